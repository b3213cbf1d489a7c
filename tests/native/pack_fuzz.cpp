// Host-side packing under AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure;
// built with g++ for the host only by tests/test_pack_sanitizers.py).
//
// Reads ligands (CSR, the layout the C ABI takes) from a binary file and packs each one with
// pack_ligand, the validation and topology packing every upload and served request goes
// through; then mutates each ligand into invalid forms (atom, bond and rotatable-bond indices
// out of range, counts beyond the limits, a ring bond made rotatable, a type beyond the
// channels) and checks they are refused; then costs the ligands and lays them out in work
// queues.  Any out-of-bounds access or undefined behaviour aborts under the sanitizers.
#include <stdio.h>
#include <stdlib.h>

#include <string>
#include <vector>

#include "exs.h"
#include "exs_pack.h"

using namespace exs;

template <class T>
static bool read_vec(FILE* f, std::vector<T>& v) {
    int64_t n = 0;
    if (fread(&n, sizeof n, 1, f) != 1 || n < 0) return false;
    v.resize((size_t)n);
    return n == 0 || fread(v.data(), sizeof(T), (size_t)n, f) == (size_t)n;
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    std::vector<int32_t> ao, bo, bij, ro, rb;
    std::vector<float> x, y, z;
    std::vector<uint8_t> type;
    if (!read_vec(f, ao) || !read_vec(f, x) || !read_vec(f, y) || !read_vec(f, z) ||
        !read_vec(f, type) || !read_vec(f, bo) || !read_vec(f, bij) || !read_vec(f, ro) ||
        !read_vec(f, rb))
        return 2;
    fclose(f);
    const int L = (int)ao.size() - 1;
    int packed = 0, refused = 0, tried = 0;
    std::vector<double> cost(L);
    std::vector<int> pocket(L);
    for (int l = 0; l < L; ++l) {
        const int a0 = ao[l], n = ao[l + 1] - a0;
        const int b0 = bo[l], nb = bo[l + 1] - b0;
        const int r0 = ro[l], nr = ro[l + 1] - r0;
        PackedLigand pk;
        std::string err;
        // copies sized exactly, so the sanitizer sees any read past a ligand's own arrays
        std::vector<int32_t> b(bij.begin() + 2 * b0, bij.begin() + 2 * (b0 + nb));
        std::vector<int32_t> r(rb.begin() + r0, rb.begin() + r0 + nr);
        std::vector<uint8_t> t(type.begin() + a0, type.begin() + a0 + n);
        std::vector<float> xs(x.begin() + a0, x.begin() + a0 + n), ys(y.begin() + a0, y.begin() + a0 + n),
            zs(z.begin() + a0, z.begin() + a0 + n);
        if (pack_ligand(n, b.data(), nb, r.data(), nr, t.data(), 8, xs.data(), ys.data(), zs.data(),
                        &pk, &err) != EXS_OK) {
            fprintf(stderr, "ligand %d refused: %s\n", l, err.c_str());
            return 1;
        }
        ++packed;
        std::vector<int16_t> m(pk.nrot);
        for (int q = 0; q < pk.nrot; ++q) m[q] = (int16_t)pk.moving[q].count();
        cost[l] = ligand_cost(pk.n, m.data(), pk.nrot, 256, 32, 2, 27);
        pocket[l] = l % 3;
        // invalid forms
        std::vector<std::vector<int32_t>> bad_bonds;
        if (nb > 0) {
            std::vector<int32_t> bb = b;
            bb[0] = n;                      // atom index past the ligand
            bad_bonds.push_back(bb);
            bb = b;
            bb[2 * nb - 1] = -1;            // negative atom index
            bad_bonds.push_back(bb);
        }
        tried += (int)bad_bonds.size();
        for (auto& bb : bad_bonds)
            refused += pack_ligand(n, bb.data(), nb, r.data(), nr, t.data(), 8, xs.data(), ys.data(),
                                   zs.data(), &pk, &err) != EXS_OK;
        if (nr > 0) {
            std::vector<int32_t> rr = r;
            tried += 2;
            rr[0] = nb;                     // rotatable bond past the bond list
            refused += pack_ligand(n, b.data(), nb, rr.data(), nr, t.data(), 8, xs.data(), ys.data(),
                                   zs.data(), &pk, &err) != EXS_OK;
            rr[0] = -1;
            refused += pack_ligand(n, b.data(), nb, rr.data(), nr, t.data(), 8, xs.data(), ys.data(),
                                   zs.data(), &pk, &err) != EXS_OK;
        }
        if (nb > 0 && n >= 3) {             // close a ring through the first rotatable bond's ends
            std::vector<int32_t> bb = b;
            int u = b[0], v = b[1];
            int w = -1;
            for (int e = 0; e < nb && w < 0; ++e) {
                if (b[2 * e] == v && b[2 * e + 1] != u) w = b[2 * e + 1];
                else if (b[2 * e + 1] == v && b[2 * e] != u) w = b[2 * e];
            }
            if (w >= 0) {
                bb.push_back(u);
                bb.push_back(w);
                std::vector<int32_t> rr{0};
                tried += 1;
                refused += pack_ligand(n, bb.data(), nb + 1, rr.data(), 1, t.data(), 8, xs.data(),
                                       ys.data(), zs.data(), &pk, &err) != EXS_OK;
            }
        }
        std::vector<uint8_t> tt = t;
        tt[n - 1] = 8;                      // type beyond the channels
        tried += 3;
        refused += pack_ligand(n, b.data(), nb, r.data(), nr, tt.data(), 8, xs.data(), ys.data(),
                               zs.data(), &pk, &err) != EXS_OK;
        refused += pack_ligand(EXS_MAX_ATOMS + 1, b.data(), nb, r.data(), nr, t.data(), 8, xs.data(),
                               ys.data(), zs.data(), &pk, &err) != EXS_OK;
        refused += pack_ligand(n, b.data(), nb, r.data(), EXS_MAX_ROT + 1, t.data(), 8, xs.data(),
                               ys.data(), zs.data(), &pk, &err) != EXS_OK;
    }
    std::vector<int32_t> order((size_t)L + kMaxWorkQueues + 1);
    for (int nq : {1, 2, 8})
        for (int pm = 0; pm < 2; ++pm)
            work_queues(L, pocket.data(), cost.data(), nq, pm != 0, order.data(), order.data() + L);
    printf("packed %d refused %d of %d\n", packed, refused, tried);
    return 0;
}
