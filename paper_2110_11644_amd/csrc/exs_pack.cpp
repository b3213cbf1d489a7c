// Host-side topology packing: bond-distance exclusion masks and the moving side
// of every torsional bond, as 128-bit rows (one bit per atom).
//
// Sec. 3.1: each torsional bond splits the ligand's atoms into two disjoint
// sets that turn about the bond axis.  The side that does not hold atom 0
// turns, so nested bonds compose in any order.  Pairs within three bonds
// (1-2, 1-3, 1-4) are excluded from the clash term.
#include "exs_pack.h"

#include <algorithm>

#include <stdio.h>

#include "exs.h"

namespace exs {

// Call f(i) for every set bit i of b, in increasing order.
template <class F>
static inline void for_each_bit(const Bits128& b, F f) {
    for (uint64_t w = b.lo; w; w &= w - 1) f(__builtin_ctzll(w));
    for (uint64_t w = b.hi; w; w &= w - 1) f(64 + __builtin_ctzll(w));
}

// Atoms reachable from `start` without crossing the edge (cut_a, cut_b).
static Bits128 flood(const Bits128* adj, int start, int cut_a, int cut_b) {
    Bits128 seen, frontier;
    seen.set(start);
    frontier.set(start);
    while (frontier.lo | frontier.hi) {
        Bits128 next;
        for_each_bit(frontier, [&](int i) {
            Bits128 a = adj[i];
            if (i == cut_a) a.clear(cut_b);
            if (i == cut_b) a.clear(cut_a);
            next |= a;
        });
        Bits128 fresh;
        fresh.lo = next.lo & ~seen.lo;
        fresh.hi = next.hi & ~seen.hi;
        seen |= fresh;
        frontier = fresh;
    }
    return seen;
}

int pack_ligand(int n, const int32_t* bond_ij, int nb, const int32_t* rot_bond, int nrot,
                const uint8_t* type, int channels, const float* x, const float* y,
                const float* z, PackedLigand* out, std::string* err) {
    char buf[256];
    if (n < 1 || n > EXS_MAX_ATOMS) {
        snprintf(buf, sizeof buf, "atom count %d outside [1, %d]", n, EXS_MAX_ATOMS);
        *err = buf;
        return EXS_EINVAL;
    }
    if (nrot < 0 || nrot > EXS_MAX_ROT) {
        snprintf(buf, sizeof buf, "%d rotatable bonds (max %d)", nrot, EXS_MAX_ROT);
        *err = buf;
        return EXS_EINVAL;
    }
    if (nb < 0) { *err = "negative bond count"; return EXS_EINVAL; }
    for (int i = 0; i < n; ++i) {
        if ((int)type[i] >= channels) {
            snprintf(buf, sizeof buf, "atom %d has type %d, pocket has %d channels", i, type[i],
                     channels);
            *err = buf;
            return EXS_EINVAL;
        }
        if (!(x[i] == x[i]) || !(y[i] == y[i]) || !(z[i] == z[i]) ||
            x[i] - x[i] != 0.0f || y[i] - y[i] != 0.0f || z[i] - z[i] != 0.0f) {
            snprintf(buf, sizeof buf, "atom %d has a non-finite coordinate", i);
            *err = buf;
            return EXS_EINVAL;
        }
    }
    Bits128 adj[EXS_MAX_ATOMS];
    for (int e = 0; e < nb; ++e) {
        int p = bond_ij[2 * e], q = bond_ij[2 * e + 1];
        if (p < 0 || p >= n || q < 0 || q >= n || p == q) {
            snprintf(buf, sizeof buf, "bond %d (%d, %d) invalid for %d atoms", e, p, q, n);
            *err = buf;
            return EXS_EINVAL;
        }
        adj[p].set(q);
        adj[q].set(p);
    }
    out->n = n;
    out->nrot = nrot;
    // bond distance <= 1, then <= 2, then <= 3
    Bits128 d1[EXS_MAX_ATOMS], d2[EXS_MAX_ATOMS];
    for (int i = 0; i < n; ++i) { d1[i] = adj[i]; d1[i].set(i); }
    for (int i = 0; i < n; ++i) for_each_bit(d1[i], [&](int j) { d2[i] |= d1[j]; });
    out->excl.assign(n, Bits128());
    for (int i = 0; i < n; ++i) for_each_bit(d2[i], [&](int j) { out->excl[i] |= d1[j]; });
    out->rot_u.resize(nrot);
    out->rot_v.resize(nrot);
    out->moving.assign(nrot, Bits128());
    for (int b = 0; b < nrot; ++b) {
        int e = rot_bond[b];
        if (e < 0 || e >= nb) {
            snprintf(buf, sizeof buf, "rotatable bond %d names bond %d of %d", b, e, nb);
            *err = buf;
            return EXS_EINVAL;
        }
        int p = bond_ij[2 * e], q = bond_ij[2 * e + 1];
        Bits128 sp = flood(adj, p, p, q);
        if (sp.test(q)) {
            snprintf(buf, sizeof buf, "rotatable bond %d (%d-%d) is in a ring", b, p, q);
            *err = buf;
            return EXS_EINVAL;
        }
        Bits128 sq = flood(adj, q, p, q);
        int u, v;
        Bits128 side;
        if (sp.test(0)) { u = p; v = q; side = sq; }
        else if (sq.test(0)) { u = q; v = p; side = sp; }
        else {
            snprintf(buf, sizeof buf, "rotatable bond %d (%d-%d) is not connected to atom 0", b,
                     p, q);
            *err = buf;
            return EXS_EINVAL;
        }
        side.clear(v);
        const double ax = (double)x[v] - x[u], ay = (double)y[v] - y[u], az = (double)z[v] - z[u];
        if (!(ax * ax + ay * ay + az * az > 1e-12)) {
            snprintf(buf, sizeof buf, "rotatable bond %d (%d-%d) has zero length", b, p, q);
            *err = buf;
            return EXS_EINVAL;
        }
        out->rot_u[b] = u;
        out->rot_v[b] = v;
        out->moving[b] = side;
    }
    double c[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i) { c[0] += (double)x[i]; c[1] += (double)y[i]; c[2] += (double)z[i]; }
    for (int a = 0; a < 3; ++a) out->centroid[a] = c[a] / (double)n;
    return EXS_OK;
}

double ligand_cost(int n, const int16_t* m, int nrot, int K, int S, int P, int T) {
    // texel lookups: the final score (n), per pass S per moving atom and T per atom;
    // pair tests: moving x static per bond and pass, plus the two full scores.
    double look = 2.0 * n, pairs = (double)n * n;
    for (int b = 0; b < nrot; ++b) {
        look += (double)P * S * m[b];
        pairs += (double)P * m[b] * (double)(n - m[b]);
    }
    look += (double)P * (T > 1 ? T : 0) * n;
    return (double)K * (look * 40.0 + pairs * 20.0);
}

void work_queues(int n, const int* pocket, const double* cost, int n_queues, bool pocket_major,
                 int32_t* order, int32_t* bounds) {
    std::vector<int32_t> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) {
        if (pocket[a] != pocket[c]) return pocket[a] < pocket[c];
        return cost[a] > cost[c];
    });
    double total = 0.0;
    for (int i = 0; i < n; ++i) total += cost[i];
    for (int q = 0; q <= n_queues; ++q) bounds[q] = n;
    bounds[0] = 0;
    double acc = 0.0;
    int q = 1;
    for (int i = 0; i < n && q < n_queues; ++i) {
        acc += cost[ord[i]];
        while (q < n_queues && acc >= total * q / n_queues) bounds[q++] = i + 1;
    }
    if (!pocket_major)
        for (int r = 0; r < n_queues; ++r)
            std::stable_sort(ord.begin() + bounds[r], ord.begin() + bounds[r + 1],
                             [&](int a, int c) { return cost[a] > cost[c]; });
    std::copy(ord.begin(), ord.end(), order);
}

}  // namespace exs
