// Host-side topology packing of ligand batches (no HIP calls; testable on the CPU).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "exs_internal.h"

namespace exs {

struct Bits128 {
    uint64_t lo = 0, hi = 0;
    bool test(int i) const { return i < 64 ? (lo >> i) & 1u : (hi >> (i - 64)) & 1u; }
    void set(int i) { if (i < 64) lo |= 1ull << i; else hi |= 1ull << (i - 64); }
    void clear(int i) { if (i < 64) lo &= ~(1ull << i); else hi &= ~(1ull << (i - 64)); }
    Bits128& operator|=(const Bits128& o) { lo |= o.lo; hi |= o.hi; return *this; }
    bool operator==(const Bits128& o) const { return lo == o.lo && hi == o.hi; }
    int count() const { return __builtin_popcountll(lo) + __builtin_popcountll(hi); }
    uint4 as_uint4() const {
        return make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    }
};

// Packed, validated topology of one ligand.
struct PackedLigand {
    int n = 0, nrot = 0;
    std::vector<Bits128> excl;     // [n]   bond distance <= 3 (self included)
    std::vector<int> rot_u, rot_v; // [nrot] u on atom 0's side
    std::vector<Bits128> moving;   // [nrot]
    double centroid[3] = {0, 0, 0};
};

// Validate and pack one ligand.  Returns 0 or a negative status with a message in *err.
int pack_ligand(int n, const int32_t* bond_ij, int nb, const int32_t* rot_bond, int nrot,
                const uint8_t* type, int channels, const float* x, const float* y,
                const float* z, PackedLigand* out, std::string* err);

// Relative search cost of one ligand (lookups and pair tests it implies), for
// longest-first ordering of the work.
// m[b] = atoms that turn with rotatable bond b.
double ligand_cost(int n, const int16_t* m, int nrot, int K, int S, int P, int T);

// Work queues of a persistent launch: items (ligands) ordered pocket-major, cut into n_queues
// contiguous ranges of equal total cost; within a range, longest first (pocket_major false) or
// pocket by pocket, longest first within a pocket (pocket_major true).  order[0..n) receives
// item indices, bounds[0..n_queues] the range starts (bounds[n_queues] = n).
void work_queues(int n, const int* pocket, const double* cost, int n_queues, bool pocket_major,
                 int32_t* order, int32_t* bounds);

}  // namespace exs
