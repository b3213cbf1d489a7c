// Internal layout shared by the host runtime and the HIP kernels of libexs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exs {

constexpr int kWave = 64;
constexpr int kMaxAtoms = 128;   // bits of one exclusion / moving mask row
constexpr int kMaxRot = 32;
constexpr int kMaxTopK = 32;
constexpr int kMaxLpw = 8;       // ligands per workgroup
constexpr int kMaxWavesPerWg = 8;
constexpr int kMaxThreadsPerWg = kMaxWavesPerWg * kWave;
constexpr int kXcds = 8;   // accelerator complex dies of an MI355X, each with its own L2

// Work queues of a persistent launch: the workgroups of XCD x start on queue x % n_queues and
// move on to the others once it is drained.  Two layouts of the order:
//  * spread: kXcds queues, contiguous pocket-major runs of equal cost, each longest first.  For
//    launches whose pockets hold fewer ligands each than the device has in flight: all of the
//    launch runs at once and its tail decides (serving iterations of <= 4,096 ligands over 15
//    pockets: capacity 152k docks/s, against 127k pocket by pocket).
//  * pocket-major: kPocketMajorQueues queues, each pocket by pocket, longest first within a
//    pocket, so that few pockets are in use at a time and their texel blocks stay in the L2s and
//    the shared last-level cache (100,000 ligands over 15 pockets, FP32: 634 ms spread; 567,
//    543, 548 ms with 1, 2, 4 pocket-major queues).
constexpr int kMaxWorkQueues = kXcds;
constexpr int kPocketMajorQueues = 2;
constexpr int kInflightWaves = 256 * 4 * 3;   // CUs x SIMDs x dock-kernel waves per SIMD
struct QueuePlan {
    int n_queues;
    bool pocket_major;
};
// Layout for n_ligands ligands over n_pockets distinct pockets, waves_per_ligand waves each.
inline QueuePlan queue_plan(int64_t n_ligands, int n_pockets, int waves_per_ligand) {
    const int64_t inflight = kInflightWaves / (waves_per_ligand > 0 ? waves_per_ligand : 1);
    if (n_pockets >= 2 && n_ligands >= inflight * n_pockets) return {kPocketMajorQueues, true};
    return {kXcds, false};
}

// Turn tables: for S in {8, 16, 32}, cos then sin of 2*pi*s/S at offset trig_offset(S).
constexpr int kTrigEntries = 2 * (8 + 16 + 32);
__host__ __device__ constexpr int trig_offset(int S) { return S == 8 ? 0 : (S == 16 ? 16 : 48); }

// cos(2 pi m / S) for 0 <= m <= S/4, FP64 values rounded to FP32 (RNE).  Every turn
// 2 pi s / S of the torsion sweep has cos and sin equal to +-qcos(m) for some m, so the
// unrolled sweep needs S/4 + 1 constants and the signs fold into FMA source modifiers.
// upload_trig_tables() checks these literals against the host's FP64 cos.
template <int S> __host__ __device__ __forceinline__ constexpr float qcos(int m);
template <> __host__ __device__ __forceinline__ constexpr float qcos<8>(int m) {
    return m == 0 ? 1.0f : (m == 1 ? 0x1.6a09e6p-1f : 0.0f);
}
template <> __host__ __device__ __forceinline__ constexpr float qcos<16>(int m) {
    return m == 0 ? 1.0f : m == 1 ? 0x1.d906bcp-1f : m == 2 ? 0x1.6a09e6p-1f
         : m == 3 ? 0x1.87de2ap-2f : 0.0f;
}
template <> __host__ __device__ __forceinline__ constexpr float qcos<32>(int m) {
    return m == 0 ? 1.0f : m == 1 ? 0x1.f6297cp-1f : m == 2 ? 0x1.d906bcp-1f
         : m == 3 ? 0x1.a9b662p-1f : m == 4 ? 0x1.6a09e6p-1f : m == 5 ? 0x1.1c73b4p-1f
         : m == 6 ? 0x1.87de2ap-2f : m == 7 ? 0x1.8f8b84p-3f : 0.0f;
}
// cos and sin of 2 pi s / S, 0 <= s < S, from the quarter-period table.
template <int S> __host__ __device__ __forceinline__ constexpr float kcos(int s) {
    constexpr int Q = S / 4;
    const int q = s / Q, r = s % Q;
    return q == 0 ? qcos<S>(r) : q == 1 ? -qcos<S>(Q - r) : q == 2 ? -qcos<S>(r) : qcos<S>(Q - r);
}
template <int S> __host__ __device__ __forceinline__ constexpr float ksin(int s) {
    constexpr int Q = S / 4;
    const int q = s / Q, r = s % Q;
    return q == 0 ? qcos<S>(Q - r) : q == 1 ? qcos<S>(r) : q == 2 ? -qcos<S>(Q - r) : -qcos<S>(r);
}

// One packed ligand (caller order).
struct LigInfo {
    int32_t atom_base;   // first atom in the packed atom arrays
    int32_t rot_base;    // first rotatable bond in the packed bond arrays
    int16_t n;           // atoms
    int16_t nrot;        // rotatable bonds
    int16_t pocket;      // index into the job's pocket table
    int16_t pad;
    float cost;          // relative search cost, for longest-first ordering
    int32_t pad2[3];
};
static_assert(sizeof(LigInfo) == 32, "LigInfo layout");

// One pocket as the kernels see it.
struct GridDesc {
    const void* tex;       // per-cell gather blocks, one channel every chan_bytes: the 8 corners
                           // of a cell, 32 B in FP32 (x pairs as a, b - a, cells x fastest),
                           // 16 B in BF16/FP16 (cells in 2 x 2 x 2 bricks of one line)
    const float* master;   // FP32 master texels [C][nz][ny][nx] (FP64 rescoring)
    int nx, ny, nz, channels;
    float ox, oy, oz, inv_h;   // origin and 1/spacing, FP32
    float cx, cy, cz, pad;     // pocket centre (grid centre), FP32
    float ux_hi, uy_hi, uz_hi, pad1;  // largest floats below N-1 per axis (grid-unit clamp)
    double h, dox, doy, doz;   // FP64 geometry for the rescoring
    double dcx, dcy, dcz, dpad;
    int32_t chan_bytes;        // bytes of one channel of the gather layout
    int32_t master_chan_bytes; // bytes of one FP32 channel
    int32_t storage;           // EXS_F32 / EXS_BF16 / EXS_F16
    int32_t pad3;
};

// Everything one dock launch reads and writes.
// Serving: the results of one iteration's ligands in contiguous host memory (one record per
// ligand, then coordinates and torsion bytes at host-computed offsets).
struct ResultRec {
    float score;
    int32_t k;
    int32_t tau;
    int32_t pad;
    double score64;
};

struct DockArgs {
    // packed ligand batch
    const LigInfo* info;
    const float4* ref;        // [A] centred input coords, type in .w (int bits)
    const double* ref64;      // [A*3] centred input coords in FP64 (rescoring)
    const uint4* excl;        // [A] bit j: pair (i, j) excluded (bond distance <= 3, or i == j)
    const uint32_t* rot_uv;   // [R] u | v << 16, u on atom 0's side
    const uint4* rot_mask;    // [R] atoms that turn with the bond
    const int32_t* order;     // ligands in processing order (pocket-major, longest first within)
    int32_t n_order;          // ligands in this launch
    int32_t n_tiles;          // ceil(n_order / lpw)
    // pockets
    const GridDesc* grids;
    // search settings
    const float* rot32;       // [K][9] orientation matrices, row-major
    const double* rot64;      // [K][9]
    int32_t K, S, P, T;
    float step, cut2, pen, pad0;
    double step64, cut2_64, pen64;
    int32_t top_k;
    int32_t lpw;              // ligands per workgroup
    int32_t wpl;              // waves per ligand = ceil(K / (64 * ppl))
    int32_t kp;               // padded orientations per ligand = wpl * 64 * ppl
    int32_t n_max;            // atoms of the largest ligand in the launch
    int32_t persistent;
    // per-workgroup-slot scratch of pose coordinates: [lpw][n_max][3][kp] floats
    float* scratch;
    int64_t slot_floats;
    int32_t* tile_counter;    // persistent launches: next tile of each queue [n_queues]
    // persistent launches: n_queues + 1 positions in `order`, queue q = [qb[q], qb[q+1]);
    // a workgroup takes tiles from queue (its XCD index mod n_queues) first, then from the
    // others.  Null, or n_queues = 1: one queue over the whole order.
    const int32_t* queue_bounds;
    int32_t n_queues;
    int32_t pad1;
    // outputs (indexed by caller ligand / rotatable-bond index)
    float* orient_score;      // [L*K]
    uint8_t* orient_theta;    // [R*K], element (rot_base+b)*K + k
    int32_t* orient_tau;      // [L*K], tau packed as 3 signed bytes
    float* best_score;        // [L]
    int32_t* best_k;          // [L]
    float* best_coords;       // [A*3]
    uint8_t* best_theta;      // [R]
    int32_t* best_tau;        // [L]
    double* best_score64;     // [L]   (top_k > 0)
    int32_t* topk_k;          // [L*top_k]
    float* topk_score;        // [L*top_k] FP32 search score
    double* topk_score64;     // [L*top_k]
    uint8_t* topk_theta;      // [R*top_k], element (rot_base+b)*top_k + t
    int32_t* topk_tau;        // [L*top_k]
    // ranking of the final poses (rank_keep > 0)
    float rank_thr2;          // RMSD threshold squared (A^2)
    int32_t rank_keep;        // ranked poses kept per ligand
    int32_t* n_clusters;      // [L]
    int32_t* ranked;          // [L*rank_keep] orientation indices, leaders first
    float* final_xyz;         // [A*3][K] final pose of every orientation (rank_keep > 0)
    // second-stage rescoring of the ranked poses (rescore2 > 0; needs rank_keep > 0)
    int32_t rescore2;
    int32_t pad2;
    const uint32_t* rot_ac;   // [R] a | c << 16 (0xffff: none): dihedral neighbours of u and v
    double eps2, w2;          // contact well depth, torsion weight of the second-stage score
    double* score2;           // [L*rank_keep] second-stage score of each ranked pose
    int32_t* best2_k;         // [L] orientation of the lowest second-stage score
    double* best2;            // [L] that score
    // serving iterations (res_rec non-null): each ligand's finish also writes its result to the
    // iteration's result buffer (mapped host memory), at position j = res_slot[l]: the record
    // res_rec[j], coordinates from res_coords + 3 res_adst[j], torsion bytes from
    // res_theta + res_rdst[j]; no kernel runs after the search
    const int32_t* res_slot;  // [L] position of each ligand in its iteration's work list
    const int32_t* res_adst;  // [work list]
    const int32_t* res_rdst;  // [work list]
    ResultRec* res_rec;
    float* res_coords;
    uint8_t* res_theta;
};

// LDS words per wave of the ranking kernel: rank, state and score per pose, the leader bits,
// the coordinates of 8 candidate leaders (3 n_max rows each, n_max the launch's largest
// ligand) and the list of uncovered poses.
__host__ __device__ inline int rank_lds_words(int K, int n_max) {
    return 4 * K + (K + 31) / 32 + 8 * 3 * n_max;
}

// Per-ligand LDS staging of a tile (topology read wave-uniformly by the search).
struct LigLds {
    float4 ref[kMaxAtoms];     // centred reference coordinates, type in .w
    uint4 excl[kMaxAtoms];     // exclusion rows
    uint4 rmask[kMaxRot];      // moving masks
    uint32_t ruv[kMaxRot];     // u | v << 16
    int32_t lig, n, nrot, pocket;
    int32_t atom_base, rot_base, pad0, pad1;
    int32_t topk[kMaxTopK];
};

// Dynamic LDS bytes of a dock launch: the tile's ligands, the FP64 rescoring poses (top_k > 0)
// and, per wave, a clash difference array of S counters per pose slot and lane.
__host__ __device__ inline size_t dock_lds_x64_offset(int lpw) { return (size_t)lpw * sizeof(LigLds); }
__host__ __device__ inline size_t dock_lds_diff_offset(int lpw, int top_k) {
    return dock_lds_x64_offset(lpw) + (top_k > 0 ? (size_t)lpw * kMaxAtoms * 3 * sizeof(double) : 0);
}
__host__ __device__ inline size_t dock_lds_bytes(int lpw, int top_k, int waves, int ppl, int S) {
    return dock_lds_diff_offset(lpw, top_k) + (size_t)waves * ppl * S * kWave * sizeof(int32_t);
}
constexpr size_t kMaxLdsBytes = 160 * 1024;   // gfx950 LDS per workgroup
// Waves of a dock workgroup for a tile of lpw ligands x wpl orientation chunks: one per chunk
// up to kMaxWavesPerWg, fewer if their clash difference arrays would not fit in LDS (the waves
// then take the chunks in turn); 0 if not even one wave fits.
__host__ __device__ inline int dock_waves(int lpw, int wpl, int top_k, int ppl, int S) {
    int w = lpw * wpl < kMaxWavesPerWg ? lpw * wpl : kMaxWavesPerWg;
    while (w > 0 && dock_lds_bytes(lpw, top_k, w, ppl, S) > kMaxLdsBytes) --w;
    return w;
}

// Launchers (dock_misc.hip).
hipError_t launch_dock(const DockArgs& a, int storage, int ppl, int n_blocks, int threads,
                       size_t lds, hipStream_t st);
// Per-cell gather layout of a pocket channel, in 16-byte entries: the 8 corners of each of the
// (nx-1)(ny-1)(nz-1) cells, two entries per cell for FP32; one per cell for 16-bit, in
// 2 x 2 x 2 bricks (8 * (nx/2)(ny/2)(nz/2) entries with the padding of odd edges).
int64_t expanded_entries(int nx, int ny, int nz, int storage);
hipError_t launch_expand_grid(const float* src, void* dst, int nx, int ny, int nz, int channels,
                              int storage, hipStream_t st);
// Gather probe over the pocket `gd` (device pointer) in `storage`: blocks x 256 lanes, nb
// (8, 16 or 32) independent lookups per round.
hipError_t launch_gather_probe(const GridDesc* gd, int storage, int nb, int64_t blocks, int per_lane,
                               float half, float walk, uint32_t seed, float* out, hipStream_t st);
// Unfolding of `n_lig` packed ligands in place (ref, ref64), S turns per bond, `passes` passes;
// turns [passes * R] receives the kept turns (or null).
// The waves take the ligands in `order` (a permutation of 0..n_lig-1, longest first).
hipError_t launch_unfold(const LigInfo* info, float4* ref, double* ref64, const uint32_t* rot_uv,
                         const uint4* rot_mask, int32_t* turns, const int32_t* order, int n_lig, int R,
                         int S, int passes, hipStream_t st);
// Ranking of the final poses of `n_lig` ligands (rank_keep > 0), one wave per ligand, the
// ligands taken in `order` (a permutation of 0..n_lig-1, longest first).
hipError_t launch_rank(const DockArgs& a, int n_lig, const int32_t* order, hipStream_t st);
// Second-stage rescoring of the ranked poses of `n_lig` ligands, one block of waves per ligand,
// the ligands taken in `order`.
hipError_t launch_rescore2(const DockArgs& a, int n_lig, const int32_t* order, hipStream_t st);
hipError_t launch_zero_ints(int* p, int n, hipStream_t st);
// dst[0..n) = src[0..n), zero[0..nz) = 0 and slot[src[lig + j]] = j for j < n_lig, one kernel;
// src may be mapped host memory (a kernel reads it over the bus, so no copy call is queued).
hipError_t launch_stage_ints(const int32_t* src, int32_t* dst, int n, int* zero, int nz, int lig,
                             int n_lig, int32_t* slot, hipStream_t st);
// *flag |= 1 if a texel is not finite, |= 2 if one overflows the 16-bit storage (storage 1, 2).
hipError_t launch_check_texels(const float* v, int64_t count, int storage, int* flag, hipStream_t st);
// K orientation matrices [K][9] (row-major), FP32 and (unless r64 is null) FP64.
hipError_t launch_orientation_table(int K, float* r32, double* r64, hipStream_t st);
hipError_t upload_trig_tables();
const void* dock_kernel_fn(int storage, int S, int ppl);

}  // namespace exs
