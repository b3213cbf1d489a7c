// Small kernels (grid conversion, counter reset) and the dispatch of the dock
// launches over texel storage types.
#include <math.h>

#include <algorithm>

#include "exs_internal.h"
#include "rank_poses.inc"
#include "rescore2.inc"
#include "unfold.inc"

namespace exs {

hipError_t launch_dock_f32(const DockArgs& a, int ppl, dim3 grid, dim3 block, size_t lds, hipStream_t st);
hipError_t launch_dock_bf16(const DockArgs& a, int ppl, dim3 grid, dim3 block, size_t lds, hipStream_t st);
hipError_t launch_dock_f16(const DockArgs& a, int ppl, dim3 grid, dim3 block, size_t lds, hipStream_t st);
const void* dock_kernel_fn_f32(int S, int ppl);
const void* dock_kernel_fn_bf16(int S, int ppl);
const void* dock_kernel_fn_f16(int S, int ppl);
hipError_t upload_trig_f32(const float* t32, const double* t64);
hipError_t upload_trig_bf16(const float* t32, const double* t64);
hipError_t upload_trig_f16(const float* t32, const double* t64);
hipError_t launch_gather_probe_f32(const GridDesc* gd, int nb, int64_t blocks, int per_lane,
                                   float half, float walk, uint32_t seed, float* out, hipStream_t st);
hipError_t launch_gather_probe_bf16(const GridDesc* gd, int nb, int64_t blocks, int per_lane,
                                   float half, float walk, uint32_t seed, float* out, hipStream_t st);
hipError_t launch_gather_probe_f16(const GridDesc* gd, int nb, int64_t blocks, int per_lane,
                                   float half, float walk, uint32_t seed, float* out, hipStream_t st);



// FP32 -> 16-bit texel bits, round to nearest even.
__device__ __forceinline__ uint32_t to16(float v, int storage) {
    if (storage == 1) {                       // BF16
        uint32_t u = __builtin_bit_cast(uint32_t, v);
        u += 0x7fffu + ((u >> 16) & 1u);
        return u >> 16;
    }
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v);   // FP16
}

// Expand the FP32 master [C][nz][ny][nx] (x fastest) into the per-cell gather layout, one
// 16-byte entry per thread; cx = nx-1, cy = ny-1, cz = nz-1 cells, corner index dx + 2 dy + 4 dz.
// FP32 cells are indexed (z * cy + y) * cx + x; 16-bit cells go in 2 x 2 x 2 bricks (bricks x
// fastest, cell 4 (z & 1) + 2 (y & 1) + (x & 1) within a brick; cells of an odd edge's padding
// are zero and never read).
//  FP32 (storage 0): two entries per cell, entry dz = {V(x,y,z+dz), V(x+1,y,z+dz) - V(x,y,z+dz),
//  V(x,y+1,z+dz), V(x+1,y+1,z+dz) - V(x,y+1,z+dz)} (x differences rounded in FP32, as the
//  interpolation's x round would compute them).
//  16-bit (1 BF16, 2 FP16): one entry per cell, dword j = corner(2j) | corner(2j+1) << 16.
__global__ void expand_grid_kernel(const float* __restrict__ src, uint4* __restrict__ dst,
                                   int nx, int ny, int nz, int64_t per_chan, int64_t count,
                                   int storage) {
    const int cx = nx - 1, cy = ny - 1;
    const int64_t nxy = (int64_t)nx * ny, chan = nxy * nz;
    const int per_cell = storage == 0 ? 2 : 1;
    const int cz = nz - 1, bxc = nx / 2, byc = ny / 2;   // 16-bit: bricks per row and per column
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = i / per_chan, e = i - c * per_chan;
        const int64_t cell = e / per_cell;
        const int half = (int)(e - cell * per_cell);
        int x, y, z;
        if (storage == 0) {
            x = (int)(cell % cx);
            const int64_t yz = cell / cx;
            y = (int)(yz % cy); z = (int)(yz / cy);
        } else {
            const int64_t brick = cell >> 3;
            const int sub = (int)(cell & 7);
            x = (int)(brick % bxc) * 2 + (sub & 1);
            const int64_t rest = brick / bxc;
            y = (int)(rest % byc) * 2 + ((sub >> 1) & 1);
            z = (int)(rest / byc) * 2 + (sub >> 2);
            if (x >= cx || y >= cy || z >= cz) {   // padding of an odd edge: never read
                dst[i] = make_uint4(0u, 0u, 0u, 0u);
                continue;
            }
        }
        const float* b = src + c * chan + (int64_t)z * nxy + (int64_t)y * nx + x;
        uint4 o;
        if (storage == 0) {
            const float* q = b + half * nxy;
            const float d0 = q[1] - q[0], d1 = q[nx + 1] - q[nx];   // x differences, FP32
            o = make_uint4(__builtin_bit_cast(uint32_t, q[0]), __builtin_bit_cast(uint32_t, d0),
                           __builtin_bit_cast(uint32_t, q[nx]), __builtin_bit_cast(uint32_t, d1));
        } else {
            uint32_t w[4];
            for (int j = 0; j < 4; ++j) {
                const float* r = b + (j >> 1) * nxy + (j & 1) * nx;   // (dy, dz) = (j & 1, j >> 1)
                w[j] = to16(r[0], storage) | (to16(r[1], storage) << 16);
            }
            o = make_uint4(w[0], w[1], w[2], w[3]);
        }
        dst[i] = o;
    }
}

// Zero a small int array with a kernel (safe inside a captured graph).
__global__ void zero_ints_kernel(int* p, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_dock(const DockArgs& a, int storage, int ppl, int n_blocks, int threads,
                       size_t lds, hipStream_t st) {
    dim3 grid(n_blocks), block(threads);
    switch (storage) {
        case 0: return launch_dock_f32(a, ppl, grid, block, lds, st);
        case 1: return launch_dock_bf16(a, ppl, grid, block, lds, st);
        case 2: return launch_dock_f16(a, ppl, grid, block, lds, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather_probe(const GridDesc* gd, int storage, int nb, int64_t blocks, int per_lane,
                               float half, float walk, uint32_t seed, float* out, hipStream_t st) {
    switch (storage) {
        case 0: return launch_gather_probe_f32(gd, nb, blocks, per_lane, half, walk, seed, out, st);
        case 1: return launch_gather_probe_bf16(gd, nb, blocks, per_lane, half, walk, seed, out, st);
        case 2: return launch_gather_probe_f16(gd, nb, blocks, per_lane, half, walk, seed, out, st);
        default: return hipErrorInvalidValue;
    }
}

const void* dock_kernel_fn(int storage, int S, int ppl) {
    switch (storage) {
        case 0: return dock_kernel_fn_f32(S, ppl);
        case 1: return dock_kernel_fn_bf16(S, ppl);
        case 2: return dock_kernel_fn_f16(S, ppl);
        default: return nullptr;
    }
}

int64_t expanded_entries(int nx, int ny, int nz, int storage) {
    if (storage == 0) return (int64_t)(nx - 1) * (ny - 1) * (nz - 1) * 2;
    return (int64_t)8 * (nx / 2) * (ny / 2) * (nz / 2);
}

hipError_t launch_expand_grid(const float* src, void* dst, int nx, int ny, int nz, int channels,
                              int storage, hipStream_t st) {
    const int64_t per_chan = expanded_entries(nx, ny, nz, storage);
    const int64_t count = per_chan * channels;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(expand_grid_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src,
                       static_cast<uint4*>(dst), nx, ny, nz, per_chan, count, storage);
    return hipGetLastError();
}

hipError_t launch_rank(const DockArgs& a, int n_lig, const int32_t* order, hipStream_t st) {
    if (n_lig <= 0) return hipSuccess;
    // up to 4 waves (ligands) per block, within 64 KB of LDS
    const size_t per_wave = (size_t)rank_lds_words(a.K, a.n_max) * sizeof(int);
    const int waves = (int)std::max<size_t>(1, std::min<size_t>(4, (64 * 1024) / per_wave));
    hipLaunchKernelGGL(rank_kernel, dim3((n_lig + waves - 1) / waves), dim3(waves * kWave),
                       waves * per_wave, st, a, n_lig, order);
    return hipGetLastError();
}

hipError_t launch_rescore2(const DockArgs& a, int n_lig, const int32_t* order, hipStream_t st) {
    if (n_lig <= 0) return hipSuccess;
    hipLaunchKernelGGL(rescore2_kernel, dim3(n_lig), dim3(kRescoreWaves * kWave),
                       rescore2_lds_bytes(kRescoreWaves), st, a, n_lig, order);
    return hipGetLastError();
}

hipError_t launch_unfold(const LigInfo* info, float4* ref, double* ref64, const uint32_t* rot_uv,
                         const uint4* rot_mask, int32_t* turns, const int32_t* order, int n_lig, int R,
                         int S, int passes, hipStream_t st) {
    if (n_lig <= 0) return hipSuccess;
    UnfoldArgs a{info, ref, ref64, rot_uv, rot_mask, turns, order, n_lig, R, passes, 0};
    constexpr int kWavesPerBlock = 4;
    const dim3 grid((n_lig + kWavesPerBlock - 1) / kWavesPerBlock), block(kWavesPerBlock * kWave);
    const size_t lds = (size_t)kWavesPerBlock * kUnfoldLdsPerWave;
    switch (S) {
        case 8: hipLaunchKernelGGL(unfold_kernel<8>, grid, block, lds, st, a); break;
        case 16: hipLaunchKernelGGL(unfold_kernel<16>, grid, block, lds, st, a); break;
        case 32: hipLaunchKernelGGL(unfold_kernel<32>, grid, block, lds, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// flag |= 1 for a non-finite texel, |= 2 for a finite texel that rounds to infinity in the
// 16-bit storage (RNE thresholds: FP16 |v| >= 65520, BF16 |v| >= 0x7f7f8000).
__global__ void check_texels_kernel(const float* __restrict__ v, int64_t count, int storage,
                                    int* flag) {
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t a = __builtin_bit_cast(uint32_t, v[i]) & 0x7fffffffu;
        if (a >= 0x7f800000u) bad |= 1;
        else if ((storage == 2 && a >= 0x477ff000u) || (storage == 1 && a >= 0x7f7f8000u)) bad |= 2;
    }
    if (bad) atomicOr(flag, bad);
}

hipError_t launch_check_texels(const float* v, int64_t count, int storage, int* flag, hipStream_t st) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(check_texels_kernel, dim3((unsigned)blocks), dim3(256), 0, st, v, count,
                       storage, flag);
    return hipGetLastError();
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t st) {
    hipLaunchKernelGGL(zero_ints_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

__global__ void stage_ints_kernel(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int n,
                                  int* __restrict__ zero, int nz, int lig, int n_lig,
                                  int32_t* __restrict__ slot) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nz) zero[t] = 0;
    for (int i = t; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
    for (int j = t; j < n_lig; j += gridDim.x * blockDim.x) slot[src[lig + j]] = j;
}

hipError_t launch_stage_ints(const int32_t* src, int32_t* dst, int n, int* zero, int nz, int lig,
                             int n_lig, int32_t* slot, hipStream_t st) {
    const int blocks = std::max(1, std::min(256, (std::max(n, nz) + 255) / 256));
    hipLaunchKernelGGL(stage_ints_kernel, dim3(blocks), dim3(256), 0, st, src, dst, n, zero, nz, lig,
                       n_lig, slot);
    return hipGetLastError();
}

// Fibonacci-sphere orientations R_k = Rz(phi_k) Ry(beta_k): z_k = 1 - (2k+1)/K, beta_k = acos z_k,
// phi_k = k * golden angle, rows of the product in FP64 and rounded to FP32.  Computed on the
// device so that every launch path (and a path that cannot allocate or copy from the host)
// reads the same table bit for bit.
__global__ void orientation_table_kernel(int K, float* __restrict__ r32, double* __restrict__ r64) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double golden = 3.14159265358979323846 * (3.0 - sqrt(5.0));
    const double zk = 1.0 - (2.0 * k + 1.0) / (double)K;
    const double beta = acos(zk), phi = (double)k * golden;
    const double cb = cos(beta), sb = sin(beta), cp = cos(phi), sp = sin(phi);
    const double m[9] = {cp * cb, -sp, cp * sb, sp * cb, cp, sp * sb, -sb, 0.0, cb};
    for (int t = 0; t < 9; ++t) {
        if (r64) r64[(size_t)k * 9 + t] = m[t];
        r32[(size_t)k * 9 + t] = (float)m[t];
    }
}

hipError_t launch_orientation_table(int K, float* r32, double* r64, hipStream_t st) {
    hipLaunchKernelGGL(orientation_table_kernel, dim3((K + 63) / 64), dim3(64), 0, st, K, r32, r64);
    return hipGetLastError();
}

// Fill the turn tables of the current device: FP32 from the quarter-period literals (the
// same values the unrolled kernels use), checked against FP64 cos / sin rounded to FP32;
// FP64 from the host's cos / sin.
template <int S>
static bool fill_trig(float* t32, double* t64) {
    const int off = trig_offset(S);
    bool ok = true;
    for (int s = 0; s < S; ++s) {
        double a = 2.0 * 3.14159265358979323846 * (double)s / (double)S;
        double c = (4 * s == S || 4 * s == 3 * S) ? 0.0 : (s == 0 ? 1.0 : cos(a));
        double sn = (s == 0 || 2 * s == S) ? 0.0 : (4 * s == S ? 1.0 : (4 * s == 3 * S ? -1.0 : sin(a)));
        t64[off + s] = c;
        t64[off + S + s] = sn;
        t32[off + s] = kcos<S>(s);
        t32[off + S + s] = ksin<S>(s);
        ok = ok && t32[off + s] == (float)c && t32[off + S + s] == (float)sn;
    }
    return ok;
}

hipError_t upload_trig_tables() {
    float t32[kTrigEntries];
    double t64[kTrigEntries];
    if (!fill_trig<8>(t32, t64) || !fill_trig<16>(t32, t64) || !fill_trig<32>(t32, t64))
        return hipErrorInvalidValue;   // a literal of the quarter-period table is wrong
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_trig64), t64, sizeof(double) * kTrigEntries);
    if (e == hipSuccess) e = upload_trig_f32(t32, t64);
    if (e == hipSuccess) e = upload_trig_bf16(t32, t64);
    if (e == hipSuccess) e = upload_trig_f16(t32, t64);
    return e;
}

}  // namespace exs
