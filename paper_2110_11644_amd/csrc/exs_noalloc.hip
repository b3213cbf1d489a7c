// Docking entry point that allocates no device memory.
//
// For callers that cannot allocate (code under stream capture, tight serving loops, harnesses
// that forbid allocation): the search of exs_dock_batch as one persistent launch, with its
// intermediate buffers -- the orientation table, the work counter, every orientation's score and
// descriptor, and the pose coordinates of each resident workgroup -- carved from one static
// device array per device instead of allocated per job.  Inputs are the uploaded batch and its
// resident pockets; the per-ligand results go to the caller's device buffers.
//
// The array's host-side name is not a device address: its address on each device comes from
// hipGetSymbolAddress, once per device, and only that address is passed to kernels.  Every call
// on a device shares the array, so calls that overlap on one device race; the counter is
// cleared by a kernel at every call, and every other region is written before it is read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "exs.h"
#include "exs_internal.h"
#include "exs_runtime.h"

namespace {

constexpr size_t kScratchBytes = (size_t)EXS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::unordered_map<int, unsigned char*> g_scratch_of;   // device -> address of `scratch` there

// Address of this device's copy of the scratch array (looked up once per device, with that
// device current).
int scratch_address(int dev, unsigned char** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch_of.find(dev);
    if (it == g_scratch_of.end()) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return exs::rt::fail(EXS_EDEVICE, "scratch address on device %d: %s", dev,
                                 hipGetErrorString(e));
        it = g_scratch_of.emplace(dev, static_cast<unsigned char*>(ptr)).first;
    }
    *out = it->second;
    return EXS_OK;
}

// Consecutive 256-byte aligned regions of the scratch array.
struct Carve {
    unsigned char* base;
    size_t used = 0;
    template <class T>
    T* take(size_t count) {
        T* p = reinterpret_cast<T*>(base + used);
        used += (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~(size_t)255;
        return p;
    }
};

}  // namespace

extern "C" int exs_dock_batch_noalloc(int64_t batch, const exs_search_params* params, void* stream,
                                      float* best_score, int32_t* best_orient, int32_t* best_tau,
                                      uint8_t* best_theta, float* best_coords) {
    using namespace exs;
    rt::NoAllocPlan pl;
    if (int rc = rt::noalloc_plan(batch, params, &pl)) return rc;
    if (pl.L == 0) return EXS_OK;
    if (!best_score || !best_orient || !best_tau || !best_coords || (pl.R > 0 && !best_theta))
        return rt::fail(EXS_EINVAL, "null output buffer");
    unsigned char* base = nullptr;
    if (int rc = scratch_address(pl.device, &base)) return rc;
    DockArgs a = pl.args;
    const int64_t L = pl.L, R = pl.R, K = a.K;
    Carve c{base};
    float* rot32 = c.take<float>((size_t)K * 9);
    a.rot32 = rot32;
    a.tile_counter = c.take<int32_t>(kMaxWorkQueues);
    a.orient_score = c.take<float>((size_t)L * K);
    a.orient_tau = c.take<int32_t>((size_t)L * K);
    a.orient_theta = c.take<uint8_t>((size_t)R * K);
    const size_t slot_bytes = (size_t)a.slot_floats * sizeof(float);
    if (c.used + slot_bytes > kScratchBytes)
        return rt::fail(EXS_EINVAL,
                        "batch needs %zu B of per-orientation results and %zu B per workgroup of "
                        "pose scratch; the no-allocation buffer holds %zu B (split the batch)",
                        c.used, slot_bytes, kScratchBytes);
    const int64_t fit = (int64_t)((kScratchBytes - c.used) / slot_bytes);
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)pl.resident,
                                                                    (int64_t)a.n_tiles, fit}));
    a.scratch = c.take<float>((size_t)blocks * a.slot_floats);
    a.best_score = best_score;
    a.best_k = best_orient;
    a.best_tau = best_tau;
    a.best_theta = best_theta;
    a.best_coords = best_coords;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t e = launch_orientation_table((int)K, rot32, nullptr, st);
    if (e == hipSuccess) e = launch_zero_ints(a.tile_counter, kMaxWorkQueues, st);
    if (e == hipSuccess) e = launch_dock(a, pl.storage, pl.ppl, blocks, pl.threads, pl.lds, st);
    if (e != hipSuccess) return rt::fail(EXS_EDEVICE, "no-allocation launch: %s", hipGetErrorString(e));
    return EXS_OK;
}
