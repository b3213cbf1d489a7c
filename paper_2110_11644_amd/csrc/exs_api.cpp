// C ABI of libexs: pocket registry, ligand-batch upload, dock jobs.
//
// Host work is limited to validation, topology packing at upload time and
// launch bookkeeping; every step of the search itself runs in the HIP kernels
// (dock_kernels.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "exs.h"
#include "exs_internal.h"
#include "exs_pack.h"
#include "exs_runtime.h"

using namespace exs;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(e_ == hipErrorOutOfMemory ? EXS_ENOMEM : EXS_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

// ---- per-device state -------------------------------------------------------------------------

struct DeviceState {
    bool ready = false;
    int cus = 0;
    std::map<int, std::pair<float*, double*>> orient_tables;   // K -> (FP32, FP64) [K][9]
};

std::mutex g_dev_mu;
std::unordered_map<int, DeviceState> g_dev;

int current_device(int* dev) {
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return fail(EXS_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    return EXS_OK;
}

int ensure_device(int dev) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceState& d = g_dev[dev];
    if (d.ready) return EXS_OK;
    HIP_TRY(upload_trig_tables());
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    d.cus = prop.multiProcessorCount;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    d.ready = true;
    return EXS_OK;
}

// Fibonacci-sphere orientation tables of K orientations, built once per (device, K) by
// orientation_table_kernel (the no-allocation entry point builds the same table on the device).
int orientation_tables(int dev, int K, const float** r32, const double** r64) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    DeviceState& d = g_dev[dev];
    auto it = d.orient_tables.find(K);
    if (it == d.orient_tables.end()) {
        float* d32 = nullptr;
        double* d64 = nullptr;
        HIP_TRY(hipMalloc(&d32, (size_t)K * 9 * sizeof(float)));
        HIP_TRY(hipMalloc(&d64, (size_t)K * 9 * sizeof(double)));
        HIP_TRY(launch_orientation_table(K, d32, d64, nullptr));
        HIP_TRY(hipStreamSynchronize(nullptr));
        it = d.orient_tables.emplace(K, std::make_pair(d32, d64)).first;
    }
    *r32 = it->second.first;
    *r64 = it->second.second;
    return EXS_OK;
}

// A finite FP32 texel that rounds (to nearest even) to infinity in 16-bit storage: FP16 from
// 65520 (halfway between 65504 and 65536, a tie that rounds to the even 65536 = inf), BF16
// from 0x7f7f8000 (halfway past the largest finite BF16, likewise).
bool overflows_storage(float v, int storage) {
    const uint32_t a = __builtin_bit_cast(uint32_t, v) & 0x7fffffffu;
    if (storage == EXS_F16) return a >= __builtin_bit_cast(uint32_t, 65520.0f);
    if (storage == EXS_BF16) return a >= 0x7f7f8000u;
    return false;
}

// ---- registries --------------------------------------------------------------------------------

struct Pocket {
    int device = 0;
    int nx = 0, ny = 0, nz = 0, channels = 0, storage = EXS_F32;
    double h = 0, origin[3] = {0, 0, 0};
    float* master = nullptr;     // FP32 texels
    void* tex = nullptr;         // per-cell gather layout (8 corners per cell)
    GridDesc desc;
    std::atomic<int> users{0};
};

// A reusable execution plan of one (batch, settings) pair: device buffers that
// outlive jobs and the launch sequence captured once in a hipGraph.
struct Plan {
    std::vector<void*> bufs;
    DockArgs args{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::atomic<bool> busy{false};
};

struct Batch {
    int device = 0;
    int L = 0, A = 0, R = 0, n_max = 1;
    std::vector<int32_t> pockets;          // pocket handle per table slot
    std::vector<int> storage_of_slot;
    std::vector<LigInfo> info;             // host copy
    std::vector<std::vector<int16_t>> mcount;   // moving-set sizes per ligand
    std::vector<int32_t> rot_base;
    LigInfo* d_info = nullptr;
    float4* d_ref = nullptr;
    double* d_ref64 = nullptr;
    uint4* d_excl = nullptr;
    uint32_t* d_rot_uv = nullptr;
    uint4* d_rot_mask = nullptr;
    GridDesc* d_grids = nullptr;
    int32_t* d_upload_order = nullptr;   // pocket by pocket, longest first (no-allocation launches)
    uint32_t* d_rot_ac = nullptr;        // [R] dihedral neighbours a | c << 16 of each rotatable bond
    void* d_block = nullptr;             // the one allocation the arrays above are carved from
    std::mutex order_mu;
    std::map<std::vector<int>, int32_t*> d_orders;   // (S, P, T, persistent, K) -> order array
    std::map<std::vector<int>, std::vector<int>> group_sizes;
    std::map<std::vector<int>, int> queue_counts;   // persistent orders: work queues
    std::map<std::vector<int64_t>, std::shared_ptr<Plan>> plans;   // graph plans by settings
};

struct Job {
    int device = 0;
    std::shared_ptr<Batch> batch;
    exs_search_params prm{};
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t ev_dock = nullptr, ev_rank = nullptr;   // eager ranked jobs: after the search, after the ranking
    int L = 0, A = 0, R = 0, K = 0, top_k = 0;
    std::vector<void*> bufs;    // stream-ordered allocations (eager jobs)
    std::shared_ptr<Plan> plan; // graph jobs: buffers belong to the plan
    DockArgs args{};
};

std::mutex g_reg_mu;
int32_t g_next_pocket = 1;
int64_t g_next_batch = 1, g_next_job = 1;
std::unordered_map<int32_t, std::shared_ptr<Pocket>> g_pockets;
std::unordered_map<int64_t, std::shared_ptr<Batch>> g_batches;
std::unordered_map<int64_t, std::shared_ptr<Job>> g_jobs;

std::shared_ptr<Pocket> find_pocket(int32_t id) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_pockets.find(id);
    return it == g_pockets.end() ? nullptr : it->second;
}
std::shared_ptr<Batch> find_batch(int64_t id) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_batches.find(id);
    return it == g_batches.end() ? nullptr : it->second;
}
std::shared_ptr<Job> find_job(int64_t id) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_jobs.find(id);
    return it == g_jobs.end() ? nullptr : it->second;
}

void free_batch(Batch* b) {
    if (b->d_block) (void)hipFree(b->d_block);
    b->d_block = nullptr;
    for (auto& kv : b->d_orders) (void)hipFree(kv.second);
    b->d_orders.clear();
    for (auto& kv : b->plans) {
        Plan& pl = *kv.second;
        if (pl.exec) (void)hipGraphExecDestroy(pl.exec);
        if (pl.graph) (void)hipGraphDestroy(pl.graph);
        for (void* q : pl.bufs) (void)hipFree(q);
    }
    b->plans.clear();
}

}  // namespace

namespace exs {
namespace rt {

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
int current_device(int* dev) { return ::current_device(dev); }
int ensure_device(int dev) { return ::ensure_device(dev); }
int orientation_tables(int dev, int K, const float** r32, const double** r64) {
    return ::orientation_tables(dev, K, r32, r64);
}
int device_cus(int dev) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    return g_dev[dev].cus;
}
bool pocket_info(int32_t id, PocketInfo* out) {
    auto p = find_pocket(id);
    if (!p) return false;
    out->device = p->device;
    out->channels = p->channels;
    out->storage = p->storage;
    out->desc = p->desc;
    return true;
}
void pocket_use(int32_t id, int delta) {
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_pockets.find(id);
    if (it != g_pockets.end()) it->second->users += delta;
}

}  // namespace rt
}  // namespace exs

// ---- C ABI -------------------------------------------------------------------------------------

extern "C" {

const char* exs_version(void) { return "exs 0.1 (gfx950)"; }

const char* exs_last_error(void) { return g_last_error.c_str(); }

int exs_load_pocket_grid(const float* values, int nx, int ny, int nz, int channels,
                         double spacing_A, const double origin_A[3], int storage,
                         int values_on_device, void* stream, int32_t* pocket_id_out) {
    try {
        if (!values || !origin_A || !pocket_id_out) return fail(EXS_EINVAL, "null argument");
        if (nx < 2 || ny < 2 || nz < 2) return fail(EXS_EINVAL, "grid %dx%dx%d: each edge must be >= 2", nx, ny, nz);
        if (channels < 1 || channels > EXS_MAX_CHANNELS)
            return fail(EXS_EINVAL, "channels %d outside [1, %d]", channels, EXS_MAX_CHANNELS);
        if (!(spacing_A > 0.0) || !isfinite(spacing_A)) return fail(EXS_EINVAL, "spacing must be > 0");
        if (storage != EXS_F32 && storage != EXS_BF16 && storage != EXS_F16)
            return fail(EXS_EINVAL, "unknown storage %d", storage);
        if ((int64_t)nx * ny >= (int64_t)1 << 23 || nz >= 1 << 23)
            return fail(EXS_EINVAL, "grid %dx%dx%d: nx*ny and nz must be below 2^23 (cell offsets use 24-bit multiplies)",
                        nx, ny, nz);
        const int64_t chan = (int64_t)nx * ny * nz;
        const int64_t tex_chan_bytes = expanded_entries(nx, ny, nz, storage) * 16;
        if (tex_chan_bytes > INT32_MAX)
            return fail(EXS_EINVAL, "a grid channel must expand to < 2 GiB (32 B per FP32 cell, 16 B per 16-bit cell)");
        const int64_t count = chan * channels;
        if (!values_on_device) {
            for (int64_t i = 0; i < count; ++i) {
                if (!isfinite(values[i])) return fail(EXS_EINVAL, "texel %lld is not finite", (long long)i);
                if (overflows_storage(values[i], storage))
                    return fail(EXS_EINVAL, "texel %lld (%g) overflows %s storage", (long long)i,
                                (double)values[i], storage == EXS_F16 ? "FP16" : "BF16");
            }
        }
        int dev;
        if (int rc = current_device(&dev)) return rc;
        if (int rc = ensure_device(dev)) return rc;
        hipStream_t st = (hipStream_t)stream;
        auto p = std::make_shared<Pocket>();
        p->device = dev; p->nx = nx; p->ny = ny; p->nz = nz; p->channels = channels;
        p->storage = storage; p->h = spacing_A;
        for (int a = 0; a < 3; ++a) p->origin[a] = origin_A[a];
        struct FreeOnFail {     // device buffers of a pocket whose load fails part way
            Pocket* p;
            bool armed = true;
            ~FreeOnFail() {
                if (!armed) return;
                if (p->master) (void)hipFree(p->master);
                if (p->tex) (void)hipFree(p->tex);
            }
        } guard{p.get()};
        HIP_TRY(hipMalloc(&p->master, (size_t)count * sizeof(float)));
        HIP_TRY(hipMemcpyAsync(p->master, values, (size_t)count * sizeof(float),
                               values_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
        HIP_TRY(hipMalloc(&p->tex, (size_t)tex_chan_bytes * channels));
        if (values_on_device) {   // the same checks on the device copy
            int* flag = nullptr;
            HIP_TRY(hipMallocAsync(&flag, sizeof(int), st));
            int bad = 0;
            hipError_t e = launch_zero_ints(flag, 1, st);
            if (e == hipSuccess) e = launch_check_texels(p->master, count, storage, flag, st);
            if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            (void)hipFreeAsync(flag, st);
            if (e != hipSuccess) return fail(EXS_EDEVICE, "texel check: %s", hipGetErrorString(e));
            if (bad & 1) return fail(EXS_EINVAL, "a texel is not finite");
            if (bad & 2)
                return fail(EXS_EINVAL, "a texel overflows %s storage", storage == EXS_F16 ? "FP16" : "BF16");
        }
        HIP_TRY(launch_expand_grid(p->master, p->tex, nx, ny, nz, channels, storage, st));
        HIP_TRY(hipStreamSynchronize(st));
        GridDesc& g = p->desc;
        memset(&g, 0, sizeof g);
        g.tex = p->tex;
        g.master = p->master;
        g.nx = nx; g.ny = ny; g.nz = nz; g.channels = channels;
        g.ox = (float)origin_A[0]; g.oy = (float)origin_A[1]; g.oz = (float)origin_A[2];
        g.inv_h = (float)(1.0 / spacing_A);
        g.h = spacing_A; g.dox = origin_A[0]; g.doy = origin_A[1]; g.doz = origin_A[2];
        g.dcx = origin_A[0] + spacing_A * (nx - 1) / 2.0;
        g.dcy = origin_A[1] + spacing_A * (ny - 1) / 2.0;
        g.dcz = origin_A[2] + spacing_A * (nz - 1) / 2.0;
        g.cx = (float)g.dcx; g.cy = (float)g.dcy; g.cz = (float)g.dcz;
        g.ux_hi = nextafterf((float)(nx - 1), 0.0f);
        g.uy_hi = nextafterf((float)(ny - 1), 0.0f);
        g.uz_hi = nextafterf((float)(nz - 1), 0.0f);
        g.chan_bytes = (int32_t)tex_chan_bytes;
        g.master_chan_bytes = (int32_t)(chan * 4);
        g.storage = storage;
        std::lock_guard<std::mutex> lk(g_reg_mu);
        int32_t id = g_next_pocket++;
        g_pockets[id] = p;
        guard.armed = false;
        *pocket_id_out = id;
        return EXS_OK;
    } catch (const std::exception& e) {
        return fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_unload_pocket(int32_t pocket_id) {
    std::shared_ptr<Pocket> p;
    {
        std::lock_guard<std::mutex> lk(g_reg_mu);
        auto it = g_pockets.find(pocket_id);
        if (it == g_pockets.end()) return fail(EXS_ENOENT, "unknown pocket %d", pocket_id);
        if (it->second->users.load() > 0)
            return fail(EXS_EINVAL, "pocket %d is used by %d uploaded batch(es)", pocket_id,
                        it->second->users.load());
        p = it->second;
        g_pockets.erase(it);
    }
    (void)hipDeviceSynchronize();
    if (p->master) (void)hipFree(p->master);
    if (p->tex) (void)hipFree(p->tex);
    return EXS_OK;
}

int exs_upload_ligands(const exs_ligand_batch* in, void* stream, int64_t* batch_out) {
    try {
        if (!in || !batch_out) return fail(EXS_EINVAL, "null argument");
        const int L = in->n_ligands;
        if (L < 0) return fail(EXS_EINVAL, "negative ligand count");
        if (L > 0 && (!in->atom_offset || !in->x || !in->y || !in->z || !in->type ||
                      !in->bond_offset || !in->rot_offset || !in->pocket_id))
            return fail(EXS_EINVAL, "null array in ligand batch");
        int dev;
        if (int rc = current_device(&dev)) return rc;
        if (int rc = ensure_device(dev)) return rc;
        auto b = std::make_shared<Batch>();
        b->device = dev;
        b->L = L;
        // pockets of the batch
        std::map<int32_t, int> slot_of;
        std::vector<std::shared_ptr<Pocket>> pk;
        std::vector<int> lig_slot(L);
        for (int l = 0; l < L; ++l) {
            int32_t id = in->pocket_id[l];
            auto it = slot_of.find(id);
            if (it == slot_of.end()) {
                auto p = find_pocket(id);
                if (!p) return fail(EXS_EINVAL, "ligand %d: unknown pocket %d", l, id);
                if (p->device != dev) return fail(EXS_EINVAL, "ligand %d: pocket %d lives on device %d", l, id, p->device);
                it = slot_of.emplace(id, (int)pk.size()).first;
                pk.push_back(p);
            }
            lig_slot[l] = it->second;
        }
        if (L > 0 && in->atom_offset[0] != 0) return fail(EXS_EINVAL, "atom_offset[0] must be 0");
        if (L > 0 && (in->bond_offset[0] != 0 || in->rot_offset[0] != 0))
            return fail(EXS_EINVAL, "bond_offset[0] and rot_offset[0] must be 0");
        for (int l = 0; l < L; ++l)
            if (in->atom_offset[l + 1] < in->atom_offset[l] || in->bond_offset[l + 1] < in->bond_offset[l] ||
                in->rot_offset[l + 1] < in->rot_offset[l])
                return fail(EXS_EINVAL, "ligand %d: offsets decrease", l);
        const int A = L ? in->atom_offset[L] : 0;
        const int R = L ? in->rot_offset[L] : 0;
        if (L > 0 && in->bond_offset[L] > 0 && !in->bond_ij) return fail(EXS_EINVAL, "null bond_ij");
        if (R > 0 && !in->rot_bond) return fail(EXS_EINVAL, "null rot_bond");
        b->A = A; b->R = R;
        // The device arrays live in one allocation, filled by one copy from a host block of the
        // same layout (regions 256-byte aligned): order [L + kMaxWorkQueues + 1], info [L],
        // ref [A], ref64 [3A], excl [A], rot_uv [R], rot_ac [R], rot_mask [R], grids [slots].
        size_t off = 0;
        auto region = [&off](size_t bytes) {
            const size_t at = off;
            off += (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
            return at;
        };
        const size_t o_order = region(sizeof(int32_t) * ((size_t)L + kMaxWorkQueues + 1));
        const size_t o_info = region(sizeof(LigInfo) * (size_t)L);
        const size_t o_ref = region(sizeof(float4) * (size_t)A);
        const size_t o_ref64 = region(sizeof(double) * 3 * (size_t)A);
        const size_t o_excl = region(sizeof(uint4) * (size_t)A);
        const size_t o_ruv = region(sizeof(uint32_t) * (size_t)R);
        const size_t o_rac = region(sizeof(uint32_t) * (size_t)R);
        const size_t o_rmask = region(sizeof(uint4) * (size_t)R);
        const size_t o_grids = region(sizeof(GridDesc) * pk.size());
        const size_t total = off;
        std::unique_ptr<unsigned char[]> host(new unsigned char[total]);   // every byte read is written
        unsigned char* hb = host.get();
        LigInfo* h_info = reinterpret_cast<LigInfo*>(hb + o_info);
        float4* ref = reinterpret_cast<float4*>(hb + o_ref);
        double* ref64 = reinterpret_cast<double*>(hb + o_ref64);
        uint4* excl = reinterpret_cast<uint4*>(hb + o_excl);
        uint32_t* ruv = reinterpret_cast<uint32_t*>(hb + o_ruv);
        uint32_t* rot_ac = reinterpret_cast<uint32_t*>(hb + o_rac);
        uint4* rmask = reinterpret_cast<uint4*>(hb + o_rmask);
        b->info.resize(L);
        b->mcount.resize(L);
        b->rot_base.resize(L);
        // validate, pack and flatten on host threads, each ligand into its own ranges
        std::vector<int> rc_of(L, EXS_OK);
        std::vector<std::string> err_of(L);
        std::vector<double> cost(L, 0.0);   // search cost at the full settings (the upload order)
        unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        if (L < 256) nth = 1;
        std::atomic<int> next{0};
        auto work = [&]() {
            PackedLigand p;   // reused across this thread's ligands (keeps its capacity)
            for (;;) {
                const int l = next.fetch_add(1);
                if (l >= L) break;
                try {   // an exception must not leave a worker thread (it would end the process)
                const int a0 = in->atom_offset[l], n = in->atom_offset[l + 1] - a0;
                const int b0 = in->bond_offset[l], nbl = in->bond_offset[l + 1] - b0;
                const int r0 = in->rot_offset[l], nr = in->rot_offset[l + 1] - r0;
                rc_of[l] = pack_ligand(n, in->bond_ij + 2 * (size_t)b0, nbl, in->rot_bond + r0, nr,
                                       in->type + a0, pk[lig_slot[l]]->channels, in->x + a0,
                                       in->y + a0, in->z + a0, &p, &err_of[l]);
                if (rc_of[l]) continue;
                LigInfo& inf = b->info[l];
                memset(&inf, 0, sizeof inf);
                inf.atom_base = a0; inf.rot_base = r0; inf.n = (int16_t)p.n; inf.nrot = (int16_t)p.nrot;
                inf.pocket = (int16_t)lig_slot[l];
                h_info[l] = inf;
                b->rot_base[l] = r0;
                for (int i = 0; i < p.n; ++i) {
                    const double dx = (double)in->x[a0 + i] - p.centroid[0];
                    const double dy = (double)in->y[a0 + i] - p.centroid[1];
                    const double dz = (double)in->z[a0 + i] - p.centroid[2];
                    const int t = in->type[a0 + i];
                    ref[a0 + i] = make_float4((float)dx, (float)dy, (float)dz, __builtin_bit_cast(float, t));
                    ref64[(size_t)(a0 + i) * 3 + 0] = dx;
                    ref64[(size_t)(a0 + i) * 3 + 1] = dy;
                    ref64[(size_t)(a0 + i) * 3 + 2] = dz;
                    excl[a0 + i] = p.excl[i].as_uint4();
                }
                b->mcount[l].resize(p.nrot);
                for (int r = 0; r < p.nrot; ++r) {
                    // lowest-index neighbours of u (other than v) and of v (other than u): the
                    // dihedral of the bond in the second-stage score
                    const int u = p.rot_u[r], v = p.rot_v[r];
                    int na = 0xffff, nc = 0xffff;
                    for (int e = 0; e < nbl; ++e) {
                        const int bi = in->bond_ij[2 * (size_t)(b0 + e)], bj = in->bond_ij[2 * (size_t)(b0 + e) + 1];
                        if (bi == u && bj != v) na = std::min(na, bj);
                        if (bj == u && bi != v) na = std::min(na, bi);
                        if (bi == v && bj != u) nc = std::min(nc, bj);
                        if (bj == v && bi != u) nc = std::min(nc, bi);
                    }
                    rot_ac[r0 + r] = (uint32_t)na | ((uint32_t)nc << 16);
                    ruv[r0 + r] = (uint32_t)p.rot_u[r] | ((uint32_t)p.rot_v[r] << 16);
                    rmask[r0 + r] = p.moving[r].as_uint4();
                    b->mcount[l][r] = (int16_t)p.moving[r].count();
                }
                cost[l] = ligand_cost(p.n, b->mcount[l].data(), p.nrot, 1, 32, 2, 27);
                } catch (const std::exception& ex) {
                    rc_of[l] = EXS_ENOMEM;
                    err_of[l] = std::string("exception: ") + ex.what();
                }
            }
        };
        {
            std::vector<std::thread> pool;
            try {
                for (unsigned t = 1; t < nth; ++t) pool.emplace_back(work);
            } catch (...) {   // fewer threads: the ones started and this one finish the work
            }
            work();
            for (auto& t : pool) t.join();
        }
        for (int l = 0; l < L; ++l)
            if (rc_of[l]) return fail(rc_of[l], "ligand %d: %s", l, err_of[l].c_str());
        for (int l = 0; l < L; ++l) b->n_max = std::max<int>(b->n_max, b->info[l].n);
        GridDesc* h_grids = reinterpret_cast<GridDesc*>(hb + o_grids);
        for (size_t sl = 0; sl < pk.size(); ++sl) {
            h_grids[sl] = pk[sl]->desc;
            b->storage_of_slot.push_back(pk[sl]->storage);
        }
        // one work queue, pocket by pocket and longest first within a pocket, by the cost at the
        // full search settings (the order of launches that cannot build one of their own)
        int32_t* up_order = reinterpret_cast<int32_t*>(hb + o_order);
        {
            std::vector<int> pocket(L);
            for (int l = 0; l < L; ++l) pocket[l] = b->info[l].pocket;
            work_queues(L, pocket.data(), cost.data(), 1, true, up_order, up_order + L);
        }
        hipStream_t st = (hipStream_t)stream;
        {
            hipError_t e = hipMalloc(&b->d_block, total);
            if (e != hipSuccess) {
                b->d_block = nullptr;
                (void)hipGetLastError();
                return fail(EXS_ENOMEM, "device allocation of %zu B for the ligand batch: %s", total,
                            hipGetErrorString(e));
            }
            unsigned char* d = static_cast<unsigned char*>(b->d_block);
            b->d_upload_order = reinterpret_cast<int32_t*>(d + o_order);
            b->d_info = reinterpret_cast<LigInfo*>(d + o_info);
            b->d_ref = reinterpret_cast<float4*>(d + o_ref);
            b->d_ref64 = reinterpret_cast<double*>(d + o_ref64);
            b->d_excl = reinterpret_cast<uint4*>(d + o_excl);
            b->d_rot_uv = reinterpret_cast<uint32_t*>(d + o_ruv);
            b->d_rot_ac = reinterpret_cast<uint32_t*>(d + o_rac);
            b->d_rot_mask = reinterpret_cast<uint4*>(d + o_rmask);
            b->d_grids = reinterpret_cast<GridDesc*>(d + o_grids);
            // one copy of the whole block (the padding between regions is zeroed first)
            const std::pair<size_t, size_t> used[] = {
                {o_order, sizeof(int32_t) * ((size_t)L + kMaxWorkQueues + 1)},
                {o_info, sizeof(LigInfo) * (size_t)L}, {o_ref, sizeof(float4) * (size_t)A},
                {o_ref64, sizeof(double) * 3 * (size_t)A}, {o_excl, sizeof(uint4) * (size_t)A},
                {o_ruv, sizeof(uint32_t) * (size_t)R}, {o_rac, sizeof(uint32_t) * (size_t)R},
                {o_rmask, sizeof(uint4) * (size_t)R}, {o_grids, sizeof(GridDesc) * pk.size()}};
            for (size_t i = 0; i < sizeof used / sizeof used[0]; ++i) {
                const size_t end = used[i].first + used[i].second;
                const size_t next_at = i + 1 < sizeof used / sizeof used[0] ? used[i + 1].first : total;
                memset(hb + end, 0, next_at - end);
            }
            e = hipMemcpyAsync(d, hb, total, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) {
                free_batch(b.get());
                return fail(EXS_EDEVICE, "upload: %s", hipGetErrorString(e));
            }
        }
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            free_batch(b.get());
            return fail(EXS_EDEVICE, "upload: %s", hipGetErrorString(e));
        }
        for (auto& p : pk) { p->users++; b->pockets.push_back(0); }
        for (auto& kv : slot_of) b->pockets[kv.second] = kv.first;
        std::lock_guard<std::mutex> lk(g_reg_mu);
        int64_t id = g_next_batch++;
        g_batches[id] = b;
        *batch_out = id;
        return EXS_OK;
    } catch (const std::exception& e) {
        return fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_pack_topology(int n, const float* x, const float* y, const float* z, const uint8_t* type,
                      int channels, int nb, const int32_t* bond_ij, int nrot,
                      const int32_t* rot_bond, uint32_t* excl, int32_t* rot_uv, uint32_t* moving) {
    try {
        if (!x || !y || !z || !type || (nb > 0 && !bond_ij) || (nrot > 0 && !rot_bond))
            return fail(EXS_EINVAL, "null argument");
        PackedLigand p;
        std::string err;
        int rc = pack_ligand(n, bond_ij, nb, rot_bond, nrot, type, channels, x, y, z, &p, &err);
        if (rc) return fail(rc, "%s", err.c_str());
        for (int i = 0; excl && i < n; ++i) {
            uint4 w = p.excl[i].as_uint4();
            excl[4 * i] = w.x; excl[4 * i + 1] = w.y; excl[4 * i + 2] = w.z; excl[4 * i + 3] = w.w;
        }
        for (int b = 0; b < nrot; ++b) {
            if (rot_uv) { rot_uv[2 * b] = p.rot_u[b]; rot_uv[2 * b + 1] = p.rot_v[b]; }
            if (moving) {
                uint4 w = p.moving[b].as_uint4();
                moving[4 * b] = w.x; moving[4 * b + 1] = w.y; moving[4 * b + 2] = w.z; moving[4 * b + 3] = w.w;
            }
        }
        return EXS_OK;
    } catch (const std::exception& e) {
        return fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_release_ligands(int64_t batch) {
    std::shared_ptr<Batch> b;
    {
        std::lock_guard<std::mutex> lk(g_reg_mu);
        auto it = g_batches.find(batch);
        if (it == g_batches.end()) return fail(EXS_ENOENT, "unknown batch %lld", (long long)batch);
        for (auto& kv : g_jobs)
            if (kv.second->batch == it->second)
                return fail(EXS_EINVAL, "batch %lld still has job %lld", (long long)batch, (long long)kv.first);
        b = it->second;
        g_batches.erase(it);
        for (int32_t id : b->pockets) {
            auto p = g_pockets.find(id);
            if (p != g_pockets.end()) p->second->users--;
        }
    }
    free_batch(b.get());
    return EXS_OK;
}

}  // extern "C"

namespace {

// Processing order.  Per-pocket launches: grouped by pocket, longest first in each group.
// Persistent launch: work queues laid out by queue_plan (spread or pocket-major); the device
// array holds the order followed by the queue bounds (kMaxWorkQueues + 1 entries reserved) and
// *n_queues receives their count.
int batch_order(Batch& b, int K, int S, int P, int T, int persistent, hipStream_t st,
                int32_t** d_order, std::vector<int>* groups, int* n_queues) {
    std::vector<int> key = {K, S, P, T, persistent};
    std::lock_guard<std::mutex> lk(b.order_mu);
    auto it = b.d_orders.find(key);
    if (it != b.d_orders.end()) {
        *d_order = it->second;
        *groups = b.group_sizes[key];
        *n_queues = b.queue_counts[key];
        return EXS_OK;
    }
    std::vector<double> cost(b.L);
    for (int l = 0; l < b.L; ++l) {
        cost[l] = ligand_cost(b.info[l].n, b.mcount[l].data(), b.info[l].nrot, K, S, P, T);
        b.info[l].cost = (float)cost[l];
    }
    std::vector<int> ord(b.L);
    std::iota(ord.begin(), ord.end(), 0);
    const int n_slots = (int)b.pockets.size();
    if (persistent) {
        std::vector<int> pocket(b.L);
        for (int l = 0; l < b.L; ++l) pocket[l] = b.info[l].pocket;
        int used = 0;
        std::vector<int> seen(n_slots, 0);
        for (int p : pocket) used += seen[p]++ == 0 ? 1 : 0;
        const QueuePlan plan = queue_plan(b.L, used, (K + kWave - 1) / kWave);
        ord.resize(b.L + kMaxWorkQueues + 1);
        work_queues(b.L, pocket.data(), cost.data(), plan.n_queues, plan.pocket_major, ord.data(),
                    ord.data() + b.L);
        groups->assign(1, b.L);
        *n_queues = plan.n_queues;
    } else {
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int c) {
            if (b.info[a].pocket != b.info[c].pocket) return b.info[a].pocket < b.info[c].pocket;
            return cost[a] > cost[c];
        });
        groups->assign(n_slots, 0);
        for (int l = 0; l < b.L; ++l) (*groups)[b.info[l].pocket]++;
    }
    int32_t* d = nullptr;
    HIP_TRY(hipMalloc(&d, std::max<size_t>(1, ord.size()) * sizeof(int32_t)));
    if (!ord.empty()) {
        HIP_TRY(hipMemcpyAsync(d, ord.data(), ord.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    b.d_orders[key] = d;
    b.group_sizes[key] = *groups;
    b.queue_counts[key] = *n_queues;
    *d_order = d;
    return EXS_OK;
}

// Device buffers of a job: stream-ordered per job (eager), or plain and owned by
// a graph plan (kept across jobs).
struct Alloc {
    std::vector<void*>* bufs;
    hipStream_t stream;
    bool stream_ordered;
};

template <class T>
int job_alloc(Alloc& al, T** p, size_t count) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    void* q = nullptr;
    if (al.stream_ordered) HIP_TRY(hipMallocAsync(&q, bytes, al.stream));
    else HIP_TRY(hipMalloc(&q, bytes));
    al.bufs->push_back(q);
    *p = (T*)q;
    return EXS_OK;
}

void free_allocs(Alloc& al) {
    for (void* p : *al.bufs) {
        if (al.stream_ordered) (void)hipFreeAsync(p, al.stream);
        else (void)hipFree(p);
    }
    al.bufs->clear();
}

void job_free(Job& j) {
    for (void* p : j.bufs) (void)hipFreeAsync(p, j.stream);
    j.bufs.clear();
    if (j.plan) { j.plan->busy = false; j.plan.reset(); }
    if (j.ev0) (void)hipEventDestroy(j.ev0);
    if (j.ev1) (void)hipEventDestroy(j.ev1);
    if (j.ev_dock) (void)hipEventDestroy(j.ev_dock);
    if (j.ev_rank) (void)hipEventDestroy(j.ev_rank);
    j.ev0 = j.ev1 = j.ev_dock = j.ev_rank = nullptr;
}

}  // namespace

namespace {

int job_wait(Job& j, int wait) {
    if (!wait) {
        hipError_t e = hipEventQuery(j.ev1);
        if (e == hipErrorNotReady) return fail(EXS_ENOTREADY, "job still running");
        if (e != hipSuccess) return fail(EXS_EDEVICE, "job: %s", hipGetErrorString(e));
        return EXS_OK;
    }
    HIP_TRY(hipEventSynchronize(j.ev1));
    return EXS_OK;
}

template <class T>
int copy_out(T* dst, const T* src, size_t count) {
    if (!dst || !count) return EXS_OK;
    HIP_TRY(hipMemcpy(dst, src, count * sizeof(T), hipMemcpyDeviceToHost));
    return EXS_OK;
}

void fill_desc(exs_pose_desc& d, float score, double s64, int k, int32_t tau_packed,
                      int nrot, const uint8_t* theta, size_t theta_stride) {
    memset(&d, 0, sizeof d);
    d.score = score;
    d.score_fp64 = s64;
    d.orient = k;
    d.tau[0] = (int8_t)(tau_packed & 0xff);
    d.tau[1] = (int8_t)((tau_packed >> 8) & 0xff);
    d.tau[2] = (int8_t)((tau_packed >> 16) & 0xff);
    d.n_rot = (uint8_t)nrot;
    for (int b = 0; b < nrot; ++b) d.theta[b] = theta[(size_t)b * theta_stride];
}

}  // namespace

namespace {

// The launch sequence of one job on `st`: a counter reset and one persistent dock
// launch, or one dock launch per pocket group.
// ev_dock / ev_rank (may be null): recorded on `st` after the search and after the ranking, so
// that an eager job can report each kernel's time (never inside a graph capture).
hipError_t enqueue_dock(const DockArgs& base, const Batch& b, const std::vector<int>& groups,
                        const int32_t* d_order, int n_queues, int storage, int ppl, bool persistent,
                        int resident, int threads, size_t lds, hipStream_t st,
                        hipEvent_t ev_dock = nullptr, hipEvent_t ev_rank = nullptr) {
    if (b.L == 0) return hipSuccess;
    if (persistent) {
        DockArgs a = base;
        a.order = d_order;
        a.n_order = b.L;
        a.n_tiles = (b.L + a.lpw - 1) / a.lpw;
        a.persistent = 1;
        a.queue_bounds = d_order + b.L;
        a.n_queues = n_queues;
        hipError_t e = launch_zero_ints(a.tile_counter, n_queues, st);
        if (e != hipSuccess) return e;
        e = launch_dock(a, storage, ppl, resident, threads, lds, st);
        if (e == hipSuccess && ev_dock) e = hipEventRecord(ev_dock, st);
        if (e == hipSuccess && a.rank_keep > 0) e = launch_rank(a, b.L, d_order, st);
        if (e == hipSuccess && ev_rank) e = hipEventRecord(ev_rank, st);
        if (e == hipSuccess && a.rescore2) e = launch_rescore2(a, b.L, d_order, st);
        return e;
    }
    int start = 0;
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const int gsz = groups[gi];
        if (gsz == 0) continue;
        DockArgs a = base;
        a.order = d_order + start;
        a.n_order = gsz;
        a.n_tiles = (gsz + a.lpw - 1) / a.lpw;
        a.persistent = 0;
        hipError_t e = launch_dock(a, b.storage_of_slot[gi], ppl, a.n_tiles, threads, lds, st);
        if (e != hipSuccess) return e;
        start += gsz;
    }
    hipError_t e = ev_dock ? hipEventRecord(ev_dock, st) : hipSuccess;
    // d_order: every pocket's ligands, longest first, one pocket after another
    if (e == hipSuccess && base.rank_keep > 0) e = launch_rank(base, b.L, d_order, st);
    if (e == hipSuccess && ev_rank) e = hipEventRecord(ev_rank, st);
    if (e == hipSuccess && base.rescore2) e = launch_rescore2(base, b.L, d_order, st);
    return e;
}

// Validated search settings of a batch and the launch shape they give.
struct LaunchShape {
    int ppl = 1, wpl = 1, lpw = 1, threads = 64, top_k = 0, storage = 0;
    size_t lds = 0;
    const void* fn = nullptr;
};

int launch_shape(const Batch& b, const exs_search_params& p, bool persistent, LaunchShape* out) {
    if (p.n_orient < 1 || p.n_orient > EXS_MAX_ORIENT)
        return fail(EXS_EINVAL, "n_orient %d outside [1, %d]", p.n_orient, EXS_MAX_ORIENT);
    if (p.torsion_steps != 8 && p.torsion_steps != 16 && p.torsion_steps != 32)
        return fail(EXS_EINVAL, "torsion_steps %d: supported 8, 16, 32", p.torsion_steps);
    if (p.passes < 0 || p.passes > 64) return fail(EXS_EINVAL, "passes %d outside [0, 64]", p.passes);
    if (p.n_offsets != 1 && p.n_offsets != 27) return fail(EXS_EINVAL, "n_offsets must be 1 or 27");
    if (!(p.offset_step_A >= 0.0f) || !(p.clash_cutoff_A >= 0.0f) || !isfinite(p.clash_penalty) ||
        !isfinite(p.offset_step_A) || !isfinite(p.clash_cutoff_A))
        return fail(EXS_EINVAL, "offset step, clash cutoff and penalty must be finite, >= 0");
    if (p.top_k < 0 || p.top_k > EXS_MAX_TOPK) return fail(EXS_EINVAL, "top_k %d outside [0, %d]", p.top_k, EXS_MAX_TOPK);
    if (p.n_offsets == 27 && p.passes > 127) return fail(EXS_EINVAL, "too many passes for offsets");
    if (p.rank_keep < 0 || p.rank_keep > p.n_orient)
        return fail(EXS_EINVAL, "rank_keep %d outside [0, n_orient]", p.rank_keep);
    if (p.rank_keep > 0 && (!(p.cluster_rmsd_A >= 0.0f) || !isfinite(p.cluster_rmsd_A)))
        return fail(EXS_EINVAL, "cluster_rmsd_A must be finite and >= 0");
    if ((p.flags & EXS_FLAG_RESCORE2) && p.rank_keep <= 0)
        return fail(EXS_EINVAL, "EXS_FLAG_RESCORE2 rescores the ranked poses: it needs rank_keep > 0");
    LaunchShape& sh = *out;
    sh.ppl = p.poses_per_lane ? p.poses_per_lane : 1;
    if (sh.ppl != 1 && sh.ppl != 2 && sh.ppl != 4)
        return fail(EXS_EINVAL, "poses_per_lane %d: supported 1, 2, 4", sh.ppl);
    const int K = p.n_orient;
    sh.wpl = (K + kWave * sh.ppl - 1) / (kWave * sh.ppl);
    sh.lpw = p.ligands_per_wg;
    if (sh.lpw == 0) sh.lpw = std::max(1, std::min(kMaxLpw, kMaxWavesPerWg / std::max(1, sh.wpl) / 2));
    if (sh.lpw != 1 && sh.lpw != 2 && sh.lpw != 4 && sh.lpw != 8)
        return fail(EXS_EINVAL, "ligands_per_wg %d: supported 1, 2, 4, 8", sh.lpw);
    sh.top_k = std::min(p.top_k, K);
    const int waves = dock_waves(sh.lpw, sh.wpl, sh.top_k, sh.ppl, p.torsion_steps);
    if (waves < 1)
        return fail(EXS_EINVAL, "tile of %d ligands x %d poses per lane does not fit in %zu B of LDS",
                    sh.lpw, sh.ppl, kMaxLdsBytes);
    sh.threads = waves * kWave;
    int storage = -1;
    for (size_t s = 0; s < b.pockets.size(); ++s) {
        auto pk = find_pocket(b.pockets[s]);
        if (!pk) return fail(EXS_ENOENT, "pocket %d of the batch was unloaded", b.pockets[s]);
        if (storage >= 0 && pk->storage != storage && persistent)
            return fail(EXS_EINVAL, "persistent launch needs one texel storage for all pockets");
        storage = storage < 0 ? pk->storage : storage;
    }
    sh.storage = storage < 0 ? 0 : storage;
    sh.lds = dock_lds_bytes(sh.lpw, sh.top_k, waves, sh.ppl, p.torsion_steps);
    sh.fn = dock_kernel_fn(sh.storage, p.torsion_steps, sh.ppl);
    if (!sh.fn) return fail(EXS_EINVAL, "no kernel for this configuration");
    if (sh.lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(sh.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
        if (e != hipSuccess) return fail(EXS_EDEVICE, "LDS %zu: %s", sh.lds, hipGetErrorString(e));
    }
    return EXS_OK;
}

// Launch arguments of batch b under settings p (batch, pocket and search fields); outputs,
// scratch and the processing order are left null.
void base_args(DockArgs& a, const Batch& b, const exs_search_params& p, const LaunchShape& sh,
               const float* r32, const double* r64) {
    memset(&a, 0, sizeof a);
    a.info = b.d_info; a.ref = b.d_ref; a.ref64 = b.d_ref64; a.excl = b.d_excl;
    a.rot_uv = b.d_rot_uv; a.rot_mask = b.d_rot_mask; a.grids = b.d_grids;
    a.rot32 = r32; a.rot64 = r64;
    a.K = p.n_orient; a.S = p.torsion_steps; a.P = p.passes; a.T = p.n_offsets;
    a.step = p.offset_step_A; a.cut2 = p.clash_cutoff_A * p.clash_cutoff_A; a.pen = p.clash_penalty;
    a.step64 = (double)p.offset_step_A;
    a.cut2_64 = (double)p.clash_cutoff_A * (double)p.clash_cutoff_A;
    a.pen64 = (double)p.clash_penalty;
    a.top_k = sh.top_k; a.lpw = sh.lpw; a.wpl = sh.wpl; a.kp = sh.wpl * kWave * sh.ppl;
    a.rank_keep = p.rank_keep;
    a.rank_thr2 = p.cluster_rmsd_A * p.cluster_rmsd_A;
    a.n_max = b.n_max;
    a.slot_floats = (int64_t)sh.lpw * a.n_max * 3 * a.kp;
    a.rescore2 = (p.flags & EXS_FLAG_RESCORE2) ? 1 : 0;
    a.rot_ac = b.d_rot_ac;
    a.eps2 = EXS_RESCORE2_CONTACT_EPS;
    a.w2 = EXS_RESCORE2_TORSION_W;
}

// Workgroups of a persistent launch of shape sh that are resident at once on device dev.
int resident_workgroups(int dev, const LaunchShape& sh) {
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sh.fn, sh.threads, sh.lds);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    return per_cu * std::max(1, g_dev[dev].cus);
}

}  // namespace

extern "C" {

int exs_dock_batch(int64_t batch, const exs_search_params* params, void* stream, int64_t* job_out) {
    try {
        if (!params || !job_out) return fail(EXS_EINVAL, "null argument");
        auto b = find_batch(batch);
        if (!b) return fail(EXS_ENOENT, "unknown batch %lld", (long long)batch);
        const exs_search_params& p = *params;
        const bool persistent = (p.flags & EXS_FLAG_PERSISTENT) != 0;
        LaunchShape sh;
        if (int rc = launch_shape(*b, p, persistent, &sh)) return rc;
        const int ppl = sh.ppl, lpw = sh.lpw, threads = sh.threads, top_k = sh.top_k;
        const int storage = sh.storage;
        const size_t lds = sh.lds;
        const int K = p.n_orient;
        int dev;
        if (int rc = current_device(&dev)) return rc;
        if (dev != b->device) return fail(EXS_EINVAL, "batch lives on device %d, current is %d", b->device, dev);
        hipStream_t st = (hipStream_t)stream;
        const float* r32;
        const double* r64;
        if (int rc = orientation_tables(dev, K, &r32, &r64)) return rc;
        int32_t* d_order = nullptr;
        std::vector<int> groups;
        int n_queues = 1;
        if (int rc = batch_order(*b, K, p.torsion_steps, p.passes, p.n_offsets, persistent, st,
                                 &d_order, &groups, &n_queues)) return rc;

        auto j = std::make_shared<Job>();
        j->device = dev; j->batch = b; j->prm = p; j->stream = st;
        j->L = b->L; j->A = b->A; j->R = b->R; j->K = K; j->top_k = top_k;
        const int L = b->L;
        // workgroup slots of pose scratch: resident workgroups (persistent) or the largest launch
        int64_t slots = 0;
        int resident = 0;
        if (persistent) {
            const int n_tiles = (L + lpw - 1) / lpw;
            resident = std::max(1, std::min(n_tiles, resident_workgroups(dev, sh)));
            slots = resident;
        } else {
            for (int gsz : groups) slots = std::max<int64_t>(slots, (gsz + lpw - 1) / lpw);
        }
        const bool graph = (p.flags & EXS_FLAG_GRAPH) != 0;
        std::shared_ptr<Plan> plan;
        std::vector<int64_t> plan_key;
        if (graph) {
            plan_key = {K, p.torsion_steps, p.passes, p.n_offsets, top_k, ppl, lpw, p.flags,
                        (int64_t)__builtin_bit_cast(uint32_t, p.offset_step_A),
                        (int64_t)__builtin_bit_cast(uint32_t, p.clash_cutoff_A),
                        (int64_t)__builtin_bit_cast(uint32_t, p.clash_penalty), p.rank_keep,
                        (int64_t)__builtin_bit_cast(uint32_t, p.cluster_rmsd_A)};
            std::lock_guard<std::mutex> lk(b->order_mu);
            auto it = b->plans.find(plan_key);
            if (it != b->plans.end()) plan = it->second;
            if (plan) {
                bool expect = false;
                if (!plan->busy.compare_exchange_strong(expect, true))
                    return fail(EXS_EINVAL, "the graph plan of these settings is held by an unreleased job");
            }
        }
        if (plan && plan->exec) {
            j->plan = plan;
            j->args = plan->args;
        } else {
            DockArgs& a = j->args;
            base_args(a, *b, p, sh, r32, r64);
            std::shared_ptr<Plan> fresh;
            if (graph) fresh = std::make_shared<Plan>();
            Alloc al{graph ? &fresh->bufs : &j->bufs, st, !graph};
            const int R = b->R, A = b->A;
            int rc;
            if ((rc = job_alloc(al, &a.orient_score, (size_t)L * K)) ||
                (rc = job_alloc(al, &a.orient_theta, (size_t)R * K)) ||
                (rc = job_alloc(al, &a.orient_tau, (size_t)L * K)) ||
                (rc = job_alloc(al, &a.best_score, (size_t)L)) ||
                (rc = job_alloc(al, &a.best_k, (size_t)L)) ||
                (rc = job_alloc(al, &a.best_coords, (size_t)A * 3)) ||
                (rc = job_alloc(al, &a.best_theta, (size_t)R)) ||
                (rc = job_alloc(al, &a.best_tau, (size_t)L)) ||
                (rc = job_alloc(al, &a.best_score64, (size_t)L)) ||
                (rc = job_alloc(al, &a.topk_k, (size_t)L * top_k)) ||
                (rc = job_alloc(al, &a.topk_score, (size_t)L * top_k)) ||
                (rc = job_alloc(al, &a.topk_score64, (size_t)L * top_k)) ||
                (rc = job_alloc(al, &a.topk_theta, (size_t)R * top_k)) ||
                (rc = job_alloc(al, &a.topk_tau, (size_t)L * top_k)) ||
                (rc = job_alloc(al, &a.n_clusters, (size_t)L)) ||
                (rc = job_alloc(al, &a.ranked, (size_t)L * p.rank_keep)) ||
                (rc = job_alloc(al, &a.final_xyz, p.rank_keep > 0 ? (size_t)A * 3 * K : (size_t)0)) ||
                (rc = job_alloc(al, &a.score2, a.rescore2 ? (size_t)L * p.rank_keep : (size_t)0)) ||
                (rc = job_alloc(al, &a.best2_k, a.rescore2 ? (size_t)L : (size_t)0)) ||
                (rc = job_alloc(al, &a.best2, a.rescore2 ? (size_t)L : (size_t)0)) ||
                (rc = job_alloc(al, &a.tile_counter, (size_t)kMaxWorkQueues)) ||
                (rc = job_alloc(al, &a.scratch, (size_t)std::max<int64_t>(slots, 1) * a.slot_floats))) {
                free_allocs(al);
                return rc;
            }
            if (graph) {
                fresh->args = a;
                // capture the launch sequence once on a private stream
                hipStream_t cs = nullptr;
                HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
                hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    e = enqueue_dock(a, *b, groups, d_order, n_queues, storage, ppl, persistent,
                                     resident, threads, lds, cs);
                    hipGraph_t gr = nullptr;
                    hipError_t e2 = hipStreamEndCapture(cs, &gr);
                    if (e == hipSuccess) e = e2;
                    fresh->graph = gr;
                    if (e == hipSuccess) e = hipGraphInstantiate(&fresh->exec, gr, nullptr, nullptr, 0);
                }
                (void)hipStreamDestroy(cs);
                if (e != hipSuccess) {
                    if (fresh->exec) (void)hipGraphExecDestroy(fresh->exec);
                    if (fresh->graph) (void)hipGraphDestroy(fresh->graph);
                    free_allocs(al);
                    return fail(EXS_EDEVICE, "graph capture: %s", hipGetErrorString(e));
                }
                fresh->busy = true;
                {
                    std::lock_guard<std::mutex> lk(b->order_mu);
                    b->plans[plan_key] = fresh;
                }
                j->plan = fresh;
            }
        }
        HIP_TRY(hipEventCreate(&j->ev0));
        HIP_TRY(hipEventCreate(&j->ev1));
        if (!j->plan && p.rank_keep > 0 && b->L > 0) {
            HIP_TRY(hipEventCreate(&j->ev_dock));
            HIP_TRY(hipEventCreate(&j->ev_rank));
        }
        HIP_TRY(hipEventRecord(j->ev0, st));
        if (j->plan) {
            HIP_TRY(hipGraphLaunch(j->plan->exec, st));
        } else {
            HIP_TRY(enqueue_dock(j->args, *b, groups, d_order, n_queues, storage, ppl, persistent,
                                 resident, threads, lds, st, j->ev_dock, j->ev_rank));
        }
        HIP_TRY(hipEventRecord(j->ev1, st));
        std::lock_guard<std::mutex> lk(g_reg_mu);
        int64_t id = g_next_job++;
        g_jobs[id] = j;
        *job_out = id;
        return EXS_OK;
    } catch (const std::exception& e) {
        return fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_get_best_poses(int64_t job, int wait, float* best_score, exs_pose_desc* desc, float* coords,
                       exs_pose_desc* topk) {
    try {
        auto j = find_job(job);
        if (!j) return fail(EXS_ENOENT, "unknown job %lld", (long long)job);
        if (int rc = job_wait(*j, wait)) return rc;
        const DockArgs& a = j->args;
        const int L = j->L, R = j->R, tk = j->top_k;
        if (best_score && tk > 0) {
            std::vector<double> b64(L);
            if (int rc = copy_out(b64.data(), a.best_score64, (size_t)L)) return rc;
            for (int l = 0; l < L; ++l) best_score[l] = (float)b64[l];
        } else if (int rc = copy_out(best_score, a.best_score, (size_t)L)) {
            return rc;
        }
        if (int rc = copy_out(coords, a.best_coords, (size_t)j->A * 3)) return rc;
        if (desc) {
            std::vector<float> bs(L);
            std::vector<int32_t> bk(L), bt(L);
            std::vector<uint8_t> th(R);
            std::vector<double> b64(L, NAN);
            if (int rc = copy_out(bs.data(), a.best_score, (size_t)L)) return rc;
            if (int rc = copy_out(bk.data(), a.best_k, (size_t)L)) return rc;
            if (int rc = copy_out(bt.data(), a.best_tau, (size_t)L)) return rc;
            if (int rc = copy_out(th.data(), a.best_theta, (size_t)R)) return rc;
            if (tk > 0)
                if (int rc = copy_out(b64.data(), a.best_score64, (size_t)L)) return rc;
            for (int l = 0; l < L; ++l) {
                const LigInfo& inf = j->batch->info[l];
                fill_desc(desc[l], bs[l], b64[l], bk[l], bt[l], inf.nrot, th.data() + inf.rot_base, 1);
            }
        }
        if (topk && tk > 0) {
            std::vector<int32_t> kk((size_t)L * tk), tt((size_t)L * tk);
            std::vector<float> sc((size_t)L * tk);
            std::vector<double> s64((size_t)L * tk);
            std::vector<uint8_t> th((size_t)R * tk);
            if (int rc = copy_out(kk.data(), a.topk_k, kk.size())) return rc;
            if (int rc = copy_out(tt.data(), a.topk_tau, tt.size())) return rc;
            if (int rc = copy_out(sc.data(), a.topk_score, sc.size())) return rc;
            if (int rc = copy_out(s64.data(), a.topk_score64, s64.size())) return rc;
            if (int rc = copy_out(th.data(), a.topk_theta, th.size())) return rc;
            for (int l = 0; l < L; ++l) {
                const LigInfo& inf = j->batch->info[l];
                for (int t = 0; t < tk; ++t) {
                    size_t o = (size_t)l * tk + t;
                    fill_desc(topk[o], sc[o], s64[o], kk[o], tt[o], inf.nrot,
                              th.data() + (size_t)inf.rot_base * tk + t, (size_t)tk);
                }
            }
        }
        return EXS_OK;
    } catch (const std::exception& e) {
        return fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_get_orientation_results(int64_t job, float* score, exs_pose_desc* desc) {
    try {
        auto j = find_job(job);
        if (!j) return fail(EXS_ENOENT, "unknown job %lld", (long long)job);
        if (int rc = job_wait(*j, 1)) return rc;
        const DockArgs& a = j->args;
        const int L = j->L, K = j->K, R = j->R;
        std::vector<float> sc((size_t)L * K);
        if (int rc = copy_out(sc.data(), a.orient_score, sc.size())) return rc;
        if (score) memcpy(score, sc.data(), sc.size() * sizeof(float));
        if (desc) {
            std::vector<int32_t> tt((size_t)L * K);
            std::vector<uint8_t> th((size_t)R * K);
            if (int rc = copy_out(tt.data(), a.orient_tau, tt.size())) return rc;
            if (int rc = copy_out(th.data(), a.orient_theta, th.size())) return rc;
            for (int l = 0; l < L; ++l) {
                const LigInfo& inf = j->batch->info[l];
                for (int k = 0; k < K; ++k) {
                    size_t o = (size_t)l * K + k;
                    fill_desc(desc[o], sc[o], NAN, k, tt[o], inf.nrot,
                              th.data() + (size_t)inf.rot_base * K + k, (size_t)K);
                }
            }
        }
        return EXS_OK;
    } catch (const std::exception& e) {
        return fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_get_rescored_poses(int64_t job, int wait, double* score2, int32_t* best_orient,
                           double* best_score2) {
    try {
        auto j = find_job(job);
        if (!j) return fail(EXS_ENOENT, "unknown job %lld", (long long)job);
        const DockArgs& a = j->args;
        if (!a.rescore2) return fail(EXS_EINVAL, "job %lld was run without EXS_FLAG_RESCORE2", (long long)job);
        if (int rc = job_wait(*j, wait)) return rc;
        if (score2)
            if (int rc = copy_out(score2, a.score2, (size_t)j->L * a.rank_keep)) return rc;
        if (best_orient)
            if (int rc = copy_out(best_orient, a.best2_k, (size_t)j->L)) return rc;
        if (best_score2)
            if (int rc = copy_out(best_score2, a.best2, (size_t)j->L)) return rc;
        return EXS_OK;
    } catch (const std::exception& e) {
        return fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_get_ranked_poses(int64_t job, int wait, int32_t* n_clusters, int32_t* ranked) {
    try {
        auto j = find_job(job);
        if (!j) return fail(EXS_ENOENT, "unknown job %lld", (long long)job);
        const DockArgs& a = j->args;
        if (a.rank_keep <= 0) return fail(EXS_EINVAL, "job %lld was run with rank_keep = 0", (long long)job);
        if (int rc = job_wait(*j, wait)) return rc;
        if (n_clusters)
            if (int rc = copy_out(n_clusters, a.n_clusters, (size_t)j->L)) return rc;
        if (ranked)
            if (int rc = copy_out(ranked, a.ranked, (size_t)j->L * a.rank_keep)) return rc;
        return EXS_OK;
    } catch (const std::exception& e) {
        return fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_job_elapsed_ms(int64_t job, float* ms) {
    auto j = find_job(job);
    if (!j) return fail(EXS_ENOENT, "unknown job %lld", (long long)job);
    if (!ms) return fail(EXS_EINVAL, "null argument");
    if (int rc = job_wait(*j, 1)) return rc;
    HIP_TRY(hipEventElapsedTime(ms, j->ev0, j->ev1));
    return EXS_OK;
}

int exs_job_stage_ms(int64_t job, float* dock_ms, float* rank_ms, float* rescore2_ms) {
    auto j = find_job(job);
    if (!j) return fail(EXS_ENOENT, "unknown job %lld", (long long)job);
    if (!dock_ms || !rank_ms || !rescore2_ms) return fail(EXS_EINVAL, "null argument");
    if (int rc = job_wait(*j, 1)) return rc;
    *rank_ms = *rescore2_ms = -1.0f;
    if (!j->ev_dock) {   // not staged: the whole job
        HIP_TRY(hipEventElapsedTime(dock_ms, j->ev0, j->ev1));
        return EXS_OK;
    }
    HIP_TRY(hipEventElapsedTime(dock_ms, j->ev0, j->ev_dock));
    if (j->args.rescore2) {
        HIP_TRY(hipEventElapsedTime(rank_ms, j->ev_dock, j->ev_rank));
        HIP_TRY(hipEventElapsedTime(rescore2_ms, j->ev_rank, j->ev1));
    } else {   // the ranking ends the job
        HIP_TRY(hipEventElapsedTime(rank_ms, j->ev_dock, j->ev1));
    }
    return EXS_OK;
}

int exs_unfold_ligands(int64_t batch, int torsion_steps, int passes, void* stream, int32_t* turns_out) {
    try {
        if (torsion_steps != 8 && torsion_steps != 16 && torsion_steps != 32)
            return fail(EXS_EINVAL, "torsion_steps %d: supported 8, 16, 32", torsion_steps);
        if (passes < 0 || passes > 64) return fail(EXS_EINVAL, "passes %d outside [0, 64]", passes);
        auto b = find_batch(batch);
        if (!b) return fail(EXS_ENOENT, "unknown ligand batch %lld", (long long)batch);
        int dev;
        if (int rc = current_device(&dev)) return rc;
        if (dev != b->device) return fail(EXS_EINVAL, "batch lives on device %d, current is %d", b->device, dev);
        hipStream_t st = (hipStream_t)stream;
        int32_t* d_turns = nullptr;
        const size_t nt = (size_t)passes * b->R;
        if (turns_out && nt > 0) HIP_TRY(hipMalloc(&d_turns, nt * sizeof(int32_t)));
        hipError_t e = launch_unfold(b->d_info, b->d_ref, b->d_ref64, b->d_rot_uv, b->d_rot_mask,
                                     d_turns, b->d_upload_order, b->L, b->R, torsion_steps, passes, st);
        if (e == hipSuccess && d_turns)
            e = hipMemcpyAsync(turns_out, d_turns, nt * sizeof(int32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (d_turns) (void)hipFree(d_turns);
        if (e != hipSuccess) return fail(EXS_EDEVICE, "unfold: %s", hipGetErrorString(e));
        return EXS_OK;
    } catch (const std::exception& ex) {
        return fail(EXS_ENOMEM, "exception: %s", ex.what());
    }
}

int exs_get_ligand_coords(int64_t batch, float* xyz) {
    try {
        if (!xyz) return fail(EXS_EINVAL, "null argument");
        auto b = find_batch(batch);
        if (!b) return fail(EXS_ENOENT, "unknown ligand batch %lld", (long long)batch);
        std::vector<float4> r((size_t)b->A);
        if (b->A > 0) HIP_TRY(hipMemcpy(r.data(), b->d_ref, r.size() * sizeof(float4), hipMemcpyDeviceToHost));
        for (size_t i = 0; i < r.size(); ++i) {
            xyz[3 * i] = r[i].x; xyz[3 * i + 1] = r[i].y; xyz[3 * i + 2] = r[i].z;
        }
        return EXS_OK;
    } catch (const std::exception& ex) {
        return fail(EXS_ENOMEM, "exception: %s", ex.what());
    }
}

int exs_gather_probe(int32_t pocket_id, int64_t n_lanes, int lookups_per_lane, int batch,
                     float half_edge_A, float walk_step_A, uint32_t seed, void* stream,
                     float* ms_out, double* checksum_out) {
    try {
        if (!ms_out) return fail(EXS_EINVAL, "null argument");
        if (batch != 8 && batch != 16 && batch != 32) return fail(EXS_EINVAL, "batch %d is not 8, 16 or 32", batch);
        if (n_lanes < 1 || n_lanes > ((int64_t)1 << 30))
            return fail(EXS_EINVAL, "n_lanes %lld outside [1, 2^30]", (long long)n_lanes);
        if (lookups_per_lane < 1 || lookups_per_lane > (1 << 20))
            return fail(EXS_EINVAL, "lookups_per_lane %d outside [1, 2^20]", lookups_per_lane);
        if (!(half_edge_A >= 0.0f) || !isfinite(half_edge_A) || !(walk_step_A >= 0.0f) || !isfinite(walk_step_A))
            return fail(EXS_EINVAL, "half edge and walk step must be finite and >= 0");
        std::shared_ptr<Pocket> pk;
        {
            std::lock_guard<std::mutex> lk(g_reg_mu);
            auto it = g_pockets.find(pocket_id);
            if (it == g_pockets.end()) return fail(EXS_ENOENT, "unknown pocket %d", pocket_id);
            pk = it->second;
        }
        int dev;
        if (int rc = current_device(&dev)) return rc;
        if (dev != pk->device) return fail(EXS_EINVAL, "pocket %d is on device %d", pocket_id, pk->device);
        hipStream_t st = (hipStream_t)stream;
        const int64_t blocks = (n_lanes + 255) / 256;
        const float inv_h = (float)(1.0 / pk->h);
        GridDesc* d_gd = nullptr;
        float* d_out = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        auto cleanup = [&]() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
            if (d_gd) (void)hipFree(d_gd);
            if (d_out) (void)hipFree(d_out);
        };
        hipError_t e = hipMalloc(&d_gd, sizeof(GridDesc));
        if (e == hipSuccess) e = hipMalloc(&d_out, (size_t)blocks * 256 * sizeof(float));
        if (e == hipSuccess) e = hipMemcpyAsync(d_gd, &pk->desc, sizeof(GridDesc), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        if (e == hipSuccess)
            e = launch_gather_probe(d_gd, pk->storage, batch, blocks, lookups_per_lane, half_edge_A * inv_h,
                                    walk_step_A * inv_h, seed, d_out, st);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(ms_out, e0, e1);
        if (e == hipSuccess && checksum_out) {
            std::vector<float> h((size_t)blocks * 256);
            e = hipMemcpy(h.data(), d_out, h.size() * sizeof(float), hipMemcpyDeviceToHost);
            double sum = 0.0;
            for (float v : h) sum += v;
            *checksum_out = sum;
        }
        cleanup();
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? EXS_ENOMEM : EXS_EDEVICE, "gather probe: %s", hipGetErrorString(e));
        return EXS_OK;
    } catch (const std::exception& ex) {
        return fail(EXS_ENOMEM, "exception: %s", ex.what());
    }
}

int exs_release_job(int64_t job) {
    std::shared_ptr<Job> j;
    {
        std::lock_guard<std::mutex> lk(g_reg_mu);
        auto it = g_jobs.find(job);
        if (it == g_jobs.end()) return fail(EXS_ENOENT, "unknown job %lld", (long long)job);
        j = it->second;
        g_jobs.erase(it);
    }
    job_free(*j);
    return EXS_OK;
}

}  // extern "C"

namespace exs {
namespace rt {

int noalloc_plan(int64_t batch, const exs_search_params* params, NoAllocPlan* out) {
    if (!params || !out) return fail(EXS_EINVAL, "null argument");
    auto b = find_batch(batch);
    if (!b) return fail(EXS_ENOENT, "unknown batch %lld", (long long)batch);
    const exs_search_params& p = *params;
    if (p.top_k != 0 || p.rank_keep != 0)
        return fail(EXS_EINVAL, "the no-allocation launch needs top_k = 0 and rank_keep = 0");
    if (p.flags & ~EXS_FLAG_PERSISTENT)
        return fail(EXS_EINVAL, "the no-allocation launch takes no flags but EXS_FLAG_PERSISTENT");
    int dev;
    if (int rc = current_device(&dev)) return rc;
    if (dev != b->device) return fail(EXS_EINVAL, "batch lives on device %d, current is %d", b->device, dev);
    LaunchShape sh;
    if (int rc = launch_shape(*b, p, true, &sh)) return rc;
    base_args(out->args, *b, p, sh, nullptr, nullptr);
    DockArgs& a = out->args;
    a.order = b->d_upload_order;
    a.n_order = b->L;
    a.n_tiles = (b->L + sh.lpw - 1) / sh.lpw;
    a.persistent = 1;
    a.queue_bounds = nullptr;
    a.n_queues = 1;
    out->device = dev;
    out->storage = sh.storage;
    out->ppl = sh.ppl;
    out->threads = sh.threads;
    out->lds = sh.lds;
    out->resident = resident_workgroups(dev, sh);
    out->L = b->L; out->A = b->A; out->R = b->R;
    return EXS_OK;
}

}  // namespace rt
}  // namespace exs
