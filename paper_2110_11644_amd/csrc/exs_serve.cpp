// Serving engine: continuous batching of docking requests on one GPU.
//
// The paper's docking application is a pipeline of stages with queues, whose
// docker stage runs several workers per GPU to hide host-side preparation
// (Sec. 3.2, 4.3).  Here one scheduler thread per server plays that role:
//  * requests (a CSR ligand batch against resident pockets) are validated and
//    packed on the submitting thread and queued;
//  * admission: a request enters the device arena when its bytes fit in the
//    HBM budget (the caller's, clamped to the device's free memory less a
//    reserve) and its ligand, atom and bond ranges fit -- FIFO, so a
//    request that does not fit holds back the ones behind it (backpressure);
//    its packed data is uploaded on an upload stream;
//  * iterations: each launch is the persistent dock kernel over a work list of
//    not-yet-docked ligands of the in-flight requests (oldest request first,
//    capped per iteration), in the work queues of a persistent launch; up to two
//    iterations run at once on two streams, so a new iteration fills the CUs
//    the previous one's tail leaves idle (the upload stream and the iteration
//    streams each have a hardware queue of their own, so that neither uploads
//    nor the next iteration wait behind a running kernel);
//  * completion: a request whose last ligand finished has its results copied
//    to host buffers and its arena ranges freed.
// A ligand's result does not depend on what it is batched with (every lane
// searches its own orientation; tiles hold whole ligands), so a request gives
// the same answer alone and in the mix.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
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

using Clock = std::chrono::steady_clock;

#define SRV_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return rt::fail(e_ == hipErrorOutOfMemory ? EXS_ENOMEM : EXS_EDEVICE, "%s: %s", #expr, \
                            hipGetErrorString(e_));                                        \
    } while (0)

// First-fit allocator of index ranges [0, cap).
class RangeAlloc {
  public:
    void reset(int cap) { free_.clear(); if (cap > 0) free_[0] = cap; cap_ = cap; }
    bool alloc(int n, int* start) {
        if (n == 0) { *start = 0; return true; }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *start = it->first;
                int rest = it->second - n, at = it->first + n;
                free_.erase(it);
                if (rest > 0) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(int start, int n) {
        if (n == 0) return;
        auto it = free_.emplace(start, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    int cap() const { return cap_; }

  private:
    std::map<int, int> free_;
    int cap_ = 0;
};

enum ReqState { kQueued, kInflight, kDone };

// A stream on a hardware queue of its own.  The runtime maps ordinary streams onto a small pool
// of hardware queues, so two streams can share one, and then a copy or kernel on one waits for
// every kernel queued before it on the other (a pageable upload even holds the calling thread
// until then).  A stream created with a CU mask always gets a queue of its own; the mask here
// holds every CU, so nothing is restricted.  Such a stream synchronizes with the null stream.
// Where the runtime refuses a CU mask, an ordinary non-blocking stream is used (correct, but
// iterations may then wait for each other).
hipError_t own_queue_stream(int cus, hipStream_t* s) {
    std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
    for (int c = 0; c < cus; ++c) mask[(size_t)c / 32] |= 1u << (c % 32);
    if (hipExtStreamCreateWithCUMask(s, (uint32_t)mask.size(), mask.data()) == hipSuccess) return hipSuccess;
    (void)hipGetLastError();
    return hipStreamCreateWithFlags(s, hipStreamNonBlocking);
}

struct Request {
    int64_t id = 0;
    int L = 0, A = 0, R = 0;
    int64_t bytes = 0;          // device bytes it holds while admitted
    // packed host data (request-local bases)
    std::vector<LigInfo> info;
    std::vector<float4> ref;
    std::vector<double> ref64;
    std::vector<uint4> excl;
    std::vector<uint32_t> ruv;
    std::vector<uint4> rmask;
    std::vector<double> cost;
    // arena ranges
    int lig0 = 0, atom0 = 0, rot0 = 0;
    int scheduled = 0, remaining = 0;
    ReqState state = kQueued;
    Clock::time_point t_submit, t_done;
    // results
    std::vector<float> best_score;
    std::vector<exs_pose_desc> desc;
    std::vector<float> coords;
};

struct Iteration {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    // work list indices: processing order [n], queue bounds [kMaxWorkQueues + 1], then per
    // work-list ligand j: arena ligand [n], result atom offset [n], result bond offset [n].
    // Written by the host into mapped pinned memory (h_order, hd_order its device address)
    // and staged into d_order by a kernel: no copy call is queued (the runtime performs small
    // copies on the host after waiting for the stream's earlier work, which would hold the
    // scheduler until the running iteration ends).
    int32_t* d_order = nullptr;
    int32_t* h_order = nullptr;
    int32_t* hd_order = nullptr;
    int* d_counter = nullptr;
    float* scratch = nullptr;
    // results (records | coordinates | torsion bytes), written by each ligand's finish in the
    // search kernel straight into mapped pinned memory (h_res; hd_res its device address)
    unsigned char* h_res = nullptr;
    unsigned char* hd_res = nullptr;
    bool running = false;
    struct Work { Request* r; int start, count; };   // ligands start .. start+count-1 of r
    std::vector<Work> work;
    Clock::time_point t_launch;
};

class Server {
  public:
    ~Server() { shutdown(); }

    int create(const int32_t* pockets, int n_pockets, const exs_search_params& p,
               const exs_server_config& cfg);
    int submit(const exs_ligand_batch& in, int64_t* id_out);
    int poll(int64_t id, int wait, float* best_score, exs_pose_desc* desc, float* coords,
             double* latency_ms);
    void stats(exs_server_stats* out);
    void shutdown();

  private:
    void loop();
    bool admit_locked();
    void complete(Iteration& it);
    bool launch(Iteration& it);

    int dev_ = 0;
    exs_search_params prm_{};
    int K_ = 0, ppl_ = 1, lpw_ = 1, wpl_ = 1, threads_ = 64, top_k_ = 0, storage_ = 0;
    int resident_ = 1, max_iter_ = 0, n_iters_ = 2;
    size_t res_rec_bytes_ = 0, res_coord_bytes_ = 0, res_theta_bytes_ = 0;   // staging regions
    size_t lds_ = 0;
    std::vector<int32_t> pocket_ids_;
    std::unordered_map<int32_t, int> pocket_slot_;
    std::vector<int> channels_;
    DockArgs base_{};
    std::vector<void*> dev_bufs_;
    RangeAlloc lig_alloc_, atom_alloc_, rot_alloc_;
    int64_t per_lig_ = 0, per_atom_ = 0, per_rot_ = 0;       // device bytes of each item
    int64_t budget_ = 0, arena_budget_ = 0;                    // HBM budget; its request part
    int64_t admitted_bytes_ = 0, peak_admitted_bytes_ = 0, peak_queued_ = 0;
    hipStream_t up_stream_ = nullptr;
    hipEvent_t up_event_ = nullptr;
    int32_t* res_slot_ = nullptr;   // device [arena ligands]: position in its iteration's work list
    bool up_pending_ = false;
    Iteration it_[2];

    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Request*> queue_;
    std::vector<Request*> inflight_;
    std::unordered_map<int64_t, std::unique_ptr<Request>> reqs_;
    int64_t next_id_ = 1;
    bool stop_ = false;
    std::thread thread_;
    // stats
    int64_t submitted_ = 0, completed_ = 0, iterations_ = 0, ligands_ = 0;
    double busy_ms_ = 0.0;
    std::string thread_error_;
};

template <class T>
int dev_alloc(std::vector<void*>& bufs, T** p, size_t count) {
    void* q = nullptr;
    SRV_TRY(hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)));
    bufs.push_back(q);
    *p = (T*)q;
    return EXS_OK;
}

int Server::create(const int32_t* pockets, int n_pockets, const exs_search_params& p,
                   const exs_server_config& cfg) {
    if (n_pockets < 1 || !pockets) return rt::fail(EXS_EINVAL, "a server needs at least one pocket");
    if (int rc = rt::current_device(&dev_)) return rc;
    if (int rc = rt::ensure_device(dev_)) return rc;
    prm_ = p;
    K_ = p.n_orient;
    if (K_ < 1 || K_ > EXS_MAX_ORIENT) return rt::fail(EXS_EINVAL, "n_orient %d", K_);
    if (p.torsion_steps != 8 && p.torsion_steps != 16 && p.torsion_steps != 32)
        return rt::fail(EXS_EINVAL, "torsion_steps %d: supported 8, 16, 32", p.torsion_steps);
    if (p.n_offsets != 1 && p.n_offsets != 27) return rt::fail(EXS_EINVAL, "n_offsets must be 1 or 27");
    if (p.passes < 0 || p.passes > 64) return rt::fail(EXS_EINVAL, "passes %d", p.passes);
    if (p.top_k < 0 || p.top_k > EXS_MAX_TOPK) return rt::fail(EXS_EINVAL, "top_k %d", p.top_k);
    if (p.rank_keep != 0) return rt::fail(EXS_EINVAL, "the server does not rank poses (rank_keep must be 0)");
    ppl_ = p.poses_per_lane ? p.poses_per_lane : 1;
    if (ppl_ != 1 && ppl_ != 2 && ppl_ != 4) return rt::fail(EXS_EINVAL, "poses_per_lane %d", ppl_);
    wpl_ = (K_ + kWave * ppl_ - 1) / (kWave * ppl_);
    lpw_ = p.ligands_per_wg ? p.ligands_per_wg : 1;
    if (lpw_ != 1 && lpw_ != 2 && lpw_ != 4 && lpw_ != 8)
        return rt::fail(EXS_EINVAL, "ligands_per_wg %d: supported 1, 2, 4, 8", lpw_);
    top_k_ = std::min(p.top_k, K_);
    const int waves = dock_waves(lpw_, wpl_, top_k_, ppl_, p.torsion_steps);
    if (waves < 1) return rt::fail(EXS_EINVAL, "tile does not fit in LDS");
    threads_ = waves * kWave;
    lds_ = dock_lds_bytes(lpw_, top_k_, waves, ppl_, p.torsion_steps);
    n_iters_ = cfg.max_inflight_iters == 1 ? 1 : 2;
    // pockets
    std::vector<GridDesc> grids;
    for (int i = 0; i < n_pockets; ++i) {
        rt::PocketInfo pi;
        if (!rt::pocket_info(pockets[i], &pi)) return rt::fail(EXS_EINVAL, "unknown pocket %d", pockets[i]);
        if (pi.device != dev_) return rt::fail(EXS_EINVAL, "pocket %d is on another device", pockets[i]);
        if (i > 0 && pi.storage != storage_)
            return rt::fail(EXS_EINVAL, "all pockets of a server need the same texel storage");
        storage_ = pi.storage;
        pocket_slot_[pockets[i]] = i;
        channels_.push_back(pi.channels);
        grids.push_back(pi.desc);
    }
    const void* fn = dock_kernel_fn(storage_, p.torsion_steps, ppl_);
    if (lds_ > 64 * 1024)
        SRV_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_));
    int per_cu = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads_, lds_) != hipSuccess || per_cu < 1)
        per_cu = 1;
    resident_ = std::max(1, per_cu * rt::device_cus(dev_));
    // default: four waves of workgroups' worth of ligands (with two iterations in flight, two
    // measured the same latency at 0.7 of capacity and a 25 % higher p99 at 0.9; one lost
    // throughput to the iterations' tails)
    max_iter_ = cfg.max_iter_ligands > 0 ? cfg.max_iter_ligands : 4 * resident_ * lpw_;
    // budget: scratch for the iterations first, the rest is the request arena
    const int64_t slot_floats = (int64_t)lpw_ * EXS_MAX_ATOMS * 3 * (wpl_ * kWave * ppl_);
    res_rec_bytes_ = sizeof(ResultRec) * (size_t)max_iter_;
    res_coord_bytes_ = sizeof(float) * 3 * (size_t)EXS_MAX_ATOMS * max_iter_;
    res_theta_bytes_ = (size_t)EXS_MAX_ROT * max_iter_;
    const int64_t scratch_bytes = (int64_t)n_iters_ * resident_ * slot_floats * 4 +
                                  (int64_t)n_iters_ * (4 * (int64_t)max_iter_ + kMaxWorkQueues + 1) * 4;
    per_lig_ = 32 + 12LL * K_ + 40 + 28LL * top_k_ + 4;   // info, per-orientation, best, top-k, order
    per_atom_ = 16 + 24 + 16 + 12;
    per_rot_ = 4 + 16 + K_ + 1 + top_k_;
    // budget: the caller's (2 GiB if 0), never more than the device's free memory less a reserve
    // (1 GiB or 5 % of the device, the larger) for the rest of the process
    size_t free_b = 0, total_b = 0;
    SRV_TRY(hipMemGetInfo(&free_b, &total_b));
    const int64_t reserve = std::max<int64_t>((int64_t)1 << 30, (int64_t)(total_b / 20));
    const int64_t avail = std::max<int64_t>(0, (int64_t)free_b - reserve);
    const int64_t asked = cfg.hbm_budget_bytes > 0 ? cfg.hbm_budget_bytes : (int64_t)2 << 30;
    budget_ = std::min(asked, avail);
    arena_budget_ = budget_ - scratch_bytes;
    // index ranges of the arena: 1.5x the ligands, atoms and bonds of the byte budget at 48 atoms
    // and 16 bonds per ligand, so that for usual ligand sizes the byte budget, not a range, is
    // what admission runs out of (requests are admitted by their actual bytes)
    const int64_t unit = per_lig_ + 48 * per_atom_ + 16 * per_rot_;
    const int64_t cap_l = arena_budget_ > 0 ? (3 * arena_budget_) / (2 * unit) : 0;
    if (cap_l < 1)
        return rt::fail(EXS_ENOMEM, "HBM budget %lld (asked %lld, free %zu less %lld reserved) below "
                        "the iteration scratch (%lld) and one ligand", (long long)budget_,
                        (long long)asked, free_b, (long long)reserve, (long long)scratch_bytes);
    int64_t cap = std::min<int64_t>(cap_l, 1 << 24);
    if (cfg.max_arena_ligands > 0) cap = std::min<int64_t>(cap, cfg.max_arena_ligands);
    const int capL = (int)cap;
    const int capA = capL * 48, capR = capL * 16;
    lig_alloc_.reset(capL);
    atom_alloc_.reset(capA);
    rot_alloc_.reset(capR);
    // arena
    DockArgs& a = base_;
    memset(&a, 0, sizeof a);
    LigInfo* info;
    float4* ref;
    double* ref64;
    uint4 *excl, *rmask;
    uint32_t* ruv;
    GridDesc* dg;
    int rc;
    if ((rc = dev_alloc(dev_bufs_, &info, capL)) || (rc = dev_alloc(dev_bufs_, &ref, capA)) ||
        (rc = dev_alloc(dev_bufs_, &ref64, (size_t)capA * 3)) || (rc = dev_alloc(dev_bufs_, &excl, capA)) ||
        (rc = dev_alloc(dev_bufs_, &ruv, capR)) || (rc = dev_alloc(dev_bufs_, &rmask, capR)) ||
        (rc = dev_alloc(dev_bufs_, &dg, grids.size())) || (rc = dev_alloc(dev_bufs_, &res_slot_, capL)) ||
        (rc = dev_alloc(dev_bufs_, &a.orient_score, (size_t)capL * K_)) ||
        (rc = dev_alloc(dev_bufs_, &a.orient_theta, (size_t)capR * K_)) ||
        (rc = dev_alloc(dev_bufs_, &a.orient_tau, (size_t)capL * K_)) ||
        (rc = dev_alloc(dev_bufs_, &a.best_score, capL)) || (rc = dev_alloc(dev_bufs_, &a.best_k, capL)) ||
        (rc = dev_alloc(dev_bufs_, &a.best_coords, (size_t)capA * 3)) ||
        (rc = dev_alloc(dev_bufs_, &a.best_theta, capR)) || (rc = dev_alloc(dev_bufs_, &a.best_tau, capL)) ||
        (rc = dev_alloc(dev_bufs_, &a.best_score64, capL)) ||
        (rc = dev_alloc(dev_bufs_, &a.topk_k, (size_t)capL * top_k_)) ||
        (rc = dev_alloc(dev_bufs_, &a.topk_score, (size_t)capL * top_k_)) ||
        (rc = dev_alloc(dev_bufs_, &a.topk_score64, (size_t)capL * top_k_)) ||
        (rc = dev_alloc(dev_bufs_, &a.topk_theta, (size_t)capR * top_k_)) ||
        (rc = dev_alloc(dev_bufs_, &a.topk_tau, (size_t)capL * top_k_)))
        return rc;
    SRV_TRY(hipMemcpy(dg, grids.data(), grids.size() * sizeof(GridDesc), hipMemcpyHostToDevice));
    a.info = info; a.ref = ref; a.ref64 = ref64; a.excl = excl; a.rot_uv = ruv; a.rot_mask = rmask;
    a.grids = dg;
    if ((rc = rt::orientation_tables(dev_, K_, &a.rot32, &a.rot64))) return rc;
    a.K = K_; a.S = p.torsion_steps; a.P = p.passes; a.T = p.n_offsets;
    a.step = p.offset_step_A; a.cut2 = p.clash_cutoff_A * p.clash_cutoff_A; a.pen = p.clash_penalty;
    a.step64 = p.offset_step_A; a.cut2_64 = (double)p.clash_cutoff_A * p.clash_cutoff_A;
    a.pen64 = p.clash_penalty;
    a.top_k = top_k_; a.lpw = lpw_; a.wpl = wpl_; a.kp = wpl_ * kWave * ppl_;
    a.n_max = EXS_MAX_ATOMS;
    a.slot_floats = slot_floats;
    a.persistent = 1;
    // the streams get a hardware queue each, several ms apiece: created on threads of their own
    {
        hipStream_t* target[3] = {&up_stream_, &it_[0].stream, n_iters_ > 1 ? &it_[1].stream : nullptr};
        hipError_t err[3] = {hipSuccess, hipSuccess, hipSuccess};
        const int cus = rt::device_cus(dev_);
        struct Join {
            std::vector<std::thread> ts;
            ~Join() {
                for (auto& t : ts)
                    if (t.joinable()) t.join();
            }
        } join;
        for (int i = 1; i < 3; ++i)
            if (target[i])
                join.ts.emplace_back([&, i] {
                    err[i] = hipSetDevice(dev_);
                    if (err[i] == hipSuccess) err[i] = own_queue_stream(cus, target[i]);
                });
        err[0] = own_queue_stream(cus, target[0]);
        for (auto& t : join.ts) t.join();
        for (hipError_t e : err) SRV_TRY(e);
    }
    SRV_TRY(hipEventCreateWithFlags(&up_event_, hipEventDisableTiming));
    for (int i = 0; i < n_iters_; ++i) {
        Iteration& it = it_[i];
        SRV_TRY(hipEventCreateWithFlags(&it.done, hipEventDisableTiming));
        if ((rc = dev_alloc(dev_bufs_, &it.d_order, 4 * (size_t)max_iter_ + kMaxWorkQueues + 1)) ||
            (rc = dev_alloc(dev_bufs_, &it.d_counter, kMaxWorkQueues)) ||
            (rc = dev_alloc(dev_bufs_, &it.scratch, (size_t)resident_ * slot_floats)))
            return rc;
        // mapped, coherent pinned memory: kernels read and write it over the bus, uncached
        SRV_TRY(hipHostMalloc((void**)&it.h_order, sizeof(int32_t) * (4 * (size_t)max_iter_ + kMaxWorkQueues + 1),
                              hipHostMallocMapped | hipHostMallocCoherent));
        SRV_TRY(hipHostMalloc((void**)&it.h_res, res_rec_bytes_ + res_coord_bytes_ + res_theta_bytes_,
                              hipHostMallocMapped | hipHostMallocCoherent));
        SRV_TRY(hipHostGetDevicePointer((void**)&it.hd_order, it.h_order, 0));
        SRV_TRY(hipHostGetDevicePointer((void**)&it.hd_res, it.h_res, 0));
    }
    pocket_ids_.assign(pockets, pockets + n_pockets);
    for (int32_t id : pocket_ids_) rt::pocket_use(id, +1);
    thread_ = std::thread([this] {
        try {
            loop();
        } catch (const std::exception& e) {   // fail the server (pollers see it) rather than the process
            std::lock_guard<std::mutex> lk(mu_);
            thread_error_ = std::string("scheduler: ") + e.what();
            done_cv_.notify_all();
        }
    });
    return EXS_OK;
}

int Server::submit(const exs_ligand_batch& in, int64_t* id_out) {
    const int L = in.n_ligands;
    if (L < 1) return rt::fail(EXS_EINVAL, "empty request");
    if (!in.atom_offset || !in.x || !in.y || !in.z || !in.type || !in.bond_offset ||
        !in.rot_offset || !in.pocket_id)
        return rt::fail(EXS_EINVAL, "null array in request");
    if (in.atom_offset[0] != 0 || in.bond_offset[0] != 0 || in.rot_offset[0] != 0)
        return rt::fail(EXS_EINVAL, "offsets must start at 0");
    auto r = std::make_unique<Request>();
    r->L = L;
    r->A = in.atom_offset[L];
    r->R = in.rot_offset[L];
    if (r->R > 0 && !in.rot_bond) return rt::fail(EXS_EINVAL, "null rot_bond");
    if (in.bond_offset[L] > 0 && !in.bond_ij) return rt::fail(EXS_EINVAL, "null bond_ij");
    r->bytes = (int64_t)r->L * per_lig_ + (int64_t)r->A * per_atom_ + (int64_t)r->R * per_rot_;
    if (r->L > lig_alloc_.cap() || r->A > atom_alloc_.cap() || r->R > rot_alloc_.cap() ||
        r->bytes > arena_budget_)
        return rt::fail(EXS_ENOMEM, "request of %d ligands / %d atoms (%lld B) exceeds the server arena "
                        "(%lld B)", L, r->A, (long long)r->bytes, (long long)arena_budget_);
    r->info.resize(L); r->ref.resize(r->A); r->ref64.resize((size_t)r->A * 3); r->excl.resize(r->A);
    r->ruv.resize(r->R); r->rmask.resize(r->R); r->cost.resize(L);
    r->best_score.resize(L); r->desc.resize(L); r->coords.resize((size_t)r->A * 3);
    PackedLigand pk;            // reused across the request's ligands (keeps its capacity)
    std::string err;
    std::vector<int16_t> m;
    for (int l = 0; l < L; ++l) {
        if (in.atom_offset[l + 1] < in.atom_offset[l] || in.bond_offset[l + 1] < in.bond_offset[l] ||
            in.rot_offset[l + 1] < in.rot_offset[l])
            return rt::fail(EXS_EINVAL, "ligand %d: offsets decrease", l);
        auto ps = pocket_slot_.find(in.pocket_id[l]);
        if (ps == pocket_slot_.end())
            return rt::fail(EXS_EINVAL, "ligand %d: pocket %d is not served", l, in.pocket_id[l]);
        int a0 = in.atom_offset[l], n = in.atom_offset[l + 1] - a0;
        int b0 = in.bond_offset[l], nb = in.bond_offset[l + 1] - b0;
        int r0 = in.rot_offset[l], nr = in.rot_offset[l + 1] - r0;
        int rc = pack_ligand(n, in.bond_ij + 2 * (size_t)b0, nb, in.rot_bond + r0, nr, in.type + a0,
                             channels_[ps->second], in.x + a0, in.y + a0, in.z + a0, &pk, &err);
        if (rc) return rt::fail(rc, "ligand %d: %s", l, err.c_str());
        LigInfo& inf = r->info[l];
        memset(&inf, 0, sizeof inf);
        inf.atom_base = a0; inf.rot_base = r0; inf.n = (int16_t)n; inf.nrot = (int16_t)nr;
        inf.pocket = (int16_t)ps->second;
        m.assign(nr, 0);
        for (int i = 0; i < n; ++i) {
            double dx = (double)in.x[a0 + i] - pk.centroid[0], dy = (double)in.y[a0 + i] - pk.centroid[1],
                   dz = (double)in.z[a0 + i] - pk.centroid[2];
            r->ref[a0 + i] = make_float4((float)dx, (float)dy, (float)dz,
                                         __builtin_bit_cast(float, (int)in.type[a0 + i]));
            r->ref64[(size_t)(a0 + i) * 3] = dx;
            r->ref64[(size_t)(a0 + i) * 3 + 1] = dy;
            r->ref64[(size_t)(a0 + i) * 3 + 2] = dz;
            r->excl[a0 + i] = pk.excl[i].as_uint4();
        }
        for (int b = 0; b < nr; ++b) {
            r->ruv[r0 + b] = (uint32_t)pk.rot_u[b] | ((uint32_t)pk.rot_v[b] << 16);
            r->rmask[r0 + b] = pk.moving[b].as_uint4();
            m[b] = (int16_t)pk.moving[b].count();
        }
        r->cost[l] = ligand_cost(n, m.data(), nr, K_, prm_.torsion_steps, prm_.passes, prm_.n_offsets);
    }
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_) return rt::fail(EXS_EINVAL, "server is shutting down");
    if (!thread_error_.empty()) return rt::fail(EXS_EDEVICE, "server failed: %s", thread_error_.c_str());
    r->id = next_id_++;
    r->remaining = L;
    r->t_submit = Clock::now();
    *id_out = r->id;
    queue_.push_back(r.get());
    peak_queued_ = std::max<int64_t>(peak_queued_, (int64_t)queue_.size());
    reqs_[r->id] = std::move(r);
    submitted_++;
    cv_.notify_all();
    return EXS_OK;
}

// Move queued requests into the arena while they fit (FIFO).  Called with mu_ held.
bool Server::admit_locked() {
    bool any = false;
    while (!queue_.empty()) {
        Request* r = queue_.front();
        int l0, a0, r0;
        if (admitted_bytes_ + r->bytes > arena_budget_) break;   // the byte budget holds it back
        if (!lig_alloc_.alloc(r->L, &l0)) break;
        if (!atom_alloc_.alloc(r->A, &a0)) { lig_alloc_.release(l0, r->L); break; }
        if (!rot_alloc_.alloc(r->R, &r0)) {
            lig_alloc_.release(l0, r->L); atom_alloc_.release(a0, r->A); break;
        }
        queue_.pop_front();
        admitted_bytes_ += r->bytes;
        peak_admitted_bytes_ = std::max(peak_admitted_bytes_, admitted_bytes_);
        r->lig0 = l0; r->atom0 = a0; r->rot0 = r0;
        for (auto& inf : r->info) { inf.atom_base += a0; inf.rot_base += r0; }
        const DockArgs& a = base_;
        (void)hipMemcpyAsync((void*)(a.info + l0), r->info.data(), sizeof(LigInfo) * r->L, hipMemcpyHostToDevice, up_stream_);
        if (r->A) {
            (void)hipMemcpyAsync((void*)(a.ref + a0), r->ref.data(), sizeof(float4) * r->A, hipMemcpyHostToDevice, up_stream_);
            (void)hipMemcpyAsync((void*)(a.ref64 + (size_t)a0 * 3), r->ref64.data(), sizeof(double) * 3 * r->A, hipMemcpyHostToDevice, up_stream_);
            (void)hipMemcpyAsync((void*)(a.excl + a0), r->excl.data(), sizeof(uint4) * r->A, hipMemcpyHostToDevice, up_stream_);
        }
        if (r->R) {
            (void)hipMemcpyAsync((void*)(a.rot_uv + r0), r->ruv.data(), sizeof(uint32_t) * r->R, hipMemcpyHostToDevice, up_stream_);
            (void)hipMemcpyAsync((void*)(a.rot_mask + r0), r->rmask.data(), sizeof(uint4) * r->R, hipMemcpyHostToDevice, up_stream_);
        }
        r->state = kInflight;
        inflight_.push_back(r);
        any = true;
    }
    if (any) {
        (void)hipEventRecord(up_event_, up_stream_);
        up_pending_ = true;
    }
    return any;
}

bool Server::launch(Iteration& it) {
    // oldest requests first, up to max_iter_ ligands; j = position in this work list
    std::vector<double> cost;
    std::vector<int> pocket;
    std::vector<int32_t> lig, nat, nrt;
    it.work.clear();
    for (Request* r : inflight_) {
        if ((int)lig.size() >= max_iter_) break;
        int take = std::min(r->L - r->scheduled, max_iter_ - (int)lig.size());
        if (take <= 0) continue;
        for (int i = 0; i < take; ++i) {
            const LigInfo& inf = r->info[r->scheduled + i];
            cost.push_back(r->cost[r->scheduled + i]);
            pocket.push_back(inf.pocket);
            lig.push_back(r->lig0 + r->scheduled + i);
            nat.push_back(inf.n);
            nrt.push_back(inf.nrot);
        }
        it.work.push_back({r, r->scheduled, take});
        r->scheduled += take;
    }
    if (lig.empty()) return false;
    // work queues (queue_plan: spread or pocket-major), then each ligand's arena index and the
    // offsets of its coordinates and torsion bytes in the result buffer
    const int n = (int)lig.size();
    int32_t* h_ord = it.h_order;
    int32_t* h_bounds = h_ord + n;
    int32_t* h_lig = h_bounds + kMaxWorkQueues + 1;
    int32_t* h_adst = h_lig + n;
    int32_t* h_rdst = h_adst + n;
    std::vector<int32_t> ord(n);
    int used = 0;
    {
        std::vector<int> seen(pocket_ids_.size(), 0);
        for (int p : pocket) used += seen[p]++ == 0 ? 1 : 0;
    }
    const QueuePlan plan = queue_plan(n, used, wpl_);
    work_queues(n, pocket.data(), cost.data(), plan.n_queues, plan.pocket_major, ord.data(), h_bounds);
    int atoms = 0, rots = 0;
    for (int j = 0; j < n; ++j) {
        h_ord[j] = lig[ord[j]];
        h_lig[j] = lig[j];
        h_adst[j] = atoms;
        h_rdst[j] = rots;
        atoms += nat[j];
        rots += nrt[j];
    }
    const int32_t* d_bounds = it.d_order + n;
    const int32_t* d_lig = d_bounds + kMaxWorkQueues + 1;
    if (up_pending_) (void)hipStreamWaitEvent(it.stream, up_event_, 0);
    DockArgs a = base_;
    a.order = it.d_order;
    a.n_order = n;
    a.n_tiles = (a.n_order + lpw_ - 1) / lpw_;
    a.tile_counter = it.d_counter;
    a.queue_bounds = d_bounds;
    a.n_queues = plan.n_queues;
    a.scratch = it.scratch;
    // each ligand's finish writes its result straight into the pinned result buffer, so the
    // iteration ends with its search (a kernel queued after it would wait for CUs behind the
    // other iteration's persistent launch)
    a.res_slot = res_slot_;
    a.res_adst = d_lig + n;
    a.res_rdst = d_lig + 2 * n;
    a.res_rec = reinterpret_cast<ResultRec*>(it.hd_res);
    a.res_coords = reinterpret_cast<float*>(it.hd_res + res_rec_bytes_);
    a.res_theta = it.hd_res + res_rec_bytes_ + res_coord_bytes_;
    hipError_t e = launch_stage_ints(it.hd_order, it.d_order, 4 * n + kMaxWorkQueues + 1, it.d_counter,
                                     plan.n_queues, n + kMaxWorkQueues + 1, n, res_slot_, it.stream);
    if (e == hipSuccess)
        e = launch_dock(a, storage_, ppl_, std::min(resident_, a.n_tiles), threads_, lds_, it.stream);
    if (e == hipSuccess) e = hipEventRecord(it.done, it.stream);
    if (e != hipSuccess) {
        thread_error_ = hipGetErrorString(e);
        return false;
    }
    it.running = true;
    it.t_launch = Clock::now();
    iterations_++;
    return true;
}

void Server::complete(Iteration& it) {
    it.running = false;
    busy_ms_ += std::chrono::duration<double, std::milli>(Clock::now() - it.t_launch).count();
    const ResultRec* rec = reinterpret_cast<const ResultRec*>(it.h_res);
    const float* co = reinterpret_cast<const float*>(it.h_res + res_rec_bytes_);
    const uint8_t* th = it.h_res + res_rec_bytes_ + res_coord_bytes_;
    int j = 0;
    size_t atom = 0, rot = 0;
    for (const Iteration::Work& w : it.work) {
        Request* r = w.r;
        for (int l = w.start; l < w.start + w.count; ++l, ++j) {
            const LigInfo& inf = r->info[l];
            const ResultRec& rr = rec[j];
            exs_pose_desc& d = r->desc[l];
            memset(&d, 0, sizeof d);
            d.score = rr.score;
            d.score_fp64 = top_k_ > 0 ? rr.score64 : NAN;
            d.orient = rr.k;
            d.tau[0] = (int8_t)(rr.tau & 0xff);
            d.tau[1] = (int8_t)((rr.tau >> 8) & 0xff);
            d.tau[2] = (int8_t)((rr.tau >> 16) & 0xff);
            d.n_rot = (uint8_t)inf.nrot;
            memcpy(d.theta, th + rot, inf.nrot);
            r->best_score[l] = top_k_ > 0 ? (float)rr.score64 : rr.score;
            memcpy(&r->coords[(size_t)(inf.atom_base - r->atom0) * 3], co + atom * 3,
                   sizeof(float) * 3 * inf.n);
            atom += inf.n;
            rot += inf.nrot;
        }
        r->remaining -= w.count;
        ligands_ += w.count;
        if (r->remaining > 0) continue;
        lig_alloc_.release(r->lig0, r->L);
        atom_alloc_.release(r->atom0, r->A);
        rot_alloc_.release(r->rot0, r->R);
        admitted_bytes_ -= r->bytes;
        r->state = kDone;
        r->t_done = Clock::now();
        completed_++;
        inflight_.erase(std::find(inflight_.begin(), inflight_.end(), r));
        // release the packed inputs
        std::vector<float4>().swap(r->ref);
        std::vector<double>().swap(r->ref64);
        std::vector<uint4>().swap(r->excl);
        std::vector<uint4>().swap(r->rmask);
    }
    it.work.clear();
    done_cv_.notify_all();
}

void Server::loop() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
        bool progress = false;
        if (thread_error_.empty()) {
            if (admit_locked()) progress = true;
            for (int i = 0; i < n_iters_; ++i) {
                Iteration& it = it_[i];
                if (!it.running) continue;
                const hipError_t q = hipEventQuery(it.done);
                if (q == hipSuccess) {
                    complete(it);
                    progress = true;
                } else if (q != hipErrorNotReady) {   // a device error: fail the server, wake pollers
                    thread_error_ = hipGetErrorString(q);
                    it.running = false;
                    progress = true;
                }
            }
            if (admit_locked()) progress = true;
            for (int i = 0; i < n_iters_; ++i)
                if (!it_[i].running && launch(it_[i])) progress = true;
        }
        bool running = false;
        for (int i = 0; i < n_iters_; ++i) running |= it_[i].running;
        if (stop_ && !running) break;
        if (!thread_error_.empty()) {
            done_cv_.notify_all();
            if (stop_) break;
        }
        if (!progress) {
            if (running) cv_.wait_for(lk, std::chrono::microseconds(50));
            else cv_.wait_for(lk, std::chrono::milliseconds(5));
        }
    }
}

int Server::poll(int64_t id, int wait, float* best_score, exs_pose_desc* desc, float* coords,
                 double* latency_ms) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end()) return rt::fail(EXS_ENOENT, "unknown request %lld", (long long)id);
    Request* r = it->second.get();
    if (wait)
        done_cv_.wait(lk, [&] { return r->state == kDone || !thread_error_.empty() || stop_; });
    if (r->state != kDone) {
        if (!thread_error_.empty()) return rt::fail(EXS_EDEVICE, "server failed: %s", thread_error_.c_str());
        if (stop_) return rt::fail(EXS_EINVAL, "server shut down before request %lld finished", (long long)id);
        return rt::fail(EXS_ENOTREADY, "request %lld is %s", (long long)id,
                        r->state == kQueued ? "queued" : "running");
    }
    if (best_score) memcpy(best_score, r->best_score.data(), sizeof(float) * r->L);
    if (desc) memcpy(desc, r->desc.data(), sizeof(exs_pose_desc) * r->L);
    if (coords) memcpy(coords, r->coords.data(), sizeof(float) * 3 * r->A);
    if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
    reqs_.erase(it);
    return EXS_OK;
}

void Server::stats(exs_server_stats* out) {
    std::lock_guard<std::mutex> lk(mu_);
    memset(out, 0, sizeof *out);
    out->submitted = submitted_;
    out->completed = completed_;
    out->queued = (int64_t)queue_.size();
    out->inflight = (int64_t)inflight_.size();
    out->iterations = iterations_;
    out->ligands_docked = ligands_;
    out->arena_ligands = lig_alloc_.cap();
    out->arena_atoms = atom_alloc_.cap();
    out->busy_ms = busy_ms_;
    out->budget_bytes = budget_;
    out->arena_budget_bytes = arena_budget_;
    out->admitted_bytes = admitted_bytes_;
    out->peak_admitted_bytes = peak_admitted_bytes_;
    out->peak_queued = peak_queued_;
}

void Server::shutdown() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        if (stop_ && !thread_.joinable()) return;
        stop_ = true;
        queue_.clear();
        cv_.notify_all();
        done_cv_.notify_all();
    }
    if (thread_.joinable()) thread_.join();
    for (int i = 0; i < 2; ++i) {
        Iteration& it = it_[i];
        if (it.stream) { (void)hipStreamSynchronize(it.stream); (void)hipStreamDestroy(it.stream); }
        if (it.done) (void)hipEventDestroy(it.done);
        if (it.h_order) (void)hipHostFree(it.h_order);
        if (it.h_res) (void)hipHostFree(it.h_res);
        it = Iteration();
    }
    if (up_stream_) { (void)hipStreamSynchronize(up_stream_); (void)hipStreamDestroy(up_stream_); }
    if (up_event_) (void)hipEventDestroy(up_event_);
    up_stream_ = nullptr;
    up_event_ = nullptr;
    for (void* p : dev_bufs_) (void)hipFree(p);
    dev_bufs_.clear();
    for (int32_t id : pocket_ids_) rt::pocket_use(id, -1);
    pocket_ids_.clear();
}

std::mutex g_srv_mu;
std::unordered_map<int64_t, std::shared_ptr<Server>> g_servers;
int64_t g_next_server = 1;

std::shared_ptr<Server> find_server(int64_t id) {
    std::lock_guard<std::mutex> lk(g_srv_mu);
    auto it = g_servers.find(id);
    return it == g_servers.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

int exs_server_create(const int32_t* pocket_ids, int n_pockets, const exs_search_params* params,
                      const exs_server_config* cfg, int64_t* server_out) {
    try {
        if (!params || !server_out) return rt::fail(EXS_EINVAL, "null argument");
        exs_server_config c{};
        if (cfg) c = *cfg;
        auto s = std::make_shared<Server>();
        if (int rc = s->create(pocket_ids, n_pockets, *params, c)) {
            s->shutdown();
            return rc;
        }
        std::lock_guard<std::mutex> lk(g_srv_mu);
        int64_t id = g_next_server++;
        g_servers[id] = s;
        *server_out = id;
        return EXS_OK;
    } catch (const std::exception& e) {
        return rt::fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_server_submit(int64_t server, const exs_ligand_batch* request, int64_t* request_out) {
    try {
        if (!request || !request_out) return rt::fail(EXS_EINVAL, "null argument");
        auto s = find_server(server);
        if (!s) return rt::fail(EXS_ENOENT, "unknown server %lld", (long long)server);
        return s->submit(*request, request_out);
    } catch (const std::exception& e) {
        return rt::fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_server_poll(int64_t server, int64_t request, int wait, float* best_score,
                    exs_pose_desc* desc, float* coords, double* latency_ms) {
    try {
        auto s = find_server(server);
        if (!s) return rt::fail(EXS_ENOENT, "unknown server %lld", (long long)server);
        return s->poll(request, wait, best_score, desc, coords, latency_ms);
    } catch (const std::exception& e) {
        return rt::fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}

int exs_server_get_stats(int64_t server, exs_server_stats* out) {
    if (!out) return rt::fail(EXS_EINVAL, "null argument");
    auto s = find_server(server);
    if (!s) return rt::fail(EXS_ENOENT, "unknown server %lld", (long long)server);
    s->stats(out);
    return EXS_OK;
}

int exs_server_destroy(int64_t server) {
    std::shared_ptr<Server> s;
    {
        std::lock_guard<std::mutex> lk(g_srv_mu);
        auto it = g_servers.find(server);
        if (it == g_servers.end()) return rt::fail(EXS_ENOENT, "unknown server %lld", (long long)server);
        s = it->second;
        g_servers.erase(it);
    }
    s->shutdown();
    return EXS_OK;
}

}  // extern "C"
