// Screening campaign on one device: a ligand library streamed through the serving engine.
//
// The paper's docking application is a pipeline -- a reader, a splitter, dockers and a
// writer joined by queues -- that keeps the GPUs fed while the host prepares the next ligands
// (Sec. 3.2), with several docking workers per GPU (Sec. 4.3).  Here, on one device:
//  * the library is validated and every ligand's search cost computed on all host threads
//    (the exact lookup / pair-test count of its search) while the server is created; the
//    ligands are then ordered pocket by pocket, most costly first within a pocket, and cut into
//    chunks (the first ones small and growing, so that the device starts while the next are
//    packed): an iteration reads few pockets' texel blocks, and the last launches hold the
//    cheapest ligands of the last pocket, so the device finishes evenly;
//  * packer threads gather chunks into CSR requests and submit them to a server, which packs
//    each on the submitting thread and docks the admitted requests in iterations of the
//    persistent kernel while the next chunks are being packed;
//  * the calling thread collects the chunks in submission order, scatters every ligand's best
//    score to its library index and keeps the hit list: the best ligands by score.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "exs.h"
#include "exs_internal.h"
#include "exs_pack.h"
#include "exs_runtime.h"

using namespace exs;

namespace {

// One chunk of the library in the CSR form a request takes.
struct Chunk {
    std::vector<int32_t> ids;                       // library indices of its ligands
    std::vector<int32_t> atom_off, bond_off, rot_off, bond_ij, rot_bond, pocket;
    std::vector<float> x, y, z;
    std::vector<uint8_t> type;
    exs_ligand_batch view() const {
        exs_ligand_batch b;
        b.n_ligands = (int32_t)ids.size();
        b.atom_offset = atom_off.data(); b.x = x.data(); b.y = y.data(); b.z = z.data();
        b.type = type.data(); b.bond_offset = bond_off.data(); b.bond_ij = bond_ij.data();
        b.rot_offset = rot_off.data(); b.rot_bond = rot_bond.data(); b.pocket_id = pocket.data();
        return b;
    }
};

void gather_chunk(const exs_ligand_batch& lib, const int32_t* ids, int n, Chunk& c) {
    c.ids.assign(ids, ids + n);
    c.atom_off.assign(1, 0); c.bond_off.assign(1, 0); c.rot_off.assign(1, 0);
    for (int t = 0; t < n; ++t) {
        const int l = ids[t];
        const int a0 = lib.atom_offset[l], a1 = lib.atom_offset[l + 1];
        const int b0 = lib.bond_offset[l], b1 = lib.bond_offset[l + 1];
        const int r0 = lib.rot_offset[l], r1 = lib.rot_offset[l + 1];
        c.x.insert(c.x.end(), lib.x + a0, lib.x + a1);
        c.y.insert(c.y.end(), lib.y + a0, lib.y + a1);
        c.z.insert(c.z.end(), lib.z + a0, lib.z + a1);
        c.type.insert(c.type.end(), lib.type + a0, lib.type + a1);
        if (b1 > b0) c.bond_ij.insert(c.bond_ij.end(), lib.bond_ij + 2 * (size_t)b0, lib.bond_ij + 2 * (size_t)b1);
        if (r1 > r0) c.rot_bond.insert(c.rot_bond.end(), lib.rot_bond + r0, lib.rot_bond + r1);
        c.pocket.push_back(lib.pocket_id[l]);
        c.atom_off.push_back(c.atom_off.back() + (a1 - a0));
        c.bond_off.push_back(c.bond_off.back() + (b1 - b0));
        c.rot_off.push_back(c.rot_off.back() + (r1 - r0));
    }
}

// Joins the threads it holds when it goes out of scope, so that an exception never leaves a
// joinable std::thread behind (which would terminate the process).
struct Joiner {
    std::vector<std::thread> ts;
    ~Joiner() {
        for (auto& t : ts)
            if (t.joinable()) t.join();
    }
};

}  // namespace

extern "C" int exs_campaign_run(const int32_t* pocket_ids, int n_pockets,
                                const exs_search_params* params, const exs_ligand_batch* library,
                                const exs_campaign_config* cfg, float* best_score,
                                int32_t* hits, int32_t* n_hits_out, exs_campaign_stats* stats) {
    try {
        if (!pocket_ids || n_pockets < 1 || !params || !library || !cfg || !n_hits_out)
            return rt::fail(EXS_EINVAL, "null argument");
        const exs_ligand_batch& lib = *library;
        const int L = lib.n_ligands;
        if (L < 0) return rt::fail(EXS_EINVAL, "negative ligand count");
        const int chunk = cfg->chunk_ligands > 0 ? cfg->chunk_ligands : 16384;
        const int packers = std::max(1, std::min(64, cfg->packers > 0 ? cfg->packers : 4));
        const double frac = cfg->hit_fraction > 0.0 ? cfg->hit_fraction : 0.01;
        if (!(frac <= 1.0)) return rt::fail(EXS_EINVAL, "hit_fraction must be in (0, 1]");
        const auto t0 = std::chrono::steady_clock::now();
        if (L > 0 && (!lib.atom_offset || !lib.x || !lib.y || !lib.z || !lib.type ||
                      !lib.bond_offset || !lib.rot_offset || !lib.pocket_id))
            return rt::fail(EXS_EINVAL, "null array in the library");
        if (L > 0 && (lib.atom_offset[0] != 0 || lib.bond_offset[0] != 0 || lib.rot_offset[0] != 0))
            return rt::fail(EXS_EINVAL, "atom_offset[0], bond_offset[0] and rot_offset[0] must be 0");
        // pockets: channels of each handle the campaign docks against
        std::vector<int> channels(n_pockets);
        for (int p = 0; p < n_pockets; ++p) {
            rt::PocketInfo info;
            if (!rt::pocket_info(pocket_ids[p], &info))
                return rt::fail(EXS_EINVAL, "unknown pocket %d", pocket_ids[p]);
            channels[p] = info.channels;
        }
        // the server is created (device buffers, streams) while the host threads validate
        int64_t server = 0;
        int create_rc = EXS_OK;
        std::string create_err;
        // a server created here is destroyed on every way out below (after the thread that
        // creates it has been joined: the guards go out of scope in reverse order)
        struct ServerGuard {
            int64_t* s;
            ~ServerGuard() {
                if (*s) (void)exs_server_destroy(*s);
            }
        } server_guard{&server};
        Joiner creator;
        creator.ts.emplace_back([&] {
            create_rc = exs_server_create(pocket_ids, n_pockets, params, &cfg->server, &server);
            if (create_rc != EXS_OK) create_err = exs_last_error();
        });
        // validate every ligand and take its search cost (host threads)
        std::vector<double> cost(L, 0.0);
        std::vector<int> rc_of(L, EXS_OK);
        std::vector<std::string> err_of(L);
        {
            std::atomic<int> next{0};
            auto work = [&]() {
                for (;;) {
                    const int l = next.fetch_add(1);
                    if (l >= L) return;
                    int slot = -1;
                    for (int p = 0; p < n_pockets; ++p)
                        if (pocket_ids[p] == lib.pocket_id[l]) { slot = p; break; }
                    if (slot < 0) {
                        rc_of[l] = EXS_EINVAL;
                        err_of[l] = "pocket not among the campaign's pockets";
                        continue;
                    }
                    const int a0 = lib.atom_offset[l], n = lib.atom_offset[l + 1] - a0;
                    const int b0 = lib.bond_offset[l], nb = lib.bond_offset[l + 1] - b0;
                    const int r0 = lib.rot_offset[l], nr = lib.rot_offset[l + 1] - r0;
                    if (n < 0 || nb < 0 || nr < 0 || (nb > 0 && !lib.bond_ij) || (nr > 0 && !lib.rot_bond)) {
                        rc_of[l] = EXS_EINVAL;
                        err_of[l] = "bad offsets";
                        continue;
                    }
                    try {   // an exception must not leave a worker thread
                        PackedLigand pk;
                        rc_of[l] = pack_ligand(n, lib.bond_ij + 2 * (size_t)b0, nb, lib.rot_bond + r0, nr,
                                               lib.type + a0, channels[slot], lib.x + a0, lib.y + a0,
                                               lib.z + a0, &pk, &err_of[l]);
                        if (rc_of[l]) continue;
                        std::vector<int16_t> m(pk.nrot);
                        for (int b = 0; b < pk.nrot; ++b) m[b] = (int16_t)pk.moving[b].count();
                        cost[l] = ligand_cost(pk.n, m.data(), pk.nrot, params->n_orient,
                                              params->torsion_steps, params->passes, params->n_offsets);
                    } catch (const std::exception& ex) {
                        rc_of[l] = EXS_ENOMEM;
                        err_of[l] = std::string("exception: ") + ex.what();
                    }
                }
            };
            // every host thread: nothing docks until this pass is done
            const int nth = std::max<int>(packers, std::min<int>(32, (int)std::thread::hardware_concurrency()));
            Joiner pool;
            for (int t = 1; t < nth; ++t) pool.ts.emplace_back(work);
            work();
        }
        const auto t_pre = std::chrono::steady_clock::now();
        creator.ts[0].join();
        for (int l = 0; l < L; ++l)
            if (rc_of[l]) return rt::fail(rc_of[l], "ligand %d: %s", l, err_of[l].c_str());
        if (create_rc != EXS_OK) return rt::fail(create_rc, "%s", create_err.c_str());
        // the order the chunks are cut from: pocket by pocket (an iteration then reads few
        // pockets' texel blocks: 185k -> 193k docks/s on the 100,000-ligand library over 15
        // pockets), most costly first within a pocket
        std::vector<int32_t> order(L);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            if (lib.pocket_id[a] != lib.pocket_id[b]) return lib.pocket_id[a] < lib.pocket_id[b];
            return cost[a] > cost[b];
        });
        // chunk c covers order[start[c], start[c+1]): the first chunks grow from 1,024 ligands,
        // doubling up to `chunk`, so that the device starts while the larger ones are packed
        std::vector<int> start(1, 0);
        for (int size = std::min(chunk, 1024); start.back() < L; size = std::min(chunk, 2 * size))
            start.push_back((int)std::min<int64_t>(L, (int64_t)start.back() + size));
        const int n_chunks = (int)start.size() - 1;
        std::vector<Chunk> chunks(n_chunks);
        std::vector<int64_t> handle(n_chunks, 0);
        std::vector<int> state(n_chunks, 0);          // 0 pending, 1 submitted, < 0 failed
        std::mutex mu;
        std::condition_variable cv;
        std::atomic<int> next{0};
        std::chrono::steady_clock::time_point t_first = t_pre;
        auto packer = [&]() {
            for (;;) {
                const int c = next.fetch_add(1);
                if (c >= n_chunks) return;
                int64_t h = 0;
                int rc;
                try {   // an exception must not leave a worker thread; the chunk fails instead
                    gather_chunk(lib, order.data() + start[c], start[c + 1] - start[c], chunks[c]);
                    const exs_ligand_batch view = chunks[c].view();
                    rc = exs_server_submit(server, &view, &h);
                } catch (const std::exception&) {
                    rc = EXS_ENOMEM;
                }
                std::lock_guard<std::mutex> lk(mu);
                if (c == 0) t_first = std::chrono::steady_clock::now();
                handle[c] = h;
                state[c] = rc == EXS_OK ? 1 : rc;
                cv.notify_all();
            }
        };
        Joiner threads;
        for (int t = 0; t < packers; ++t) threads.ts.emplace_back(packer);
        std::vector<float> best(L, INFINITY);
        std::vector<float> part;
        int status = EXS_OK;
        std::string msg;
        for (int c = 0; c < n_chunks; ++c) {
            int st;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return state[c] != 0; });
                st = state[c];
            }
            if (st < 0) {
                if (status == EXS_OK) { status = st; msg = exs_last_error(); }
                continue;
            }
            const Chunk& ch = chunks[c];
            part.assign(ch.ids.size(), 0.0f);
            const int rc = exs_server_poll(server, handle[c], 1, part.data(), nullptr, nullptr, nullptr);
            if (rc != EXS_OK) {
                if (status == EXS_OK) { status = rc; msg = exs_last_error(); }
                continue;
            }
            for (size_t t = 0; t < ch.ids.size(); ++t) best[ch.ids[t]] = part[t];
            chunks[c] = Chunk();   // the server holds its own copy since the submit
        }
        for (auto& t : threads.ts) t.join();
        exs_server_stats ss;
        memset(&ss, 0, sizeof ss);
        (void)exs_server_get_stats(server, &ss);
        (void)exs_server_destroy(server);
        server = 0;
        if (status != EXS_OK) return rt::fail(status, "campaign: %s", msg.c_str());
        // hit list: the best round(L * frac) ligands (at least one), score then index ascending
        const int n_hits = L == 0 ? 0 : std::max(1, std::min(L, (int)llround((double)L * frac)));
        std::vector<int32_t> ids(L);
        std::iota(ids.begin(), ids.end(), 0);
        auto better = [&](int a, int b) {
            const float sa = best[a] == best[a] ? best[a] : INFINITY;
            const float sb = best[b] == best[b] ? best[b] : INFINITY;
            return sa < sb || (sa == sb && a < b);
        };
        std::partial_sort(ids.begin(), ids.begin() + n_hits, ids.end(), better);
        if (hits) std::copy(ids.begin(), ids.begin() + n_hits, hits);
        *n_hits_out = n_hits;
        if (best_score) std::copy(best.begin(), best.end(), best_score);
        if (stats) {
            stats->ligands = L;
            stats->chunks = n_chunks;
            stats->iterations = ss.iterations;
            stats->hits = n_hits;
            stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            stats->prepass_seconds = std::chrono::duration<double>(t_pre - t0).count();
            stats->first_submit_seconds = std::chrono::duration<double>(t_first - t0).count();
        }
        return EXS_OK;
    } catch (const std::exception& e) {
        return rt::fail(EXS_ENOMEM, "exception: %s", e.what());
    }
}
