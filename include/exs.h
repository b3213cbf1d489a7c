/*
 * exs.h -- C ABI of the MI355X docking hot path (libexs.so).
 *
 * The library docks flexible ligands into rigid, pre-computed pocket grids and
 * keeps each ligand's best pose, the data-parallel core of the screening
 * method of the paper (Sec. 3.1 "The dock and score algorithm"; Sec. 3.2 "The
 * only information required to dock and score a ligand in the target binding
 * site is their description" -- every ligand x pocket pair is independent).
 *
 * Calls return 0 (EXS_OK) or a negative status; no C++ exception crosses the
 * ABI.  exs_last_error() gives a message for the calling thread's last
 * failure.  Every call is thread-safe.  Pointers are plain host pointers
 * unless a comment says "device".  The library owns every device buffer it
 * allocates (pocket grids, uploaded ligand batches, job results) until the
 * matching unload/release call.  A `stream` argument is a hipStream_t passed
 * as void* (NULL = the null stream); work and copies of a job are ordered on
 * the stream it was launched on.
 */
#ifndef EXS_H
#define EXS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
    EXS_OK = 0,
    EXS_EINVAL = -1,    /* invalid argument or input; nothing was queued     */
    EXS_ENOMEM = -2,    /* device or host allocation failed / over budget    */
    EXS_EDEVICE = -3,   /* a HIP runtime call failed                         */
    EXS_ENOTREADY = -4, /* job still running (only with wait = 0)            */
    EXS_ENOENT = -5     /* unknown pocket, batch or job handle               */
};

/* ---- texel storage of a pocket grid ------------------------------------- */
enum { EXS_F32 = 0, EXS_BF16 = 1, EXS_F16 = 2 };

/* ---- search flags -------------------------------------------------------- */
enum {
    EXS_FLAG_PERSISTENT = 1, /* one persistent launch pulling ligand tiles from work queues */
    EXS_FLAG_GRAPH = 2,      /* capture the job's launches in a hipGraph and replay it   */
    EXS_FLAG_RESCORE2 = 4    /* rescore the ranked poses with the second-stage score     */
};

/* ---- limits -------------------------------------------------------------- */
#define EXS_MAX_ATOMS 128     /* atoms per ligand                    */
#define EXS_MAX_ROT 32        /* rotatable bonds per ligand          */
#define EXS_MAX_CHANNELS 16   /* atom types (grid channels) per pocket */
#define EXS_MAX_ORIENT 1024   /* initial orientations per ligand     */
#define EXS_MAX_TOPK 32       /* poses rescored in FP64 per ligand   */

/* Library version string (static storage). */
const char* exs_version(void);

/* Message of the calling thread's last failed call ("" if none). */
const char* exs_last_error(void);

/*
 * Load a pocket grid and keep it resident on the current device.
 * The pocket is constant during a run and fetched once (Sec. 3.2: pocket data
 * is fetched once per process and placed where the implementation likes).
 *   values      [channels][nz][ny][nx] FP32 texels, x fastest; one channel per
 *               ligand atom type.  Host pointer, or device pointer when
 *               values_on_device = 1.  Copied; the caller keeps ownership.
 *   nx, ny, nz  texels per axis, each >= 2; nx * ny and nz below 2^23 (the search
 *               forms cell offsets with 24-bit multiplies).
 *   spacing_A   texel spacing (A), > 0.  Texel (i,j,k) sits at
 *               origin_A + spacing_A * (i,j,k); the pocket centre is the grid
 *               centre, where each ligand's centroid is placed.
 *   storage     EXS_F32, EXS_BF16 or EXS_F16: texels are stored in this type
 *               (round to nearest even); interpolation and accumulation run in
 *               FP32.  The search reads a copy expanded per cell: the 8
 *               corners of every cell together (32 B FP32, 16 B 16-bit), so a
 *               lookup is one contiguous block; this costs 8x (FP32) or 4x
 *               (16-bit) the bytes of the input, and each channel's expanded
 *               copy must stay below 2 GiB.  The FP32 master copy is always
 *               kept as well: it feeds the FP64 rescoring of the top poses.
 *   pocket_id_out  receives the handle.
 * Errors: EXS_EINVAL (bad sizes, nx * ny or nz of 2^23 or more, channels >
 * EXS_MAX_CHANNELS, non-finite texels, an expanded channel of 2 GiB or more),
 * EXS_ENOMEM, EXS_EDEVICE.
 */
int exs_load_pocket_grid(const float* values, int nx, int ny, int nz, int channels,
                         double spacing_A, const double origin_A[3], int storage,
                         int values_on_device, void* stream, int32_t* pocket_id_out);

/*
 * Unfold the uploaded ligands in place before docking (Sec. 3.1, first step: the
 * ligand is flattened, independently of the protein, by turning its torsional
 * bonds so that the sum of the distances between all its atoms grows).  Per
 * pass, every rotatable bond in list order tries the S-1 relative turns
 * 2*pi*s/S (S = torsion_steps: 8, 16 or 32) of the side without atom 0 and
 * keeps the largest distance sum if strictly larger (ties keep the shape, then
 * the lower s); `passes` passes (0..64).  FP32 on the device; a ligand whose
 * shape changed is then re-centred on its centroid (the docking places that
 * centroid at the pocket centre), one that kept its shape is left as uploaded.  Runs on `stream` and waits for it; order it
 * before any docking of the batch.
 *   turns_out  [passes * R] kept turn s per pass and rotatable bond (the
 *              batch's bonds in CSR order), or NULL.
 * Errors: EXS_EINVAL (torsion_steps, passes, device), EXS_ENOENT, EXS_EDEVICE.
 */
int exs_unfold_ligands(int64_t batch, int torsion_steps, int passes, void* stream,
                       int32_t* turns_out);

/* The batch's current coordinates [A][3] (centred on each ligand's centroid), to host. */
int exs_get_ligand_coords(int64_t batch, float* xyz);

/*
 * Ranked poses of a job run with rank_keep > 0 (Sec. 3.1, third step: cluster
 * leaders first, then the other poses, each by score).
 *   n_clusters  [L] clusters (leaders) per ligand, or NULL
 *   ranked      [L * rank_keep] orientation indices per ligand in ranked order,
 *               or NULL
 * wait = 0 returns EXS_ENOTREADY while the job runs.  Errors: EXS_ENOENT,
 * EXS_EINVAL (the job did not rank), EXS_EDEVICE.
 */
int exs_get_ranked_poses(int64_t job, int wait, int32_t* n_clusters, int32_t* ranked);

/*
 * Second-stage rescoring of a job run with rank_keep > 0 and EXS_FLAG_RESCORE2 (Sec. 3.1,
 * fourth step: the first poses of each ligand's ranked list are rescored with a richer score;
 * the paper's chemical score is not defined there, so the library uses a stand-in), in FP64 on
 * the device, each pose rebuilt from its descriptor:
 *   E2(X) = sum_i g(X_i, t_i)                                   grid term on the FP32 master
 *         + sum over pairs four or more bonds apart (or unbonded) of
 *           EXS_RESCORE2_CONTACT_EPS * ((s/d')^12 - 2 (s/d')^6), d' = max(d, s/2), s = clash cutoff
 *         + sum over rotatable bonds of EXS_RESCORE2_TORSION_W * (1 + cos 3 phi), phi the dihedral
 *           a-u-v-c, a / c the lowest-index neighbours of u / v other than each other (none, or an
 *           undefined dihedral: no term).
 * The ligand's final pose is the lowest E2 of its ranked list (ties: the earlier entry).
 *   score2       [L * rank_keep] E2 of the ranked poses, in ranked order (or NULL)
 *   best_orient  [L] orientation of the lowest E2 (or NULL)
 *   best_score2  [L] that E2 (or NULL)
 * wait = 0 returns EXS_ENOTREADY while the job runs.  Errors: EXS_ENOENT, EXS_EINVAL (the job
 * was run without the flag), EXS_EDEVICE.
 */
#define EXS_RESCORE2_CONTACT_EPS 0.25
#define EXS_RESCORE2_TORSION_W 0.5
int exs_get_rescored_poses(int64_t job, int wait, double* score2, int32_t* best_orient,
                           double* best_score2);

/*
 * Gather probe: the docking kernels' texel lookup (same per-cell blocks, loads and FP32
 * trilinear arithmetic) alone, to measure the lookup rate the search is held against
 * (Sec. 3.1: the score of a pose is a lookup per atom in the pocket's grids).
 * n_lanes lanes (rounded up to a multiple of 256) each do lookups_per_lane lookups (rounded
 * up to a multiple of batch), issued `batch` (8, 16 or 32) at a time independently of each
 * other, at 4, 3 or 2 waves per SIMD respectively, in runs of 32 lookups like the search's
 * lookups of one atom: a run keeps one channel (the next run takes the next) and starts at a
 * pseudo-random point of the cube of half edge half_edge_A (A) around the pocket centre; its
 * further points are independent points of the cube when walk_step_A = 0, else a walk of at
 * most walk_step_A per axis and step, clamped to the cube.  Runs on `stream` and waits for it.
 *   ms_out        device time of the probe kernel (HIP events).
 *   checksum_out  sum of the lanes' lookup sums (may be NULL).
 * Errors: EXS_EINVAL (sizes, batch, non-finite or negative lengths, pocket on another device),
 * EXS_ENOENT (unknown pocket), EXS_ENOMEM, EXS_EDEVICE.
 */
int exs_gather_probe(int32_t pocket_id, int64_t n_lanes, int lookups_per_lane, int batch,
                     float half_edge_A, float walk_step_A, uint32_t seed, void* stream,
                     float* ms_out, double* checksum_out);

/* Free a pocket's device grids.  Jobs still using it must be released first. */
int exs_unload_pocket(int32_t pocket_id);

/*
 * A batch of ligands in CSR form (host pointers; every array is read during
 * exs_upload_ligands and not kept).  A ligand is its atoms' positions and
 * types and its bonds (Sec. 4.1: atom positions, types and bonds), plus the
 * list of torsional (rotatable) bonds (Sec. 3.1).
 *   atom_offset [L+1]  ligand l owns atoms atom_offset[l] .. atom_offset[l+1]-1
 *   x, y, z     [A]    input conformation (A)
 *   type        [A]    atom type = grid channel, < channels of its pocket
 *   bond_offset [L+1], bond_ij [2*nb]   bonds as pairs of ligand-local indices
 *   rot_offset  [L+1], rot_bond [R]     rotatable bonds, as indices into the
 *                                       ligand's own bond list, in search order
 *   pocket_id   [L]    pocket handle each ligand is docked against
 * A rotatable bond must be a bridge of the bond graph (not in a ring) with
 * atom 0 on one side; the side without atom 0 turns.
 */
typedef struct {
    int32_t n_ligands;
    const int32_t* atom_offset;
    const float* x;
    const float* y;
    const float* z;
    const uint8_t* type;
    const int32_t* bond_offset;
    const int32_t* bond_ij;
    const int32_t* rot_offset;
    const int32_t* rot_bond;
    const int32_t* pocket_id;
} exs_ligand_batch;

/*
 * Validate a ligand batch, pack its topology (bond-distance exclusion masks,
 * moving-atom masks of every rotatable bond, per-ligand cost) and upload it to
 * the device on `stream`.  All-or-nothing: any invalid ligand gives EXS_EINVAL
 * naming the ligand, and nothing is uploaded.  Invalid: n < 1 or
 * n > EXS_MAX_ATOMS, more than EXS_MAX_ROT rotatable bonds, an atom type not
 * below its pocket's channel count, a bond or rotatable-bond index out of
 * range, a rotatable bond in a ring or not connected to atom 0, an unknown
 * pocket.  batch_out receives the handle.
 */
int exs_upload_ligands(const exs_ligand_batch* batch, void* stream, int64_t* batch_out);

/* Free an uploaded batch (jobs using it must be released first). */
int exs_release_ligands(int64_t batch);

/*
 * Host-only view of how the library reads one ligand (no device call): the
 * same validation as exs_upload_ligands (with `channels` standing for the
 * pocket's channel count) and the packed topology it uploads.  Outputs (any
 * may be NULL):
 *   excl   [4*n]      exclusion row of atom i as 4 x uint32: bit j%32 of word
 *                     j/32 set = pair (i, j) is left out of the clash term
 *                     (bond distance <= 3, i.e. 1-2, 1-3, 1-4 pairs, or i == j)
 *   rot_uv [2*nrot]   u, v of each rotatable bond, u on atom 0's side
 *   moving [4*nrot]   atoms that turn with the bond (v's side, v excluded)
 */
int exs_pack_topology(int n, const float* x, const float* y, const float* z, const uint8_t* type,
                      int channels, int nb, const int32_t* bond_ij, int nrot,
                      const int32_t* rot_bond, uint32_t* excl, int32_t* rot_uv, uint32_t* moving);

/*
 * Search settings (Sec. 3.1: greedy optimisation with restarts; the paper
 * uses 256 initial poses per ligand).
 *   n_orient       K initial orientations (Fibonacci sphere), 1..EXS_MAX_ORIENT
 *   torsion_steps  S: each rotatable bond tries the S-1 turns 2*pi*s/S;
 *                  one of 8, 16, 32
 *   passes         P optimisation passes (all bonds, then the rigid offsets)
 *   n_offsets      1 (no rigid offsets) or 27 (offset_step_A * {-1,0,1}^3)
 *   clash_cutoff_A, clash_penalty   penalty per non-1-2/1-3/1-4 atom pair
 *                  closer than the cutoff
 *   top_k          0, or 1..EXS_MAX_TOPK: rescore each ligand's top_k poses in
 *                  FP64 from the FP32 master grid and pick the best by FP64
 *   poses_per_lane 0 = auto, or 1, 2, 4 (orientations searched by one lane)
 *   ligands_per_wg 0 = auto, or 1, 2, 4, 8 (ligands per workgroup)
 *   flags          EXS_FLAG_* bits
 *   cluster_rmsd_A, rank_keep   ranking of each ligand's K final poses (Sec. 3.1,
 *                  third step), when rank_keep > 0: poses by score (lower
 *                  first, ties to the lower orientation), greedy clusters (a pose
 *                  leads a new cluster unless its RMSD, over all atoms in the
 *                  pocket frame, to an earlier leader is below cluster_rmsd_A),
 *                  then the leaders by score followed by the other poses by
 *                  score; the first rank_keep (<= n_orient) orientations of that
 *                  list are kept (exs_get_ranked_poses).  0 = no ranking.  Not
 *                  supported by the serving engine.
 */
typedef struct {
    int32_t n_orient;
    int32_t torsion_steps;
    int32_t passes;
    int32_t n_offsets;
    float offset_step_A;
    float clash_cutoff_A;
    float clash_penalty;
    int32_t top_k;
    int32_t poses_per_lane;
    int32_t ligands_per_wg;
    int32_t flags;
    float cluster_rmsd_A;
    int32_t rank_keep;
} exs_search_params;

/*
 * A pose descriptor: the pose it names is
 *   X = c + offset_step * tau + R_orient * FK_theta(X0 - mean(X0))
 * where c is the pocket centre, R_orient the orientation's rotation and
 * FK_theta turns each rotatable bond's moving side by theta[b] * 2*pi/S.
 * Poses are deterministic, so a descriptor regenerates its pose (Sec. 3.1).
 */
typedef struct {
    float score;        /* FP32 search score (lower is better)             */
    float pad0;
    double score_fp64;  /* FP64 rescoring score, or NaN when top_k = 0      */
    int32_t orient;     /* orientation index k                              */
    int8_t tau[3];      /* accumulated rigid offsets, units of offset_step  */
    uint8_t n_rot;      /* rotatable bonds of the ligand                    */
    uint8_t theta[EXS_MAX_ROT]; /* torsion of each rotatable bond, units 2*pi/S */
} exs_pose_desc;

/*
 * Dock every ligand of an uploaded batch against its pocket, asynchronously
 * on `stream` (Sec. 3.1: per ligand, restarts from the initial orientations,
 * each a greedy optimisation of the torsions and the rigid roto-translation
 * driven by the pocket score; the ligand's score is its best pose's; Sec. 3.2:
 * every ligand x pocket pair is independent).  One launch per pocket (default),
 * or one persistent launch over all pockets (EXS_FLAG_PERSISTENT).  job_out
 * receives the handle.  The batch and its pockets must stay loaded until the job
 * is released.
 * Errors: EXS_EINVAL (settings), EXS_ENOENT (unknown batch or a pocket
 * unloaded since upload), EXS_ENOMEM, EXS_EDEVICE.
 */
int exs_dock_batch(int64_t batch, const exs_search_params* params, void* stream,
                   int64_t* job_out);

/*
 * Best pose of every ligand of a job (the ligand's score is the score of its
 * best pose, Sec. 3.1).  wait = 1 blocks until the job is done; wait = 0
 * returns EXS_ENOTREADY while it runs.  Outputs (host, any may be NULL):
 *   best_score [L]          FP32 score of the best pose (FP64 value when top_k > 0,
 *                           rounded to float)
 *   desc       [L]          descriptor of the best pose
 *   coords     [A*3]        best-pose coordinates, atom-major x,y,z
 *   topk       [L*top_k]    the top_k poses by FP32 score, ascending (top_k > 0)
 */
int exs_get_best_poses(int64_t job, int wait, float* best_score, exs_pose_desc* desc,
                       float* coords, exs_pose_desc* topk);

/*
 * Final score and descriptor of every orientation of every ligand:
 * score [L*K], desc [L*K] (host, either may be NULL).  Waits for the job.
 */
int exs_get_orientation_results(int64_t job, float* score, exs_pose_desc* desc);

/*
 * Dock an uploaded batch without allocating device memory: for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid allocation).  The
 * search of exs_dock_batch (same settings, same per-ligand results bit for bit) as one
 * persistent launch on `stream`, enqueued and not waited for; no job handle.  Its
 * intermediate buffers (orientation table, work counter, every orientation's score and
 * descriptor, per-workgroup pose coordinates) live in one static device buffer of
 * EXS_NOALLOC_SCRATCH_BYTES that the library holds on every device it runs this call on, until
 * the process ends.  Calls on one device share that buffer: calls that overlap on a device
 * race, so order them (for example on one stream); the batch and its pockets must stay loaded
 * until the stream has finished the call's work.
 *   params       top_k = 0, rank_keep = 0, flags 0 or EXS_FLAG_PERSISTENT (the launch is
 *                persistent either way); tiles as for exs_dock_batch
 *   best_score   [L] device, FP32 score of each ligand's best pose
 *   best_orient  [L] device, its orientation
 *   best_tau     [L] device, its rigid offsets packed as (uint8)tau_x | tau_y << 8 | tau_z << 16
 *   best_theta   [R] device, its torsion of each rotatable bond (the batch's bonds, CSR order)
 *   best_coords  [A*3] device, its coordinates, atom-major x, y, z
 * Errors: EXS_EINVAL (settings, null outputs, or a batch whose per-orientation results
 * L * K * 8 + R * K bytes plus one workgroup's pose scratch exceed the buffer: split it),
 * EXS_ENOENT (unknown batch, unloaded pocket), EXS_EDEVICE.
 */
#define EXS_NOALLOC_SCRATCH_BYTES (256u << 20)
int exs_dock_batch_noalloc(int64_t batch, const exs_search_params* params, void* stream,
                           float* best_score, int32_t* best_orient, int32_t* best_tau,
                           uint8_t* best_theta, float* best_coords);

/* Device time of the job's kernels in ms (waits for the job). */
int exs_job_elapsed_ms(int64_t job, float* ms);

/*
 * Device time of each step of the job in ms (waits for the job), from events recorded between
 * its kernels on the job's stream: the search (Sec. 3.1, second step), the ranking of the final
 * poses (third step) and the second-stage rescoring (fourth step).  A step the job did not run
 * reads -1.  A job launched from a graph (EXS_FLAG_GRAPH) or without ranking is not staged:
 * dock_ms is then the whole job, as exs_job_elapsed_ms gives it.
 * Errors: EXS_ENOENT (unknown job), EXS_EINVAL (null output), EXS_EDEVICE.
 */
int exs_job_stage_ms(int64_t job, float* dock_ms, float* rank_ms, float* rescore2_ms);

/* Free a job's device results. */
int exs_release_job(int64_t job);

/* ---- serving: continuous batching of docking requests -------------------
 *
 * A server keeps a set of resident pockets and an arena of device memory
 * (sized by hbm_budget_bytes) for admitted requests.  A request is a ligand
 * batch (exs_ligand_batch, pocket_id = handles of the server's pockets); it is
 * validated and packed on the submitting thread (an invalid request fails
 * alone with EXS_EINVAL and nothing is queued), queued, admitted when its
 * ligands fit in the arena (FIFO; a request that does not fit waits: this is
 * the backpressure of the budget), and docked by iteration launches of the
 * persistent kernel over the not-yet-docked ligands of every admitted request
 * (up to max_iter_ligands per launch, up to max_inflight_iters launches in
 * flight on separate streams, so requests arriving while others run join the
 * next launch and overlap on the device).  Results do not depend on what a
 * request is batched with.  Mirrors the paper's staged pipeline with queues
 * and several GPU workers per device (Sec. 3.2, 4.3).
 */
typedef struct {
    int64_t hbm_budget_bytes;   /* device memory for scratch + admitted requests (0: 2 GiB);
                                   clamped to the free device memory (hipMemGetInfo) less a
                                   reserve of max(1 GiB, 5 % of the device) at creation */
    int32_t max_iter_ligands;   /* ligands per iteration launch (0: four waves of workgroups) */
    int32_t max_inflight_iters; /* 1 or 2 (0: 2)                                             */
    int32_t max_arena_ligands;  /* cap on the arena's ligand slots (0: from the budget)       */
    int32_t pad;
} exs_server_config;

typedef struct {
    int64_t submitted, completed, queued, inflight;
    int64_t iterations, ligands_docked;
    int64_t arena_ligands, arena_atoms;   /* arena capacity */
    double busy_ms;                       /* summed wall time of iteration launches */
    int64_t budget_bytes;                 /* HBM budget after the free-memory clamp */
    int64_t arena_budget_bytes;           /* its part for admitted requests */
    int64_t admitted_bytes;               /* bytes of the requests admitted now */
    int64_t peak_admitted_bytes;          /* the most ever admitted at once */
    int64_t peak_queued;                  /* the most requests ever waiting for admission */
} exs_server_stats;

/* Start a server on the current device for the given pockets (same texel
 * storage) and search settings.  Errors: EXS_EINVAL, EXS_ENOMEM (budget below
 * the fixed iteration scratch), EXS_EDEVICE. */
int exs_server_create(const int32_t* pocket_ids, int n_pockets, const exs_search_params* params,
                      const exs_server_config* cfg, int64_t* server_out);

/* Queue one request (host arrays, copied).  It is admitted when its device bytes
 * (L * (76 + 12 K + 28 top_k) + 68 A + R * (21 + K + top_k)) fit in the arena budget beside
 * the requests admitted before it (FIFO).  EXS_ENOMEM if it can never fit.  request_out
 * receives its handle. */
int exs_server_submit(int64_t server, const exs_ligand_batch* request, int64_t* request_out);

/* Results of a request: best_score [L], desc [L], coords [A*3] (any may be
 * NULL) and its latency (submit to completion, ms).  wait = 0 gives
 * EXS_ENOTREADY while it is queued or running.  A successful poll releases
 * the request. */
int exs_server_poll(int64_t server, int64_t request, int wait, float* best_score,
                    exs_pose_desc* desc, float* coords, double* latency_ms);

int exs_server_get_stats(int64_t server, exs_server_stats* out);

/* Stop the server: requests not yet admitted are dropped; admitted ones are docked to the
 * end before it returns. */
int exs_server_destroy(int64_t server);

/* ---- campaign: a library screened on one device ---------------------------
 *
 * The paper's docking application is a pipeline of a reader, a splitter, docking workers and a
 * writer joined by queues, which keeps the GPUs fed while the host prepares ligands (Sec. 3.2,
 * several workers per GPU in Sec. 4.3).  exs_campaign_run does that on one device for a library
 * in host memory: it validates every ligand and computes its search cost on the host's
 * threads, cuts the library -- pocket by pocket, most costly ligands first within a pocket --
 * into chunks of chunk_ligands (the first ones 1,024, 2,048, ... ligands, doubling up to that,
 * so the device starts early), and streams the chunks through a server (exs_server_*, created
 * while the library is validated) configured by `server`: `packers` threads pack and submit
 * chunks while earlier ones dock.  It returns when every ligand is docked.
 */
typedef struct {
    int32_t chunk_ligands;      /* ligands per chunk (0: 16384)                              */
    int32_t packers;            /* host threads that validate, pack and submit (0: 4)       */
    double hit_fraction;        /* hits kept: the best round(L * hit_fraction), at least 1
                                   (0: 0.01, the top 1 %)                                    */
    exs_server_config server;   /* the serving engine the chunks go through                 */
} exs_campaign_config;

typedef struct {
    int64_t ligands, chunks, iterations;
    int32_t hits, pad;
    double seconds;             /* wall time of the call */
    double prepass_seconds;     /* of it, the validation and cost pass over the library */
    double first_submit_seconds;/* call start to the first chunk submitted */
} exs_campaign_stats;

/* Screen `library` (host CSR batch; pocket_id = handles among pocket_ids, all of one texel
 * storage) with `params` (top_k allowed: the best score is then the FP64 one; rank_keep must be
 * 0).  Outputs: best_score [L] (host, or NULL) each ligand's best score, by library index; hits
 * [round(L * hit_fraction)] (host, or NULL) the library indices of the best ligands, best first
 * (ties to the lower index, NaN last); *n_hits_out their count; stats (or NULL).  All-or-nothing
 * validation: an invalid ligand gives EXS_EINVAL naming it before any docking.  Errors:
 * EXS_EINVAL, EXS_ENOMEM (the server's budget, or a chunk larger than its arena), EXS_EDEVICE. */
int exs_campaign_run(const int32_t* pocket_ids, int n_pockets, const exs_search_params* params,
                     const exs_ligand_batch* library, const exs_campaign_config* cfg,
                     float* best_score, int32_t* hits, int32_t* n_hits_out,
                     exs_campaign_stats* stats);

#ifdef __cplusplus
}
#endif
#endif /* EXS_H */
