/*
 * ffs.h -- C ABI of the MI355X (gfx950) library for the dual heterogeneous
 * island genetic algorithm on the flexible flow shop (Luo & El Baz,
 * arXiv 1903.10722).
 *
 * Problem (paper, Section 3): J jobs pass S stages in the same order; stage s
 * has M_s machines; every operation runs on one machine of its stage without
 * preemption.  In this library the machines of a stage are identical (one
 * processing time p[j][s] per job and stage), there are no release or due
 * dates, and the objective is the makespan C_max.  A solution is a job
 * permutation, decoded by list scheduling: stage 1 in permutation order,
 * every later stage first-in-first-out by the previous stage's completion
 * time (ties: earlier dispatch first), each job to the machine that becomes
 * free first (ties: lowest machine index).
 *
 * Conventions for every function:
 *   - Return value: FFS_OK (0) or a negative FFS_E* status.  No C++
 *     exception crosses this boundary.  On error, outputs are left untouched
 *     and ffs_last_error() describes the failure.
 *   - Ownership: input arrays are read during the call only (copied where
 *     kept); the caller keeps ownership of every buffer it passes.  The
 *     library allocates no device memory: the caller supplies one device
 *     workspace (ffs_workspace_size / ffs_bind_workspace) and owns it.
 *   - Streams: all device work of a context is enqueued on the HIP stream
 *     given at ffs_ctx_create, in call order.  Functions marked "(syncs)"
 *     wait for that stream before returning.
 *   - Threading: a context must not be used from two threads at once.
 *   - Pointers are host pointers unless the argument says "device".
 */
#ifndef FFS_H
#define FFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ffs_ctx ffs_ctx;

enum {
    FFS_OK = 0,
    FFS_EINVAL = -1,        /* an argument is out of range or inconsistent      */
    FFS_ENOMEM = -2,        /* the bound workspace is too small                 */
    FFS_EDEVICE = -3,       /* a HIP call failed or a kernel reported a fault   */
    FFS_ESTATE = -4,        /* call out of order (e.g. evolve before bind)      */
    FFS_EUNSUPPORTED = -5   /* valid problem outside this library's limits        */
};

/* One island.  Paper Section 4.1: island A runs the cellular GA, island B the
 * pseudo GA, each with its own crossover / mutation rates (parameter level).
 *   kind 0 (cellular): individuals on a rows x cols torus (rows, cols >= 3);
 *          each cell picks two parents in its von Neumann neighbourhood
 *          (self, north, east, south, west) by `selection`, applies order
 *          crossover with probability p_c and a swap mutation with
 *          probability p_m, and keeps the child only if its makespan is
 *          strictly lower.  selection (the paper only says two individuals
 *          of the nearby area are selected, Section 4.2):
 *            0: the two best by (makespan, neighbourhood order);
 *            1: the cell itself and the best of north, east, south, west;
 *            2: two binary tournaments: draws 6 and 7 of the cell's CELL
 *               block each give x uniform in [0, 25), the neighbourhood
 *               positions x / 5 and x % 5, and the better of the two by
 *               (makespan, position) is the parent.
 *          sweep (the paper gives one thread per cell, Section 4.2, and no
 *          update order): 0 = synchronous, every cell from generation g-1;
 *          1 = asynchronous line sweep, the cells in row-major order, each
 *          seeing the cells before it already updated in this generation
 *          (run as one launch per anti-diagonal r + c; needs the lane
 *          mapping's limits: at most 8 machines per stage and 160 in all;
 *          no pre-screen).
 *   kind 1 (pseudo): `size` individuals (even, >= 2) in fixed pairs; each pair
 *          mates its better member with that member's complement (the
 *          reversed permutation) and both children replace the pair.
 * Island sizes are limited to 16384 individuals in this library.             */
typedef struct {
    int32_t kind;
    int32_t rows, cols;   /* kind 0 */
    int32_t size;         /* kind 1; ignored for kind 0 (rows*cols)           */
    double p_c, p_m;      /* in [0, 1]                                        */
    int32_t selection;    /* kind 0: 0, 1 or 2 (above); kind 1: must be 0     */
    int32_t sweep;        /* kind 0: 0 or 1 (above); kind 1: must be 0        */
} ffs_island_spec;

/* Migration (paper Section 4.3).  Islands are paired (i, i + H), H = half the
 * island count, which must be even.  Every `migration_interval` generations
 * (0 = never) one migration epoch runs:
 *   topology 0: for each pair, the penetration rule of equations (1)-(2):
 *               fitness = E - best makespan with E = sum of all processing
 *               times; migrate iff the fitnesses differ and 1 - beta < theta;
 *               ceil(alpha * min(N_A, N_B)) best individuals of the fitter
 *               island overwrite as many worst individuals of the other.
 *   topology 1: first a ring (island order 0, H, 1, H+1, ...): every island's
 *               best overwrites its successor's worst; then topology 0.
 *   topology 2: the rule of topology 0 on every edge of that ring in turn,
 *               (0, H), (H, 1), (1, H+1), ..., (2H-1, 0), each edge on the
 *               state the previous edges left (two islands: the one edge
 *               (0, 1)); an alternative reading for more than two islands. */
typedef struct {
    int32_t migration_interval;
    int32_t topology;
    double theta;         /* in [0, 1]; the paper's experiments use 1.0       */
    /* Learned pre-screen of the cellular island (0 or 1 = off, 2..64 = on; at
     * most one instance per context).  Each cell builds `surrogate_k`
     * candidate children from candidate streams 0..k-1 (stream 0 is the
     * plain GA's), a 256-512-512-1 BF16 MLP ranks them, and only the best
     * ranked one is decoded exactly and replaces the cell if strictly
     * better.  The first `surrogate_warmup` generations use stream 0 only.
     * After every generation each decoded cellular child (features, exact
     * (C - LB) / LB) enters a replay ring of 65536 rows and the network
     * takes one Adam step (lr 1e-3) on 4096 rows sampled from it.  Makespans
     * always come from exact decodes.                                       */
    int32_t surrogate_k;
    int32_t surrogate_warmup;
} ffs_ga_config;

/* Create / destroy a context bound to a HIP stream (hipStream_t as void*;
 * NULL = the null stream).  The device current at creation is used.        */
int ffs_ctx_create(void *hip_stream, ffs_ctx **out);
void ffs_ctx_destroy(ffs_ctx *ctx);

/* Text of the last error on this context (never NULL; static storage owned
 * by the context, valid until the next call on it).                         */
const char *ffs_last_error(const ffs_ctx *ctx);

/* Register one FFS instance with its islands (Section 3's problem statement).
 *   n_jobs >= 1, n_stages in [1, 64]; machines[n_stages], each in [1, 16];
 *   p[n_jobs * n_stages], job-major (p[j * n_stages + s]), each in [1, 65535];
 *   islands[n_islands], n_islands even >= 2 (or 1 with no migration);
 *   seed: the random stream key together with the instance id.
 * Limits of this library: n_jobs <= 4096, and the packed schedule key
 * needs sum(p) < 2^(32 - ceil(log2 n_jobs)) - 1 (FFS_EUNSUPPORTED otherwise).
 * Must be called before ffs_bind_workspace.  *out_instance_id = 0, 1, ...  */
int ffs_create_instance(ffs_ctx *ctx, int32_t n_jobs, int32_t n_stages,
                        const int32_t *machines, const int32_t *p,
                        const ffs_island_spec *islands, int32_t n_islands,
                        const ffs_ga_config *cfg, uint64_t seed,
                        int32_t *out_instance_id);

/* Tile shape of the generation kernels: waves per workgroup (1, 2, 4 or 8).
 * Results never depend on it.  May be called before or after
 * ffs_bind_workspace (after: waits for the stream, then re-plans the
 * workgroups; FFS_EUNSUPPORTED if the tile does not fit in LDS).            */
int ffs_set_waves_per_block(ffs_ctx *ctx, int32_t waves);

/* Lane mapping of the decode (Section 4.2: fitness evaluations are
 * independent, so they can be spread over the GPU in any arrangement).
 *   0: per stage -- a group of n_stages lanes decodes one chromosome, one
 *      lane per stage, jobs handed from stage to stage between lanes;
 *   1: per lane -- one lane decodes one chromosome through all stages;
 *  -1: automatic (the default): per lane when every instance fits it and the
 *      context holds at least 131072 individuals (ffs_evaluate: at least
 *      65536 rows of at least 8 stages), per stage otherwise.
 * The per-lane mapping needs at most 8 machines per stage, a sum of machine
 * counts <= 160 and no pre-screen; otherwise per stage is used whatever the
 * request.  Results never depend on the mapping.  May be called before or
 * after ffs_bind_workspace (after: waits for the stream and re-plans).
 * ffs_get_mapping reports the mapping the generation launches use: 0 or 1,
 * or 2 when instances use different ones (ffs_set_instance_tile).          */
int ffs_set_mapping(ffs_ctx *ctx, int32_t mapping);
int ffs_get_mapping(ffs_ctx *ctx, int32_t *used);

/* Launch chains (islands are independent between migration epochs, Section
 * 4.3): with 2, the islands of every instance alternate between two groups
 * whose generations of a migration epoch run as two launch sequences side by
 * side (two branches of the captured epoch graph, joined before the epoch's
 * migration), so one group's next generation fills the GPU while the other's
 * last workgroups finish.  Each group keeps its own best-ever record per
 * instance; ffs_best returns the better of the two by (makespan, generation,
 * island, slot), which is the record a single sequence keeps.  1 = one
 * sequence.  -1 (default) = automatic: 2 when allowed and the context holds
 * at least 131072 individuals (a generation larger than one round of
 * resident waves; smaller ones only pay a second launch).  Two chains need
 * a single launch class (all instances with the same tile and LDS class), no
 * line-sweep island and no pre-screen; otherwise one is used whatever the
 * request.  Results never depend on it.  Eager generations (no graph) launch
 * the two groups in turn.  May be called before or after ffs_bind_workspace
 * (after: waits for the stream and re-plans).  ffs_get_chains reports the
 * number in use.                                                            */
int ffs_set_chains(ffs_ctx *ctx, int32_t chains);
int ffs_get_chains(ffs_ctx *ctx, int32_t *used);

/* Tile of one instance (overrides the context's for it): mapping -1 / 0 / 1
 * as in ffs_set_mapping (-1: the context's), waves per workgroup 1, 2, 4, 8
 * (0: the context's; narrowed automatically while a workgroup would exceed
 * the device's LDS).  Instances with the same tile and similar LDS needs
 * share one launch per generation.  Results never depend on tiles.  Before
 * or after ffs_bind_workspace (after: waits for the stream and re-plans).  */
int ffs_set_instance_tile(ffs_ctx *ctx, int32_t inst, int32_t mapping, int32_t waves);

/* When a generation has several launches (instances of different tiles or
 * LDS needs), run them side by side on streams forked from and joined back
 * into the context's stream (parallel branches of the captured graph), or
 * one after another (enable = 0).  Default: side by side.  Results are
 * identical.                                                               */
int ffs_set_concurrent(ffs_ctx *ctx, int32_t enable);

/* ffs_evolve replays whole migration epochs (or chunks of 16 generations
 * when nothing migrates) from one captured HIP graph when enable != 0 (the
 * default), the stream is not the null stream, timing is off, and every
 * migrating instance has the same interval.  Results are identical.        */
int ffs_set_graphs(ffs_ctx *ctx, int32_t enable);

/* Device bytes needed by all instances created so far.                      */
int ffs_workspace_size(const ffs_ctx *ctx, size_t *bytes);

/* Bind a device workspace (>= ffs_workspace_size bytes, 256-byte aligned,
 * owned by the caller, kept alive until ffs_ctx_destroy) and enqueue
 * generation 0: random permutations (Fisher-Yates), complementary pairs on
 * pseudo islands, decode of every individual, best-ever record.  (syncs)    */
int ffs_bind_workspace(ffs_ctx *ctx, void *device_ptr, size_t bytes);

/* Decode `count` permutations of instance `inst` (paper Section 3; the
 * rule is stated at the top of this header).
 *   perms: device, int32 [count * n_jobs], row-major, one permutation per row;
 *   out_makespans: device, int32 [count].
 * A row that is not a permutation of 0..n_jobs-1 gets makespan -1 and the
 * call returns FFS_EINVAL after the valid rows are written.  (syncs)        */
int ffs_evaluate(ffs_ctx *ctx, int32_t inst, const int32_t *perms, int32_t count,
                 int32_t *out_makespans);

/* ffs_evaluate with host pointers: perms int32 [count * n_jobs] and
 * out_makespans int32 [count] in host memory.  Rows are copied through a
 * 4 MiB staging region of the workspace in chunks (pageable copies on the
 * context's stream), so the figure it gives includes the host transfers.
 * Same validation and status as ffs_evaluate.  (syncs)                      */
int ffs_evaluate_host(ffs_ctx *ctx, int32_t inst, const int32_t *perms, int32_t count,
                      int32_t *out_makespans);

/* ffs_evaluate for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no context, no workspace, and no hipMalloc / hipFree or other allocating
 * routine.  The instance is given here and used for this call only:
 *   machines: host, int32 [n_stages], each in [1, 16];
 *   p: host, int32 [n_jobs * n_stages], job-major, each in [1, 65535];
 *   perms: device, int32 [count * n_jobs]; out_makespans: device, int32 [count];
 *   hip_stream: a stream of the current device (NULL = the null stream).
 * Limits: n_jobs <= 4096, n_stages <= 64, the packed-key limit of
 * ffs_create_instance, and 256 + 256 + 4 n S + S * n_pad * w bytes of state
 * within 1 MiB (n_pad = n rounded up to 32, w = 1 if every p <= 255 else 2),
 * else FFS_EUNSUPPORTED.  The state lives in a statically allocated device
 * array (1 MiB per GPU, held until the process ends) that every call on a
 * GPU shares: calls that overlap on one GPU (other threads, other streams)
 * race and must be serialised by the caller.  Same rows, makespans and
 * statuses as ffs_evaluate (invalid rows: -1 and FFS_EINVAL); no error text
 * (there is no context).  (syncs)                                          */
int ffs_evaluate_noalloc(void *hip_stream, int32_t n_jobs, int32_t n_stages, const int32_t *machines,
                         const int32_t *p, const int32_t *perms, int32_t count, int32_t *out_makespans);

/* Run `generations` generations of every instance.  Per generation: every
 * cellular cell and pseudo pair produces its children from generation g-1
 * (synchronous update), the best-ever record is updated, and when
 * g % migration_interval == 0 a migration epoch follows.  evolve(a) then
 * evolve(b) equals evolve(a + b).  Asynchronous (enqueued on the stream).  */
int ffs_evolve(ffs_ctx *ctx, int32_t generations);

/* Run one migration epoch of instance `inst` now, outside the schedule.    */
int ffs_migrate(ffs_ctx *ctx, int32_t inst);

/* Best-ever individual of `inst`: makespan, the generation it was found,
 * and (if out_perm != NULL) its permutation, int32 [n_jobs].  (syncs)      */
int ffs_best(ffs_ctx *ctx, int32_t inst, int32_t *out_makespan, int32_t *out_generation,
             int32_t *out_perm);

/* Current population of one island: genes int32 [size * n_jobs] (row per
 * slot; cellular slot = row * cols + col) and makespans int32 [size];
 * either pointer may be NULL.  (syncs)                                      */
int ffs_get_population(ffs_ctx *ctx, int32_t inst, int32_t island, int32_t *genes,
                       int32_t *makespans);

/* Generations completed so far (0 after bind).                              */
int ffs_generation(const ffs_ctx *ctx, int32_t *out_generation);

/* Migration counters of `inst` since bind: epochs with a migration, and
 * individuals moved by the adaptive rule (ring moves not counted).  (syncs) */
int ffs_migration_counters(ffs_ctx *ctx, int32_t inst, int64_t *migrations, int64_t *migrants);

/* Timing of the generation kernel: when enabled, every launch of it is
 * bracketed by HIP events on the context's stream; ffs_kernel_time returns
 * the summed milliseconds and the launch count since enabling.  (syncs)     */
int ffs_set_timing(ffs_ctx *ctx, int32_t enable);
int ffs_kernel_time(ffs_ctx *ctx, double *total_ms, int64_t *launches);

/* ---- checkpoint / restore --------------------------------------------------
 * A checkpoint is a host byte image of the whole context at its current
 * generation: the generation count, every island's genes and makespans, the
 * best-ever records with their permutations, the migration counters and,
 * for a pre-screened instance, the network's FP32 parameters, both Adam
 * moments and the step count, the replay ring and the cells' candidate
 * choices.  It begins with a fingerprint of the instances (sizes, machines,
 * processing times, island specs, GA configs, seeds).  ffs_checkpoint_load
 * accepts it only on a bound context created with the same instances in the
 * same order (tile shape and graph use may differ); evolving from there
 * gives exactly the trajectory the saved context would have followed
 * (Section 4's GA is a deterministic function of this state and the seeds).
 *   size: bytes of the image; save: host buffer of at least that size;
 *   load: FFS_EINVAL when the image is not one, is truncated, or was taken
 *   from other instances (the context is then unchanged).  (syncs)          */
int ffs_checkpoint_size(ffs_ctx *ctx, size_t *bytes);
int ffs_checkpoint_save(ffs_ctx *ctx, void *host, size_t bytes);
int ffs_checkpoint_load(ffs_ctx *ctx, const void *host, size_t bytes);

/* ---- learned pre-screen (instances with surrogate_k > 1) ------------------
 * Parameters: one FP32 vector of 394753 values, W1 [512][256] (row = output
 * unit), b1 [512], W2 [512][512], b2 [512], w3 [512], b3 [1]; the products
 * use BF16 copies of W1, W2, w3 with FP32 accumulation (MFMA).  Features:
 * BF16 rows of 256 (uint16 bit patterns): for B = floor(240 / S) position
 * buckets (position t in bucket floor(t B / n)) and stage k, entry b*S + k =
 * B * (processing time at stage k of the jobs in bucket b) / (stage k's total
 * processing time); entries 240..251: parents' makespans / LB, cut points /
 * n, crossover and mutation flags, swap positions / n, LB / sum(p), n / 1000,
 * S / 20, sum(m) / (6 S); the rest 0.  LB = max(max_k ceil(P_k / m_k),
 * max_j sum_k p_jk).  Every ratio is one correctly rounded FP32 division.   */

/* Copy the FP32 parameters out / in (in: the BF16 copies are refreshed, the
 * Adam moments kept).  host: float [394753].  (syncs)                       */
int ffs_surrogate_params(ffs_ctx *ctx, int32_t inst, float *host);
int ffs_surrogate_set_params(ffs_ctx *ctx, int32_t inst, const float *host);

/* Forward pass of `rows` rows (positive multiple of 128).  X: device BF16
 * [rows][256]; y: device float [rows]; H1, H2: device BF16 [rows][512]
 * receiving the hidden activations (may be NULL when rows <= 4096).  (syncs) */
int ffs_mlp_forward(ffs_ctx *ctx, int32_t inst, const uint16_t *X, int32_t rows, float *y, uint16_t *H1,
                    uint16_t *H2);

/* Gradients of mean((y - t)^2) over rows (multiple of 128, <= 4096) without
 * an update.  X: device BF16 [rows][256]; t: device float [rows]; grad:
 * device float [394753] in the parameter layout; dZ2, dZ1: device BF16
 * [rows][512] receiving the back-propagated pre-activation gradients of
 * layers 2 and 1 (may be NULL).  (syncs)                                    */
int ffs_mlp_gradients(ffs_ctx *ctx, int32_t inst, const uint16_t *X, const float *t, int32_t rows, float *grad,
                      uint16_t *dZ2, uint16_t *dZ1);

/* One training step (gradients as above, then Adam) on caller data.  (syncs) */
int ffs_mlp_train_step(ffs_ctx *ctx, int32_t inst, const uint16_t *X, const float *t, int32_t rows);

/* Score the candidates the next generation would consider: X_host BF16
 * [cells * k][256] (row cell * k + c), pred_host float [cells * k],
 * exact_host float [cells * k] (exact (C - LB) / LB of every candidate, only
 * when exact != 0), choice_host int32 [cells].  Cells are numbered over the
 * instance's cellular islands in island order, row-major within a grid.
 * Any output may be NULL.  The population is not changed.  (syncs)          */
int ffs_surrogate_candidates(ffs_ctx *ctx, int32_t inst, int32_t exact, uint16_t *X_host, float *pred_host,
                             float *exact_host, int32_t *choice_host);

/* Candidate stream each cell used in the last screened generation (int32
 * [cells]).  (syncs)                                                        */
int ffs_surrogate_choices(ffs_ctx *ctx, int32_t inst, int32_t *host);

/* Rows [first, first + count) of the replay ring (features BF16 [count][256],
 * targets float [count]); row ((g - 1) * cells + cell) mod 65536 holds the
 * child decoded for `cell` in generation g.  (syncs)                        */
int ffs_surrogate_ring(ffs_ctx *ctx, int32_t inst, int32_t first, int32_t count, uint16_t *X_host, float *t_host);

#ifdef __cplusplus
}
#endif
#endif /* FFS_H */
