/*
 * ffs_tt.h -- C ABI of the paper-faithful variant of the island GA (Luo &
 * El Baz, arXiv 1903.10722) on MI355X (gfx950).
 *
 * Problem (Section 3): J jobs pass S stages in order; stage s has M_s
 * unrelated machines (processing time P[j][s][m] depends on the machine);
 * job j is released at R_j and due at D_j; the objective is
 * WT * sum_j T_j + C_max with T_j = max(0, C_j - D_j), C_j the job's
 * completion at the last stage.  Every time is an integer number of
 * hundredths of a time unit (Table 1's due dates are fractional).
 *
 * Genotype (Section 4.1, genotype level): a string of J * S machine indices,
 * gene j * S + s = the machine of job j at stage s.  The pseudo GA's lower
 * layer is the complement: machine m of stage s -> M_s - 1 - m (for two
 * machines, the bit complement).  Sequencing (the paper gives only the
 * assignment; this library's reading): stage 1 takes the jobs by (R_j, j),
 * every later stage first in, first out by the previous stage's completion
 * (ties: the previous stage's order); a job waits for its assigned machine.
 *
 * Islands (Sections 4.1, 4.2): ffs_island_spec of ffs.h, kind 0 (cellular:
 * the two best of the von Neumann neighbourhood, two-point crossover with
 * probability p_c, with probability p_m one gene moved to another machine of
 * its stage, the child kept if strictly better) or kind 1 (pseudo: pairs
 * (X, complement of X); the better of a pair mates with its complement by
 * two-point crossover with probability p_c, the two children replace the
 * pair; each child then mutates with probability p_m).  `selection` and
 * `sweep` must be 0 (the update schedule is set per context, below).
 * Migration (Section 4.3, equations (1) and (2)) pairs island i with island
 * i + H (H = islands / 2) every `interval` generations on the fitness
 * max(E_max - objective, 0), E_max = WT * sum_j max(0, H_t - D_j) + H_t with
 * H_t = max_j R_j + sum_j sum_s max_m P[j][s][m].
 *
 * Runs: a context holds `runs` independent GA runs of one instance (run r
 * draws its random numbers with instance id r); one launch steps all of them.
 *
 * Conventions (as in ffs.h): FFS_OK or a negative FFS_E* status, error text
 * from ffs_tt_last_error(); inputs are copied; the caller owns every buffer
 * and supplies the one device workspace; all device work runs in call order
 * on the HIP stream given at creation; "(syncs)" functions wait for it.
 * Pointers are host pointers unless the argument says "device".
 */
#ifndef FFS_TT_H
#define FFS_TT_H

#include <stddef.h>
#include <stdint.h>

#include "ffs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ffs_tt_ctx ffs_tt_ctx;

/* Limits of this library: J <= 1024, S <= 32, M_s <= 4, WT >= 0, islands <= 8,
 * island size <= 4096 (even for pseudo islands), runs <= 1024, every time
 * and H_t below 2^30, E_max below 2^39.  Violations give FFS_EUNSUPPORTED. */

/* New context on HIP `stream` (a hipStream_t, may be NULL for the default
 * stream) of the current device.  *out receives the handle. */
int ffs_tt_create(void* stream, ffs_tt_ctx** out);
int ffs_tt_destroy(ffs_tt_ctx* ctx);
const char* ffs_tt_last_error(const ffs_tt_ctx* ctx);

/* The instance.  M[S]; P[J][S][MX] with MX = max_s M_s, entries for
 * m >= M_s ignored, every used entry >= 1; R[J] >= 0; D[J]; all in
 * hundredths.  (Section 3; Table 1 generates such data.) */
int ffs_tt_set_instance(ffs_tt_ctx* ctx, int32_t J, int32_t S, const int32_t* M, int32_t MX, const int32_t* P,
                        const int32_t* R, const int64_t* D, int64_t WT);

/* Append an island (see the header comment).  Islands are numbered in order. */
int ffs_tt_add_island(ffs_tt_ctx* ctx, const ffs_island_spec* spec);

/* Migration every `interval` generations (0: never; needs an even number of
 * islands), threshold theta in [0, 1], base seed, number of runs. */
int ffs_tt_configure(ffs_tt_ctx* ctx, int32_t interval, double theta, uint64_t seed, int32_t runs);

/* Device workspace: size needed, then bind (device pointer, 256-byte
 * aligned, at least that size).  Binding initialises every run's
 * generation 0 (random assignments; a pseudo pair = X and its complement)
 * and its best record. */
int ffs_tt_workspace_size(const ffs_tt_ctx* ctx, size_t* bytes);
int ffs_tt_bind_workspace(ffs_tt_ctx* ctx, void* device_ptr, size_t bytes);

/* `generations` generations of every run (each: every island steps, the best
 * record is updated, then migration on multiples of the interval). */
int ffs_tt_evolve(ffs_tt_ctx* ctx, int32_t generations);

/* One migration epoch now (on the current generation). */
int ffs_tt_migrate(ffs_tt_ctx* ctx);

/* Completed generations. */
int ffs_tt_generation(const ffs_tt_ctx* ctx, int32_t* gen);

/* (syncs) Island `island` of run `run`: genes[size][J*S] as int32 machine
 * indices (may be NULL), objectives[size] (may be NULL). */
int ffs_tt_get_population(ffs_tt_ctx* ctx, int32_t run, int32_t island, int32_t* genes, int64_t* objectives);

/* (syncs) Replace island `island` of run `run` (genes[size][J*S] with every
 * gene in [0, M_s), objectives as the caller states them) and set the
 * completed-generation counter (test access: restores a saved state). */
int ffs_tt_set_population(ffs_tt_ctx* ctx, int32_t run, int32_t island, const int32_t* genes,
                          const int64_t* objectives);
int ffs_tt_set_generation(ffs_tt_ctx* ctx, int32_t gen);

/* (syncs) Best-ever of run `run`: objective, generation, island, slot and its
 * genes (J*S int32, may be NULL).  Strict improvements only; ties inside a
 * generation go to the lowest island, then slot. */
int ffs_tt_best(ffs_tt_ctx* ctx, int32_t run, int64_t* objective, int32_t* gen, int32_t* island, int32_t* slot,
                int32_t* genes);

/* (syncs) Migration epochs with moves and migrants moved, of run `run`. */
int ffs_tt_counters(ffs_tt_ctx* ctx, int32_t run, int64_t* migrations, int64_t* migrants);

/* Objectives of `count` caller-supplied assignments: genes (device) is
 * count x (J*S) uint8 machine indices, row-major; out (device) receives
 * count int64 objectives.  A gene out of range gives -1 for its row. */
int ffs_tt_evaluate(ffs_tt_ctx* ctx, const void* genes, int32_t count, void* out);

/* Update schedule of the cellular islands (an alternative reading of
 * Section 4.2, which gives none): 0 = synchronous (every cell reads the
 * previous generation; the default), 1 = asynchronous line sweep (cells in
 * row-major order, each reading its neighbours as already updated in this
 * generation).  May be changed between calls to ffs_tt_evolve. */
int ffs_tt_set_update(ffs_tt_ctx* ctx, int32_t mode);

/* Timing of the generation kernel: on = 1 brackets the kernel launches of
 * every generation with HIP events; ffs_tt_kernel_time (syncs) returns the
 * summed milliseconds and the number of generations since timing was
 * switched on. */
int ffs_tt_set_timing(ffs_tt_ctx* ctx, int32_t on);
int ffs_tt_kernel_time(ffs_tt_ctx* ctx, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
