/*
 * ffs_oracle.c -- slow, single-threaded CPU oracle for the dual heterogeneous
 * island GA on the flexible flow shop (Luo & El Baz, arXiv 1903.10722).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP
 * library: every step is written here again, plainly, from the paper's
 * description and the readings documented beside the project.
 *
 * What it computes, with the passage each part follows:
 *   - Problem model (Section 3): J jobs visit S stages in order, stage s has
 *     M_s identical machines, one machine per stage, no preemption.  The
 *     objective used here is the makespan C_max (reading: no release dates,
 *     no tardiness term, identical machines within a stage).
 *   - Decoding a job permutation into a schedule (Section 3 says a solution is
 *     a job sequence on target machines; the rule itself is our reading):
 *     stage 1 in permutation order, later stages first-in-first-out by the
 *     previous stage's completion time (ties: earlier dispatch first), each
 *     job to the machine that becomes free first (ties: lowest index).
 *     Implemented below as "dispatch, then stable sort" -- the plainest form.
 *   - Cellular GA (Section 4.1 operator level, Section 4.2): individuals on a
 *     2-D torus, two parents from the neighbourhood, one child, mutation,
 *     replace the cell if the child is strictly better; synchronous update,
 *     or, as an alternative reading of the update schedule, an asynchronous
 *     line sweep (cells in row-major order, in place).
 *   - Pseudo GA (Section 4.1 operator level): fixed complementary parent
 *     pairs; children replace both parents.  Complement of a permutation is
 *     its reversal (reading of the binary lower layer).
 *   - Migration (Section 4.3, equations (1) and (2)): threshold theta, rate
 *     alpha = 1 - beta, direction from the ratio of the island bests.
 *   - Randomness: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11), counter
 *     based, so one seed fixes one trajectory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11, "Parallel random numbers: as easy as
 * 1, 2, 3").  Round: (hi,lo)=M0*x0, (hi',lo')=M1*x2,
 * x <- (hi' ^ x1 ^ k0, lo', hi ^ x3 ^ k1, lo); key bumped by the Weyl
 * constants before every round but the first.                              */
/* ------------------------------------------------------------------------ */
static void mul64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t hi0, lo0, hi1, lo1;
        mul64(M0, x0, &hi0, &lo0);
        mul64(M1, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream layout (the project's convention for which random number feeds
 * which decision): key = (seed, instance id); counter word 0 = block index
 * inside the stream, word 1 = (island << 32) | slot, word 2 = (sub << 32) |
 * generation, word 3 = purpose.  Draw d of a stream is the 32-bit half
 * (d % 2, low half first) of 64-bit word (d % 8) / 2 of block d / 8.        */
enum { OR_INIT = 3, OR_CELL = 4, OR_PAIR = 5 };

uint32_t or_draw(uint64_t seed, uint64_t inst, uint32_t island, uint32_t slot,
                 uint32_t sub, uint32_t gen, uint32_t purpose, uint32_t d)
{
    uint64_t ctr[4], key[2], out[4];
    key[0] = seed; key[1] = inst;
    ctr[0] = d / 8;
    ctr[1] = ((uint64_t)island << 32) | slot;
    ctr[2] = ((uint64_t)sub << 32) | gen;
    ctr[3] = purpose;
    or_philox4x64_10(ctr, key, out);
    uint64_t w = out[(d % 8) / 2];
    return (d % 2 == 0) ? (uint32_t)(w & 0xFFFFFFFFu) : (uint32_t)(w >> 32);
}

/* Integer in [0, r) from a 32-bit draw: multiply-shift (no rejection). */
static uint32_t uniform_below(uint32_t u, uint32_t r)
{
    return (uint32_t)(((uint64_t)u * (uint64_t)r) >> 32);
}

/* Bernoulli(p) from a 32-bit draw: u < floor(p * 2^32).  The threshold is a
 * 64-bit integer so that p = 1 is "always".                                 */
static uint64_t rate_threshold(double p)
{
    if (p <= 0.0) return 0;
    if (p >= 1.0) return 4294967296ULL;
    return (uint64_t)(p * 4294967296.0); /* exact: scaling by a power of 2 */
}

/* ------------------------------------------------------------------------ */
/* Decoder: permutation -> schedule -> makespan.                             */
/* ------------------------------------------------------------------------ */

/* Sort jobs[0..n) by (C[job], position in jobs[]) -- a stable insertion sort
 * on C, chosen for being obviously correct rather than fast.               */
static void stable_sort_by_completion(int n, int *jobs, const int64_t *C)
{
    for (int i = 1; i < n; ++i) {
        int j = jobs[i];
        int t = i - 1;
        while (t >= 0 && C[jobs[t]] > C[j]) { jobs[t + 1] = jobs[t]; --t; }
        jobs[t + 1] = j;
    }
}

/* p is job-major: p[j*S + k].  out_start / out_machine (job-major, may be
 * NULL) receive every operation's start time and machine.                  */
int64_t or_decode(int n, int S, const int *m, const int *p, const int *perm,
                  int64_t *out_start, int *out_machine)
{
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    int64_t *ready = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *C = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int mmax = 1;
    for (int k = 0; k < S; ++k) if (m[k] > mmax) mmax = m[k];
    int64_t *freet = (int64_t *)malloc(sizeof(int64_t) * (size_t)mmax);

    for (int i = 0; i < n; ++i) { order[i] = perm[i]; ready[i] = 0; }
    for (int k = 0; k < S; ++k) {
        for (int q = 0; q < m[k]; ++q) freet[q] = 0;
        for (int idx = 0; idx < n; ++idx) {
            int j = order[idx];
            int best = 0;                       /* first-available machine,   */
            for (int q = 1; q < m[k]; ++q)      /* lowest index on ties       */
                if (freet[q] < freet[best]) best = q;
            int64_t st = freet[best] > ready[j] ? freet[best] : ready[j];
            C[j] = st + p[(size_t)j * S + k];
            freet[best] = C[j];
            if (out_start) out_start[(size_t)j * S + k] = st;
            if (out_machine) out_machine[(size_t)j * S + k] = best;
        }
        /* next stage: first-in-first-out by completion, ties by dispatch
         * position; order[] is in dispatch position, so a stable sort.     */
        stable_sort_by_completion(n, order, C);
        for (int i = 0; i < n; ++i) ready[i] = C[i];
    }
    int64_t cmax = 0;
    for (int i = 0; i < n; ++i) if (ready[i] > cmax) cmax = ready[i];
    free(order); free(ready); free(C); free(freet);
    return cmax;
}

/* ------------------------------------------------------------------------ */
/* Genetic operators.                                                        */
/* ------------------------------------------------------------------------ */

/* Order crossover (Davis): child[a..b] = p1[a..b]; the remaining positions
 * b+1 .. n-1, 0 .. a-1 are filled, in that order, with the genes of p2 read
 * cyclically from position b+1, skipping genes already in the segment.      */
void or_ox(int n, const int *p1, const int *p2, int a, int b, int *child)
{
    char *used = (char *)calloc((size_t)n, 1);
    for (int t = a; t <= b; ++t) { child[t] = p1[t]; used[p1[t]] = 1; }
    int pos = (b + 1) % n;
    for (int s = 0; s < n; ++s) {
        int g = p2[(b + 1 + s) % n];
        if (used[g]) continue;
        child[pos] = g;
        pos = (pos + 1) % n;
    }
    free(used);
}

/* Fisher-Yates shuffle from the INIT stream of (island, slot). */
void or_fisher_yates(int n, uint64_t seed, uint64_t inst, int island, int slot, int *out)
{
    for (int i = 0; i < n; ++i) out[i] = i;
    for (int i = n - 1; i >= 1; --i) {
        uint32_t u = or_draw(seed, inst, (uint32_t)island, (uint32_t)slot, 0, 0, OR_INIT,
                             (uint32_t)(n - 1 - i));
        int j = (int)uniform_below(u, (uint32_t)(i + 1));
        int t = out[i]; out[i] = out[j]; out[j] = t;
    }
}

/* Parent choice on the torus: the von Neumann neighbourhood in the fixed
 * order (self, north, east, south, west); P1 is the best by (makespan, order
 * position), P2 the best of the other four.                                 */
/* Parent selection variants (the paper only says two individuals are
 * selected from the nearby area; Section 4.2):
 *   sel 0: P1 = the best of (self, N, E, S, W) by (makespan, order position),
 *          P2 = the best of the other four;
 *   sel 1: P1 = self, P2 = the best of (N, E, S, W) by (makespan, order);
 *   sel 2: binary tournaments: draw d6 gives x uniform in [0, 25), the
 *          positions x / 5 and x % 5 of the neighbourhood, and P1 is the
 *          better of the two by (makespan, order position); draw d7 gives P2
 *          the same way (P2 may equal P1).                                   */
static int better_pos(const int *mk, const int *nb, int i, int j)
{
    if (mk[nb[j]] < mk[nb[i]]) return j;
    if (mk[nb[j]] == mk[nb[i]] && j < i) return j;
    return i;
}

void or_cell_parents_sel(int rows, int cols, const int *mk, int slot, int sel, uint32_t d6, uint32_t d7,
                         int *p1, int *p2)
{
    int r = slot / cols, c = slot % cols;
    int nb[5];
    nb[0] = slot;
    nb[1] = ((r - 1 + rows) % rows) * cols + c;
    nb[2] = r * cols + (c + 1) % cols;
    nb[3] = ((r + 1) % rows) * cols + c;
    nb[4] = r * cols + (c - 1 + cols) % cols;
    if (sel == 1) {
        int b = 1;
        for (int t = 2; t < 5; ++t) if (mk[nb[t]] < mk[nb[b]]) b = t;
        *p1 = nb[0];
        *p2 = nb[b];
        return;
    }
    if (sel == 2) {
        uint32_t x = uniform_below(d6, 25u), y = uniform_below(d7, 25u);
        *p1 = nb[better_pos(mk, nb, (int)(x / 5), (int)(x % 5))];
        *p2 = nb[better_pos(mk, nb, (int)(y / 5), (int)(y % 5))];
        return;
    }
    int b1 = 0;
    for (int t = 1; t < 5; ++t) if (mk[nb[t]] < mk[nb[b1]]) b1 = t;
    int b2 = -1;
    for (int t = 0; t < 5; ++t) {
        if (t == b1) continue;
        if (b2 < 0 || mk[nb[t]] < mk[nb[b2]]) b2 = t;
    }
    *p1 = nb[b1];
    *p2 = nb[b2];
}

void or_cell_parents(int rows, int cols, const int *mk, int slot, int *p1, int *p2)
{
    or_cell_parents_sel(rows, cols, mk, slot, 0, 0u, 0u, p1, p2);
}

/* Migration decision for one island pair (Section 4.3, eq. (1)-(2)), with
 * fitness = E - makespan (Section 3's transform, E = sum of all processing
 * times) and every real-number comparison carried out in exact integers:
 *   beta = lo/hi, migrate iff 1 - beta < theta  <=>  (hi-lo)*2^32 < T*hi,
 *   T = floor(theta * 2^32); count = ceil(alpha * N), N = min(N_A, N_B).
 * Returns the number of migrants (0 = none); *emigrant_is_a says which side
 * sends (the side with the larger fitness, i.e. the smaller makespan).     */
int64_t or_migration_policy(int64_t E, int64_t best_a, int64_t best_b,
                            int64_t n_a, int64_t n_b, double theta, int *emigrant_is_a)
{
    int64_t fa = E - best_a, fb = E - best_b;
    if (fa < 0) fa = 0;
    if (fb < 0) fb = 0;
    *emigrant_is_a = fa > fb;
    if (fa == fb) return 0;
    uint64_t hi = (uint64_t)(fa > fb ? fa : fb), lo = (uint64_t)(fa > fb ? fb : fa);
    if (hi == 0) return 0;
    uint64_t T = rate_threshold(theta);
    if (!(((hi - lo) << 32) < T * hi)) return 0;
    uint64_t N = (uint64_t)(n_a < n_b ? n_a : n_b);
    uint64_t count = (N * (hi - lo) + hi - 1) / hi;
    if (count > N) count = N;
    return (int64_t)count;
}

/* ------------------------------------------------------------------------ */
/* The island GA.                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind;            /* 0 cellular grid, 1 pseudo (complementary pairs)  */
    int rows, cols;      /* cellular                                          */
    int size;            /* number of individuals                            */
    uint64_t tc, tm;     /* crossover / mutation thresholds                  */
    int sel;             /* cellular parent selection variant (or_cell_parents_sel) */
    int sweep;           /* cellular update: 0 synchronous, 1 line sweep     */
    int *genes;          /* size * n, current generation                     */
    int *mk;             /* size                                             */
} or_island_t;

typedef struct {
    int n, S;
    int *m, *p;
    int64_t E;
    int n_islands;
    or_island_t *isl;
    int interval, topology;
    double theta;
    uint64_t seed, inst;
    int gen;
    int64_t best_mk;
    int best_gen, best_island, best_slot;
    int *best_perm;
    int64_t migrations, migrants;  /* counters, for tests */
    int **choice;                  /* per island: candidate stream of each cell for the next step, or NULL */
} or_ga_t;

static int64_t dec(or_ga_t *g, const int *perm)
{
    return or_decode(g->n, g->S, g->m, g->p, perm, NULL, NULL);
}

/* best-ever: strict improvement only; ties inside one generation go to the
 * lowest (island, slot).                                                    */
static void update_best(or_ga_t *g)
{
    int bi = -1, bs = -1;
    int64_t bm = 0;
    for (int i = 0; i < g->n_islands; ++i)
        for (int s = 0; s < g->isl[i].size; ++s)
            if (bi < 0 || g->isl[i].mk[s] < bm) { bm = g->isl[i].mk[s]; bi = i; bs = s; }
    if (g->best_island < 0 || bm < g->best_mk) {
        g->best_mk = bm; g->best_gen = g->gen; g->best_island = bi; g->best_slot = bs;
        memcpy(g->best_perm, g->isl[bi].genes + (size_t)bs * g->n, sizeof(int) * (size_t)g->n);
    }
}

void *or_ga_create(int n, int S, const int *m, const int *p, int n_islands,
                   const int *kinds, const int *rows, const int *cols, const int *sizes,
                   const double *pc, const double *pm, int interval, double theta,
                   int topology, uint64_t seed, uint64_t inst)
{
    or_ga_t *g = (or_ga_t *)calloc(1, sizeof(or_ga_t));
    g->n = n; g->S = S;
    g->m = (int *)malloc(sizeof(int) * (size_t)S);
    g->p = (int *)malloc(sizeof(int) * (size_t)n * S);
    memcpy(g->m, m, sizeof(int) * (size_t)S);
    memcpy(g->p, p, sizeof(int) * (size_t)n * S);
    g->E = 0;
    for (size_t i = 0; i < (size_t)n * S; ++i) g->E += p[i];
    g->n_islands = n_islands;
    g->isl = (or_island_t *)calloc((size_t)n_islands, sizeof(or_island_t));
    g->interval = interval; g->theta = theta; g->topology = topology;
    g->seed = seed; g->inst = inst;
    g->best_perm = (int *)malloc(sizeof(int) * (size_t)n);
    g->best_island = -1;
    g->choice = (int **)calloc((size_t)n_islands, sizeof(int *));
    for (int i = 0; i < n_islands; ++i) {
        or_island_t *I = &g->isl[i];
        I->kind = kinds[i];
        if (I->kind == 0) { I->rows = rows[i]; I->cols = cols[i]; I->size = rows[i] * cols[i]; }
        else { I->rows = 0; I->cols = 0; I->size = sizes[i]; }
        I->tc = rate_threshold(pc[i]);
        I->tm = rate_threshold(pm[i]);
        I->genes = (int *)malloc(sizeof(int) * (size_t)I->size * n);
        I->mk = (int *)malloc(sizeof(int) * (size_t)I->size);
        /* generation 0: random permutations; a pseudo pair starts as a
         * permutation and its complement (reversal).                       */
        if (I->kind == 0) {
            for (int s = 0; s < I->size; ++s)
                or_fisher_yates(n, seed, inst, i, s, I->genes + (size_t)s * n);
        } else {
            for (int q = 0; q < I->size / 2; ++q) {
                int *A = I->genes + (size_t)(2 * q) * n, *B = I->genes + (size_t)(2 * q + 1) * n;
                or_fisher_yates(n, seed, inst, i, q, A);
                for (int t = 0; t < n; ++t) B[t] = A[n - 1 - t];
            }
        }
        for (int s = 0; s < I->size; ++s) I->mk[s] = (int)dec(g, I->genes + (size_t)s * n);
    }
    g->gen = 0;
    update_best(g);
    return g;
}

void or_ga_destroy(void *h)
{
    or_ga_t *g = (or_ga_t *)h;
    for (int i = 0; i < g->n_islands; ++i) { free(g->isl[i].genes); free(g->isl[i].mk); free(g->choice[i]); }
    free(g->choice);
    free(g->isl); free(g->m); free(g->p); free(g->best_perm); free(g);
}

/* Swap mutation (Section 4.2 names a mutation step; the operator is our
 * reading): with probability tm the genes at positions i and j != i trade
 * places, i uniform in [0, n) from draw di and j = (i + 1 + r) mod n with r
 * uniform in [0, n - 1) from draw dj, so every other position is equally
 * likely.  Exported for the tests.                                          */
void or_swap_mutation(int n, int *x, uint32_t dflag, uint32_t di, uint32_t dj, uint64_t tm)
{
    if (!((uint64_t)dflag < tm)) return;
    int i = (int)uniform_below(di, (uint32_t)n);
    int j = (i + 1 + (int)uniform_below(dj, (uint32_t)(n > 1 ? n - 1 : 0))) % n;
    int t = x[i]; x[i] = x[j]; x[j] = t;
}

/* Offspring of cell s at generation g->gen from candidate stream `sub` of
 * the CELL purpose (sub 0 is the plain GA's only stream).  meta (may be NULL)
 * receives p1, p2, crossover flag, a, b, mutation flag, i, j.              */
static void cell_offspring(or_ga_t *g, int island, int s, int sub, int *child, int *meta)
{
    or_island_t *I = &g->isl[island];
    int n = g->n;
    int p1, p2;
    uint32_t d[8];
    for (int t = 0; t < 8; ++t)
        d[t] = or_draw(g->seed, g->inst, (uint32_t)island, (uint32_t)s, (uint32_t)sub, (uint32_t)g->gen, OR_CELL,
                       (uint32_t)t);
    or_cell_parents_sel(I->rows, I->cols, I->mk, s, I->sel, d[6], d[7], &p1, &p2);
    const int *P1 = I->genes + (size_t)p1 * n, *P2 = I->genes + (size_t)p2 * n;
    int cx = (uint64_t)d[0] < I->tc;
    int u = (int)uniform_below(d[1], (uint32_t)n), v = (int)uniform_below(d[2], (uint32_t)n);
    int a = u < v ? u : v, b = u < v ? v : u;
    if (cx) or_ox(n, P1, P2, a, b, child);
    else memcpy(child, P1, sizeof(int) * (size_t)n);
    or_swap_mutation(n, child, d[3], d[4], d[5], I->tm);
    if (meta) {
        int mx = (uint64_t)d[3] < I->tm;
        int mi = (int)uniform_below(d[4], (uint32_t)n);
        int mj = (mi + 1 + (int)uniform_below(d[5], (uint32_t)(n > 1 ? n - 1 : 0))) % n;
        meta[0] = p1; meta[1] = p2; meta[2] = cx; meta[3] = a; meta[4] = b;
        meta[5] = mx; meta[6] = mi; meta[7] = mj;
    }
}

/* Parent selection variant of a cellular island (see or_cell_parents_sel). */
void or_ga_set_selection(void *h, int island, int sel)
{
    or_ga_t *g = (or_ga_t *)h;
    g->isl[island].sel = sel;
}

/* Update schedule of a cellular island: 0 synchronous (Section 4.2, every
 * cell from generation g-1), 1 asynchronous line sweep (an alternative
 * reading: cells in row-major order, in place).                            */
void or_ga_set_sweep(void *h, int island, int sweep)
{
    or_ga_t *g = (or_ga_t *)h;
    g->isl[island].sweep = sweep;
}

/* Test access: the offspring a cell would get at the next generation from
 * candidate stream `sub`, with its meta data (see cell_offspring).          */
void or_ga_cell_candidate(void *h, int island, int slot, int sub, int *child, int *meta)
{
    or_ga_t *g = (or_ga_t *)h;
    g->gen += 1;
    cell_offspring(g, island, slot, sub, child, meta);
    g->gen -= 1;
}

/* Candidate stream of every cell of `island` for the next generation only
 * (the choice of a learned pre-screen, replayed); NULL restores stream 0.  */
void or_ga_set_cell_choices(void *h, int island, const int *choices)
{
    or_ga_t *g = (or_ga_t *)h;
    free(g->choice[island]);
    g->choice[island] = NULL;
    if (choices) {
        g->choice[island] = (int *)malloc(sizeof(int) * (size_t)g->isl[island].size);
        memcpy(g->choice[island], choices, sizeof(int) * (size_t)g->isl[island].size);
    }
}

/* one generation of a cellular island, synchronous (reads generation g-1
 * only, writes a fresh copy).                                              */
static void cellular_step(or_ga_t *g, int island)
{
    or_island_t *I = &g->isl[island];
    int n = g->n;
    int *ng = (int *)malloc(sizeof(int) * (size_t)I->size * n);
    int *nm = (int *)malloc(sizeof(int) * (size_t)I->size);
    int *child = (int *)malloc(sizeof(int) * (size_t)n);
    for (int s = 0; s < I->size; ++s) {
        int sub = g->choice[island] ? g->choice[island][s] : 0;
        cell_offspring(g, island, s, sub, child, NULL);
        int cm = (int)dec(g, child);
        if (cm < I->mk[s]) {
            memcpy(ng + (size_t)s * n, child, sizeof(int) * (size_t)n);
            nm[s] = cm;
        } else {
            memcpy(ng + (size_t)s * n, I->genes + (size_t)s * n, sizeof(int) * (size_t)n);
            nm[s] = I->mk[s];
        }
    }
    free(I->genes); free(I->mk); free(child);
    I->genes = ng; I->mk = nm;
    free(g->choice[island]);
    g->choice[island] = NULL;
}

/* one generation of a cellular island as an asynchronous line sweep: the
 * cells in row-major order, each updated in place, so a cell's parents are
 * taken from the state its earlier neighbours have already reached in this
 * generation.  Draws, operators and the strict replacement rule are those of
 * cellular_step.                                                           */
static void cellular_sweep(or_ga_t *g, int island)
{
    or_island_t *I = &g->isl[island];
    int n = g->n;
    int *child = (int *)malloc(sizeof(int) * (size_t)n);
    for (int s = 0; s < I->size; ++s) {
        int sub = g->choice[island] ? g->choice[island][s] : 0;
        cell_offspring(g, island, s, sub, child, NULL);
        int cm = (int)dec(g, child);
        if (cm < I->mk[s]) {
            memcpy(I->genes + (size_t)s * n, child, sizeof(int) * (size_t)n);
            I->mk[s] = cm;
        }
    }
    free(child);
    free(g->choice[island]);
    g->choice[island] = NULL;
}

/* The two children of one complementary pair (Section 4.1, operator level:
 * a parent mates with its complement, and the pseudo GA's children take the
 * parents' places).  X is the pair's better member, Y = reverse(X) its
 * complement.  With probability tc (draw d[0]) the children are
 * C1 = OX(X, Y; a, b) and C2 = OX(Y, X; a, b) with one pair of cut points
 * from draws d[1], d[2]; otherwise C1 = X and C2 = Y.  C1 then takes a swap
 * mutation from draws d[3..5] and C2 one from d[6..8].  Exported for the
 * tests.                                                                    */
void or_pseudo_children(int n, const int *X, const uint32_t *d, uint64_t tc, uint64_t tm, int *C1, int *C2)
{
    int *Y = (int *)malloc(sizeof(int) * (size_t)n);
    for (int t = 0; t < n; ++t) Y[t] = X[n - 1 - t];
    if ((uint64_t)d[0] < tc) {
        int u = (int)uniform_below(d[1], (uint32_t)n), v = (int)uniform_below(d[2], (uint32_t)n);
        int a = u < v ? u : v, b = u < v ? v : u;
        or_ox(n, X, Y, a, b, C1);
        or_ox(n, Y, X, a, b, C2);
    } else {
        memcpy(C1, X, sizeof(int) * (size_t)n);
        memcpy(C2, Y, sizeof(int) * (size_t)n);
    }
    or_swap_mutation(n, C1, d[3], d[4], d[5], tm);
    or_swap_mutation(n, C2, d[6], d[7], d[8], tm);
    free(Y);
}

/* one generation of a pseudo island: per pair, the better parent X (lower
 * makespan, the even slot on ties) and its complement mate; the two
 * children replace the pair.                                                */
static void pseudo_step(or_ga_t *g, int island)
{
    or_island_t *I = &g->isl[island];
    int n = g->n;
    int *ng = (int *)malloc(sizeof(int) * (size_t)I->size * n);
    int *nm = (int *)malloc(sizeof(int) * (size_t)I->size);
    int *X = (int *)malloc(sizeof(int) * (size_t)n);
    for (int q = 0; q < I->size / 2; ++q) {
        int s0 = 2 * q, s1 = 2 * q + 1;
        int xs = (I->mk[s0] <= I->mk[s1]) ? s0 : s1;
        memcpy(X, I->genes + (size_t)xs * n, sizeof(int) * (size_t)n);
        uint32_t d[9];
        for (int t = 0; t < 9; ++t)
            d[t] = or_draw(g->seed, g->inst, (uint32_t)island, (uint32_t)q, 0, (uint32_t)g->gen, OR_PAIR, (uint32_t)t);
        int *C1 = ng + (size_t)s0 * n, *C2 = ng + (size_t)s1 * n;
        or_pseudo_children(n, X, d, I->tc, I->tm, C1, C2);
        nm[s0] = (int)dec(g, C1);
        nm[s1] = (int)dec(g, C2);
    }
    free(I->genes); free(I->mk); free(X);
    I->genes = ng; I->mk = nm;
}

/* slot order of an island by (makespan, slot), ascending */
static void rank_slots(const or_island_t *I, int *order)
{
    for (int s = 0; s < I->size; ++s) order[s] = s;
    for (int i = 1; i < I->size; ++i) {       /* insertion sort: plain */
        int x = order[i], t = i - 1;
        while (t >= 0 && (I->mk[order[t]] > I->mk[x] ||
                          (I->mk[order[t]] == I->mk[x] && order[t] > x))) {
            order[t + 1] = order[t]; --t;
        }
        order[t + 1] = x;
    }
}

static void copy_individual(or_ga_t *g, int di, int ds, const int *genes, int mk)
{
    memcpy(g->isl[di].genes + (size_t)ds * g->n, genes, sizeof(int) * (size_t)g->n);
    g->isl[di].mk[ds] = mk;
}

/* adaptive (penetration) migration between islands a and b */
static void adaptive_pair(or_ga_t *g, int a, int b)
{
    or_island_t *A = &g->isl[a], *B = &g->isl[b];
    int *oa = (int *)malloc(sizeof(int) * (size_t)A->size), *ob = (int *)malloc(sizeof(int) * (size_t)B->size);
    rank_slots(A, oa);
    rank_slots(B, ob);
    int a_emigrates = 0;
    int64_t count = or_migration_policy(g->E, A->mk[oa[0]], B->mk[ob[0]], A->size, B->size,
                                        g->theta, &a_emigrates);
    if (count > 0) {
        int src = a_emigrates ? a : b, dst = a_emigrates ? b : a;
        int *os = a_emigrates ? oa : ob, *od = a_emigrates ? ob : oa;
        int nd = g->isl[dst].size;
        for (int64_t r = 0; r < count; ++r) {
            int ss = os[r], ds = od[nd - 1 - r];   /* r-th best -> r-th worst */
            copy_individual(g, dst, ds, g->isl[src].genes + (size_t)ss * g->n, g->isl[src].mk[ss]);
        }
        g->migrations += 1;
        g->migrants += count;
    }
    free(oa); free(ob);
}

/* one migration epoch.  Islands are paired (i, i + H), H = n_islands / 2.
 * Topology 1 first runs a ring c0, p0, c1, p1, ... in which every island's
 * best (taken from a snapshot) overwrites its successor's worst.
 * Topology 2 (an alternative reading of the multi-island case) applies the
 * penetration rule of equations (1)-(2) to every edge of that ring in turn,
 * (c0, p0), (p0, c1), ..., (p_{H-1}, c0), each on the state the previous
 * edges left; two islands have the single edge (c0, p0).                   */
void or_ga_migrate(void *h)
{
    or_ga_t *g = (or_ga_t *)h;
    int H = g->n_islands / 2;
    if (H == 0) return;
    if (g->topology == 2) {
        int L = 2 * H;
        int edges = (L == 2) ? 1 : L;
        for (int t = 0; t < edges; ++t) {
            int x = (t % 2 == 0) ? t / 2 : H + t / 2;
            int u = (t + 1) % L;
            int y = (u % 2 == 0) ? u / 2 : H + u / 2;
            adaptive_pair(g, x, y);
        }
        return;
    }
    if (g->topology == 1) {
        int L = 2 * H;
        int *ring = (int *)malloc(sizeof(int) * (size_t)L);
        for (int i = 0; i < H; ++i) { ring[2 * i] = i; ring[2 * i + 1] = i + H; }
        /* snapshot of every island's best individual and worst slot */
        int **bg = (int **)malloc(sizeof(int *) * (size_t)L);
        int *bm = (int *)malloc(sizeof(int) * (size_t)L), *ws = (int *)malloc(sizeof(int) * (size_t)L);
        for (int t = 0; t < L; ++t) {
            or_island_t *I = &g->isl[ring[t]];
            int *o = (int *)malloc(sizeof(int) * (size_t)I->size);
            rank_slots(I, o);
            bg[t] = (int *)malloc(sizeof(int) * (size_t)g->n);
            memcpy(bg[t], I->genes + (size_t)o[0] * g->n, sizeof(int) * (size_t)g->n);
            bm[t] = I->mk[o[0]];
            ws[t] = o[I->size - 1];
            free(o);
        }
        for (int t = 0; t < L; ++t) {
            int dt = (t + 1) % L;
            copy_individual(g, ring[dt], ws[dt], bg[t], bm[t]);
        }
        for (int t = 0; t < L; ++t) free(bg[t]);
        free(bg); free(bm); free(ws); free(ring);
    }
    for (int i = 0; i < H; ++i) adaptive_pair(g, i, i + H);
}

/* G generations.  Per generation: every island steps from generation g-1,
 * the best-ever record is updated, and on every generation that is a
 * multiple of the migration interval one migration epoch runs.              */
void or_ga_evolve(void *h, int G)
{
    or_ga_t *g = (or_ga_t *)h;
    for (int it = 0; it < G; ++it) {
        g->gen += 1;
        for (int i = 0; i < g->n_islands; ++i) {
            if (g->isl[i].kind == 0) {
                if (g->isl[i].sweep) cellular_sweep(g, i);
                else cellular_step(g, i);
            } else {
                pseudo_step(g, i);
            }
        }
        update_best(g);
        if (g->interval > 0 && g->gen % g->interval == 0) or_ga_migrate(g);
    }
}

int or_ga_generation(void *h) { return ((or_ga_t *)h)->gen; }

/* Test access: set the generation counter (with or_ga_set this restores a
 * state taken from elsewhere), and run the step of one island for the next
 * generation without touching the others, the counter or the best record. */
void or_ga_set_generation(void *h, int gen) { ((or_ga_t *)h)->gen = gen; }

void or_ga_step_island(void *h, int island)
{
    or_ga_t *g = (or_ga_t *)h;
    g->gen += 1;
    if (g->isl[island].kind == 0) {
        if (g->isl[island].sweep) cellular_sweep(g, island);
        else cellular_step(g, island);
    } else {
        pseudo_step(g, island);
    }
    g->gen -= 1;
}

void or_ga_get(void *h, int island, int *genes, int *mk)
{
    or_ga_t *g = (or_ga_t *)h;
    or_island_t *I = &g->isl[island];
    if (genes) memcpy(genes, I->genes, sizeof(int) * (size_t)I->size * g->n);
    if (mk) memcpy(mk, I->mk, sizeof(int) * (size_t)I->size);
}

void or_ga_set(void *h, int island, const int *genes, const int *mk)
{
    or_ga_t *g = (or_ga_t *)h;
    or_island_t *I = &g->isl[island];
    memcpy(I->genes, genes, sizeof(int) * (size_t)I->size * g->n);
    memcpy(I->mk, mk, sizeof(int) * (size_t)I->size);
}

void or_ga_best(void *h, int64_t *mk, int *gen, int *island, int *slot, int *perm)
{
    or_ga_t *g = (or_ga_t *)h;
    *mk = g->best_mk; *gen = g->best_gen; *island = g->best_island; *slot = g->best_slot;
    if (perm) memcpy(perm, g->best_perm, sizeof(int) * (size_t)g->n);
}

void or_ga_counters(void *h, int64_t *migrations, int64_t *migrants)
{
    or_ga_t *g = (or_ga_t *)h;
    *migrations = g->migrations; *migrants = g->migrants;
}
