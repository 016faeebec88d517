/*
 * ffs_tt_oracle.c -- slow, single-threaded CPU oracle of the paper-faithful
 * variant of the dual heterogeneous island GA (Luo & El Baz, arXiv
 * 1903.10722): unrelated machines, release and due dates, the objective
 * WT * sum T_j + C_max, and the two-layer machine-assignment genotype.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP
 * library.  It is built into the same shared object as ffs_oracle.c and uses
 * that file's counter-based generator (or_draw).
 *
 * What it computes, with the passage each part follows:
 *   - Problem (Section 3): J jobs, S stages, M_s unrelated machines at stage
 *     s, processing time P[j][s][m], release R_j, due date D_j, tardiness
 *     T_j = max(0, C_j - D_j) with C_j the job's completion at the last
 *     stage, objective WT * sum_j T_j + C_max.  All times are integers in
 *     hundredths of a time unit (Table 1's due dates are fractional; Table 2
 *     reports two decimals), so every comparison is exact.
 *   - Genotype (Section 4.1, genotype level): gene i = j * S + s is the index
 *     of the machine of job j at stage s.  The lower (binary) layer of the
 *     pseudo GA is the same string; its complement maps machine m to
 *     M_s - 1 - m, which for two machines is the bit complement (reading).
 *   - Sequencing (reading; the paper gives only the assignment): stage 1
 *     takes the jobs by (R_j, j); every later stage takes them first in,
 *     first out by the previous stage's completion, ties by the previous
 *     stage's order; each job waits for its assigned machine.
 *   - Cellular GA (Sections 4.1, 4.2): the two best of the von Neumann
 *     neighbourhood, two-point crossover (reading), mutation of one gene to
 *     another machine of its stage (reading), replacement if strictly better.
 *     Update schedule: synchronous (every cell reads the previous
 *     generation), or, as an alternative reading, an asynchronous line sweep:
 *     cells in row-major order, each reading its neighbours as they are at
 *     that moment (already updated ones included).
 *   - Pseudo GA (Section 4.1): pairs (X, complement of X); X = the better of
 *     the pair mates with its complement, the two children replace the pair.
 *   - Migration (Section 4.3, equations (1) and (2)) on the fitness
 *     max(E_max - objective, 0) (Section 3), E_max = WT * sum_j max(0, H -
 *     D_j) + H with H = max_j R_j + sum_j sum_s max_m P[j][s][m], a bound on
 *     every schedule's objective (reading of "estimated maximum").
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

uint32_t or_draw(uint64_t seed, uint64_t inst, uint32_t island, uint32_t slot,
                 uint32_t sub, uint32_t gen, uint32_t purpose, uint32_t d);

enum { TT_INIT = 3, TT_CELL = 4, TT_PAIR = 5 };

static uint32_t below(uint32_t u, uint32_t r)
{
    return (uint32_t)(((uint64_t)u * (uint64_t)r) >> 32);
}

static uint64_t threshold(double p)
{
    if (p <= 0.0) return 0;
    if (p >= 1.0) return 4294967296ULL;
    return (uint64_t)(p * 4294967296.0);
}

/* ------------------------------------------------------------------------ */
/* Decoder.                                                                  */
/* ------------------------------------------------------------------------ */

/* Stable insertion sort of order[0..J) by key[order[t]]: equal keys keep
 * their positions' order.  Plain and obviously correct.                     */
static void stable_sort_by(int J, int *order, const int64_t *key)
{
    for (int i = 1; i < J; ++i) {
        int x = order[i], t = i - 1;
        while (t >= 0 && key[order[t]] > key[x]) { order[t + 1] = order[t]; --t; }
        order[t + 1] = x;
    }
}

/* P is indexed ((j * S) + s) * MX + m, MX = max_s M_s.  genes[j * S + s] is
 * job j's machine at stage s.  out_C (may be NULL) receives every completion,
 * out_C[j * S + s] for job j at stage s; out_cmax / out_tard (may be NULL)
 * C_max and sum_j T_j.  Returns WT * sum_j T_j + C_max.                     */
int64_t or_tt_decode(int J, int S, const int *M, int MX, const int *P, const int *R, const int64_t *D,
                     int64_t WT, const int *genes, int64_t *out_C, int64_t *out_cmax, int64_t *out_tard)
{
    int *order = (int *)malloc(sizeof(int) * (size_t)J);
    int64_t *ready = (int64_t *)calloc((size_t)J, sizeof(int64_t));
    int64_t *C = (int64_t *)malloc(sizeof(int64_t) * (size_t)J);
    int64_t *freeat = (int64_t *)malloc(sizeof(int64_t) * (size_t)(MX > 0 ? MX : 1));
    for (int j = 0; j < J; ++j) { order[j] = j; ready[j] = R[j]; }
    stable_sort_by(J, order, ready);                 /* stage 1: by (R_j, j) */
    for (int s = 0; s < S; ++s) {
        for (int m = 0; m < M[s]; ++m) freeat[m] = 0;
        for (int t = 0; t < J; ++t) {
            int j = order[t];
            int m = genes[j * S + s];
            int64_t st = freeat[m] > ready[j] ? freeat[m] : ready[j];
            C[j] = st + P[((size_t)j * S + s) * MX + m];
            freeat[m] = C[j];
            if (out_C) out_C[(size_t)j * S + s] = C[j];
        }
        for (int j = 0; j < J; ++j) ready[j] = C[j];
        stable_sort_by(J, order, ready);             /* next stage: FIFO     */
    }
    int64_t cmax = 0, tard = 0;
    for (int j = 0; j < J; ++j) {
        if (C[j] > cmax) cmax = C[j];
        if (C[j] > D[j]) tard += C[j] - D[j];
    }
    if (out_cmax) *out_cmax = cmax;
    if (out_tard) *out_tard = tard;
    free(order); free(ready); free(C); free(freeat);
    return WT * tard + cmax;
}

/* E_max of the migration fitness (see the header). */
int64_t or_tt_emax(int J, int S, const int *M, int MX, const int *P, const int *R, const int64_t *D, int64_t WT)
{
    int64_t H = 0, rmax = 0;
    for (int j = 0; j < J; ++j) {
        if (R[j] > rmax) rmax = R[j];
        for (int s = 0; s < S; ++s) {
            int64_t mx = 0;
            for (int m = 0; m < M[s]; ++m) {
                int64_t v = P[((size_t)j * S + s) * MX + m];
                if (v > mx) mx = v;
            }
            H += mx;
        }
    }
    H += rmax;
    int64_t e = H;
    for (int j = 0; j < J; ++j) if (H > D[j]) e += WT * (H - D[j]);
    return e;
}

/* ------------------------------------------------------------------------ */
/* Operators on the assignment string (length L = J * S).                    */
/* ------------------------------------------------------------------------ */

/* Two-point crossover: child = P1 on [a, b], P2 elsewhere. */
void or_tt_two_point(int L, const int *p1, const int *p2, int a, int b, int *child)
{
    for (int i = 0; i < L; ++i) child[i] = (i >= a && i <= b) ? p1[i] : p2[i];
}

/* Complement of the lower layer: machine m of stage s -> M_s - 1 - m. */
void or_tt_complement(int J, int S, const int *M, const int *x, int *y)
{
    for (int j = 0; j < J; ++j)
        for (int s = 0; s < S; ++s) y[j * S + s] = M[s] - 1 - x[j * S + s];
}

/* Mutation: with probability tm, gene i (uniform) moves to another machine
 * of its stage, (old + 1 + r) mod M_s with r uniform in [0, M_s - 1); a stage
 * with one machine is left alone.  Exported for the tests.                  */
void or_tt_mutate(int J, int S, const int *M, int *x, uint32_t dflag, uint32_t di, uint32_t dr, uint64_t tm)
{
    (void)J;
    if (!((uint64_t)dflag < tm)) return;
    int L = J * S;
    int i = (int)below(di, (uint32_t)L);
    int ms = M[i % S];
    if (ms < 2) return;
    int r = (int)below(dr, (uint32_t)(ms - 1));
    x[i] = (x[i] + 1 + r) % ms;
}

/* Random assignment of slot `slot` of island `island` (INIT stream, draw i
 * for gene i). */
void or_tt_random_genes(int J, int S, const int *M, uint64_t seed, uint64_t inst, int island, int slot, int *x)
{
    for (int i = 0; i < J * S; ++i)
        x[i] = (int)below(or_draw(seed, inst, (uint32_t)island, (uint32_t)slot, 0, 0, TT_INIT, (uint32_t)i),
                          (uint32_t)M[i % S]);
}

/* Migration decision on int64 objectives (equations (1) and (2), exact).
 * Same convention as the makespan variant: beta = lo / hi of the two best
 * fitness values, migrate iff (hi - lo) * 2^32 < floor(theta * 2^32) * hi,
 * count = ceil(alpha * N), the fitter island sends.                         */
int64_t or_tt_migration_policy(int64_t E, int64_t best_a, int64_t best_b, int64_t n_a, int64_t n_b,
                               double theta, int *emigrant_is_a)
{
    int64_t fa = E - best_a, fb = E - best_b;
    if (fa < 0) fa = 0;
    if (fb < 0) fb = 0;
    *emigrant_is_a = fa > fb;
    if (fa == fb) return 0;
    unsigned __int128 hi = (unsigned __int128)(fa > fb ? fa : fb), lo = (unsigned __int128)(fa > fb ? fb : fa);
    if (hi == 0) return 0;
    unsigned __int128 T = threshold(theta);
    if (!(((hi - lo) << 32) < T * hi)) return 0;
    unsigned __int128 N = (unsigned __int128)(n_a < n_b ? n_a : n_b);
    unsigned __int128 count = (N * (hi - lo) + hi - 1) / hi;
    if (count > N) count = N;
    return (int64_t)count;
}

/* ------------------------------------------------------------------------ */
/* The island GA of the variant.                                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int kind, rows, cols, size;
    uint64_t tc, tm;
    int *genes;          /* size * L */
    int64_t *obj;        /* size */
} tt_island_t;

typedef struct {
    int J, S, MX, L;
    int *M, *P, *R;
    int64_t *D, WT, E;
    int n_islands;
    tt_island_t *isl;
    int interval;
    double theta;
    uint64_t seed, inst;
    int sweep;           /* cellular update: 0 synchronous, 1 line sweep */
    int gen;
    int64_t best_obj;
    int best_gen, best_island, best_slot;
    int *best_genes;
    int64_t migrations, migrants;
} tt_ga_t;

static int64_t tt_obj(tt_ga_t *g, const int *x)
{
    return or_tt_decode(g->J, g->S, g->M, g->MX, g->P, g->R, g->D, g->WT, x, NULL, NULL, NULL);
}

static void tt_update_best(tt_ga_t *g)
{
    int bi = -1, bs = -1;
    int64_t bo = 0;
    for (int i = 0; i < g->n_islands; ++i)
        for (int s = 0; s < g->isl[i].size; ++s)
            if (bi < 0 || g->isl[i].obj[s] < bo) { bo = g->isl[i].obj[s]; bi = i; bs = s; }
    if (g->best_island < 0 || bo < g->best_obj) {
        g->best_obj = bo; g->best_gen = g->gen; g->best_island = bi; g->best_slot = bs;
        memcpy(g->best_genes, g->isl[bi].genes + (size_t)bs * g->L, sizeof(int) * (size_t)g->L);
    }
}

void *or_tt_ga_create(int J, int S, const int *M, int MX, const int *P, const int *R, const int64_t *D,
                      int64_t WT, int n_islands, const int *kinds, const int *rows, const int *cols,
                      const int *sizes, const double *pc, const double *pm, int interval, double theta,
                      uint64_t seed, uint64_t inst)
{
    tt_ga_t *g = (tt_ga_t *)calloc(1, sizeof(tt_ga_t));
    g->J = J; g->S = S; g->MX = MX; g->L = J * S; g->WT = WT;
    g->M = (int *)malloc(sizeof(int) * (size_t)S);
    memcpy(g->M, M, sizeof(int) * (size_t)S);
    g->P = (int *)malloc(sizeof(int) * (size_t)J * S * MX);
    memcpy(g->P, P, sizeof(int) * (size_t)J * S * MX);
    g->R = (int *)malloc(sizeof(int) * (size_t)J);
    memcpy(g->R, R, sizeof(int) * (size_t)J);
    g->D = (int64_t *)malloc(sizeof(int64_t) * (size_t)J);
    memcpy(g->D, D, sizeof(int64_t) * (size_t)J);
    g->E = or_tt_emax(J, S, M, MX, P, R, D, WT);
    g->n_islands = n_islands;
    g->isl = (tt_island_t *)calloc((size_t)n_islands, sizeof(tt_island_t));
    g->interval = interval; g->theta = theta; g->seed = seed; g->inst = inst;
    g->best_genes = (int *)malloc(sizeof(int) * (size_t)g->L);
    g->best_island = -1;
    int L = g->L;
    for (int i = 0; i < n_islands; ++i) {
        tt_island_t *I = &g->isl[i];
        I->kind = kinds[i];
        if (I->kind == 0) { I->rows = rows[i]; I->cols = cols[i]; I->size = rows[i] * cols[i]; }
        else I->size = sizes[i];
        I->tc = threshold(pc[i]);
        I->tm = threshold(pm[i]);
        I->genes = (int *)malloc(sizeof(int) * (size_t)I->size * L);
        I->obj = (int64_t *)malloc(sizeof(int64_t) * (size_t)I->size);
        if (I->kind == 0) {
            for (int s = 0; s < I->size; ++s)
                or_tt_random_genes(J, S, M, seed, inst, i, s, I->genes + (size_t)s * L);
        } else {
            for (int q = 0; q < I->size / 2; ++q) {
                int *A = I->genes + (size_t)(2 * q) * L, *B = I->genes + (size_t)(2 * q + 1) * L;
                or_tt_random_genes(J, S, M, seed, inst, i, q, A);
                or_tt_complement(J, S, M, A, B);
            }
        }
        for (int s = 0; s < I->size; ++s) I->obj[s] = tt_obj(g, I->genes + (size_t)s * L);
    }
    g->gen = 0;
    tt_update_best(g);
    return g;
}

void or_tt_ga_destroy(void *h)
{
    tt_ga_t *g = (tt_ga_t *)h;
    for (int i = 0; i < g->n_islands; ++i) { free(g->isl[i].genes); free(g->isl[i].obj); }
    free(g->isl); free(g->M); free(g->P); free(g->R); free(g->D); free(g->best_genes); free(g);
}

/* better of slots x, y of a neighbourhood listed in order: smaller objective,
 * ties to the earlier position */
static void tt_two_best(const int64_t *obj, const int *nb, int *p1, int *p2)
{
    int b = 0;
    for (int t = 1; t < 5; ++t) if (obj[nb[t]] < obj[nb[b]]) b = t;
    int c = -1;
    for (int t = 0; t < 5; ++t) {
        if (t == b) continue;
        if (c < 0 || obj[nb[t]] < obj[nb[c]]) c = t;
    }
    *p1 = nb[b]; *p2 = nb[c];
}

/* one generation of a cellular island as an asynchronous line sweep: cells
 * in row-major order, in place, each seeing the current state. */
static void tt_cellular_sweep(tt_ga_t *g, int island)
{
    tt_island_t *I = &g->isl[island];
    int L = g->L;
    int *child = (int *)malloc(sizeof(int) * (size_t)L);
    for (int s = 0; s < I->size; ++s) {
        int r = s / I->cols, c = s % I->cols;
        int nb[5] = {s, ((r + I->rows - 1) % I->rows) * I->cols + c, r * I->cols + (c + 1) % I->cols,
                     ((r + 1) % I->rows) * I->cols + c, r * I->cols + (c + I->cols - 1) % I->cols};
        int p1, p2;
        tt_two_best(I->obj, nb, &p1, &p2);
        uint32_t d[6];
        for (int t = 0; t < 6; ++t)
            d[t] = or_draw(g->seed, g->inst, (uint32_t)island, (uint32_t)s, 0, (uint32_t)g->gen, TT_CELL, (uint32_t)t);
        const int *P1 = I->genes + (size_t)p1 * L, *P2 = I->genes + (size_t)p2 * L;
        if ((uint64_t)d[0] < I->tc) {
            int u = (int)below(d[1], (uint32_t)L), v = (int)below(d[2], (uint32_t)L);
            or_tt_two_point(L, P1, P2, u < v ? u : v, u < v ? v : u, child);
        } else {
            memcpy(child, P1, sizeof(int) * (size_t)L);
        }
        or_tt_mutate(g->J, g->S, g->M, child, d[3], d[4], d[5], I->tm);
        int64_t co = tt_obj(g, child);
        if (co < I->obj[s]) {
            memcpy(I->genes + (size_t)s * L, child, sizeof(int) * (size_t)L);
            I->obj[s] = co;
        }
    }
    free(child);
}

static void tt_cellular_step(tt_ga_t *g, int island)
{
    tt_island_t *I = &g->isl[island];
    int L = g->L;
    int *ng = (int *)malloc(sizeof(int) * (size_t)I->size * L);
    int64_t *no = (int64_t *)malloc(sizeof(int64_t) * (size_t)I->size);
    int *child = (int *)malloc(sizeof(int) * (size_t)L);
    for (int s = 0; s < I->size; ++s) {
        int r = s / I->cols, c = s % I->cols;
        int nb[5] = {s, ((r + I->rows - 1) % I->rows) * I->cols + c, r * I->cols + (c + 1) % I->cols,
                     ((r + 1) % I->rows) * I->cols + c, r * I->cols + (c + I->cols - 1) % I->cols};
        int p1, p2;
        tt_two_best(I->obj, nb, &p1, &p2);
        uint32_t d[6];
        for (int t = 0; t < 6; ++t)
            d[t] = or_draw(g->seed, g->inst, (uint32_t)island, (uint32_t)s, 0, (uint32_t)g->gen, TT_CELL, (uint32_t)t);
        const int *P1 = I->genes + (size_t)p1 * L, *P2 = I->genes + (size_t)p2 * L;
        if ((uint64_t)d[0] < I->tc) {
            int u = (int)below(d[1], (uint32_t)L), v = (int)below(d[2], (uint32_t)L);
            or_tt_two_point(L, P1, P2, u < v ? u : v, u < v ? v : u, child);
        } else {
            memcpy(child, P1, sizeof(int) * (size_t)L);
        }
        or_tt_mutate(g->J, g->S, g->M, child, d[3], d[4], d[5], I->tm);
        int64_t co = tt_obj(g, child);
        if (co < I->obj[s]) {
            memcpy(ng + (size_t)s * L, child, sizeof(int) * (size_t)L);
            no[s] = co;
        } else {
            memcpy(ng + (size_t)s * L, I->genes + (size_t)s * L, sizeof(int) * (size_t)L);
            no[s] = I->obj[s];
        }
    }
    free(I->genes); free(I->obj); free(child);
    I->genes = ng; I->obj = no;
}

static void tt_pseudo_step(tt_ga_t *g, int island)
{
    tt_island_t *I = &g->isl[island];
    int L = g->L;
    int *ng = (int *)malloc(sizeof(int) * (size_t)I->size * L);
    int64_t *no = (int64_t *)malloc(sizeof(int64_t) * (size_t)I->size);
    int *X = (int *)malloc(sizeof(int) * (size_t)L), *Y = (int *)malloc(sizeof(int) * (size_t)L);
    for (int q = 0; q < I->size / 2; ++q) {
        int s0 = 2 * q, s1 = 2 * q + 1;
        int xs = (I->obj[s0] <= I->obj[s1]) ? s0 : s1;
        memcpy(X, I->genes + (size_t)xs * L, sizeof(int) * (size_t)L);
        or_tt_complement(g->J, g->S, g->M, X, Y);
        uint32_t d[9];
        for (int t = 0; t < 9; ++t)
            d[t] = or_draw(g->seed, g->inst, (uint32_t)island, (uint32_t)q, 0, (uint32_t)g->gen, TT_PAIR, (uint32_t)t);
        int *C1 = ng + (size_t)s0 * L, *C2 = ng + (size_t)s1 * L;
        if ((uint64_t)d[0] < I->tc) {
            int u = (int)below(d[1], (uint32_t)L), v = (int)below(d[2], (uint32_t)L);
            int a = u < v ? u : v, b = u < v ? v : u;
            or_tt_two_point(L, X, Y, a, b, C1);
            or_tt_two_point(L, Y, X, a, b, C2);
        } else {
            memcpy(C1, X, sizeof(int) * (size_t)L);
            memcpy(C2, Y, sizeof(int) * (size_t)L);
        }
        or_tt_mutate(g->J, g->S, g->M, C1, d[3], d[4], d[5], I->tm);
        or_tt_mutate(g->J, g->S, g->M, C2, d[6], d[7], d[8], I->tm);
        no[s0] = tt_obj(g, C1);
        no[s1] = tt_obj(g, C2);
    }
    free(I->genes); free(I->obj); free(X); free(Y);
    I->genes = ng; I->obj = no;
}

/* slots by (objective, slot) ascending: insertion sort */
static void tt_rank(const tt_island_t *I, int *order)
{
    for (int s = 0; s < I->size; ++s) order[s] = s;
    for (int i = 1; i < I->size; ++i) {
        int x = order[i], t = i - 1;
        while (t >= 0 && (I->obj[order[t]] > I->obj[x] || (I->obj[order[t]] == I->obj[x] && order[t] > x))) {
            order[t + 1] = order[t]; --t;
        }
        order[t + 1] = x;
    }
}

/* one migration epoch: islands paired (i, i + H), H = n_islands / 2, the
 * r-th best of the sending island overwrites the r-th worst of the other. */
void or_tt_ga_migrate(void *h)
{
    tt_ga_t *g = (tt_ga_t *)h;
    int H = g->n_islands / 2, L = g->L;
    for (int i = 0; i < H; ++i) {
        tt_island_t *A = &g->isl[i], *B = &g->isl[i + H];
        int *oa = (int *)malloc(sizeof(int) * (size_t)A->size), *ob = (int *)malloc(sizeof(int) * (size_t)B->size);
        tt_rank(A, oa);
        tt_rank(B, ob);
        int a_sends = 0;
        int64_t count = or_tt_migration_policy(g->E, A->obj[oa[0]], B->obj[ob[0]], A->size, B->size, g->theta,
                                               &a_sends);
        if (count > 0) {
            tt_island_t *src = a_sends ? A : B, *dst = a_sends ? B : A;
            int *os = a_sends ? oa : ob, *od = a_sends ? ob : oa;
            for (int64_t r = 0; r < count; ++r) {
                int ss = os[r], ds = od[dst->size - 1 - r];
                memcpy(dst->genes + (size_t)ds * L, src->genes + (size_t)ss * L, sizeof(int) * (size_t)L);
                dst->obj[ds] = src->obj[ss];
            }
            g->migrations += 1;
            g->migrants += count;
        }
        free(oa); free(ob);
    }
}

void or_tt_ga_evolve(void *h, int G)
{
    tt_ga_t *g = (tt_ga_t *)h;
    for (int it = 0; it < G; ++it) {
        g->gen += 1;
        for (int i = 0; i < g->n_islands; ++i) {
            if (g->isl[i].kind == 0) {
                if (g->sweep) tt_cellular_sweep(g, i);
                else tt_cellular_step(g, i);
            } else {
                tt_pseudo_step(g, i);
            }
        }
        tt_update_best(g);
        if (g->interval > 0 && g->gen % g->interval == 0) or_tt_ga_migrate(g);
    }
}

int or_tt_ga_generation(void *h) { return ((tt_ga_t *)h)->gen; }
void or_tt_ga_set_update(void *h, int sweep) { ((tt_ga_t *)h)->sweep = sweep; }
void or_tt_ga_set_generation(void *h, int gen) { ((tt_ga_t *)h)->gen = gen; }
int64_t or_tt_ga_emax(void *h) { return ((tt_ga_t *)h)->E; }

void or_tt_ga_get(void *h, int island, int *genes, int64_t *obj)
{
    tt_ga_t *g = (tt_ga_t *)h;
    tt_island_t *I = &g->isl[island];
    if (genes) memcpy(genes, I->genes, sizeof(int) * (size_t)I->size * g->L);
    if (obj) memcpy(obj, I->obj, sizeof(int64_t) * (size_t)I->size);
}

void or_tt_ga_set(void *h, int island, const int *genes, const int64_t *obj)
{
    tt_ga_t *g = (tt_ga_t *)h;
    tt_island_t *I = &g->isl[island];
    memcpy(I->genes, genes, sizeof(int) * (size_t)I->size * g->L);
    memcpy(I->obj, obj, sizeof(int64_t) * (size_t)I->size);
}

void or_tt_ga_best(void *h, int64_t *obj, int *gen, int *island, int *slot, int *genes)
{
    tt_ga_t *g = (tt_ga_t *)h;
    *obj = g->best_obj; *gen = g->best_gen; *island = g->best_island; *slot = g->best_slot;
    if (genes) memcpy(genes, g->best_genes, sizeof(int) * (size_t)g->L);
}

void or_tt_ga_counters(void *h, int64_t *migrations, int64_t *migrants)
{
    tt_ga_t *g = (tt_ga_t *)h;
    *migrations = g->migrations; *migrants = g->migrants;
}
