// ffs_tt.hip -- the paper-faithful variant of the island GA on gfx950: the
// machine-assignment genotype (Section 4.1), unrelated machines with release
// and due dates and the objective WT * sum T_j + C_max (Section 3), the
// cellular and pseudo islands and the penetration migration (Sections
// 4.1-4.3).  Host side of include/ffs_tt.h and its kernels.
//
// Mapping: one wave per individual.  A workgroup copies the instance tables
// (processing times, due dates, release times, stage-1 order, machine
// counts, complement base), which the host stores as their LDS image, into
// LDS once; each wave builds its child there and decodes it stage by stage
// with the whole wave:
//   - the completions of one stage come from a (max, +) scan per machine
//     along the stage's order: job k on machine m finishes at
//     max(free_m, ready_k) + p_k, and "wait for x, then run p" composes
//     associatively: (A1, B1) then (A2, B2) is (max(A1, A2 - B1), B1 + B2)
//     applied as x -> max(x, A) + B;
//   - the next stage's order (first in, first out by completion, ties by
//     this stage's order) merges the machines' lists, each already sorted by
//     (completion, position) because a machine finishes its jobs in order:
//     with at most two machines by a merge path (each lane finds its share
//     of the merged order by one binary search on its diagonal, then merges
//     it), otherwise by rank (a job's index in its own list plus, for every
//     other machine, the number of that machine's entries below it, each a
//     binary search).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ffs_tt.h"
#include "philox.h"

namespace tt {

using flowshop::Block4;
using flowshop::below;
using flowshop::draw32;
using flowshop::stream_block;

constexpr int kMaxJ = 1024, kMaxS = 32, kMaxM = 4, kMaxIsl = 8, kMaxIslSize = 4096, kMaxRuns = 1024;
constexpr int kNeg = -(1 << 30) - 1;  // A of the identity; every real A is >= 0
constexpr int kSortThreads = 1024;

struct TtIsland {
    int kind, rows, cols, size, off;  // off: first individual of the island inside a run
    unsigned long long tc, tm;        // crossover / mutation thresholds (draw < t)
};

struct TtDesc {
    int J, S, MX, L, Lp, Jp, N, n_isl, runs, H;
    long long WT, E;
    unsigned long long theta_T;
    const uint4* tab;           // the LDS image of the tables (see tab_off), tab_vec 16-byte vectors
    int tab_vec;
    uint8_t* genes[2];          // [runs][N][Lp], by generation parity
    long long* obj[2];          // [runs][N]
    unsigned long long* genkey; // [runs][n_isl][2]: min of (objective << 13 | slot)
    long long* best;            // [runs][4]: objective, generation, island, slot
    uint8_t* best_genes;        // [runs][Lp]
    long long* counters;        // [runs][2]: epochs with moves, migrants
    int* err;                   // device error flag
    uint64_t seed;
    TtIsland isl[kMaxIsl];
};

// Island i of the descriptor, read with static indices only (a dynamic index
// into a kernel argument would place the argument in scratch memory).
__device__ __forceinline__ TtIsland island_at(const TtDesc& d, int i)
{
    TtIsland r = d.isl[0];
#pragma unroll
    for (int q = 1; q < kMaxIsl; ++q)
        if (q == i) r = d.isl[q];
    return r;
}

// 32-bit lane of a 16-byte vector, by static index
__device__ __forceinline__ uint32_t word_of(const uint4& v, int w)
{
    return w == 0 ? v.x : (w == 1 ? v.y : (w == 2 ? v.z : v.w));
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

// Byte offsets of the shared tables in LDS, each piece 16-byte aligned:
// P[J][S][MX] (u16), D[J] and R[J] (int), the stage-1 order ord0[J] (u16),
// M[S] (int) and cb[Lp] (u8: M_s - 1 of gene i's stage, 0 past the string,
// the complement base).  The host writes the same image into the workspace,
// so that a workgroup stages it with one vector copy.
struct TabOff {
    int P, D, R, ord0, M, cb, bytes;
};
__host__ __device__ inline TabOff tab_off(int J, int S, int MX, int Lp)
{
    TabOff o;
    o.P = 0;
    o.D = o.P + align16(J * S * MX * 2);
    o.R = o.D + align16(J * 4);
    o.ord0 = o.R + align16(J * 4);
    o.M = o.ord0 + align16(J * 2);
    o.cb = o.M + align16(S * 4);
    o.bytes = o.cb + Lp;   // Lp is a multiple of 16
    return o;
}

// LDS bytes of the shared tables and of one wave's work area.
__host__ __device__ inline int tables_bytes(int J, int S, int MX, int Lp) { return tab_off(J, S, MX, Lp).bytes; }
__host__ __device__ inline int wave_bytes(int Lp, int Jp) { return Lp + Jp * 2 * 2 + Jp * 4 * 2 + Jp * 8; }

struct Smem {
    uint16_t* P;
    int* D;
    int* R;
    uint16_t* ord0;
    int* M;
    uint8_t* cb;   // [Lp]: M_s - 1 of gene i's stage (0 past the string): complement base
};

__device__ __forceinline__ Smem smem_tables(unsigned char* base, const TtDesc& d)
{
    const TabOff o = tab_off(d.J, d.S, d.MX, d.Lp);
    Smem s;
    s.P = reinterpret_cast<uint16_t*>(base + o.P);
    s.D = reinterpret_cast<int*>(base + o.D);
    s.R = reinterpret_cast<int*>(base + o.R);
    s.ord0 = reinterpret_cast<uint16_t*>(base + o.ord0);
    s.M = reinterpret_cast<int*>(base + o.M);
    s.cb = base + o.cb;
    return s;
}

// Copy of the table image into LDS at `base`: every thread issues its (up to
// four) 16-byte global reads before its LDS writes, so a workgroup waits for
// one round trip per 4 x blockDim vectors.  Past the end a thread reads and
// writes the last vector again, with the same value, so that no branch pulls
// a read down to its write.
typedef uint32_t tab_vec4 __attribute__((ext_vector_type(4)));

__device__ void stage_tables(const TtDesc& d, unsigned char* base)
{
    constexpr int U = 4;
    const auto* src = (const __attribute__((address_space(1))) tab_vec4*)d.tab;   // global, not flat, reads
    tab_vec4* dst = reinterpret_cast<tab_vec4*>(base);
    const int nv = d.tab_vec;
    for (int v0 = threadIdx.x; v0 < nv; v0 += U * blockDim.x) {
        tab_vec4 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * (int)blockDim.x;
            x[u] = src[v < nv ? v : nv - 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * (int)blockDim.x;
            dst[v < nv ? v : nv - 1] = x[u];
        }
    }
}

// Wave-wide inclusive scans in registers (DPP): row_shr 1, 2, 4, 8 inside
// each 16-lane row, then row_bcast 15 (rows 1 and 3 take the last lane of the
// row before) and row_bcast 31 (rows 2 and 3 take lane 31).  A lane whose
// source is outside its row, or whose row is masked off, reads the identity.
template <int CTRL, int ROWS>
__device__ __forceinline__ void maxplus_step(int& A, int& B)
{
    const int Al = __builtin_amdgcn_update_dpp(kNeg, A, CTRL, ROWS, 0xF, false);
    int Bl = __builtin_amdgcn_update_dpp(0, B, CTRL, ROWS, 0xF, false);
    // keep the shifted value in its own register: fused into the subtraction
    // (v_subrev_u32_dpp) the shift was measured to apply to the other operand
    asm volatile("" : "+v"(Bl));
    const int a2 = A - Bl;
    A = Al > a2 ? Al : a2;
    B = Bl + B;
}

// (A, B) under "left then right": (max(A_l, A_r - B_l), B_l + B_r)
__device__ __forceinline__ void scan_maxplus(int& A, int& B)
{
    maxplus_step<0x111, 0xF>(A, B);
    maxplus_step<0x112, 0xF>(A, B);
    maxplus_step<0x114, 0xF>(A, B);
    maxplus_step<0x118, 0xF>(A, B);
    maxplus_step<0x142, 0xA>(A, B);
    maxplus_step<0x143, 0xC>(A, B);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ int add_step(int x)
{
    return x + __builtin_amdgcn_update_dpp(0, x, CTRL, ROWS, 0xF, false);
}

__device__ __forceinline__ int scan_add(int x)
{
    x = add_step<0x111, 0xF>(x);
    x = add_step<0x112, 0xF>(x);
    x = add_step<0x114, 0xF>(x);
    x = add_step<0x118, 0xF>(x);
    x = add_step<0x142, 0xA>(x);
    x = add_step<0x143, 0xC>(x);
    return x;
}

// value of lane - 1 (lane 0 reads `first`)
__device__ __forceinline__ int from_lane_below(int x, int first)
{
    return __builtin_amdgcn_update_dpp(first, x, 0x138 /* wave_shr:1 */, 0xF, 0xF, false);
}

// Key of a position in its machine's list: ordered by (completion, position),
// with the job in the low bits for whoever writes the merged order.
__device__ __forceinline__ unsigned long long order_key(int c, int t, int j)
{
    return ((unsigned long long)(unsigned)c << 32) | ((unsigned)t << 16) | (unsigned)j;
}

// The largest power of two not above x (x >= 1).
__device__ __forceinline__ int top_pow2(int x)
{
    return 1 << (31 - __builtin_clz((unsigned)x));
}

// The objective of the assignment in `child` (LDS, J*S genes), decoded by
// the whole wave; -1 if a gene is out of range.  Work arrays in LDS:
// ord/rdy (two buffers each, Jp entries) and keys (Jp entries).  A lane owns
// K = ceil(J / 64) <= KMAX consecutive positions.
template <int KMAX, int MMX>
__device__ long long decode_wave(const TtDesc& d, const Smem& sm, const uint8_t* child, uint16_t* ordA,
                                 uint16_t* ordB, int* rdyA, int* rdyB, unsigned long long* keys, int lane)
{
    const int J = d.J, S = d.S, MX = d.MX;
    const int K = (J + 63) >> 6;
    const int t0 = lane * K;
    bool bad = false;
    for (int u = 0; u < K; ++u) {
        const int t = t0 + u;
        if (t < J) {
            const int j = sm.ord0[t];
            ordA[t] = (uint16_t)j;
            rdyA[t] = sm.R[j];
        }
    }
    wave_sync();
    int cloc[KMAX];
    int jloc[KMAX];
    for (int s = 0; s < S; ++s) {
        const int Ms = sm.M[s];
        int mloc[KMAX], rloc[KMAX], ploc[KMAX];
        int A[MMX], B[MMX], cnt[MMX];
#pragma unroll
        for (int m = 0; m < MMX; ++m) {
            A[m] = kNeg;
            B[m] = 0;
            cnt[m] = 0;
        }
        // the lane's positions: machine, ready time, processing time
#pragma unroll
        for (int u = 0; u < KMAX; ++u) {
            mloc[u] = -1;
            if (u < K && t0 + u < J) {
                const int t = t0 + u;
                const int j = ordA[t];
                int m = child[j * S + s];
                if (m >= Ms) {
                    bad = true;
                    m = 0;
                }
                const int r = rdyA[t];
                const int p = sm.P[(j * S + s) * MX + m];
                jloc[u] = j;
                mloc[u] = m;
                rloc[u] = r;
                ploc[u] = p;
#pragma unroll
                for (int mm = 0; mm < MMX; ++mm)
                    if (mm == m) {
                        const int a2 = r - B[mm];
                        A[mm] = A[mm] > a2 ? A[mm] : a2;
                        B[mm] += p;
                        cnt[mm] += 1;
                    }
            }
        }
        // across lanes: exclusive prefix of every machine's (A, B) and count
        int off[MMX], tot[MMX];
        int run_off = 0;
#pragma unroll
        for (int m = 0; m < MMX; ++m) {
            off[m] = run_off;
            tot[m] = 0;
            if (m < Ms) {   // the stage's machines only (uniform)
                int Ai = A[m], Bi = B[m];
                scan_maxplus(Ai, Bi);
                A[m] = from_lane_below(Ai, kNeg);   // exclusive prefix
                B[m] = from_lane_below(Bi, 0);
                if (MMX == 2 && m == 1) {
                    // two machines: the lanes below hold min(t0, J) positions,
                    // those not on machine 0 are on machine 1
                    tot[1] = J - tot[0];
                    cnt[1] = (t0 < J ? t0 : J) - cnt[0];
                } else {
                    const int ci = scan_add(cnt[m]);
                    tot[m] = __builtin_amdgcn_readlane(ci, 63);
                    cnt[m] = ci - cnt[m];   // exclusive: entries of machine m before this lane
                }
                run_off += tot[m];
            }
        }
        // completions; except at the last stage (whose order nobody reads),
        // each machine's list of keys (completion << 32 | position << 16 |
        // job), sorted by (completion, position): first in, first out on a
        // machine, ties to the earlier position
        const bool more = s + 1 < S;
        int own[KMAX];
#pragma unroll
        for (int u = 0; u < KMAX; ++u) {
            if (mloc[u] >= 0) {
                const int m = mloc[u];
                int c = 0, idx = 0, base = 0;
#pragma unroll
                for (int mm = 0; mm < MMX; ++mm)
                    if (mm == m) {
                        const int a2 = rloc[u] - B[mm];
                        A[mm] = A[mm] > a2 ? A[mm] : a2;
                        B[mm] += ploc[u];
                        c = (A[mm] > 0 ? A[mm] : 0) + B[mm];
                        idx = cnt[mm]++;
                        base = off[mm];
                    }
                cloc[u] = c;
                own[u] = idx;
                if (more) keys[base + idx] = order_key(c, t0 + u, jloc[u]);
            }
        }
        if (!more) break;
        wave_sync();
        if constexpr (MMX == 2) {
            // two lists (the second empty when M_s = 1): a merge path.  Lane
            // l writes merged positions [l K, l K + K): a binary search on
            // that diagonal finds how many of them come from the first list,
            // then the lane merges its K outputs in order.
            const unsigned long long* X = keys + off[0];
            const unsigned long long* Y = keys + off[1];
            const int nx = tot[0], ny = tot[1];
            const int dg = t0 < J ? t0 : J;
            int lo = dg - ny > 0 ? dg - ny : 0;
            int hi = dg < nx ? dg : nx;
            // the first list's share of positions [0, dg): the least i in
            // [lo, hi] with X[i] > Y[dg - 1 - i] (i = hi if none); hi - lo is
            // at most min(nx, ny), and every round halves the candidates
            const int span = nx < ny ? nx : ny;
            for (int step = span > 0 ? top_pow2(span) : 0; step > 0; step >>= 1) {
                if (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const bool x_first = X[mid] < Y[dg - 1 - mid];
                    lo = x_first ? mid + 1 : lo;
                    hi = x_first ? hi : mid;
                }
            }
            int i = lo, jy = dg - lo;
#pragma unroll
            for (int u = 0; u < KMAX; ++u) {
                if (u < K && dg + u < J) {
                    const unsigned long long x = i < nx ? X[i] : ~0ull;
                    const unsigned long long y = jy < ny ? Y[jy] : ~0ull;
                    const bool tx = x < y;
                    const unsigned long long kk = tx ? x : y;
                    i += tx ? 1 : 0;
                    jy += tx ? 0 : 1;
                    ordB[dg + u] = (uint16_t)(kk & 0xFFFFull);
                    rdyB[dg + u] = (int)(kk >> 32);
                }
            }
        } else {
            // rank in the next stage's order: own index plus, in every other
            // machine's list, the number of entries below the key -- a
            // power-of-two search with a fixed step sequence, run for all of
            // the lane's positions in lockstep so that their LDS reads overlap
            unsigned long long key[KMAX];
#pragma unroll
            for (int u = 0; u < KMAX; ++u)
                key[u] = order_key(mloc[u] >= 0 ? cloc[u] : 0, t0 + u, mloc[u] >= 0 ? jloc[u] : 0);
            const int top = top_pow2(J) << 1;
            for (int oi = 1; oi < Ms; ++oi) {
                // position u searches machine (m_u + oi) mod Ms: each other machine once
                int lb[KMAX], n[KMAX], pos[KMAX];
#pragma unroll
                for (int u = 0; u < KMAX; ++u) {
                    int om = (mloc[u] >= 0 ? mloc[u] : 0) + oi;
                    om = om >= Ms ? om - Ms : om;
                    int ob = 0, on = 0;
#pragma unroll
                    for (int mm = 0; mm < MMX; ++mm)
                        if (mm == om) {
                            ob = off[mm];
                            on = tot[mm];
                        }
                    lb[u] = ob - 1;
                    n[u] = (mloc[u] >= 0) ? on : 0;
                    pos[u] = 0;
                }
                for (int step = top >> 1; step > 0; step >>= 1) {
#pragma unroll
                    for (int u = 0; u < KMAX; ++u) {
                        if (u < K) {   // uniform
                            const int at = pos[u] + step;
                            // entries lst[0..at) all below the key: advance
                            if (at <= n[u] && keys[lb[u] + at] < key[u]) pos[u] = at;
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < KMAX; ++u)
                    if (mloc[u] >= 0) own[u] += pos[u];
            }
#pragma unroll
            for (int u = 0; u < KMAX; ++u)
                if (mloc[u] >= 0) {
                    ordB[own[u]] = (uint16_t)jloc[u];
                    rdyB[own[u]] = cloc[u];
                }
        }
        wave_sync();
        uint16_t* to = ordA;
        ordA = ordB;
        ordB = to;
        int* tr = rdyA;
        rdyA = rdyB;
        rdyB = tr;
    }
    // the last stage's completions are in cloc (jobs jloc)
    long long tard = 0;
    int cmax = 0;
#pragma unroll
    for (int u = 0; u < KMAX; ++u)
        if (u < K && t0 + u < J) {
            const int late = cloc[u] - sm.D[jloc[u]];
            if (late > 0) tard += late;
            cmax = cloc[u] > cmax ? cloc[u] : cmax;
        }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        tard += __shfl_xor(tard, o, 64);
        const int c2 = __shfl_xor(cmax, o, 64);
        cmax = c2 > cmax ? c2 : cmax;
    }
    const bool anybad = __any(bad);
    return anybad ? -1ll : d.WT * tard + (long long)cmax;
}

struct WaveMem {
    uint8_t* child;
    uint16_t *ordA, *ordB;
    int *rdyA, *rdyB;
    unsigned long long* keys;
};

__device__ __forceinline__ WaveMem wave_mem(unsigned char* base, int Lp, int Jp)
{
    WaveMem w;
    w.child = base;
    base += Lp;
    w.ordA = reinterpret_cast<uint16_t*>(base);
    base += Jp * 2;
    w.ordB = reinterpret_cast<uint16_t*>(base);
    base += Jp * 2;
    w.rdyA = reinterpret_cast<int*>(base);
    base += Jp * 4;
    w.rdyB = reinterpret_cast<int*>(base);
    base += Jp * 4;
    w.keys = reinterpret_cast<unsigned long long*>(base);
    return w;
}

extern __shared__ __align__(16) unsigned char tt_smem[];

// Generation `gen` of every run:
//   mode 1: generation 0 (random assignments; a pseudo pair = X and its
//           complement), every individual;
//   mode 0: every island steps from generation gen - 1 (synchronous update);
//   mode 2: the cells of cellular island `sel` on anti-diagonal `diag`
//           (r + c = diag) of a line-sweep generation.  In row-major order a
//           neighbour precedes the cell exactly when its diagonal is lower
//           (the torus's wrapped neighbours included), so it is read from the
//           new generation's buffer then and from the previous one otherwise;
//           the diagonals run in order, one launch each;
//   mode 3: the individuals of the pseudo islands only (`count` per run).
template <int KMAX, int MMX>
__global__ void __launch_bounds__(256) k_tt_generation(TtDesc d, int gen, int mode, int sel, int diag, int count)
{
    const Smem sm = smem_tables(tt_smem, d);
    stage_tables(d, tt_smem);
    __syncthreads();
    const int wpb = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long wg = (long long)blockIdx.x * wpb + wave;
    const int per_run = (mode <= 1) ? d.N : count;
    if (wg >= (long long)d.runs * per_run) return;
    const int run = (int)(wg / per_run), q0 = (int)(wg - (long long)run * per_run);
    int isl = 0, slot = 0;
    if (mode <= 1) {
#pragma unroll
        for (int i = 1; i < kMaxIsl; ++i)
            if (i < d.n_isl && q0 >= d.isl[i].off) isl = i;
        slot = q0 - island_at(d, isl).off;
    } else if (mode == 2) {
        const TtIsland C = island_at(d, sel);
        const int rlo = diag - (C.cols - 1) > 0 ? diag - (C.cols - 1) : 0;
        const int r = rlo + q0;
        isl = sel;
        slot = r * C.cols + (diag - r);
    } else {
        // q0-th individual among the pseudo islands, in island order
        int left = q0;
#pragma unroll
        for (int i = 0; i < kMaxIsl; ++i) {
            const TtIsland X = d.isl[i];
            if (i < d.n_isl && X.kind == 1 && left >= 0) {
                if (left < X.size) {
                    isl = i;
                    slot = left;
                }
                left -= X.size;
            }
        }
    }
    const TtIsland I = island_at(d, isl);
    const int L = d.L, Lp = d.Lp, S = d.S;
    const WaveMem w = wave_mem(tt_smem + tables_bytes(d.J, S, d.MX, d.Lp) + wave * wave_bytes(Lp, d.Jp), Lp, d.Jp);
    const int cur = (gen + 1) & 1, nxt = gen & 1;
    const long long rowbase = (long long)run * d.N + I.off;   // individual index of slot 0
    uint8_t* child = w.child;

    if (mode == 1) {
        const int src = (I.kind == 0) ? slot : (slot >> 1);
        const bool comp = (I.kind == 1) && (slot & 1);
        const int nblk = (L + 7) >> 3;
        for (int blk = lane; blk < nblk; blk += 64) {
            const Block4 b = stream_block(d.seed, (uint64_t)run, (uint32_t)isl, (uint32_t)src, 0, 0, flowshop::kInit,
                                          (uint32_t)blk);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i = blk * 8 + q;
                if (i < L) {
                    const int ms = sm.M[i % S];
                    const int g = (int)below(draw32(b, q), (uint32_t)ms);
                    child[i] = (uint8_t)(comp ? ms - 1 - g : g);
                }
            }
        }
    } else if (I.kind == 0) {
        const int r = slot / I.cols, c = slot - r * I.cols;
        const int rn = (r == 0) ? I.rows - 1 : r - 1, rs = (r == I.rows - 1) ? 0 : r + 1;
        const int ce = (c == I.cols - 1) ? 0 : c + 1, cw = (c == 0) ? I.cols - 1 : c - 1;
        const int nb[5] = {slot, rn * I.cols + c, r * I.cols + ce, rs * I.cols + c, r * I.cols + cw};
        // buffer of each neighbour: the new generation's for the cells a line
        // sweep has already updated (lower diagonal), else the previous one
        const int nd[5] = {r + c, rn + c, r + ce, rs + c, r + cw};
        int buf[5];
        long long v[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            buf[q] = (mode == 2 && q > 0 && nd[q] < diag) ? nxt : cur;
            v[q] = d.obj[buf[q]][rowbase + nb[q]];
        }
        // the two best by (objective, neighbourhood order)
        int b = 0, p1 = nb[0], b1 = buf[0];
        long long bv = v[0];
#pragma unroll
        for (int q = 1; q < 5; ++q)
            if (v[q] < bv) {
                bv = v[q];
                b = q;
                p1 = nb[q];
                b1 = buf[q];
            }
        int s2 = -1, p2 = nb[0], b2 = buf[0];
        long long sv = 0;
#pragma unroll
        for (int q = 0; q < 5; ++q)
            if (q != b && (s2 < 0 || v[q] < sv)) {
                sv = v[q];
                s2 = q;
                p2 = nb[q];
                b2 = buf[q];
            }
        const Block4 bk = stream_block(d.seed, (uint64_t)run, (uint32_t)isl, (uint32_t)slot, 0, (uint32_t)gen,
                                       flowshop::kCell, 0);
        const bool cx = (unsigned long long)draw32(bk, 0) < I.tc;
        const int u = (int)below(draw32(bk, 1), (uint32_t)L), v2 = (int)below(draw32(bk, 2), (uint32_t)L);
        const int a = u < v2 ? u : v2, e = u < v2 ? v2 : u;
        const uint8_t* P1 = d.genes[b1] + (rowbase + p1) * Lp;
        const uint8_t* P2 = d.genes[b2] + (rowbase + p2) * Lp;
        for (int i0 = lane * 16; i0 < Lp; i0 += 64 * 16) {
            const uint4 x1 = *reinterpret_cast<const uint4*>(P1 + i0);
            const uint4 x2 = *reinterpret_cast<const uint4*>(P2 + i0);
            uint32_t o[4];
#pragma unroll
            for (int wd = 0; wd < 4; ++wd) {
                // byte mask of the positions taken from P1
                uint32_t mask = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = i0 + wd * 4 + q;
                    if (!cx || (i >= a && i <= e)) mask |= 0xFFu << (8 * q);
                }
                o[wd] = (word_of(x1, wd) & mask) | (word_of(x2, wd) & ~mask);
            }
            *reinterpret_cast<uint4*>(child + i0) = make_uint4(o[0], o[1], o[2], o[3]);
        }
        wave_sync();
        if (lane == 0 && (unsigned long long)draw32(bk, 3) < I.tm) {
            const int i = (int)below(draw32(bk, 4), (uint32_t)L);
            const int ms = sm.M[i % S];
            if (ms >= 2) child[i] = (uint8_t)((child[i] + 1 + (int)below(draw32(bk, 5), (uint32_t)(ms - 1))) % ms);
        }
    } else {
        const long long* ob = d.obj[cur] + rowbase;
        const int q = slot >> 1;
        const bool odd = slot & 1;
        const int xs = (ob[2 * q] <= ob[2 * q + 1]) ? 2 * q : 2 * q + 1;
        const Block4 b0 = stream_block(d.seed, (uint64_t)run, (uint32_t)isl, (uint32_t)q, 0, (uint32_t)gen,
                                       flowshop::kPair, 0);
        const Block4 b1 = stream_block(d.seed, (uint64_t)run, (uint32_t)isl, (uint32_t)q, 0, (uint32_t)gen,
                                       flowshop::kPair, 1);
        const bool cx = (unsigned long long)draw32(b0, 0) < I.tc;
        const int u = (int)below(draw32(b0, 1), (uint32_t)L), v2 = (int)below(draw32(b0, 2), (uint32_t)L);
        const int a = u < v2 ? u : v2, e = u < v2 ? v2 : u;
        const uint32_t dm = odd ? draw32(b0, 6) : draw32(b0, 3);
        const uint32_t di = odd ? draw32(b0, 7) : draw32(b0, 4);
        const uint32_t dr = odd ? draw32(b1, 0) : draw32(b0, 5);
        const uint8_t* X = d.genes[cur] + (rowbase + xs) * Lp;
        for (int i0 = lane * 16; i0 < Lp; i0 += 64 * 16) {
            const uint4 x1 = *reinterpret_cast<const uint4*>(X + i0);
            const uint4 c1 = *reinterpret_cast<const uint4*>(sm.cb + i0);
            uint32_t o[4];
#pragma unroll
            for (int wd = 0; wd < 4; ++wd) {
                const uint32_t xw = word_of(x1, wd);
                // complement of four genes at once: every byte of the base is
                // >= the gene below it, so the subtraction borrows only in the
                // padding past the string (higher bytes)
                const uint32_t yw = word_of(c1, wd) - xw;
                uint32_t mask = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = i0 + wd * 4 + q;
                    // even child: X on [a, b], complement elsewhere (X if no
                    // crossover); odd child: the opposite
                    const bool takex = cx ? ((i >= a && i <= e) != odd) : !odd;
                    if (takex) mask |= 0xFFu << (8 * q);
                }
                o[wd] = (xw & mask) | (yw & ~mask);
            }
            *reinterpret_cast<uint4*>(child + i0) = make_uint4(o[0], o[1], o[2], o[3]);
        }
        wave_sync();
        if (lane == 0 && (unsigned long long)dm < I.tm) {
            const int i = (int)below(di, (uint32_t)L);
            const int ms = sm.M[i % S];
            if (ms >= 2) child[i] = (uint8_t)((child[i] + 1 + (int)below(dr, (uint32_t)(ms - 1))) % ms);
        }
    }
    wave_sync();
    const long long o = decode_wave<KMAX, MMX>(d, sm, child, w.ordA, w.ordB, w.rdyA, w.rdyB, w.keys, lane);
    // replacement (cellular: only if strictly better) and write-out
    uint8_t* dst = d.genes[nxt] + (rowbase + slot) * Lp;
    long long onew = o;
    const uint8_t* srow = child;
    if (mode != 1 && I.kind == 0) {
        const long long oold = d.obj[cur][rowbase + slot];
        if (!(o < oold)) {
            onew = oold;
            srow = d.genes[cur] + (rowbase + slot) * Lp;
        }
    }
    for (int i0 = lane * 16; i0 < Lp; i0 += 64 * 16)
        *reinterpret_cast<uint4*>(dst + i0) = *reinterpret_cast<const uint4*>(srow + i0);
    if (lane == 0) {
        d.obj[nxt][rowbase + slot] = onew;
        if (o < 0) atomicOr(d.err, 1);
        atomicMin(d.genkey + ((long long)run * d.n_isl + isl) * 2 + (gen & 1),
                  ((unsigned long long)onew << 13) | (unsigned)slot);
    }
}

// Best-ever record of every run after generation `gen`, one wave per run:
// the minimum (objective, island, slot) of the generation replaces the
// record if its objective is strictly lower; the generation's keys are
// reset.  Every lane reads the keys and the record and takes the same
// decision; the wave copies the row, and lane 0 writes the keys and the
// record after the reads they depend on.
__global__ void __launch_bounds__(64) k_tt_fold(TtDesc d, int gen)
{
    const int run = blockIdx.x, lane = threadIdx.x;
    if (run >= d.runs) return;
    const int par = gen & 1;
    unsigned long long* gk = d.genkey + (long long)run * d.n_isl * 2 + par;   // island i at gk[2 i]
    long long bo = 0;
    int bi = -1, bs = 0;
    for (int i = 0; i < d.n_isl; ++i) {
        const unsigned long long v = gk[2 * i];
        const long long oi = (long long)(v >> 13);
        // every island posts a key each generation; an unset key is skipped
        if (v != ~0ull && (bi < 0 || oi < bo)) {
            bo = oi;
            bi = i;
            bs = (int)(v & 8191u);
        }
    }
    long long* rec = d.best + (long long)run * 4;
    const bool better = bi >= 0 && (rec[2] < 0 || bo < rec[0]);
    if (better) {
        const uint4* s4 =
            reinterpret_cast<const uint4*>(d.genes[par] + ((long long)run * d.N + island_at(d, bi).off + bs) * d.Lp);
        uint4* d4 = reinterpret_cast<uint4*>(d.best_genes + (long long)run * d.Lp);
        for (int v = lane; v < d.Lp / 16; v += 64) d4[v] = s4[v];
    }
    if (lane == 0) {
        for (int i = 0; i < d.n_isl; ++i) gk[2 * i] = ~0ull;
        if (better) {
            rec[0] = bo;
            rec[1] = gen;
            rec[2] = bi;
            rec[3] = bs;
        }
    }
}

// Slots of one island by (objective, slot) ascending into keys[0..size):
// bitonic sort of objective << 13 | slot over a power-of-two span.
__device__ void sort_island(unsigned long long* keys, const long long* obj, int size)
{
    int span = 1;
    while (span < size) span <<= 1;
    for (int i = threadIdx.x; i < span; i += blockDim.x)
        keys[i] = (i < size) ? (((unsigned long long)obj[i] << 13) | (unsigned)i) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= span; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < span; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long x = keys[i], y = keys[l];
                    const bool up = (i & k) == 0;
                    if ((x > y) == up) {
                        keys[i] = y;
                        keys[l] = x;
                    }
                }
            }
            __syncthreads();
        }
}

// Migration epoch of island pair (i, i + H) of run blockIdx.x / H on the
// completed generation `gen` (equations (1) and (2), exact integers).
__global__ void __launch_bounds__(kSortThreads) k_tt_migrate(TtDesc d, int gen)
{
    const int run = blockIdx.x / d.H, pi = blockIdx.x - run * d.H;
    const int par = gen & 1;
    const TtIsland IA = island_at(d, pi), IB = island_at(d, pi + d.H);
    long long* oa = d.obj[par] + (long long)run * d.N + IA.off;
    long long* ob = d.obj[par] + (long long)run * d.N + IB.off;
    unsigned long long* ka = reinterpret_cast<unsigned long long*>(tt_smem);
    unsigned long long* kb = ka + kMaxIslSize;
    sort_island(ka, oa, IA.size);
    sort_island(kb, ob, IB.size);
    __shared__ long long s_count;
    __shared__ int s_a_sends;
    if (threadIdx.x == 0) {
        long long fa = d.E - (long long)(ka[0] >> 13), fb = d.E - (long long)(kb[0] >> 13);
        fa = fa < 0 ? 0 : fa;
        fb = fb < 0 ? 0 : fb;
        long long count = 0;
        const int a_sends = fa > fb;
        if (fa != fb) {
            const unsigned __int128 hi = (unsigned __int128)(unsigned long long)(fa > fb ? fa : fb);
            const unsigned __int128 lo = (unsigned __int128)(unsigned long long)(fa > fb ? fb : fa);
            if (hi != 0 && ((hi - lo) << 32) < (unsigned __int128)d.theta_T * hi) {
                const unsigned __int128 n = (unsigned __int128)(IA.size < IB.size ? IA.size : IB.size);
                unsigned __int128 c = (n * (hi - lo) + hi - 1) / hi;
                if (c > n) c = n;
                count = (long long)c;
            }
        }
        s_count = count;
        s_a_sends = a_sends;
        if (count > 0) {
            // the pairs of one run update its counters from different workgroups
            atomicAdd(reinterpret_cast<unsigned long long*>(d.counters + run * 2 + 0), 1ull);
            atomicAdd(reinterpret_cast<unsigned long long*>(d.counters + run * 2 + 1), (unsigned long long)count);
        }
    }
    __syncthreads();
    const long long count = s_count;
    if (count == 0) return;
    const bool a_sends = s_a_sends;
    const unsigned long long* ks = a_sends ? ka : kb;
    const unsigned long long* kd = a_sends ? kb : ka;
    const TtIsland Is = a_sends ? IA : IB, Id = a_sends ? IB : IA;
    long long* os = a_sends ? oa : ob;
    long long* od = a_sends ? ob : oa;
    const int vpr = d.Lp / 16;
    for (long long x = threadIdx.x; x < count * vpr; x += blockDim.x) {
        const int r = (int)(x / vpr), v = (int)(x - (long long)r * vpr);
        const int ss = (int)(ks[r] & 8191u), ds = (int)(kd[Id.size - 1 - r] & 8191u);
        const uint4* s4 = reinterpret_cast<const uint4*>(d.genes[par] + ((long long)run * d.N + Is.off + ss) * d.Lp);
        uint4* d4 = reinterpret_cast<uint4*>(d.genes[par] + ((long long)run * d.N + Id.off + ds) * d.Lp);
        d4[v] = s4[v];
        if (v == 0) od[ds] = os[ss];
    }
}

// Objectives of caller-supplied assignments (count rows of L genes).
template <int KMAX, int MMX>
__global__ void __launch_bounds__(256) k_tt_evaluate(TtDesc d, const uint8_t* genes, int count, long long* out)
{
    const Smem sm = smem_tables(tt_smem, d);
    stage_tables(d, tt_smem);
    __syncthreads();
    const int wpb = blockDim.x >> 6, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long row = (long long)blockIdx.x * wpb + wave;
    if (row >= count) return;
    const WaveMem w = wave_mem(tt_smem + tables_bytes(d.J, d.S, d.MX, d.Lp) + wave * wave_bytes(d.Lp, d.Jp), d.Lp, d.Jp);
    const uint8_t* src = genes + row * d.L;
    for (int i = lane; i < d.L; i += 64) w.child[i] = src[i];
    wave_sync();
    const long long o = decode_wave<KMAX, MMX>(d, sm, w.child, w.ordA, w.ordB, w.rdyA, w.rdyB, w.keys, lane);
    if (lane == 0) out[row] = o;
}

}  // namespace tt

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace tt;

struct ffs_tt_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    std::string err;
    // instance
    bool have_inst = false;
    int J = 0, S = 0, MX = 0, L = 0, Lp = 0, Jp = 0;
    std::vector<int> M, R, D;
    std::vector<uint16_t> P, ord0;
    long long WT = 0, E = 0;
    // islands and configuration
    std::vector<ffs_island_spec> isl;
    int interval = 0, runs = 1;
    double theta = 1.0;
    uint64_t seed = 0;
    bool configured = false;
    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    int gen = 0;
    TtDesc desc{};
    int sweep = 0;   // cellular update: 0 synchronous, 1 line sweep
    int wpb = 4;
    int kmax = 16;   // positions per lane bound of the decode (8 when J <= 512)
    int mmx = 4;     // machines per stage bound of the decode (2 when every M_s <= 2)
    size_t lds_gen = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    double t_ms = 0;
    long long t_n = 0;
};

namespace {

int fail(ffs_tt_ctx* c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define TT_HIP(c, call)                                                                         \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return fail((c), FFS_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

unsigned long long rate_T(double p)
{
    if (p <= 0.0) return 0ull;
    if (p >= 1.0) return 4294967296ull;
    return (unsigned long long)(p * 4294967296.0);
}

struct Layout {
    size_t genes[2], obj[2], genkey, best, best_genes, counters, err, tab, total;
};

Layout layout_of(const ffs_tt_ctx* c)
{
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) & ~(size_t)255;
        return at;
    };
    size_t N = 0;
    for (const auto& s : c->isl) N += (size_t)((s.kind == 0) ? s.rows * s.cols : s.size);
    const size_t R = (size_t)c->runs;
    for (int p = 0; p < 2; ++p) l.genes[p] = take(R * N * c->Lp);
    for (int p = 0; p < 2; ++p) l.obj[p] = take(R * N * 8);
    l.genkey = take(R * c->isl.size() * 2 * 8);
    l.best = take(R * 4 * 8);
    l.best_genes = take(R * c->Lp);
    l.counters = take(R * 2 * 8);
    l.err = take(4);
    l.tab = take((size_t)tables_bytes(c->J, c->S, c->MX, c->Lp));
    l.total = off;
    return l;
}

int check_ready(ffs_tt_ctx* c)
{
    if (!c) return FFS_EINVAL;
    if (!c->bound) return fail(c, FFS_ESTATE, "workspace not bound");
    return FFS_OK;
}

int launch_one(ffs_tt_ctx* c, int gen, int mode, int sel, int diag, int count, long long waves)
{
    if (waves <= 0) return FFS_OK;
    const unsigned blocks = (unsigned)((waves + c->wpb - 1) / c->wpb);
    const TtDesc& d = c->desc;
    if (c->kmax == 8 && c->mmx == 2)
        hipLaunchKernelGGL((k_tt_generation<8, 2>), dim3(blocks), dim3(64 * c->wpb), c->lds_gen, c->stream, d, gen,
                           mode, sel, diag, count);
    else if (c->kmax == 8)
        hipLaunchKernelGGL((k_tt_generation<8, 4>), dim3(blocks), dim3(64 * c->wpb), c->lds_gen, c->stream, d, gen,
                           mode, sel, diag, count);
    else if (c->mmx == 2)
        hipLaunchKernelGGL((k_tt_generation<16, 2>), dim3(blocks), dim3(64 * c->wpb), c->lds_gen, c->stream, d, gen,
                           mode, sel, diag, count);
    else
        hipLaunchKernelGGL((k_tt_generation<16, 4>), dim3(blocks), dim3(64 * c->wpb), c->lds_gen, c->stream, d, gen,
                           mode, sel, diag, count);
    TT_HIP(c, hipGetLastError());
    return FFS_OK;
}

// One generation (mode 1: generation 0; mode 0: a step, synchronous or as a
// line sweep: the pseudo islands in one launch, then every cellular island
// one anti-diagonal per launch), then the best-ever fold.
int launch_gen(ffs_tt_ctx* c, int gen, int mode)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        while (c->ev.size() < c->ev_used + 2) {
            hipEvent_t e;
            TT_HIP(c, hipEventCreate(&e));
            c->ev.push_back(e);
        }
        e0 = c->ev[c->ev_used++];
        e1 = c->ev[c->ev_used++];
        TT_HIP(c, hipEventRecord(e0, c->stream));
    }
    int rc = FFS_OK;
    const TtDesc& d = c->desc;
    if (mode == 1 || !c->sweep) {
        rc = launch_one(c, gen, mode, 0, 0, 0, (long long)c->runs * d.N);
    } else {
        int np = 0;
        for (int i = 0; i < d.n_isl; ++i)
            if (d.isl[i].kind == 1) np += d.isl[i].size;
        rc = launch_one(c, gen, 3, 0, 0, np, (long long)c->runs * np);
        for (int i = 0; i < d.n_isl && rc == FFS_OK; ++i) {
            if (d.isl[i].kind != 0) continue;
            const int rows = d.isl[i].rows, cols = d.isl[i].cols;
            for (int g = 0; g <= rows + cols - 2 && rc == FFS_OK; ++g) {
                const int rlo = std::max(0, g - (cols - 1)), rhi = std::min(rows - 1, g);
                rc = launch_one(c, gen, 2, i, g, rhi - rlo + 1, (long long)c->runs * (rhi - rlo + 1));
            }
        }
    }
    if (rc != FFS_OK) return rc;
    if (c->timing) TT_HIP(c, hipEventRecord(e1, c->stream));
    hipLaunchKernelGGL(k_tt_fold, dim3((unsigned)c->runs), dim3(64), 0, c->stream, c->desc, gen);
    TT_HIP(c, hipGetLastError());
    return FFS_OK;
}

int launch_migrate(ffs_tt_ctx* c, int gen)
{
    if (c->desc.H == 0) return FFS_OK;
    const size_t lds = (size_t)2 * kMaxIslSize * 8;
    hipLaunchKernelGGL(k_tt_migrate, dim3((unsigned)(c->runs * c->desc.H)), dim3(kSortThreads), lds, c->stream,
                       c->desc, gen);
    TT_HIP(c, hipGetLastError());
    return FFS_OK;
}

int collect_timing(ffs_tt_ctx* c)
{
    if (c->ev_used == 0) return FFS_OK;
    TT_HIP(c, hipStreamSynchronize(c->stream));
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.f;
        TT_HIP(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        c->t_ms += ms;
        c->t_n += 1;
    }
    c->ev_used = 0;
    return FFS_OK;
}

}  // namespace

extern "C" {

int ffs_tt_create(void* stream, ffs_tt_ctx** out)
{
    if (!out) return FFS_EINVAL;
    ffs_tt_ctx* c = new (std::nothrow) ffs_tt_ctx();
    if (!c) return FFS_ENOMEM;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return FFS_EDEVICE;
    }
    *out = c;
    return FFS_OK;
}

int ffs_tt_destroy(ffs_tt_ctx* c)
{
    if (!c) return FFS_EINVAL;
    if (c->stream || c->bound) (void)hipStreamSynchronize(c->stream);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    delete c;
    return FFS_OK;
}

const char* ffs_tt_last_error(const ffs_tt_ctx* c) { return c ? c->err.c_str() : "null context"; }

int ffs_tt_set_instance(ffs_tt_ctx* c, int32_t J, int32_t S, const int32_t* M, int32_t MX, const int32_t* P,
                        const int32_t* R, const int64_t* D, int64_t WT)
{
    if (!c) return FFS_EINVAL;
    if (c->bound) return fail(c, FFS_ESTATE, "instance set after bind");
    if (!M || !P || !R || !D) return fail(c, FFS_EINVAL, "null array");
    if (J < 1 || S < 1 || MX < 1 || WT < 0) return fail(c, FFS_EINVAL, "bad sizes J=%d S=%d MX=%d WT=%lld", J, S, MX, (long long)WT);
    if (J > kMaxJ || S > kMaxS || MX > kMaxM)
        return fail(c, FFS_EUNSUPPORTED, "J=%d S=%d MX=%d beyond 1024 / 32 / 4", J, S, MX);
    int mx = 0;
    for (int s = 0; s < S; ++s) {
        if (M[s] < 1 || M[s] > MX) return fail(c, FFS_EINVAL, "M[%d]=%d outside [1, MX]", s, M[s]);
        mx = std::max(mx, (int)M[s]);
    }
    if (mx != MX) return fail(c, FFS_EINVAL, "MX=%d is not max M_s=%d", MX, mx);
    long long H = 0, rmax = 0;
    for (int j = 0; j < J; ++j) {
        if (R[j] < 0) return fail(c, FFS_EINVAL, "R[%d] < 0", j);
        rmax = std::max(rmax, (long long)R[j]);
        if (D[j] < -(1ll << 30) || D[j] > (1ll << 30)) return fail(c, FFS_EUNSUPPORTED, "D[%d] beyond 2^30", j);
        for (int s = 0; s < S; ++s) {
            long long pm = 0;
            for (int m = 0; m < M[s]; ++m) {
                const int v = P[((size_t)j * S + s) * MX + m];
                if (v < 1) return fail(c, FFS_EINVAL, "P[%d][%d][%d]=%d < 1", j, s, m, v);
                if (v > 65535) return fail(c, FFS_EUNSUPPORTED, "P[%d][%d][%d]=%d beyond 65535", j, s, m, v);
                pm = std::max(pm, (long long)v);
            }
            H += pm;
        }
    }
    H += rmax;
    if (H >= (1ll << 30)) return fail(c, FFS_EUNSUPPORTED, "schedule bound %lld beyond 2^30", H);
    long long E = H;
    for (int j = 0; j < J; ++j)
        if (H > D[j]) E += WT * (H - D[j]);
    if (E >= (1ll << 39)) return fail(c, FFS_EUNSUPPORTED, "objective bound %lld beyond 2^39", E);
    c->J = J;
    c->S = S;
    c->MX = MX;
    c->L = J * S;
    c->Lp = (c->L + 15) & ~15;
    c->Jp = (J + 7) & ~7;
    c->M.assign(M, M + S);
    c->R.assign(R, R + J);
    c->D.resize(J);
    for (int j = 0; j < J; ++j) c->D[j] = (int)D[j];
    c->P.resize((size_t)J * S * MX);
    for (size_t i = 0; i < c->P.size(); ++i) c->P[i] = (uint16_t)std::max(0, (int)P[i]);
    std::vector<int> ord(J);
    for (int j = 0; j < J; ++j) ord[j] = j;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return R[a] < R[b]; });
    c->ord0.assign(ord.begin(), ord.end());
    c->WT = WT;
    c->E = E;
    c->have_inst = true;
    return FFS_OK;
}

int ffs_tt_add_island(ffs_tt_ctx* c, const ffs_island_spec* s)
{
    if (!c || !s) return FFS_EINVAL;
    if (c->bound) return fail(c, FFS_ESTATE, "island added after bind");
    if ((int)c->isl.size() >= kMaxIsl) return fail(c, FFS_EUNSUPPORTED, "more than %d islands", kMaxIsl);
    if (s->kind != 0 && s->kind != 1) return fail(c, FFS_EINVAL, "kind %d", s->kind);
    if (s->selection != 0) return fail(c, FFS_EINVAL, "selection must be 0");
    if (s->sweep != 0) return fail(c, FFS_EINVAL, "sweep must be 0 (the update schedule is set per context)");
    if (!(s->p_c >= 0.0 && s->p_c <= 1.0 && s->p_m >= 0.0 && s->p_m <= 1.0)) return fail(c, FFS_EINVAL, "rates outside [0, 1]");
    const int size = (s->kind == 0) ? s->rows * s->cols : s->size;
    if (s->kind == 0 && (s->rows < 3 || s->cols < 3)) return fail(c, FFS_EINVAL, "cellular grid below 3x3");
    if (s->kind == 1 && (s->size < 2 || (s->size & 1))) return fail(c, FFS_EINVAL, "pseudo size must be even and >= 2");
    if (size > kMaxIslSize) return fail(c, FFS_EUNSUPPORTED, "island of %d beyond %d", size, kMaxIslSize);
    c->isl.push_back(*s);
    return FFS_OK;
}

int ffs_tt_configure(ffs_tt_ctx* c, int32_t interval, double theta, uint64_t seed, int32_t runs)
{
    if (!c) return FFS_EINVAL;
    if (c->bound) return fail(c, FFS_ESTATE, "configure after bind");
    if (interval < 0 || !(theta >= 0.0 && theta <= 1.0)) return fail(c, FFS_EINVAL, "interval %d theta %g", interval, theta);
    if (runs < 1 || runs > kMaxRuns) return fail(c, FFS_EUNSUPPORTED, "runs %d outside [1, %d]", runs, kMaxRuns);
    c->interval = interval;
    c->theta = theta;
    c->seed = seed;
    c->runs = runs;
    c->configured = true;
    return FFS_OK;
}

int ffs_tt_workspace_size(const ffs_tt_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return FFS_EINVAL;
    if (!c->have_inst || c->isl.empty()) return FFS_ESTATE;
    *bytes = layout_of(c).total;
    return FFS_OK;
}

int ffs_tt_bind_workspace(ffs_tt_ctx* c, void* ptr, size_t bytes)
{
    if (!c) return FFS_EINVAL;
    if (c->bound) return fail(c, FFS_ESTATE, "already bound");
    if (!c->have_inst || c->isl.empty()) return fail(c, FFS_ESTATE, "no instance or island");
    if (c->interval > 0 && (c->isl.size() & 1)) return fail(c, FFS_EINVAL, "migration needs an even island count");
    if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255)) return fail(c, FFS_EINVAL, "workspace not 256-byte aligned");
    const Layout l = layout_of(c);
    if (bytes < l.total) return fail(c, FFS_ENOMEM, "workspace %zu < %zu", bytes, l.total);
    // LDS: tables + waves; up to 4 waves per workgroup, fewer if that does not fit
    const size_t tb = (size_t)tables_bytes(c->J, c->S, c->MX, c->Lp), wb = (size_t)wave_bytes(c->Lp, c->Jp);
    int wpb = 4;
    while (wpb > 1 && tb + wpb * wb > 160 * 1024) --wpb;
    if (tb + wpb * wb > 160 * 1024) return fail(c, FFS_EUNSUPPORTED, "instance tables need %zu bytes of LDS", tb + wb);
    c->wpb = wpb;
    c->lds_gen = tb + wpb * wb;
    c->kmax = (c->J <= 512) ? 8 : 16;
    c->mmx = (c->MX <= 2) ? 2 : 4;
    const void* kg[4] = {reinterpret_cast<const void*>(&k_tt_generation<8, 2>),
                         reinterpret_cast<const void*>(&k_tt_generation<8, 4>),
                         reinterpret_cast<const void*>(&k_tt_generation<16, 2>),
                         reinterpret_cast<const void*>(&k_tt_generation<16, 4>)};
    const void* ke[4] = {reinterpret_cast<const void*>(&k_tt_evaluate<8, 2>),
                         reinterpret_cast<const void*>(&k_tt_evaluate<8, 4>),
                         reinterpret_cast<const void*>(&k_tt_evaluate<16, 2>),
                         reinterpret_cast<const void*>(&k_tt_evaluate<16, 4>)};
    const int kv = (c->kmax == 8 ? 0 : 2) + (c->mmx == 2 ? 0 : 1);
    TT_HIP(c, hipFuncSetAttribute(kg[kv], hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_gen));
    TT_HIP(c, hipFuncSetAttribute(ke[kv], hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_gen));
    TT_HIP(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tt_migrate),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 2 * kMaxIslSize * 8));
    c->ws = reinterpret_cast<char*>(ptr);
    c->ws_bytes = bytes;
    TtDesc& d = c->desc;
    d = TtDesc{};
    d.J = c->J;
    d.S = c->S;
    d.MX = c->MX;
    d.L = c->L;
    d.Lp = c->Lp;
    d.Jp = c->Jp;
    d.runs = c->runs;
    d.n_isl = (int)c->isl.size();
    d.H = (c->interval > 0 || d.n_isl >= 2) ? d.n_isl / 2 : 0;
    d.WT = c->WT;
    d.E = c->E;
    d.theta_T = rate_T(c->theta);
    d.seed = c->seed;
    int off = 0;
    for (int i = 0; i < d.n_isl; ++i) {
        const auto& s = c->isl[i];
        TtIsland& I = d.isl[i];
        I.kind = s.kind;
        I.rows = s.kind == 0 ? s.rows : 0;
        I.cols = s.kind == 0 ? s.cols : 0;
        I.size = s.kind == 0 ? s.rows * s.cols : s.size;
        I.off = off;
        I.tc = rate_T(s.p_c);
        I.tm = rate_T(s.p_m);
        off += I.size;
    }
    d.N = off;
    char* w = c->ws;
    for (int p = 0; p < 2; ++p) {
        d.genes[p] = reinterpret_cast<uint8_t*>(w + l.genes[p]);
        d.obj[p] = reinterpret_cast<long long*>(w + l.obj[p]);
    }
    d.genkey = reinterpret_cast<unsigned long long*>(w + l.genkey);
    d.best = reinterpret_cast<long long*>(w + l.best);
    d.best_genes = reinterpret_cast<uint8_t*>(w + l.best_genes);
    d.counters = reinterpret_cast<long long*>(w + l.counters);
    d.err = reinterpret_cast<int*>(w + l.err);
    // the tables as the LDS image that every workgroup copies (tab_off)
    const TabOff to = tab_off(c->J, c->S, c->MX, c->Lp);
    std::vector<unsigned char> img((size_t)to.bytes, 0);
    std::memcpy(img.data() + to.P, c->P.data(), c->P.size() * 2);
    std::memcpy(img.data() + to.D, c->D.data(), c->D.size() * 4);
    std::memcpy(img.data() + to.R, c->R.data(), c->R.size() * 4);
    std::memcpy(img.data() + to.ord0, c->ord0.data(), c->ord0.size() * 2);
    std::memcpy(img.data() + to.M, c->M.data(), c->M.size() * 4);
    for (int i = 0; i < c->L; ++i) img[(size_t)to.cb + i] = (unsigned char)(c->M[i % c->S] - 1);
    d.tab = reinterpret_cast<const uint4*>(w + l.tab);
    d.tab_vec = to.bytes / 16;
    TT_HIP(c, hipMemcpyAsync(w + l.tab, img.data(), img.size(), hipMemcpyHostToDevice, c->stream));
    std::vector<unsigned long long> gk((size_t)c->runs * d.n_isl * 2, ~0ull);
    TT_HIP(c, hipMemcpyAsync(w + l.genkey, gk.data(), gk.size() * 8, hipMemcpyHostToDevice, c->stream));
    std::vector<long long> best((size_t)c->runs * 4, 0);
    for (int r = 0; r < c->runs; ++r) {
        best[r * 4 + 0] = LLONG_MAX;
        best[r * 4 + 2] = -1;
    }
    TT_HIP(c, hipMemcpyAsync(w + l.best, best.data(), best.size() * 8, hipMemcpyHostToDevice, c->stream));
    std::vector<long long> zeros((size_t)c->runs * 2, 0);
    TT_HIP(c, hipMemcpyAsync(w + l.counters, zeros.data(), zeros.size() * 8, hipMemcpyHostToDevice, c->stream));
    const int zero = 0;
    TT_HIP(c, hipMemcpyAsync(w + l.err, &zero, 4, hipMemcpyHostToDevice, c->stream));
    TT_HIP(c, hipStreamSynchronize(c->stream));   // the host vectors above go out of scope
    c->bound = true;
    c->gen = 0;
    int rc = launch_gen(c, 0, 1);
    if (rc != FFS_OK) {
        c->bound = false;
        return rc;
    }
    return FFS_OK;
}

int ffs_tt_evolve(ffs_tt_ctx* c, int32_t generations)
{
    int rc = check_ready(c);
    if (rc != FFS_OK) return rc;
    if (generations < 0) return fail(c, FFS_EINVAL, "generations < 0");
    for (int it = 0; it < generations; ++it) {
        const int g = c->gen + 1;
        if ((rc = launch_gen(c, g, 0)) != FFS_OK) return rc;
        c->gen = g;
        if (c->interval > 0 && g % c->interval == 0)
            if ((rc = launch_migrate(c, g)) != FFS_OK) return rc;
    }
    return FFS_OK;
}

int ffs_tt_migrate(ffs_tt_ctx* c)
{
    int rc = check_ready(c);
    if (rc != FFS_OK) return rc;
    if (c->isl.size() & 1) return fail(c, FFS_EINVAL, "migration needs an even island count");
    return launch_migrate(c, c->gen);
}

int ffs_tt_generation(const ffs_tt_ctx* c, int32_t* gen)
{
    if (!c || !gen) return FFS_EINVAL;
    *gen = c->gen;
    return FFS_OK;
}

static int island_args(ffs_tt_ctx* c, int run, int island, int* size, size_t* first)
{
    int rc = check_ready(c);
    if (rc != FFS_OK) return rc;
    if (run < 0 || run >= c->runs || island < 0 || island >= c->desc.n_isl)
        return fail(c, FFS_EINVAL, "run %d island %d", run, island);
    *size = c->desc.isl[island].size;
    *first = (size_t)run * c->desc.N + c->desc.isl[island].off;
    return FFS_OK;
}

int ffs_tt_get_population(ffs_tt_ctx* c, int32_t run, int32_t island, int32_t* genes, int64_t* objectives)
{
    int size = 0;
    size_t first = 0;
    int rc = island_args(c, run, island, &size, &first);
    if (rc != FFS_OK) return rc;
    const int par = c->gen & 1;
    std::vector<uint8_t> g((size_t)size * c->Lp);
    TT_HIP(c, hipMemcpyAsync(g.data(), c->desc.genes[par] + first * c->Lp, g.size(), hipMemcpyDeviceToHost, c->stream));
    std::vector<long long> o(size);
    TT_HIP(c, hipMemcpyAsync(o.data(), c->desc.obj[par] + first, (size_t)size * 8, hipMemcpyDeviceToHost, c->stream));
    TT_HIP(c, hipStreamSynchronize(c->stream));
    if (genes)
        for (int s = 0; s < size; ++s)
            for (int i = 0; i < c->L; ++i) genes[(size_t)s * c->L + i] = g[(size_t)s * c->Lp + i];
    if (objectives)
        for (int s = 0; s < size; ++s) objectives[s] = o[s];
    return FFS_OK;
}

int ffs_tt_set_population(ffs_tt_ctx* c, int32_t run, int32_t island, const int32_t* genes, const int64_t* objectives)
{
    int size = 0;
    size_t first = 0;
    int rc = island_args(c, run, island, &size, &first);
    if (rc != FFS_OK) return rc;
    if (!genes || !objectives) return fail(c, FFS_EINVAL, "null array");
    std::vector<uint8_t> g((size_t)size * c->Lp, 0);
    for (int s = 0; s < size; ++s)
        for (int i = 0; i < c->L; ++i) {
            const int v = genes[(size_t)s * c->L + i];
            if (v < 0 || v >= c->M[i % c->S]) return fail(c, FFS_EINVAL, "gene %d of slot %d out of range", i, s);
            g[(size_t)s * c->Lp + i] = (uint8_t)v;
        }
    for (int s = 0; s < size; ++s)
        if (objectives[s] < 0 || objectives[s] >= (1ll << 39)) return fail(c, FFS_EINVAL, "objective of slot %d", s);
    const int par = c->gen & 1;
    TT_HIP(c, hipMemcpyAsync(c->desc.genes[par] + first * c->Lp, g.data(), g.size(), hipMemcpyHostToDevice, c->stream));
    TT_HIP(c, hipMemcpyAsync(c->desc.obj[par] + first, objectives, (size_t)size * 8, hipMemcpyHostToDevice, c->stream));
    TT_HIP(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_tt_set_generation(ffs_tt_ctx* c, int32_t gen)
{
    int rc = check_ready(c);
    if (rc != FFS_OK) return rc;
    if (gen < 0) return fail(c, FFS_EINVAL, "generation < 0");
    if ((gen & 1) != (c->gen & 1)) {
        // keep the parity of the buffers the state lives in
        const size_t n = (size_t)c->runs * c->desc.N;
        const int from = c->gen & 1, to = gen & 1;
        TT_HIP(c, hipMemcpyAsync(c->desc.genes[to], c->desc.genes[from], n * c->Lp, hipMemcpyDeviceToDevice, c->stream));
        TT_HIP(c, hipMemcpyAsync(c->desc.obj[to], c->desc.obj[from], n * 8, hipMemcpyDeviceToDevice, c->stream));
        TT_HIP(c, hipStreamSynchronize(c->stream));
    }
    c->gen = gen;
    return FFS_OK;
}

int ffs_tt_best(ffs_tt_ctx* c, int32_t run, int64_t* objective, int32_t* gen, int32_t* island, int32_t* slot,
                int32_t* genes)
{
    int rc = check_ready(c);
    if (rc != FFS_OK) return rc;
    if (run < 0 || run >= c->runs) return fail(c, FFS_EINVAL, "run %d", run);
    long long rec[4];
    std::vector<uint8_t> g(c->Lp);
    TT_HIP(c, hipMemcpyAsync(rec, c->desc.best + (size_t)run * 4, sizeof rec, hipMemcpyDeviceToHost, c->stream));
    TT_HIP(c, hipMemcpyAsync(g.data(), c->desc.best_genes + (size_t)run * c->Lp, c->Lp, hipMemcpyDeviceToHost, c->stream));
    int err = 0;
    TT_HIP(c, hipMemcpyAsync(&err, c->desc.err, 4, hipMemcpyDeviceToHost, c->stream));
    TT_HIP(c, hipStreamSynchronize(c->stream));
    if (err) return fail(c, FFS_EDEVICE, "a kernel met an out-of-range gene");
    if (objective) *objective = rec[0];
    if (gen) *gen = (int32_t)rec[1];
    if (island) *island = (int32_t)rec[2];
    if (slot) *slot = (int32_t)rec[3];
    if (genes)
        for (int i = 0; i < c->L; ++i) genes[i] = g[i];
    return FFS_OK;
}

int ffs_tt_counters(ffs_tt_ctx* c, int32_t run, int64_t* migrations, int64_t* migrants)
{
    int rc = check_ready(c);
    if (rc != FFS_OK) return rc;
    if (run < 0 || run >= c->runs) return fail(c, FFS_EINVAL, "run %d", run);
    long long v[2];
    TT_HIP(c, hipMemcpyAsync(v, c->desc.counters + (size_t)run * 2, sizeof v, hipMemcpyDeviceToHost, c->stream));
    TT_HIP(c, hipStreamSynchronize(c->stream));
    if (migrations) *migrations = v[0];
    if (migrants) *migrants = v[1];
    return FFS_OK;
}

int ffs_tt_evaluate(ffs_tt_ctx* c, const void* genes, int32_t count, void* out)
{
    int rc = check_ready(c);
    if (rc != FFS_OK) return rc;
    if (count < 0 || (count > 0 && (!genes || !out))) return fail(c, FFS_EINVAL, "count %d", count);
    if (count == 0) return FFS_OK;
    const unsigned blocks = (unsigned)((count + c->wpb - 1) / c->wpb);
    const uint8_t* g = reinterpret_cast<const uint8_t*>(genes);
    long long* o = reinterpret_cast<long long*>(out);
    if (c->kmax == 8 && c->mmx == 2)
        hipLaunchKernelGGL((k_tt_evaluate<8, 2>), dim3(blocks), dim3(64 * c->wpb), c->lds_gen, c->stream, c->desc, g,
                           count, o);
    else if (c->kmax == 8)
        hipLaunchKernelGGL((k_tt_evaluate<8, 4>), dim3(blocks), dim3(64 * c->wpb), c->lds_gen, c->stream, c->desc, g,
                           count, o);
    else if (c->mmx == 2)
        hipLaunchKernelGGL((k_tt_evaluate<16, 2>), dim3(blocks), dim3(64 * c->wpb), c->lds_gen, c->stream, c->desc, g,
                           count, o);
    else
        hipLaunchKernelGGL((k_tt_evaluate<16, 4>), dim3(blocks), dim3(64 * c->wpb), c->lds_gen, c->stream, c->desc, g,
                           count, o);
    TT_HIP(c, hipGetLastError());
    return FFS_OK;
}

int ffs_tt_set_update(ffs_tt_ctx* c, int32_t mode)
{
    if (!c) return FFS_EINVAL;
    if (mode != 0 && mode != 1) return fail(c, FFS_EINVAL, "update mode %d", mode);
    c->sweep = mode;
    return FFS_OK;
}

int ffs_tt_set_timing(ffs_tt_ctx* c, int32_t on)
{
    if (!c) return FFS_EINVAL;
    c->timing = on != 0;
    c->t_ms = 0;
    c->t_n = 0;
    c->ev_used = 0;
    return FFS_OK;
}

int ffs_tt_kernel_time(ffs_tt_ctx* c, double* ms, int64_t* launches)
{
    if (!c || !ms || !launches) return FFS_EINVAL;
    int rc = collect_timing(c);
    if (rc != FFS_OK) return rc;
    *ms = c->t_ms;
    *launches = c->t_n;
    return FFS_OK;
}

}  // extern "C"
