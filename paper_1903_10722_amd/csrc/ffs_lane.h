// ffs_lane.h -- lane-per-chromosome mapping of the decode and of the
// generation step, for populations large enough to fill the chip with it.
//
// The decode (the list-scheduling rule of include/ffs.h over the Section 3
// problem) runs one chromosome per lane.  A lane walks every stage itself,
// so the stage that runs is the same on all 64 lanes of a wave: the
// insertion network of a stage has exactly m_k entries (a branch on the
// wave-uniform m_k), and nothing moves between lanes.
//
// Slots.  Stage k dispatches its n jobs at slots off_k .. off_k + n - 1
// (off_k = m_0 + ... + m_{k-1}); the key it removes at a dispatch (the
// machine's previous job, completion << jb | job) is written back to the
// slot it read, so the slot sequence of stage k's writes is its release
// order.  The first m_k of them are the machines' initial empty entries;
// after its last dispatch the stage writes its remaining entries, in order,
// to slots off_k + n .. off_k + n + m_k - 1.  Stage k + 1 therefore reads
// exactly its input order at slots off_{k+1} .. off_{k+1} + n - 1.
// Entries of one stage leave in (completion, dispatch order) order -- the
// first-in-first-out rule at the next stage -- because a newly dispatched
// job is inserted after every entry whose completion is not later than its
// own.
//
// Windows.  The slots are processed in windows of kLaneD held in registers:
// for each window, stage 0, 1, ..., S-1 in turn transform the window in
// place.  A stage's m_k sorted keys stay in LDS between windows.  Windows
// that lie inside a stage's dispatch range run unguarded; the first and
// last windows of a stage run with per-slot (wave-uniform) guards.
//
// The generation kernel of this mapping builds each wave's 64 children one
// after the other with the operators of ffs_kernels.h on all 64 lanes,
// writes them to the next generation's rows, decodes them one per lane from
// there, then writes back the parent's row of every cellular cell whose
// child is not strictly better.
#pragma once
#include "ffs_kernels.h"

namespace flowshop {

constexpr int kLaneD = 16;           // slots per window
constexpr int kLaneMaxMsum = 160;    // machine entries per lane (sum over stages) kept in LDS

// LDS of one wave of the lane generation kernel: the operators' three rows,
// later reused for the decode state (64 lanes x msum keys).
__host__ __device__ inline size_t lane_gen_wave_lds(int n_pad, int msum)
{
    const size_t ops = (size_t)group_stride(n_pad) * 2;
    const size_t st = (size_t)64 * msum * 4;
    return align16(ops > st ? ops : st);
}

// LDS of one wave of the lane decode of caller-supplied rows: the per-lane
// bit sets of the validity check, later reused for the decode state.
__host__ __device__ inline size_t lane_eval_wave_lds(int n, int msum)
{
    const size_t st = (size_t)64 * msum * 4;
    const size_t seen = (size_t)64 * ((n + 31) / 32) * 4;
    return align16(st > seen ? st : seen);
}

// One stage over one window.  r[i] holds slot lo + i: a key from the
// previous stage, or a gene at stage 0 (completion 0).  Key formats:
//   F = false: completion << jb | job.  A new key goes after every entry
//     with the same completion (those were dispatched earlier), by a
//     threshold compare per entry.
//   F = true:  completion << sh | dispatch index << jb | job (sh = 2 jb),
//     the dispatch index counting this stage's dispatches.  Keys of one
//     list are then distinct and their numeric order is (completion,
//     dispatch order), so the new key goes in by one min, max or median
//     per entry.  The completions must stay below 2^(32 - sh): cor
//     collects the bits of every completion for the caller's check.
// With GUARD, slot i dispatches only if bit i of `act` is set, and if bit i
// of `fl` is set it receives the list's first entry, which leaves the list
// (the flush after the last dispatch); job indices are clamped to n - 1 for
// the table read.
template <int M, bool GUARD, bool F, typename PT>
__device__ __forceinline__ void lane_stage(uint32_t (&r)[kLaneD], uint32_t (&key)[M], const PT* prow,
                                           uint32_t jb, uint32_t jmask, uint32_t act, uint32_t fl, uint32_t nmax,
                                           uint32_t sh, int dbase, uint32_t& cor)
{
    uint32_t jj[kLaneD], pj[kLaneD];
#pragma unroll
    for (int i = 0; i < kLaneD; ++i) {
        const uint32_t j = r[i] & jmask;
        jj[i] = GUARD ? (j < nmax ? j : nmax) : j;
    }
#pragma unroll
    for (int i = 0; i < kLaneD; ++i) pj[i] = (uint32_t)prow[jj[i]];
#pragma unroll
    for (int i = 0; i < kLaneD; ++i) {
        if (!GUARD || ((act >> i) & 1u)) {
            // start = max(machine free, job ready): the larger key has the
            // larger (or equal) time in its high bits
            const uint32_t o = key[0];
            const uint32_t mx = o > r[i] ? o : r[i];
            if (F) {
                const uint32_t c = (mx >> sh) + pj[i];
                cor |= c;
                if (M == 1) {
                    key[0] = (c << sh) | jj[i];
                } else {
                    const uint32_t nk = (c << sh) | ((uint32_t)(dbase + i) << jb) | jj[i];
                    // sorted list key[1 .. M-1] with nk added
                    uint32_t nkey[M];
                    nkey[0] = key[1] < nk ? key[1] : nk;
#pragma unroll
                    for (int q = 1; q + 1 < M; ++q) nkey[q] = umed3(key[q], nk, key[q + 1]);
                    nkey[M - 1] = key[M - 1] > nk ? key[M - 1] : nk;
#pragma unroll
                    for (int q = 0; q < M; ++q) key[q] = nkey[q];
                }
            } else {
                const uint32_t c = (mx >> jb) + pj[i];
                const uint32_t nk = (c << jb) | jj[i];
                if (M == 1) {
                    key[0] = nk;
                } else {
                    // drop entry 0, insert nk after every entry with completion <= c
                    const uint32_t thr = (c + 1u) << jb;
                    uint32_t nkey[M];
                    bool prev = true;
#pragma unroll
                    for (int q = 0; q + 1 < M; ++q) {
                        const bool lt = key[q + 1] < thr;
                        nkey[q] = lt ? key[q + 1] : (prev ? nk : key[q]);
                        prev = lt;
                    }
                    nkey[M - 1] = prev ? nk : key[M - 1];
#pragma unroll
                    for (int q = 0; q < M; ++q) key[q] = nkey[q];
                }
            }
            r[i] = o;
        } else if (GUARD && ((fl >> i) & 1u)) {
            r[i] = key[0];
#pragma unroll
            for (int q = 0; q + 1 < M; ++q) key[q] = key[q + 1];
        }
    }
}

// Stage k (m_k = M) over window [lo, lo + kLaneD): its dispatch slots are
// [d0, d0 + n), its flush slots [d0 + n, d0 + n + M) unless it is the last
// stage.  Keys live at st[q * 64] (q < M) between windows (during a flush
// that spans two windows, the entries not yet written, first at q = 0).  Returns the
// makespan on the last window of the last stage, else 0.
template <int M, bool F, typename PT>
__device__ __forceinline__ uint32_t lane_stage_window(uint32_t (&r)[kLaneD], uint32_t* st, const PT* prow, int lo,
                                                      int d0, int n, bool last, uint32_t jb, uint32_t jmask,
                                                      uint32_t sh, uint32_t& cor)
{
    const int d1 = d0 + n, end = last ? d1 : d1 + M;
    uint32_t key[M];
    if (d0 >= lo) {
#pragma unroll
        for (int q = 0; q < M; ++q) key[q] = 0u;
    } else {
#pragma unroll
        for (int q = 0; q < M; ++q) key[q] = st[q * 64];
    }
    if (d0 <= lo && lo + kLaneD <= d1) {
        lane_stage<M, false, F, PT>(r, key, prow, jb, jmask, 0u, 0u, 0u, sh, lo - d0, cor);
    } else {
        const int a0 = d0 > lo ? d0 - lo : 0, a1 = (d1 < lo + kLaneD ? d1 : lo + kLaneD) - lo;
        const uint32_t act = (a1 > a0) ? ((0xFFFFFFFFu >> (32 - (a1 - a0))) << a0) : 0u;
        uint32_t fl = 0u;
        if (!last) {
            const int f0 = (d1 > lo ? d1 : lo) - lo, f1 = (end < lo + kLaneD ? end : lo + kLaneD) - lo;
            fl = (f1 > f0) ? ((0xFFFFFFFFu >> (32 - (f1 - f0))) << f0) : 0u;
        }
        lane_stage<M, true, F, PT>(r, key, prow, jb, jmask, act, fl, (uint32_t)(n - 1), sh, lo - d0, cor);
    }
    if (end <= lo + kLaneD) return last ? (key[M - 1] >> (F ? sh : jb)) : 0u;
#pragma unroll
    for (int q = 0; q < M; ++q) st[q * 64] = key[q];
    return 0u;
}

// Genes of slots [lo, lo + kLaneD) of a row (positions past the row's end
// read the row's padding; the guards never dispatch them).
struct GenesU16 {
    const uint16_t* row;   // n_pad entries, 64-byte aligned
    __device__ __forceinline__ void load(int lo, uint32_t (&g)[kLaneD]) const
    {
        const auto* v = as_global(reinterpret_cast<const u32x4*>(row + lo));
        const u32x4 a = v[0], b = v[1];
        const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            g[2 * i] = w[i] & 0xFFFFu;
            g[2 * i + 1] = w[i] >> 16;
        }
    }
};

// Caller-supplied int32 rows of exactly n entries: values outside [0, n)
// become 0 (the row is reported invalid separately).
struct GenesI32 {
    const int* row;
    int n;
    __device__ __forceinline__ void load(int lo, uint32_t (&g)[kLaneD]) const
    {
        const auto* p = as_global(row);
#pragma unroll
        for (int i = 0; i < kLaneD; ++i) {
            const int t = lo + i;
            const int x = p[t < n ? t : n - 1];
            g[i] = ((unsigned)x < (unsigned)n) ? (uint32_t)x : 0u;
        }
    }
};

// Makespan of one chromosome per lane with the key format F (see
// lane_stage).  pT is the LDS table (row stride pts), mach the stage machine
// counts, st this wave's LDS state (msum keys per lane, lane-interleaved).
template <int MMAX, bool F, typename PT, typename Src>
__device__ __forceinline__ uint32_t lane_decode_keys(const Src& src, const PT* pT, int pts, const int* mach, int S, int n, int jb,
                                     uint32_t sh, uint32_t* st, int lane, uint32_t& cor)
{
    const uint32_t ujb = (uint32_t)jb, jmask = (1u << jb) - 1u;
    int off_last = 0;
    for (int k = 0; k + 1 < S; ++k) off_last += mach[k];
    const int nwin = (off_last + n + kLaneD - 1) / kLaneD;
    uint32_t cmax = 0u;
    uint32_t gnext[kLaneD];
    src.load(0, gnext);
    for (int w = 0; w < nwin; ++w) {
        const int lo = w * kLaneD;
        uint32_t r[kLaneD];
#pragma unroll
        for (int i = 0; i < kLaneD; ++i) r[i] = gnext[i];
        if (lo + kLaneD < n) src.load(lo + kLaneD, gnext);
        int off = 0;
        for (int k = 0; k < S; ++k) {
            const int M = mach[k];
            const bool last = (k == S - 1);
            const int end = off + n + (last ? 0 : M);
            if (off >= lo + kLaneD) break;   // this and later stages start after the window
            if (end > lo) {
                const PT* prow = pT + (size_t)k * pts;
                uint32_t* sk = st + (size_t)off * 64 + lane;
                uint32_t cm = 0u;
                switch (M) {
#define FFS_LANE_CASE(MM)                                                                       \
    case MM:                                                                                    \
        if (MM <= MMAX)                                                                         \
            cm = lane_stage_window<(MM <= MMAX ? MM : 1), F, PT>(r, sk, prow, lo, off, n, last, ujb, jmask, sh, cor); \
        break;
                    FFS_LANE_CASE(1) FFS_LANE_CASE(2) FFS_LANE_CASE(3) FFS_LANE_CASE(4)
                    FFS_LANE_CASE(5) FFS_LANE_CASE(6) FFS_LANE_CASE(7) FFS_LANE_CASE(8)
#undef FFS_LANE_CASE
                    default: break;
                }
                cmax = last ? (cm > cmax ? cm : cmax) : cmax;
            }
            off += M;
        }
    }
    return cmax;
}

// The two-field decode as a function of its own (the fallback of the
// three-field one, whose code stays out of the kernel's main path).
template <int MMAX, typename PT, typename Src>
__device__ __attribute__((noinline)) uint32_t lane_decode_twofield(const Src& src, const PT* pT, int pts,
                                                                   const int* mach, int S, int n, int jb,
                                                                   uint32_t* st, int lane)
{
    uint32_t cor = 0u;
    return lane_decode_keys<MMAX, false, PT>(src, pT, pts, mach, S, n, jb, 0u, st, lane, cor);
}

// Makespan of one chromosome per lane.  With fsh > 0 (the instance's
// completions can fit below 2^(32 - fsh), fsh = 2 jb) the three-field key
// goes first; if any lane's completions outgrow it, the wave decodes again
// with the two-field key and those lanes take that result.
template <int MMAX, typename PT, typename Src>
__device__ __forceinline__ uint32_t lane_decode(const Src& src, const PT* pT, int pts, const int* mach, int S, int n, int jb,
                                int fsh, uint32_t* st, int lane)
{
    uint32_t cor = 0u;
    if (fsh > 0) {
        const uint32_t cm = lane_decode_keys<MMAX, true, PT>(src, pT, pts, mach, S, n, jb, (uint32_t)fsh, st, lane, cor);
        const bool redo = (cor >> (32 - fsh)) != 0u;
        if (__ballot(redo) == 0ull) return cm;
        // rare: out of line
        const uint32_t cm2 = lane_decode_twofield<MMAX, PT>(src, pT, pts, mach, S, n, jb, st, lane);
        return redo ? cm2 : cm;
    }
    return lane_decode_keys<MMAX, false, PT>(src, pT, pts, mach, S, n, jb, 0u, st, lane, cor);
}

// ---- one generation (mode 0) or generation 0 (mode 1), lane mapping --------
// Work item = up to 64 * waves chromosomes of one island; wave w takes 64 of
// them.  Same generation bookkeeping, best-ever workgroup and XCD placement
// as k_generation.  Mode 0 leaves line-sweep islands alone; mode 2 runs the
// cells of anti-diagonal `cnt_off` of line-sweep island work[blockIdx.y]
// for the generation the last mode-0 launch counted (one launch per
// anti-diagonal, in order, after that launch).
template <int MMAX, typename PT>
__global__ void __launch_bounds__(512) k_generation_lane(const InstDesc* __restrict__ insts,
                                                         const IslandDesc* __restrict__ isls,
                                                         const WorkItem* __restrict__ work, Control* ctl, int n_inst,
                                                         int mode, int cnt_off, int has_extra)
{
    __shared__ int s_gen;
    const bool sweep = mode == 2;
    if (threadIdx.x == 0) {
        int gg = 0;
        if (mode == 0) {
            int* cnt = ctl->counts + cnt_off + blockIdx.x;
            const int t = *cnt;
            *cnt = t + 1;
            gg = ctl->base + 1 + t;
        } else if (sweep) {
            gg = completed_gen(ctl);
        }
        s_gen = gg;
    }
    // has_extra = 1 + group: the last workgroup folds that fold group's
    // previous generation
    if (has_extra && blockIdx.x == gridDim.x - 1) {
        __syncthreads();
        const int prev = s_gen - 1, group = has_extra - 1;
        if (ctl->best_gen[group] < prev)
            fold_best(insts, isls, n_inst, prev, ctl, reinterpret_cast<int*>(ffs_smem), group);
        return;
    }
    const int nw = (int)gridDim.x - (has_extra ? 1 : 0);
    int widx = sweep ? (int)blockIdx.y : (int)blockIdx.x;
    if (!sweep && nw <= 256) {
        const int per = (nw + 7) / 8, full = nw - 8 * (per - 1);
        const int xcd = widx & 7, rnk = widx >> 3;
        widx = (xcd < full) ? xcd * per + rnk : full * per + (xcd - full) * (per - 1) + rnk;
    }
    const WorkItem wi = work[widx];
    const InstDesc* I = insts + wi.inst;
    const IslandDesc* L = isls + wi.island;
    if (mode == 0 && L->sweep) return;   // line-sweep islands have launches of their own
    // line sweep: the cells of anti-diagonal diag, rows rlo .. rlo + dcount - 1
    const int diag = sweep ? cnt_off : -1;
    int rlo = 0, dcount = 0;
    if (sweep) {
        rlo = diag - (L->cols - 1) > 0 ? diag - (L->cols - 1) : 0;
        const int rhi = diag < L->rows - 1 ? diag : L->rows - 1;
        dcount = rhi - rlo + 1;
        if (dcount <= 0) return;
    }
    const int n = I->n, S = I->S, n_pad = I->n_pad, jb = I->jb;

    PT* pT = reinterpret_cast<PT*>(ffs_smem);
    stage_pt<PT>(pT, I->pT, S, n_pad);
    __syncthreads();
    const int gen = s_gen;
    const int cur = (gen + 1) & 1, nxt = gen & 1;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    unsigned char* wbase = ffs_smem + pt_lds_bytes<PT>(S, n_pad) + (size_t)wave * I->lane_wlds;
    // chromosome i of this wave sits in slot slot_of(sbase + i)
    const int w0 = wave * kWave + (sweep ? (int)blockIdx.x * (int)blockDim.x : 0);
    const int total = sweep ? dcount : wi.count;
    const int wcount = total - w0 < 0 ? 0 : (total - w0 > kWave ? kWave : total - w0);
    const int sbase = sweep ? w0 : wi.slot0 + w0;
    const int lcols = L->cols;
    auto slot_of = [&](int i) { return sweep ? (rlo + i) * lcols + (diag - rlo - i) : i; };

    // children, one at a time on all 64 lanes, into the next generation's
    // rows.  Lane c first takes the parents and draws of child c (one Philox
    // block per cell, two per pair); while a child is built, the parents'
    // rows of the next one are already on their way into registers.
    {
        uint16_t* A = reinterpret_cast<uint16_t*>(wbase);
        uint16_t* B = A + n_pad;
        uint16_t* V = B + n_pad;
        if (mode == 1) {
            for (int c = 0; c < wcount; ++c) {
                make_child<true>(I, L, slot_of(sbase + c), 0u, gen, cur, 1, A, B, V, lane, kWave, 0, true);
                row_l2g(L->genes[nxt] + (size_t)slot_of(sbase + c) * n_pad, A, n_pad, lane, kWave);
                wave_sync();
            }
        } else if (wcount > 0) {
            const bool cell = L->kind == 0;
            const int pslot = slot_of(sbase + (lane < wcount ? lane : 0));
            uint32_t w_src, w_cut, w_mut;
            if (cell) {
                // slots < 2^14; bits 15 and 31: that parent's row is the new generation's
                const CellPlan pl = cell_plan(I, L, pslot, 0u, gen, cur, diag);
                w_src = (uint32_t)pl.p1 | ((uint32_t)pl.p2 << 16) | (pl.n1 ? 1u << 15 : 0u) | (pl.n2 ? 1u << 31 : 0u);
                w_cut = (uint32_t)pl.meta.a | ((uint32_t)pl.meta.b << 12) | (pl.meta.cx ? 1u << 24 : 0u) |
                        (pl.meta.mx ? 1u << 25 : 0u);
                w_mut = (uint32_t)pl.meta.mi | ((uint32_t)pl.meta.mj << 12);
            } else {
                const PairPlan pl = pair_plan(I, L, pslot, gen, cur);
                w_src = (uint32_t)pl.xs | (pl.odd ? 1u << 31 : 0u);
                w_cut = (uint32_t)pl.a | ((uint32_t)pl.b << 12) | (pl.cx ? 1u << 24 : 0u) | (pl.mx ? 1u << 25 : 0u);
                w_mut = (uint32_t)pl.mi | ((uint32_t)pl.mj << 12);
            }
            const int nv = n_pad >> 3;                   // 16-byte vectors per row
            constexpr int PV = 2;                         // vectors per lane per row held in registers
            const bool pre = nv <= PV * kWave;            // rows of up to 1024 genes
            const auto* g4 = as_global(reinterpret_cast<const u32x4*>(L->genes[cur]));
            const auto* g4n = as_global(reinterpret_cast<const u32x4*>(L->genes[nxt]));
            u32x4 ra[PV], rb[PV];
            auto fetch = [&](int c) {
                const uint32_t src = (uint32_t)__builtin_amdgcn_readlane((int)w_src, c);
                const size_t r1 = (size_t)(cell ? (src & 0x7FFFu) : (src & 0x7FFFFFFFu)) * nv;
                const size_t r2 = (size_t)((src >> 16) & 0x7FFFu) * nv;
                const auto* s1 = (cell && (src & 0x8000u)) ? g4n : g4;
                const auto* s2 = (cell && (src >> 31)) ? g4n : g4;
#pragma unroll
                for (int v = 0; v < PV; ++v) {
                    const int x = lane + v * kWave;
                    if (x < nv) {
                        ra[v] = s1[r1 + x];
                        if (cell) rb[v] = s2[r2 + x];
                    }
                }
            };
            if (pre) fetch(0);
            for (int c = 0; c < wcount; ++c) {
                const uint32_t src = (uint32_t)__builtin_amdgcn_readlane((int)w_src, c);
                const uint32_t cut = (uint32_t)__builtin_amdgcn_readlane((int)w_cut, c);
                const uint32_t mut = (uint32_t)__builtin_amdgcn_readlane((int)w_mut, c);
                const int slot = slot_of(sbase + c);
                if (pre) {
                    u32x4* da = reinterpret_cast<u32x4*>(cell ? A : V);
                    u32x4* db = reinterpret_cast<u32x4*>(B);
#pragma unroll
                    for (int v = 0; v < PV; ++v) {
                        const int x = lane + v * kWave;
                        if (x < nv) {
                            da[x] = ra[v];
                            if (cell) db[x] = rb[v];
                        }
                    }
                } else if (cell) {
                    rows_g2l(A, L->genes[(src & 0x8000u) ? nxt : cur] + (size_t)(src & 0x7FFFu) * n_pad, B,
                             L->genes[(src >> 31) ? nxt : cur] + (size_t)((src >> 16) & 0x7FFFu) * n_pad, n_pad,
                             lane, kWave);
                } else {
                    row_g2l(V, L->genes[cur] + (size_t)(src & 0x7FFFFFFFu) * n_pad, n_pad, lane, kWave);
                }
                wave_sync();
                if (pre && c + 1 < wcount) fetch(c + 1);
                if (!cell) pair_parents(A, B, V, n, (src >> 31) != 0u, lane, kWave, true);
                ox_group<true, false>(A, B, V, n, (int)(cut & 0xFFFu), (int)((cut >> 12) & 0xFFFu),
                                      ((cut >> 24) & 1u) != 0u, lane, kWave, 0);
                swap_genes(A, ((cut >> 25) & 1u) != 0u && lane == 0, (int)(mut & 0xFFFu), (int)(mut >> 12));
                row_l2g(L->genes[nxt] + (size_t)slot * n_pad, A, n_pad, lane, kWave);
                wave_sync();
            }
        }
    }
    // the rows just written are read back by other lanes of this wave
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

    const bool active = lane < wcount;
    const int slot = slot_of(sbase + (active ? lane : 0));
    unsigned long long wkey = ~0ull;
    if (wcount > 0) {
        const GenesU16 src{L->genes[nxt] + (size_t)slot * n_pad};
        const uint32_t cm = lane_decode<MMAX, PT>(src, pT, pt_stride<PT>(n_pad), I->mach, S, n, jb, I->fsh,
                                                  reinterpret_cast<uint32_t*>(wbase), lane);
        bool keep_old = false;
        if (active) {
            int mk_new = (int)cm;
            if (mode != 1 && L->kind == 0) {
                const int mk_old = as_global(L->mk[cur])[slot];
                keep_old = !((int)cm < mk_old);
                mk_new = keep_old ? mk_old : (int)cm;
            }
            L->mk[nxt][slot] = mk_new;
            wkey = ((unsigned long long)(unsigned)mk_new << 32) | (unsigned)slot;
        }
        // cells that keep their individual get the parent's row back, four
        // rows at a time by the whole wave
        unsigned long long km = __ballot(keep_old);
        const int nv = n_pad >> 3;
        const u32x4* s4 = reinterpret_cast<const u32x4*>(L->genes[cur]);
        u32x4* d4 = reinterpret_cast<u32x4*>(L->genes[nxt]);
        while (km) {
            int rows[4];
            int cnt = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                rows[t] = -1;
                if (km) {
                    rows[t] = slot_of(sbase + (int)__builtin_ctzll(km));
                    km &= km - 1ull;
                    ++cnt;
                }
            }
            for (int v0 = lane; v0 < nv; v0 += kWave) {
                u32x4 x[4];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (rows[t] >= 0) x[t] = as_global(s4)[(size_t)rows[t] * nv + v0];
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (rows[t] >= 0) as_global(d4)[(size_t)rows[t] * nv + v0] = x[t];
            }
            (void)cnt;
        }
    }
#pragma unroll
    for (int offx = 32; offx > 0; offx >>= 1) {
        const unsigned long long o = __shfl_xor(wkey, offx, 64);
        wkey = o < wkey ? o : wkey;
    }
    __shared__ unsigned long long s_wmin[8];
    if (lane == 0) s_wmin[wave] = wkey;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long mn = ~0ull;
        for (int x = 0; x < (int)(blockDim.x >> 6); ++x) mn = s_wmin[x] < mn ? s_wmin[x] : mn;
        if (mn != ~0ull) atomicMin(L->genkey + (gen & 1), mn);
    }
}

// ---- decode of caller-supplied permutations, lane mapping ------------------
// One row per lane.  A row is invalid if a value lies outside [0, n) or
// repeats (per-lane bit set in LDS); its makespan is then -1 and bit 0 of
// the control block's error word is set.
template <int MMAX, typename PT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_evaluate_lane(const InstDesc* __restrict__ I, const int* __restrict__ perms,
                                                       int count, int* __restrict__ out, Control* ctl)
{
    const int n = I->n, S = I->S, n_pad = I->n_pad, jb = I->jb;
    PT* pT = reinterpret_cast<PT*>(ffs_smem);
    stage_pt<PT>(pT, I->pT, S, n_pad);
    __syncthreads();
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t* wbase = reinterpret_cast<uint32_t*>(ffs_smem + pt_lds_bytes<PT>(S, n_pad) +
                                                  (size_t)wave * I->lane_wlds_eval);
    const long long base = ((long long)blockIdx.x * wpb + wave) * kWave;
    if (base >= count) return;
    const long long idx = base + lane;
    const bool active = idx < count;
    const int* row = perms + (active ? idx : base) * (long long)n;
    // validity: each value in range and seen once
    const int nwords = (n + 31) >> 5;
    for (int q = 0; q < nwords; ++q) wbase[q * 64 + lane] = 0u;
    bool bad = false;
    {
        const auto* p = as_global(row);
        for (int t = 0; t < n; ++t) {
            const int x = p[t];
            if ((unsigned)x >= (unsigned)n) {
                bad = true;
            } else {
                const uint32_t bit = 1u << (x & 31);
                const uint32_t old = atomicOr(&wbase[(x >> 5) * 64 + lane], bit);
                bad |= (old & bit) != 0u;
            }
        }
    }
    wave_sync();
    const GenesI32 src{row, n};
    const uint32_t cm = lane_decode<MMAX, PT>(src, pT, pt_stride<PT>(n_pad), I->mach, S, n, jb, I->fsh, wbase, lane);
    if (active) out[idx] = bad ? -1 : (int)cm;
    if (active && bad) atomicOr(&ctl->err, 1);
}

}  // namespace flowshop

namespace flowshop {

// ---- candidates of the learned pre-screen, one wave per cell ----------------
// Features of the chromosome in A (n genes) as features_group computes them,
// from the job-major table pJ (row of job j at pJ + j * rsb bytes, the
// stages' processing times, zero past S): lane l sums the positions
// [l C, l C + C) (C = ceil(n / 64)) stage by stage in registers and adds each
// bucket's partial sums into acc[b * S + k] in LDS (integer sums: the order
// does not matter), then the 256 entries are written to out.
template <int SM, typename PT>
__device__ __forceinline__ void cand_features(const uint16_t* A, const unsigned char* pJ, int rsb, const InstDesc* I,
                                              const CellMeta& cm, uint32_t* acc, int lane, uint16_t* out)
{
    const int n = I->n, S = I->S, B = 240 / S;
    for (int e = lane; e < B * S; e += kWave) acc[e] = 0u;
    wave_sync();
    const int C = (n + kWave - 1) / kWave;
    const int t0 = lane * C < n ? lane * C : n, t1 = t0 + C < n ? t0 + C : n;
    // per-lane sums over at most 64 positions; with one-byte processing
    // times (<= 255) they fit in 16 bits, so stages 4d + {0, 2} and
    // 4d + {1, 3} share a register and are added pairwise (integer packed adds)
    constexpr bool PK = sizeof(PT) == 1;
    constexpr int NR = PK ? (SM + 1) / 2 : SM;   // accumulator registers
    uint32_t s[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) s[k] = 0u;
    int cb = (int)(((long long)t0 * B) / n);
    int next = (int)(((long long)(cb + 1) * n + B - 1) / B);   // first position of bucket cb + 1
    auto add_row = [&](uint32_t* x, int t) {
        const PT* row = reinterpret_cast<const PT*>(pJ + (size_t)A[t] * rsb);
        constexpr int PV = 16 / (int)sizeof(PT);   // processing times per 16-byte read
        constexpr int NB = (SM + PV - 1) / PV;     // 16-byte reads per row
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            const uint4 w = reinterpret_cast<const uint4*>(row)[v];
            const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
            if (PK) {
                typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
#pragma unroll
                for (int d = 0; d < 4; ++d) {
                    const int r = 2 * (v * 4 + d);   // registers of stages 4 (4v + d) + {0, 2} and + {1, 3}
                    if (r < NR) {
                        const u16x2 lo = __builtin_bit_cast(u16x2, ww[d] & 0x00FF00FFu);
                        const u16x2 hi = __builtin_bit_cast(u16x2, (ww[d] >> 8) & 0x00FF00FFu);
                        x[r] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, x[r]) + lo);
                        x[r + 1] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, x[r + 1]) + hi);
                    }
                }
            } else {
#pragma unroll
                for (int q = 0; q < PV; ++q)
                    if (v * PV + q < SM) x[v * PV + q] += (ww[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
            }
        }
    };
    auto flush = [&]() {
#pragma unroll
        for (int k = 0; k < SM; ++k)
            if (k < S) {
                // stage k sits in register 2 (k / 4) + (k & 1), half (k >> 1) & 1
                const uint32_t v = PK ? (s[2 * (k >> 2) + (k & 1)] >> (16 * ((k >> 1) & 1))) & 0xFFFFu : s[k];
                if (v) atomicAdd(&acc[cb * S + k], v);
            }
#pragma unroll
        for (int k = 0; k < NR; ++k) s[k] = 0u;
    };
    if (n / B >= C) {
        // every bucket holds at least C positions, so [t0, t1) meets at most
        // one boundary, tb: the sums are snapshotted there (a select per
        // register, no divergent flush inside the loop) and split after it
        const int tb = next < t1 ? next : t1;
        uint32_t snap[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) snap[k] = 0u;
#pragma unroll 2
        for (int t = t0; t < t1; ++t) {
            const bool at = t == tb;
#pragma unroll
            for (int k = 0; k < NR; ++k) snap[k] = at ? s[k] : snap[k];
            add_row(s, t);
        }
        if (tb >= t1) {
#pragma unroll
            for (int k = 0; k < NR; ++k) snap[k] = s[k];
        }
        // s - snap per 16-bit half (each half only grows, so no borrow crosses)
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            if (PK) {
                typedef uint16_t u16x2 __attribute__((ext_vector_type(2)));
                s[k] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, s[k]) - __builtin_bit_cast(u16x2, snap[k]));
            } else {
                s[k] -= snap[k];
            }
        }
#pragma unroll
        for (int k = 0; k < SM; ++k)
            if (k < S && t0 < t1) {
                const uint32_t v0 = PK ? (snap[2 * (k >> 2) + (k & 1)] >> (16 * ((k >> 1) & 1))) & 0xFFFFu : snap[k];
                const uint32_t v1 = PK ? (s[2 * (k >> 2) + (k & 1)] >> (16 * ((k >> 1) & 1))) & 0xFFFFu : s[k];
                if (v0) atomicAdd(&acc[cb * S + k], v0);
                if (v1) atomicAdd(&acc[(cb + 1) * S + k], v1);
            }
    } else {
        for (int t = t0; t < t1; ++t) {
            if (t >= next) {
                flush();
                cb += 1;
                next = (int)(((long long)(cb + 1) * n + B - 1) / B);
            }
            add_row(s, t);
        }
        if (t0 < t1) flush();
    }
    wave_sync();
    const float fn = (float)n, fLB = (float)I->LB;
    for (int e = lane; e < kFeat; e += kWave) {
        float v = 0.f;
        if (e < B * S) {
            const int k = e - (e / S) * S;
            v = __fdiv_rn((float)((uint64_t)acc[e] * (uint64_t)B), (float)I->Pk[k]);
        } else {
            switch (e - 240) {
                case 0: v = __fdiv_rn((float)cm.mk1, fLB); break;
                case 1: v = __fdiv_rn((float)cm.mk2, fLB); break;
                case 2: v = __fdiv_rn((float)cm.a, fn); break;
                case 3: v = __fdiv_rn((float)cm.b, fn); break;
                case 4: v = cm.cx ? 1.f : 0.f; break;
                case 5: v = cm.mx ? 1.f : 0.f; break;
                case 6: v = __fdiv_rn((float)cm.mi, fn); break;
                case 7: v = __fdiv_rn((float)cm.mj, fn); break;
                case 8: v = __fdiv_rn(fLB, (float)I->E); break;
                case 9: v = __fdiv_rn(fn, 1000.f); break;
                case 10: v = __fdiv_rn((float)S, 20.f); break;
                case 11: v = __fdiv_rn((float)I->msum, (float)(6 * S)); break;
                default: break;
            }
        }
        out[e] = f32_to_bf16(v);
    }
}

// One wave per cell of the pre-screened instance's cellular islands: lane c
// (< K) takes the parents and draws of candidate c (candidate stream c of
// the CELL purpose, generation completed + 1); the wave then builds each
// candidate on all 64 lanes (order crossover, swap mutation) and writes its
// features to Xout[(cell * K + c) * 256].  LDS: the job-major table (rows of
// rsb bytes), then per wave three rows and B * S bucket sums.
template <int SM, typename PT>
__global__ void __launch_bounds__(1024) k_cand_features(const InstDesc* __restrict__ insts,
                                                       const IslandDesc* __restrict__ isls, int inst,
                                                       const Control* ctl, int cells, uint16_t* __restrict__ Xout)
{
    const InstDesc* I = insts + inst;
    const int n = I->n, S = I->S, n_pad = I->n_pad, K = I->surr_k;
    const int rsb = I->pj_row_bytes;
    const int done = completed_gen(ctl);
    const int gen = done + 1, cur = done & 1;
    unsigned char* pJ = ffs_smem;
    {
        const size_t words = (size_t)n * rsb / 16;
        const auto* s4 = as_global(reinterpret_cast<const u32x4*>(I->pJ));
        u32x4* d4 = reinterpret_cast<u32x4*>(pJ);
        for (size_t v = threadIdx.x; v < words; v += blockDim.x) d4[v] = s4[v];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cell = blockIdx.x * (blockDim.x >> 6) + wave;
    if (cell >= cells) return;
    uint16_t* A = reinterpret_cast<uint16_t*>(pJ + align16((size_t)n * rsb) +
                                              (size_t)wave * (group_stride(n_pad) * 2 + 240 * 4));
    uint16_t* B = A + n_pad;
    uint16_t* V = B + n_pad;
    uint32_t* acc = reinterpret_cast<uint32_t*>(A + group_stride(n_pad));
    // the cellular island holding this cell
    const IslandDesc* L = isls + I->island0;
    int slot = 0;
    for (int x = 0; x < I->n_islands; ++x) {
        const IslandDesc* X = isls + I->island0 + x;
        if (X->kind == 0 && cell >= X->cell_base && cell < X->cell_base + X->size) {
            L = X;
            slot = cell - X->cell_base;
        }
    }
    const CellPlan pl = cell_plan(I, L, slot, (uint32_t)(lane < K ? lane : 0), gen, cur);
    const uint32_t w_src = (uint32_t)pl.p1 | ((uint32_t)pl.p2 << 16);
    const uint32_t w_cut = (uint32_t)pl.meta.a | ((uint32_t)pl.meta.b << 12) | (pl.meta.cx ? 1u << 24 : 0u) |
                           (pl.meta.mx ? 1u << 25 : 0u);
    const uint32_t w_mut = (uint32_t)pl.meta.mi | ((uint32_t)pl.meta.mj << 12);
    const uint16_t* gp = L->genes[cur];
    // the parents' rows of the next candidate are read into registers while
    // the current one is built (rows of up to 1024 genes)
    const int nv = n_pad >> 3;
    constexpr int PV2 = 2;
    const bool pre = nv <= PV2 * kWave;
    const auto* g4 = as_global(reinterpret_cast<const u32x4*>(gp));
    u32x4 ra[PV2], rb[PV2];
    auto fetch = [&](int c) {
        const uint32_t src = (uint32_t)__builtin_amdgcn_readlane((int)w_src, c);
#pragma unroll
        for (int v = 0; v < PV2; ++v) {
            const int x = lane + v * kWave;
            if (x < nv) {
                ra[v] = g4[(size_t)(src & 0xFFFFu) * nv + x];
                rb[v] = g4[(size_t)(src >> 16) * nv + x];
            }
        }
    };
    if (pre) fetch(0);
    for (int c = 0; c < K; ++c) {
        const uint32_t src = (uint32_t)__builtin_amdgcn_readlane((int)w_src, c);
        const uint32_t cut = (uint32_t)__builtin_amdgcn_readlane((int)w_cut, c);
        const uint32_t mut = (uint32_t)__builtin_amdgcn_readlane((int)w_mut, c);
        CellMeta cm;
        cm.mk1 = __builtin_amdgcn_readlane(pl.meta.mk1, c);
        cm.mk2 = __builtin_amdgcn_readlane(pl.meta.mk2, c);
        cm.a = (int)(cut & 0xFFFu);
        cm.b = (int)((cut >> 12) & 0xFFFu);
        cm.cx = ((cut >> 24) & 1u) != 0u;
        cm.mx = ((cut >> 25) & 1u) != 0u;
        cm.mi = (int)(mut & 0xFFFu);
        cm.mj = (int)(mut >> 12);
        if (pre) {
            u32x4* da = reinterpret_cast<u32x4*>(A);
            u32x4* db = reinterpret_cast<u32x4*>(B);
#pragma unroll
            for (int v = 0; v < PV2; ++v) {
                const int x = lane + v * kWave;
                if (x < nv) {
                    da[x] = ra[v];
                    db[x] = rb[v];
                }
            }
        } else {
            rows_g2l(A, gp + (size_t)(src & 0xFFFFu) * n_pad, B, gp + (size_t)(src >> 16) * n_pad, n_pad, lane,
                     kWave);
        }
        wave_sync();
        if (pre && c + 1 < K) fetch(c + 1);
        ox_group<true, false, 16>(A, B, V, n, cm.a, cm.b, cm.cx, lane, kWave, 0);
        swap_genes(A, cm.mx && lane == 0, cm.mi, cm.mj);
        cand_features<SM, PT>(A, pJ, rsb, I, cm, acc, lane, Xout + ((size_t)cell * K + c) * kFeat);
        wave_sync();
    }
}

// LDS bytes of a k_cand_features workgroup of `waves` waves.
__host__ __device__ inline size_t cand_lds_bytes(int n, int n_pad, int rsb, int waves)
{
    return align16((size_t)n * rsb) + (size_t)waves * ((size_t)group_stride(n_pad) * 2 + 240 * 4);
}

}  // namespace flowshop
