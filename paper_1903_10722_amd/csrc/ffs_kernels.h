// ffs_kernels.h -- gfx950 kernels of the island GA hot path.
//
// Mapping (one wave = 64 lanes):
//   * a wave holds G = floor(64 / S) chromosomes; lane g*S + k works on
//     stage k of chromosome g ("group" g).  Lanes beyond G*S idle.
//   * decode (paper Section 3 problem; list-scheduling rule documented in
//     include/ffs.h) runs as a systolic pipeline along the group: the lane of
//     stage k keeps the m_k machine-free times of its stage, sorted, in
//     registers, dispatches one job per step and releases finished jobs, in
//     (completion, dispatch order), through a small LDS ring to stage k+1.
//     A job can be released once the stage has started a later job at or
//     after its completion time: later starts never decrease and every
//     processing time is >= 1, so no later completion can precede it.
//   * the genetic operators (Section 4.1-4.2: neighbourhood choice, order
//     crossover, swap mutation, complementary pairs) run on the same group of
//     lanes on chromosomes staged in LDS; the crossover's fill uses a wave
//     ballot and a per-group prefix count.
//   * populations live in HBM as rows of n_pad uint16 genes (slot-major,
//     64-byte aligned rows), double buffered by generation parity.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ffs_mlp.h"
#include "philox.h"

namespace flowshop {

constexpr int kWave = 64;
constexpr int kMaxStages = 64;
constexpr int kMaxMachines = 16;

// The islands of a context form fold groups: the islands whose generations
// one launch sequence runs (a launch chain of a large instance's islands, or
// a launch class's instances), whose best individuals the extra workgroup of
// that sequence's launches folds into the best-ever records.  Between
// migration epochs the groups' sequences are independent.  An instance split
// over two chains keeps a record per chain (record slot); its record is the
// better of the two by (makespan, generation, island, slot).
constexpr int kChains = 2;      // record slots per instance
constexpr int kMaxGroups = 16;  // fold groups per context

struct InstDesc {
    const void* pT;          // [S][n_pad] processing times, uint8 or uint16
    uint16_t* best_perm;     // [kChains][n_pad]
    int* best_rec;           // [kChains][4]: makespan, generation, island (local), slot
    long long* counters;     // migration epochs with moves, migrants
    unsigned long long seed;
    unsigned long long theta_T;  // floor(theta * 2^32)
    long long E;                 // sum of all processing times
    int inst_id;
    int n, S, n_pad, jb, G;
    int fsh;                     // lane decode: completion shift of the three-field key (2 jb), 0: not used
    int psh;                     // pipelined decode: the same where every completion fits, 0: not used
    int island0, n_islands;
    int interval, topology;
    // learned pre-screen (surr_k > 1): candidate streams per cell, replay ring
    int surr_k, surr_warmup, n_cells, ring_size;
    int* surr_choice;            // [n_cells] candidate chosen for the next generation
    const uint16_t* surr_X;      // [n_cells * surr_k][256] features of the scored candidates
    uint16_t* ring_X;            // [ring_size][256] features of decoded children
    float* ring_T;               // [ring_size] (C - LB) / LB
    int LB, msum;
    int lane_wlds, lane_wlds_eval;   // lane mapping: LDS bytes per wave (generation, ffs_evaluate)
    const void* pJ;              // pre-screen: job-major processing times, rows of pj_row_bytes
    int pj_row_bytes;
    int mach[kMaxStages];
    int Pk[kMaxStages];          // sum over jobs of p[j][k]
};

struct IslandDesc {
    uint16_t* genes[2];          // [size][n_pad] per generation parity
    int* mk[2];                  // [size]
    unsigned long long* genkey;  // [2]: min of (makespan << 32 | slot), by generation parity
    unsigned long long* minmax;  // [2] min / max keys (ring migration)
    int* sorted;                 // [size] slots by (makespan, slot) (migration)
    int* sortbest;               // [1] island minimum makespan when `sorted` was built
    unsigned long long tc, tm;   // crossover / mutation thresholds (< tc, < tm)
    int kind, rows, cols, size;
    int inst;
    int local;                   // island index inside its instance
    int cell_base;               // index of slot 0 among the instance's cellular cells
    int sel;                     // cellular parent selection variant (0, 1, 2)
    int sweep;                   // cellular update: 0 synchronous, 1 line sweep
    int chain;                   // fold group of the island's generations
    int rec;                     // its instance's record slot for that group
};

struct WorkItem {
    int island, slot0, count, inst;
};

struct PairDesc {
    int a, b, inst, pad;
};

// Generation bookkeeping without a last-workgroup handshake or a shared
// counter: workgroup b of every generation launch keeps its own count of the
// launches it has run, counts[b], so launch number counts[b] after `base`
// runs generation base + 1 + counts[b]; the counts of all workgroups agree
// between launches, and kernels that run between launches read counts[0].
struct Control {
    int* counts;                 // [workgroups per generation launch]
    int base;                    // completed generation when the counts were zero
    int best_gen[kMaxGroups];    // per fold group: last generation folded into the records
    int err;                     // bit 0: invalid permutation, bit 1: decode fault
};

__device__ __forceinline__ int completed_gen(const Control* c)
{
    return c->base + c->counts[0];
}

extern __shared__ __align__(16) unsigned char ffs_smem[];

// Global-memory views of generic pointers: accesses through them compile to
// global (not flat) instructions, which the compiler may keep in flight
// across LDS accesses.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* as_global(const T* p)
{
    return (const __attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS of one group: three n_pad rows of uint16 and 16 bytes of padding, so
// that the groups of a wave start 4 banks apart and same-offset accesses of
// different groups do not collide.
__host__ __device__ inline int group_stride(int n_pad) { return 3 * n_pad + 8; }

__host__ __device__ inline size_t wave_lds_bytes(int G, int n_pad)
{
    return (size_t)G * group_stride(n_pad) * 2;
}

// The processing-time table is staged into LDS stage-major with each row
// padded by 4 bytes, so that the S rows start on different LDS banks (the S
// lanes of a group read the same job in S different rows).
template <typename PT>
__host__ __device__ inline int pt_stride(int n_pad) { return n_pad + 4 / (int)sizeof(PT); }

template <typename PT>
__host__ __device__ inline size_t pt_lds_bytes(int S, int n_pad)
{
    return align16((size_t)S * pt_stride<PT>(n_pad) * sizeof(PT));
}

// HBM rows of n_pad elements -> LDS rows of pt_stride elements (32-bit words).
template <typename PT>
__device__ __forceinline__ void stage_pt(PT* dst, const void* src, int S, int n_pad)
{
    constexpr int U = 4;
    const int wpr = (int)(n_pad * sizeof(PT) / 4), ld = wpr + 1, nw = S * wpr;
    const auto* s = as_global(reinterpret_cast<const uint32_t*>(src));
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    for (int w0 = threadIdx.x; w0 < nw; w0 += U * blockDim.x) {
        uint32_t x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int w = w0 + u * blockDim.x;
            x[u] = s[w < nw ? w : nw - 1];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // past the end: the last word again, with the same value
            const int w = w0 + u * blockDim.x < nw ? w0 + u * blockDim.x : nw - 1;
            const int r = w / wpr, c = w - r * wpr;
            d[r * ld + c] = x[u];
        }
    }
}

// ---- row copies by the S lanes of a group (16-byte vectors) ---------------
// The global reads of a row are all issued before the LDS writes.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void rows_g2l(uint16_t* dA, const uint16_t* sA, uint16_t* dB, const uint16_t* sB,
                                         int n_pad, int k, int S)
{
    constexpr int U = 4;
    const auto* a4 = as_global(reinterpret_cast<const u32x4*>(sA));
    const auto* b4 = as_global(reinterpret_cast<const u32x4*>(sB));
    u32x4* da = reinterpret_cast<u32x4*>(dA);
    u32x4* db = reinterpret_cast<u32x4*>(dB);
    const int nv = n_pad >> 3;
    for (int v0 = k; v0 < nv; v0 += U * S) {
        u32x4 xa[U], xb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * S < nv ? v0 + u * S : nv - 1;
            xa[u] = a4[v];
            xb[u] = b4[v];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // past the end: the last vector again, with the same value
            const int v = v0 + u * S < nv ? v0 + u * S : nv - 1;
            da[v] = xa[u];
            db[v] = xb[u];
        }
    }
}

__device__ __forceinline__ void row_g2l(uint16_t* dst, const uint16_t* src, int n_pad, int k, int S)
{
    constexpr int U = 4;
    const auto* s4 = as_global(reinterpret_cast<const u32x4*>(src));
    u32x4* d4 = reinterpret_cast<u32x4*>(dst);
    const int nv = n_pad >> 3;
    for (int v0 = k; v0 < nv; v0 += U * S) {
        u32x4 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * S < nv ? v0 + u * S : nv - 1;
            x[u] = s4[v];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int v = v0 + u * S < nv ? v0 + u * S : nv - 1;
            d4[v] = x[u];
        }
    }
}

__device__ __forceinline__ void row_g2g(uint16_t* dst, const uint16_t* src, int n_pad, int k, int S)
{
    constexpr int U = 4;
    const auto* s4 = as_global(reinterpret_cast<const u32x4*>(src));
    auto* d4 = as_global(reinterpret_cast<u32x4*>(dst));
    const int nv = n_pad >> 3;
    for (int v0 = k; v0 < nv; v0 += U * S) {
        u32x4 x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = s4[v0 + u * S < nv ? v0 + u * S : nv - 1];
#pragma unroll
        for (int u = 0; u < U; ++u) d4[v0 + u * S < nv ? v0 + u * S : nv - 1] = x[u];
    }
}

__device__ __forceinline__ void row_l2g(uint16_t* dst, const uint16_t* src, int n_pad, int k, int S)
{
    const u32x4* s4 = reinterpret_cast<const u32x4*>(src);
    auto* d4 = as_global(reinterpret_cast<u32x4*>(dst));
    const int nv = n_pad >> 3;
#pragma unroll 4
    for (int v = k; v < nv; v += S) d4[v] = s4[v];
}

// ---- pipelined decode -----------------------------------------------------
// Value of `x` held by lane - 1 (whole-wave shift right by one lane, DPP;
// lane 0 reads 0).
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}

// One step of stage k (see decode_pipelined).  With PRED the lane acts only
// while rel < n_act and takes a job only while rel < n; without it the caller
// guarantees both for every lane that matters.
// Median of three unsigned words (one VALU operation).
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Key formats: F = false, completion << jb | job, a new key entering after
// the entries of equal completion by a threshold compare per entry; F =
// true, completion << sh | dispatch index << jb | job (sh = 2 jb, the
// dispatch index counting stage k's dispatches, dsh = that index << jb), whose
// numeric order is (completion, dispatch order), so the new key enters by
// one min, median or max per entry.
template <int MMAX, bool PRED, bool F, typename PT>
__device__ __forceinline__ void pipe_step(uint32_t (&key)[MMAX], uint32_t& o_key, uint32_t& o_p, uint32_t& pn_pre,
                                          uint32_t ap, uint32_t rel, uint32_t n_act, uint32_t un, bool first,
                                          uint32_t jb, uint32_t jmask, const PT* prow_next, uint32_t sh,
                                          uint32_t dsh)
{
    constexpr uint32_t PAD = 0xFFFFFFFFu;
    const uint32_t in_key = from_prev_lane(o_key);
    const uint32_t in_p = from_prev_lane(o_p);
    if (!PRED || rel < n_act) {
        const bool have = !PRED || rel < un;
        // stage 0 takes its job word (p << jb | job) from AP, the others the
        // handed-on key and processing time
        const uint32_t x = first ? ap : in_key;
        const uint32_t j = x & jmask;
        const uint32_t o = key[0];
        uint32_t nkey[MMAX];
        if (F) {
            const uint32_t mx = first ? o : (o > in_key ? o : in_key);
            const uint32_t pj = first ? (ap >> jb) : in_p;
            const uint32_t c = (mx >> sh) + pj;
            const uint32_t nk = have ? ((c << sh) | dsh | j) : PAD;
            if (MMAX == 1) {
                nkey[0] = nk;
            } else {
                nkey[0] = key[1 < MMAX ? 1 : 0] < nk ? key[1 < MMAX ? 1 : 0] : nk;
#pragma unroll
                for (int i = 1; i + 1 < MMAX; ++i) nkey[i] = umed3(key[i], nk, key[i + 1]);
                nkey[MMAX - 1] = key[MMAX - 1] > nk ? key[MMAX - 1] : nk;
            }
        } else {
            const uint32_t hi = x >> jb;
            const uint32_t r = first ? 0u : hi;
            const uint32_t pj = first ? hi : in_p;
            const uint32_t f = o >> jb;
            const uint32_t st = f > r ? f : r;
            const uint32_t c = st + pj;
            const uint32_t nk = have ? ((c << jb) | j) : PAD;
            const uint32_t ithr = have ? ((c + 1u) << jb) : PAD;
            bool prev = true;
#pragma unroll
            for (int i = 0; i < MMAX; ++i) {
                const bool lt = (i + 1 < MMAX) ? (key[(i + 1 < MMAX) ? i + 1 : i] < ithr) : false;
                nkey[i] = lt ? key[(i + 1 < MMAX) ? i + 1 : i] : (prev ? nk : key[i]);
                prev = lt;
            }
        }
#pragma unroll
        for (int i = 0; i < MMAX; ++i) key[i] = nkey[i];
        o_key = o;
        o_p = pn_pre;
    }
    // every lane holds real jobs while all stages dispatch, so only the
    // predicated fill and drain steps clamp the index
    const uint32_t q = key[0] & jmask;
    pn_pre = (uint32_t)prow_next[PRED ? min(q, un - 1u) : q];
}

// One group of S lanes decodes one permutation; lane k runs stage k.
//
// Stage k keeps its m_k machine-free times as a sorted list of keys (one of
// pipe_step's two formats) in registers; a machine that has not run a job yet
// holds key 0, a padding entry (fewer than MMAX machines) 0xFFFFFFFF.  Each
// step dispatches the next job: it takes the machine of entry 0 (free first;
// ties on time only relabel machines), starts at max(free, ready) and inserts
// its completion.  The removed entry 0 is handed to stage k+1: entries leave
// the list in (completion, dispatch order) order, which is the order in which
// stage k+1 must dispatch them.  After its last job a stage hands on its
// remaining entries, one per step.
//
// The timing of this pipeline does not depend on the data: stage k acts in
// steps [a_k, a_k + n) (dispatch) and, unless it is the last stage, in
// [a_k + n, a_k + n + m_k) (hand-on of the rest); the first m_k entries it
// removes are the never-used machines, so its real jobs leave in steps
// [a_k + m_k, a_k + m_k + n) and stage k+1 starts at a_{k+1} = a_k + m_k + 1.
// The decode therefore runs exactly n + sum_{k<S-1} (m_k + 1) steps, and a
// job handed on in one step is taken by the next lane in the next step, so
// one register pair per lane carries it: (key, processing time at k+1).
// In steps [a_{S-1}, n) every stage is dispatching, so that stretch runs
// without per-lane predication; lanes of unused groups then compute values
// nobody reads (their loads stay in bounds).
//
// AP[t] = (p[job][0] << jb) | job for the permutation's t-th job.  Returns
// the makespan on the lane of the last stage.
template <int MMAX, bool F, typename PT>
__device__ __forceinline__ uint32_t decode_pipelined_keys(const uint32_t* AP, const PT* prow_next, const int* mach,
                                                          int k, int S, int n, int jb, bool active)
{
    constexpr uint32_t PAD = 0xFFFFFFFFu;
    int a_k = 0, total = n;
    for (int i = 0; i + 1 < S; ++i) {
        const int step = mach[i] + 1;
        if (i < k) a_k += step;
        total += step;
    }
    const int a_last = total - n;
    const int mstage = mach[k];
    uint32_t key[MMAX];
#pragma unroll
    for (int i = 0; i < MMAX; ++i) key[i] = (i < mstage) ? 0u : PAD;
    uint32_t o_key = 0, o_p = 0;
    const bool first = (k == 0), last = (k == S - 1);
    const uint32_t jmask = (1u << jb) - 1u;
    const uint32_t ujb = (uint32_t)jb;
    const uint32_t un = (uint32_t)n;
    const uint32_t n_act = active ? (last ? un : un + (uint32_t)mstage) : 0u;
    uint32_t pn_pre = (uint32_t)prow_next[0];
    // three-field keys: the dispatch index of step it is it - a_k
    const uint32_t sh = 2u * ujb, dstep = 1u << ujb;
    uint32_t dsh = F ? (uint32_t)(0 - a_k) << ujb : 0u;
    // the steady stretch starts on a multiple of 4 so that its job words can
    // be read four at a time (AP is 16-byte aligned)
    const int steady0 = (a_last + 3) & ~3;
    const int fill_end = steady0 < n ? steady0 : n;
    int it = 0;
    for (; it < fill_end; ++it) {
        pipe_step<MMAX, true, F, PT>(key, o_key, o_p, pn_pre, AP[it], (uint32_t)(it - a_k), n_act, un, first, ujb,
                                     jmask, prow_next, sh, dsh);
        dsh += dstep;
    }
    if (it + 3 < n) {
        uint4 cur = *reinterpret_cast<const uint4*>(AP + it);
        for (; it + 3 < n; it += 4) {
            const int nx = (it + 7 < n) ? it + 4 : it;
            const uint4 nxt = *reinterpret_cast<const uint4*>(AP + nx);
            asm volatile("" ::: "memory");   // keep the read ahead of the four steps
            pipe_step<MMAX, false, F, PT>(key, o_key, o_p, pn_pre, cur.x, 0u, 0u, un, first, ujb, jmask, prow_next,
                                          sh, dsh);
            pipe_step<MMAX, false, F, PT>(key, o_key, o_p, pn_pre, cur.y, 0u, 0u, un, first, ujb, jmask, prow_next,
                                          sh, dsh + dstep);
            pipe_step<MMAX, false, F, PT>(key, o_key, o_p, pn_pre, cur.z, 0u, 0u, un, first, ujb, jmask, prow_next,
                                          sh, dsh + 2u * dstep);
            pipe_step<MMAX, false, F, PT>(key, o_key, o_p, pn_pre, cur.w, 0u, 0u, un, first, ujb, jmask, prow_next,
                                          sh, dsh + 3u * dstep);
            dsh += 4u * dstep;
            cur = nxt;
        }
    }
    for (; it < total; ++it) {
        pipe_step<MMAX, true, F, PT>(key, o_key, o_p, pn_pre, AP[it < n ? it : n - 1], (uint32_t)(it - a_k), n_act,
                                     un, first, ujb, jmask, prow_next, sh, dsh);
        dsh += dstep;
    }
    // the last stage's list now holds every machine's final completion time
    uint32_t cmax = 0;
#pragma unroll
    for (int i = 0; i < MMAX; ++i) {
        const uint32_t c = (key[i] == PAD) ? 0u : (key[i] >> (F ? sh : ujb));
        cmax = c > cmax ? c : cmax;
    }
    return cmax;
}

// The pipelined decode with the instance's key format: three-field keys
// where every completion fits their completion field (psh = 2 jb, set when
// the sum of all processing times does), else two-field keys.
template <int MMAX, typename PT>
__device__ __forceinline__ uint32_t decode_pipelined(const uint32_t* AP, const PT* prow_next, const int* mach,
                                                     int k, int S, int n, int jb, int psh, bool active)
{
    if (psh > 0) return decode_pipelined_keys<MMAX, true, PT>(AP, prow_next, mach, k, S, n, jb, active);
    return decode_pipelined_keys<MMAX, false, PT>(AP, prow_next, mach, k, S, n, jb, active);
}

// AP[t] = (p[A[t]][0] << jb) | A[t], built by the group's lanes.
template <typename PT>
__device__ __forceinline__ void build_ap(uint32_t* AP, const uint16_t* A, const PT* prow0, int n, int jb, int k,
                                         int S, bool active)
{
    constexpr int U = 4;
    if (active)
        for (int t0 = k; t0 < n; t0 += U * S) {
            uint32_t j[U], pj[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * S;
                j[u] = A[t < n ? t : 0];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) pj[u] = prow0[j[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * S;
                if (t < n) AP[t] = (pj[u] << jb) | j[u];
            }
        }
    wave_sync();
}

// ---- order crossover on a group -------------------------------------------
// A = parent 1 (becomes the child), B = parent 2, V = scratch for the inverse
// of parent 1.  child[a..b] = P1[a..b]; P2 read cyclically from b+1 fills
// b+1, ..., n-1, 0, ..., a-1 with the genes not in the segment.  Lane k of
// the group owns the cyclic offsets [kC, kC + C) of P2 (C = ceil(n / S)):
// it counts the genes it keeps, an exclusive scan over the group's lanes
// gives its first destination, and a second pass writes them.  REG and MID
// select which register-holding paths are compiled (REG up to RMAX genes
// per lane); without both only the two-pass path remains (fewest registers).
__device__ __forceinline__ uint32_t wrap_sub(uint32_t x, uint32_t n)
{
    const uint32_t y = x - n;   // x < 2n: x mod n
    return y < x ? y : x;
}

// Register path for C <= kOxReg: each lane reads its parent-1 and parent-2
// genes once, so the whole crossover costs three LDS round trips plus the
// group scan.
constexpr int kOxReg = 24;
constexpr int kOxMid = 64;   // rows with up to this many positions per lane keep P2 in registers

__device__ __forceinline__ int group_exclusive_scan(int v, int k, int S)
{
    int incl = v;
    for (int d = 1; d < S; d <<= 1) {
        const int up = __shfl_up(incl, d, 64);
        if (k >= d) incl += up;
    }
    return incl - v;
}

// Register path: lane k holds positions [o0, o1) of parent 1 and cyclic
// offsets [o0, o1) of parent 2 (o1 - o0 <= CM), so the crossover costs three
// LDS round trips plus the group scan.
template <int CM>
__device__ __forceinline__ void ox_reg(uint16_t* A, const uint16_t* B, uint16_t* V, uint32_t un, uint32_t ua,
                                       uint32_t ub, bool doit, int k, int S, int o0, int o1)
{
    // lane k: positions [o0, o1) of parent 1 and cyclic offsets [o0, o1) of parent 2
    uint32_t x1[CM], x2[CM];
#pragma unroll
    for (int u = 0; u < CM; ++u) {
        const bool ok = o0 + u < o1;
        x1[u] = A[ok ? o0 + u : 0];
        x2[u] = B[ok ? wrap_sub(ub + 1u + (uint32_t)(o0 + u), un) : 0u];
    }
    if (doit) {
#pragma unroll
        for (int u = 0; u < CM; ++u)
            if (o0 + u < o1) V[x1[u]] = (uint16_t)(o0 + u);
    }
    wave_sync();
    uint32_t keep = 0;
    int cnt = 0;
#pragma unroll
    for (int u = 0; u < CM; ++u) {
        const uint32_t iv = V[x2[u]];
        const bool kp = (o0 + u < o1) && (iv < ua || iv > ub);
        keep |= kp ? (1u << u) : 0u;
        cnt += kp ? 1 : 0;
    }
    const int pre = group_exclusive_scan(cnt, k, S);
    if (doit) {
        uint32_t dst = wrap_sub(ub + 1u + (uint32_t)pre, un);
#pragma unroll
        for (int u = 0; u < CM; ++u)
            if (keep & (1u << u)) {
                A[dst] = (uint16_t)x2[u];
                dst = wrap_sub(dst + 1u, un);
            }
    }
    wave_sync();
}

// Middle path: P2's genes held in registers between the count and the write.
template <int CM>
__device__ __forceinline__ void ox_mid(uint16_t* A, const uint16_t* B, uint16_t* V, uint32_t un, uint32_t ua,
                                       uint32_t ub, bool doit, int k, int S, int o0, int o1)
{
    constexpr int U = 8;
    if (doit) {
        for (int t0 = o0; t0 < o1; t0 += U) {
            uint32_t x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = A[t0 + u < o1 ? t0 + u : 0];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (t0 + u < o1) V[x[u]] = (uint16_t)(t0 + u);
        }
    }
    wave_sync();
    uint32_t x2[CM];
    unsigned long long keep = 0ull;
    int cnt = 0;
    if (doit) {
#pragma unroll
        for (int u = 0; u < CM; ++u) {
            const uint32_t p = wrap_sub(ub + 1u + (uint32_t)(o0 + u), un);
            x2[u] = B[(o0 + u < o1) ? p : 0u];
        }
#pragma unroll
        for (int u = 0; u < CM; ++u) {
            const uint32_t iv = V[x2[u]];
            const bool kp = (o0 + u < o1) && (iv < ua || iv > ub);
            keep |= kp ? (1ull << u) : 0ull;
            cnt += kp ? 1 : 0;
        }
    }
    const int pre = group_exclusive_scan(cnt, k, S);
    if (doit) {
        uint32_t dst = wrap_sub(ub + 1u + (uint32_t)pre, un);
#pragma unroll
        for (int u = 0; u < CM; ++u)
            if (keep & (1ull << u)) {
                A[dst] = (uint16_t)x2[u];
                dst = wrap_sub(dst + 1u, un);
            }
    }
    wave_sync();
}

template <bool REG = true, bool MID = true, int RMAX = kOxReg>
__device__ __forceinline__ void ox_group(uint16_t* A, const uint16_t* B, uint16_t* V, int n, int a, int b,
                                         bool doit, int k, int S, int g)
{
    const uint32_t un = (uint32_t)n, ua = (uint32_t)a, ub = (uint32_t)b;
    const int C = (n + S - 1) / S;
    const int o0 = k * C, o1 = (o0 + C < n) ? o0 + C : n;
    if (REG && C <= 8) {
        ox_reg<8>(A, B, V, un, ua, ub, doit, k, S, o0, o1);
        return;
    }
    if (REG && RMAX >= 16 && C <= 16) {
        ox_reg<16>(A, B, V, un, ua, ub, doit, k, S, o0, o1);
        return;
    }
    if (REG && RMAX >= kOxReg && C <= kOxReg) {
        ox_reg<kOxReg>(A, B, V, un, ua, ub, doit, k, S, o0, o1);
        return;
    }
    if (MID && C <= 32) {
        ox_mid<32>(A, B, V, un, ua, ub, doit, k, S, o0, o1);
        return;
    }
    if (MID && C <= kOxMid) {
        ox_mid<kOxMid>(A, B, V, un, ua, ub, doit, k, S, o0, o1);
        return;
    }
    // long rows: two passes over P2 in chunks of U
    constexpr int U = 8;
    if (doit) {
        for (int t0 = o0; t0 < o1; t0 += U) {
            uint32_t x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) x[u] = A[t0 + u < o1 ? t0 + u : 0];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (t0 + u < o1) V[x[u]] = (uint16_t)(t0 + u);
        }
    }
    wave_sync();
    int cnt = 0;
    if (doit) {
        for (int ob = o0; ob < o1; ob += U) {
            uint32_t x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t p = wrap_sub(ub + 1u + (uint32_t)(ob + u), un);
                x[u] = B[(ob + u < o1) ? p : 0u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t iv = V[x[u]];
                cnt += (ob + u < o1 && (iv < ua || iv > ub)) ? 1 : 0;
            }
        }
    }
    const int pre = group_exclusive_scan(cnt, k, S);
    if (doit) {
        uint32_t dst = wrap_sub(ub + 1u + (uint32_t)pre, un);
        for (int ob = o0; ob < o1; ob += U) {
            uint32_t x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t p = wrap_sub(ub + 1u + (uint32_t)(ob + u), un);
                x[u] = B[(ob + u < o1) ? p : 0u];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t iv = V[x[u]];
                if (ob + u < o1 && (iv < ua || iv > ub)) {
                    A[dst] = (uint16_t)x[u];
                    dst = wrap_sub(dst + 1u, un);
                }
            }
        }
    }
    wave_sync();
}

__device__ __forceinline__ void swap_genes(uint16_t* A, bool doit, int i, int j)
{
    if (doit) {
        const uint16_t x = A[i], y = A[j];
        A[i] = y;
        A[j] = x;
    }
    wave_sync();
}

// ---- cellular offspring ----------------------------------------------------
struct CellMeta {
    int mk1, mk2, a, b, mi, mj;
    bool cx, mx;
};

// Parents and draws of the child of cell `slot` at generation `gen` from
// candidate stream `sub` (sub 0 is the plain GA's stream): P1, P2 = the two
// best of (self, N, E, S, W) by (makespan, that order) in generation gen-1
// (or the selection variant of the island), then the crossover flag and
// cuts and the swap mutation's flag and positions.
struct CellPlan {
    int p1, p2;
    bool n1, n2;      // line sweep: the parent's row is already the new generation's
    CellMeta meta;
};

// Parents and draws of cell `slot` at generation `gen` (Section 4.2).  With
// sdiag >= 0 (the cell's anti-diagonal r + c in a line sweep) a neighbour on
// a lower anti-diagonal precedes the cell in row-major order, the torus's
// wrapped neighbours included, so its makespan and row are read from the
// generation being built (buffer cur ^ 1); the others and the cell itself
// from generation gen - 1.
__device__ __forceinline__ CellPlan cell_plan(const InstDesc* I, const IslandDesc* L, int slot, uint32_t sub, int gen,
                                              int cur, int sdiag = -1)
{
    const int n = I->n;
    const auto* mkp = as_global(L->mk[cur]);
    const auto* mkn = as_global(L->mk[cur ^ 1]);
    const int rows = L->rows, cols = L->cols;
    const int r = slot / cols, c = slot - r * cols;
    const int nb0 = slot;
    const int nb1 = ((r == 0) ? rows - 1 : r - 1) * cols + c;
    const int nb2 = r * cols + ((c == cols - 1) ? 0 : c + 1);
    const int nb3 = ((r == rows - 1) ? 0 : r + 1) * cols + c;
    const int nb4 = r * cols + ((c == 0) ? cols - 1 : c - 1);
    const bool sw = sdiag >= 0;
    const bool u1 = sw && r > 0, u2 = sw && c == cols - 1, u3 = sw && r == rows - 1, u4 = sw && c > 0;
    const int v0 = mkp[nb0];
    const int v1 = (u1 ? mkn : mkp)[nb1], v2 = (u2 ? mkn : mkp)[nb2];
    const int v3 = (u3 ? mkn : mkp)[nb3], v4 = (u4 ? mkn : mkp)[nb4];
    const Block4 bk = stream_block(I->seed, (uint64_t)I->inst_id, (uint32_t)L->local, (uint32_t)slot, sub,
                                   (uint32_t)gen, kCell, 0);
    int bv, bs, sv, ss;
    const int sel = L->sel;
    if (sel == 1) {
        // self + the best of (N, E, S, W) by (makespan, order)
        bv = v0;
        bs = nb0;
        sv = v1;
        ss = nb1;
        if (v2 < sv) { sv = v2; ss = nb2; }
        if (v3 < sv) { sv = v3; ss = nb3; }
        if (v4 < sv) { sv = v4; ss = nb4; }
    } else if (sel == 2) {
        // binary tournaments: draws 6 and 7 each pick two positions of the
        // neighbourhood (x / 5, x % 5 with x uniform in [0, 25)); the better
        // by (makespan, position) wins
        const int vv[5] = {v0, v1, v2, v3, v4}, nn[5] = {nb0, nb1, nb2, nb3, nb4};
        int win[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int x = (int)below(draw32(bk, 6 + t), 25u);
            const int i = x / 5, j = x - 5 * (x / 5);
            int vi = vv[0], vj = vv[0];
#pragma unroll
            for (int q = 1; q < 5; ++q) {
                vi = (i == q) ? vv[q] : vi;
                vj = (j == q) ? vv[q] : vj;
            }
            win[t] = (vj < vi || (vj == vi && j < i)) ? j : i;
        }
        bv = vv[0]; bs = nn[0]; sv = vv[0]; ss = nn[0];
#pragma unroll
        for (int q = 1; q < 5; ++q) {
            if (win[0] == q) { bv = vv[q]; bs = nn[q]; }
            if (win[1] == q) { sv = vv[q]; ss = nn[q]; }
        }
    } else {
        // the two best of (self, N, E, S, W) by (makespan, order)
        int bo = 0;
        bv = v0;
        bs = nb0;
        if (v1 < bv) { bv = v1; bs = nb1; bo = 1; }
        if (v2 < bv) { bv = v2; bs = nb2; bo = 2; }
        if (v3 < bv) { bv = v3; bs = nb3; bo = 3; }
        if (v4 < bv) { bv = v4; bs = nb4; bo = 4; }
        sv = 0x7FFFFFFF;
        ss = -1;
        if (bo != 0 && v0 < sv) { sv = v0; ss = nb0; }
        if (bo != 1 && v1 < sv) { sv = v1; ss = nb1; }
        if (bo != 2 && v2 < sv) { sv = v2; ss = nb2; }
        if (bo != 3 && v3 < sv) { sv = v3; ss = nb3; }
        if (bo != 4 && v4 < sv) { sv = v4; ss = nb4; }
        if (ss < 0) ss = nb1;   // only when every makespan is INT_MAX (never)
    }
    CellPlan pl;
    pl.p1 = bs;
    pl.p2 = ss;
    pl.n1 = (bs == nb1 && u1) || (bs == nb2 && u2) || (bs == nb3 && u3) || (bs == nb4 && u4);
    pl.n2 = (ss == nb1 && u1) || (ss == nb2 && u2) || (ss == nb3 && u3) || (ss == nb4 && u4);
    pl.meta.mk1 = bv;
    pl.meta.mk2 = sv;
    pl.meta.cx = (uint64_t)draw32(bk, 0) < L->tc;
    const int u = (int)below(draw32(bk, 1), (uint32_t)n), w = (int)below(draw32(bk, 2), (uint32_t)n);
    pl.meta.a = u < w ? u : w;
    pl.meta.b = u < w ? w : u;
    pl.meta.mx = (uint64_t)draw32(bk, 3) < L->tm;
    pl.meta.mi = (int)below(draw32(bk, 4), (uint32_t)n);
    int mj = pl.meta.mi + 1 + (int)below(draw32(bk, 5), (uint32_t)(n - 1));
    if (mj >= n) mj -= n;
    pl.meta.mj = mj;
    return pl;
}

// The child of cell `slot` (cell_plan) built on the group's LDS rows: order
// crossover of P1 and P2, then the swap mutation.  A receives the child.
template <bool LEAN = false>
__device__ __forceinline__ CellMeta cellular_offspring(const InstDesc* I, const IslandDesc* L, int slot, uint32_t sub,
                                                   int gen, int cur, uint16_t* A, uint16_t* B, uint16_t* V, int k,
                                                   int S, int g, bool active)
{
    const int n = I->n, n_pad = I->n_pad;
    const CellPlan pl = cell_plan(I, L, slot, sub, gen, cur);
    const uint16_t* gp = L->genes[cur];
    if (active) rows_g2l(A, gp + (size_t)pl.p1 * n_pad, B, gp + (size_t)pl.p2 * n_pad, n_pad, k, S);
    wave_sync();
    ox_group<!LEAN, !LEAN>(A, B, V, n, pl.meta.a, pl.meta.b, pl.meta.cx && active, k, S, g);
    swap_genes(A, pl.meta.mx && active && k == 0, pl.meta.mi, pl.meta.mj);
    return pl.meta;
}

// Draws of the pseudo island's slot `slot` at generation `gen` (Section
// 4.1, complementary parents): X = the better of its pair (2q, 2q + 1) by
// (makespan, slot) in generation gen-1; the even slot gets OX(X, Y), the odd
// one OX(Y, X) with Y = reverse(X), both with the pair's cuts; each child has
// its own mutation draws.
struct PairPlan {
    int xs;
    bool odd, cx, mx;
    int a, b, mi, mj;
};

__device__ __forceinline__ PairPlan pair_plan(const InstDesc* I, const IslandDesc* L, int slot, int gen, int cur)
{
    const int n = I->n;
    const auto* mkp = as_global(L->mk[cur]);
    const int q = slot >> 1;
    PairPlan pl;
    pl.odd = slot & 1;
    pl.xs = (mkp[2 * q] <= mkp[2 * q + 1]) ? 2 * q : 2 * q + 1;
    const uint64_t seed = I->seed, iid = (uint64_t)I->inst_id;
    const uint32_t isl_local = (uint32_t)L->local;
    const Block4 b0 = stream_block(seed, iid, isl_local, (uint32_t)q, 0, (uint32_t)gen, kPair, 0);
    const Block4 b1 = stream_block(seed, iid, isl_local, (uint32_t)q, 0, (uint32_t)gen, kPair, 1);
    pl.cx = (uint64_t)draw32(b0, 0) < L->tc;
    const int u = (int)below(draw32(b0, 1), (uint32_t)n), w = (int)below(draw32(b0, 2), (uint32_t)n);
    pl.a = u < w ? u : w;
    pl.b = u < w ? w : u;
    const uint32_t dm = pl.odd ? draw32(b0, 6) : draw32(b0, 3);
    const uint32_t di = pl.odd ? draw32(b0, 7) : draw32(b0, 4);
    const uint32_t dj = pl.odd ? draw32(b1, 0) : draw32(b0, 5);
    pl.mx = (uint64_t)dm < L->tm;
    pl.mi = (int)below(di, (uint32_t)n);
    int mj = pl.mi + 1 + (int)below(dj, (uint32_t)(n - 1));
    if (mj >= n) mj -= n;
    pl.mj = mj;
    return pl;
}

// A = X (even slot) or reverse(X) (odd slot) and B the other, from X in V.
__device__ __forceinline__ void pair_parents(uint16_t* A, uint16_t* B, const uint16_t* V, int n, bool odd, int k,
                                             int S, bool active)
{
    if (active) {
        constexpr int U = 4;
        for (int t0 = k; t0 < n; t0 += U * S) {
            uint16_t x[U], xr[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * S < n ? t0 + u * S : n - 1;
                x[u] = V[t];
                xr[u] = V[n - 1 - t];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * S < n ? t0 + u * S : n - 1;
                A[t] = odd ? xr[u] : x[u];
                B[t] = odd ? x[u] : xr[u];
            }
        }
    }
    wave_sync();
}

// Pre-screen input of the chromosome in A (the group's S lanes): lane k sums
// stage k's processing times over each of B = floor(240 / S) position
// buckets (position t is in bucket floor(t B / n)) and writes
// bf16(fp32(load * B) / fp32(P_k)) at index b * S + k; indices B*S .. 239 and
// 252 .. 255 are 0; 240 .. 251 hold the scalars (parents' makespans / LB,
// cut points / n, crossover flag, mutation flag, swap positions / n, LB / E,
// n / 1000, S / 20, sum m / (6 S)).  Every ratio is one correctly rounded
// FP32 division.
template <typename PT>
__device__ __forceinline__ void features_group(const uint16_t* A, const PT* pT, const InstDesc* I, int k, bool active,
                                               const CellMeta& cm, uint16_t* out)
{
    if (!active) return;
    const int n = I->n, S = I->S, n_pad = I->n_pad;
    const int B = 240 / S;
    const PT* prow = pT + (size_t)k * pt_stride<PT>(n_pad);
    const float Pk = (float)I->Pk[k];
    int t = 0;
    for (int bb = 0; bb < B; ++bb) {
        const int tend = ((bb + 1) * n + B - 1) / B;
        uint32_t load = 0;
#pragma unroll 8
        for (; t < tend; ++t) load += prow[A[t]];
        out[bb * S + k] = f32_to_bf16(__fdiv_rn((float)((uint64_t)load * (uint64_t)B), Pk));
    }
    const float fn = (float)n, fLB = (float)I->LB;
    for (int e = B * S + k; e < kFeat; e += S) {
        float v = 0.f;
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
        out[e] = f32_to_bf16(v);
    }
}

// The chromosome of `slot` at generation `gen`, built in row A of a group of
// S lanes (lane k) with B and V as scratch: generation 0 (mode 1) draws it;
// a cellular cell gets the child of its neighbourhood's two best from
// candidate stream `sub`; a pseudo slot gets its pair's complementary child.
template <bool LEAN = false>
__device__ __forceinline__ CellMeta make_child(const InstDesc* I, const IslandDesc* L, int slot, uint32_t sub,
                                               int gen, int cur, int mode, uint16_t* A, uint16_t* B, uint16_t* V,
                                               int k, int S, int g, bool active)
{
    const int n = I->n, n_pad = I->n_pad;
    const uint64_t seed = I->seed, iid = (uint64_t)I->inst_id;
    const uint32_t isl_local = (uint32_t)L->local;
    CellMeta meta{};
    if (mode == 1) {
        // generation 0: Fisher-Yates from the INIT stream; a pseudo pair is a
        // permutation (even slot) and its reversal (odd slot).
        const int fy_slot = (L->kind == 0) ? slot : (slot >> 1);
        const bool rev = (L->kind == 1) && (slot & 1);
        uint32_t* D = reinterpret_cast<uint32_t*>(B);   // B..V: n_pad words >= n - 1
        const int nblk = (n - 1 + 7) / 8;
        if (active) {
            for (int blk = k; blk < nblk; blk += S) {
                const Block4 bb = stream_block(seed, iid, isl_local, (uint32_t)fy_slot, 0, 0, kInit, (uint32_t)blk);
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int idx = blk * 8 + d;
                    if (idx < n - 1) D[idx] = draw32(bb, d);
                }
            }
            for (int t = k; t < n; t += S) A[t] = (uint16_t)t;
        }
        wave_sync();
        if (active && k == 0) {
            for (int i = n - 1; i >= 1; --i) {
                const int j = (int)below(D[n - 1 - i], (uint32_t)(i + 1));
                const uint16_t x = A[i], y = A[j];
                A[i] = y;
                A[j] = x;
            }
        }
        wave_sync();
        if (active && rev) {
            for (int t = k; t < n / 2; t += S) {
                const uint16_t x = A[t], y = A[n - 1 - t];
                A[t] = y;
                A[n - 1 - t] = x;
            }
        }
        wave_sync();
    } else if (L->kind == 0) {
        meta = cellular_offspring<LEAN>(I, L, slot, sub, gen, cur, A, B, V, k, S, g, active);
    } else {
        // pseudo: X = better of the pair, Y = reverse(X); even slot gets
        // OX(X, Y), odd slot OX(Y, X), with shared cut points.
        const PairPlan pl = pair_plan(I, L, slot, gen, cur);
        if (active) row_g2l(V, L->genes[cur] + (size_t)pl.xs * n_pad, n_pad, k, S);
        wave_sync();
        pair_parents(A, B, V, n, pl.odd, k, S, active);
        ox_group<!LEAN, !LEAN>(A, B, V, n, pl.a, pl.b, pl.cx && active, k, S, g);
        swap_genes(A, pl.mx && active && k == 0, pl.mi, pl.mj);
    }
    return meta;
}

// ---- best-ever records ------------------------------------------------------
// Folds generation g into the best-ever records of every instance: the
// minimum (makespan, slot) key of each island, ties on makespan to the lowest
// island; a strictly better makespan replaces the record and copies the
// permutation from generation g's population.  Resets the islands' keys of
// g's parity for generation g + 2.  Run by one workgroup; s_tmp holds
// 3 * blockDim.x ints (fold_lds_bytes).
__host__ __device__ inline size_t fold_lds_bytes(int threads) { return (size_t)3 * sizeof(int) * threads; }

__device__ void fold_best(const InstDesc* __restrict__ insts, const IslandDesc* __restrict__ isls, int n_inst,
                          int g, Control* ctl, int* s_tmp, int group)
{
    const int par = g & 1;
    int* s_imp = s_tmp;
    int* s_isl = s_imp + blockDim.x;
    int* s_slot = s_isl + blockDim.x;
    for (int base = 0; base < n_inst; base += blockDim.x) {
        const int ii = base + threadIdx.x;
        int imp = 0, bisl = -1, bslot = -1;
        if (ii < n_inst) {
            const InstDesc* J = insts + ii;
            unsigned long long bkey = ~0ull;
            for (int x = 0; x < J->n_islands; ++x) {
                if (isls[J->island0 + x].chain != group) continue;
                unsigned long long* gk = isls[J->island0 + x].genkey + par;
                const unsigned long long v = __hip_atomic_load(gk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (bisl < 0 || (v >> 32) < (bkey >> 32)) {
                    bkey = v;
                    bisl = x;
                }
                __hip_atomic_store(gk, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (bisl >= 0) {
                const int slot = isls[J->island0 + bisl].rec;
                int* rec = J->best_rec + 4 * slot;
                bslot = (int)(bkey & 0xFFFFFFFFu);
                const int bmk = (int)(bkey >> 32);
                if (bmk < rec[0]) {
                    rec[0] = bmk;
                    rec[1] = g;
                    rec[2] = bisl;
                    rec[3] = bslot;
                    imp = 1;
                }
            }
        }
        s_imp[threadIdx.x] = imp;
        s_isl[threadIdx.x] = bisl;
        s_slot[threadIdx.x] = bslot;
        __syncthreads();
        const int lim = (n_inst - base) < (int)blockDim.x ? (n_inst - base) : (int)blockDim.x;
        for (int t = 0; t < lim; ++t) {
            if (!s_imp[t]) continue;
            const InstDesc* J = insts + base + t;
            const IslandDesc* X = isls + J->island0 + s_isl[t];
            const uint4* s4 = reinterpret_cast<const uint4*>(X->genes[par] + (size_t)s_slot[t] * J->n_pad);
            uint4* d4 = reinterpret_cast<uint4*>(J->best_perm + (size_t)X->rec * J->n_pad);
            for (int v = threadIdx.x; v < (J->n_pad >> 3); v += blockDim.x) d4[v] = s4[v];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) ctl->best_gen[group] = g;
}

// Folds the completed generation into the best-ever records of every fold
// group that has not done so yet (one workgroup).
__global__ void __launch_bounds__(256) k_best_flush(const InstDesc* __restrict__ insts,
                                                    const IslandDesc* __restrict__ isls, Control* ctl, int n_inst,
                                                    int groups)
{
    __shared__ int s_tmp[3 * 256];
    const int g = completed_gen(ctl);
    for (int group = 0; group < groups; ++group)
        if (ctl->best_gen[group] < g) fold_best(insts, isls, n_inst, g, ctl, s_tmp, group);
}

// ---- one generation (mode 0) or generation 0 (mode 1) of every island -----
template <int MMAX, typename PT>
__global__ void __launch_bounds__(512) k_generation(const InstDesc* __restrict__ insts,
                                                    const IslandDesc* __restrict__ isls,
                                                    const WorkItem* __restrict__ work, Control* ctl, int n_inst,
                                                    int mode, int cnt_off, int has_extra)
{
    // generation number from this workgroup's launch count (generation 0 has none)
    __shared__ int s_gen;
    if (threadIdx.x == 0) {
        int gg = 0;
        if (mode == 0) {
            int* cnt = ctl->counts + cnt_off + blockIdx.x;
            const int t = *cnt;
            *cnt = t + 1;
            gg = ctl->base + 1 + t;
        }
        s_gen = gg;
    }
    // the workgroup after the work items folds the previous generation into
    // the best-ever records while the others run this one
    // has_extra = 1 + group: the last workgroup folds that fold group's
    // previous generation
    if (has_extra && blockIdx.x == gridDim.x - 1) {
        __syncthreads();
        const int prev = s_gen - 1, group = has_extra - 1;
        if (ctl->best_gen[group] < prev)
            fold_best(insts, isls, n_inst, prev, ctl, reinterpret_cast<int*>(ffs_smem), group);
        return;
    }
    // When every workgroup is resident at once, give each XCD (the hardware
    // places workgroup b on XCD b % 8) a contiguous run of work items, so
    // that neighbouring cells share an L2; larger grids keep the
    // largest-first order.
    const int nw = (int)gridDim.x - (has_extra ? 1 : 0);
    int widx = (int)blockIdx.x;
    if (nw <= 256) {
        const int per = (nw + 7) / 8, full = nw - 8 * (per - 1);
        const int xcd = widx & 7, rnk = widx >> 3;
        widx = (xcd < full) ? xcd * per + rnk : full * per + (xcd - full) * (per - 1) + rnk;
    }
    const WorkItem wi = work[widx];
    const InstDesc* I = insts + wi.inst;
    const IslandDesc* L = isls + wi.island;
    if (mode == 0 && L->sweep) return;   // line-sweep islands have launches of their own
    const int n = I->n, S = I->S, n_pad = I->n_pad, jb = I->jb, G = I->G;

    PT* pT = reinterpret_cast<PT*>(ffs_smem);
    stage_pt<PT>(pT, I->pT, S, n_pad);
    __syncthreads();
    const int gen = s_gen;
    const int cur = (gen + 1) & 1, nxt = gen & 1;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint16_t* gbase = reinterpret_cast<uint16_t*>(ffs_smem + pt_lds_bytes<PT>(S, n_pad) +
                                                  wave * wave_lds_bytes(G, n_pad));
    const int g = lane / S, k = lane - g * S;
    const int local = wave * G + g;
    const bool active = (g < G) && (local < wi.count);
    uint16_t* A = gbase + (size_t)(active ? g : 0) * group_stride(n_pad);
    uint16_t* B = A + n_pad;
    uint16_t* V = B + n_pad;
    const int slot = wi.slot0 + (active ? local : 0);
    const PT* prow_next = pT + (size_t)(k + 1 < S ? k + 1 : S - 1) * pt_stride<PT>(n_pad);

    const bool screened = mode == 0 && L->kind == 0 && I->surr_k > 1 && gen > I->surr_warmup;
    const uint32_t sub = screened ? (uint32_t)I->surr_choice[L->cell_base + slot] : 0u;
    const CellMeta meta = make_child(I, L, slot, sub, gen, cur, mode, A, B, V, k, S, g, active);

    uint32_t* AP = reinterpret_cast<uint32_t*>(B);   // B..V: n_pad words
    build_ap<PT>(AP, A, pT, n, jb, k, S, active);
    const uint32_t cm = decode_pipelined<MMAX, PT>(AP, prow_next, I->mach, k, S, n, jb, I->psh, active);
    const int src = active ? (g * S + S - 1) : lane;
    const int cmg = __shfl((int)cm, src, 64);

    unsigned long long wkey = ~0ull;
    if (active) {
        uint16_t* dstrow = L->genes[nxt] + (size_t)slot * n_pad;
        int mk_new;
        if (mode == 1 || L->kind == 1) {
            mk_new = cmg;
            row_l2g(dstrow, A, n_pad, k, S);
        } else {
            const int mk_old = as_global(L->mk[cur])[slot];
            const bool rep = cmg < mk_old;
            mk_new = rep ? cmg : mk_old;
            if (rep) {
                row_l2g(dstrow, A, n_pad, k, S);
            } else {
                row_g2g(dstrow, L->genes[cur] + (size_t)slot * n_pad, n_pad, k, S);
            }
        }
        if (k == 0) L->mk[nxt][slot] = mk_new;
        wkey = (k == 0) ? (((unsigned long long)(unsigned)mk_new << 32) | (unsigned)slot) : ~0ull;
    }
    if (mode == 0 && L->kind == 0 && I->surr_k > 1) {
        // training data of the pre-screen: the decoded child and its exact
        // makespan; a screened child's features were computed when it was scored
        const int cell = L->cell_base + slot;
        const long long ri = ((long long)(gen - 1) * I->n_cells + cell) % I->ring_size;
        uint16_t* dst = I->ring_X + ri * kFeat;
        if (gen > I->surr_warmup) {
            if (active) {
                const uint4* s4 = reinterpret_cast<const uint4*>(
                    I->surr_X + ((size_t)cell * I->surr_k + (size_t)I->surr_choice[cell]) * kFeat);
                uint4* d4 = reinterpret_cast<uint4*>(dst);
                for (int v = k; v < kFeat / 8; v += S) d4[v] = s4[v];
            }
        } else {
            features_group<PT>(A, pT, I, k, active, meta, dst);
        }
        if (active && k == 0) I->ring_T[ri] = __fdiv_rn((float)(cmg - I->LB), (float)I->LB);
    }
    // island minimum of (makespan, slot): wave reduction, then one atomic per workgroup
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(wkey, off, 64);
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

// ---- decode of caller-supplied permutations -------------------------------
template <int MMAX, typename PT>
__global__ void __launch_bounds__(512) k_evaluate(const InstDesc* __restrict__ I, const int* __restrict__ perms,
                                                  int count, int* __restrict__ out, Control* ctl)
{
    const int n = I->n, S = I->S, n_pad = I->n_pad, jb = I->jb, G = I->G;
    PT* pT = reinterpret_cast<PT*>(ffs_smem);
    stage_pt<PT>(pT, I->pT, S, n_pad);
    __syncthreads();
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint16_t* gbase = reinterpret_cast<uint16_t*>(ffs_smem + pt_lds_bytes<PT>(S, n_pad) +
                                                  wave * wave_lds_bytes(G, n_pad));
    const int g = lane / S, k = lane - g * S;
    const long long idx = ((long long)blockIdx.x * wpb + wave) * G + g;
    const bool active = (g < G) && (idx < count);
    uint16_t* A = gbase + (size_t)(active ? g : 0) * group_stride(n_pad);
    uint16_t* V = A + 2 * n_pad;
    bool bad = false;
    if (active) {
        const int* row = perms + idx * (long long)n;
        for (int t = k; t < n; t += S) {
            const int x = row[t];
            const bool ob = (unsigned)x >= (unsigned)n;
            bad |= ob;
            A[t] = ob ? (uint16_t)0 : (uint16_t)x;
            if (!ob) V[x] = (uint16_t)t;
        }
    }
    wave_sync();
    if (active)
        for (int t = k; t < n; t += S) bad |= (V[A[t]] != (uint16_t)t);
    const uint64_t gmask = (S >= 64) ? ~0ull : ((1ull << S) - 1ull);
    const uint64_t bb = __ballot(bad && active);
    const int shift = g * S;
    const bool gbad = ((shift < 64 ? (bb >> shift) : 0ull) & gmask) != 0ull;
    uint32_t* AP = reinterpret_cast<uint32_t*>(A + n_pad);   // B..V: n_pad words
    build_ap<PT>(AP, A, pT, n, jb, k, S, active);
    const uint32_t cm = decode_pipelined<MMAX, PT>(AP, pT + (size_t)(k + 1 < S ? k + 1 : S - 1) * pt_stride<PT>(n_pad), I->mach,
                                                   k, S, n, jb, I->psh, active);
    if (active && k == S - 1) out[idx] = gbad ? -1 : (int)cm;
    if (active && k == 0 && gbad) atomicOr(&ctl->err, 1);
}

// ---- candidates of the learned pre-screen ----------------------------------
// Row q = cell * K + c: the child cell `cell` would get at the next
// generation from candidate stream c, as features (Xout[q]) and, when Tout
// is given, its exact (C - LB) / LB (the judge of the pre-screen's ranking).
template <int MMAX, typename PT>
__global__ void __launch_bounds__(512) k_candidates(const InstDesc* __restrict__ insts,
                                                    const IslandDesc* __restrict__ isls, int inst,
                                                    const Control* ctl, int Nc, uint16_t* __restrict__ Xout,
                                                    float* __restrict__ Tout)
{
    const InstDesc* I = insts + inst;
    const int n = I->n, S = I->S, n_pad = I->n_pad, jb = I->jb, G = I->G, K = I->surr_k;
    const int done = completed_gen(ctl);
    const int gen = done + 1, cur = done & 1;
    PT* pT = reinterpret_cast<PT*>(ffs_smem);
    stage_pt<PT>(pT, I->pT, S, n_pad);
    __syncthreads();
    const int wpb = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint16_t* gbase = reinterpret_cast<uint16_t*>(ffs_smem + pt_lds_bytes<PT>(S, n_pad) +
                                                  wave * wave_lds_bytes(G, n_pad));
    const int g = lane / S, k = lane - g * S;
    const int q = (blockIdx.x * wpb + wave) * G + g;
    const bool active = (g < G) && (q < Nc);
    const int qq = active ? q : 0;
    const int cell = qq / K, c = qq - cell * K;
    const IslandDesc* L = isls + I->island0;
    int slot = 0;
    for (int x = 0; x < I->n_islands; ++x) {
        const IslandDesc* X = isls + I->island0 + x;
        if (X->kind == 0 && cell >= X->cell_base && cell < X->cell_base + X->size) {
            L = X;
            slot = cell - X->cell_base;
        }
    }
    uint16_t* A = gbase + (size_t)(active ? g : 0) * group_stride(n_pad);
    uint16_t* B = A + n_pad;
    uint16_t* V = B + n_pad;
    const CellMeta meta = cellular_offspring(I, L, slot, (uint32_t)c, gen, cur, A, B, V, k, S, g, active);
    features_group<PT>(A, pT, I, k, active, meta, Xout + (size_t)qq * kFeat);
    if (Tout) {
        uint32_t* AP = reinterpret_cast<uint32_t*>(B);
        build_ap<PT>(AP, A, pT, n, jb, k, S, active);
        const uint32_t cm = decode_pipelined<MMAX, PT>(AP, pT + (size_t)(k + 1 < S ? k + 1 : S - 1) * pt_stride<PT>(n_pad),
                                                       I->mach, k, S, n, jb, I->psh, active);
        const int cmg = __shfl((int)cm, active ? (g * S + S - 1) : lane, 64);
        if (active && k == 0) Tout[q] = __fdiv_rn((float)(cmg - I->LB), (float)I->LB);
    }
}

// Parameters of the 256-512-512-1 network, one FP32 vector: W1 [512][256],
// b1 [512], W2 [512][512], b2 [512], w3 [512], b3.  Weights uniform in
// +-sqrt(6 / fan_in) from the MLP_INIT stream (slot = tensor index, draw =
// element index), biases 0; Adam moments 0.
constexpr int kP_W1 = 0, kP_b1 = 131072, kP_W2 = 131584, kP_b2 = 393728, kP_w3 = 394240, kP_b3 = 394752;
constexpr int kParams = 394753;

__global__ void __launch_bounds__(256) k_mlp_init(uint64_t seed, uint64_t inst, float* __restrict__ w,
                                                  uint16_t* __restrict__ wb, float* __restrict__ m,
                                                  float* __restrict__ v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kParams) return;
    int tensor, elem, fan_in;
    if (i < kP_b1) { tensor = 0; elem = i; fan_in = 256; }
    else if (i < kP_W2) { tensor = 1; elem = i - kP_b1; fan_in = 0; }
    else if (i < kP_b2) { tensor = 2; elem = i - kP_W2; fan_in = 512; }
    else if (i < kP_w3) { tensor = 3; elem = i - kP_b2; fan_in = 0; }
    else if (i < kP_b3) { tensor = 4; elem = i - kP_w3; fan_in = 512; }
    else { tensor = 5; elem = 0; fan_in = 0; }
    float x = 0.f;
    if (fan_in > 0) {
        const Block4 b = stream_block(seed, inst, 0, (uint32_t)tensor, 0, 0, kMlpInit, (uint32_t)(elem >> 3));
        const uint64_t word = b.w[(elem & 7) >> 1];
        const uint32_t u = (elem & 1) ? (uint32_t)(word >> 32) : (uint32_t)word;
        const float f = ((float)(u >> 8) + 0.5f) * 5.9604644775390625e-08f;   // (0, 1), 2^-24 steps
        x = (2.f * f - 1.f) * sqrtf(6.f / (float)fan_in);
    }
    w[i] = x;
    wb[i] = f32_to_bf16(x);
    m[i] = 0.f;
    v[i] = 0.f;
}

// Minibatch rows of the training step after the last completed generation
// g: uniform over the filled part of the replay ring (min(g * cells, ring)
// rows), from the MLP_BATCH stream of step g (draw r -> row r).  The
// generation comes from the control block, so a captured graph replays it.
__global__ void __launch_bounds__(256) k_batch_idx(uint64_t seed, uint64_t inst, const Control* __restrict__ ctl,
                                                   int cells, int ring, int rows, int* __restrict__ idx)
{
    const int blk = blockIdx.x * blockDim.x + threadIdx.x;
    if (blk * 8 >= rows) return;
    const int gen = completed_gen(ctl);
    const long long f = (long long)gen * cells;
    const uint32_t filled = (uint32_t)(f < ring ? f : ring);
    const Block4 b = stream_block(seed, inst, 0, 0, 0, (uint32_t)gen, kMlpBatch, (uint32_t)blk);
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int r = blk * 8 + d;
        if (r < rows) idx[r] = (int)below(draw32(b, d), filled);
    }
}

__global__ void __launch_bounds__(256) k_zero_u32(uint32_t* __restrict__ p, size_t count)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// ---- migration (paper Section 4.3) -----------------------------------------
__device__ __forceinline__ bool migrating_now(const InstDesc* I, int inst, int gen, int force_inst)
{
    if (force_inst >= 0) return inst == force_inst;
    return I->interval > 0 && gen > 0 && (gen % I->interval) == 0;
}

__global__ void __launch_bounds__(256) k_mig_minmax(const InstDesc* __restrict__ insts,
                                                    const IslandDesc* __restrict__ isls, const Control* ctl,
                                                    int force_inst)
{
    const IslandDesc* L = isls + blockIdx.x;
    const InstDesc* I = insts + L->inst;
    const int gen = completed_gen(ctl);
    if (!migrating_now(I, L->inst, gen, force_inst) || I->topology != 1) return;
    const int* mk = L->mk[gen & 1];
    unsigned long long mn = ~0ull, mx = 0ull;
    for (int s = threadIdx.x; s < L->size; s += blockDim.x) {
        const unsigned long long v = ((unsigned long long)(unsigned)mk[s] << 32) | (unsigned)s;
        mn = v < mn ? v : mn;
        mx = v > mx ? v : mx;
    }
    __shared__ unsigned long long smn[256], smx[256];
    smn[threadIdx.x] = mn;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            smn[threadIdx.x] = smn[threadIdx.x + w] < smn[threadIdx.x] ? smn[threadIdx.x + w] : smn[threadIdx.x];
            smx[threadIdx.x] = smx[threadIdx.x + w] > smx[threadIdx.x] ? smx[threadIdx.x + w] : smx[threadIdx.x];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        L->minmax[0] = smn[0];
        L->minmax[1] = smx[0];
    }
}

// ring c0, p0, c1, p1, ...: island x receives its predecessor's best into its worst slot
__global__ void __launch_bounds__(256) k_mig_ring(const InstDesc* __restrict__ insts,
                                                  const IslandDesc* __restrict__ isls, const Control* ctl,
                                                  int force_inst)
{
    const IslandDesc* L = isls + blockIdx.x;
    const InstDesc* I = insts + L->inst;
    const int gen = completed_gen(ctl);
    if (!migrating_now(I, L->inst, gen, force_inst) || I->topology != 1) return;
    const int H = I->n_islands / 2;
    if (H == 0) return;
    const int l = L->local;
    const int pos = (l < H) ? 2 * l : 2 * (l - H) + 1;
    const int pp = (pos == 0) ? 2 * H - 1 : pos - 1;
    const int pl = (pp & 1) ? H + (pp >> 1) : (pp >> 1);
    const IslandDesc* P = isls + I->island0 + pl;
    const int par = gen & 1;
    const int ss = (int)(P->minmax[0] & 0xFFFFFFFFu);
    const int ds = (int)(L->minmax[1] & 0xFFFFFFFFu);
    const int n_pad = I->n_pad;
    const uint4* s4 = reinterpret_cast<const uint4*>(P->genes[par] + (size_t)ss * n_pad);
    uint4* d4 = reinterpret_cast<uint4*>(L->genes[par] + (size_t)ds * n_pad);
    for (int v = threadIdx.x; v < (n_pad >> 3); v += blockDim.x) d4[v] = s4[v];
    if (threadIdx.x == 0) L->mk[par][ds] = P->mk[par][ss];
}

// Stable sort of one island's slots by makespan (ties keep slot order): a
// least-significant-digit-first radix sort over the bits of (makespan -
// island minimum), two bits per pass.  1024 threads hold R = max(1, P/1024)
// items each in striped order (item i = r * 1024 + thread); per pass, a wave
// ballot per digit value and the per-(digit, r, wave) counts, prefixed in
// that order, give every item its place; a pass is three block barriers, and
// an island whose makespans span 2^b values needs ceil(b / 2) passes.
// Padding items (i >= size) carry all ones and stay at the end.
constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortRMax = 16;
constexpr int kSortDigits = 4;   // two bits per pass
constexpr int kSortEnt = kSortDigits * kSortRMax * kSortWaves;   // counts per pass, at most

__host__ __device__ inline size_t sort_lds_bytes(int R)
{
    return (size_t)R * kSortThreads * (sizeof(uint32_t) + sizeof(uint16_t)) +
           (size_t)2 * kSortEnt * sizeof(uint32_t) + (size_t)2 * kSortWaves * sizeof(uint32_t);
}

__global__ void __launch_bounds__(kSortThreads) k_mig_sort(const InstDesc* __restrict__ insts,
                                                           const IslandDesc* __restrict__ isls,
                                                           const Control* ctl, int force_inst, int only_inst)
{
    const IslandDesc* L = isls + blockIdx.x;
    const InstDesc* I = insts + L->inst;
    const int gen = completed_gen(ctl);
    if (only_inst >= 0 && L->inst != only_inst) return;
    if (!migrating_now(I, L->inst, gen, force_inst)) return;
    const int N = L->size;
    int R = 1;
    while (R * kSortThreads < N) R <<= 1;
    const int P = R * kSortThreads;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    uint32_t* dbuf = reinterpret_cast<uint32_t*>(ffs_smem);
    uint16_t* sbuf = reinterpret_cast<uint16_t*>(dbuf + P);
    uint32_t* zcnt = reinterpret_cast<uint32_t*>(sbuf + P);      // [digit][r][wave] counts
    uint32_t* zpre = zcnt + kSortEnt;                            // their exclusive prefix, same order
    uint32_t* misc = zpre + kSortEnt;                            // [0..15] wave minima, [16..31] maxima
    const int* mk = L->mk[gen & 1];

    uint32_t d[kSortRMax], sl[kSortRMax];
    uint32_t mn = 0xFFFFFFFFu, mx = 0u;
#pragma unroll
    for (int r = 0; r < kSortRMax; ++r) {
        const int i = r * kSortThreads + t;
        d[r] = 0xFFFFFFFFu;
        sl[r] = (uint32_t)i;
        if (r < R && i < N) {
            d[r] = (uint32_t)mk[i];
            mn = d[r] < mn ? d[r] : mn;
            mx = d[r] > mx ? d[r] : mx;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint32_t a = (uint32_t)__shfl_xor((int)mn, o, 64), b = (uint32_t)__shfl_xor((int)mx, o, 64);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    if (lane == 0) {
        misc[wave] = mn;
        misc[kSortWaves + wave] = mx;
    }
    __syncthreads();
    mn = 0xFFFFFFFFu;
    mx = 0u;
    for (int w = 0; w < kSortWaves; ++w) {
        const uint32_t a = misc[w], b = misc[kSortWaves + w];
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    // the island's best makespan, read by the migration decision (the rows
    // that the migration rewrites cannot change it afterwards)
    if (t == 0) L->sortbest[0] = (int)mn;
    const uint32_t span = mx - mn;   // N >= 1, so mn <= mx
    const int bits = span == 0u ? 0 : 32 - __clz((int)span);
#pragma unroll
    for (int r = 0; r < kSortRMax; ++r)
        if (r < R && r * kSortThreads + t < N) d[r] -= mn;

    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int nent = kSortDigits * R * kSortWaves;
    for (int bit = 0; bit < bits; bit += 2) {
        // items of each digit value per (r, wave)
#pragma unroll
        for (int r = 0; r < kSortRMax; ++r)
            if (r < R) {
                const uint32_t dg = (d[r] >> bit) & 3u;
#pragma unroll
                for (int v = 0; v < kSortDigits; ++v) {
                    const uint64_t bm = __ballot(dg == (uint32_t)v);
                    if (lane == 0) zcnt[(v * R + r) * kSortWaves + wave] = (uint32_t)__popcll(bm);
                }
            }
        __syncthreads();
        // exclusive prefix over (digit, r, wave) order, by wave 0: up to 16
        // consecutive entries per lane
        if (wave == 0) {
            const int per = (nent + 63) >> 6;
            uint32_t v[kSortEnt / 64], run = 0;
#pragma unroll
            for (int e = 0; e < kSortEnt / 64; ++e) {
                const int idx = lane * per + e;
                v[e] = (e < per && idx < nent) ? zcnt[idx] : 0u;
                run += v[e];
            }
            uint32_t incl = run;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t up = (uint32_t)__shfl_up((int)incl, o, 64);
                if (lane >= o) incl += up;
            }
            uint32_t ex = incl - run;
#pragma unroll
            for (int e = 0; e < kSortEnt / 64; ++e) {
                const int idx = lane * per + e;
                if (e < per && idx < nent) zpre[idx] = ex;
                ex += v[e];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortRMax; ++r)
            if (r < R) {
                const uint32_t dg = (d[r] >> bit) & 3u;
                // the lanes of this wave whose item has the same digit
                uint64_t m = 0;
#pragma unroll
                for (int v = 0; v < kSortDigits; ++v) {
                    const uint64_t bm = __ballot(dg == (uint32_t)v);
                    m = (dg == (uint32_t)v) ? bm : m;
                }
                const uint32_t pos = zpre[(dg * R + r) * kSortWaves + wave] + (uint32_t)__popcll(m & below);
                dbuf[pos] = d[r];
                sbuf[pos] = (uint16_t)sl[r];
            }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSortRMax; ++r)
            if (r < R) {
                d[r] = dbuf[r * kSortThreads + t];
                sl[r] = sbuf[r * kSortThreads + t];
            }
    }
    int* out = L->sorted;
#pragma unroll
    for (int r = 0; r < kSortRMax; ++r) {
        const int i = r * kSortThreads + t;
        if (r < R && i < N) out[i] = (int)sl[r];
    }
}

// adaptive penetration rule of equations (1)-(2) on one island pair, and the
// copy of the r-th best emigrant over the r-th worst immigrant.  Every block
// of the pair takes the decision from the bests that k_mig_sort recorded
// before any row moved, so all blocks agree whatever their order (when every
// immigrant slot is replaced, the immigrant's best row itself is rewritten).
constexpr int kMigRows = 32;

__global__ void __launch_bounds__(256) k_mig_adapt(const InstDesc* __restrict__ insts,
                                                   const IslandDesc* __restrict__ isls,
                                                   const PairDesc* __restrict__ pairs, const Control* ctl,
                                                   int force_inst)
{
    const PairDesc pd = pairs[blockIdx.x];
    const InstDesc* I = insts + pd.inst;
    const int gen = completed_gen(ctl);
    if (!migrating_now(I, pd.inst, gen, force_inst)) return;
    const IslandDesc* A = isls + pd.a;
    const IslandDesc* B = isls + pd.b;
    const int par = gen & 1;
    const long long ba = A->sortbest[0], bb = B->sortbest[0];
    long long fa = I->E - ba, fb = I->E - bb;
    if (fa < 0) fa = 0;
    if (fb < 0) fb = 0;
    if (fa == fb) return;
    const unsigned long long hi = (unsigned long long)(fa > fb ? fa : fb);
    const unsigned long long lo = (unsigned long long)(fa > fb ? fb : fa);
    if (hi == 0) return;
    if (!(((hi - lo) << 32) < I->theta_T * hi)) return;
    const unsigned long long N = (unsigned long long)(A->size < B->size ? A->size : B->size);
    unsigned long long count = (N * (hi - lo) + hi - 1) / hi;
    if (count > N) count = N;
    const IslandDesc* Em = (fa > fb) ? A : B;
    const IslandDesc* Im = (fa > fb) ? B : A;
    if (blockIdx.y == 0 && threadIdx.x == 0) {
        atomicAdd((unsigned long long*)&I->counters[0], 1ull);
        atomicAdd((unsigned long long*)&I->counters[1], count);
    }
    const int r0 = blockIdx.y * kMigRows;
    const int r1 = (int)((unsigned long long)(r0 + kMigRows) < count ? (unsigned long long)(r0 + kMigRows) : count);
    if (r0 >= r1) return;
    const int n_pad = I->n_pad, nv = n_pad >> 3;
    const int rows = r1 - r0;
    for (int e = threadIdx.x; e < rows * nv; e += blockDim.x) {
        const int r = r0 + e / nv, v = e - (e / nv) * nv;
        const int ss = Em->sorted[r];
        const int ds = Im->sorted[Im->size - 1 - r];
        const uint4* s4 = reinterpret_cast<const uint4*>(Em->genes[par] + (size_t)ss * n_pad);
        uint4* d4 = reinterpret_cast<uint4*>(Im->genes[par] + (size_t)ds * n_pad);
        d4[v] = s4[v];
    }
    for (int r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const int ss = Em->sorted[r];
        const int ds = Im->sorted[Im->size - 1 - r];
        Im->mk[par][ds] = Em->mk[par][ss];
    }
}

}  // namespace flowshop
