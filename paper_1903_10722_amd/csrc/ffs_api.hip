// ffs_api.hip -- host side of the C ABI declared in include/ffs.h.
//
// Host orchestration: instance validation, workspace layout (the library
// never allocates device memory), descriptor upload, kernel selection by the
// largest machine count (template MMAX) and the processing-time width, the
// generation loop with the migration schedule, and result download.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "ffs.h"
#include "ffs_kernels.h"
#include "ffs_lane.h"

using namespace flowshop;

// Device memory of the allocation-free decode (ffs_evaluate_noalloc): the
// control word, the instance descriptor, the caller's processing times and
// the stage-major table built from them.  One copy per GPU, for the life of
// the process; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = (size_t)1 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Stage-major table of an instance from its job-major processing times:
// pT[k][j] = p[j][k] for j < n, 0 in the padding up to n_pad.
__global__ void __launch_bounds__(256) k_build_table(const int* __restrict__ p, int n, int S, int n_pad, int ptb,
                                                     void* __restrict__ pT)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * n_pad) return;
    const int k = i / n_pad, j = i - k * n_pad;
    const int v = j < n ? p[(size_t)j * S + k] : 0;
    if (ptb == 1) reinterpret_cast<uint8_t*>(pT)[i] = (uint8_t)v;
    else reinterpret_cast<uint16_t*>(pT)[i] = (uint16_t)v;
}

// Completion shifts of the three-field decode key (completion, dispatch
// index, job): the lane decode's where its completion field holds 1.5 times
// the lower bound LB (makespans above it fall back to the two-field key),
// the pipelined decode's where every completion (at most the sum E of all
// processing times) fits, the key 0xFFFFFFFF staying padding; 0: not used.
static void key_shifts(int jb, long long LB, long long E, int& fsh, int& psh)
{
    const bool ok = 2 * jb <= 30;
    const long long cap = ok ? (1ll << (32 - 2 * jb)) : 0;
    fsh = (ok && 3 * LB < 2 * cap) ? 2 * jb : 0;
    psh = (ok && E < cap - 1) ? 2 * jb : 0;
}

namespace {

struct HostIsland {
    ffs_island_spec spec;
    int size;
    int cell_base;
    int chain = 0;                // fold group of its generations
    int rec = 0;                  // its instance's record slot
    size_t off_genes[2], off_mk[2], off_genkey, off_minmax, off_sorted, off_sortbest;
};

struct HostInstance {
    int n, S;
    std::vector<int> m, p;
    long long E;
    int maxP, mmax, jb, n_pad, G;
    std::vector<HostIsland> isl;
    ffs_ga_config cfg;
    uint64_t seed;
    long long LB;
    int msum, n_cells;
    std::vector<long long> Pk;
    size_t off_pT, off_best_perm, off_best_rec, off_counters;
    int edge0 = 0, n_edges = 0;   // topology 2: this instance's ring edges in the pair list
    int isl_base = 0;
    size_t lds = 0;               // LDS bytes of one generation workgroup
    size_t lane_wlds = 0, lane_wlds_eval = 0;   // lane mapping: LDS bytes per wave
    bool lane_ok = false;         // the lane mapping can run this instance
    int tile_map = -1, tile_wpb = 0;   // requested tile (-1 / 0: the context's)
    int map_eff = 0, wpb_eff = 4;      // tile the generation launches use
    int lds_bucket = 0, cls = 0;  // its LDS class
};

using GenKernel = void (*)(const InstDesc*, const IslandDesc*, const WorkItem*, Control*, int, int, int, int);
using EvalKernel = void (*)(const InstDesc*, const int*, int, int*, Control*);

template <int M, typename PT>
void* gen_ptr() { return reinterpret_cast<void*>(&k_generation<M, PT>); }
template <int M, typename PT>
void* eval_ptr() { return reinterpret_cast<void*>(&k_evaluate<M, PT>); }
template <int M, typename PT>
void* cand_ptr() { return reinterpret_cast<void*>(&k_candidates<M, PT>); }
template <int M, typename PT>
void* gen_lane_ptr() { return reinterpret_cast<void*>(&k_generation_lane<M, PT>); }
template <int M, typename PT>
void* eval_lane_ptr() { return reinterpret_cast<void*>(&k_evaluate_lane<M, PT>); }

const int kMmaxList[] = {2, 3, 4, 5, 6, 8, 16};

void* pick_gen(int mm, int ptb)
{
#define FFS_CASE(M)                                                          \
    if (mm == M) return ptb == 1 ? gen_ptr<M, uint8_t>() : gen_ptr<M, uint16_t>();
    FFS_CASE(2) FFS_CASE(3) FFS_CASE(4) FFS_CASE(5) FFS_CASE(6) FFS_CASE(8) FFS_CASE(16)
#undef FFS_CASE
    return nullptr;
}

void* pick_cand_features(int sm, int ptb)
{
#define FFS_CASE(SM)                                                                             \
    if (sm == SM) return ptb == 1 ? reinterpret_cast<void*>(&k_cand_features<SM, uint8_t>)      \
                                  : reinterpret_cast<void*>(&k_cand_features<SM, uint16_t>);
    FFS_CASE(8) FFS_CASE(16) FFS_CASE(20) FFS_CASE(24) FFS_CASE(32)
#undef FFS_CASE
    return nullptr;
}

void* pick_cand(int mm, int ptb)
{
#define FFS_CASE(M)                                                          \
    if (mm == M) return ptb == 1 ? cand_ptr<M, uint8_t>() : cand_ptr<M, uint16_t>();
    FFS_CASE(2) FFS_CASE(3) FFS_CASE(4) FFS_CASE(5) FFS_CASE(6) FFS_CASE(8) FFS_CASE(16)
#undef FFS_CASE
    return nullptr;
}

void* pick_eval(int mm, int ptb)
{
#define FFS_CASE(M)                                                          \
    if (mm == M) return ptb == 1 ? eval_ptr<M, uint8_t>() : eval_ptr<M, uint16_t>();
    FFS_CASE(2) FFS_CASE(3) FFS_CASE(4) FFS_CASE(5) FFS_CASE(6) FFS_CASE(8) FFS_CASE(16)
#undef FFS_CASE
    return nullptr;
}

// Lane-mapping kernels exist for machine counts up to 8.
void* pick_gen_lane(int mm, int ptb)
{
#define FFS_CASE(M)                                                          \
    if (mm == M) return ptb == 1 ? gen_lane_ptr<M, uint8_t>() : gen_lane_ptr<M, uint16_t>();
    FFS_CASE(2) FFS_CASE(3) FFS_CASE(4) FFS_CASE(5) FFS_CASE(6) FFS_CASE(8)
#undef FFS_CASE
    return nullptr;
}

void* pick_eval_lane(int mm, int ptb)
{
#define FFS_CASE(M)                                                          \
    if (mm == M) return ptb == 1 ? eval_lane_ptr<M, uint8_t>() : eval_lane_ptr<M, uint16_t>();
    FFS_CASE(2) FFS_CASE(3) FFS_CASE(4) FFS_CASE(5) FFS_CASE(6) FFS_CASE(8)
#undef FFS_CASE
    return nullptr;
}

// Below this many individuals in a context the lane mapping leaves most
// SIMDs idle (one wave per 64 individuals), and the per-stage lane mapping
// of k_generation is chosen when the mapping is automatic.
constexpr long long kLaneAutoMin = 131072;
constexpr long long kChainAutoMin = 131072;   // individuals per context for two launch chains
// ffs_evaluate takes the lane mapping from this many rows of at least this
// many stages (a million random rows: 1.45x and 1.65x faster at 10 and 20
// stages, 2.3x slower at 5, where the per-stage groups fill the wave too)
constexpr int kLaneEvalAutoMin = 65536;
constexpr int kLaneEvalMinStages = 8;

int round_mmax(int m)
{
    for (int v : kMmaxList)
        if (m <= v) return v;
    return -1;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int kBatch = 4096;    // training minibatch of the pre-screen
constexpr size_t kStageBytes = (size_t)4 << 20;   // staging of ffs_evaluate_host
constexpr int kRing = 65536;    // replay ring entries
constexpr float kLr = 1e-3f, kBeta1 = 0.9f, kBeta2 = 0.999f, kEps = 1e-8f;
constexpr int kBcSteps = 32768;
constexpr int kSweepWaves = 2;   // waves per workgroup of a line-sweep launch  // Adam steps with a bias-correction table entry (both 1 in FP32 after)

uint64_t rate_threshold(double p)
{
    if (p <= 0.0) return 0;
    if (p >= 1.0) return 4294967296ull;
    return (uint64_t)std::floor(p * 4294967296.0);
}

}  // namespace

struct ffs_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    std::vector<HostInstance> inst;
    int wpb = 4;
    int mapping = -1;            // requested decode mapping: -1 automatic, 0 per stage, 1 per lane
    bool lane = false;           // generation launches use the lane mapping
    bool bound = false;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    int gen = 0;
    std::string err;
    // layout
    size_t off_ctl = 0, off_insts = 0, off_isls = 0, off_work = 0, off_pairs = 0, off_counts = 0, total = 0;
    size_t off_stage = 0;            // host-pointer decode: staged rows and results
    int max_work = 0;
    int n_isl = 0, n_work = 0, n_pairs = 0, max_size = 0, max_edges = 0, n_cls = 1;
    std::vector<int> cls_w0;         // work range of class k: [cls_w0[k], cls_w0[k+1])
    std::vector<size_t> cls_lds;     // LDS bytes of class k's launch
    std::vector<void*> cls_kern;     // generation kernel of class k
    std::vector<int> cls_wpb;        // waves per workgroup of class k
    int max_lds = 65536;             // dynamic LDS bytes a workgroup may use on this device
    bool concurrent = true;          // classes of one generation run side by side
    std::vector<hipStream_t> aux;    // streams of classes 1.. (forked from `stream`)
    std::vector<hipEvent_t> fork_ev; // fork and join events, one per class
    int mm = 2, ptb = 1;
    size_t lds_gen = 0, lds_sort = 0;
    bool any_ring = false;
    void* keval = nullptr;
    std::vector<WorkItem> work;
    std::vector<PairDesc> pairs;
    // line-sweep islands: one work item each, launched one anti-diagonal at a
    // time after every generation launch
    std::vector<WorkItem> sweep;
    // launch chains: with two, the islands form two groups whose generations
    // of an epoch run as two launch sequences side by side (graph branches),
    // joined before the epoch's migration
    int chains = -1;               // requested: -1 automatic, 1, 2
    int nchain = 1;                // in use
    int chain_w0[3] = {0, 0, 0};   // work ranges of the chains (single class)
    // with several launch classes, each class is a fold group whose
    // generations of an epoch run as one branch of the epoch graph
    bool class_groups = false;
    int ngroup = 1;                // fold groups
    int sweep_diags = 0;
    size_t off_sweep = 0, sweep_lds = 0;
    void* sweep_kern = nullptr;
    // learned pre-screen (at most one instance per context)
    int surr = -1;                 // instance with the pre-screen, or -1
    int surr_K = 0, surr_warmup = 0, surr_cells = 0, surr_Nc = 0, surr_Ncp = 0;
    void* kcand = nullptr;
    void* kcandf = nullptr;          // one-wave-per-cell candidate features (stages <= 32)
    int cand_sm = 0, cand_rsb = 0;   // its stage tier and job-major row bytes
    int cand_waves = 16;             // its waves per workgroup (cells per workgroup)
    size_t o_pJ = 0;
    size_t o_w = 0, o_wb = 0, o_m = 0, o_v = 0, o_g = 0;
    size_t o_Xall = 0, o_H1all = 0, o_H2all = 0, o_yall = 0, o_Tall = 0, o_choice = 0;
    size_t o_idx = 0, o_Xb = 0, o_tb = 0, o_H1b = 0, o_H2b = 0, o_yb = 0, o_dy = 0, o_dZ2 = 0, o_dZ1 = 0;
    size_t o_part = 0, o_cpart = 0, o_dpart = 0, o_ringX = 0, o_ringT = 0;
    size_t o_adam = 0, o_bc = 0;     // Adam step count (int64) + its corrections; correction table
    // graph of one migration epoch (or a fixed chunk when nothing migrates)
    bool use_graphs = true;
    hipGraphExec_t epoch_exec = nullptr;
    int epoch_len = 0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used;
    double timed_ms = 0.0;
    long long timed_launches = 0;
};

namespace {

int fail(ffs_ctx* c, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIP_TRY(c, call)                                                                    \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) return fail((c), FFS_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Compute offsets of everything in the workspace (a pure function of the
// instances and the tile shape).
void layout(ffs_ctx* c)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al256(bytes);
        return o;
    };
    c->n_isl = 0;
    c->max_size = 0;
    c->any_ring = false;
    int mmax = 1, maxP = 1;
    for (auto& I : c->inst) {
        c->n_isl += (int)I.isl.size();
        mmax = std::max(mmax, I.mmax);
        maxP = std::max(maxP, I.maxP);
        if (I.cfg.topology == 1 && I.cfg.migration_interval >= 0) c->any_ring = true;
        for (auto& L : I.isl) c->max_size = std::max(c->max_size, L.size);
    }
    c->mm = round_mmax(mmax);
    c->ptb = (maxP <= 255) ? 1 : 2;
    // the context's mapping for instances without a tile of their own
    {
        long long total = 0;
        for (auto& I : c->inst)
            for (auto& L : I.isl) total += L.size;
        c->lane = c->mapping == 1 || (c->mapping < 0 && total >= kLaneAutoMin);
    }
    // each instance's tile: mapping (the lane mapping only where it can run)
    // and waves per workgroup, narrowed until its workgroup fits in LDS
    for (auto& I : c->inst) {
        const int want = I.tile_map >= 0 ? I.tile_map : (c->lane ? 1 : 0);
        I.map_eff = (want == 1 && I.lane_ok && c->mm <= 8 && I.cfg.surrogate_k <= 1) ? 1 : 0;
        I.wpb_eff = I.tile_wpb > 0 ? I.tile_wpb : c->wpb;
        for (;;) {
            I.lds = align16((size_t)I.S * ((size_t)I.n_pad * c->ptb + 4)) +
                    (size_t)I.wpb_eff * (I.map_eff ? I.lane_wlds : wave_lds_bytes(I.G, I.n_pad));
            if (I.lds <= (size_t)c->max_lds || I.wpb_eff == 1) break;
            I.wpb_eff >>= 1;
        }
    }
    // classes: instances with the same tile whose workgroups need LDS within
    // the same half-octave bucket (8 KB * sqrt(2)^b) share a launch sized for
    // the class, so small instances are not held to the occupancy of the
    // largest one
    std::vector<long long> keys;
    auto class_key = [](const HostInstance& I) {
        return ((long long)I.lds_bucket << 8) | ((long long)I.wpb_eff << 1) | I.map_eff;
    };
    for (auto& I : c->inst) {
        int b = 0;
        while ((size_t)(8192.0 * std::pow(1.41421356, (double)b)) < I.lds) ++b;
        I.lds_bucket = b;
        const long long k = class_key(I);
        if (std::find(keys.begin(), keys.end(), k) == keys.end()) keys.push_back(k);
    }
    std::sort(keys.begin(), keys.end(), std::greater<long long>());
    for (auto& I : c->inst) I.cls = (int)(std::find(keys.begin(), keys.end(), class_key(I)) - keys.begin());
    c->n_cls = (int)keys.size();
    // fold groups.  Launch chains: possible when a single class holds every
    // instance, no island is swept and no instance has the pre-screen (those
    // launches read the context-wide generation count); automatic from
    // 131072 individuals, where a generation needs more than one round of
    // resident waves and the other chain's next generation fills the last
    // round (a smaller generation only pays a second launch).  Islands
    // alternate between the chains in index order.  Several classes (at
    // most kMaxGroups, no swept island): one group per class.
    {
        bool can = true;
        int islands = 0;
        long long total = 0;
        for (auto& I : c->inst) {
            islands += (int)I.isl.size();
            if (I.cfg.surrogate_k > 1) can = false;
            for (auto& L : I.isl) {
                total += L.size;
                if (L.spec.kind == 0 && L.spec.sweep) can = false;
            }
        }
        const bool want = c->chains == 2 || (c->chains < 0 && total >= kChainAutoMin);
        c->nchain = (can && c->n_cls == 1 && islands >= 2 && want) ? 2 : 1;
        c->class_groups = can && c->n_cls > 1 && c->n_cls <= kMaxGroups;
        for (auto& I : c->inst)
            for (size_t x = 0; x < I.isl.size(); ++x) {
                auto& L = I.isl[x];
                L.chain = c->class_groups ? I.cls : ((c->nchain == 2) ? (int)(x % 2) : 0);
                L.rec = (c->nchain == 2) ? L.chain : 0;
            }
    }
    // work items: per island, chunks of (waves per block) x G chromosomes,
    // ordered by cost (n * S * count), largest first
    c->work.clear();
    c->pairs.clear();
    int isl_base = 0;
    for (size_t ii = 0; ii < c->inst.size(); ++ii) {
        auto& I = c->inst[ii];
        const int chunk = I.wpb_eff * (I.map_eff ? kWave : I.G);
        for (size_t x = 0; x < I.isl.size(); ++x) {
            for (int s0 = 0; s0 < I.isl[x].size; s0 += chunk) {
                WorkItem w;
                w.island = isl_base + (int)x;
                w.slot0 = s0;
                w.count = std::min(chunk, I.isl[x].size - s0);
                w.inst = (int)ii;
                c->work.push_back(w);
            }
        }
        const int H = (int)I.isl.size() / 2;
        if (I.cfg.topology != 2)
            for (int i = 0; i < H; ++i) c->pairs.push_back(PairDesc{isl_base + i, isl_base + i + H, (int)ii, 0});
        I.isl_base = isl_base;
        isl_base += (int)I.isl.size();
    }
    c->n_pairs = (int)c->pairs.size();
    // line-sweep islands (lane kernel, two waves: a torus of at most 16384
    // cells has anti-diagonals of at most 128)
    c->sweep.clear();
    c->sweep_diags = 0;
    c->sweep_lds = 0;
    for (size_t ii = 0; ii < c->inst.size(); ++ii) {
        const auto& I = c->inst[ii];
        for (size_t x = 0; x < I.isl.size(); ++x) {
            const auto& L = I.isl[x];
            if (L.spec.kind != 0 || !L.spec.sweep) continue;
            c->sweep.push_back(WorkItem{I.isl_base + (int)x, 0, L.size, (int)ii});
            c->sweep_diags = std::max(c->sweep_diags, L.spec.rows + L.spec.cols - 1);
            c->sweep_lds = std::max(c->sweep_lds, align16((size_t)I.S * ((size_t)I.n_pad * c->ptb + 4)) +
                                                      (size_t)kSweepWaves * I.lane_wlds);
        }
    }
    c->sweep_kern = c->sweep.empty() ? nullptr : pick_gen_lane(c->mm, c->ptb);
    // topology 2: the ring c0, p0, c1, p1, ... as a list of edges after the pairs
    c->max_edges = 0;
    for (size_t ii = 0; ii < c->inst.size(); ++ii) {
        auto& I = c->inst[ii];
        I.edge0 = (int)c->pairs.size();
        I.n_edges = 0;
        const int H = (int)I.isl.size() / 2;
        if (I.cfg.topology != 2 || H == 0) continue;
        const int L = 2 * H, edges = (L == 2) ? 1 : L;
        auto ring = [&](int q) { return I.isl_base + ((q % 2 == 0) ? q / 2 : H + q / 2); };
        for (int e = 0; e < edges; ++e) c->pairs.push_back(PairDesc{ring(e), ring((e + 1) % L), (int)ii, 0});
        I.n_edges = edges;
        c->max_edges = std::max(c->max_edges, edges);
    }
    auto chain_of = [&](const WorkItem& w) { return c->inst[w.inst].isl[w.island - c->inst[w.inst].isl_base].chain; };
    std::stable_sort(c->work.begin(), c->work.end(), [&](const WorkItem& a, const WorkItem& b) {
        const auto& A = c->inst[a.inst];
        const auto& B = c->inst[b.inst];
        if (A.cls != B.cls) return A.cls < B.cls;
        if (chain_of(a) != chain_of(b)) return chain_of(a) < chain_of(b);
        return (long long)A.n * A.S * a.count > (long long)B.n * B.S * b.count;
    });
    c->n_work = (int)c->work.size();
    c->chain_w0[0] = 0;
    c->chain_w0[1] = c->chain_w0[2] = c->n_work;
    if (c->nchain == 2) {
        for (int i = 0; i < c->n_work; ++i)
            if (chain_of(c->work[i]) == 1) {
                c->chain_w0[1] = i;
                break;
            }
        if (c->chain_w0[1] == c->n_work) {   // nothing in chain 1: one chain
            c->nchain = 1;
            for (auto& I : c->inst)
                for (auto& L : I.isl) L.chain = L.rec = 0;
        }
    }
    c->ngroup = c->class_groups ? c->n_cls : c->nchain;
    // one launch per class: its work range, LDS bytes and launch-count slots
    // (the first class's launch also carries the best-ever workgroup)
    c->cls_w0.assign(c->n_cls + 1, 0);
    c->cls_lds.assign(c->n_cls, 0);
    for (auto& w : c->work) c->cls_w0[c->inst[w.inst].cls + 1] += 1;
    for (int k = 0; k < c->n_cls; ++k) c->cls_w0[k + 1] += c->cls_w0[k];
    c->cls_kern.assign(c->n_cls, nullptr);
    c->cls_wpb.assign(c->n_cls, 1);
    for (auto& I : c->inst) {
        c->cls_lds[I.cls] = std::max(c->cls_lds[I.cls], I.lds);
        c->cls_kern[I.cls] = I.map_eff ? pick_gen_lane(c->mm, c->ptb) : pick_gen(c->mm, c->ptb);
        c->cls_wpb[I.cls] = I.wpb_eff;
    }
    // a class's launch can carry a best-ever workgroup (the first class's
    // always, every class's with one fold group per class), whose scratch is
    // dynamic LDS too
    for (int k = 0; k < c->n_cls; ++k)
        c->cls_lds[k] = std::max(c->cls_lds[k], fold_lds_bytes(64 * c->cls_wpb[k]));

    c->off_ctl = take(sizeof(Control));
    c->off_insts = take(sizeof(InstDesc) * c->inst.size());
    c->off_isls = take(sizeof(IslandDesc) * (size_t)c->n_isl);
    // reserve room for the finest tile (one wave per block) so that the
    // workspace size does not depend on the tile shape chosen at bind
    size_t max_work = 0;
    for (auto& I : c->inst)
        for (auto& L : I.isl) max_work += (size_t)((L.size + I.G - 1) / I.G);
    c->off_work = take(sizeof(WorkItem) * std::max<size_t>(1, max_work));
    c->max_work = (int)max_work;
    c->off_counts = take(sizeof(int) * (max_work + 16));
    c->off_stage = take(kStageBytes);
    c->off_pairs = take(sizeof(PairDesc) * std::max<size_t>(1, c->pairs.size()));
    c->off_sweep = take(sizeof(WorkItem) * std::max<size_t>(1, c->sweep.size()));
    c->lds_gen = 0;
    for (auto& I : c->inst) {
        I.off_pT = take((size_t)I.S * I.n_pad * c->ptb);
        I.off_best_perm = take((size_t)kChains * I.n_pad * 2);
        I.off_best_rec = take((size_t)kChains * 4 * sizeof(int));
        I.off_counters = take(2 * sizeof(long long));
        for (auto& L : I.isl) {
            for (int b = 0; b < 2; ++b) {
                L.off_genes[b] = take((size_t)L.size * I.n_pad * 2);
                L.off_mk[b] = take((size_t)L.size * sizeof(int));
            }
            L.off_genkey = take(16);
            L.off_minmax = take(16);
            L.off_sorted = take((size_t)L.size * sizeof(int));
            L.off_sortbest = take(sizeof(int));
        }
        c->lds_gen = std::max(c->lds_gen, I.lds);
    }
    for (size_t k = 0; k < c->cls_lds.size(); ++k) c->lds_gen = std::max(c->lds_gen, c->cls_lds[k]);
    c->lds_gen = std::max(c->lds_gen, c->sweep_lds);
    int R = 1;
    while (R * kSortThreads < c->max_size) R <<= 1;
    c->lds_sort = sort_lds_bytes(R);
    // learned pre-screen: parameters, scoring and training buffers, replay ring
    c->surr = -1;
    for (size_t ii = 0; ii < c->inst.size(); ++ii)
        if (c->inst[ii].cfg.surrogate_k > 1) c->surr = (int)ii;
    if (c->surr >= 0) {
        const auto& I = c->inst[c->surr];
        c->surr_K = I.cfg.surrogate_k;
        c->surr_warmup = I.cfg.surrogate_warmup;
        c->surr_cells = I.n_cells;
        c->surr_Nc = I.n_cells * c->surr_K;
        c->surr_Ncp = (c->surr_Nc + 127) / 128 * 128;
        const size_t Pn = kParams, Ncp = c->surr_Ncp, Bt = kBatch;
        c->o_w = take(Pn * 4);
        c->o_wb = take(Pn * 2);
        c->o_m = take(Pn * 4);
        c->o_v = take(Pn * 4);
        c->o_g = take(Pn * 4);
        c->o_Xall = take(Ncp * kFeat * 2);
        c->o_H1all = take(Ncp * kHidden * 2);
        c->o_H2all = take(Ncp * kHidden * 2);
        c->o_yall = take(Ncp * 4);
        c->o_Tall = take(Ncp * 4);
        c->o_choice = take((size_t)I.n_cells * 4);
        c->o_idx = take(Bt * 4);
        c->o_Xb = take(Bt * kFeat * 2);
        c->o_tb = take(Bt * 4);
        c->o_H1b = take(Bt * kHidden * 2);
        c->o_H2b = take(Bt * kHidden * 2);
        c->o_yb = take(Bt * 4);
        c->o_dy = take(Bt * 4);
        c->o_dZ2 = take(Bt * kHidden * 2);
        c->o_dZ1 = take(Bt * kHidden * 2);
        c->o_part = take((size_t)(kBatch / 128) * kHidden * kHidden * 4);
        c->o_cpart = take((size_t)(kBatch / 64) * 3 * kHidden * 4);
        c->o_dpart = take((size_t)(kBatch / 64) * 4);
        c->o_ringX = take((size_t)kRing * kFeat * 2);
        c->o_ringT = take((size_t)kRing * 4);
        c->o_adam = take(16);
        c->o_bc = take((size_t)kBcSteps * 8);
        // job-major processing times for the candidates' features
        c->cand_sm = I.S <= 8 ? 8 : (I.S <= 16 ? 16 : (I.S <= 20 ? 20 : (I.S <= 24 ? 24 : (I.S <= 32 ? 32 : 0))));
        c->cand_rsb = (c->cand_sm * c->ptb + 15) / 16 * 16;
        c->o_pJ = take((size_t)I.n * std::max(c->cand_rsb, 16));
    }
    c->total = off;
}

int check_bound(ffs_ctx* c)
{
    if (!c) return FFS_EINVAL;
    if (!c->bound) return fail(c, FFS_ESTATE, "workspace not bound");
    return FFS_OK;
}

int read_ctl(ffs_ctx* c, Control* out)
{
    HIP_TRY(c, hipMemcpyAsync(out, c->ws + c->off_ctl, sizeof(Control), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int check_faults(ffs_ctx* c)
{
    Control ctl;
    int rc = read_ctl(c, &ctl);
    if (rc) return rc;
    if (ctl.err & 2) return fail(c, FFS_EDEVICE, "decode kernel exceeded its step bound");
    return FFS_OK;
}

// One generation of every island (mode 0; mode 1: generation 0).  chain >= 0
// (a fold group, for the branches of a captured epoch) launches only that
// group's work: with two launch chains that chain's islands, chain 1 on the
// first auxiliary stream; with class groups that class, class k on auxiliary
// stream k - 1 (the caller forks and joins the streams).  chain < 0 launches
// everything: both chains in turn on the context's stream, or the classes
// side by side, forked and joined here.
int launch_generation(ffs_ctx* c, int mode, int chain = -1)
{
    const InstDesc* di = reinterpret_cast<const InstDesc*>(c->ws + c->off_insts);
    const IslandDesc* dl = reinterpret_cast<const IslandDesc*>(c->ws + c->off_isls);
    const WorkItem* dw = reinterpret_cast<const WorkItem*>(c->ws + c->off_work);
    Control* ctl = reinterpret_cast<Control*>(c->ws + c->off_ctl);
    int n_inst = (int)c->inst.size();
    int cnt_off = 0, extra = 0;
    const WorkItem* dwk = dw;
    void* args[] = {(void*)&di, (void*)&dl, (void*)&dwk, (void*)&ctl, (void*)&n_inst, (void*)&mode, (void*)&cnt_off,
                    (void*)&extra};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing && mode == 0) {
        while (c->ev_pool.size() < 2) {
            hipEvent_t e;
            HIP_TRY(c, hipEventCreate(&e));
            c->ev_pool.push_back(e);
        }
        e0 = c->ev_pool.back();
        c->ev_pool.pop_back();
        e1 = c->ev_pool.back();
        c->ev_pool.pop_back();
        HIP_TRY(c, hipEventRecord(e0, c->stream));
    }
    if (mode == 0 && c->nchain == 2) {
        // a launch per chain, each with one workgroup more than its work
        // items, which folds the chain's previous generation
        for (int ch = 0; ch < 2; ++ch) {
            if (chain >= 0 && ch != chain) continue;
            const int nw = c->chain_w0[ch + 1] - c->chain_w0[ch];
            extra = 1 + ch;
            cnt_off = ch == 0 ? 0 : (c->chain_w0[1] - c->chain_w0[0]) + 1;
            dwk = dw + c->chain_w0[ch];
            hipStream_t st = (chain == 1) ? c->aux[0] : c->stream;
            HIP_TRY(c, hipLaunchKernel(c->cls_kern[0], dim3((unsigned)(nw + 1)), dim3(64 * c->cls_wpb[0]), args,
                                       c->cls_lds[0], st));
        }
        if (e0) {
            HIP_TRY(c, hipEventRecord(e1, c->stream));
            c->ev_used.emplace_back(e0, e1);
        }
        return FFS_OK;
    }
    // one launch per class; the first has one workgroup more than work
    // items, which folds the previous generation into the best-ever records.
    // Classes touch disjoint islands, so with several of them the launches
    // after the first go to their own streams, forked from and joined back
    // into the context's stream (parallel branches when captured in a graph)
    // (with class groups every class's launch carries the workgroup that
    // folds its own group; a group >= 0 launches only that class, class k on
    // auxiliary stream k - 1, for the caller's epoch branches)
    const bool fork = chain < 0 && c->concurrent && c->n_cls > 1 && (int)c->aux.size() >= c->n_cls - 1;
    if (fork) HIP_TRY(c, hipEventRecord(c->fork_ev[0], c->stream));
    cnt_off = 0;
    for (int k = 0; k < c->n_cls; ++k) {
        const int nw = c->cls_w0[k + 1] - c->cls_w0[k];
        extra = (mode != 0) ? 0 : (c->class_groups ? 1 + k : (k == 0 ? 1 : 0));
        if (nw + (extra ? 1 : 0) == 0) continue;
        if (chain >= 0 && k != chain) {
            cnt_off += nw + (extra ? 1 : 0);
            continue;
        }
        dwk = dw + c->cls_w0[k];
        hipStream_t st = c->stream;
        if (chain >= 0 && k > 0) st = c->aux[k - 1];
        if (fork && k > 0) {
            st = c->aux[k - 1];
            HIP_TRY(c, hipStreamWaitEvent(st, c->fork_ev[0], 0));
        }
        HIP_TRY(c, hipLaunchKernel(c->cls_kern[k], dim3((unsigned)(nw + (extra ? 1 : 0))), dim3(64 * c->cls_wpb[k]),
                                   args, c->cls_lds[k], st));
        if (fork && k > 0) {
            HIP_TRY(c, hipEventRecord(c->fork_ev[k], st));
            HIP_TRY(c, hipStreamWaitEvent(c->stream, c->fork_ev[k], 0));
        }
        cnt_off += nw + (extra ? 1 : 0);
    }
    if (mode == 0 && !c->sweep.empty()) {
        // line sweep: anti-diagonal d of every line-sweep island, d in order
        const WorkItem* ds = reinterpret_cast<const WorkItem*>(c->ws + c->off_sweep);
        int smode = 2, diag = 0, none = 0;
        void* sargs[] = {(void*)&di, (void*)&dl, (void*)&ds, (void*)&ctl, (void*)&n_inst, (void*)&smode, (void*)&diag,
                         (void*)&none};
        for (diag = 0; diag < c->sweep_diags; ++diag)
            HIP_TRY(c, hipLaunchKernel(c->sweep_kern, dim3(1, (unsigned)c->sweep.size()), dim3(64 * kSweepWaves), sargs,
                                       c->sweep_lds, c->stream));
    }
    if (e0) {
        HIP_TRY(c, hipEventRecord(e1, c->stream));
        c->ev_used.emplace_back(e0, e1);
    }
    return FFS_OK;
}

// Folds the completed generation into the best-ever records if the next
// generation launch has not done so yet.
int flush_best(ffs_ctx* c)
{
    const InstDesc* di = reinterpret_cast<const InstDesc*>(c->ws + c->off_insts);
    const IslandDesc* dl = reinterpret_cast<const IslandDesc*>(c->ws + c->off_isls);
    Control* ctl = reinterpret_cast<Control*>(c->ws + c->off_ctl);
    hipLaunchKernelGGL(k_best_flush, dim3(1), dim3(256), 0, c->stream, di, dl, ctl, (int)c->inst.size(), c->ngroup);
    HIP_TRY(c, hipGetLastError());
    return FFS_OK;
}

int launch_migration(ffs_ctx* c, int force_inst)
{
    // migration rewrites rows of the completed generation: record its best first
    int frc = flush_best(c);
    if (frc) return frc;
    const InstDesc* di = reinterpret_cast<const InstDesc*>(c->ws + c->off_insts);
    const IslandDesc* dl = reinterpret_cast<const IslandDesc*>(c->ws + c->off_isls);
    const PairDesc* dp = reinterpret_cast<const PairDesc*>(c->ws + c->off_pairs);
    const Control* ctl = reinterpret_cast<const Control*>(c->ws + c->off_ctl);
    if (c->any_ring) {
        hipLaunchKernelGGL(k_mig_minmax, dim3(c->n_isl), dim3(256), 0, c->stream, di, dl, ctl, force_inst);
        hipLaunchKernelGGL(k_mig_ring, dim3(c->n_isl), dim3(256), 0, c->stream, di, dl, ctl, force_inst);
    }
    const int chunks = (c->max_size + kMigRows - 1) / kMigRows;
    hipLaunchKernelGGL(k_mig_sort, dim3(c->n_isl), dim3(kSortThreads), c->lds_sort, c->stream, di, dl, ctl, force_inst,
                       -1);
    if (c->n_pairs > 0)
        hipLaunchKernelGGL(k_mig_adapt, dim3(c->n_pairs, chunks), dim3(256), 0, c->stream, di, dl, dp, ctl,
                           force_inst);
    // topology 2: the edges of each ring in turn, each on the state the
    // previous edge left (re-sorted)
    for (size_t ii = 0; ii < c->inst.size(); ++ii) {
        const auto& I = c->inst[ii];
        if (I.n_edges == 0 || (force_inst >= 0 && force_inst != (int)ii)) continue;
        for (int e = 0; e < I.n_edges; ++e) {
            if (e > 0)
                hipLaunchKernelGGL(k_mig_sort, dim3(c->n_isl), dim3(kSortThreads), c->lds_sort, c->stream, di, dl, ctl,
                                   force_inst, (int)ii);
            hipLaunchKernelGGL(k_mig_adapt, dim3(1, chunks), dim3(256), 0, c->stream, di, dl, dp + I.edge0 + e, ctl,
                               force_inst);
        }
    }
    HIP_TRY(c, hipGetLastError());
    return FFS_OK;
}

void drop_graph(ffs_ctx* c)
{
    if (c->epoch_exec) (void)hipGraphExecDestroy(c->epoch_exec);
    c->epoch_exec = nullptr;
    c->epoch_len = 0;
}

// Common migration interval of every instance that migrates: >0 the
// interval, 0 when no instance migrates, -1 when the intervals differ.
int common_interval(const ffs_ctx* c)
{
    int I = 0;
    for (auto& x : c->inst) {
        if (x.isl.size() < 2 || x.cfg.migration_interval == 0) continue;
        if (I == 0) I = x.cfg.migration_interval;
        else if (I != x.cfg.migration_interval) return -1;
    }
    return I;
}

// Generation kernels of the classes (dynamic LDS limit of each) and the
// streams and events that run the classes side by side.
int prepare_classes(ffs_ctx* c)
{
    for (int k = 0; k < c->n_cls; ++k) {
        if (!c->cls_kern[k]) return fail(c, FFS_EUNSUPPORTED, "no kernel for %d machines", c->mm);
        HIP_TRY(c, hipFuncSetAttribute(c->cls_kern[k], hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_gen));
    }
    if (!c->sweep.empty()) {
        if (!c->sweep_kern) return fail(c, FFS_EUNSUPPORTED, "the line sweep needs at most 8 machines per stage");
        HIP_TRY(c, hipFuncSetAttribute(c->sweep_kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_gen));
    }
    while ((int)c->aux.size() < std::max(c->n_cls, c->nchain) - 1) {
        hipStream_t st = nullptr;
        HIP_TRY(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        c->aux.push_back(st);
    }
    while ((int)c->fork_ev.size() < std::max(c->n_cls, c->nchain)) {
        hipEvent_t e = nullptr;
        HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        c->fork_ev.push_back(e);
    }
    return FFS_OK;
}

// Upload the work list of the current tiles and size the LDS of the
// generation kernels for it.
int apply_tile(ffs_ctx* c)
{
    int max_lds = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    layout(c);
    if (c->lds_gen > (size_t)max_lds)
        return fail(c, FFS_EUNSUPPORTED, "a workgroup needs %zu bytes of LDS (limit %d)", c->lds_gen, max_lds);
    int rc = prepare_classes(c);
    if (rc) return rc;
    if (c->n_work)
        HIP_TRY(c, hipMemcpy(c->ws + c->off_work, c->work.data(), sizeof(WorkItem) * c->work.size(),
                             hipMemcpyHostToDevice));
    if (c->bound) {
        // new launch width: count launches afresh from the current generation
        // (its best individuals folded first), and the islands' chains
        rc = flush_best(c);
        if (rc) return rc;
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        std::vector<int> zeros(c->max_work + 16, 0);
        HIP_TRY(c, hipMemcpy(c->ws + c->off_counts, zeros.data(), zeros.size() * sizeof(int), hipMemcpyHostToDevice));
        const int base = c->gen;
        HIP_TRY(c, hipMemcpy(c->ws + c->off_ctl + offsetof(Control, base), &base, sizeof base, hipMemcpyHostToDevice));
        int bg[kMaxGroups];
        std::fill(bg, bg + kMaxGroups, base);
        HIP_TRY(c, hipMemcpy(c->ws + c->off_ctl + offsetof(Control, best_gen), bg, sizeof bg, hipMemcpyHostToDevice));
        int x = 0;
        for (auto& I : c->inst)
            for (auto& L : I.isl) {
                const int cr[2] = {L.chain, L.rec};
                HIP_TRY(c, hipMemcpy(c->ws + c->off_isls + sizeof(IslandDesc) * x + offsetof(IslandDesc, chain), cr,
                                     sizeof cr, hipMemcpyHostToDevice));
                ++x;
            }
    }
    drop_graph(c);
    return FFS_OK;
}

template <bool TA, bool TB, int EPI>
int gemm(ffs_ctx* c, const uint16_t* A, const uint16_t* B, int M, int N, int K, int lda, int ldb, float* Cf,
         uint16_t* Cb, int ldc, const float* bias, const uint16_t* mask, int splits)
{
    if (M % GBM || N % GBN || K % (GBK * splits))
        return fail(c, FFS_EINVAL, "gemm shape %dx%dx%d (splits %d) not tiled", M, N, K, splits);
    hipLaunchKernelGGL((k_gemm<TA, TB, EPI>), dim3(N / GBN, M / GBM, splits), dim3(256), 0, c->stream, A, B, M, N, K,
                       lda, ldb, Cf, Cb, ldc, bias, mask);
    return FFS_OK;
}

template <typename T>
T* at(ffs_ctx* c, size_t off) { return reinterpret_cast<T*>(c->ws + off); }

// y = MLP(X) for `rows` rows (multiple of 128; the output layer covers the
// first out_rows); H1, H2 receive the hidden activations; with K > 0 also
// choice[cell] = argmin over each cell's K consecutive rows.  out_rows = 0:
// the hidden layers only (training fuses the output layer with its gradient).
int mlp_forward(ffs_ctx* c, const uint16_t* X, int rows, uint16_t* H1, uint16_t* H2, float* y, int K, int* choice,
                int out_rows)
{
    const float* w = at<float>(c, c->o_w);
    const uint16_t* wb = at<uint16_t>(c, c->o_wb);
    int rc = gemm<false, true, EPI_BIAS_RELU_BF16>(c, X, wb + kP_W1, rows, kHidden, kFeat, kFeat, kFeat, nullptr, H1,
                                                   kHidden, w + kP_b1, nullptr, 1);
    if (rc) return rc;
    rc = gemm<false, true, EPI_BIAS_RELU_BF16>(c, H1, wb + kP_W2, rows, kHidden, kHidden, kHidden, kHidden, nullptr, H2,
                                               kHidden, w + kP_b2, nullptr, 1);
    if (rc) return rc;
    if (out_rows == 0) return FFS_OK;
    const int waves = (K > 0) ? out_rows / K : out_rows;
    hipLaunchKernelGGL(k_mlp_out, dim3((waves + 3) / 4), dim3(256), 0, c->stream, H2, wb + kP_w3, w + kP_b3,
                       K > 0 ? waves * K : out_rows, K, y, choice);
    return FFS_OK;
}

// Gradients of mean((y - t)^2) for `rows` rows of X into grad (parameter
// layout).  H1, H2, y, dZ2, dZ1 are the batch buffers unless given.  With
// `step` an Adam step follows: the step count advances on the device.
int mlp_gradients(ffs_ctx* c, const uint16_t* X, const float* t, int rows, float* grad, uint16_t* dZ2o,
                  uint16_t* dZ1o, bool step)
{
    if (rows < 128 || rows > kBatch || rows % 128) return fail(c, FFS_EINVAL, "rows must be a multiple of 128 in [128, %d]", kBatch);
    uint16_t* H1 = at<uint16_t>(c, c->o_H1b);
    uint16_t* H2 = at<uint16_t>(c, c->o_H2b);
    float* y = at<float>(c, c->o_yb);
    float* dy = at<float>(c, c->o_dy);
    uint16_t* dZ2 = dZ2o ? dZ2o : at<uint16_t>(c, c->o_dZ2);
    uint16_t* dZ1 = dZ1o ? dZ1o : at<uint16_t>(c, c->o_dZ1);
    const uint16_t* wb = at<uint16_t>(c, c->o_wb);
    float* part = at<float>(c, c->o_part);
    int rc = mlp_forward(c, X, rows, H1, H2, y, 0, nullptr, 0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_mlp_out_dz2, dim3(rows / 4), dim3(256), 0, c->stream, (const uint16_t*)H2, wb + kP_w3,
                       at<const float>(c, c->o_w) + kP_b3, t, rows, y, dy, dZ2);
    const int splits = rows / 128;
    rc = gemm<true, false, EPI_F32>(c, dZ2, H1, kHidden, kHidden, rows, kHidden, kHidden, part, nullptr, kHidden,
                                    nullptr, nullptr, splits);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sum_splits, dim3(kHidden * kHidden / 256), dim3(256), 0, c->stream, part, splits,
                       (size_t)kHidden * kHidden, grad + kP_W2);
    rc = gemm<false, false, EPI_MASK_BF16>(c, dZ2, wb + kP_W2, rows, kHidden, kHidden, kHidden, kHidden, nullptr, dZ1,
                                           kHidden, nullptr, H1, 1);
    if (rc) return rc;
    {
        // bias gradients and the output layer's weight gradient: column
        // sums of dy * H2, dZ2 and dZ1 in one launch, then their chunk sums
        Colsum3 cs;
        cs.X[0] = H2;
        cs.X[1] = dZ2;
        cs.X[2] = dZ1;
        cs.out[0] = grad + kP_w3;
        cs.out[1] = grad + kP_b2;
        cs.out[2] = grad + kP_b1;
        float* cpart = at<float>(c, c->o_cpart);
        float* dpart = at<float>(c, c->o_dpart);
        const int chunks = rows / 64;
        hipLaunchKernelGGL(k_colsum3, dim3(1, chunks, 3), dim3(256), 0, c->stream, cs, (const float*)dy, cpart, dpart);
        hipLaunchKernelGGL(k_colsum3_sum, dim3((3 * kHidden + 1 + 255) / 256), dim3(256), 0, c->stream, cs,
                           (const float*)cpart, chunks, (const float*)dpart, grad + kP_b3,
                           step ? at<long long>(c, c->o_adam) : nullptr, at<const float2>(c, c->o_bc), kBcSteps,
                           reinterpret_cast<float*>(c->ws + c->o_adam + 8));
    }
    rc = gemm<true, false, EPI_F32>(c, dZ1, X, kHidden, kFeat, rows, kHidden, kFeat, part, nullptr, kFeat, nullptr,
                                    nullptr, splits);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sum_splits, dim3(kHidden * kFeat / 256), dim3(256), 0, c->stream, part, splits,
                       (size_t)kHidden * kFeat, grad + kP_W1);
    HIP_TRY(c, hipGetLastError());
    return FFS_OK;
}

// One Adam step; the step count and its bias corrections were advanced by
// the gradients' column-sum kernel (mlp_gradients with `step` set).
int mlp_adam(ffs_ctx* c)
{
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, c->stream, at<float>(c, c->o_w),
                       at<float>(c, c->o_m), at<float>(c, c->o_v), at<const float>(c, c->o_g),
                       at<uint16_t>(c, c->o_wb), kParams, kLr, kBeta1, kBeta2, kEps,
                       reinterpret_cast<const float*>(c->ws + c->o_adam + 8));
    HIP_TRY(c, hipGetLastError());
    return FFS_OK;
}

// One training step after the last completed generation (read from the
// control block): a minibatch from the replay ring, gradients, Adam.
int surrogate_train(ffs_ctx* c)
{
    const auto& I = c->inst[c->surr];
    const Control* ctl = reinterpret_cast<const Control*>(c->ws + c->off_ctl);
    int* idx = at<int>(c, c->o_idx);
    hipLaunchKernelGGL(k_batch_idx, dim3((kBatch / 8 + 255) / 256), dim3(256), 0, c->stream, (uint64_t)I.seed,
                       (uint64_t)c->surr, ctl, c->surr_cells, kRing, kBatch, idx);
    hipLaunchKernelGGL(k_gather_batch, dim3(kBatch / 8), dim3(256), 0, c->stream, at<const uint16_t>(c, c->o_ringX),
                       at<const float>(c, c->o_ringT), (const int*)idx, kBatch, at<uint16_t>(c, c->o_Xb),
                       at<float>(c, c->o_tb));
    int rc = mlp_gradients(c, at<const uint16_t>(c, c->o_Xb), at<const float>(c, c->o_tb), kBatch,
                           at<float>(c, c->o_g), nullptr, nullptr, true);
    if (rc) return rc;
    return mlp_adam(c);
}

// Candidates of every cell for the next generation: features (and exact
// targets when Tout), predictions, and the chosen stream per cell.
int surrogate_score(ffs_ctx* c, float* Tout)
{
    const auto& I = c->inst[c->surr];
    const InstDesc* di = reinterpret_cast<const InstDesc*>(c->ws + c->off_insts);
    const IslandDesc* dl = reinterpret_cast<const IslandDesc*>(c->ws + c->off_isls);
    const Control* ctl = reinterpret_cast<const Control*>(c->ws + c->off_ctl);
    int inst = c->surr, Nc = c->surr_Nc;
    uint16_t* X = at<uint16_t>(c, c->o_Xall);
    if (!Tout && c->kcandf) {
        // features only: one wave per cell, up to 16 cells per workgroup
        int cells = c->surr_cells;
        const int wv = c->cand_waves;
        void* args[] = {(void*)&di, (void*)&dl, (void*)&inst, (void*)&ctl, (void*)&cells, (void*)&X};
        HIP_TRY(c, hipLaunchKernel(c->kcandf, dim3((cells + wv - 1) / wv), dim3(64 * wv), args,
                                   cand_lds_bytes(I.n, I.n_pad, c->cand_rsb, wv), c->stream));
    } else {
        const int per_block = I.wpb_eff * I.G;
        const int blocks = (c->surr_Nc + per_block - 1) / per_block;
        void* args[] = {(void*)&di, (void*)&dl, (void*)&inst, (void*)&ctl, (void*)&Nc, (void*)&X, (void*)&Tout};
        HIP_TRY(c, hipLaunchKernel(c->kcand, dim3(blocks), dim3(64 * I.wpb_eff), args, I.lds, c->stream));
    }
    return mlp_forward(c, X, c->surr_Ncp, at<uint16_t>(c, c->o_H1all), at<uint16_t>(c, c->o_H2all),
                       at<float>(c, c->o_yall), c->surr_K, at<int>(c, c->o_choice), c->surr_Nc);
}

// Decode `count` device rows of `perms` (int32 [count][n]) into out (int32 [count]).
int launch_eval(ffs_ctx* c, int inst, const int32_t* perms, int count, int32_t* out)
{
    const auto& I = c->inst[inst];
    const InstDesc* di = reinterpret_cast<const InstDesc*>(c->ws + c->off_insts) + inst;
    Control* ctl = reinterpret_cast<Control*>(c->ws + c->off_ctl);
    void* kl = I.lane_ok ? pick_eval_lane(c->mm, c->ptb) : nullptr;
    const bool lane = kl && (c->mapping == 1 || (c->mapping < 0 && count >= kLaneEvalAutoMin &&
                                                 I.S >= kLaneEvalMinStages));
    const int per_block = c->wpb * (lane ? kWave : I.G);
    const int blocks = (count + per_block - 1) / per_block;
    const size_t lds = align16((size_t)I.S * ((size_t)I.n_pad * c->ptb + 4)) +
                       (size_t)c->wpb * (lane ? I.lane_wlds_eval : wave_lds_bytes(I.G, I.n_pad));
    void* args[] = {(void*)&di, (void*)&perms, (void*)&count, (void*)&out, (void*)&ctl};
    HIP_TRY(c, hipLaunchKernel(lane ? kl : c->keval, dim3(blocks), dim3(64 * c->wpb), args, lds, c->stream));
    return FFS_OK;
}

// Waits for the decodes and turns the control block's flags into a status
// (clearing the invalid-row flag for the next call).
int eval_status(ffs_ctx* c, int inst)
{
    Control h;
    int rc = read_ctl(c, &h);
    if (rc) return rc;
    if (h.err & 2) return fail(c, FFS_EDEVICE, "decode kernel exceeded its step bound");
    if (h.err & 1) {
        h.err &= ~1;
        HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_ctl + offsetof(Control, err), &h.err, sizeof(int),
                                  hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        return fail(c, FFS_EINVAL, "some rows are not permutations of 0..%d (makespan -1)", c->inst[inst].n - 1);
    }
    return FFS_OK;
}

// ---- checkpoint image --------------------------------------------------------
// A flat byte string: header, then per instance the best-ever record, its
// permutation (n_pad uint16), the migration counters, and per island the
// genes (size * n_pad uint16) and makespans (size int32) of the current
// generation's buffers; then, with a pre-screen, the Adam step count, the
// FP32 parameters, both moments, the replay ring and the cells' choices.
constexpr uint64_t kCkptMagic = 0x3154504B43534646ull;   // "FFSCKPT1"

struct CkptHeader {
    uint64_t magic, fingerprint, bytes;
    int32_t generation, n_inst;
};

uint64_t fnv(uint64_t h, const void* p, size_t n)
{
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

// Fingerprint of everything that defines the trajectory (not the tile shape).
uint64_t fingerprint(const ffs_ctx* c)
{
    uint64_t h = 0xCBF29CE484222325ull;
    for (const auto& I : c->inst) {
        h = fnv(h, &I.n, sizeof I.n);
        h = fnv(h, &I.S, sizeof I.S);
        h = fnv(h, I.m.data(), I.m.size() * sizeof(int));
        h = fnv(h, I.p.data(), I.p.size() * sizeof(int));
        for (const auto& L : I.isl) {
            const ffs_island_spec& s = L.spec;
            const int32_t v[6] = {s.kind, s.rows, s.cols, L.size, s.selection, s.sweep};
            h = fnv(h, v, sizeof v);
            h = fnv(h, &s.p_c, sizeof s.p_c);
            h = fnv(h, &s.p_m, sizeof s.p_m);
        }
        const int32_t cv[4] = {I.cfg.migration_interval, I.cfg.topology, I.cfg.surrogate_k, I.cfg.surrogate_warmup};
        h = fnv(h, cv, sizeof cv);
        h = fnv(h, &I.cfg.theta, sizeof I.cfg.theta);
        h = fnv(h, &I.seed, sizeof I.seed);
    }
    return h;
}

size_t ckpt_bytes(const ffs_ctx* c)
{
    size_t b = sizeof(CkptHeader);
    for (const auto& I : c->inst) {
        b += (size_t)kChains * (4 * sizeof(int32_t) + (size_t)I.n_pad * 2) + 2 * sizeof(int64_t);
        for (const auto& L : I.isl) b += (size_t)L.size * I.n_pad * 2 + (size_t)L.size * 4;
    }
    if (c->surr >= 0)
        b += sizeof(int64_t) + (size_t)3 * kParams * 4 + (size_t)kRing * kFeat * 2 + (size_t)kRing * 4 +
             (size_t)c->surr_cells * 4;
    return b;
}

// The pieces of the image after the header, in order: device offset and
// bytes, and for rows of permutations (u16, n_pad per row) the genes per row,
// whose padding the image stores as zeros (kernels leave it undefined).
struct CkptPiece {
    size_t off, bytes;
    int n = 0, n_pad = 0;
    CkptPiece(size_t o, size_t b, int nn = 0, int np = 0) : off(o), bytes(b), n(nn), n_pad(np) {}
};

std::vector<CkptPiece> ckpt_pieces(const ffs_ctx* c)
{
    std::vector<CkptPiece> v;
    const int par = c->gen & 1;
    for (const auto& I : c->inst) {
        v.emplace_back(I.off_best_rec, (size_t)kChains * 4 * sizeof(int32_t));
        v.emplace_back(I.off_best_perm, (size_t)kChains * I.n_pad * 2, I.n, I.n_pad);
        v.emplace_back(I.off_counters, 2 * sizeof(int64_t));
        for (const auto& L : I.isl) {
            v.emplace_back(L.off_genes[par], (size_t)L.size * I.n_pad * 2, I.n, I.n_pad);
            v.emplace_back(L.off_mk[par], (size_t)L.size * 4);
        }
    }
    if (c->surr >= 0) {
        v.emplace_back(c->o_w, (size_t)kParams * 4);
        v.emplace_back(c->o_m, (size_t)kParams * 4);
        v.emplace_back(c->o_v, (size_t)kParams * 4);
        v.emplace_back(c->o_ringX, (size_t)kRing * kFeat * 2);
        v.emplace_back(c->o_ringT, (size_t)kRing * 4);
        v.emplace_back(c->o_choice, (size_t)c->surr_cells * 4);
        v.emplace_back(c->o_adam, sizeof(int64_t));   // Adam steps taken
    }
    return v;
}

bool migration_due(const ffs_ctx* c, int g)
{
    for (auto& I : c->inst)
        if (I.cfg.migration_interval > 0 && g % I.cfg.migration_interval == 0 && I.isl.size() >= 2) return true;
    return false;
}

}  // namespace

extern "C" {

int ffs_ctx_create(void* hip_stream, ffs_ctx** out)
{
    if (!out) return FFS_EINVAL;
    ffs_ctx* c = new (std::nothrow) ffs_ctx();
    if (!c) return FFS_ENOMEM;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) {
        delete c;
        return FFS_EDEVICE;
    }
    c->max_lds -= 256;   // the generation kernels' static LDS (generation number, wave minima)
    *out = c;
    return FFS_OK;
}

void ffs_ctx_destroy(ffs_ctx* c)
{
    if (!c) return;
    if (c->bound) (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto e : c->fork_ev) (void)hipEventDestroy(e);
    for (auto st : c->aux) (void)hipStreamDestroy(st);
    for (auto& pr : c->ev_used) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    delete c;
}

const char* ffs_last_error(const ffs_ctx* c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

int ffs_create_instance(ffs_ctx* c, int32_t n, int32_t S, const int32_t* machines, const int32_t* p,
                        const ffs_island_spec* islands, int32_t n_islands, const ffs_ga_config* cfg,
                        uint64_t seed, int32_t* out_id)
{
    if (!c) return FFS_EINVAL;
    if (c->bound) return fail(c, FFS_ESTATE, "instances must be created before the workspace is bound");
    if (!machines || !p || !islands || !cfg || !out_id) return fail(c, FFS_EINVAL, "null argument");
    if (n < 1) return fail(c, FFS_EINVAL, "n_jobs must be >= 1");
    if (S < 1 || S > kMaxStages) return fail(c, FFS_EINVAL, "n_stages must be in [1, %d]", kMaxStages);
    if (n > 4096) return fail(c, FFS_EUNSUPPORTED, "n_jobs above 4096 is outside this library's limits");
    if (n_islands < 1) return fail(c, FFS_EINVAL, "need at least one island");
    if (n_islands > 1 && (n_islands % 2) != 0) return fail(c, FFS_EINVAL, "island count must be even (pairs)");
    if (cfg->migration_interval < 0) return fail(c, FFS_EINVAL, "migration_interval must be >= 0");
    if (cfg->topology < 0 || cfg->topology > 2) return fail(c, FFS_EINVAL, "topology must be 0, 1 or 2");
    if (!(cfg->theta >= 0.0 && cfg->theta <= 1.0)) return fail(c, FFS_EINVAL, "theta must be in [0, 1]");
    HostInstance I;
    I.n = n;
    I.S = S;
    I.m.assign(machines, machines + S);
    I.p.assign(p, p + (size_t)n * S);
    I.mmax = 1;
    for (int k = 0; k < S; ++k) {
        if (I.m[k] < 1 || I.m[k] > kMaxMachines)
            return fail(c, FFS_EINVAL, "machines[%d] = %d outside [1, %d]", k, I.m[k], kMaxMachines);
        I.mmax = std::max(I.mmax, I.m[k]);
    }
    I.E = 0;
    I.maxP = 1;
    for (size_t i = 0; i < I.p.size(); ++i) {
        if (I.p[i] < 1 || I.p[i] > 65535) return fail(c, FFS_EINVAL, "p[%zu] = %d outside [1, 65535]", i, I.p[i]);
        I.E += I.p[i];
        I.maxP = std::max(I.maxP, I.p[i]);
    }
    int jb = 1;
    while ((1 << jb) < n) ++jb;
    I.jb = jb;
    if (I.E >= ((1ll << (32 - jb)) - 1))
        return fail(c, FFS_EUNSUPPORTED, "sum of processing times %lld too large for the packed key (limit %lld)",
                    I.E, (1ll << (32 - jb)) - 1);
    I.n_pad = (n + 31) & ~31;
    // chromosomes per wave: one lane per stage, capped so that a wave's
    // three LDS rows per chromosome stay within 32 KB
    I.G = std::min(kWave / S, std::max(1, 32768 / (2 * group_stride(I.n_pad))));
    for (int x = 0; x < n_islands; ++x) {
        const ffs_island_spec& sp = islands[x];
        HostIsland L;
        L.spec = sp;
        if (!(sp.p_c >= 0.0 && sp.p_c <= 1.0 && sp.p_m >= 0.0 && sp.p_m <= 1.0))
            return fail(c, FFS_EINVAL, "island %d: rates must be in [0, 1]", x);
        if (sp.kind == 0) {
            if (sp.rows < 3 || sp.cols < 3) return fail(c, FFS_EINVAL, "island %d: grid must be at least 3x3", x);
            if (sp.selection < 0 || sp.selection > 2)
                return fail(c, FFS_EINVAL, "island %d: selection must be 0, 1 or 2", x);
            if (sp.sweep != 0 && sp.sweep != 1) return fail(c, FFS_EINVAL, "island %d: sweep must be 0 or 1", x);
            if ((long long)sp.rows * sp.cols > 16384)
                return fail(c, FFS_EUNSUPPORTED, "island %d: more than 16384 individuals", x);
            L.size = sp.rows * sp.cols;
        } else if (sp.kind == 1) {
            if (sp.size < 2 || (sp.size % 2) != 0) return fail(c, FFS_EINVAL, "island %d: pseudo size must be even >= 2", x);
            if (sp.selection != 0) return fail(c, FFS_EINVAL, "island %d: selection applies to cellular islands", x);
            if (sp.sweep != 0) return fail(c, FFS_EINVAL, "island %d: the line sweep applies to cellular islands", x);
            if (sp.size > 16384) return fail(c, FFS_EUNSUPPORTED, "island %d: more than 16384 individuals", x);
            L.size = sp.size;
        } else {
            return fail(c, FFS_EINVAL, "island %d: kind must be 0 or 1", x);
        }
        I.isl.push_back(L);
    }
    I.cfg = *cfg;
    I.seed = seed;
    // lower bound max(max_k ceil(P_k / m_k), max_j sum_k p_jk), stage totals
    I.Pk.assign(S, 0);
    long long jobmax = 0;
    for (int j = 0; j < n; ++j) {
        long long sj = 0;
        for (int k = 0; k < S; ++k) {
            I.Pk[k] += I.p[(size_t)j * S + k];
            sj += I.p[(size_t)j * S + k];
        }
        jobmax = std::max(jobmax, sj);
    }
    I.LB = jobmax;
    I.msum = 0;
    for (int k = 0; k < S; ++k) {
        I.LB = std::max(I.LB, (I.Pk[k] + I.m[k] - 1) / I.m[k]);
        I.msum += I.m[k];
    }
    // lane mapping: the operators' rows of one child per wave, then the
    // decode's msum keys per lane, in LDS
    I.lane_wlds = lane_gen_wave_lds(I.n_pad, I.msum);
    I.lane_wlds_eval = lane_eval_wave_lds(n, I.msum);
    I.lane_ok = I.msum <= kLaneMaxMsum && I.mmax <= 8;
    for (int x = 0; x < n_islands; ++x) {
        if (!islands[x].sweep) continue;
        if (!I.lane_ok)
            return fail(c, FFS_EUNSUPPORTED, "island %d: the line sweep needs the lane mapping (at most 8 machines "
                        "per stage, at most %d in all)", x, kLaneMaxMsum);
        if (cfg->surrogate_k > 1) return fail(c, FFS_EUNSUPPORTED, "island %d: the line sweep has no pre-screen", x);
    }
    I.n_cells = 0;
    for (auto& L : I.isl) {
        L.cell_base = (L.spec.kind == 0) ? I.n_cells : -1;
        if (L.spec.kind == 0) I.n_cells += L.size;
    }
    if (cfg->surrogate_k < 0 || cfg->surrogate_k > 64) return fail(c, FFS_EINVAL, "surrogate_k must be in [0, 64]");
    if (cfg->surrogate_warmup < 0) return fail(c, FFS_EINVAL, "surrogate_warmup must be >= 0");
    if (cfg->surrogate_k > 1) {
        if (I.n_cells == 0) return fail(c, FFS_EINVAL, "the pre-screen needs a cellular island");
        if (!c->inst.empty()) return fail(c, FFS_EUNSUPPORTED, "the pre-screen needs a context with a single instance");
    }
    for (auto& x : c->inst)
        if (x.cfg.surrogate_k > 1) return fail(c, FFS_EUNSUPPORTED, "the pre-screen needs a context with a single instance");
    c->inst.push_back(I);
    *out_id = (int32_t)(c->inst.size() - 1);
    return FFS_OK;
}

int ffs_set_waves_per_block(ffs_ctx* c, int32_t waves)
{
    if (!c) return FFS_EINVAL;
    if (waves != 1 && waves != 2 && waves != 4 && waves != 8) return fail(c, FFS_EINVAL, "waves must be 1, 2, 4 or 8");
    if (!c->bound) {
        c->wpb = waves;
        return FFS_OK;
    }
    // bound: only the work list and the LDS size change; the workspace
    // layout reserves room for the finest tile
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int old = c->wpb;
    c->wpb = waves;
    int rc = apply_tile(c);
    if (rc) {
        c->wpb = old;
        (void)apply_tile(c);
        return rc;
    }
    return FFS_OK;
}

int ffs_set_mapping(ffs_ctx* c, int32_t mapping)
{
    if (!c) return FFS_EINVAL;
    if (mapping < -1 || mapping > 1) return fail(c, FFS_EINVAL, "mapping must be -1, 0 or 1");
    if (!c->bound) {
        c->mapping = mapping;
        return FFS_OK;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int old = c->mapping;
    c->mapping = mapping;
    int rc = apply_tile(c);
    if (rc) {
        c->mapping = old;
        (void)apply_tile(c);
        return rc;
    }
    return FFS_OK;
}

int ffs_set_chains(ffs_ctx* c, int32_t chains)
{
    if (!c) return FFS_EINVAL;
    if (chains != -1 && chains != 1 && chains != 2) return fail(c, FFS_EINVAL, "chains must be -1, 1 or 2");
    if (!c->bound) {
        c->chains = chains;
        return FFS_OK;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int old = c->chains;
    c->chains = chains;
    int rc = apply_tile(c);
    if (rc) {
        c->chains = old;
        (void)apply_tile(c);
        return rc;
    }
    return FFS_OK;
}

int ffs_get_chains(ffs_ctx* c, int32_t* used)
{
    if (!c || !used) return FFS_EINVAL;
    if (!c->inst.empty()) layout(c);
    *used = c->nchain;
    return FFS_OK;
}

int ffs_get_mapping(ffs_ctx* c, int32_t* used)
{
    if (!c || !used) return FFS_EINVAL;
    if (c->inst.empty()) return fail(c, FFS_ESTATE, "no instance created");
    if (!c->bound) layout(c);
    int lane = 0, stage = 0;
    for (const auto& I : c->inst) (I.map_eff ? lane : stage) += 1;
    *used = (lane && stage) ? 2 : (lane ? 1 : 0);
    return FFS_OK;
}

int ffs_set_instance_tile(ffs_ctx* c, int32_t inst, int32_t mapping, int32_t waves)
{
    if (!c) return FFS_EINVAL;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FFS_EINVAL, "no instance %d", inst);
    if (mapping < -1 || mapping > 1) return fail(c, FFS_EINVAL, "mapping must be -1, 0 or 1");
    if (waves != 0 && waves != 1 && waves != 2 && waves != 4 && waves != 8)
        return fail(c, FFS_EINVAL, "waves must be 0, 1, 2, 4 or 8");
    auto& I = c->inst[inst];
    if (!c->bound) {
        I.tile_map = mapping;
        I.tile_wpb = waves;
        return FFS_OK;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const int om = I.tile_map, ow = I.tile_wpb;
    I.tile_map = mapping;
    I.tile_wpb = waves;
    int rc = apply_tile(c);
    if (rc) {
        I.tile_map = om;
        I.tile_wpb = ow;
        (void)apply_tile(c);
        return rc;
    }
    return FFS_OK;
}

int ffs_set_concurrent(ffs_ctx* c, int32_t enable)
{
    if (!c) return FFS_EINVAL;
    if (c->bound) HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->concurrent = enable != 0;
    drop_graph(c);
    return FFS_OK;
}

int ffs_workspace_size(const ffs_ctx* cc, size_t* bytes)
{
    ffs_ctx* c = const_cast<ffs_ctx*>(cc);
    if (!c || !bytes) return FFS_EINVAL;
    if (c->inst.empty()) return fail(c, FFS_ESTATE, "no instance created");
    layout(c);
    *bytes = c->total;
    return FFS_OK;
}

int ffs_bind_workspace(ffs_ctx* c, void* dptr, size_t bytes)
{
    if (!c) return FFS_EINVAL;
    if (c->bound) return fail(c, FFS_ESTATE, "workspace already bound");
    if (c->inst.empty()) return fail(c, FFS_ESTATE, "no instance created");
    if (!dptr) return fail(c, FFS_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(dptr) % 256 != 0) return fail(c, FFS_EINVAL, "workspace must be 256-byte aligned");
    layout(c);
    if (bytes < c->total) return fail(c, FFS_ENOMEM, "workspace too small: %zu < %zu", bytes, c->total);
    const int max_lds = c->max_lds;
    if (c->lds_gen > (size_t)max_lds)
        return fail(c, FFS_EUNSUPPORTED, "instance needs %zu bytes of LDS per workgroup (limit %d)", c->lds_gen, max_lds);
    if (c->lds_sort > (size_t)max_lds)
        return fail(c, FFS_EUNSUPPORTED, "island sort needs %zu bytes of LDS (limit %d)", c->lds_sort, max_lds);
    c->keval = pick_eval(c->mm, c->ptb);
    if (!c->keval) return fail(c, FFS_EUNSUPPORTED, "no kernel for %d machines", c->mm);
    {
        int prc = prepare_classes(c);
        if (prc) return prc;
    }
    HIP_TRY(c, hipFuncSetAttribute(c->keval, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds));
    if (void* kl = pick_eval_lane(c->mm, c->ptb))
        HIP_TRY(c, hipFuncSetAttribute(kl, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds));
    HIP_TRY(c, hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mig_sort),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_sort));
    c->ws = reinterpret_cast<char*>(dptr);
    c->ws_bytes = bytes;

    // host images of the descriptors and per-instance tables
    std::vector<InstDesc> hi(c->inst.size());
    std::vector<IslandDesc> hl;
    int isl_base = 0;
    for (size_t ii = 0; ii < c->inst.size(); ++ii) {
        auto& I = c->inst[ii];
        InstDesc d;
        memset(&d, 0, sizeof d);
        d.pT = c->ws + I.off_pT;
        d.best_perm = reinterpret_cast<uint16_t*>(c->ws + I.off_best_perm);
        d.best_rec = reinterpret_cast<int*>(c->ws + I.off_best_rec);
        d.counters = reinterpret_cast<long long*>(c->ws + I.off_counters);
        d.seed = I.seed;
        d.theta_T = rate_threshold(I.cfg.theta);
        d.E = I.E;
        d.inst_id = (int)ii;
        d.n = I.n;
        d.S = I.S;
        d.n_pad = I.n_pad;
        d.jb = I.jb;
        d.G = I.G;
        key_shifts(I.jb, I.LB, I.E, d.fsh, d.psh);
        d.island0 = isl_base;
        d.n_islands = (int)I.isl.size();
        d.interval = (I.isl.size() >= 2) ? I.cfg.migration_interval : 0;
        d.topology = I.cfg.topology;
        for (int k = 0; k < I.S; ++k) {
            d.mach[k] = I.m[k];
            d.Pk[k] = (int)I.Pk[k];
        }
        d.LB = (int)I.LB;
        d.msum = I.msum;
        d.lane_wlds = (int)I.lane_wlds;
        d.lane_wlds_eval = (int)I.lane_wlds_eval;
        d.n_cells = I.n_cells;
        d.surr_k = (c->surr == (int)ii) ? c->surr_K : 0;
        d.surr_warmup = I.cfg.surrogate_warmup;
        d.ring_size = kRing;
        if (c->surr == (int)ii) {
            d.surr_choice = reinterpret_cast<int*>(c->ws + c->o_choice);
            d.surr_X = reinterpret_cast<const uint16_t*>(c->ws + c->o_Xall);
            d.ring_X = reinterpret_cast<uint16_t*>(c->ws + c->o_ringX);
            d.ring_T = reinterpret_cast<float*>(c->ws + c->o_ringT);
            d.pJ = c->ws + c->o_pJ;
            d.pj_row_bytes = c->cand_rsb;
        }
        hi[ii] = d;
        for (size_t x = 0; x < I.isl.size(); ++x) {
            auto& L = I.isl[x];
            IslandDesc e;
            memset(&e, 0, sizeof e);
            for (int b = 0; b < 2; ++b) {
                e.genes[b] = reinterpret_cast<uint16_t*>(c->ws + L.off_genes[b]);
                e.mk[b] = reinterpret_cast<int*>(c->ws + L.off_mk[b]);
            }
            e.genkey = reinterpret_cast<unsigned long long*>(c->ws + L.off_genkey);
            e.minmax = reinterpret_cast<unsigned long long*>(c->ws + L.off_minmax);
            e.sorted = reinterpret_cast<int*>(c->ws + L.off_sorted);
            e.sortbest = reinterpret_cast<int*>(c->ws + L.off_sortbest);
            e.tc = rate_threshold(L.spec.p_c);
            e.tm = rate_threshold(L.spec.p_m);
            e.kind = L.spec.kind;
            e.rows = L.spec.kind == 0 ? L.spec.rows : 0;
            e.cols = L.spec.kind == 0 ? L.spec.cols : 0;
            e.size = L.size;
            e.inst = (int)ii;
            e.local = (int)x;
            e.cell_base = L.cell_base;
            e.sel = L.spec.kind == 0 ? L.spec.selection : 0;
            e.sweep = L.spec.kind == 0 ? L.spec.sweep : 0;
            e.chain = L.chain;
            e.rec = L.rec;
            hl.push_back(e);
        }
        isl_base += (int)I.isl.size();
    }
    Control ctl;
    memset(&ctl, 0, sizeof ctl);
    ctl.counts = reinterpret_cast<int*>(c->ws + c->off_counts);
    for (int gi = 0; gi < kMaxGroups; ++gi) ctl.best_gen[gi] = -1;
    {
        std::vector<int> zeros(c->max_work + 16, 0);
        HIP_TRY(c, hipMemcpy(c->ws + c->off_counts, zeros.data(), zeros.size() * sizeof(int), hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipMemcpy(c->ws + c->off_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->ws + c->off_insts, hi.data(), sizeof(InstDesc) * hi.size(), hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->ws + c->off_isls, hl.data(), sizeof(IslandDesc) * hl.size(), hipMemcpyHostToDevice));
    if (c->n_work)
        HIP_TRY(c, hipMemcpy(c->ws + c->off_work, c->work.data(), sizeof(WorkItem) * c->work.size(),
                             hipMemcpyHostToDevice));
    if (c->n_pairs)
        HIP_TRY(c, hipMemcpy(c->ws + c->off_pairs, c->pairs.data(), sizeof(PairDesc) * c->pairs.size(),
                             hipMemcpyHostToDevice));
    if (!c->sweep.empty())
        HIP_TRY(c, hipMemcpy(c->ws + c->off_sweep, c->sweep.data(), sizeof(WorkItem) * c->sweep.size(),
                             hipMemcpyHostToDevice));
    for (auto& I : c->inst) {
        // processing times, stage-major, padded rows
        std::vector<uint8_t> pt((size_t)I.S * I.n_pad * c->ptb, 0);
        for (int k = 0; k < I.S; ++k)
            for (int j = 0; j < I.n; ++j) {
                const int v = I.p[(size_t)j * I.S + k];
                if (c->ptb == 1) pt[(size_t)k * I.n_pad + j] = (uint8_t)v;
                else reinterpret_cast<uint16_t*>(pt.data())[(size_t)k * I.n_pad + j] = (uint16_t)v;
            }
        HIP_TRY(c, hipMemcpy(c->ws + I.off_pT, pt.data(), pt.size(), hipMemcpyHostToDevice));
        const int rec[4 * kChains] = {INT_MAX, -1, -1, -1, INT_MAX, -1, -1, -1};
        HIP_TRY(c, hipMemcpy(c->ws + I.off_best_rec, rec, sizeof rec, hipMemcpyHostToDevice));
        const long long cnt[2] = {0, 0};
        HIP_TRY(c, hipMemcpy(c->ws + I.off_counters, cnt, sizeof cnt, hipMemcpyHostToDevice));
        for (auto& L : I.isl) {
            const unsigned long long gk[2] = {~0ull, ~0ull};
            HIP_TRY(c, hipMemcpy(c->ws + L.off_genkey, gk, sizeof gk, hipMemcpyHostToDevice));
        }
    }
    if (c->surr >= 0) {
        c->kcand = pick_cand(c->mm, c->ptb);
        if (!c->kcand) return fail(c, FFS_EUNSUPPORTED, "no candidate kernel for %d machines", c->mm);
        HIP_TRY(c, hipFuncSetAttribute(c->kcand, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_gen));
        c->kcandf = pick_cand_features(c->cand_sm, c->ptb);
        if (c->kcandf) {
            const auto& I = c->inst[c->surr];
            c->cand_waves = 16;
            while (c->cand_waves > 1 && cand_lds_bytes(I.n, I.n_pad, c->cand_rsb, c->cand_waves) > (size_t)c->max_lds)
                c->cand_waves >>= 1;
            const size_t lds = cand_lds_bytes(I.n, I.n_pad, c->cand_rsb, c->cand_waves);
            if (lds > (size_t)c->max_lds) {
                c->kcandf = nullptr;
            } else {
                HIP_TRY(c, hipFuncSetAttribute(c->kcandf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
                // job-major table, rows of cand_sm entries, zero past the last stage
                std::vector<uint8_t> pj((size_t)I.n * c->cand_rsb, 0);
                for (int j = 0; j < I.n; ++j)
                    for (int k = 0; k < I.S; ++k) {
                        const int v = I.p[(size_t)j * I.S + k];
                        if (c->ptb == 1) pj[(size_t)j * c->cand_rsb + k] = (uint8_t)v;
                        else reinterpret_cast<uint16_t*>(pj.data() + (size_t)j * c->cand_rsb)[k] = (uint16_t)v;
                    }
                HIP_TRY(c, hipMemcpy(c->ws + c->o_pJ, pj.data(), pj.size(), hipMemcpyHostToDevice));
            }
        }
        hipLaunchKernelGGL(k_mlp_init, dim3((kParams + 255) / 256), dim3(256), 0, c->stream, (uint64_t)c->inst[c->surr].seed,
                           (uint64_t)c->surr, at<float>(c, c->o_w), at<uint16_t>(c, c->o_wb), at<float>(c, c->o_m),
                           at<float>(c, c->o_v));
        const size_t xw = (size_t)c->surr_Ncp * kFeat / 2;
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((xw + 255) / 256)), dim3(256), 0, c->stream,
                           at<uint32_t>(c, c->o_Xall), xw);
        hipLaunchKernelGGL(k_zero_u32, dim3((c->surr_cells + 255) / 256), dim3(256), 0, c->stream,
                           at<uint32_t>(c, c->o_choice), (size_t)c->surr_cells);
        // the replay ring starts empty (zeros, so that checkpoint images of
        // equal states are equal)
        const size_t rw = (size_t)kRing * kFeat / 2;
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((rw + 255) / 256)), dim3(256), 0, c->stream,
                           at<uint32_t>(c, c->o_ringX), rw);
        hipLaunchKernelGGL(k_zero_u32, dim3((kRing + 255) / 256), dim3(256), 0, c->stream,
                           at<uint32_t>(c, c->o_ringT), (size_t)kRing);
        // Adam: no steps taken; bias corrections of steps 1..kBcSteps
        std::vector<float> bct(2 * (size_t)kBcSteps);
        for (int t = 1; t <= kBcSteps; ++t) {
            bct[2 * (size_t)(t - 1)] = (float)(1.0 - std::pow((double)kBeta1, (double)t));
            bct[2 * (size_t)(t - 1) + 1] = (float)(1.0 - std::pow((double)kBeta2, (double)t));
        }
        if (bct[2 * (size_t)kBcSteps - 2] != 1.f || bct[2 * (size_t)kBcSteps - 1] != 1.f)
            return fail(c, FFS_EUNSUPPORTED, "Adam bias corrections are not 1 after %d steps", kBcSteps);
        HIP_TRY(c, hipMemcpy(c->ws + c->o_bc, bct.data(), bct.size() * 4, hipMemcpyHostToDevice));
        const int64_t zero16[2] = {0, 0};
        HIP_TRY(c, hipMemcpy(c->ws + c->o_adam, zero16, sizeof zero16, hipMemcpyHostToDevice));
        HIP_TRY(c, hipGetLastError());
    }
    c->bound = true;
    c->gen = 0;
    int rc = launch_generation(c, 1);
    if (rc) return rc;
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return check_faults(c);
}

int ffs_evaluate(ffs_ctx* c, int32_t inst, const int32_t* perms, int32_t count, int32_t* out)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FFS_EINVAL, "no instance %d", inst);
    if (count < 0) return fail(c, FFS_EINVAL, "count must be >= 0");
    if (count == 0) return FFS_OK;
    if (!perms || !out) return fail(c, FFS_EINVAL, "null buffer");
    rc = launch_eval(c, inst, perms, count, out);
    if (rc) return rc;
    return eval_status(c, inst);
}

int ffs_evaluate_host(ffs_ctx* c, int32_t inst, const int32_t* perms, int32_t count, int32_t* out)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FFS_EINVAL, "no instance %d", inst);
    if (count < 0) return fail(c, FFS_EINVAL, "count must be >= 0");
    if (count == 0) return FFS_OK;
    if (!perms || !out) return fail(c, FFS_EINVAL, "null buffer");
    const int n = c->inst[inst].n;
    // rows per chunk: n int32 in, one int32 out, within the staging region
    const size_t row_bytes = (size_t)n * 4 + 4;
    const int chunk = (int)std::min<size_t>((size_t)count, (kStageBytes - 256) / row_bytes);
    int32_t* dperm = reinterpret_cast<int32_t*>(c->ws + c->off_stage);
    int32_t* dout = reinterpret_cast<int32_t*>(c->ws + c->off_stage + al256((size_t)chunk * n * 4));
    for (int r0 = 0; r0 < count; r0 += chunk) {
        const int rows = std::min(chunk, count - r0);
        HIP_TRY(c, hipMemcpyAsync(dperm, perms + (size_t)r0 * n, (size_t)rows * n * 4, hipMemcpyHostToDevice,
                                  c->stream));
        rc = launch_eval(c, inst, dperm, rows, dout);
        if (rc) return rc;
        HIP_TRY(c, hipMemcpyAsync(out + r0, dout, (size_t)rows * 4, hipMemcpyDeviceToHost, c->stream));
    }
    return eval_status(c, inst);
}

int ffs_evolve(ffs_ctx* c, int32_t generations)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (generations < 0) return fail(c, FFS_EINVAL, "generations must be >= 0");
    const int I = common_interval(c);
    // whole epochs replay one captured graph: the kernels read the generation
    // (and the pre-screen its Adam step) from device memory, so the same
    // graph serves every epoch; with the pre-screen only epochs past its
    // warm-up, where every generation scores candidates
    const bool graphs = c->use_graphs && !c->timing && c->stream != nullptr && I >= 0;
    const int L = (I > 0) ? I : 16;
    int left = generations;
    while (left > 0) {
        if (graphs && c->gen % L == 0 && left >= L && (c->surr < 0 || c->gen >= c->surr_warmup)) {
            if (!c->epoch_exec || c->epoch_len != L) {
                drop_graph(c);
                hipGraph_t graph = nullptr;
                HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
                int crc = FFS_OK;
                if (c->nchain == 2) {
                    // the chains' generations of the epoch as two branches
                    HIP_TRY(c, hipEventRecord(c->fork_ev[0], c->stream));
                    HIP_TRY(c, hipStreamWaitEvent(c->aux[0], c->fork_ev[0], 0));
                    for (int t = 0; t < L && crc == FFS_OK; ++t) {
                        crc = launch_generation(c, 0, 0);
                        if (crc == FFS_OK) crc = launch_generation(c, 0, 1);
                    }
                    HIP_TRY(c, hipEventRecord(c->fork_ev[1], c->aux[0]));
                    HIP_TRY(c, hipStreamWaitEvent(c->stream, c->fork_ev[1], 0));
                } else if (c->class_groups && c->concurrent && (int)c->aux.size() >= c->n_cls - 1) {
                    // each class's generations of the epoch as one branch
                    HIP_TRY(c, hipEventRecord(c->fork_ev[0], c->stream));
                    for (int k = 1; k < c->n_cls; ++k) HIP_TRY(c, hipStreamWaitEvent(c->aux[k - 1], c->fork_ev[0], 0));
                    for (int t = 0; t < L && crc == FFS_OK; ++t)
                        for (int k = 0; k < c->n_cls && crc == FFS_OK; ++k) crc = launch_generation(c, 0, k);
                    for (int k = 1; k < c->n_cls; ++k) {
                        HIP_TRY(c, hipEventRecord(c->fork_ev[k], c->aux[k - 1]));
                        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->fork_ev[k], 0));
                    }
                } else {
                    for (int t = 0; t < L && crc == FFS_OK; ++t) {
                        if (c->surr >= 0) crc = surrogate_score(c, nullptr);
                        if (crc == FFS_OK) crc = launch_generation(c, 0);
                        if (crc == FFS_OK && c->surr >= 0) crc = surrogate_train(c);
                    }
                }
                if (crc == FFS_OK && I > 0) crc = launch_migration(c, -1);
                hipError_t ec = hipStreamEndCapture(c->stream, &graph);
                if (crc) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return crc;
                }
                if (ec != hipSuccess) return fail(c, FFS_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
                hipError_t ei = hipGraphInstantiate(&c->epoch_exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ei != hipSuccess) {
                    c->epoch_exec = nullptr;
                    return fail(c, FFS_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
                }
                c->epoch_len = L;
            }
            HIP_TRY(c, hipGraphLaunch(c->epoch_exec, c->stream));
            c->gen += L;
            left -= L;
            continue;
        }
        const int g = c->gen + 1;
        if (c->surr >= 0 && g > c->surr_warmup) {
            rc = surrogate_score(c, nullptr);     // choose the candidate each cell decodes
            if (rc) return rc;
        }
        rc = launch_generation(c, 0);
        if (rc) return rc;
        c->gen = g;
        if (c->surr >= 0) {
            rc = surrogate_train(c);
            if (rc) return rc;
        }
        if (migration_due(c, g)) {
            rc = launch_migration(c, -1);
            if (rc) return rc;
        }
        --left;
    }
    HIP_TRY(c, hipGetLastError());
    return FFS_OK;
}

int ffs_migrate(ffs_ctx* c, int32_t inst)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FFS_EINVAL, "no instance %d", inst);
    if (c->inst[inst].isl.size() < 2) return FFS_OK;
    return launch_migration(c, inst);
}

int ffs_best(ffs_ctx* c, int32_t inst, int32_t* out_mk, int32_t* out_gen, int32_t* out_perm)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FFS_EINVAL, "no instance %d", inst);
    const auto& I = c->inst[inst];
    rc = flush_best(c);
    if (rc) return rc;
    // the chains' records: the better by (makespan, generation, island, slot)
    int rec[4 * kChains];
    std::vector<uint16_t> perm((size_t)kChains * I.n_pad);
    HIP_TRY(c, hipMemcpyAsync(rec, c->ws + I.off_best_rec, sizeof rec, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(perm.data(), c->ws + I.off_best_perm, perm.size() * 2, hipMemcpyDeviceToHost, c->stream));
    rc = check_faults(c);
    if (rc) return rc;
    int b = 0;
    for (int ch = 1; ch < kChains; ++ch) {
        const int* x = rec + 4 * ch;
        const int* y = rec + 4 * b;
        if (std::lexicographical_compare(x, x + 4, y, y + 4)) b = ch;
    }
    if (out_mk) *out_mk = rec[4 * b];
    if (out_gen) *out_gen = rec[4 * b + 1];
    if (out_perm)
        for (int j = 0; j < I.n; ++j) out_perm[j] = perm[(size_t)b * I.n_pad + j];
    return FFS_OK;
}

int ffs_get_population(ffs_ctx* c, int32_t inst, int32_t island, int32_t* genes, int32_t* mk)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FFS_EINVAL, "no instance %d", inst);
    const auto& I = c->inst[inst];
    if (island < 0 || island >= (int)I.isl.size()) return fail(c, FFS_EINVAL, "no island %d", island);
    const auto& L = I.isl[island];
    const int par = c->gen & 1;
    std::vector<uint16_t> g;
    if (genes) {
        g.resize((size_t)L.size * I.n_pad);
        HIP_TRY(c, hipMemcpyAsync(g.data(), c->ws + L.off_genes[par], g.size() * 2, hipMemcpyDeviceToHost, c->stream));
    }
    if (mk) HIP_TRY(c, hipMemcpyAsync(mk, c->ws + L.off_mk[par], (size_t)L.size * 4, hipMemcpyDeviceToHost, c->stream));
    rc = check_faults(c);
    if (rc) return rc;
    if (genes)
        for (int s = 0; s < L.size; ++s)
            for (int j = 0; j < I.n; ++j) genes[(size_t)s * I.n + j] = g[(size_t)s * I.n_pad + j];
    return FFS_OK;
}

int ffs_generation(const ffs_ctx* c, int32_t* out)
{
    if (!c || !out) return FFS_EINVAL;
    *out = c->gen;
    return FFS_OK;
}

int ffs_migration_counters(ffs_ctx* c, int32_t inst, int64_t* migrations, int64_t* migrants)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FFS_EINVAL, "no instance %d", inst);
    long long v[2];
    HIP_TRY(c, hipMemcpyAsync(v, c->ws + c->inst[inst].off_counters, sizeof v, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (migrations) *migrations = v[0];
    if (migrants) *migrants = v[1];
    return FFS_OK;
}

int ffs_set_graphs(ffs_ctx* c, int32_t enable)
{
    if (!c) return FFS_EINVAL;
    c->use_graphs = enable != 0;
    if (!c->use_graphs) drop_graph(c);
    return FFS_OK;
}

int ffs_set_timing(ffs_ctx* c, int32_t enable)
{
    if (!c) return FFS_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& pr : c->ev_used) {
        c->ev_pool.push_back(pr.first);
        c->ev_pool.push_back(pr.second);
    }
    c->ev_used.clear();
    c->timing = enable != 0;
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    return FFS_OK;
}

int ffs_kernel_time(ffs_ctx* c, double* total_ms, int64_t* launches)
{
    if (!c) return FFS_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (auto& pr : c->ev_used) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, pr.first, pr.second));
        c->timed_ms += ms;
        c->timed_launches += 1;
        c->ev_pool.push_back(pr.first);
        c->ev_pool.push_back(pr.second);
    }
    c->ev_used.clear();
    if (total_ms) *total_ms = c->timed_ms;
    if (launches) *launches = c->timed_launches;
    return FFS_OK;
}

static int check_surr(ffs_ctx* c, int32_t inst)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (inst < 0 || inst >= (int)c->inst.size()) return fail(c, FFS_EINVAL, "no instance %d", inst);
    if (c->surr != inst) return fail(c, FFS_EINVAL, "instance %d has no pre-screen", inst);
    return FFS_OK;
}

int ffs_surrogate_params(ffs_ctx* c, int32_t inst, float* host)
{
    int rc = check_surr(c, inst);
    if (rc) return rc;
    if (!host) return fail(c, FFS_EINVAL, "null buffer");
    HIP_TRY(c, hipMemcpyAsync(host, c->ws + c->o_w, (size_t)kParams * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_surrogate_set_params(ffs_ctx* c, int32_t inst, const float* host)
{
    int rc = check_surr(c, inst);
    if (rc) return rc;
    if (!host) return fail(c, FFS_EINVAL, "null buffer");
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->o_w, host, (size_t)kParams * 4, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_to_bf16, dim3((kParams + 255) / 256), dim3(256), 0, c->stream, at<const float>(c, c->o_w),
                       at<uint16_t>(c, c->o_wb), kParams);
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_mlp_forward(ffs_ctx* c, int32_t inst, const uint16_t* X, int32_t rows, float* y, uint16_t* H1, uint16_t* H2)
{
    int rc = check_surr(c, inst);
    if (rc) return rc;
    if (!X || !y) return fail(c, FFS_EINVAL, "null buffer");
    if (rows < 128 || rows % 128) return fail(c, FFS_EINVAL, "rows must be a positive multiple of 128");
    if ((!H1 || !H2) && rows > kBatch) return fail(c, FFS_EINVAL, "give H1 and H2 for more than %d rows", kBatch);
    rc = mlp_forward(c, X, rows, H1 ? H1 : at<uint16_t>(c, c->o_H1b), H2 ? H2 : at<uint16_t>(c, c->o_H2b), y, 0,
                     nullptr, rows);
    if (rc) return rc;
    HIP_TRY(c, hipGetLastError());
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_mlp_gradients(ffs_ctx* c, int32_t inst, const uint16_t* X, const float* t, int32_t rows, float* grad,
                      uint16_t* dZ2, uint16_t* dZ1)
{
    int rc = check_surr(c, inst);
    if (rc) return rc;
    if (!X || !t || !grad) return fail(c, FFS_EINVAL, "null buffer");
    rc = mlp_gradients(c, X, t, rows, grad, dZ2, dZ1, false);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_mlp_train_step(ffs_ctx* c, int32_t inst, const uint16_t* X, const float* t, int32_t rows)
{
    int rc = check_surr(c, inst);
    if (rc) return rc;
    if (!X || !t) return fail(c, FFS_EINVAL, "null buffer");
    rc = mlp_gradients(c, X, t, rows, at<float>(c, c->o_g), nullptr, nullptr, true);
    if (rc) return rc;
    rc = mlp_adam(c);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_surrogate_candidates(ffs_ctx* c, int32_t inst, int32_t exact, uint16_t* X_host, float* pred_host,
                             float* exact_host, int32_t* choice_host)
{
    int rc = check_surr(c, inst);
    if (rc) return rc;
    rc = surrogate_score(c, exact ? at<float>(c, c->o_Tall) : nullptr);
    if (rc) return rc;
    const size_t Nc = (size_t)c->surr_Nc;
    if (X_host) HIP_TRY(c, hipMemcpyAsync(X_host, c->ws + c->o_Xall, Nc * kFeat * 2, hipMemcpyDeviceToHost, c->stream));
    if (pred_host) HIP_TRY(c, hipMemcpyAsync(pred_host, c->ws + c->o_yall, Nc * 4, hipMemcpyDeviceToHost, c->stream));
    if (exact_host && exact)
        HIP_TRY(c, hipMemcpyAsync(exact_host, c->ws + c->o_Tall, Nc * 4, hipMemcpyDeviceToHost, c->stream));
    if (choice_host)
        HIP_TRY(c, hipMemcpyAsync(choice_host, c->ws + c->o_choice, (size_t)c->surr_cells * 4, hipMemcpyDeviceToHost,
                                  c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_surrogate_choices(ffs_ctx* c, int32_t inst, int32_t* host)
{
    int rc = check_surr(c, inst);
    if (rc) return rc;
    if (!host) return fail(c, FFS_EINVAL, "null buffer");
    HIP_TRY(c, hipMemcpyAsync(host, c->ws + c->o_choice, (size_t)c->surr_cells * 4, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_surrogate_ring(ffs_ctx* c, int32_t inst, int32_t first, int32_t count, uint16_t* X_host, float* t_host)
{
    int rc = check_surr(c, inst);
    if (rc) return rc;
    if (first < 0 || count < 0 || first + count > kRing) return fail(c, FFS_EINVAL, "ring rows out of range");
    if (X_host)
        HIP_TRY(c, hipMemcpyAsync(X_host, c->ws + c->o_ringX + (size_t)first * kFeat * 2, (size_t)count * kFeat * 2,
                                  hipMemcpyDeviceToHost, c->stream));
    if (t_host)
        HIP_TRY(c, hipMemcpyAsync(t_host, c->ws + c->o_ringT + (size_t)first * 4, (size_t)count * 4,
                                  hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

int ffs_checkpoint_size(ffs_ctx* c, size_t* bytes)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (!bytes) return fail(c, FFS_EINVAL, "null argument");
    *bytes = ckpt_bytes(c);
    return FFS_OK;
}

int ffs_checkpoint_save(ffs_ctx* c, void* host, size_t bytes)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (!host) return fail(c, FFS_EINVAL, "null buffer");
    const size_t need = ckpt_bytes(c);
    if (bytes < need) return fail(c, FFS_EINVAL, "checkpoint buffer too small: %zu < %zu", bytes, need);
    // the records must include the current generation
    rc = flush_best(c);
    if (rc) return rc;
    unsigned char* out = static_cast<unsigned char*>(host);
    CkptHeader h;
    memset(&h, 0, sizeof h);
    h.magic = kCkptMagic;
    h.fingerprint = fingerprint(c);
    h.bytes = need;
    h.generation = c->gen;
    h.n_inst = (int32_t)c->inst.size();
    memcpy(out, &h, sizeof h);
    size_t pos = sizeof h;
    const auto pieces = ckpt_pieces(c);
    for (const auto& pc : pieces) {
        HIP_TRY(c, hipMemcpyAsync(out + pos, c->ws + pc.off, pc.bytes, hipMemcpyDeviceToHost, c->stream));
        pos += pc.bytes;
    }
    rc = check_faults(c);   // waits for the copies
    if (rc) return rc;
    pos = sizeof h;
    for (const auto& pc : pieces) {
        if (pc.n_pad > pc.n) {
            uint16_t* rows = reinterpret_cast<uint16_t*>(out + pos);
            for (size_t r = 0; r < pc.bytes / 2 / (size_t)pc.n_pad; ++r)
                std::fill(rows + r * pc.n_pad + pc.n, rows + (r + 1) * pc.n_pad, (uint16_t)0);
        }
        pos += pc.bytes;
    }
    return FFS_OK;
}

int ffs_checkpoint_load(ffs_ctx* c, const void* host, size_t bytes)
{
    int rc = check_bound(c);
    if (rc) return rc;
    if (!host) return fail(c, FFS_EINVAL, "null buffer");
    const size_t need = ckpt_bytes(c);
    CkptHeader h;
    if (bytes < sizeof h) return fail(c, FFS_EINVAL, "checkpoint too short");
    memcpy(&h, host, sizeof h);
    if (h.magic != kCkptMagic) return fail(c, FFS_EINVAL, "not a checkpoint image");
    if (h.fingerprint != fingerprint(c) || h.n_inst != (int32_t)c->inst.size())
        return fail(c, FFS_EINVAL, "checkpoint was taken from other instances");
    if (h.bytes != need || bytes < need) return fail(c, FFS_EINVAL, "checkpoint size %zu, expected %zu", bytes, need);
    if (h.generation < 0) return fail(c, FFS_EINVAL, "bad generation in checkpoint");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->gen = h.generation;
    const unsigned char* in = static_cast<const unsigned char*>(host);
    size_t pos = sizeof h;
    for (const auto& pc : ckpt_pieces(c)) {
        HIP_TRY(c, hipMemcpyAsync(c->ws + pc.off, in + pos, pc.bytes, hipMemcpyHostToDevice, c->stream));
        pos += pc.bytes;
    }
    if (c->surr >= 0) {
        hipLaunchKernelGGL(k_to_bf16, dim3((kParams + 255) / 256), dim3(256), 0, c->stream, at<const float>(c, c->o_w),
                           at<uint16_t>(c, c->o_wb), kParams);
        HIP_TRY(c, hipGetLastError());
    }
    // generation bookkeeping restarts at the loaded generation: no launches
    // counted, records already hold it, island minima empty
    std::vector<int> zeros(c->max_work + 16, 0);
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_counts, zeros.data(), zeros.size() * sizeof(int), hipMemcpyHostToDevice,
                              c->stream));
    Control ctl;
    HIP_TRY(c, hipMemcpyAsync(&ctl, c->ws + c->off_ctl, sizeof ctl, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    ctl.base = c->gen;
    for (int gi = 0; gi < kMaxGroups; ++gi) ctl.best_gen[gi] = c->gen;
    ctl.err = 0;
    HIP_TRY(c, hipMemcpyAsync(c->ws + c->off_ctl, &ctl, sizeof ctl, hipMemcpyHostToDevice, c->stream));
    const unsigned long long gk[2] = {~0ull, ~0ull};
    for (const auto& I : c->inst)
        for (const auto& L : I.isl)
            HIP_TRY(c, hipMemcpyAsync(c->ws + L.off_genkey, gk, sizeof gk, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return FFS_OK;
}

// ---- allocation-free decode ---------------------------------------------------
// The address of `scratch` on each device, taken once per device with that
// device current.
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};
}  // namespace

int ffs_evaluate_noalloc(void* hip_stream, int32_t n, int32_t S, const int32_t* machines, const int32_t* p,
                         const int32_t* perms, int32_t count, int32_t* out)
{
    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    if (!machines || !p) return FFS_EINVAL;
    if (n < 1 || n > 4096 || S < 1 || S > kMaxStages) return FFS_EINVAL;
    if (count < 0) return FFS_EINVAL;
    if (count > 0 && (!perms || !out)) return FFS_EINVAL;
    int mmax = 1, msum = 0, maxP = 1;
    for (int k = 0; k < S; ++k) {
        if (machines[k] < 1 || machines[k] > kMaxMachines) return FFS_EINVAL;
        mmax = std::max(mmax, machines[k]);
        msum += machines[k];
    }
    long long E = 0;
    for (long long i = 0; i < (long long)n * S; ++i) {
        if (p[i] < 1 || p[i] > 65535) return FFS_EINVAL;
        E += p[i];
        maxP = std::max(maxP, p[i]);
    }
    int jb = 1;
    while ((1 << jb) < n) ++jb;
    if (E >= ((1ll << (32 - jb)) - 1)) return FFS_EUNSUPPORTED;
    if (count == 0) return FFS_OK;
    const int n_pad = (n + 31) & ~31, ptb = maxP <= 255 ? 1 : 2;
    // scratch layout: control block, descriptor, processing times, table
    const size_t o_ctl = 0, o_desc = al256(sizeof(Control)), o_p = o_desc + al256(sizeof(InstDesc));
    const size_t o_pt = o_p + al256((size_t)n * S * 4);
    if (o_pt + (size_t)S * n_pad * ptb > kScratchBytes) return FFS_EUNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return FFS_EDEVICE;
    char* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_dev[dev]) {
            void* ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FFS_EDEVICE;
            g_scratch_dev[dev] = ptr;
        }
        base = static_cast<char*>(g_scratch_dev[dev]);
    }
    const int mm = round_mmax(mmax);
    InstDesc d;
    memset(&d, 0, sizeof d);
    d.pT = base + o_pt;
    d.n = n;
    d.S = S;
    d.n_pad = n_pad;
    d.jb = jb;
    {
        // lower bound: the longest job, and every stage's work over its machines
        long long LB = 0;
        for (int j = 0; j < n; ++j) {
            long long sj = 0;
            for (int k = 0; k < S; ++k) sj += p[(size_t)j * S + k];
            LB = std::max(LB, sj);
        }
        for (int k = 0; k < S; ++k) {
            long long pk = 0;
            for (int j = 0; j < n; ++j) pk += p[(size_t)j * S + k];
            LB = std::max(LB, (pk + machines[k] - 1) / machines[k]);
        }
        key_shifts(jb, LB, E, d.fsh, d.psh);
    }
    d.G = std::min(kWave / S, std::max(1, 32768 / (2 * group_stride(n_pad))));
    d.msum = msum;
    for (int k = 0; k < S; ++k) d.mach[k] = machines[k];
    d.lane_wlds_eval = (int)lane_eval_wave_lds(n, msum);
    // the automatic choice of ffs_evaluate at four waves per workgroup
    constexpr int wpb = 4;
    void* kl = (msum <= kLaneMaxMsum && mmax <= 8) ? pick_eval_lane(mm, ptb) : nullptr;
    const bool lane = kl && count >= kLaneEvalAutoMin && S >= kLaneEvalMinStages;
    void* kern = lane ? kl : pick_eval(mm, ptb);
    if (!kern) return FFS_EUNSUPPORTED;
    const size_t lds = align16((size_t)S * ((size_t)n_pad * ptb + 4)) +
                       (size_t)wpb * (lane ? (size_t)d.lane_wlds_eval : wave_lds_bytes(d.G, n_pad));
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return FFS_EDEVICE;
    if (lds > (size_t)max_lds) return FFS_EUNSUPPORTED;
    if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return FFS_EDEVICE;
    // the previous call's contents stay in scratch: descriptor, times and
    // table are rewritten, the error word cleared by a kernel
    if (hipMemcpyAsync(base + o_desc, &d, sizeof d, hipMemcpyHostToDevice, stream) != hipSuccess) return FFS_EDEVICE;
    if (hipMemcpyAsync(base + o_p, p, (size_t)n * S * 4, hipMemcpyHostToDevice, stream) != hipSuccess)
        return FFS_EDEVICE;
    uint32_t* ctlw = reinterpret_cast<uint32_t*>(base + o_ctl);
    const size_t ctl_words = sizeof(Control) / 4;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, stream, ctlw, ctl_words);
    hipLaunchKernelGGL(k_build_table, dim3((S * n_pad + 255) / 256), dim3(256), 0, stream,
                       reinterpret_cast<const int*>(base + o_p), n, S, n_pad, ptb, (void*)(base + o_pt));
    const InstDesc* di = reinterpret_cast<const InstDesc*>(base + o_desc);
    Control* ctl = reinterpret_cast<Control*>(base + o_ctl);
    const int per_block = wpb * (lane ? kWave : d.G);
    const int blocks = (count + per_block - 1) / per_block;
    void* args[] = {(void*)&di, (void*)&perms, (void*)&count, (void*)&out, (void*)&ctl};
    if (hipLaunchKernel(kern, dim3(blocks), dim3(64 * wpb), args, lds, stream) != hipSuccess) return FFS_EDEVICE;
    int err = 0;
    if (hipMemcpyAsync(&err, base + o_ctl + offsetof(Control, err), sizeof err, hipMemcpyDeviceToHost, stream) !=
        hipSuccess)
        return FFS_EDEVICE;
    if (hipStreamSynchronize(stream) != hipSuccess) return FFS_EDEVICE;
    if (err & 2) return FFS_EDEVICE;
    if (err & 1) return FFS_EINVAL;
    return FFS_OK;
}

}  // extern "C"
