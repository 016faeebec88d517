// ffs_mlp.h -- the learned pre-screen on gfx950: BF16 MLP 256-512-512-1 on
// MFMA with FP32 accumulation (forward, backward, Adam), its input features,
// and candidate selection.
//
// Storage: weights row-major [out][in] (W1 512x256, W2 512x512, w3 512) in
// BF16 for the products plus FP32 master copies; biases FP32; activations
// BF16 row-major [rows][512]; features BF16 [rows][256].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flowshop {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t gu32x4_t __attribute__((ext_vector_type(4)));

constexpr int kFeat = 256;
constexpr int kHidden = 512;

// FP32 -> BF16 bits, round to nearest even (finite values).
__device__ __forceinline__ uint16_t f32_to_bf16(float x)
{
    const uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---- tiled GEMM on MFMA ------------------------------------------------------
// C[M x N] = opA[M x K] * opB[K x N], BF16 operands, FP32 accumulation.
//   TA = false: A stored [M][K] (row stride lda);  true: stored [K][M].
//   TB = false: B stored [K][N] (row stride ldb);  true: stored [N][K].
// Block tile 128 x 128, K step 64, four waves of 64 x 64 (2 x 2 MFMA 32x32x16).
// v_mfma_f32_32x32x16_bf16 lane layout: lane l supplies row (l % 32) of A and
// column (l % 32) of B for k = 8 (l / 32) .. + 7; it receives column (l % 32)
// of D at rows 8 (r / 4) + 4 (l / 32) + r % 4, r = 0..15.
// Both operands sit in LDS k-contiguous per row ([i][k], [j][k]).  The next K
// tile is read from HBM into registers while the MFMAs run on the current
// one.  A K-contiguous operand is read as 16-byte rows (four per thread); an
// operand stored k-major ([K][M] or [K][N]) is read by half the workgroup as
// 8 x 8 blocks (eight 16-byte rows of k), transposed in registers with byte
// permutes and written as eight 16-byte rows of i.
// blockIdx.z splits K into gridDim.z equal ranges (EPI_F32 writes each
// split's partial product to its own M x N slice).
enum GemmEpi { EPI_F32 = 0, EPI_BIAS_RELU_BF16 = 1, EPI_MASK_BF16 = 2 };
constexpr int GBM = 128, GBN = 128, GBK = 64, GLD = GBK + 8;

// Transpose of an 8 x 8 block of 16-bit values: x[r] holds row r (element c
// in half c % 2 of word c / 2); y[c] receives column c.
__device__ __forceinline__ void transpose8x8_u16(const gu32x4_t (&x)[8], gu32x4_t (&y)[8])
{
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint32_t sel = (c & 1) ? 0x07060302u : 0x05040100u;
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            w[q] = __builtin_amdgcn_perm(x[2 * q + 1][c >> 1], x[2 * q][c >> 1], sel);
        }
        y[c] = gu32x4_t{w[0], w[1], w[2], w[3]};
    }
}

// One operand's share of a K tile, HBM -> registers -> LDS ([x][k] rows of
// GLD).  KM = false: the operand is k-contiguous per row, 1024 16-byte rows
// of 8 k, four per thread.  KM = true: stored k-major, one 8 x 8 block per
// thread of the half `half` of the workgroup, transposed in registers.
template <bool KM>
struct GemmStage {
    gu32x4_t r[KM ? 8 : 4];

    __device__ __forceinline__ void load(const uint16_t* __restrict__ X, int ld, int x0, int k0, int tid, int half)
    {
        if constexpr (!KM) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = tid + 256 * u, x = v >> 3, kk = (v & 7) * 8;
                r[u] = *reinterpret_cast<const gu32x4_t*>(&X[(size_t)(x0 + x) * ld + k0 + kk]);
            }
        } else {
            if ((tid >> 7) == half) {
                const int q = tid & 127, kb = (q & 7) * 8, xb = (q >> 3) * 8;
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    r[t] = *reinterpret_cast<const gu32x4_t*>(&X[(size_t)(k0 + kb + t) * ld + x0 + xb]);
            }
        }
    }

    __device__ __forceinline__ void store(uint16_t* Xs, int tid, int half) const
    {
        if constexpr (!KM) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int v = tid + 256 * u, x = v >> 3, kk = (v & 7) * 8;
                *reinterpret_cast<gu32x4_t*>(&Xs[x * GLD + kk]) = r[u];
            }
        } else {
            if ((tid >> 7) == half) {
                // eight consecutive threads fill the eight 16-byte k-chunks of
                // one LDS row: no bank conflicts
                const int q = tid & 127, kb = (q & 7) * 8, xb = (q >> 3) * 8;
                gu32x4_t y[8];
                transpose8x8_u16(r, y);
#pragma unroll
                for (int c = 0; c < 8; ++c) *reinterpret_cast<gu32x4_t*>(&Xs[(xb + c) * GLD + kb]) = y[c];
            }
        }
    }
};

template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_gemm(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
                                              int M, int N, int K, int lda, int ldb, float* __restrict__ Cf,
                                              uint16_t* __restrict__ Cb, int ldc, const float* __restrict__ bias,
                                              const uint16_t* __restrict__ mask)
{
    __shared__ __align__(16) uint16_t As[GBM * GLD];
    __shared__ __align__(16) uint16_t Bs[GBN * GLD];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int bm = blockIdx.y * GBM, bn = blockIdx.x * GBN;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    const int ks = K / gridDim.z, kbeg = blockIdx.z * ks, kend = kbeg + ks;
    f32x16_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

    // the mask of this thread's outputs, read before the K loop so that its
    // latency hides behind the MFMAs
    uint32_t mk[EPI == EPI_MASK_BF16 ? 64 : 1];
    if constexpr (EPI == EPI_MASK_BF16) {
#pragma unroll
        for (int ti = 0; ti < 2; ++ti)
#pragma unroll
            for (int tj = 0; tj < 2; ++tj)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int i = bm + wm + ti * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    const int j = bn + wn + tj * 32 + (lane & 31);
                    mk[(ti * 2 + tj) * 16 + r] = mask[(size_t)i * ldc + j];
                }
    }
    // k-major operands: A by threads 0..127, B by threads 128..255
    GemmStage<TA> sa;
    GemmStage<!TB> sb;
    sa.load(A, lda, bm, kbeg, tid, 0);
    sb.load(B, ldb, bn, kbeg, tid, 1);
    sa.store(As, tid, 0);
    sb.store(Bs, tid, 1);
    __syncthreads();
    auto mfma_tile = [&]() {
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 16) {
            bf16x8_t a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = *reinterpret_cast<const bf16x8_t*>(&As[(wm + t * 32 + (lane & 31)) * GLD + kk + 8 * (lane >> 5)]);
                b[t] = *reinterpret_cast<const bf16x8_t*>(&Bs[(wn + t * 32 + (lane & 31)) * GLD + kk + 8 * (lane >> 5)]);
            }
#pragma unroll
            for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
        }
    };
    // every K tile but the last: the next one's HBM reads are in flight
    // during this one's MFMAs
    for (int k0 = kbeg; k0 + GBK < kend; k0 += GBK) {
        sa.load(A, lda, bm, k0 + GBK, tid, 0);
        sb.load(B, ldb, bn, k0 + GBK, tid, 1);
        __builtin_amdgcn_sched_barrier(0);   // issue the reads before the MFMAs
        mfma_tile();
        __syncthreads();
        sa.store(As, tid, 0);
        sb.store(Bs, tid, 1);
        __syncthreads();
    }
    mfma_tile();
    float* Cz = (EPI == EPI_F32) ? Cf + (size_t)blockIdx.z * M * ldc : nullptr;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = bm + wm + ti * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int j = bn + wn + tj * 32 + (lane & 31);
                const float v = acc[ti][tj][r];
                const size_t o = (size_t)i * ldc + j;
                if (EPI == EPI_F32) {
                    Cz[o] = v;
                } else if (EPI == EPI_BIAS_RELU_BF16) {
                    const float z = v + bias[j];
                    Cb[o] = f32_to_bf16(z > 0.f ? z : 0.f);
                } else {
                    Cb[o] = (bf16_to_f32((uint16_t)mk[(ti * 2 + tj) * 16 + r]) > 0.f) ? f32_to_bf16(v) : (uint16_t)0;
                }
            }
}

// sum of x[y * stride], y = 0 .. n - 1, added in that order; the reads of
// 16 terms are issued before their sums.
__device__ __forceinline__ float sum_strided(const float* __restrict__ x, size_t stride, int n)
{
    float s = 0.f;
    int y = 0;
    for (; y + 16 <= n; y += 16) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = x[(size_t)(y + u) * stride];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += v[u];
    }
    for (; y < n; ++y) s += x[(size_t)y * stride];
    return s;
}

// out[i] = sum over splits s of part[s][i]  (fixed order: deterministic)
__global__ void __launch_bounds__(256) k_sum_splits(const float* __restrict__ part, int splits, size_t count,
                                                    float* __restrict__ out)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    out[i] = sum_strided(part + i, count, splits);
}

// ---- output layer --------------------------------------------------------
// y[i] = H2[i] . w3 + b3, one wave per row (64 lanes x 8 columns).  With
// K > 0 (scoring) the wave then handles the K candidates of one cell and
// writes the index of the smallest prediction (ties: lowest index).
__global__ void __launch_bounds__(256) k_mlp_out(const uint16_t* __restrict__ H2, const uint16_t* __restrict__ w3,
                                                 const float* __restrict__ b3, int rows, int K,
                                                 float* __restrict__ y, int* __restrict__ choice)
{
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
    const int per = K > 0 ? K : 1;
    const int r0 = wave * per;
    if (r0 >= rows) return;
    const uint4 wv = *reinterpret_cast<const uint4*>(&w3[lane * 8]);
    const uint16_t* we = reinterpret_cast<const uint16_t*>(&wv);
    float best = 0.f;
    int bi = 0;
    for (int c = 0; c < per; ++c) {
        const uint4 hv = *reinterpret_cast<const uint4*>(&H2[(size_t)(r0 + c) * kHidden + lane * 8]);
        const uint16_t* he = reinterpret_cast<const uint16_t*>(&hv);
        float s = 0.f;
#pragma unroll
        for (int t = 0; t < 8; ++t) s += bf16_to_f32(he[t]) * bf16_to_f32(we[t]);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        s += b3[0];
        if (lane == 0) y[r0 + c] = s;
        if (c == 0 || s < best) {
            best = s;
            bi = c;
        }
    }
    if (K > 0 && lane == 0) choice[wave] = bi;
}

// ---- backward pieces -------------------------------------------------------
// Output layer and its gradient for training, one wave per row:
// y[i] = H2[i] . w3 + b3 (as k_mlp_out), dy[i] = 2 (y[i] - t[i]) / rows and
// dZ2[i][j] = bf16(dy[i] * w3[j]) where H2[i][j] > 0.
__global__ void __launch_bounds__(256) k_mlp_out_dz2(const uint16_t* __restrict__ H2, const uint16_t* __restrict__ w3,
                                                     const float* __restrict__ b3, const float* __restrict__ t,
                                                     int rows, float* __restrict__ y, float* __restrict__ dy,
                                                     uint16_t* __restrict__ dZ2)
{
    const int i = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63;
    if (i >= rows) return;
    const uint4 wv = *reinterpret_cast<const uint4*>(&w3[lane * 8]);
    const uint16_t* we = reinterpret_cast<const uint16_t*>(&wv);
    const uint4 hv = *reinterpret_cast<const uint4*>(&H2[(size_t)i * kHidden + lane * 8]);
    const uint16_t* he = reinterpret_cast<const uint16_t*>(&hv);
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) s += bf16_to_f32(he[q]) * bf16_to_f32(we[q]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    s += b3[0];
    const float d = 2.f * (s - t[i]) / (float)rows;
    if (lane == 0) {
        y[i] = s;
        dy[i] = d;
    }
    uint16_t o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (bf16_to_f32(he[q]) > 0.f) ? f32_to_bf16(d * bf16_to_f32(we[q])) : (uint16_t)0;
    *reinterpret_cast<uint4*>(&dZ2[(size_t)i * kHidden + lane * 8]) = *reinterpret_cast<const uint4*>(o);
}

// Column sums of three BF16 matrices [rows][512] in one launch, in two
// fixed-order stages (deterministic).  Block (0, y, m) sums rows
// [64 y, 64 y + 64) of matrix m: thread (r, g) adds rows 64 y + 16 r .. + 15
// for columns 8 g .. 8 g + 7 (16-byte reads), the four row groups are added
// in order through LDS, and part[y][m * 512 + j] receives the chunk's sum.
// Matrix 0 is weighted by dy[i]; block y of matrix 0 also writes
// dpart[y] = sum of dy over its rows.  k_colsum3_sum adds the chunks.
struct Colsum3 {
    const uint16_t* X[3];
    float* out[3];
};

__global__ void __launch_bounds__(256) k_colsum3(Colsum3 a, const float* __restrict__ dy, float* __restrict__ part,
                                                 float* __restrict__ dpart)
{
    __shared__ float red[4][kHidden];
    const int m = blockIdx.z, y = blockIdx.y;
    const int r = threadIdx.x >> 6, g = threadIdx.x & 63;
    const uint16_t* X = a.X[m];
    float acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = 0.f;
    const int i0 = y * 64 + r * 16;
    uint4 v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = *reinterpret_cast<const uint4*>(&X[(size_t)(i0 + u) * kHidden + 8 * g]);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const uint16_t* e = reinterpret_cast<const uint16_t*>(&v[u]);
        const float w = (m == 0) ? dy[i0 + u] : 1.f;
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] += (m == 0) ? bf16_to_f32(e[t]) * w : bf16_to_f32(e[t]);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) red[r][8 * g + t] = acc[t];
    __syncthreads();
    for (int j = threadIdx.x; j < kHidden; j += 256)
        part[(size_t)y * 3 * kHidden + m * kHidden + j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    if (m == 0 && threadIdx.x == 0) {
        float sd = 0.f;
        for (int u = 0; u < 64; ++u) sd += dy[y * 64 + u];
        dpart[y] = sd;
    }
}

// out_m[j] = sum over chunks y (in order) of part[y][m * 512 + j]; dsum =
// sum of dpart in order.  With step non-null (a training step follows) one
// thread also advances the Adam step count t kept in device memory (so a
// captured graph can replay training steps without the host knowing their
// number) and writes step t + 1's bias corrections 1 - beta^(t+1) to bc,
// from `table` (computed on the host in FP64 and rounded to FP32; entry t for
// t < steps, both exactly 1 beyond).
__global__ void __launch_bounds__(256) k_colsum3_sum(Colsum3 a, const float* __restrict__ part, int chunks,
                                                     const float* __restrict__ dpart, float* __restrict__ dsum,
                                                     long long* step, const float2* __restrict__ table, int steps,
                                                     float* __restrict__ bc)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 3 * kHidden) a.out[e / kHidden][e % kHidden] = sum_strided(part + e, (size_t)3 * kHidden, chunks);
    if (e == 3 * kHidden) {
        *dsum = sum_strided(dpart, 1, chunks);
        if (step) {
            const long long t = *step + 1;
            *step = t;
            const float2 b = (t <= steps) ? table[t - 1] : make_float2(1.f, 1.f);
            bc[0] = b.x;
            bc[1] = b.y;
        }
    }
}

// Adam (Kingma & Ba) on FP32 master weights; writes the BF16 copy when given.
// One Adam step on every parameter with the bias corrections bc[0] =
// 1 - beta1^t, bc[1] = 1 - beta2^t of step t, which k_colsum3_sum looked up
// when it advanced the step count kept in device memory.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, uint16_t* __restrict__ wb, int count,
                                              float lr, float beta1, float beta2, float eps,
                                              const float* __restrict__ bc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float bc1 = bc[0], bc2 = bc[1];
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f32_to_bf16(wi);
}

__global__ void __launch_bounds__(256) k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) y[i] = f32_to_bf16(x[i]);
}

// Minibatch gather: rows idx_b (Philox stream of the training step) of the
// replay ring into contiguous X / t.
__global__ void __launch_bounds__(256) k_gather_batch(const uint16_t* __restrict__ ringX,
                                                      const float* __restrict__ ringT, const int* __restrict__ idx,
                                                      int rows, uint16_t* __restrict__ X, float* __restrict__ t)
{
    const int r = blockIdx.x * 8 + (threadIdx.x >> 5), lane = threadIdx.x & 31;   // 32 lanes x 8 features
    if (r >= rows) return;
    const int src = idx[r];
    *reinterpret_cast<uint4*>(&X[(size_t)r * kFeat + lane * 8]) =
        *reinterpret_cast<const uint4*>(&ringX[(size_t)src * kFeat + lane * 8]);
    if (lane == 0) t[r] = ringT[src];
}

}  // namespace flowshop
