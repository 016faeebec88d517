// lds_probe.hip -- achievable LDS read bandwidth of the device (measurement
// helper of the benchmark, not part of the GA library).
//
// Every workgroup fills 32 KB of LDS, then each thread reads 16-byte vectors
// at consecutive addresses of its wave (a wave reads 1 KB contiguous per
// instruction: no bank conflicts), `iters` times, folding them into one word
// that is written out so the reads cannot be dropped.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeBytes = 32768;

__global__ void __launch_bounds__(kProbeThreads) k_lds_probe(int iters, int step, uint32_t* __restrict__ out)
{
    __shared__ __align__(16) uint32_t buf[kProbeBytes / 4];
    for (int i = threadIdx.x; i < kProbeBytes / 4; i += kProbeThreads) buf[i] = (uint32_t)(i * 2654435761u);
    __syncthreads();
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    // the address step is a run-time argument, so every read is issued
    // (the table does not change, and repeated addresses could otherwise be
    // served from registers)
    const u32x4* v = reinterpret_cast<const u32x4*>(buf);
    constexpr int nv = kProbeBytes / 16;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int idx = (wave * 64 + lane) & (nv - 1);
    uint32_t acc = 0u;
    for (int it = 0; it < iters; it += 4) {
        u32x4 x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = v[(idx + u * kProbeThreads) & (nv - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += x[u].x + x[u].y + x[u].z + x[u].w;
        idx = (idx + step) & (nv - 1);
    }
    out[blockIdx.x * kProbeThreads + threadIdx.x] = acc;
}

}  // namespace

// Runs `blocks` workgroups of 256 threads, each thread reading `iters`
// (a multiple of 4) 16-byte vectors, on `stream`; `out` is device scratch of
// blocks * 256 words.  Returns 0 and the kernel's time (HIP events) and the
// bytes read, or a HIP error code.
extern "C" int lds_probe(void* stream, int blocks, int iters, uint32_t* out, float* ms, double* bytes)
{
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return (int)e;
    e = hipEventCreate(&e1);
    if (e != hipSuccess) return (int)e;
    const int step = 4 * kProbeThreads + 64;   // a whole wave's worth: reads stay conflict-free
    hipLaunchKernelGGL(k_lds_probe, dim3(blocks), dim3(kProbeThreads), 0, st, iters, step, out);   // warm-up
    (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL(k_lds_probe, dim3(blocks), dim3(kProbeThreads), 0, st, iters, step, out);
    (void)hipEventRecord(e1, st);
    e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *bytes = (double)blocks * kProbeThreads * (double)iters * 16.0;
    return (int)e;
}
