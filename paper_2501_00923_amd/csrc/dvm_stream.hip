// Streaming reference kernels for the roofline of the sweeps (gfx950):
// plain HBM streams with the read/write mixes of the sweeps, 16-byte loads
// per lane as the sweeps move their rows, stores plain or non-temporal,
// grid-stride or one-pass launches of 256-thread workgroups, timed with HIP
// events on the caller's stream.  Measurement infrastructure only: nothing
// in libdvm calls it.
//
//   kind 0: c = a         (1 read + 1 write: the primal sweep's own-row mix)
//   kind 1: c = a + b     (2 reads + 1 write: the adjoint sweep's mix)
//   kind 2: c = 0         (write only)
//   kind 3: sum of a      (read only; one value per workgroup written)

#include <hip/hip_runtime.h>
#include <stddef.h>

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;

template <bool NT>
__device__ __forceinline__ void put(const f4 &v, f4 *p)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void k_stream_copy(const f4 *__restrict__ a, f4 *__restrict__ c, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kThreads * kUnroll;
    for (size_t i0 = (size_t)blockIdx.x * kThreads * kUnroll + threadIdx.x; i0 < n; i0 += stride) {
        f4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const size_t i = i0 + (size_t)u * kThreads;
            v[u] = i < n ? a[i] : f4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const size_t i = i0 + (size_t)u * kThreads;
            if (i < n) put<NT>(v[u], &c[i]);
        }
    }
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void k_stream_add(const f4 *__restrict__ a, const f4 *__restrict__ b,
                                                         f4 *__restrict__ c, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kThreads * kUnroll;
    for (size_t i0 = (size_t)blockIdx.x * kThreads * kUnroll + threadIdx.x; i0 < n; i0 += stride) {
        f4 v[kUnroll], w[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const size_t i = i0 + (size_t)u * kThreads;
            v[u] = i < n ? a[i] : f4{0, 0, 0, 0};
            w[u] = i < n ? b[i] : f4{0, 0, 0, 0};
        }
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const size_t i = i0 + (size_t)u * kThreads;
            if (i < n) put<NT>(v[u] + w[u], &c[i]);
        }
    }
}

template <bool NT>
__global__ __launch_bounds__(kThreads) void k_stream_fill(f4 *__restrict__ c, size_t n)
{
    const size_t stride = (size_t)gridDim.x * kThreads;
    for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
        put<NT>(f4{0, 0, 0, 0}, &c[i]);
}

__global__ __launch_bounds__(kThreads) void k_stream_read(const f4 *__restrict__ a, float *__restrict__ out, size_t n)
{
    __shared__ float red[kThreads];
    const size_t stride = (size_t)gridDim.x * kThreads * kUnroll;
    f4 s = {0, 0, 0, 0};
    for (size_t i0 = (size_t)blockIdx.x * kThreads * kUnroll + threadIdx.x; i0 < n; i0 += stride) {
#pragma unroll
        for (int u = 0; u < kUnroll; u++) {
            const size_t i = i0 + (size_t)u * kThreads;
            if (i < n) s += a[i];
        }
    }
    red[threadIdx.x] = s.x + s.y + s.z + s.w;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace

extern "C" {

// Time `iters` launches of stream kind `kind` over arrays of `bytes` bytes
// each (a multiple of 16; a, b: inputs, c: output; for kind 3, c holds
// `blocks` floats), `blocks` workgroups of 256 threads (0: one pass, a
// workgroup per 1024 16-byte elements), non-temporal stores if `nt`, after
// `warmup` launches; *ms receives the average time per launch.  Returns 0
// or a HIP error code.
int dvm_stream_time(int kind, const void *a, const void *b, void *c, size_t bytes, int blocks, int nt, int warmup,
                    int iters, void *hip_stream, float *ms)
{
    if (bytes % 16 || blocks < 0 || iters <= 0 || kind < 0 || kind > 3) return (int)hipErrorInvalidValue;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const size_t n = bytes / 16;
    if (blocks == 0) {
        const size_t one_pass = (n + (size_t)kThreads * kUnroll - 1) / ((size_t)kThreads * kUnroll);
        if (kind == 3 || one_pass > 0x7fffffff) return (int)hipErrorInvalidValue;
        blocks = (int)one_pass;
    }
    auto launch = [&]() {
        switch (kind) {
        case 0:
            if (nt)
                hipLaunchKernelGGL(k_stream_copy<true>, dim3(blocks), dim3(kThreads), 0, st,
                                   static_cast<const f4 *>(a), static_cast<f4 *>(c), n);
            else
                hipLaunchKernelGGL(k_stream_copy<false>, dim3(blocks), dim3(kThreads), 0, st,
                                   static_cast<const f4 *>(a), static_cast<f4 *>(c), n);
            break;
        case 1:
            if (nt)
                hipLaunchKernelGGL(k_stream_add<true>, dim3(blocks), dim3(kThreads), 0, st,
                                   static_cast<const f4 *>(a), static_cast<const f4 *>(b), static_cast<f4 *>(c), n);
            else
                hipLaunchKernelGGL(k_stream_add<false>, dim3(blocks), dim3(kThreads), 0, st,
                                   static_cast<const f4 *>(a), static_cast<const f4 *>(b), static_cast<f4 *>(c), n);
            break;
        case 2:
            if (nt)
                hipLaunchKernelGGL(k_stream_fill<true>, dim3(blocks), dim3(kThreads), 0, st, static_cast<f4 *>(c), n);
            else
                hipLaunchKernelGGL(k_stream_fill<false>, dim3(blocks), dim3(kThreads), 0, st, static_cast<f4 *>(c), n);
            break;
        default:
            hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(kThreads), 0, st, static_cast<const f4 *>(a),
                               static_cast<float *>(c), n);
        }
        return hipGetLastError();
    };
    for (int i = 0; i < warmup; i++)
        if (hipError_t e = launch()) return (int)e;
    hipEvent_t e0, e1;
    if (hipError_t e = hipEventCreate(&e0)) return (int)e;
    if (hipError_t e = hipEventCreate(&e1)) {
        (void)hipEventDestroy(e0);
        return (int)e;
    }
    hipError_t err = hipEventRecord(e0, st);
    for (int i = 0; i < iters && !err; i++) err = launch();
    if (!err) err = hipEventRecord(e1, st);
    if (!err) err = hipEventSynchronize(e1);
    float t = 0;
    if (!err) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!err) *ms = t / iters;
    return (int)err;
}

}  // extern "C"
