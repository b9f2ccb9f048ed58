// Device helpers shared by the HIP sources of libdvm (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "dvm_internal.h"

namespace dvm {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

constexpr double kPi = 3.14159265358979323846;

// Sum N doubles over the workgroup; result valid in thread 0.  Fixed order.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double *lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < N; i++) v[i] += __shfl_xor(v[i], off, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < N; i++) lds[wv * N + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < N; i++) v[i] = ((lds[i] + lds[N + i]) + lds[2 * N + i]) + lds[3 * N + i];
    }
}

// Sum N doubles over the wave (xor butterfly: every lane ends with the same
// bits, the order is fixed).
template <int N>
__device__ __forceinline__ void wave_sum(double (&v)[N])
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < N; i++) v[i] += __shfl_xor(v[i], off, kWave);
    }
}

__device__ __forceinline__ double mJ_of(int objective, double v1, double v2)
{
    return objective == 0 ? v1 : 0.5 * (v1 * v1 + v2 * v2);
}

// Values that are the same in every lane of a wave (per-cell constants of a
// patch sweep), moved to scalar registers so that they do not occupy
// vector registers through the velocity loop.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
__device__ __forceinline__ double uni(double x)
{
    const long long v = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(v & 0xffffffffLL));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Workgroups are handed to the 8 XCDs round-robin; give each XCD a
// contiguous stretch of the sweep order (n items: cells or patches) so that
// the neighbour rows a workgroup reads were fetched moments before by a
// workgroup of the same XCD and are still in its L2.  Returns -1 for the
// padding workgroups of the last stretch.
__device__ __forceinline__ int xcd_item(int n, int b)
{
    const int per = (n + 7) >> 3;
    const int idx = (b & 7) * per + (b >> 3);
    return idx < n ? idx : -1;
}
static inline int xcd_grid(int n) { return ((n + 7) >> 3) << 3; }

// Instantiate for the storage type of a solve: float (mixed) or double (FP64).
#define DVM_DISPATCH(mixed, ...) \
    do {                          \
        if (mixed) {              \
            using T = float;      \
            __VA_ARGS__;          \
        } else {                  \
            using T = double;     \
            __VA_ARGS__;          \
        }                         \
    } while (0)

}  // namespace dvm
