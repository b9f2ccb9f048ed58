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

// Sum N doubles over each aligned group of G lanes (xor butterfly: every
// lane of a group ends with the same bits, the order is fixed).
template <int G, int N>
__device__ __forceinline__ void group_sum(double (&v)[N])
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int i = 0; i < N; i++) v[i] += __shfl_xor(v[i], off, G);
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

// Solve a 4x4 system A x = b (Gaussian elimination, partial pivoting; A and
// b are overwritten).  Called with the same values in every lane.
__device__ __forceinline__ void solve4(double (&A)[4][4], double (&b)[4], double (&x)[4])
{
#pragma unroll
    for (int col = 0; col < 4; col++) {
        int piv = col;
#pragma unroll
        for (int r = col + 1; r < 4; r++)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
#pragma unroll
        for (int r = 0; r < 4; r++)
            if (r == piv && r != col) {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const double t = A[col][k];
                    A[col][k] = A[r][k];
                    A[r][k] = t;
                }
                const double t = b[col];
                b[col] = b[r];
                b[r] = t;
            }
#pragma unroll
        for (int r = col + 1; r < 4; r++) {
            const double fct = A[r][col] / A[col][col];
#pragma unroll
            for (int k = col; k < 4; k++) A[r][k] -= fct * A[col][k];
            b[r] -= fct * b[col];
        }
    }
#pragma unroll
    for (int r = 3; r >= 0; r--) {
        double acc = b[r];
#pragma unroll
        for (int k = r + 1; k < 4; k++) acc -= A[r][k] * x[k];
        x[r] = acc / A[r][r];
    }
}

// Discrete-conservative equilibrium (the reading of the equilibrium on a
// discrete velocity grid): the parameters P = (rho, u1, u2, theta) of the
// reduced Maxwellian whose grid moments equal W.  Newton from the primitive
// variables of W, kEqNewton steps.  The Maxwellian factors as
// rho/(2 pi theta) X(v1) Y(v2) on the tensor grid, so each step needs only
// the 1-D sums R_p = sum_a wx_a X_a vx_a^p, T_p = sum_b wy_b Y_b vy_b^p
// (p <= 4), summed per lane and reduced across a group of G lanes (the
// wave, or a part of it that serves one cell) in a fixed order: every lane
// of the group ends with the same P.  Minv (may be null) receives
// (dm/dP)^{-1} = dP/dW at the final P, row q = parameter, column m = moment.
constexpr int kEqNewton = 6;

template <int G = kWave>
__device__ __forceinline__ void eq_moments_jac(const DevSolve &d, const double (&P)[4], double (&m)[4],
                                               double (&J)[4][4])
{
    const int lane = threadIdx.x % G;
    const double u1 = P[1], u2 = P[2], th = P[3], h = 0.5 / th;
    double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = lane; i < d.n1; i += G) {
        const double v = d.vx[i], e = v - u1, X = d.wx[i] * exp(-e * e * h);
        s[0] += X;
        s[1] += X * v;
        s[2] += X * v * v;
        s[3] += X * v * v * v;
        s[4] += X * v * v * v * v;
    }
    for (int i = lane; i < d.n2; i += G) {
        const double v = d.vy[i], e = v - u2, Y = d.wy[i] * exp(-e * e * h);
        s[5] += Y;
        s[6] += Y * v;
        s[7] += Y * v * v;
        s[8] += Y * v * v * v;
        s[9] += Y * v * v * v * v;
    }
    group_sum<G, 10>(s);
    const double *R = s, *T = s + 5;
    const double kap = P[0] / (2.0 * kPi * th);
    // d R_p / d u1 and d R_p / d theta (p = 0..2), likewise T with u2
    double Ru[3], Rt[3], Tu[3], Tt[3];
    const double i2t2 = 1.0 / (2.0 * th * th);
#pragma unroll
    for (int q = 0; q < 3; q++) {
        Ru[q] = (R[q + 1] - u1 * R[q]) / th;
        Tu[q] = (T[q + 1] - u2 * T[q]) / th;
        Rt[q] = (R[q + 2] - 2.0 * u1 * R[q + 1] + u1 * u1 * R[q]) * i2t2;
        Tt[q] = (T[q + 2] - 2.0 * u2 * T[q + 1] + u2 * u2 * T[q]) * i2t2;
    }
    const double b0 = R[0] * T[0], b1 = R[1] * T[0], b2 = R[0] * T[1];
    const double b3 = 0.5 * (R[2] * T[0] + R[0] * T[2]) + 0.5 * th * R[0] * T[0];
    m[0] = kap * b0;
    m[1] = kap * b1;
    m[2] = kap * b2;
    m[3] = kap * b3;
    // columns: rho, u1, u2, theta
    J[0][0] = m[0] / P[0];
    J[1][0] = m[1] / P[0];
    J[2][0] = m[2] / P[0];
    J[3][0] = m[3] / P[0];
    J[0][1] = kap * Ru[0] * T[0];
    J[1][1] = kap * Ru[1] * T[0];
    J[2][1] = kap * Ru[0] * T[1];
    J[3][1] = kap * (0.5 * (Ru[2] * T[0] + Ru[0] * T[2]) + 0.5 * th * Ru[0] * T[0]);
    J[0][2] = kap * R[0] * Tu[0];
    J[1][2] = kap * R[1] * Tu[0];
    J[2][2] = kap * R[0] * Tu[1];
    J[3][2] = kap * (0.5 * (R[2] * Tu[0] + R[0] * Tu[2]) + 0.5 * th * R[0] * Tu[0]);
    const double db0 = Rt[0] * T[0] + R[0] * Tt[0];
    J[0][3] = kap * (db0 - b0 / th);
    J[1][3] = kap * (Rt[1] * T[0] + R[1] * Tt[0] - b1 / th);
    J[2][3] = kap * (Rt[0] * T[1] + R[0] * Tt[1] - b2 / th);
    J[3][3] = kap * (0.5 * (Rt[2] * T[0] + R[2] * Tt[0] + Rt[0] * T[2] + R[0] * Tt[2]) + 0.5 * R[0] * T[0] +
                     0.5 * th * db0 - b3 / th);
}

template <int G = kWave>
__device__ __forceinline__ void eq_conservative(const DevSolve &d, const double (&W)[4], double (&P)[4],
                                                double *Minv)
{
    const double P0[4] = {P[0], P[1], P[2], P[3]};
    for (int it = 0; it < kEqNewton; it++) {
        double m[4], J[4][4], r[4], dP[4];
        eq_moments_jac<G>(d, P, m, J);
#pragma unroll
        for (int a = 0; a < 4; a++) r[a] = W[a] - m[a];
        solve4(J, r, dP);
#pragma unroll
        for (int a = 0; a < 4; a++) P[a] += dP[a];
    }
    // a grid too coarse for the state (a Maxwellian much narrower than the
    // velocity spacing) can leave Newton without a usable root: the cell then
    // keeps the pointwise Maxwellian of its primitive variables
    if (!(P[0] > 0) || !(P[3] > 0) || !isfinite(P[1]) || !isfinite(P[2])) {
#pragma unroll
        for (int a = 0; a < 4; a++) P[a] = P0[a];
        if (Minv) {
            const double rho = P0[0], u1 = P0[1], u2 = P0[2], E = W[3] / W[0], ir = 1.0 / rho, k23 = 2.0 / 3.0;
            const double J[16] = {1.0, 0.0, 0.0, 0.0, -u1 * ir, ir, 0.0, 0.0, -u2 * ir, 0.0, ir, 0.0,
                                  k23 * (u1 * u1 + u2 * u2 - E) * ir, -k23 * u1 * ir, -k23 * u2 * ir, k23 * ir};
#pragma unroll
            for (int q = 0; q < 16; q++) Minv[q] = J[q];
        }
        return;
    }
    if (Minv) {
        double m[4], J[4][4];
        eq_moments_jac<G>(d, P, m, J);
#pragma unroll
        for (int b = 0; b < 4; b++) {
            double A[4][4], e[4] = {0, 0, 0, 0}, x[4];
#pragma unroll
            for (int r = 0; r < 4; r++)
#pragma unroll
                for (int k = 0; k < 4; k++) A[r][k] = J[r][k];
            e[b] = 1.0;
            solve4(A, e, x);
#pragma unroll
            for (int a = 0; a < 4; a++) Minv[4 * a + b] = x[a];
        }
    }
}

// The member of a group that owns launch cell i (pre ascending, pre[0] = 0).
__device__ __forceinline__ int group_member(const MacroGroup &g, int i)
{
    int lo = 0, hi = g.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.pre[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

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
