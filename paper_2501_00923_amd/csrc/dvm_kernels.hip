// HIP kernels of libdvm for gfx950 (CDNA4).
//
// Layout: f and phi are [cell][velocity][2] (the two reduced distributions
// of Sec. 2.2 interleaved), so one cell's row of 2*nv values is contiguous
// and a wave64 reading consecutive velocities streams whole cache lines.
// One workgroup of 256 threads owns one cell for a sweep: it reads the
// cell's own row and the upwind rows of its (at most four) neighbours,
// writes the new row, and reduces the FP64 velocity moments of the new row
// in its epilogue (wave shuffles, then the 4 wave partials through LDS), so
// the next sweep finds W^{n+1} ready and f is streamed once per sweep.
// The Maxwellian is evaluated as rho/(2 pi theta) * ex[a] * ey[b] with the
// per-cell 1-D factors in LDS (tensor-product velocity grid), i.e. n1 + n2
// exponentials per cell instead of n1*n2.

#include <math.h>

#include <algorithm>

#include "dvm_internal.h"

namespace dvm {

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

constexpr double kPi = 3.14159265358979323846;

// Workgroups are handed to the 8 XCDs round-robin; give each XCD a
// contiguous stretch of the sweep order (16x16-cell tiles marching along
// grid strips) so that the upwind neighbour rows a workgroup reads were
// fetched moments before by a workgroup of the same XCD and are still in
// its L2.  Returns -1 for the padding workgroups of the last stretch.
__device__ __forceinline__ int xcd_cell(const DevSolve &d, int b)
{
    const int per = (d.nc + 7) >> 3;
    const int idx = (b & 7) * per + (b >> 3);
    return idx < d.nc ? d.order[idx] : -1;
}
static inline int xcd_grid(int n) { return ((n + 7) >> 3) << 3; }

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

// Per-cell velocity tables in LDS.
template <typename T>
struct CellLds {
    double vx[kMaxN1D], vy[kMaxN1D], wx[kMaxN1D], wy[kMaxN1D];
    T ex[kMaxN1D], ey[kMaxN1D];
    double red[4 * 12];
};

template <typename T>
__device__ __forceinline__ void load_vel_tables(const DevSolve &d, CellLds<T> &sm, double u1, double u2,
                                                double inv2th)
{
    const int t = threadIdx.x;
    if (t < d.n1) {
        const double x = d.vx[t];
        sm.vx[t] = x;
        sm.wx[t] = d.wx[t];
        const double c = x - u1;
        sm.ex[t] = (T)exp(-c * c * inv2th);
    } else if (t - d.n1 < d.n2) {
        const int b = t - d.n1;
        const double y = d.vy[b];
        sm.vy[b] = y;
        sm.wy[b] = d.wy[b];
        const double c = y - u2;
        sm.ey[b] = (T)exp(-c * c * inv2th);
    }
}

__device__ __forceinline__ double mJ_of(int objective, double v1, double v2)
{
    return objective == 0 ? v1 : 0.5 * (v1 * v1 + v2 * v2);
}

// ---------------------------------------------------------------------------
// primal sweep of one cell: eq. (numerpr_gov), first-order upwind, Jacobi
// point-implicit: f^{n+1} = (sum_in |v.S| f_up + V g/tau) / (sum_out v.S + V/tau)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void primal_cell(const DevSolve &d, int c, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ CellLds<T> sm;
    const int tid = threadIdx.x;
    const int nv = d.nv, n1 = d.n1;
    const T2 *__restrict__ fin = static_cast<const T2 *>(d.f[par]);
    T2 *__restrict__ fout = static_cast<T2 *>(d.f[par ^ 1]);

    const double *Win = d.W[par] + 4 * c;
    const double W0 = Win[0], W1 = Win[1], W2 = Win[2], W3 = Win[3];
    const double rho = W0, u1 = W1 / rho, u2 = W2 / rho;
    const double th = (2.0 / 3.0) * (W3 / rho - 0.5 * (u1 * u1 + u2 * u2));
    const double itau = d.inv_tau_inf * rho * sqrt(2.0 * th);
    const double Vt = d.vol[c] * itau;
    load_vel_tables<T>(d, sm, u1, u2, 0.5 / th);

    int nb[4];
    T Sx[4], Sy[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        nb[q] = d.nbr[4 * c + q];
        Sx[q] = (T)d.S[8 * c + 2 * q];
        Sy[q] = (T)d.S[8 * c + 2 * q + 1];
    }
    const int wl = nb[0] <= -2 ? -2 - nb[0] : -1;
    T wcoef = 0;
    double S0x = 0, S0y = 0;
    if (wl >= 0) {
        wcoef = (T)(d.F[par][wl] / d.D[wl]);
        S0x = d.S[8 * c];
        S0y = d.S[8 * c + 1];
    }
    // one source row per face, all of the storage pair type: the upwind
    // cell's row, the far-field table, or the wall table (g_M1, theta_w/2 g_M1)
    // scaled by F_l / D_l
    const T2 *src[4];
    T sc[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int n = nb[q];
        src[q] = n >= 0 ? fin + (size_t)n * nv
                        : static_cast<const T2 *>(n == -1 ? d.fd : d.gw2);
        sc[q] = n <= -2 ? wcoef : (T)1;
    }
    const T th2 = (T)(0.5 * th);
    const T gc = (T)(rho / (2.0 * kPi * th)), VtT = (T)Vt;
    __syncthreads();

    double m0 = 0, m1 = 0, m2 = 0, m3 = 0, mF = 0;
    int a = tid % n1, b = tid / n1;
    const int da = kBlock % n1, db = kBlock / n1;
    const size_t row = (size_t)c * nv;
    for (int k = tid; k < nv; k += kBlock) {
        const double v1d = sm.vx[a], v2d = sm.vy[b];
        const T v1 = (T)v1d, v2 = (T)v2d;
        // The face kind is uniform over the workgroup, only the sign of v.S
        // differs between lanes: issue every face's source load first (no
        // wait between them), then pick upwind values with selects.
        T2 up[4];
#pragma unroll
        for (int q = 0; q < 4; q++) up[q] = src[q][k];
        T out = 0, in1 = 0, in2 = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const T s = v1 * Sx[q] + v2 * Sy[q];
            if (s > 0) {
                out += s;
            } else {
                in1 -= s * (sc[q] * up[q].x);
                in2 -= s * (sc[q] * up[q].y);
            }
        }
        const T g1 = gc * sm.ex[a] * sm.ey[b];
        const T g2 = th2 * g1;
        const T den = out + VtT;
        T2 r;
        r.x = (in1 + VtT * g1) / den;
        r.y = (in2 + VtT * g2) / den;
        // streaming stores: the new row is not read again in this sweep, so
        // keep it from displacing the neighbour rows other workgroups reuse
        __builtin_nontemporal_store(r.x, &fout[row + k].x);
        __builtin_nontemporal_store(r.y, &fout[row + k].y);
        const double w = sm.wx[a] * sm.wy[b];
        const double f1 = (double)r.x, f2 = (double)r.y;
        const double wf1 = w * f1;
        m0 += wf1;
        m1 += wf1 * v1d;
        m2 += wf1 * v2d;
        m3 += wf1 * (0.5 * (v1d * v1d + v2d * v2d)) + w * f2;
        if (wl >= 0) {
            const double s0 = v1d * S0x + v2d * S0y;
            if (s0 > 0) mF += wf1 * s0;
        }
        a += da;
        b += db;
        if (a >= n1) {
            a -= n1;
            b++;
        }
    }
    double acc[5] = {m0, m1, m2, m3, mF};
    block_sum<5>(acc, sm.red);
    if (tid == 0) {
        double *Wo = d.W[par ^ 1] + 4 * c;
        Wo[0] = acc[0];
        Wo[1] = acc[1];
        Wo[2] = acc[2];
        Wo[3] = acc[3];
        if (wl >= 0) d.F[par ^ 1][wl] = acc[4] / d.wall_A[wl];
        const double e0 = acc[0] - W0, e1 = acc[1] - W1, e2 = acc[2] - W2, e3 = acc[3] - W3;
        d.red[2 * c] = e0 * e0 + e1 * e1 + e2 * e2 + e3 * e3;
        d.red[2 * c + 1] = W0 * W0 + W1 * W1 + W2 * W2 + W3 * W3;
    }
}

// moments W and wall flux F of f[par] for one cell (no update)
template <typename T>
__device__ __forceinline__ void moments_cell(const DevSolve &d, int c, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ CellLds<T> sm;
    const int tid = threadIdx.x, nv = d.nv, n1 = d.n1;
    load_vel_tables<T>(d, sm, 0.0, 0.0, 0.0);
    const int l0 = d.nbr[4 * c];
    const int wl = l0 <= -2 ? -2 - l0 : -1;
    const double S0x = d.S[8 * c], S0y = d.S[8 * c + 1];
    const T2 *__restrict__ f = static_cast<const T2 *>(d.f[par]);
    __syncthreads();
    double m0 = 0, m1 = 0, m2 = 0, m3 = 0, mF = 0;
    int a = tid % n1, b = tid / n1;
    const int da = kBlock % n1, db = kBlock / n1;
    for (int k = tid; k < nv; k += kBlock) {
        const double v1d = sm.vx[a], v2d = sm.vy[b];
        const T2 r = f[(size_t)c * nv + k];
        const double w = sm.wx[a] * sm.wy[b];
        const double f1 = (double)r.x, f2 = (double)r.y;
        const double wf1 = w * f1;
        m0 += wf1;
        m1 += wf1 * v1d;
        m2 += wf1 * v2d;
        m3 += wf1 * (0.5 * (v1d * v1d + v2d * v2d)) + w * f2;
        if (wl >= 0) {
            const double s0 = v1d * S0x + v2d * S0y;
            if (s0 > 0) mF += wf1 * s0;
        }
        a += da;
        b += db;
        if (a >= n1) {
            a -= n1;
            b++;
        }
    }
    double acc[5] = {m0, m1, m2, m3, mF};
    block_sum<5>(acc, sm.red);
    if (tid == 0) {
        double *Wo = d.W[par] + 4 * c;
        Wo[0] = acc[0];
        Wo[1] = acc[1];
        Wo[2] = acc[2];
        Wo[3] = acc[3];
        if (wl >= 0) d.F[par][wl] = acc[4] / d.wall_A[wl];
    }
}

// ---------------------------------------------------------------------------
// adjoint sweep of one cell: eq. (numerad_gov) with the wall and far-field
// conditions of eq. (formula_adjointbgk), Jacobi point-implicit:
// phi^{n+1} = (sum_out v.S phi_down + V (phi_eq/tau + phi_tau)) / (sum_out v.S + V/tau)
// Epilogue: What (eq. adjoint_macdefines, via primitive variables),
// rho_tau, the wall multiplier Phi_l and the residual partials of phi^{n+1}.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void adjoint_cell(const DevSolve &d, int c, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ CellLds<T> sm;
    const int tid = threadIdx.x;
    const int nv = d.nv, n1 = d.n1;
    const T2 *__restrict__ pin = static_cast<const T2 *>(d.phi[par]);
    T2 *__restrict__ pout = static_cast<T2 *>(d.phi[par ^ 1]);
    const T2 *__restrict__ fst = static_cast<const T2 *>(d.fstar);

    const double *ac = d.acoef + 16 * c;
    const double rho = ac[0], u1 = ac[1], u2 = ac[2], th = ac[3], itau = ac[4], gcoef = ac[5];
    const double dt0 = ac[6], dt1 = ac[7], dt2 = ac[8], dt3 = ac[9];
    const double Vv = d.vol[c];
    const double *aw = d.aW[par] + 8 * c;
    const double rt = aw[4];
    // source phi_eq / tau + phi_tau = C0 + C1 v1 + C2 v2 + C3 |v|^2/2 (first), C3 (second)
    const double C0 = aw[0] * itau - rt * dt0, C1 = aw[1] * itau - rt * dt1;
    const double C2 = aw[2] * itau - rt * dt2, C3 = aw[3] * itau - rt * dt3;
    load_vel_tables<T>(d, sm, u1, u2, 0.5 / th);

    int nb[4];
    T Sx[4], Sy[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        nb[q] = d.nbr[4 * c + q];
        Sx[q] = (T)d.S[8 * c + 2 * q];
        Sy[q] = (T)d.S[8 * c + 2 * q + 1];
    }
    const int wl = nb[0] <= -2 ? -2 - nb[0] : -1;
    T Phi_w = 0;
    double S0x = 0, S0y = 0;
    if (wl >= 0) {
        Phi_w = (T)d.Phi[par][wl];
        S0x = d.S[8 * c];
        S0y = d.S[8 * c + 1];
    }
    const T *__restrict__ gM = static_cast<const T *>(d.gM);
    // downstream rows of interior faces; boundary faces read their own row
    // (a valid address) and ignore it
    const T2 *dsrc[4];
#pragma unroll
    for (int q = 0; q < 4; q++) dsrc[q] = pin + (size_t)(nb[q] >= 0 ? nb[q] : c) * nv;
    const int obj = d.objective;
    const T VT = (T)Vv, den0 = (T)(Vv * itau);
    const T Ct0 = (T)C0, Ct1 = (T)C1, Ct2 = (T)C2, Ct3 = (T)C3;
    const T gc = (T)gcoef, th2 = (T)(0.5 * th);
    const double thw2 = 0.5 * d.theta_w;
    __syncthreads();

    double A0 = 0, A1 = 0, A2 = 0, A3 = 0, A4 = 0, R = 0, Pw = 0, dn = 0, dd = 0;
    int a = tid % n1, b = tid / n1;
    const int da = kBlock % n1, db = kBlock / n1;
    const size_t row = (size_t)c * nv;
    for (int k = tid; k < nv; k += kBlock) {
        const double v1d = sm.vx[a], v2d = sm.vy[b];
        const T v1 = (T)v1d, v2 = (T)v2d;
        const T mj = (T)mJ_of(obj, v1d, v2d);
        // all loads of this velocity first (own phi^n, frozen f, the
        // downstream rows of interior faces), then the select-based update
        const T2 old = pin[row + k];
        const T2 fs = fst[row + k];
        T2 dwn[4];
#pragma unroll
        for (int q = 0; q < 4; q++) dwn[q] = dsrc[q][k];
        T out = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const T s = v1 * Sx[q] + v2 * Sy[q];
            if (s > 0) {
                out += s;
                if (nb[q] >= 0) {
                    a1 += s * dwn[q].x;
                    a2 += s * dwn[q].y;
                } else if (nb[q] <= -2) {
                    a1 += s * (Phi_w - mj);
                }
            }
        }
        const T vv2 = (T)0.5 * (v1 * v1 + v2 * v2);
        const T s1 = Ct0 + Ct1 * v1 + Ct2 * v2 + Ct3 * vv2;
        const T den = out + den0;
        T2 r;
        r.x = (a1 + VT * s1) / den;
        r.y = (a2 + VT * Ct3) / den;
        __builtin_nontemporal_store(r.x, &pout[row + k].x);
        __builtin_nontemporal_store(r.y, &pout[row + k].y);
        // epilogue accumulations from phi^{n+1}
        const double w = sm.wx[a] * sm.wy[b];
        const double p1 = (double)r.x, p2 = (double)r.y;
        const double g1 = (double)(gc * sm.ex[a] * sm.ey[b]);
        const double g2 = (double)(th2 * (T)g1);
        const double q = p1 + 0.5 * th * p2;
        const double c1 = v1d - u1, c2 = v2d - u2;
        const double wg = w * g1;
        A0 += wg * q;
        A1 += wg * q * c1;
        A2 += wg * q * c2;
        A3 += wg * q * (c1 * c1 + c2 * c2);
        A4 += wg * p2;
        R += w * (p1 * (g1 - (double)fs.x) + p2 * (g2 - (double)fs.y));
        if (wl >= 0) {
            const double s0 = v1d * S0x + v2d * S0y;
            if (s0 <= 0) Pw += w * s0 * (double)gM[k] * ((p1 + mJ_of(obj, v1d, v2d)) + thw2 * p2);
        }
        const double e1 = p1 - (double)old.x, e2 = p2 - (double)old.y;
        dn += w * (e1 * e1 + e2 * e2);
        dd += w * (p1 * p1 + p2 * p2);
        a += da;
        b += db;
        if (a >= n1) {
            a -= n1;
            b++;
        }
    }
    double acc[9] = {A0, A1, A2, A3, A4, R, Pw, dn, dd};
    block_sum<9>(acc, sm.red);
    if (tid == 0) {
        // phi . dg/dP with P = (rho, u1, u2, theta)
        const double P0 = acc[0] / rho;
        const double P1 = acc[1] / th, P2 = acc[2] / th;
        const double P3 = acc[3] / (2.0 * th * th) - acc[0] / th + 0.5 * acc[4];
        const double E = ac[10];
        const double ir = 1.0 / rho;
        double *ao = d.aW[par ^ 1] + 8 * c;
        // What_m = sum_q P_q dP_q/dW_m
        ao[0] = P0 - P1 * u1 * ir - P2 * u2 * ir + P3 * (2.0 / 3.0) * (u1 * u1 + u2 * u2 - E) * ir;
        ao[1] = P1 * ir - P3 * (2.0 / 3.0) * u1 * ir;
        ao[2] = P2 * ir - P3 * (2.0 / 3.0) * u2 * ir;
        ao[3] = P3 * (2.0 / 3.0) * ir;
        ao[4] = acc[5] * itau;
        if (wl >= 0) d.Phi[par ^ 1][wl] = -acc[6] / (d.wall_A[wl] * d.D[wl]);
        d.red[2 * c] = acc[7];
        d.red[2 * c + 1] = acc[8];
    }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_primal_sweep(DevSolve d, int par)
{
    const int c = xcd_cell(d, blockIdx.x);
    if (c < 0) return;
    primal_cell<T>(d, c, par);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments(DevSolve d, int par)
{
    const int c = xcd_cell(d, blockIdx.x);
    if (c < 0) return;
    moments_cell<T>(d, c, par);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adjoint_sweep(DevSolve d, int par)
{
    const int c = xcd_cell(d, blockIdx.x);
    if (c < 0) return;
    adjoint_cell<T>(d, c, par);
}

// one sweep of the primal-phase (or adjoint-phase) members of a batch; a
// block owns one (solve, cell).  The two phases are separate kernels so
// that each gets the occupancy of its own register footprint.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_primal(const DevSolve *tab, const int32_t *blk_solve,
                                                         const int32_t *blk_cell, const int32_t *par0, int step)
{
    const int s = blk_solve[blockIdx.x];
    if (s < 0) return;
    primal_cell<T>(tab[s], blk_cell[blockIdx.x], (par0[s] + step) & 1);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_batch_adjoint(const DevSolve *tab, const int32_t *blk_solve,
                                                          const int32_t *blk_cell, const int32_t *par0, int step)
{
    const int s = blk_solve[blockIdx.x];
    if (s < 0) return;
    adjoint_cell<T>(tab[s], blk_cell[blockIdx.x], (par0[s] + step) & 1);
}

// f = far-field Maxwellian everywhere (storage type)
template <typename T>
__global__ void k_fill_fd(DevSolve d, int par)
{
    using T2 = typename Vec2<T>::type;
    const T2 *fd = static_cast<const T2 *>(d.fd);
    T2 *f = static_cast<T2 *>(d.f[par]);
    const size_t n = (size_t)d.nc * d.nv;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        f[i] = fd[i % d.nv];
}

template <typename T>
__global__ void k_zero(T *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// per-cell adjoint coefficients from the frozen moments
__global__ void k_adjoint_coef(DevSolve d, const double *Wst)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    const double *W = Wst + 4 * c;
    const double rho = W[0], u1 = W[1] / rho, u2 = W[2] / rho, E = W[3] / rho;
    const double th = (2.0 / 3.0) * (E - 0.5 * (u1 * u1 + u2 * u2));
    const double itau = d.inv_tau_inf * rho * sqrt(2.0 * th);
    double *ac = d.acoef + 16 * c;
    ac[0] = rho;
    ac[1] = u1;
    ac[2] = u2;
    ac[3] = th;
    ac[4] = itau;
    ac[5] = rho / (2.0 * kPi * th);
    // (1/tau) dtau/dW, tau ~ 1 / (rho sqrt(theta)) (hard sphere)
    const double ir = 1.0 / rho, k23 = 2.0 / 3.0;
    const double dth0 = k23 * (u1 * u1 + u2 * u2 - E) * ir, dth1 = -k23 * u1 * ir, dth2 = -k23 * u2 * ir,
                 dth3 = k23 * ir;
    const double h = 0.5 / th;
    ac[6] = -ir - h * dth0;
    ac[7] = -h * dth1;
    ac[8] = -h * dth2;
    ac[9] = -h * dth3;
    ac[10] = E;
}

// Phi_l of phi = 0 (only the objective's m_J term): one block per element
template <typename T>
__global__ __launch_bounds__(kBlock) void k_wall_phi0(DevSolve d, int par)
{
    __shared__ double red[4 * 1];
    const int l = blockIdx.x;
    const T *gM = static_cast<const T *>(d.gM);
    const double n1 = d.wall_n[2 * l], n2 = d.wall_n[2 * l + 1];
    double s = 0;
    for (int k = threadIdx.x; k < d.nv; k += kBlock) {
        const double v1 = d.vx[k % d.n1], v2 = d.vy[k / d.n1];
        const double vn = v1 * n1 + v2 * n2;
        if (vn <= 0) s += d.wx[k % d.n1] * d.wy[k / d.n1] * vn * mJ_of(d.objective, v1, v2) * (double)gM[k];
    }
    double acc[1] = {s};
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) d.Phi[par][l] = -acc[0] / d.D[l];
}

// deterministic sum of the per-cell residual partials: out[0..1]
__global__ __launch_bounds__(kBlock) void k_residual(const double *red, int nc, double *out)
{
    __shared__ double lds[4 * 2];
    double a = 0, b = 0;
    for (int c = threadIdx.x; c < nc; c += kBlock) {
        a += red[2 * c];
        b += red[2 * c + 1];
    }
    double acc[2] = {a, b};
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        out[0] = acc[0];
        out[1] = acc[1];
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_residual(const DevSolve *tab, double *out)
{
    __shared__ double lds[4 * 2];
    const DevSolve &d = tab[blockIdx.x];
    double a = 0, b = 0;
    for (int c = threadIdx.x; c < d.nc; c += kBlock) {
        a += d.red[2 * c];
        b += d.red[2 * c + 1];
    }
    double acc[2] = {a, b};
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = acc[0];
        out[2 * blockIdx.x + 1] = acc[1];
    }
}

// J_l = A_l sum_k w m_J (v.n) f1_{l,k}, eq. (numer_J): one block per element
template <typename T>
__global__ __launch_bounds__(kBlock) void k_objective_elem(DevSolve d, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ double red[4];
    const int l = blockIdx.x;
    const int c = d.wall_cell[l];
    const T2 *f = static_cast<const T2 *>(d.f[par]);
    const T *gM = static_cast<const T *>(d.gM);
    const double n1 = d.wall_n[2 * l], n2 = d.wall_n[2 * l + 1];
    const double FD = d.F[par][l] / d.D[l];
    double s = 0;
    for (int k = threadIdx.x; k < d.nv; k += kBlock) {
        const int a = k % d.n1, b = k / d.n1;
        const double v1 = d.vx[a], v2 = d.vy[b];
        const double vn = v1 * n1 + v2 * n2;
        const double f1 = vn > 0 ? (double)f[(size_t)c * d.nv + k].x : FD * (double)gM[k];
        s += d.wx[a] * d.wy[b] * mJ_of(d.objective, v1, v2) * vn * f1;
    }
    double acc[1] = {s};
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) d.Jl[l] = d.wall_A[l] * acc[0];
}

__global__ __launch_bounds__(kBlock) void k_objective_sum(DevSolve d)
{
    __shared__ double red[4];
    double s = 0;
    for (int l = threadIdx.x; l < d.nw; l += kBlock) s += d.Jl[l];
    double acc[1] = {s};
    block_sum<1>(acc, red);
    if (threadIdx.x == 0) {
        d.out[0] = acc[0];
        d.out[1] = acc[0] / d.cd_scale;
    }
}

// ---------------------------------------------------------------------------
// wall sensitivity, eqs. (sens_J_itf), (gaussgrad), (sens_B_itf): one block
// per wall element
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_wall_sens(DevSolve d, int fpar, int ppar)
{
    using T2 = typename Vec2<T>::type;
    __shared__ double red[4 * 12];
    const int l = blockIdx.x;
    const int c = d.wall_cell[l];
    const T2 *f = static_cast<const T2 *>(d.f[fpar]);
    const T2 *ph = static_cast<const T2 *>(d.phi[ppar]);
    const T2 *fd = static_cast<const T2 *>(d.fd);
    const T *gM = static_cast<const T *>(d.gM);
    const double n1 = d.wall_n[2 * l], n2 = d.wall_n[2 * l + 1], A = d.wall_A[l];
    const double iD = 1.0 / d.D[l], F = d.F[fpar][l], thw2 = 0.5 * d.theta_w;
    const double iV = 1.0 / d.vol[c];
    int nb[4];
    double Sx[4], Sy[4];
    for (int q = 0; q < 4; q++) {
        nb[q] = d.nbr[4 * c + q];
        Sx[q] = d.S[8 * c + 2 * q];
        Sy[q] = d.S[8 * c + 2 * q + 1];
    }
    double sa = 0, jx0 = 0, jx1 = 0, jn0 = 0, jn1 = 0, M0 = 0, M1 = 0, G0 = 0, G1 = 0, bx0 = 0, bx1 = 0, Pw = 0;
    const size_t row = (size_t)c * d.nv;
    for (int k = threadIdx.x; k < d.nv; k += kBlock) {
        const int a = k % d.n1, b = k / d.n1;
        const double v1 = d.vx[a], v2 = d.vy[b], w = d.wx[a] * d.wy[b];
        const double vn = v1 * n1 + v2 * n2;
        const double mj = mJ_of(d.objective, v1, v2);
        const T2 fc = f[row + k];
        const double gw1 = F * (double)gM[k] * iD;
        const double f1l = vn > 0 ? (double)fc.x : gw1;
        // Green-Gauss gradient with the scheme's upwind face values
        double g10 = 0, g11 = 0, g20 = 0, g21 = 0;
        for (int q = 0; q < 4; q++) {
            const double s = v1 * Sx[q] + v2 * Sy[q];
            double a1, a2;
            if (s > 0) {
                a1 = (double)fc.x;
                a2 = (double)fc.y;
            } else if (nb[q] >= 0) {
                const T2 u = f[(size_t)nb[q] * d.nv + k];
                a1 = (double)u.x;
                a2 = (double)u.y;
            } else if (nb[q] == -1) {
                const T2 u = fd[k];
                a1 = (double)u.x;
                a2 = (double)u.y;
            } else {
                a1 = gw1;
                a2 = thw2 * gw1;
            }
            g10 += a1 * Sx[q];
            g11 += a1 * Sy[q];
            g20 += a2 * Sx[q];
            g21 += a2 * Sy[q];
        }
        g10 *= iV;
        g11 *= iV;
        g20 *= iV;
        g21 *= iV;
        sa += w * mj * vn * f1l;
        jx0 += w * mj * vn * g10;
        jx1 += w * mj * vn * g11;
        jn0 += w * mj * v1 * f1l;
        jn1 += w * mj * v2 * f1l;
        M0 += w * v1 * f1l;
        M1 += w * v2 * f1l;
        if (vn > 0) {
            G0 += w * vn * g10;
            G1 += w * vn * g11;
        } else {
            const T2 pc = ph[row + k];
            const double pw1 = -vn * ((double)pc.x + mj), pw2 = -vn * (double)pc.y;
            bx0 += w * (pw1 * g10 + pw2 * g20);
            bx1 += w * (pw1 * g11 + pw2 * g21);
            const double gb1 = (double)gM[k] * iD;
            Pw += w * (pw1 * gb1 + pw2 * thw2 * gb1);
        }
    }
    double acc[12] = {sa, jx0, jx1, jn0, jn1, M0, M1, G0, G1, bx0, bx1, Pw};
    block_sum<12>(acc, red);
    if (threadIdx.x == 0) {
        double *o = d.sens + 5 * l;
        const double Phi = acc[11];
        o[0] = acc[0];
        o[1] = A * (acc[1] + acc[9] - Phi * acc[7]);
        o[2] = A * (acc[2] + acc[10] - Phi * acc[8]);
        o[3] = A * (acc[3] - Phi * acc[5]);
        o[4] = A * (acc[4] - Phi * acc[6]);
    }
}

// element -> node transform, eq. (sens_nod), then dJ/dalpha = dJ/dx . dx/dalpha
__global__ __launch_bounds__(kBlock) void k_nodes_params(DevSolve d, int n_params)
{
    __shared__ double red[4];
    const int nw = d.nw;
    for (int m = threadIdx.x; m < nw; m += kBlock) {
        double g[2] = {0, 0};
        for (int side = 0; side < 2; side++) {
            const int l = side == 0 ? m : (m + nw - 1) % nw;   // m is x_{l,1} of l = m, x_{l,2} of l = m-1
            const double *o = d.sens + 5 * l;
            const double ax = d.wall_a[2 * l], ay = d.wall_a[2 * l + 1];
            const double bx = d.wall_b[2 * l], by = d.wall_b[2 * l + 1];
            const double A = d.wall_A[l], n1 = d.wall_n[2 * l], n2 = d.wall_n[2 * l + 1];
            const double sg = ((ax - bx) * n2 - (ay - by) * n1) > 0 ? 1.0 : -1.0;
            const double sgn = side == 0 ? 1.0 : -1.0;     // d/db = -d/da for A and n
            const double dA0 = (ax - bx) / A, dA1 = (ay - by) / A;
            // (dn/da)^T S_n, dn/da = sg/A [[-n1 n2, -n2^2], [n1^2, n1 n2]]
            const double t0 = sg / A * (-n1 * n2 * o[3] + n1 * n1 * o[4]);
            const double t1 = sg / A * (-n2 * n2 * o[3] + n1 * n2 * o[4]);
            g[0] += sgn * (o[0] * dA0 + t0) + 0.5 * o[1];
            g[1] += sgn * (o[0] * dA1 + t1) + 0.5 * o[2];
        }
        d.dJdn[2 * m] = g[0];
        d.dJdn[2 * m + 1] = g[1];
    }
    __threadfence_block();
    __syncthreads();
    for (int p = 0; p < n_params; p++) {
        double s = 0;
        for (int m = threadIdx.x; m < nw; m += kBlock)
            s += d.dJdn[2 * m] * d.jac[(2 * m) * kMaxParams + p] + d.dJdn[2 * m + 1] * d.jac[(2 * m + 1) * kMaxParams + p];
        double acc[1] = {s};
        block_sum<1>(acc, red);
        if (threadIdx.x == 0) d.dJda[p] = acc[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
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

static inline int ew_grid(size_t n) { return (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192); }

hipError_t launch_primal_init(const DevSolve &d, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_fill_fd<T>, dim3(ew_grid((size_t)d.nc * d.nv)), dim3(kBlock), 0, st, d, 0));
    if (hipError_t e = hipGetLastError()) return e;
    return launch_moments(d, 0, st);
}

hipError_t launch_moments(const DevSolve &d, int par, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_moments<T>, dim3(xcd_grid(d.nc)), dim3(kBlock), 0, st, d, par));
    return hipGetLastError();
}

hipError_t launch_primal_sweep(const DevSolve &d, int par, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_primal_sweep<T>, dim3(xcd_grid(d.nc)), dim3(kBlock), 0, st, d, par));
    return hipGetLastError();
}

hipError_t launch_residual(const DevSolve &d, int adjoint, hipStream_t st)
{
    hipLaunchKernelGGL(k_residual, dim3(1), dim3(kBlock), 0, st, d.red, d.nc, d.out + (adjoint ? 4 : 2));
    return hipGetLastError();
}

hipError_t launch_objective(const DevSolve &d, int par, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_objective_elem<T>, dim3(d.nw), dim3(kBlock), 0, st, d, par));
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_objective_sum, dim3(1), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_adjoint_init(const DevSolve &d, int fpar, hipStream_t st)
{
    hipLaunchKernelGGL(k_adjoint_coef, dim3((d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d, d.W[fpar]);
    if (hipError_t e = hipGetLastError()) return e;
    const size_t n = (size_t)d.nc * d.nv * 2;
    if (d.mixed)
        hipLaunchKernelGGL(k_zero<float>, dim3(ew_grid(n)), dim3(kBlock), 0, st, static_cast<float *>(d.phi[0]), n);
    else
        hipLaunchKernelGGL(k_zero<double>, dim3(ew_grid(n)), dim3(kBlock), 0, st, static_cast<double *>(d.phi[0]), n);
    if (hipError_t e = hipGetLastError()) return e;
    // both ping-pong buffers: slots 5..7 of each cell are padding that the
    // sweep never writes, and checkpoints copy them
    for (int p = 0; p < 2; p++) {
        hipLaunchKernelGGL(k_zero<double>, dim3(ew_grid((size_t)8 * d.nc)), dim3(kBlock), 0, st, d.aW[p],
                           (size_t)8 * d.nc);
        if (hipError_t e = hipGetLastError()) return e;
    }
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_wall_phi0<T>, dim3(d.nw), dim3(kBlock), 0, st, d, 0));
    return hipGetLastError();
}

hipError_t launch_adjoint_sweep(const DevSolve &d, int par, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_adjoint_sweep<T>, dim3(xcd_grid(d.nc)), dim3(kBlock), 0, st, d, par));
    return hipGetLastError();
}

hipError_t launch_wall_sens(const DevSolve &d, int fpar, int ppar, int n_params, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_wall_sens<T>, dim3(d.nw), dim3(kBlock), 0, st, d, fpar, ppar));
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_nodes_params, dim3(1), dim3(kBlock), 0, st, d, n_params);
    return hipGetLastError();
}

hipError_t launch_batch(const DevSolve *tab, const int32_t *blk_solve, const int32_t *blk_cell,
                        const int32_t *par0, int step, int nblocks, int mixed, int adjoint, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (adjoint)
        DVM_DISPATCH(mixed, hipLaunchKernelGGL(k_batch_adjoint<T>, dim3(nblocks), dim3(kBlock), 0, st, tab,
                                               blk_solve, blk_cell, par0, step));
    else
        DVM_DISPATCH(mixed, hipLaunchKernelGGL(k_batch_primal<T>, dim3(nblocks), dim3(kBlock), 0, st, tab,
                                               blk_solve, blk_cell, par0, step));
    return hipGetLastError();
}

hipError_t launch_batch_residual(const DevSolve *tab, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_residual, dim3(n), dim3(kBlock), 0, st, tab, out);
    return hipGetLastError();
}

}  // namespace dvm
