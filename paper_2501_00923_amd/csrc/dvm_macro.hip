// Macroscopic prediction of the primal iteration (gfx950).
//
// Sec. 3.1 accelerates the kinetic iterations with "prediction" solutions of
// approximate macroscopic equations from the continuum limit.  Every K
// sweeps (first-order scheme):
//   1. k_macro_state: each cell's equilibrium parameters P' and dP'/dW (the
//      pointwise ones, or the discrete-conservative ones by Newton);
//   2. k_macro_assemble: the moments r of the kinetic residual of eq.
//      (numerpr_gov) at the current f, and the linearised macroscopic system
//      A dW = -r with A the moments of the scheme's upwind transport of
//      equilibrium perturbations: the outflow faces carry the cell's own
//      dg/dW, the inflow faces the neighbour's, the far field nothing and
//      the wall face the diffuse value's response gbar dF_l; plus the
//      pseudo-time term (|u| + c) sum_q |S_q| / CFL (CFL 1000) on the
//      diagonal, which keeps near-singular modes of the steady operator (a
//      slow wake, a sonic region) from being amplified; stored as the
//      inverse of each cell's own block and the blocks of its four face
//      neighbours;
//   3. k_macro_rbgs: red-black block Gauss-Seidel half steps from dW = 0
//      (colour (i + j) % 2 in mesh numbering, each half step reading one
//      array and writing the other);
//   4. k_macro_apply: W += dW, limited so that rho and theta change by at
//      most 20%: the next sweep relaxes towards the predicted moments.
// The residual's moments vanish at the discrete solution, so the prediction
// leaves the solution of the plain iteration unchanged.  The work is small
// next to the sweeps (a few passes over the velocity grid per cell, every K
// sweeps), so it favours plain, fixed-order FP64 code: one velocity per
// lane, moment sums reduced across the wave in a fixed order.

#include <math.h>

#include "dvm_device.h"

namespace dvm {

constexpr int kMacroState = 20;   // doubles per cell: P' (4), dP'/dW (16, row = parameter)
constexpr double kMacroCFL = 1000.0;

// ---------------------------------------------------------------------------
// per-cell equilibrium parameters and their derivative, one wave per cell
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_macro_state(DevSolve d, int par)
{
    const int c = blockIdx.x * (kBlock / kWave) + (int)(threadIdx.x / kWave);
    if (c >= d.nc) return;                      // whole waves; the kernel has no block barrier
    const double *W = d.W[par] + 4 * c;
    const double rho = W[0], u1 = W[1] / rho, u2 = W[2] / rho, E = W[3] / rho;
    const double th = (2.0 / 3.0) * (E - 0.5 * (u1 * u1 + u2 * u2));
    double P[4] = {rho, u1, u2, th}, M[16];
    if (d.equil) {
        const double Wv[4] = {W[0], W[1], W[2], W[3]};
        eq_conservative(d, Wv, P, M);
    } else {
        const double ir = 1.0 / rho, k23 = 2.0 / 3.0;
        const double J[16] = {1.0, 0.0, 0.0, 0.0, -u1 * ir, ir, 0.0, 0.0, -u2 * ir, 0.0, ir, 0.0,
                              k23 * (u1 * u1 + u2 * u2 - E) * ir, -k23 * u1 * ir, -k23 * u2 * ir, k23 * ir};
#pragma unroll
        for (int q = 0; q < 16; q++) M[q] = J[q];
    }
    if (threadIdx.x % kWave != 0) return;
    double *o = d.mstate + kMacroState * c;
#pragma unroll
    for (int a = 0; a < 4; a++) o[a] = P[a];
#pragma unroll
    for (int q = 0; q < 16; q++) o[4 + q] = M[q];
}

// derivatives of (g1, g2) with respect to the equilibrium parameters
// (rho, u1, u2, theta) at velocity (v1, v2), with g1 = kap X Y from the tables
__device__ __forceinline__ void dg_dP(double kap, const double *P, double X, double Y, double v1, double v2,
                                      double &g1, double &g2, double (&d1)[4], double (&d2)[4])
{
    const double th = P[3], c1 = v1 - P[1], c2 = v2 - P[2];
    g1 = kap * X * Y;
    g2 = 0.5 * th * g1;
    d1[0] = g1 / P[0];
    d1[1] = g1 * c1 / th;
    d1[2] = g1 * c2 / th;
    d1[3] = g1 * ((c1 * c1 + c2 * c2) / (2.0 * th * th) - 1.0 / th);
#pragma unroll
    for (int p = 0; p < 4; p++) d2[p] = 0.5 * th * d1[p];
    d2[3] += 0.5 * g1;
}

// this wave's 1-D factor tables X(v1), Y(v2) of the Maxwellian of state P
__device__ __forceinline__ void macro_tables(const DevSolve &d, const double *P, double *X, double *Y)
{
    const int lane = threadIdx.x % kWave;
    const double h = 0.5 / P[3];
    for (int i = lane; i < d.n1; i += kWave) {
        const double e = d.vx[i] - P[1];
        X[i] = exp(-e * e * h);
    }
    for (int i = lane; i < d.n2; i += kWave) {
        const double e = d.vy[i] - P[2];
        Y[i] = exp(-e * e * h);
    }
}

// ---------------------------------------------------------------------------
// assembly, one wave per cell; every wave of a workgroup runs the same
// passes (the table exchange between passes is a workgroup barrier)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_macro_assemble(DevSolve d, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ double tabX[kBlock / kWave][kMaxN1D], tabY[kBlock / kWave][kMaxN1D];
    const int w = (int)(threadIdx.x / kWave), lane = threadIdx.x % kWave;
    const int c0 = blockIdx.x * (kBlock / kWave) + w;
    const bool act = c0 < d.nc;
    const int c = act ? c0 : d.nc - 1;
    const int nv = d.nv, n1 = d.n1;
    const T2 *__restrict__ f = static_cast<const T2 *>(d.f[par]);
    const T2 *__restrict__ fd = static_cast<const T2 *>(d.fd);
    const T *__restrict__ gM = static_cast<const T *>(d.gM);
    const double *ms = d.mstate + kMacroState * c;
    double P[4];
#pragma unroll
    for (int a = 0; a < 4; a++) P[a] = ms[a];
    const double kap = P[0] / (2.0 * kPi * P[3]);
    // 1/tau of the cell's own rho and theta
    const double *W = d.W[par] + 4 * c;
    const double rho = W[0], u1 = W[1] / rho, u2 = W[2] / rho;
    const double th = (2.0 / 3.0) * (W[3] / rho - 0.5 * (u1 * u1 + u2 * u2));
    const double Vt = d.vol[c] * d.inv_tau_inf * rho * sqrt(2.0 * th);
    int nb[4];
    double Sx[4], Sy[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        nb[q] = d.nbr[4 * c + q];
        Sx[q] = d.S[8 * c + 2 * q];
        Sy[q] = d.S[8 * c + 2 * q + 1];
    }
    const int wl = nb[0] <= -2 ? -2 - nb[0] : -1;
    const double Fw = wl >= 0 ? d.F[par][wl] : 0.0, Dw = wl >= 0 ? d.D[wl] : 1.0;
    const double n1w = wl >= 0 ? d.wall_n[2 * wl] : 0.0, n2w = wl >= 0 ? d.wall_n[2 * wl + 1] : 0.0;
    const double thw2 = 0.5 * d.theta_w;
    const size_t row = (size_t)c * nv;

    // pass 0: r, the cell's own block (in dg/dP' form), the wall coupling
    macro_tables(d, P, tabX[w], tabY[w]);
    __syncthreads();
    double acc[28];
#pragma unroll
    for (int i = 0; i < 28; i++) acc[i] = 0.0;
    double *r = acc, *Dp = acc + 4, *wall1 = acc + 20, *dFp = acc + 24;
    for (int k = lane; k < nv; k += kWave) {
        const int a = k % n1, b = k / n1;
        const double v1 = d.vx[a], v2 = d.vy[b], wt = d.wx[a] * d.wy[b];
        const double psi[4] = {1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2)};
        double g1, g2, d1[4], d2[4];
        dg_dP(kap, P, tabX[w][a], tabY[w][b], v1, v2, g1, g2, d1, d2);
        const T2 fk = f[row + k];
        const double f1 = (double)fk.x, f2 = (double)fk.y;
        const double e1 = Vt * (f1 - g1), e2 = Vt * (f2 - g2);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const double s = v1 * Sx[q] + v2 * Sy[q];
            double a1, a2;
            if (s > 0) {
                a1 = f1;
                a2 = f2;
#pragma unroll
                for (int x = 0; x < 4; x++)
#pragma unroll
                    for (int p = 0; p < 4; p++) Dp[4 * x + p] += wt * s * (psi[x] * d1[p] + (x == 3 ? d2[p] : 0.0));
            } else if (nb[q] >= 0) {
                const T2 u = f[(size_t)nb[q] * nv + k];
                a1 = (double)u.x;
                a2 = (double)u.y;
            } else if (nb[q] == -1) {
                const T2 u = fd[k];
                a1 = (double)u.x;
                a2 = (double)u.y;
            } else {
                const double gb1 = (double)gM[k] / Dw, gb2 = thw2 * gb1;
                a1 = Fw * gb1;
                a2 = Fw * gb2;
#pragma unroll
                for (int x = 0; x < 4; x++) wall1[x] += wt * s * (psi[x] * gb1 + (x == 3 ? gb2 : 0.0));
            }
#pragma unroll
            for (int x = 0; x < 4; x++) r[x] += wt * s * (psi[x] * a1 + (x == 3 ? a2 : 0.0));
        }
#pragma unroll
        for (int x = 0; x < 4; x++) r[x] += wt * (psi[x] * e1 + (x == 3 ? e2 : 0.0));
        if (wl >= 0) {
            const double vn = v1 * n1w + v2 * n2w;
            if (vn > 0) {
#pragma unroll
                for (int p = 0; p < 4; p++) dFp[p] += wt * vn * d1[p];
            }
        }
    }
    wave_sum<28>(acc);
    const double *M = ms + 4;
    if (act && lane == 0) {
        // D = Dp M + wall1 (dFp M)
        double Dm[4][4], dF[4];
#pragma unroll
        for (int m = 0; m < 4; m++) {
            dF[m] = ((dFp[0] * M[m] + dFp[1] * M[4 + m]) + dFp[2] * M[8 + m]) + dFp[3] * M[12 + m];
#pragma unroll
            for (int x = 0; x < 4; x++)
                Dm[x][m] = ((Dp[4 * x] * M[m] + Dp[4 * x + 1] * M[4 + m]) + Dp[4 * x + 2] * M[8 + m]) +
                           Dp[4 * x + 3] * M[12 + m];
        }
#pragma unroll
        for (int x = 0; x < 4; x++)
#pragma unroll
            for (int m = 0; m < 4; m++) Dm[x][m] += wall1[x] * dF[m];
        // pseudo-time term V/dt of the cell
        double sS = 0.0;
#pragma unroll
        for (int q = 0; q < 4; q++) sS += hypot(Sx[q], Sy[q]);
        const double lam = (sqrt(u1 * u1 + u2 * u2) + sqrt(5.0 / 3.0 * th)) * sS / kMacroCFL;
#pragma unroll
        for (int x = 0; x < 4; x++) Dm[x][x] += lam;
        double *Di = d.mDinv + 16 * c;
#pragma unroll
        for (int b2 = 0; b2 < 4; b2++) {
            double A[4][4], e[4] = {0, 0, 0, 0}, x[4];
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 4; j++) A[i][j] = Dm[i][j];
            e[b2] = 1.0;
            solve4(A, e, x);
#pragma unroll
            for (int a2 = 0; a2 < 4; a2++) Di[4 * a2 + b2] = x[a2];
        }
#pragma unroll
        for (int x = 0; x < 4; x++) d.mr[4 * c + x] = r[x];
    }

    // passes 1-4: the blocks of the face neighbours (inflow faces, the
    // neighbour's equilibrium)
    for (int q = 0; q < 4; q++) {
        const int n = nb[q];
        const double *mn = d.mstate + kMacroState * (n >= 0 ? n : c);
        double Pn[4];
#pragma unroll
        for (int a = 0; a < 4; a++) Pn[a] = mn[a];
        const double kapn = Pn[0] / (2.0 * kPi * Pn[3]);
        __syncthreads();                         // the previous pass is done with the tables
        macro_tables(d, Pn, tabX[w], tabY[w]);
        __syncthreads();
        double Op[16];
#pragma unroll
        for (int i = 0; i < 16; i++) Op[i] = 0.0;
        if (n >= 0) {
            for (int k = lane; k < nv; k += kWave) {
                const int a = k % n1, b = k / n1;
                const double v1 = d.vx[a], v2 = d.vy[b];
                const double s = v1 * Sx[q] + v2 * Sy[q];
                if (s > 0) continue;
                const double wt = d.wx[a] * d.wy[b];
                const double psi[4] = {1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2)};
                double g1, g2, d1[4], d2[4];
                dg_dP(kapn, Pn, tabX[w][a], tabY[w][b], v1, v2, g1, g2, d1, d2);
#pragma unroll
                for (int x = 0; x < 4; x++)
#pragma unroll
                    for (int p = 0; p < 4; p++) Op[4 * x + p] += wt * s * (psi[x] * d1[p] + (x == 3 ? d2[p] : 0.0));
            }
        }
        wave_sum<16>(Op);
        if (act && lane == 0) {
            const double *Mn = mn + 4;
            double *Oq = d.mO + 64 * c + 16 * q;
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int m = 0; m < 4; m++)
                    Oq[4 * x + m] = n >= 0 ? ((Op[4 * x] * Mn[m] + Op[4 * x + 1] * Mn[4 + m]) + Op[4 * x + 2] * Mn[8 + m]) +
                                                 Op[4 * x + 3] * Mn[12 + m]
                                           : 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// one colour of a red-black block Gauss-Seidel step, a thread per cell
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_macro_rbgs(DevSolve d, int colour, const double *__restrict__ src,
                                                       double *__restrict__ dst)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    const int m = d.cell_of[c];
    const int i = m % d.ni, j = m / d.ni;
    if (((i + j) & 1) != colour) {
#pragma unroll
        for (int a = 0; a < 4; a++) dst[4 * c + a] = src[4 * c + a];
        return;
    }
    double b[4];
#pragma unroll
    for (int a = 0; a < 4; a++) b[a] = -d.mr[4 * c + a];
    for (int q = 0; q < 4; q++) {
        const int n = d.nbr[4 * c + q];
        if (n < 0) continue;
        const double *O = d.mO + 64 * c + 16 * q;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int e = 0; e < 4; e++) b[a] -= O[4 * a + e] * src[4 * n + e];
    }
    const double *Di = d.mDinv + 16 * c;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        double acc = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) acc += Di[4 * a + e] * b[e];
        dst[4 * c + a] = acc;
    }
}

__global__ __launch_bounds__(kBlock) void k_macro_zero(double *x, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

// W += dW, limited: rho and theta change by at most kMacroLimit
constexpr double kMacroLimit = 0.2;

__device__ __forceinline__ double theta_of(const double *W)
{
    const double u1 = W[1] / W[0], u2 = W[2] / W[0];
    return (2.0 / 3.0) * (W[3] / W[0] - 0.5 * (u1 * u1 + u2 * u2));
}

__global__ __launch_bounds__(kBlock) void k_macro_apply(DevSolve d, int par, const double *__restrict__ x)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    double *W = d.W[par] + 4 * c;
    double Wt[4];
#pragma unroll
    for (int a = 0; a < 4; a++) Wt[a] = W[a] + x[4 * c + a];
    const double th0 = theta_of(W), th1 = theta_of(Wt);
    const double ch = fmax(fabs(x[4 * c]) / W[0], fabs(th1 - th0) / th0);
    double fac = 0.0;
    if (Wt[0] > 0 && th1 > 0 && isfinite(ch)) fac = ch > kMacroLimit ? kMacroLimit / ch : 1.0;
#pragma unroll
    for (int a = 0; a < 4; a++) W[a] += fac * x[4 * c + a];
}

hipError_t launch_macro_predict(const DevSolve &d, int par, int inner, hipStream_t st)
{
    constexpr int per_block = kBlock / kWave;
    const int gw = (d.nc + per_block - 1) / per_block, gt = (d.nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_macro_state, dim3(gw), dim3(kBlock), 0, st, d, par);
    if (hipError_t e = hipGetLastError()) return e;
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_macro_assemble<T>, dim3(gw), dim3(kBlock), 0, st, d, par));
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_macro_zero, dim3((4 * d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d.mx[0], 4 * d.nc);
    if (hipError_t e = hipGetLastError()) return e;
    for (int it = 0; it < inner; it++) {
        hipLaunchKernelGGL(k_macro_rbgs, dim3(gt), dim3(kBlock), 0, st, d, 0, d.mx[0], d.mx[1]);
        hipLaunchKernelGGL(k_macro_rbgs, dim3(gt), dim3(kBlock), 0, st, d, 1, d.mx[1], d.mx[0]);
        if (hipError_t e = hipGetLastError()) return e;
    }
    hipLaunchKernelGGL(k_macro_apply, dim3(gt), dim3(kBlock), 0, st, d, par, d.mx[0]);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// adjoint prediction: the transpose of the primal's accelerated sweep.
// Linearised at the converged f, the primal sweep after a prediction is
// f' = f + D^-1 Q R'(f), Q = I - H L M (M the moments, L the Gauss-Seidel
// map above, H = dg/dW V/tau + (g - f) d(V/tau)/dW: how the predicted
// moments enter the sweep).  Its transpose for the adjoint equation is
// phi' = phi_s - Psi L^T (H^T (phi_s - phi)), phi_s the plain adjoint
// sweep's result: every K-th adjoint sweep
//   1. k_macro_adj_y: y = H^T (phi_s - phi) per cell, from the adjoint
//      moments the two sweeps left (What and rho_tau are linear in phi):
//      y = V (What_s - What) / tau - V (1/tau dtau/dW) (rho_tau,s - rho_tau);
//   2. k_macro_rbgs_adj: z = L^T y, the Gauss-Seidel half steps transposed
//      in reverse order (the neighbour blocks transposed once, at the
//      adjoint's start, by k_macro_transpose);
//   3. k_macro_adj_correct: phi_s -= (z . Psi, z_3), then the adjoint
//      moments of the corrected phi (k_adjoint_moments).
// The accelerated adjoint cycle then has the eigenvalues of the primal's,
// and the correction vanishes with the sweep's change (the adjoint solution
// is the plain iteration's).
// ---------------------------------------------------------------------------

// the transposed neighbour blocks: OT[c][q] = O[n][q']^T for the face q' of
// n = nbr[c][q] that faces c, a thread per cell
__global__ __launch_bounds__(kBlock) void k_macro_transpose(DevSolve d)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    for (int q = 0; q < 4; q++) {
        double *o = d.mOT + 64 * c + 16 * q;
        const int n = d.nbr[4 * c + q];
        int qb = -1;
        if (n >= 0)
            for (int t = 0; t < 4; t++)
                if (d.nbr[4 * n + t] == c) {
                    qb = t;
                    break;
                }
        const double *src = d.mO + 64 * (size_t)(n >= 0 ? n : c) + 16 * (qb >= 0 ? qb : 0);
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) o[4 * a + b] = qb >= 0 ? src[4 * b + a] : 0.0;
    }
}

// y_c = H_c^T (phi_s - phi) from the adjoint moments of phi_s (aW[pnew]) and
// of phi (aW[pnew ^ 1]), written as the seed of the transposed solve
__global__ __launch_bounds__(kBlock) void k_macro_adj_y(DevSolve d, int pnew, double *__restrict__ y)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= d.nc) return;
    const double *an = d.aW[pnew] + 8 * c, *ao = d.aW[pnew ^ 1] + 8 * c;
    const double *ac = d.acoef + kAcoef * c;
    const double V = d.vol[c], itau = ac[4], drt = an[4] - ao[4];
#pragma unroll
    for (int m = 0; m < 4; m++) y[4 * c + m] = V * (itau * (an[m] - ao[m]) - ac[6 + m] * drt);
}

__device__ __forceinline__ bool macro_colour(const DevSolve &d, int c, int colour)
{
    const int m = d.cell_of[c];
    return (((m % d.ni) + (m / d.ni)) & 1) == colour;
}

// one transposed half step of k_macro_rbgs (colour `colour`), a thread per
// cell: the forward step set x_c = Dinv_c (-r_c - sum_q O_cq src_nbr) on its
// colour and copied the rest; given the adjoint ob of its output, t_c =
// -Dinv_c^T ob_c joins rbar on the colour, and the adjoint of its input is
// ib_m = (m off the colour: ob_m) + sum_q OT_mq t_nbr (neighbours on the
// colour)
__global__ __launch_bounds__(kBlock) void k_macro_rbgs_adj(DevSolve d, int colour, const double *__restrict__ ob,
                                                           double *__restrict__ ib, double *__restrict__ rbar)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= d.nc) return;
    double acc[4];
    const bool on = macro_colour(d, m, colour);
#pragma unroll
    for (int a = 0; a < 4; a++) acc[a] = on ? 0.0 : ob[4 * m + a];
    for (int q = 0; q < 4; q++) {
        const int n = d.nbr[4 * m + q];
        if (n < 0 || !macro_colour(d, n, colour)) continue;
        const double *Di = d.mDinv + 16 * n;
        double t[4];
#pragma unroll
        for (int a = 0; a < 4; a++) {
            double s = 0;
#pragma unroll
            for (int e = 0; e < 4; e++) s += Di[4 * e + a] * ob[4 * n + e];
            t[a] = -s;
        }
        const double *OT = d.mOT + 64 * m + 16 * q;
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int e = 0; e < 4; e++) acc[a] += OT[4 * a + e] * t[e];
    }
#pragma unroll
    for (int a = 0; a < 4; a++) ib[4 * m + a] = acc[a];
    if (on) {
        const double *Di = d.mDinv + 16 * m;
#pragma unroll
        for (int a = 0; a < 4; a++) {
            double s = 0;
#pragma unroll
            for (int e = 0; e < 4; e++) s += Di[4 * e + a] * ob[4 * m + e];
            rbar[4 * m + a] -= s;
        }
    }
}

// phi[pnew] -= (z . Psi, z_3), a thread per (cell, velocity)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_macro_adj_correct(DevSolve d, int pnew, const double *__restrict__ z)
{
    using T2 = typename Vec2<T>::type;
    T2 *__restrict__ ph = static_cast<T2 *>(d.phi[pnew]);
    const size_t n = (size_t)d.nc * d.nv, stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int c = (int)(i / d.nv), k = (int)(i % d.nv);
        const double v1 = d.vx[k % d.n1], v2 = d.vy[k / d.n1];
        const double *zc = z + 4 * c;
        T2 p = ph[i];
        const double s1 = ((zc[0] + zc[1] * v1) + zc[2] * v2) + zc[3] * (0.5 * (v1 * v1 + v2 * v2));
        p.x = (T)((double)p.x - s1);
        p.y = (T)((double)p.y - zc[3]);
        ph[i] = p;
    }
}

hipError_t launch_macro_adjoint_setup(const DevSolve &d, int fpar, hipStream_t st)
{
    constexpr int per_block = kBlock / kWave;
    const int gw = (d.nc + per_block - 1) / per_block, gt = (d.nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_macro_state, dim3(gw), dim3(kBlock), 0, st, d, fpar);
    if (hipError_t e = hipGetLastError()) return e;
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_macro_assemble<T>, dim3(gw), dim3(kBlock), 0, st, d, fpar));
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_macro_transpose, dim3(gt), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_macro_adjoint_predict(const DevSolve &d, int pnew, int inner, hipStream_t st)
{
    const int gt = (d.nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_macro_adj_y, dim3(gt), dim3(kBlock), 0, st, d, pnew, d.mx[0]);
    hipLaunchKernelGGL(k_macro_zero, dim3((4 * d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d.mr, 4 * d.nc);
    if (hipError_t e = hipGetLastError()) return e;
    // the forward steps ran it = 0 .. inner-1, colour 0 (x -> y) then 1
    // (y -> x); here it = inner-1 .. 0, colour 1 (adjoint of x -> of y) then 0
    for (int it = 0; it < inner; it++) {
        hipLaunchKernelGGL(k_macro_rbgs_adj, dim3(gt), dim3(kBlock), 0, st, d, 1, d.mx[0], d.mx[1], d.mr);
        hipLaunchKernelGGL(k_macro_rbgs_adj, dim3(gt), dim3(kBlock), 0, st, d, 0, d.mx[1], d.mx[0], d.mr);
        if (hipError_t e = hipGetLastError()) return e;
    }
    const size_t pairs = (size_t)d.nc * d.nv;
    const int gp = (int)std::min<size_t>((pairs + kBlock - 1) / kBlock, 16384);
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_macro_adj_correct<T>, dim3(gp), dim3(kBlock), 0, st, d, pnew, d.mr));
    if (hipError_t e = hipGetLastError()) return e;
    return launch_adjoint_moments(d, pnew, st);
}

}  // namespace dvm
