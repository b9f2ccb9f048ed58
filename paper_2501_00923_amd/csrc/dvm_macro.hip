// Macroscopic prediction of the primal iteration (gfx950).
//
// Sec. 3.1 accelerates the kinetic iterations with "prediction" solutions of
// approximate macroscopic equations from the continuum limit.  Every K
// sweeps (first-order scheme):
//   1. k_eq_params: each cell's discrete-conservative equilibrium
//      parameters P' and dP'/dW by Newton;
//   2. k_macro_resid, k_macro_blocks: the moments r of the kinetic residual
//      of eq. (numerpr_gov) at the current f, and the linearised macroscopic
//      system A dW = -r with A the moments of the scheme's upwind transport of
//      equilibrium perturbations: the outflow faces carry the cell's own
//      dg/dW, the inflow faces the neighbour's, the far field nothing and
//      the wall face the diffuse value's response gbar dF_l; plus the
//      pseudo-time term (|u| + c) sum_q |S_q| / CFL (CFL 1000) on the
//      diagonal, which keeps near-singular modes of the steady operator (a
//      slow wake, a sonic region) from being amplified; stored as the
//      inverse of each cell's own block and the outflow block of each face
//      (the neighbours' inflow blocks);
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

constexpr double kMacroCFL = 1000.0;

// derivatives of (g1, g2) with respect to the equilibrium parameters
// (rho, u1, u2, theta) at velocity (v1, v2), with g1 = kap X Y from the tables
// (ir = 1/rho, it = 1/theta, ih = 1/(2 theta^2) of the cell, computed once)
struct DgCell {
    double kap, u1, u2, hth, ir, it, ih;
};

__device__ __forceinline__ DgCell dg_cell(const double *P)
{
    return {P[0] / (2.0 * kPi * P[3]), P[1], P[2], 0.5 * P[3], 1.0 / P[0], 1.0 / P[3], 1.0 / (2.0 * P[3] * P[3])};
}

__device__ __forceinline__ void dg_dP(const DgCell &q, double X, double Y, double v1, double v2, double &g1,
                                      double &g2, double (&d1)[4], double (&d2)[4])
{
    const double c1 = v1 - q.u1, c2 = v2 - q.u2;
    g1 = q.kap * X * Y;
    g2 = q.hth * g1;
    d1[0] = g1 * q.ir;
    d1[1] = g1 * c1 * q.it;
    d1[2] = g1 * c2 * q.it;
    d1[3] = g1 * ((c1 * c1 + c2 * c2) * q.ih - q.it);
#pragma unroll
    for (int p = 0; p < 4; p++) d2[p] = q.hth * d1[p];
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
// r_c, the moments of the kinetic residual at the current f, one wave per
// cell: the own row, the upwind neighbours' rows (far-field table, diffuse
// wall), the collision part V/tau (f - g).  A workgroup per sweep patch in
// the sweeps' XCD order, so neighbour rows are read from the XCD's own L2.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kPatchCells * kWave) void k_macro_resid(DevSolve d, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ double tabX[kPatchCells][kMaxN1D], tabY[kPatchCells][kMaxN1D];
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;                          // whole workgroups
    const int w = (int)(threadIdx.x / kWave), lane = threadIdx.x % kWave;
    const int c0 = d.patch[p], cnt = d.patch[p + 1] - c0;
    const bool act = w < cnt;                   // idle waves of a partial patch only join the barrier
    const int c = c0 + (act ? w : 0);
    const int nv = d.nv, n1 = d.n1;
    const T2 *__restrict__ f = static_cast<const T2 *>(d.f[par]);
    const T2 *__restrict__ fd = static_cast<const T2 *>(d.fd);
    const T *__restrict__ gM = static_cast<const T *>(d.gM);
    const double *ms = d.mstate + kEqState * c;
    const double P[4] = {ms[0], ms[1], ms[2], ms[3]};
    const double kap = P[0] / (2.0 * kPi * P[3]), th2 = 0.5 * P[3];
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
    const double thw2 = 0.5 * d.theta_w;
    const size_t row = (size_t)c * nv;
    // the 1-D velocity tables in LDS (threads 0 .. n1 + n2 - 1)
    __shared__ double svx[kMaxN1D], svy[kMaxN1D], swx[kMaxN1D], swy[kMaxN1D];
    {
        const int t = threadIdx.x, n2 = d.n2;
        if (t < n1) {
            svx[t] = d.vx[t];
            swx[t] = d.wx[t];
        } else if (t - n1 < n2) {
            svy[t - n1] = d.vy[t - n1];
            swy[t - n1] = d.wy[t - n1];
        }
    }
    macro_tables(d, P, tabX[w], tabY[w]);
    // one source row per face for its inflow velocities: the neighbour's
    // row or the far-field table (the wall's value is computed)
    const T2 *src[4];
#pragma unroll
    for (int q = 0; q < 4; q++) src[q] = nb[q] >= 0 ? f + (size_t)nb[q] * nv : (nb[q] == -1 ? fd : f + row);
    __syncthreads();
    double r[4] = {0, 0, 0, 0};
    int a = lane % n1, b = lane / n1;
    const int da = kWave % n1, db = kWave / n1;
    for (int k = lane; k < nv; k += kWave) {
        const double v1 = svx[a], v2 = svy[b], wt = swx[a] * swy[b];
        const double psi[4] = {1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2)};
        const double g1 = kap * tabX[w][a] * tabY[w][b], g2 = th2 * g1;
        // every load of this velocity before its arithmetic: the own row,
        // and each face's source row where the face is inflow
        const T2 fk = f[row + k];
        double s[4];
        T2 u[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            s[q] = v1 * Sx[q] + v2 * Sy[q];
            u[q] = T2{0, 0};
            if (!(s[q] > 0) && nb[q] >= -1) u[q] = src[q][k];
        }
        const double gw = wl >= 0 ? (double)gM[k] : 0.0;
        const double f1 = (double)fk.x, f2 = (double)fk.y;
        double in1 = Vt * (f1 - g1), in2 = Vt * (f2 - g2);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            double a1, a2;
            if (s[q] > 0) {
                a1 = f1;
                a2 = f2;
            } else if (nb[q] >= -1) {
                a1 = (double)u[q].x;
                a2 = (double)u[q].y;
            } else {
                const double gb1 = gw / Dw;
                a1 = Fw * gb1;
                a2 = Fw * (thw2 * gb1);
            }
            in1 += s[q] * a1;
            in2 += s[q] * a2;
        }
#pragma unroll
        for (int x = 0; x < 4; x++) r[x] += wt * (psi[x] * in1 + (x == 3 ? in2 : 0.0));
        a += da;
        b += db;
        if (a >= n1) {
            a -= n1;
            b++;
        }
    }
    wave_sum<4>(r);
    if (act && lane == 0) {
#pragma unroll
        for (int x = 0; x < 4; x++) d.mr[4 * c + x] = r[x];
    }
}

// ---------------------------------------------------------------------------
// the macroscopic blocks of each cell, two waves per cell (faces 0-1 and
// 2-3), no distribution read: each face q gets its outflow block
//   B_cq = sum_{k: v.S_q > 0} w (v.S_q) Psi_k dg_c,k/dW,
// and the cell's own block is D_c = sum_q B_cq + wall1 dF + lam I (wall1 dF:
// the diffuse wall's re-emission of the outgoing flux; lam the pseudo-time
// term).  The inflow block of the neighbour n across face q is -B_nq' (q'
// the face of n that faces c: S_nq' = -S_cq, so n's outflow half-space
// through q' is c's inflow half-space through q and the sums agree term by
// term).  The Gauss-Seidel steps read the neighbours' B instead of a
// separate off-diagonal table.
// ---------------------------------------------------------------------------
constexpr int kBlkCells = kBlock / (2 * kWave);

__global__ __launch_bounds__(kBlock) void k_macro_blocks(DevSolve d, int par)
{
    __shared__ double tabX[kBlkCells][kMaxN1D], tabY[kBlkCells][kMaxN1D];
    __shared__ double vx[kMaxN1D], vy[kMaxN1D], wx[kMaxN1D], wy[kMaxN1D];
    __shared__ double Dpart[kBlkCells][2][16];
    const int wv = (int)(threadIdx.x / kWave), lane = threadIdx.x % kWave;
    const int cl = wv >> 1, h = wv & 1;          // cell of the workgroup, half (faces 2h, 2h+1)
    const int c0 = blockIdx.x * kBlkCells + cl;
    const bool act = c0 < d.nc;                 // idle waves of the last workgroup only join the barriers
    const int c = act ? c0 : d.nc - 1;
    const int nv = d.nv, n1 = d.n1, n2 = d.n2;
    const double *ms = d.mstate + kEqState * c;
    const double P[4] = {ms[0], ms[1], ms[2], ms[3]};
    const DgCell qc = dg_cell(P);
    const double hh = 0.5 / P[3];
    for (int i = threadIdx.x; i < n1; i += kBlock) {
        vx[i] = d.vx[i];
        wx[i] = d.wx[i];
    }
    for (int i = threadIdx.x; i < n2; i += kBlock) {
        vy[i] = d.vy[i];
        wy[i] = d.wy[i];
    }
    // the cell's 1-D factor tables: X by the first wave of the cell, Y by the second
    if (h == 0)
        for (int i = lane; i < n1; i += kWave) {
            const double e = d.vx[i] - P[1];
            tabX[cl][i] = exp(-e * e * hh);
        }
    else
        for (int i = lane; i < n2; i += kWave) {
            const double e = d.vy[i] - P[2];
            tabY[cl][i] = exp(-e * e * hh);
        }
    double Sx[2], Sy[2];
#pragma unroll
    for (int t = 0; t < 2; t++) {
        Sx[t] = d.S[8 * c + 2 * (2 * h + t)];
        Sy[t] = d.S[8 * c + 2 * (2 * h + t) + 1];
    }
    const int nb0 = d.nbr[4 * c];
    const int wl = (h == 0 && nb0 <= -2) ? -2 - nb0 : -1;     // the wall face is face 0
    const double Dw = wl >= 0 ? d.D[wl] : 1.0;
    const double n1w = wl >= 0 ? d.wall_n[2 * wl] : 0.0, n2w = wl >= 0 ? d.wall_n[2 * wl + 1] : 0.0;
    const double thw2 = 0.5 * d.theta_w;
    const double *gMd = static_cast<const double *>(d.gM);
    const float *gMf = static_cast<const float *>(d.gM);
    __syncthreads();
    // Bp: B of the two faces in dg/dP form (2 x 16)
    double Bp[32];
#pragma unroll
    for (int i = 0; i < 32; i++) Bp[i] = 0.0;
    for (int k = lane; k < nv; k += kWave) {
        const int a = k % n1, b = k / n1;
        const double v1 = vx[a], v2 = vy[b], wt = wx[a] * wy[b];
        const double psi[4] = {1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2)};
        double g1, g2, d1[4], d2[4];
        dg_dP(qc, tabX[cl][a], tabY[cl][b], v1, v2, g1, g2, d1, d2);
        const double s0 = v1 * Sx[0] + v2 * Sy[0], s1 = v1 * Sx[1] + v2 * Sy[1];
        // B_q[x][p] += w s Psi_x dg1/dP_p (+ w s dg2/dP_p in row x = 3) for
        // each outflow face, as fused multiply-adds on (w s Psi_x)
#pragma unroll
        for (int t = 0; t < 2; t++) {
            const double st = t == 0 ? s0 : s1;
            if (st > 0) {
                const double ws = wt * st;
                double *Bq = Bp + 16 * t;
#pragma unroll
                for (int x = 0; x < 4; x++) {
                    const double wsp = ws * psi[x];
#pragma unroll
                    for (int p = 0; p < 4; p++) Bq[4 * x + p] = fma(wsp, d1[p], Bq[4 * x + p]);
                }
#pragma unroll
                for (int p = 0; p < 4; p++) Bq[12 + p] = fma(ws, d2[p], Bq[12 + p]);
            }
        }
    }
    wave_sum<32>(Bp);
    const double *M = ms + 4;
    if (act && lane == 0) {
        // this half's faces: B_q = Bp_q M into the table, and their share of D
        double Dm[16];
#pragma unroll
        for (int i = 0; i < 16; i++) Dm[i] = 0.0;
#pragma unroll
        for (int t = 0; t < 2; t++) {
            const double *Bq = Bp + 16 * t;
            double *Bo = d.mO + 64 * c + 16 * (2 * h + t);
#pragma unroll
            for (int x = 0; x < 4; x++)
#pragma unroll
                for (int m = 0; m < 4; m++) {
                    const double v = ((Bq[4 * x] * M[m] + Bq[4 * x + 1] * M[4 + m]) + Bq[4 * x + 2] * M[8 + m]) +
                                     Bq[4 * x + 3] * M[12 + m];
                    Bo[4 * x + m] = v;
                    Dm[4 * x + m] += v;
                }
        }
#pragma unroll
        for (int i = 0; i < 16; i++) Dpart[cl][h][i] = Dm[i];
    }
    // the wall face (face 0, first wave of a wall cell), in a loop of its
    // own so that the face sums above need not stay live beside its sums:
    // where the face is inflow, the diffuse value's response wall1; the
    // outgoing flux's response dF (dg/dP form)
    if (wl >= 0) {
        double wacc[8];
#pragma unroll
        for (int i = 0; i < 8; i++) wacc[i] = 0.0;
        double *wall1 = wacc, *dFp = wacc + 4;
        for (int k = lane; k < nv; k += kWave) {
            const int a = k % n1, b = k / n1;
            const double v1 = vx[a], v2 = vy[b], wt = wx[a] * wy[b];
            const double psi[4] = {1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2)};
            double g1, g2, d1[4], d2[4];
            dg_dP(qc, tabX[cl][a], tabY[cl][b], v1, v2, g1, g2, d1, d2);
            const double s = v1 * Sx[0] + v2 * Sy[0];
            if (!(s > 0)) {
                const double gb1 = (d.mixed ? (double)gMf[k] : gMd[k]) / Dw, gb2 = thw2 * gb1;
#pragma unroll
                for (int x = 0; x < 4; x++) wall1[x] += wt * s * (psi[x] * gb1 + (x == 3 ? gb2 : 0.0));
            }
            const double vn = v1 * n1w + v2 * n2w;
            if (vn > 0) {
#pragma unroll
                for (int p = 0; p < 4; p++) dFp[p] += wt * vn * d1[p];
            }
        }
        wave_sum<8>(wacc);
        if (act && lane == 0) {
#pragma unroll
            for (int m = 0; m < 4; m++) {
                const double dF = ((dFp[0] * M[m] + dFp[1] * M[4 + m]) + dFp[2] * M[8 + m]) + dFp[3] * M[12 + m];
#pragma unroll
                for (int x = 0; x < 4; x++) Dpart[cl][h][4 * x + m] += wall1[x] * dF;
            }
        }
    }
    __syncthreads();
    if (!act || h != 0 || lane != 0) return;
    // D = both halves + the pseudo-time term V/dt of the cell, inverted
    const double *W = d.W[par] + 4 * c;
    const double rho = W[0], u1 = W[1] / rho, u2 = W[2] / rho;
    const double th = (2.0 / 3.0) * (W[3] / rho - 0.5 * (u1 * u1 + u2 * u2));
    double sS = 0.0;
#pragma unroll
    for (int q = 0; q < 4; q++) sS += hypot(d.S[8 * c + 2 * q], d.S[8 * c + 2 * q + 1]);
    const double lam = (sqrt(u1 * u1 + u2 * u2) + sqrt(5.0 / 3.0 * th)) * sS / kMacroCFL;
    double Dm[4][4];
#pragma unroll
    for (int x = 0; x < 4; x++)
#pragma unroll
        for (int m = 0; m < 4; m++) Dm[x][m] = Dpart[cl][0][4 * x + m] + Dpart[cl][1][4 * x + m] + (x == m ? lam : 0.0);
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
}

// the face of cell n that faces cell c (n a face neighbour of c)
__device__ __forceinline__ int back_face(const DevSolve &d, int n, int c)
{
    int qb = 0;
#pragma unroll
    for (int t = 3; t >= 0; t--)
        if (d.nbr[4 * n + t] == c) qb = t;
    return qb;
}

// ---------------------------------------------------------------------------
// one colour of a red-black block Gauss-Seidel step for cell c: on its colour
// x_c = Dinv_c (-r_c - sum_q O_cq src_nbr), the rest copied.  The cell's four
// components sit on four lanes (component a = lane % 4): each lane sums its
// row of the neighbours' blocks, the lanes exchange the right-hand side and
// each applies its row of D^-1, so a launch has four threads per cell (the
// kernel is latency-bound: one thread per cell gives 2 waves per CU on
// 32,768 cells).  All four lanes of a cell take the same branches; callers
// launch whole cells.
// ---------------------------------------------------------------------------
static_assert(kBlock % 4 == 0, "the Gauss-Seidel launches keep a cell's four lanes in one workgroup");
__device__ __forceinline__ void rbgs_cell(const DevSolve &d, int c, int a, int colour, const double *__restrict__ src,
                                           double *__restrict__ dst)
{
    const int m = d.cell_of[c];
    const int i = m % d.ni, j = m / d.ni;
    if (((i + j) & 1) != colour) {
        dst[4 * c + a] = src[4 * c + a];
        return;
    }
    double ba = -d.mr[4 * c + a];
    for (int q = 0; q < 4; q++) {
        const int n = d.nbr[4 * c + q];
        if (n < 0) continue;
        // the inflow block of n across face q is -B_nq'
        const double *B = d.mO + 64 * n + 16 * back_face(d, n, c);
#pragma unroll
        for (int e = 0; e < 4; e++) ba += B[4 * a + e] * src[4 * n + e];
    }
    double b[4];
#pragma unroll
    for (int e = 0; e < 4; e++) b[e] = __shfl(ba, e, 4);
    const double *Di = d.mDinv + 16 * c;
    double acc = 0;
#pragma unroll
    for (int e = 0; e < 4; e++) acc += Di[4 * a + e] * b[e];
    dst[4 * c + a] = acc;
}

__global__ __launch_bounds__(kBlock) void k_macro_rbgs(DevSolve d, int colour, const double *__restrict__ src,
                                                       double *__restrict__ dst)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;     // 4 lanes per cell
    if ((t >> 2) < d.nc) rbgs_cell(d, t >> 2, t & 3, colour, src, dst);
}

// Several solves of a batch in one launch: a thread per cell of the
// group's members in turn (member a owns cells pre[a] .. pre[a+1]-1), each
// member's DevSolve read from the batch's table; the per-cell arithmetic
// is the single-solve kernel's, so the results are bitwise the same.
__global__ __launch_bounds__(kBlock) void k_macro_rbgs_group(const DevSolve *__restrict__ tab, MacroGroup g,
                                                             int colour, int from)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;     // 4 lanes per cell
    const int i = t >> 2;
    if (i >= g.pre[g.n]) return;
    const int a = group_member(g, i);
    const DevSolve &d = tab[g.idx[a]];
    rbgs_cell(d, i - g.pre[a], t & 3, colour, d.mx[from], d.mx[from ^ 1]);
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

// P' and dP'/dW of W[par], then the blocks; with_r: also the residual's moments
static hipError_t macro_system(const DevSolve &d, int par, bool with_r, hipStream_t st)
{
    if (hipError_t e = launch_eq_params(d, par, 1, st)) return e;
    if (with_r) {
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_macro_resid<T>, dim3(xcd_grid(d.np)), dim3(kPatchCells * kWave), 0,
                                                 st, d, par));
        if (hipError_t e = hipGetLastError()) return e;
    }
    hipLaunchKernelGGL(k_macro_blocks, dim3((d.nc + kBlkCells - 1) / kBlkCells), dim3(kBlock), 0, st, d, par);
    return hipGetLastError();
}

hipError_t launch_macro_predict_begin(const DevSolve &d, int par, hipStream_t st)
{
    if (hipError_t e = macro_system(d, par, true, st)) return e;
    hipLaunchKernelGGL(k_macro_zero, dim3((4 * d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d.mx[0], 4 * d.nc);
    return hipGetLastError();
}

hipError_t launch_macro_predict_end(const DevSolve &d, int par, hipStream_t st)
{
    hipLaunchKernelGGL(k_macro_apply, dim3((d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d, par, d.mx[0]);
    return hipGetLastError();
}

hipError_t launch_macro_predict(const DevSolve &d, int par, int inner, hipStream_t st)
{
    const int gt = (4 * d.nc + kBlock - 1) / kBlock;          // k_macro_rbgs: 4 lanes per cell
    if (hipError_t e = launch_macro_predict_begin(d, par, st)) return e;
    for (int it = 0; it < inner; it++) {
        hipLaunchKernelGGL(k_macro_rbgs, dim3(gt), dim3(kBlock), 0, st, d, 0, d.mx[0], d.mx[1]);
        hipLaunchKernelGGL(k_macro_rbgs, dim3(gt), dim3(kBlock), 0, st, d, 1, d.mx[1], d.mx[0]);
        if (hipError_t e = hipGetLastError()) return e;
    }
    return launch_macro_predict_end(d, par, st);
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
//      in reverse order;
//   3. k_adjoint_correct_moments: phi_s -= (z . Psi, z_3) and the adjoint
//      moments of the corrected phi, in one pass.
// The accelerated adjoint cycle then has the eigenvalues of the primal's,
// and the correction vanishes with the sweep's change (the adjoint solution
// is the plain iteration's).
// ---------------------------------------------------------------------------

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

// one transposed half step of k_macro_rbgs (colour `colour`) for cell m: the
// forward step set x_c = Dinv_c (-r_c - sum_q O_cq src_nbr) on its colour and
// copied the rest; given the adjoint ob of its output, t_c = -Dinv_c^T ob_c
// joins rbar on the colour, and the adjoint of its input is
// ib_m = (m off the colour: ob_m) + sum_q O_nq'^T t_n over neighbours n on
// the colour, where O_nq' (n's inflow block from m) is -B_mq.  Four lanes
// per cell as in rbgs_cell: lane a computes component a of each t_n, the
// lanes exchange t_n, and each accumulates its component of ib_m and rbar_m
// (the sums in the order of one thread per cell: bitwise the same).
__device__ __forceinline__ void rbgs_adj_cell(const DevSolve &d, int m, int a, int colour,
                                              const double *__restrict__ ob, double *__restrict__ ib,
                                              double *__restrict__ rbar)
{
    const bool on = macro_colour(d, m, colour);
    double acc = on ? 0.0 : ob[4 * m + a];
    for (int q = 0; q < 4; q++) {
        const int n = d.nbr[4 * m + q];
        if (n < 0 || !macro_colour(d, n, colour)) continue;
        const double *Di = d.mDinv + 16 * n;
        double s = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) s += Di[4 * e + a] * ob[4 * n + e];
        const double ta = -s;
        double t[4];
#pragma unroll
        for (int e = 0; e < 4; e++) t[e] = __shfl(ta, e, 4);
        const double *B = d.mO + 64 * m + 16 * q;
#pragma unroll
        for (int e = 0; e < 4; e++) acc -= B[4 * e + a] * t[e];
    }
    ib[4 * m + a] = acc;
    if (on) {
        const double *Di = d.mDinv + 16 * m;
        double s = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) s += Di[4 * e + a] * ob[4 * m + e];
        rbar[4 * m + a] -= s;
    }
}

__global__ __launch_bounds__(kBlock) void k_macro_rbgs_adj(DevSolve d, int colour, const double *__restrict__ ob,
                                                           double *__restrict__ ib, double *__restrict__ rbar)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;     // 4 lanes per cell
    if ((t >> 2) < d.nc) rbgs_adj_cell(d, t >> 2, t & 3, colour, ob, ib, rbar);
}

__global__ __launch_bounds__(kBlock) void k_macro_rbgs_adj_group(const DevSolve *__restrict__ tab, MacroGroup g,
                                                                 int colour, int from)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;     // 4 lanes per cell
    const int i = t >> 2;
    if (i >= g.pre[g.n]) return;
    const int a = group_member(g, i);
    const DevSolve &d = tab[g.idx[a]];
    rbgs_adj_cell(d, i - g.pre[a], t & 3, colour, d.mx[from], d.mx[from ^ 1], d.mr);
}

hipError_t launch_macro_adjoint_setup(const DevSolve &d, int fpar, hipStream_t st)
{
    return macro_system(d, fpar, false, st);
}

hipError_t launch_macro_adjoint_begin(const DevSolve &d, int pnew, hipStream_t st)
{
    const int gt = (d.nc + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_macro_adj_y, dim3(gt), dim3(kBlock), 0, st, d, pnew, d.mx[0]);
    hipLaunchKernelGGL(k_macro_zero, dim3((4 * d.nc + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d.mr, 4 * d.nc);
    return hipGetLastError();
}

hipError_t launch_macro_adjoint_end(const DevSolve &d, int pnew, hipStream_t st)
{
    // phi -= (z . Psi, z_3) and the adjoint moments of the result, one pass
    return launch_adjoint_correct_moments(d, pnew, d.mr, st);
}

hipError_t launch_macro_adjoint_predict(const DevSolve &d, int pnew, int inner, hipStream_t st)
{
    const int gt = (4 * d.nc + kBlock - 1) / kBlock;          // k_macro_rbgs_adj: 4 lanes per cell
    if (hipError_t e = launch_macro_adjoint_begin(d, pnew, st)) return e;
    // the forward steps ran it = 0 .. inner-1, colour 0 (x -> y) then 1
    // (y -> x); here it = inner-1 .. 0, colour 1 (adjoint of x -> of y) then 0
    for (int it = 0; it < inner; it++) {
        hipLaunchKernelGGL(k_macro_rbgs_adj, dim3(gt), dim3(kBlock), 0, st, d, 1, d.mx[0], d.mx[1], d.mr);
        hipLaunchKernelGGL(k_macro_rbgs_adj, dim3(gt), dim3(kBlock), 0, st, d, 0, d.mx[1], d.mx[0], d.mr);
        if (hipError_t e = hipGetLastError()) return e;
    }
    return launch_macro_adjoint_end(d, pnew, st);
}

// the Gauss-Seidel steps of a group of batch members with the same inner
// count, one launch per half step for the whole group
hipError_t launch_macro_gs_group(const DevSolve *tab, const MacroGroup &g, int inner, int adjoint, hipStream_t st)
{
    if (g.n <= 0) return hipSuccess;
    const int gt4 = (4 * g.pre[g.n] + kBlock - 1) / kBlock;  // 4 lanes per cell
    for (int it = 0; it < inner; it++) {
        if (adjoint) {
            hipLaunchKernelGGL(k_macro_rbgs_adj_group, dim3(gt4), dim3(kBlock), 0, st, tab, g, 1, 0);
            hipLaunchKernelGGL(k_macro_rbgs_adj_group, dim3(gt4), dim3(kBlock), 0, st, tab, g, 0, 1);
        } else {
            hipLaunchKernelGGL(k_macro_rbgs_group, dim3(gt4), dim3(kBlock), 0, st, tab, g, 0, 0);
            hipLaunchKernelGGL(k_macro_rbgs_group, dim3(gt4), dim3(kBlock), 0, st, tab, g, 1, 1);
        }
        if (hipError_t e = hipGetLastError()) return e;
    }
    return hipSuccess;
}

}  // namespace dvm
