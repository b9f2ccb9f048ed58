// HIP kernels of libdvm for the shape derivative: the wall sensitivity of
// Sec. 3.2 (paper mode) and the exact discrete derivative in the mesh node
// coordinates.  Each runs once per solve, after the adjoint.

#include <math.h>

#include "dvm_device.h"

namespace dvm {

// ---------------------------------------------------------------------------
// wall sensitivity, eqs. (sens_J_itf), (gaussgrad), (sens_B_itf): one block
// per wall element.  SO (second-order scheme): the formulas take that
// scheme's values -- wall and face values reconstructed on the upwind side
// from the slopes G of f (k_so_slope of the same f, which also leaves dF)
// and the wall flux F + dF.
// ---------------------------------------------------------------------------
template <typename T, bool SO>
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
    const double iD = 1.0 / d.D[l], F = SO ? d.F[fpar][l] + d.dF[l] : d.F[fpar][l], thw2 = 0.5 * d.theta_w;
    const double iV = 1.0 / d.vol[c];
    const T2 *G = static_cast<const T2 *>(d.G);
    int nb[4];
    double Sx[4], Sy[4], rx[4] = {}, ry[4] = {}, nx[4] = {}, ny[4] = {};
    for (int q = 0; q < 4; q++) {
        nb[q] = d.nbr[4 * c + q];
        Sx[q] = d.S[8 * c + 2 * q];
        Sy[q] = d.S[8 * c + 2 * q + 1];
        if (SO) {
            rx[q] = d.rf[8 * c + 2 * q];
            ry[q] = d.rf[8 * c + 2 * q + 1];
            nx[q] = d.rn[8 * c + 2 * q];
            ny[q] = d.rn[8 * c + 2 * q + 1];
        }
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
        T2 gc1 = {0, 0}, gc2 = {0, 0};
        if (SO) {
            gc1 = G[2 * (row + k)];
            gc2 = G[2 * (row + k) + 1];
        }
        // the outgoing wall value: the cell value, reconstructed at order 2
        const double f1l = vn > 0 ? (double)fc.x + (SO ? (double)(gc1.x * (T)rx[0] + gc1.y * (T)ry[0]) : 0.0) : gw1;
        // Green-Gauss gradient with the scheme's upwind face values
        double g10 = 0, g11 = 0, g20 = 0, g21 = 0;
        for (int q = 0; q < 4; q++) {
            const double s = v1 * Sx[q] + v2 * Sy[q];
            double a1, a2;
            if (s > 0) {
                a1 = (double)fc.x;
                a2 = (double)fc.y;
                if (SO) {
                    a1 += (double)(gc1.x * (T)rx[q] + gc1.y * (T)ry[q]);
                    a2 += (double)(gc2.x * (T)rx[q] + gc2.y * (T)ry[q]);
                }
            } else if (nb[q] >= 0) {
                const size_t nr = (size_t)nb[q] * d.nv + k;
                const T2 u = f[nr];
                a1 = (double)u.x;
                a2 = (double)u.y;
                if (SO) {
                    const T2 h1 = G[2 * nr], h2 = G[2 * nr + 1];
                    a1 += (double)(h1.x * (T)nx[q] + h1.y * (T)ny[q]);
                    a2 += (double)(h2.x * (T)nx[q] + h2.y * (T)ny[q]);
                }
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
// exact discrete shape derivative: dL/d(node coordinates) of the Lagrangian
// L = J + sum_{c,k} w_k phi_{c,k} . R_{c,k}, with R the residual of eq.
// (numerpr_gov) and J that of eq. (numer_J), f and phi held fixed.  At
// converged f and phi this is dJ/dx of the discrete problem under mesh
// motion, the volume-mesh terms included (the wall-only derivative of
// Sec. 2.5 leaves them out).  Per cell: G_q = dL/dS_q = sum_k w v
// (phi . f_face) for each face vector (upwind face values), H = dL/dV =
// sum_k w phi . (f - g) / tau; chained to the cell's corners through
// S_q = (y_{q+1} - y_q, -(x_{q+1} - x_q)) and V = (d1 x d2)/2, d1 = x_2 - x_0,
// d2 = x_3 - x_1.  Per wall element: the dependence of the diffuse wall
// value F_l/D_l and of J_l on the element's normal and length.  Per node:
// the sum over the cells that have it as a corner, in a fixed order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mesh_sens_cell(DevSolve d, int fpar, int ppar)
{
    using T2 = typename Vec2<T>::type;
    const int w = (int)(threadIdx.x / kWave), lane = threadIdx.x % kWave;
    const int c = blockIdx.x * (kBlock / kWave) + w;
    if (c >= d.nc) return;                      // whole waves; the kernel has no block barrier
    const int nv = d.nv, n1 = d.n1;
    const T2 *f = static_cast<const T2 *>(d.f[fpar]);
    const T2 *ph = static_cast<const T2 *>(d.phi[ppar]);
    const T2 *fd = static_cast<const T2 *>(d.fd);
    const T *gM = static_cast<const T *>(d.gM);
    // the frozen state's equilibrium (parameters and 1/tau from the adjoint
    // coefficients)
    const double *ac = d.acoef + kAcoef * c;
    const double u1 = ac[1], u2 = ac[2], th = ac[3], itau = ac[4], gc = ac[5];
    int nb[4];
    double Sx[4], Sy[4];
    for (int q = 0; q < 4; q++) {
        nb[q] = d.nbr[4 * c + q];
        Sx[q] = d.S[8 * c + 2 * q];
        Sy[q] = d.S[8 * c + 2 * q + 1];
    }
    const int wl = nb[0] <= -2 ? -2 - nb[0] : -1;
    const double rw = wl >= 0 ? d.F[fpar][wl] / d.D[wl] : 0.0;
    const double thw2 = 0.5 * d.theta_w;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // G_0..G_3 (x, y), H
    const size_t row = (size_t)c * nv;
    for (int k = lane; k < nv; k += kWave) {
        const int a = k % n1, b = k / n1;
        const double v1 = d.vx[a], v2 = d.vy[b], wt = d.wx[a] * d.wy[b];
        const T2 fc = f[row + k], pc = ph[row + k];
        const double f1 = (double)fc.x, f2 = (double)fc.y, p1 = (double)pc.x, p2 = (double)pc.y;
        for (int q = 0; q < 4; q++) {
            const double s = v1 * Sx[q] + v2 * Sy[q];
            double a1, a2;
            if (s > 0) {
                a1 = f1;
                a2 = f2;
            } else if (nb[q] >= 0) {
                const T2 u = f[(size_t)nb[q] * nv + k];
                a1 = (double)u.x;
                a2 = (double)u.y;
            } else if (nb[q] == -1) {
                const T2 u = fd[k];
                a1 = (double)u.x;
                a2 = (double)u.y;
            } else {
                a1 = rw * (double)gM[k];
                a2 = thw2 * a1;
            }
            const double pa = wt * (p1 * a1 + p2 * a2);
            acc[2 * q] += pa * v1;
            acc[2 * q + 1] += pa * v2;
        }
        const double e1 = v1 - u1, e2 = v2 - u2;
        const double g1 = gc * exp(-(e1 * e1 + e2 * e2) / (2.0 * th)), g2 = 0.5 * th * g1;
        acc[8] += wt * itau * (p1 * (f1 - g1) + p2 * (f2 - g2));
    }
    wave_sum<9>(acc);
    if (lane == 0) {
        double cx[4] = {0, 0, 0, 0}, cy[4] = {0, 0, 0, 0};   // dL/dx, dL/dy of corners 0..3
        for (int q = 0; q < 4; q++) {
            const int r = (q + 1) & 3;
            cx[q] += acc[2 * q + 1];
            cx[r] -= acc[2 * q + 1];
            cy[q] -= acc[2 * q];
            cy[r] += acc[2 * q];
        }
        // corner edges e_q = x_{q+1} - x_q = (-S_q,y, S_q,x); d1 = e0 + e1, d2 = e1 + e2
        const double d1x = -(Sy[0] + Sy[1]), d1y = Sx[0] + Sx[1];
        const double d2x = -(Sy[1] + Sy[2]), d2y = Sx[1] + Sx[2];
        const double H = 0.5 * acc[8];
        cx[0] -= H * d2y;
        cx[1] += H * d1y;
        cx[2] += H * d2y;
        cx[3] -= H * d1y;
        cy[0] += H * d2x;
        cy[1] -= H * d1x;
        cy[2] -= H * d2x;
        cy[3] += H * d1x;
        double *o = d.msens + 8 * d.cell_of[c];
        for (int q = 0; q < 4; q++) {
            o[2 * q] = cx[q];
            o[2 * q + 1] = cy[q];
        }
    }
}

// Second-order scheme.  The area centroid of a quadrilateral from its
// corners relative to corner 0 (the two triangles (0,1,2), (0,2,3)), on
// values carrying one derivative direction.
struct Dual {
    double v, d;
};
__device__ __forceinline__ Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }

__device__ void centroid_rel(const Dual (&X)[4], const Dual (&Y)[4], Dual &cx, Dual &cy)
{
    const Dual r1x = X[1] - X[0], r1y = Y[1] - Y[0], r2x = X[2] - X[0], r2y = Y[2] - Y[0];
    const Dual r3x = X[3] - X[0], r3y = Y[3] - Y[0];
    const Dual a1 = r1x * r2y - r1y * r2x, a2 = r2x * r3y - r2y * r3x;
    const Dual three = {3.0, 0.0}, den = three * (a1 + a2);
    cx = (a1 * (r1x + r2x) + a2 * (r2x + r3x)) / den;
    cy = (a1 * (r1y + r2y) + a2 * (r2y + r3y)) / den;
}

// Second-order scheme, one wave per cell c: dL/d(c's geometry) with f, phi
// and the limiter factors psi of f fixed.  L reads c's face vectors S_q
// (the face fluxes, with the reconstructed face values, and the slopes
// G_c = psi (1/V) sum_q fbar_q S_q), its volume (the collision term and
// G_c), its face midpoints m_q (the values reconstructed at them for c's
// own balance, and at the wall for F_l and J_l too) and its centroid x_c
// (the values c sends through its outflow faces, into its own balance and
// its downstream neighbour's).  Per outflow face the weight of a sent value
// is phi_c - phi_down: the neighbour's phi, 0 at the far field,
// (Phi_l - m_J, 0) at the wall (Phi_l: the wall multiplier of this phi).
// The per-face and per-cell sums are mapped to c's four corners.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mesh_sens_cell_so(DevSolve d, int fpar, int ppar)
{
    using T2 = typename Vec2<T>::type;
    const int w = (int)(threadIdx.x / kWave), lane = threadIdx.x % kWave;
    const int c = blockIdx.x * (kBlock / kWave) + w;
    if (c >= d.nc) return;                      // whole waves; the kernel has no block barrier
    const int nv = d.nv, n1 = d.n1, obj = d.objective;
    const T2 *f = static_cast<const T2 *>(d.f[fpar]);
    const T2 *ph = static_cast<const T2 *>(d.phi[ppar]);
    const T2 *fd = static_cast<const T2 *>(d.fd);
    const T *gM = static_cast<const T *>(d.gM);
    const T *Gs = static_cast<const T *>(d.G);
    const T2 *ps = static_cast<const T2 *>(d.psi);
    // the frozen state's equilibrium (parameters and 1/tau from the adjoint
    // coefficients)
    const double *ac = d.acoef + kAcoef * c;
    const double u1 = ac[1], u2 = ac[2], th = ac[3], itau = ac[4], gc = ac[5];
    int nb[4];
    double Sx[4], Sy[4], rfx[4], rfy[4], rnx[4], rny[4];
    for (int q = 0; q < 4; q++) {
        nb[q] = d.nbr[4 * c + q];
        Sx[q] = d.S[8 * c + 2 * q];
        Sy[q] = d.S[8 * c + 2 * q + 1];
        rfx[q] = d.rf[8 * c + 2 * q];
        rfy[q] = d.rf[8 * c + 2 * q + 1];
        rnx[q] = d.rn[8 * c + 2 * q];
        rny[q] = d.rn[8 * c + 2 * q + 1];
    }
    const int wl = nb[0] <= -2 ? -2 - nb[0] : -1;
    const double rw = wl >= 0 ? (d.F[fpar][wl] + d.dF[wl]) / d.D[wl] : 0.0;
    const double Phi = wl >= 0 ? d.Phi[ppar][wl] : 0.0;
    const double thw2 = 0.5 * d.theta_w;
    // dL/dS_q direct (8), dL/dm_q (8), dL/dx_c (2), dL/dS_q through G_c times V (8),
    // dL/dV direct (1), dL/dV through G_c times -V (1)
    double acc[28] = {};
    const size_t row = (size_t)c * nv;
    for (int k = lane; k < nv; k += kWave) {
        const int a = k % n1, b = k / n1;
        const double v1 = d.vx[a], v2 = d.vy[b], wt = d.wx[a] * d.wy[b];
        const double mj = mJ_of(obj, v1, v2);
        const T2 fc = f[row + k], pc = ph[row + k], pk = ps[row + k];
        const double f1 = (double)fc.x, f2 = (double)fc.y, p1 = (double)pc.x, p2 = (double)pc.y;
        const T *gk = Gs + 4 * (row + k);
        const double g1x = (double)gk[0], g1y = (double)gk[1], g2x = (double)gk[2], g2y = (double)gk[3];
        double P1x = 0, P1y = 0, P2x = 0, P2y = 0, fb1[4], fb2[4];
        for (int q = 0; q < 4; q++) {
            const double s = v1 * Sx[q] + v2 * Sy[q];
            double fn1 = f1, fn2 = f2;
            if (nb[q] >= 0) {
                const T2 u = f[(size_t)nb[q] * nv + k];
                fn1 = (double)u.x;
                fn2 = (double)u.y;
                fb1[q] = 0.5 * (f1 + fn1);
                fb2[q] = 0.5 * (f2 + fn2);
            } else {
                fb1[q] = f1;
                fb2[q] = f2;
            }
            double a1, a2;
            if (s > 0) {
                a1 = f1 + g1x * rfx[q] + g1y * rfy[q];
                a2 = f2 + g2x * rfx[q] + g2y * rfy[q];
                double d1 = 0, d2 = 0;
                if (nb[q] >= 0) {
                    const T2 pn = ph[(size_t)nb[q] * nv + k];
                    d1 = (double)pn.x;
                    d2 = (double)pn.y;
                } else if (nb[q] <= -2) {
                    d1 = Phi - mj;
                }
                const double e1 = p1 - d1, e2 = p2 - d2;
                const double m1 = nb[q] <= -2 ? e1 : p1, m2 = nb[q] <= -2 ? e2 : p2;
                acc[8 + 2 * q] += wt * s * (m1 * g1x + m2 * g2x);
                acc[8 + 2 * q + 1] += wt * s * (m1 * g1y + m2 * g2y);
                acc[16] -= wt * s * (e1 * g1x + e2 * g2x);
                acc[17] -= wt * s * (e1 * g1y + e2 * g2y);
                P1x += s * e1 * rfx[q];
                P1y += s * e1 * rfy[q];
                P2x += s * e2 * rfx[q];
                P2y += s * e2 * rfy[q];
            } else if (nb[q] >= 0) {
                const T *gn = Gs + 4 * ((size_t)nb[q] * nv + k);
                const double n1x = (double)gn[0], n1y = (double)gn[1], n2x = (double)gn[2], n2y = (double)gn[3];
                a1 = fn1 + n1x * rnx[q] + n1y * rny[q];
                a2 = fn2 + n2x * rnx[q] + n2y * rny[q];
                acc[8 + 2 * q] += wt * s * (p1 * n1x + p2 * n2x);
                acc[8 + 2 * q + 1] += wt * s * (p1 * n1y + p2 * n2y);
            } else if (nb[q] == -1) {
                const T2 u = fd[k];
                a1 = (double)u.x;
                a2 = (double)u.y;
            } else {
                a1 = rw * (double)gM[k];
                a2 = thw2 * a1;
            }
            const double pa = wt * (p1 * a1 + p2 * a2);
            acc[2 * q] += pa * v1;
            acc[2 * q + 1] += pa * v2;
        }
        // through G_c: dG[m][x]/dS_q[x] = psi_m fbar_q[m] / V, dG/dV = -G / V
        const double q1 = wt * (double)pk.x, q2 = wt * (double)pk.y;
        for (int q = 0; q < 4; q++) {
            acc[18 + 2 * q] += P1x * q1 * fb1[q] + P2x * q2 * fb2[q];
            acc[18 + 2 * q + 1] += P1y * q1 * fb1[q] + P2y * q2 * fb2[q];
        }
        acc[27] += wt * (P1x * g1x + P1y * g1y + P2x * g2x + P2y * g2y);
        const double e1 = v1 - u1, e2 = v2 - u2;
        const double g1 = gc * exp(-(e1 * e1 + e2 * e2) / (2.0 * th)), g2 = 0.5 * th * g1;
        acc[26] += wt * itau * (p1 * (f1 - g1) + p2 * (f2 - g2));
    }
    wave_sum<28>(acc);
    if (lane == 0) {
        const double iV = 1.0 / d.vol[c];
        double cx[4] = {0, 0, 0, 0}, cy[4] = {0, 0, 0, 0};   // dL/dx, dL/dy of corners 0..3
        for (int q = 0; q < 4; q++) {
            const int r = (q + 1) & 3;
            const double gSx = acc[2 * q] + acc[18 + 2 * q] * iV, gSy = acc[2 * q + 1] + acc[18 + 2 * q + 1] * iV;
            cx[q] += gSy;
            cx[r] -= gSy;
            cy[q] -= gSx;
            cy[r] += gSx;
            // face midpoint: half to each end of the face
            cx[q] += 0.5 * acc[8 + 2 * q];
            cx[r] += 0.5 * acc[8 + 2 * q];
            cy[q] += 0.5 * acc[8 + 2 * q + 1];
            cy[r] += 0.5 * acc[8 + 2 * q + 1];
        }
        // volume: corner edges e_q = x_{q+1} - x_q = (-S_q,y, S_q,x); d1 = e0 + e1, d2 = e1 + e2
        const double d1x = -(Sy[0] + Sy[1]), d1y = Sx[0] + Sx[1];
        const double d2x = -(Sy[1] + Sy[2]), d2y = Sx[1] + Sx[2];
        const double H = 0.5 * (acc[26] - acc[27] * iV);
        cx[0] -= H * d2y;
        cx[1] += H * d1y;
        cx[2] += H * d2y;
        cx[3] -= H * d1y;
        cy[0] += H * d2x;
        cy[1] -= H * d1x;
        cy[2] -= H * d2x;
        cy[3] += H * d1x;
        // centroid: derivatives with respect to corners 1..3 (relative to
        // corner 0, rebuilt from the edges); corner 0 by translation invariance
        const double ex[3] = {-Sy[0], -Sy[1], -Sy[2]}, ey[3] = {Sx[0], Sx[1], Sx[2]};
        double X[4] = {0, ex[0], ex[0] + ex[1], ex[0] + ex[1] + ex[2]};
        double Y[4] = {0, ey[0], ey[0] + ey[1], ey[0] + ey[1] + ey[2]};
        double sx0 = 0, sy0 = 0;
        for (int q = 1; q < 4; q++)
            for (int dir = 0; dir < 2; dir++) {
                Dual Xd[4], Yd[4];
                for (int t = 0; t < 4; t++) {
                    Xd[t] = {X[t], (t == q && dir == 0) ? 1.0 : 0.0};
                    Yd[t] = {Y[t], (t == q && dir == 1) ? 1.0 : 0.0};
                }
                Dual kx, ky;
                centroid_rel(Xd, Yd, kx, ky);
                const double gq = acc[16] * kx.d + acc[17] * ky.d;
                if (dir == 0) {
                    cx[q] += gq;
                    sx0 += gq;
                } else {
                    cy[q] += gq;
                    sy0 += gq;
                }
            }
        cx[0] += acc[16] - sx0;
        cy[0] += acc[17] - sy0;
        double *o = d.msens + 8 * d.cell_of[c];
        for (int q = 0; q < 4; q++) {
            o[2 * q] = cx[q];
            o[2 * q + 1] = cy[q];
        }
    }
}

// wall element l (one workgroup): rho_l = F_l / D_l enters R through the
// diffuse wall value of the wall cell's incoming velocities and J_l through
// f on Xi^-; F_l = sum_{v.n>0} w (v.n) f1, D_l = -sum_{v.n<=0} w (v.n) g_M1
// depend on the normal n = S_0 / A, and J_l = sum_k w m_J (v.S_0) f1_l on S_0.
// Adds the resulting dL/dS_0 to the two corners of the wall face.  SO
// (second-order scheme): F_l + dF_l and the reconstructed outgoing values
// (their dependence on the slopes, face midpoint and centroid is taken by
// the per-cell kernel).
template <typename T, bool SO>
__global__ __launch_bounds__(kBlock) void k_mesh_sens_wall(DevSolve d, int fpar, int ppar)
{
    using T2 = typename Vec2<T>::type;
    __shared__ double red[4 * 8];
    const int l = blockIdx.x, c = d.wall_cell[l], nv = d.nv, n1 = d.n1;
    const T2 *f = static_cast<const T2 *>(d.f[fpar]);
    const T2 *ph = static_cast<const T2 *>(d.phi[ppar]);
    const T *gM = static_cast<const T *>(d.gM);
    const double nx = d.wall_n[2 * l], ny = d.wall_n[2 * l + 1], A = d.wall_A[l];
    const double F = SO ? d.F[fpar][l] + d.dF[l] : d.F[fpar][l], D = d.D[l], rw = F / D, thw2 = 0.5 * d.theta_w;
    const T *Gs = static_cast<const T *>(d.G);
    const double r0x = SO ? d.rf[8 * c] : 0.0, r0y = SO ? d.rf[8 * c + 1] : 0.0;
    // dF/dn (2), dD/dn (2), dL/drho from R (1), dJ/drho / A (1), dJ/dS_0 at fixed rho (2)
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const size_t row = (size_t)c * nv;
    for (int k = threadIdx.x; k < nv; k += kBlock) {
        const int a = k % n1, b = k / n1;
        const double v1 = d.vx[a], v2 = d.vy[b], wt = d.wx[a] * d.wy[b];
        const double vn = v1 * nx + v2 * ny, mj = mJ_of(d.objective, v1, v2);
        const T2 fc = f[row + k], pc = ph[row + k];
        double f1 = (double)fc.x;
        const double g = (double)gM[k];
        if constexpr (SO) {
            if (vn > 0) f1 += (double)Gs[4 * (row + k)] * r0x + (double)Gs[4 * (row + k) + 1] * r0y;
        }
        if (vn > 0) {
            acc[0] += wt * v1 * f1;
            acc[1] += wt * v2 * f1;
            acc[6] += wt * mj * v1 * f1;
            acc[7] += wt * mj * v2 * f1;
        } else {
            acc[2] -= wt * v1 * g;
            acc[3] -= wt * v2 * g;
            acc[4] += wt * (A * vn) * g * ((double)pc.x + thw2 * (double)pc.y);
            acc[5] += wt * mj * vn * g;
            const double fw = rw * g;
            acc[6] += wt * mj * v1 * fw;
            acc[7] += wt * mj * v2 * fw;
        }
    }
    block_sum<8>(acc, red);
    if (threadIdx.x == 0) {
        const double dLdr = acc[4] + A * acc[5];
        const double gx = dLdr * (acc[0] / D - F * acc[2] / (D * D));
        const double gy = dLdr * (acc[1] / D - F * acc[3] / (D * D));
        const double gn = nx * gx + ny * gy;          // dn/dS_0 = (I - n n^T) / A
        const double G0 = (gx - nx * gn) / A + acc[6], G1 = (gy - ny * gn) / A + acc[7];
        double *o = d.msens + 8 * d.cell_of[c];       // face 0 joins corners 0 -> 1
        o[0] += G1;
        o[2] -= G1;
        o[1] -= G0;
        o[3] += G0;
    }
}

// node (i, j) is corner 0 of cell (i, j), 1 of (i-1, j), 2 of (i-1, j-1) and
// 3 of (i, j-1) (mesh numbering)
__global__ __launch_bounds__(kBlock) void k_mesh_sens_nodes(DevSolve d)
{
    const int m = blockIdx.x * kBlock + threadIdx.x;
    const int ni = d.ni, nj = d.nj;
    if (m >= (ni + 1) * (nj + 1)) return;
    const int im = m % (ni + 1), jm = m / (ni + 1);
    const int ci[4] = {im, im - 1, im - 1, im}, cj[4] = {jm, jm, jm - 1, jm - 1};
    double gx = 0, gy = 0;
    for (int p = 0; p < 4; p++) {
        if (ci[p] < 0 || ci[p] >= ni || cj[p] < 0 || cj[p] >= nj) continue;
        const double *o = d.msens + 8 * (ci[p] + ni * cj[p]) + 2 * p;
        gx += o[0];
        gy += o[1];
    }
    d.dJdx[2 * m] = gx;
    d.dJdx[2 * m + 1] = gy;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_wall_sens(const DevSolve &d, int fpar, int ppar, int n_params, hipStream_t st)
{
    if (d.order == 2) {
        // slopes and dF of the frozen f (the slope buffer holds the adjoint's
        // B between corrections; B is recomputed at the next one)
        if (hipError_t e = launch_so_slopes(d, fpar, st)) return e;
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_wall_sens<T, true>), dim3(d.nw), dim3(kBlock), 0, st, d, fpar, ppar));
    } else {
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_wall_sens<T, false>), dim3(d.nw), dim3(kBlock), 0, st, d, fpar, ppar));
    }
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_nodes_params, dim3(1), dim3(kBlock), 0, st, d, n_params);
    return hipGetLastError();
}

hipError_t launch_mesh_sens(const DevSolve &d, int fpar, int ppar, hipStream_t st)
{
    constexpr int per_block = kBlock / kWave;
    const dim3 grid((d.nc + per_block - 1) / per_block);
    if (d.order == 2) {
        // slopes and dF of the frozen f into the slope buffer (it holds the
        // adjoint's B between corrections; B is recomputed at the next one)
        if (hipError_t e = launch_so_slopes(d, fpar, st)) return e;
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_mesh_sens_cell_so<T>, grid, dim3(kBlock), 0, st, d, fpar, ppar));
    } else {
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_mesh_sens_cell<T>, grid, dim3(kBlock), 0, st, d, fpar, ppar));
    }
    if (hipError_t e = hipGetLastError()) return e;
    if (d.nw > 0) {
        if (d.order == 2)
            DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_mesh_sens_wall<T, true>), dim3(d.nw), dim3(kBlock), 0, st, d,
                                                     fpar, ppar));
        else
            DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_mesh_sens_wall<T, false>), dim3(d.nw), dim3(kBlock), 0, st, d,
                                                     fpar, ppar));
        if (hipError_t e = hipGetLastError()) return e;
    }
    const int nn = (d.ni + 1) * (d.nj + 1);
    hipLaunchKernelGGL(k_mesh_sens_nodes, dim3((nn + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace dvm
