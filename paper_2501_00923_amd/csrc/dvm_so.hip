// Second-order reconstruction kernels of libdvm (Sec. 3.1 states
// second-order accuracy in physical space for the primal and the adjoint
// balance and leaves the scheme to its references).  The scheme: cell
// values at the cell centroids, Green-Gauss slopes with the face mean of
// the two cell values (the cell value on a boundary face), the
// Venkatakrishnan limiter (smoothing relative to the cell value), and face
// values reconstructed on the upwind side
// (far-field and wall inflow are not reconstructed; the wall flux F_l sums
// the reconstructed outgoing values).
//
// It is applied by defect correction: every K sweeps
//   k_so_slope  limited slopes G of f and the wall-flux correction dF,
//   k_so_corr   c = sum_q (v.S_q) (second- minus first-order face value),
// and the first-order sweep subtracts the held c and uses F + dF.  The
// adjoint linearises with the limiter factors of the converged f frozen
// (k_so_slope in its psi mode) and holds, every K sweeps,
//   k_so_adj_b  B_u = psi_u sum_{outflow q} (v.S_q)(phi_u - phi_down)(m_q - x_u),
//   k_so_adj_e  E_m, the transpose of the Green-Gauss sum applied to B,
// which the adjoint sweep subtracts.
//
// Layout and launch as in the sweeps: one workgroup per patch (XCD-aware
// order), one wave per cell, a lane per velocity; per-cell constants in
// scalar registers.  Each kernel reads its cell's row and its interior
// neighbours' rows (in L2 for the same reasons as in the sweeps) and writes
// one row.

#include "dvm_device.h"

namespace dvm {

namespace {

constexpr int kSoBlock = kPatchCells * kWave;

// Per-cell constants of one wave's cell c: neighbour codes, face vectors,
// the face-midpoint offsets from c's centroid (r) and from the neighbours'
// centroids (rn), 1 / V.
template <typename T>
struct Cell {
    int c, nb[4];
    size_t row, nrow[4];     // first pair of c's row; of each neighbour's (c's own for boundary faces)
    T Sx[4], Sy[4], rx[4], ry[4], nx[4], ny[4];
    T iV, iVn[4];
};

template <typename T>
__device__ __forceinline__ Cell<T> load_cell(const DevSolve &d, int c, bool want_rn)
{
    Cell<T> g;
    g.c = c;
    g.row = (size_t)c * d.nv;
    g.iV = uni((T)(1.0 / d.vol[c]));
#pragma unroll
    for (int q = 0; q < 4; q++) {
        g.nb[q] = uni(d.nbr[4 * c + q]);
        g.nrow[q] = g.nb[q] >= 0 ? (size_t)g.nb[q] * d.nv : g.row;
        g.Sx[q] = uni((T)d.S[8 * c + 2 * q]);
        g.Sy[q] = uni((T)d.S[8 * c + 2 * q + 1]);
        g.rx[q] = uni((T)d.rf[8 * c + 2 * q]);
        g.ry[q] = uni((T)d.rf[8 * c + 2 * q + 1]);
        if (want_rn) {
            g.nx[q] = uni((T)d.rn[8 * c + 2 * q]);
            g.ny[q] = uni((T)d.rn[8 * c + 2 * q + 1]);
            g.iVn[q] = uni((T)(g.nb[q] >= 0 ? 1.0 / d.vol[g.nb[q]] : 0.0));
        } else {
            g.nx[q] = g.ny[q] = g.iVn[q] = 0;
        }
    }
    return g;
}

// Venkatakrishnan smoothing relative to the cell value: e = kVkKappa |f_c|
constexpr double kVkKappa = 1e-3;

// Limited slope of one component: Green-Gauss gradient from the cell value
// fc and the interior neighbours' values fn, then the Venkatakrishnan factor
// p = min(1, min_q (D^2 + e^2 + 2 d D) / (D^2 + 2 d^2 + d D + e^2)) with d
// the face's unlimited increment grad . r_q and D the room to the
// neighbourhood's max (d > 0) or min, each term evaluated in the order
// written here.  The smallest of the four fractions is found by comparing
// cross products, then divided once (IEEE).  The limiter arithmetic is FP64
// for both storage types, on d, D and e rescaled by the power of two nearest
// 1 / |f_c| (exact, and the fractions are homogeneous of degree 0): squares
// of values near the Maxwellian's tail (f ~ 1e-22 and below on common grids)
// underflow in FP32, and the adjoint uses p on its own, not only p grad f.
template <typename T>
__device__ __forceinline__ void slope1(const Cell<T> &g, T fc, const T (&fn)[4], int lim, T &gx, T &gy, T &p)
{
    T lo = fc, hi = fc;
    gx = 0;
    gy = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        T b = fc;
        if (g.nb[q] >= 0) {
            b = (T)0.5 * (fc + fn[q]);
            lo = fmin(lo, fn[q]);
            hi = fmax(hi, fn[q]);
        }
        gx += b * g.Sx[q];
        gy += b * g.Sy[q];
    }
    gx *= g.iV;
    gy *= g.iV;
    double pd = 1.0;
    if (lim) {
        int ex = 0;
        (void)frexp((double)fc, &ex);
        const double sc = ldexp(1.0, -ex);
        const double fcd = (double)fc * sc, e = kVkKappa * fcd, e2 = e * e;
        const double hid = (double)hi * sc, lod = (double)lo * sc, gxd = (double)gx * sc, gyd = (double)gy * sc;
        double bn = 1.0, bd = 1.0;   // smallest fraction so far (the cap 1 / 1)
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const double dq = gxd * (double)g.rx[q] + gyd * (double)g.ry[q];
            const double D = dq > 0 ? hid - fcd : lod - fcd;
            const double den = D * D + 2.0 * dq * dq + dq * D + e2;
            const double num = D * D + e2 + 2.0 * dq * D;
            if (den > 0 && num * bd < bn * den) {
                bn = num;
                bd = den;
            }
        }
        pd = bn / bd;
    }
    p = (T)pd;
}

// the wave's cell of patch p, or -1 for an idle wave of a partial patch
__device__ __forceinline__ int patch_cell(const DevSolve &d, int p)
{
    const int w = uni((int)(threadIdx.x / kWave));
    const int c0 = uni(d.patch[p]), cnt = uni(d.patch[p + 1]) - c0;
    return w < cnt ? c0 + w : -1;
}

// Limited slopes of f[par] into G and the wall cell's dF (PSI = false), or
// the limiter factors into psi (PSI = true).
template <typename T, bool PSI>
__global__ __launch_bounds__(kSoBlock) void k_so_slope(DevSolve d, int par)
{
    using T2 = typename Vec2<T>::type;
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;
    const int c = patch_cell(d, p);
    if (c < 0) return;   // no barrier in this kernel
    const int lane = threadIdx.x % kWave, nv = d.nv, n1 = d.n1, lim = d.limiter;
    const Cell<T> g = load_cell<T>(d, c, false);
    const T2 *__restrict__ f = static_cast<const T2 *>(d.f[par]);
    T2 *__restrict__ G = static_cast<T2 *>(d.G);
    T2 *__restrict__ psi = static_cast<T2 *>(d.psi);
    const int wl = g.nb[0] <= -2 ? -2 - g.nb[0] : -1;
    double S0x = 0, S0y = 0, mdF = 0;
    if (wl >= 0) {
        S0x = uni(d.S[8 * c]);
        S0y = uni(d.S[8 * c + 1]);
    }
    int a = lane % n1, b = lane / n1;
    const int da = kWave % n1, db = kWave / n1;
    for (int k = lane; k < nv; k += kWave) {
        const T2 fc = f[g.row + k];
        T f1[4], f2[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const T2 t = f[g.nrow[q] + k];   // boundary faces read the own row and ignore it
            f1[q] = t.x;
            f2[q] = t.y;
        }
        T g1x, g1y, p1, g2x, g2y, p2;
        slope1(g, fc.x, f1, lim, g1x, g1y, p1);
        slope1(g, fc.y, f2, lim, g2x, g2y, p2);
        if constexpr (PSI) {
            __builtin_nontemporal_store(p1, &psi[g.row + k].x);
            __builtin_nontemporal_store(p2, &psi[g.row + k].y);
        } else {
            T2 o1, o2;
            o1.x = p1 * g1x;
            o1.y = p1 * g1y;
            o2.x = p2 * g2x;
            o2.y = p2 * g2y;
            __builtin_nontemporal_store(o1.x, &G[2 * (g.row + k)].x);
            __builtin_nontemporal_store(o1.y, &G[2 * (g.row + k)].y);
            __builtin_nontemporal_store(o2.x, &G[2 * (g.row + k) + 1].x);
            __builtin_nontemporal_store(o2.y, &G[2 * (g.row + k) + 1].y);
            if (wl >= 0) {
                const double s0 = d.vx[a] * S0x + d.vy[b] * S0y;
                if (s0 > 0) mdF += d.wx[a] * d.wy[b] * s0 * (double)(o1.x * g.rx[0] + o1.y * g.ry[0]);
            }
        }
        a += da;
        b += db;
        if (a >= n1) {
            a -= n1;
            b++;
        }
    }
    if constexpr (!PSI) {
        if (wl >= 0) {
            double acc[1] = {mdF};
            wave_sum<1>(acc);
            if (lane == 0) d.dF[wl] = acc[0] / d.wall_A[wl];
        }
    }
}

// c = sum_q (v.S_q) G_u . (m_q - x_u) with u the upwind cell of face q
// (nothing for inflow through a boundary)
template <typename T>
__global__ __launch_bounds__(kSoBlock) void k_so_corr(DevSolve d)
{
    using T2 = typename Vec2<T>::type;
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;
    const int c = patch_cell(d, p);
    if (c < 0) return;
    const int lane = threadIdx.x % kWave, nv = d.nv, n1 = d.n1;
    const Cell<T> g = load_cell<T>(d, c, true);
    const T2 *__restrict__ G = static_cast<const T2 *>(d.G);
    T2 *__restrict__ out = static_cast<T2 *>(d.corr);
    int a = lane % n1, b = lane / n1;
    const int da = kWave % n1, db = kWave / n1;
    for (int k = lane; k < nv; k += kWave) {
        const T v1 = (T)d.vx[a], v2 = (T)d.vy[b];
        const T2 o1 = G[2 * (g.row + k)], o2 = G[2 * (g.row + k) + 1];
        // a neighbour's slopes are needed only where it is upwind
        T sq[4];
        T2 n1v[4], n2v[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            sq[q] = v1 * g.Sx[q] + v2 * g.Sy[q];
            n1v[q] = n2v[q] = T2{0, 0};
            if (!(sq[q] > 0) && g.nb[q] >= 0) {
                n1v[q] = G[2 * (g.nrow[q] + k)];
                n2v[q] = G[2 * (g.nrow[q] + k) + 1];
            }
        }
        T c1 = 0, c2 = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const T s = sq[q];
            if (s > 0) {
                c1 += s * (o1.x * g.rx[q] + o1.y * g.ry[q]);
                c2 += s * (o2.x * g.rx[q] + o2.y * g.ry[q]);
            } else if (g.nb[q] >= 0) {
                c1 += s * (n1v[q].x * g.nx[q] + n1v[q].y * g.ny[q]);
                c2 += s * (n2v[q].x * g.nx[q] + n2v[q].y * g.ny[q]);
            }
        }
        __builtin_nontemporal_store(c1, &out[g.row + k].x);
        __builtin_nontemporal_store(c2, &out[g.row + k].y);
        a += da;
        b += db;
        if (a >= n1) {
            a -= n1;
            b++;
        }
    }
}

// B_u = psi_u sum_{q: v.S_q > 0} (v.S_q)(phi_u - phi_down,q)(m_q - x_u), with
// phi_down the neighbour's phi, 0 at the far field, (Phi_l - m_J, 0) at the wall
template <typename T>
__global__ __launch_bounds__(kSoBlock) void k_so_adj_b(DevSolve d, int par)
{
    using T2 = typename Vec2<T>::type;
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;
    const int c = patch_cell(d, p);
    if (c < 0) return;
    const int lane = threadIdx.x % kWave, nv = d.nv, n1 = d.n1, obj = d.objective;
    const Cell<T> g = load_cell<T>(d, c, false);
    const T2 *__restrict__ phi = static_cast<const T2 *>(d.phi[par]);
    const T2 *__restrict__ psi = static_cast<const T2 *>(d.psi);
    T2 *__restrict__ B = static_cast<T2 *>(d.G);
    const int wl = g.nb[0] <= -2 ? -2 - g.nb[0] : -1;
    const T Phi_w = wl >= 0 ? uni((T)d.Phi[par][wl]) : (T)0;
    int a = lane % n1, b = lane / n1;
    const int da = kWave % n1, db = kWave / n1;
    for (int k = lane; k < nv; k += kWave) {
        const double v1d = d.vx[a], v2d = d.vy[b];
        const T v1 = (T)v1d, v2 = (T)v2d;
        const T2 pu = phi[g.row + k], ps = psi[g.row + k];
        // a neighbour's phi is needed only where it is downwind
        T sq[4];
        T2 pd[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            sq[q] = v1 * g.Sx[q] + v2 * g.Sy[q];
            pd[q] = T2{0, 0};
            if (sq[q] > 0 && g.nb[q] >= 0) pd[q] = phi[g.nrow[q] + k];
        }
        T b1x = 0, b1y = 0, b2x = 0, b2y = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const T s = sq[q];
            if (s > 0) {
                T d1 = 0, d2 = 0;
                if (g.nb[q] >= 0) {
                    d1 = pd[q].x;
                    d2 = pd[q].y;
                } else if (g.nb[q] <= -2) {
                    d1 = Phi_w - (T)mJ_of(obj, v1d, v2d);
                }
                const T a1 = s * (pu.x - d1), a2 = s * (pu.y - d2);
                b1x += a1 * g.rx[q];
                b1y += a1 * g.ry[q];
                b2x += a2 * g.rx[q];
                b2y += a2 * g.ry[q];
            }
        }
        // plain stores: non-temporal ones made this kernel 0.26 ms slower on
        // the 256x128 C-grid with 2304 velocities (they help the slopes' G)
        T2 o1, o2;
        o1.x = b1x * ps.x;
        o1.y = b1y * ps.x;
        o2.x = b2x * ps.y;
        o2.y = b2y * ps.y;
        B[2 * (g.row + k)] = o1;
        B[2 * (g.row + k) + 1] = o2;
        a += da;
        b += db;
        if (a >= n1) {
            a -= n1;
            b++;
        }
    }
}

// E_m = d/df_m of sum_u B_u . grad f_u with grad f_u = (1/V_u) sum_q fbar_q S_uq:
// the own part (1/2 on interior faces, 1 on boundary faces) and, through each
// interior face q, the neighbour's part with its face vector -S_q.
template <typename T>
__global__ __launch_bounds__(kSoBlock) void k_so_adj_e(DevSolve d)
{
    using T2 = typename Vec2<T>::type;
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;
    const int c = patch_cell(d, p);
    if (c < 0) return;
    const int lane = threadIdx.x % kWave, nv = d.nv;
    const Cell<T> g = load_cell<T>(d, c, true);
    const T2 *__restrict__ B = static_cast<const T2 *>(d.G);
    T2 *__restrict__ out = static_cast<T2 *>(d.corr);
    for (int k = lane; k < nv; k += kWave) {
        const T2 o1 = B[2 * (g.row + k)], o2 = B[2 * (g.row + k) + 1];
        T2 n1v[4], n2v[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            n1v[q] = B[2 * (g.nrow[q] + k)];
            n2v[q] = B[2 * (g.nrow[q] + k) + 1];
        }
        T e1 = 0, e2 = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const T t1 = (o1.x * g.Sx[q] + o1.y * g.Sy[q]) * g.iV;
            const T t2 = (o2.x * g.Sx[q] + o2.y * g.Sy[q]) * g.iV;
            if (g.nb[q] >= 0) {
                const T u1 = (n1v[q].x * g.Sx[q] + n1v[q].y * g.Sy[q]) * g.iVn[q];
                const T u2 = (n2v[q].x * g.Sx[q] + n2v[q].y * g.Sy[q]) * g.iVn[q];
                e1 += (T)0.5 * (t1 - u1);
                e2 += (T)0.5 * (t2 - u2);
            } else {
                e1 += t1;
                e2 += t2;
            }
        }
        __builtin_nontemporal_store(e1, &out[g.row + k].x);
        __builtin_nontemporal_store(e2, &out[g.row + k].y);
    }
}

// J_l = A_l sum_k w m_J (v.n) f1_{l,k} with the outgoing wall values
// reconstructed from f[par] and the incoming ones (F_l + dF_l) gbar1, dF_l
// of the same f: one block per element.  With H = sum_{Xi^-} w m_J (v.n)
// gbar1, J_l = A_l (sum_{Xi^+} w m_J (v.n) f1 + (F_l + dF_l) H).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_so_objective_elem(DevSolve d, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ double red[4 * 3];
    const int l = blockIdx.x;
    const int c = d.wall_cell[l];
    const T2 *f = static_cast<const T2 *>(d.f[par]);
    const T *gM = static_cast<const T *>(d.gM);
    const Cell<T> g = load_cell<T>(d, c, false);
    const double n1 = d.wall_n[2 * l], n2 = d.wall_n[2 * l + 1], iD = 1.0 / d.D[l];
    double jp = 0, dF = 0, H = 0;
    for (int k = threadIdx.x; k < d.nv; k += kBlock) {
        const int a = k % d.n1, b = k / d.n1;
        const double v1 = d.vx[a], v2 = d.vy[b];
        const double vn = v1 * n1 + v2 * n2;
        const double wm = d.wx[a] * d.wy[b] * mJ_of(d.objective, v1, v2);
        if (vn > 0) {
            const T2 fc = f[g.row + k];
            T f1[4];
#pragma unroll
            for (int q = 0; q < 4; q++) f1[q] = f[g.nrow[q] + k].x;
            T gx, gy, p1;
            slope1(g, fc.x, f1, d.limiter, gx, gy, p1);
            const double delta = (double)((p1 * gx) * g.rx[0] + (p1 * gy) * g.ry[0]);
            jp += wm * vn * ((double)fc.x + delta);
            dF += d.wx[a] * d.wy[b] * vn * delta;
        } else {
            H += wm * vn * (double)gM[k] * iD;
        }
    }
    double acc[3] = {jp, dF, H};
    block_sum<3>(acc, red);
    if (threadIdx.x == 0) d.Jl[l] = d.wall_A[l] * (acc[0] + (d.F[par][l] + acc[1]) * acc[2]);
}

}  // namespace

hipError_t launch_so_slopes(const DevSolve &d, int par, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_so_slope<T, false>), dim3(xcd_grid(d.np)), dim3(kSoBlock), 0, st, d, par));
    return hipGetLastError();
}

hipError_t launch_so_correction(const DevSolve &d, int par, hipStream_t st)
{
    if (hipError_t e = launch_so_slopes(d, par, st)) return e;
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_so_corr<T>, dim3(xcd_grid(d.np)), dim3(kSoBlock), 0, st, d));
    return hipGetLastError();
}

hipError_t launch_so_freeze(const DevSolve &d, int fpar, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_so_slope<T, true>), dim3(xcd_grid(d.np)), dim3(kSoBlock), 0, st, d, fpar));
    return hipGetLastError();
}

hipError_t launch_so_adjoint_term(const DevSolve &d, int par, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_so_adj_b<T>, dim3(xcd_grid(d.np)), dim3(kSoBlock), 0, st, d, par));
    if (hipError_t e = hipGetLastError()) return e;
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_so_adj_e<T>, dim3(xcd_grid(d.np)), dim3(kSoBlock), 0, st, d));
    return hipGetLastError();
}

hipError_t launch_so_objective_elem(const DevSolve &d, int par, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_so_objective_elem<T>, dim3(d.nw), dim3(kBlock), 0, st, d, par));
    return hipGetLastError();
}

}  // namespace dvm
