// HIP kernels of libdvm for gfx950 (CDNA4).
//
// Layout: f and phi are [cell][velocity][2] (the two reduced distributions
// of Sec. 2.2 interleaved), so one cell's row of 2*nv values is contiguous
// and a wave64 reading consecutive velocities streams whole cache lines.
// Cells are numbered on the device in sweep order (see dvm_internal.h).
//
// Sweeps: one workgroup per patch of up to kPatchCells cells, one wave per
// cell.  A wave walks its cell's velocities 64 at a time; at each step every
// wave puts its own row's values into LDS, and after one barrier a face
// whose neighbour lies in the same patch reads the neighbour's values from
// LDS, a face to a cell outside the patch reads them from global memory
// (L2 in the common case: the neighbouring patch ran shortly before or runs
// alongside on the same XCD), and a boundary face reads the far-field or
// wall table.  The loads of the next step are issued before the current
// step's arithmetic.  The FP64 velocity moments of the new row are summed
// in registers and reduced across the wave with shuffles in a fixed order,
// so the next sweep finds W^{n+1} ready and f is streamed once per sweep.
// The Maxwellian is evaluated as rho/(2 pi theta) * ex[a] * ey[b] with the
// per-cell 1-D factors in LDS (tensor-product velocity grid), i.e. n1 + n2
// exponentials per cell instead of n1*n2.

#include <math.h>

#include <algorithm>
#include <mutex>

#include "dvm_device.h"

namespace dvm {

// In FP32 a lane can take two adjacent velocities of one velocity-grid row
// (n1 even): the pair's (f1, f2, f1', f2') is one 16-byte load or store, as
// one velocity is in FP64.  Measured on the 256x128 C-grid with 2304
// velocities: mixed primal sweep 325 -> 299 us.
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ bool pair_velocities(int n1)
{
    return sizeof(T) == 4 && (n1 & 1) == 0;
}

// LDS of a patch sweep: the velocity tables, each cell's Maxwellian
// factors and, for a sweep that exchanges rows (XCH), the double-buffered
// exchange of the patch's own rows.
template <typename T, bool XCH>
struct PatchLds {
    double vx[kMaxN1D], vy[kMaxN1D], wx[kMaxN1D], wy[kMaxN1D];
    T ex[kPatchCells][kMaxN1D], ey[kPatchCells][kMaxN1D];
    typename Vec2<T>::type xch[XCH ? 2 : 1][XCH ? kPatchCells : 1][kWave];
};

// Non-temporal load of a (x, y) pair: rows read by their own cell only (the
// frozen f of the adjoint, held corrections) so that they do not push the
// neighbour rows other cells reuse out of L2 (FP64 adjoint sweep on the
// 256x128 C-grid with 2304 velocities: 735 -> 727 us).
template <typename V>
__device__ __forceinline__ V ntload2(const V *p)
{
    V r;
    r.x = __builtin_nontemporal_load(&p->x);
    r.y = __builtin_nontemporal_load(&p->y);
    return r;
}

// Reciprocal for the FP64 update: hardware estimate and two Newton steps
// (error about one ulp; the IEEE division costs twice the instructions).
// FP32 keeps the IEEE division: a one-ulp reciprocal there raised the
// mixed-precision drag error against FP64 from 1e-8 to 2e-7 relative.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) { return 1.0f / x; }

// The adjoint sweep exchanges the patch's rows through LDS in FP64 (4%
// faster than every face reading global memory on the 256x128 C-grid with
// 2304 velocities); in FP32 and in the primal sweep the per-step barrier
// costs more than the L2 requests it saves.
template <typename T>
constexpr bool kAdjointExchange = sizeof(T) == 8;

// Shared velocity tables (threads 0 .. n1+n2-1; a patch workgroup has at
// least 4 waves, n1 + n2 <= 256) and this wave's Maxwellian factors
// exp(-(v - u)^2 / (2 theta)) per direction.
template <typename T, bool XCH>
__device__ __forceinline__ void patch_tables(const DevSolve &d, PatchLds<T, XCH> &sm, int w, int lane, double u1,
                                             double u2, double inv2th)
{
    const int t = threadIdx.x, n1 = d.n1, n2 = d.n2;
    if (t < n1) {
        sm.vx[t] = d.vx[t];
        sm.wx[t] = d.wx[t];
    } else if (t - n1 < n2) {
        sm.vy[t - n1] = d.vy[t - n1];
        sm.wy[t - n1] = d.wy[t - n1];
    }
    for (int i = lane; i < n1 + n2; i += kWave) {
        if (i < n1) {
            const double e = d.vx[i] - u1;
            sm.ex[w][i] = (T)exp(-e * e * inv2th);
        } else {
            const double e = d.vy[i - n1] - u2;
            sm.ey[w][i - n1] = (T)exp(-e * e * inv2th);
        }
    }
}

// ---------------------------------------------------------------------------
// primal sweep of one patch: eq. (numerpr_gov), first-order upwind, Jacobi
// point-implicit: f^{n+1} = (sum_in |v.S| f_up + V g/tau) / (sum_out v.S + V/tau)
// SO (second-order scheme, defect correction): the held correction c is
// subtracted from the numerator and the wall flux is F + dF.
// ---------------------------------------------------------------------------
template <typename T, bool SO>
__device__ __forceinline__ void primal_patch(const DevSolve &d, int p, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ PatchLds<T, false> sm;
    const int w = uni((int)(threadIdx.x / kWave)), lane = threadIdx.x % kWave;
    const int c0 = uni(d.patch[p]), cnt = uni(d.patch[p + 1]) - c0;
    const bool act = w < cnt;                   // idle waves of a partial patch only join the barrier
    const int c = c0 + (act ? w : 0);
    const int nv = d.nv, n1 = d.n1;
    const T2 *__restrict__ fin = static_cast<const T2 *>(d.f[par]);
    T2 *__restrict__ fout = static_cast<T2 *>(d.f[par ^ 1]);
    const T2 *__restrict__ corr = static_cast<const T2 *>(d.corr);

    const double *Win = d.W[par] + 4 * c;
    const double W0 = uni(Win[0]), W1 = uni(Win[1]), W2 = uni(Win[2]), W3 = uni(Win[3]);
    const double rho = W0, u1 = W1 / rho, u2 = W2 / rho;
    const double th = (2.0 / 3.0) * (W3 / rho - 0.5 * (u1 * u1 + u2 * u2));
    const double itau = d.inv_tau_inf * rho * sqrt(2.0 * th);
    const double Vt = d.vol[c] * itau;
    // the equilibrium's parameters: the primitive variables, or those whose
    // grid moments equal W (found by k_eq_params before the sweep; tau keeps
    // the cell's own rho and theta)
    double Pe[4] = {rho, u1, u2, th};
    if (d.equil) {
        const double *pe = d.mstate + kEqState * c;
#pragma unroll
        for (int a = 0; a < 4; a++) Pe[a] = uni(pe[a]);
    }
    patch_tables<T, false>(d, sm, w, lane, Pe[1], Pe[2], 0.5 / Pe[3]);

    const size_t row = (size_t)c * nv;
    int nb[4];
    T Sx[4], Sy[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        nb[q] = uni(d.nbr[4 * c + q]);
        Sx[q] = uni((T)d.S[8 * c + 2 * q]);
        Sy[q] = uni((T)d.S[8 * c + 2 * q + 1]);
    }
    const int wl = nb[0] <= -2 ? -2 - nb[0] : -1;
    T wcoef = 0;
    double S0x = 0, S0y = 0;
    if (wl >= 0) {
        wcoef = uni((T)((SO ? d.F[par][wl] + d.dF[wl] : d.F[par][wl]) / d.D[wl]));
        S0x = uni(d.S[8 * c]);
        S0y = uni(d.S[8 * c + 1]);
    }
    // one source row per face: the neighbour's row (a neighbour in the same
    // patch was read moments before by its own wave on this CU and is in
    // L1), the far-field table, or the wall table (g_M1, theta_w/2 g_M1)
    // scaled by F_l / D_l
    const T2 *src[4];
    T sc[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int n = nb[q];
        src[q] = n >= 0 ? fin + (size_t)n * nv : static_cast<const T2 *>(n == -1 ? d.fd : d.gw2);
        sc[q] = n <= -2 ? wcoef : (T)1;
    }
    const T th2 = uni((T)(0.5 * Pe[3]));
    const T gc = uni((T)(Pe[0] / (2.0 * kPi * Pe[3]))), VtT = uni((T)Vt);
    __syncthreads();

    double m0 = 0, m1 = 0, m2 = 0, m3 = 0, mF = 0;
    // one velocity (1-D indices a, b): the point-implicit update from the
    // four face sources, and the new value's share of the FP64 moments
    auto update = [&](int a, int b, const T2 (&up)[4], T2 cr) {
        const T v1 = (T)sm.vx[a], v2 = (T)sm.vy[b];
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
        if constexpr (SO) {
            in1 -= cr.x;
            in2 -= cr.y;
        }
        const T g1 = gc * sm.ex[w][a] * sm.ey[w][b];
        const T g2 = th2 * g1;
        const T rden = recip(out + VtT);
        T2 r;
        r.x = (in1 + VtT * g1) * rden;
        r.y = (in2 + VtT * g2) * rden;
        return r;
    };
    auto accumulate = [&](int a, int b, T2 r) {
        const double v1d = sm.vx[a], v2d = sm.vy[b];
        const double wt = sm.wx[a] * sm.wy[b];
        const double f1 = (double)r.x, f2 = (double)r.y;
        const double wf1 = wt * f1;
        m0 += wf1;
        m1 = fma(wf1, v1d, m1);
        m2 = fma(wf1, v2d, m2);
        m3 = fma(wf1, 0.5 * fma(v1d, v1d, v2d * v2d), fma(wt, f2, m3));
        if (wl >= 0) {
            const double s0 = v1d * S0x + v2d * S0y;
            if (s0 > 0) mF = fma(wf1, s0, mF);
        }
    };
    if (pair_velocities<T>(n1)) {
        // FP32 with an even n1: two adjacent velocities (same b) per lane,
        // 16-byte loads and stores
        int a = (2 * lane) % n1, b = (2 * lane) / n1;
        const int da = (2 * kWave) % n1, db = (2 * kWave) / n1;
        const int nstep = (nv + 2 * kWave - 1) / (2 * kWave);
        for (int t = 0; t < nstep; t++) {
            const int k = 2 * (t * kWave + lane);
            if (act && k < nv) {
                // a face's source row only where it is upwind for either velocity
                f4 u4[4];
                {
                    const T v1a = (T)sm.vx[a], v1b = (T)sm.vx[a + 1], v2 = (T)sm.vy[b];
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        u4[q] = f4{0, 0, 0, 0};
                        if (!(v1a * Sx[q] + v2 * Sy[q] > 0) || !(v1b * Sx[q] + v2 * Sy[q] > 0))
                            u4[q] = *reinterpret_cast<const f4 *>(src[q] + k);
                    }
                }
                T2 u0[4], u1[4], cr0 = {0, 0}, cr1 = {0, 0};
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    u0[q].x = u4[q].x;
                    u0[q].y = u4[q].y;
                    u1[q].x = u4[q].z;
                    u1[q].y = u4[q].w;
                }
                if constexpr (SO) {
                    const f4 c4 = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(corr + row + k));
                    cr0.x = c4.x;
                    cr0.y = c4.y;
                    cr1.x = c4.z;
                    cr1.y = c4.w;
                }
                const T2 r0 = update(a, b, u0, cr0), r1 = update(a + 1, b, u1, cr1);
                const f4 r4 = {(float)r0.x, (float)r0.y, (float)r1.x, (float)r1.y};
                __builtin_nontemporal_store(r4, reinterpret_cast<f4 *>(fout + row + k));
                accumulate(a, b, r0);
                accumulate(a + 1, b, r1);
            }
            a += da;
            b += db;
            if (a >= n1) {
                a -= n1;
                b++;
            }
        }
    } else {
        int a = lane % n1, b = lane / n1;
        const int da = kWave % n1, db = kWave / n1;
        const int nstep = (nv + kWave - 1) / kWave;
        for (int t = 0; t < nstep; t++) {
            const int k = t * kWave + lane;
            if (act && k < nv) {
                // a face's source row only where the face is upwind (the
                // lanes of a wave split by the sign of v.S): about half the
                // L2 requests of loading all four (primal 557 -> 511 us on
                // the 256x128 C-grid with 2304 velocities; the adjoint's
                // downstream loads gain nothing from the same masking)
                T2 up[4], cr = {0, 0};
                {
                    const T v1 = (T)sm.vx[a], v2 = (T)sm.vy[b];
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        up[q] = T2{0, 0};
                        if (!(v1 * Sx[q] + v2 * Sy[q] > 0)) up[q] = src[q][k];
                    }
                }
                if constexpr (SO) cr = ntload2(&corr[row + k]);
                const T2 r = update(a, b, up, cr);
                // streaming stores: the new row is not read again in this sweep
                __builtin_nontemporal_store(r.x, &fout[row + k].x);
                __builtin_nontemporal_store(r.y, &fout[row + k].y);
                accumulate(a, b, r);
            }
            a += da;
            b += db;
            if (a >= n1) {
                a -= n1;
                b++;
            }
        }
    }
    double acc[5] = {m0, m1, m2, m3, mF};
    wave_sum<5>(acc);
    if (act && lane == 0) {
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

// moments W and wall flux F of f[par] for one cell (no update), one wave
// per cell: the same lane <-> velocity map, expressions and summation order
// as the primal sweep's epilogue, so a state loaded from a checkpoint
// continues bit for bit.
template <typename T>
__device__ __forceinline__ void moments_wave(const DevSolve &d, int c, int par)
{
    using T2 = typename Vec2<T>::type;
    const int lane = threadIdx.x % kWave, nv = d.nv, n1 = d.n1;
    const int l0 = d.nbr[4 * c];
    const int wl = l0 <= -2 ? -2 - l0 : -1;
    const double S0x = d.S[8 * c], S0y = d.S[8 * c + 1];
    const T2 *__restrict__ f = static_cast<const T2 *>(d.f[par]);
    double m0 = 0, m1 = 0, m2 = 0, m3 = 0, mF = 0;
    auto accumulate = [&](int a, int b, T2 r) {
        const double v1d = d.vx[a], v2d = d.vy[b];
        const double wt = d.wx[a] * d.wy[b];
        const double f1 = (double)r.x, f2 = (double)r.y;
        const double wf1 = wt * f1;
        m0 += wf1;
        m1 = fma(wf1, v1d, m1);
        m2 = fma(wf1, v2d, m2);
        m3 = fma(wf1, 0.5 * fma(v1d, v1d, v2d * v2d), fma(wt, f2, m3));
        if (wl >= 0) {
            const double s0 = v1d * S0x + v2d * S0y;
            if (s0 > 0) mF = fma(wf1, s0, mF);
        }
    };
    const size_t row = (size_t)c * nv;
    if (pair_velocities<T>(n1)) {
        int a = (2 * lane) % n1, b = (2 * lane) / n1;
        const int da = (2 * kWave) % n1, db = (2 * kWave) / n1;
        for (int k = 2 * lane; k < nv; k += 2 * kWave) {
            T2 r0, r1;
            r0 = f[row + k];
            r1 = f[row + k + 1];
            accumulate(a, b, r0);
            accumulate(a + 1, b, r1);
            a += da;
            b += db;
            if (a >= n1) {
                a -= n1;
                b++;
            }
        }
    } else {
        int a = lane % n1, b = lane / n1;
        const int da = kWave % n1, db = kWave / n1;
        for (int k = lane; k < nv; k += kWave) {
            accumulate(a, b, f[row + k]);
            a += da;
            b += db;
            if (a >= n1) {
                a -= n1;
                b++;
            }
        }
    }
    double acc[5] = {m0, m1, m2, m3, mF};
    wave_sum<5>(acc);
    if (lane == 0) {
        double *Wo = d.W[par] + 4 * c;
        Wo[0] = acc[0];
        Wo[1] = acc[1];
        Wo[2] = acc[2];
        Wo[3] = acc[3];
        if (wl >= 0) d.F[par][wl] = acc[4] / d.wall_A[wl];
    }
}

// Per-cell constants of the adjoint moments: the frozen velocity u, theta/2,
// theta_w/2, the wall face vector and wall element (-1: none), objective.
struct AdjCell {
    double u1, u2, hth, thw2, S0x, S0y;
    int wl, obj;
};

// One velocity's share of the FP64 adjoint moments of phi (eqs.
// adjoint_macdefines, formula_adjointbgk): phi . dg/dP for P = (rho, u1, u2,
// theta) summed as A0..A4, the rho_tau sum R and the wall multiplier sum Pw
// (incoming velocities of the wall face).  g1, g2: the frozen Maxwellian at
// this velocity; gM[k]: g_M1(1, 0, theta_w) there, read only in wall cells.
// Shared by the adjoint sweep's epilogue and k_adjoint_moments, so both give
// the same bits.
template <typename T>
__device__ __forceinline__ void adjoint_terms(double &A0, double &A1, double &A2, double &A3, double &A4, double &R,
                                              double &Pw, const AdjCell &q, double v1d, double v2d, double wt,
                                              double g1, double g2, double p1, double p2, double fs1, double fs2,
                                              const T *__restrict__ gM, int k)
{
    const double qq = fma(q.hth, p2, p1);
    const double c1 = v1d - q.u1, c2 = v2d - q.u2;
    const double wg = wt * g1, wq = wg * qq;
    A0 += wq;
    A1 = fma(wq, c1, A1);
    A2 = fma(wq, c2, A2);
    A3 = fma(wq, fma(c1, c1, c2 * c2), A3);
    A4 = fma(wg, p2, A4);
    R = fma(wt, fma(p1, g1 - fs1, p2 * (g2 - fs2)), R);
    if (q.wl >= 0) {
        const double s0 = v1d * q.S0x + v2d * q.S0y;
        if (s0 <= 0) Pw += wt * s0 * (double)gM[k] * ((p1 + mJ_of(q.obj, v1d, v2d)) + q.thw2 * p2);
    }
}

// The wave-reduced sums acc[0..6] of adjoint_terms -> What (4) and rho_tau
// of the cell (ao[0..4]) and the wall multiplier Phi_l of its wall element.
__device__ __forceinline__ void adjoint_store(const DevSolve &d, const double *ac, int wl, const double *acc,
                                              double *ao, double *Phi)
{
    const double rho = ac[0], th = ac[3], itau = ac[4];
    const double *M = ac + 16;      // dP/dW, P = the equilibrium's (rho, u1, u2, theta)
    // phi . dg/dP
    double Pq[4];
    Pq[0] = acc[0] / rho;
    Pq[1] = acc[1] / th;
    Pq[2] = acc[2] / th;
    Pq[3] = acc[3] / (2.0 * th * th) - acc[0] / th + 0.5 * acc[4];
    // What_m = sum_q (phi . dg/dP_q) dP_q/dW_m
#pragma unroll
    for (int m = 0; m < 4; m++)
        ao[m] = ((Pq[0] * M[m] + Pq[1] * M[4 + m]) + Pq[2] * M[8 + m]) + Pq[3] * M[12 + m];
    ao[4] = acc[5] * itau;
    if (wl >= 0) Phi[wl] = -acc[6] / (d.wall_A[wl] * d.D[wl]);
}

// ---------------------------------------------------------------------------
// adjoint sweep of one patch: eq. (numerad_gov) with the wall and far-field
// conditions of eq. (formula_adjointbgk), Jacobi point-implicit:
// phi^{n+1} = (sum_out v.S phi_down + V (phi_eq/tau + phi_tau)) / (sum_out v.S + V/tau)
// Epilogue: What (eq. adjoint_macdefines, via primitive variables),
// rho_tau, the wall multiplier Phi_l and the residual partials of phi^{n+1}.
// SO (second-order scheme): the held reconstruction term E is subtracted
// from the numerator.
// ---------------------------------------------------------------------------
template <typename T, bool XCH, bool SO>
__device__ __forceinline__ void adjoint_patch(const DevSolve &d, int p, int par)
{
    using T2 = typename Vec2<T>::type;
    __shared__ PatchLds<T, XCH> sm;
    const int w = uni((int)(threadIdx.x / kWave)), lane = threadIdx.x % kWave;
    const int c0 = uni(d.patch[p]), cnt = uni(d.patch[p + 1]) - c0;
    const bool act = w < cnt;
    const int c = c0 + (act ? w : 0);
    const int nv = d.nv, n1 = d.n1;
    const T2 *__restrict__ pin = static_cast<const T2 *>(d.phi[par]);
    T2 *__restrict__ pout = static_cast<T2 *>(d.phi[par ^ 1]);
    const T2 *__restrict__ fst = static_cast<const T2 *>(d.fstar);
    const T2 *__restrict__ eterm = static_cast<const T2 *>(d.corr);

    const double *ac = d.acoef + kAcoef * c;
    const double u1 = uni(ac[1]), u2 = uni(ac[2]), th = uni(ac[3]), itau = uni(ac[4]);
    const double gcoef = ac[5];
    const double dt0 = ac[6], dt1 = ac[7], dt2 = ac[8], dt3 = ac[9];
    const double Vv = d.vol[c];
    const double *aw = d.aW[par] + 8 * c;
    const double rt = aw[4];
    // source phi_eq / tau + phi_tau = C0 + C1 v1 + C2 v2 + C3 |v|^2/2 (first), C3 (second)
    const double C0 = aw[0] * itau - rt * dt0, C1 = aw[1] * itau - rt * dt1;
    const double C2 = aw[2] * itau - rt * dt2, C3 = aw[3] * itau - rt * dt3;
    patch_tables<T, XCH>(d, sm, w, lane, u1, u2, 0.5 / th);

    const size_t row = (size_t)c * nv;
    int nb[4], slot[4];
    T Sx[4], Sy[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        nb[q] = uni(d.nbr[4 * c + q]);
        Sx[q] = uni((T)d.S[8 * c + 2 * q]);
        Sy[q] = uni((T)d.S[8 * c + 2 * q + 1]);
        slot[q] = XCH && nb[q] >= c0 && nb[q] < c0 + cnt ? nb[q] - c0 : -1;
    }
    const int wl = nb[0] <= -2 ? -2 - nb[0] : -1;
    T Phi_w = 0;
    double S0x = 0, S0y = 0;
    if (wl >= 0) {
        Phi_w = uni((T)d.Phi[par][wl]);
        S0x = uni(d.S[8 * c]);
        S0y = uni(d.S[8 * c + 1]);
    }
    const T *__restrict__ gM = static_cast<const T *>(d.gM);
    // downstream rows of faces to cells not exchanged through LDS; every
    // other face reads the own row (loaded anyway, an L1 hit) and ignores it
    const T2 *dsrc[4];
#pragma unroll
    for (int q = 0; q < 4; q++) dsrc[q] = pin + (size_t)(nb[q] >= 0 && slot[q] < 0 ? nb[q] : c) * nv;
    const int obj = d.objective;
    const T VT = uni((T)Vv), den0 = uni((T)(Vv * itau));
    const T Ct0 = uni((T)C0), Ct1 = uni((T)C1), Ct2 = uni((T)C2), Ct3 = uni((T)C3);
    const T gc = uni((T)gcoef), th2 = uni((T)(0.5 * th));
    const double thw2 = 0.5 * d.theta_w, hth = 0.5 * th;
    __syncthreads();

    double A0 = 0, A1 = 0, A2 = 0, A3 = 0, A4 = 0, R = 0, Pw = 0, dn = 0, dd = 0;
    // one velocity (1-D indices a, b): the point-implicit update from the
    // downstream values of the four faces, and the new value's share of the
    // FP64 adjoint moments, the wall multiplier and the residual
    auto update = [&](int a, int b, const T2 (&dwn)[4], T2 e) {
        const double v1d = sm.vx[a], v2d = sm.vy[b];
        const T v1 = (T)v1d, v2 = (T)v2d;
        const T mj = (T)mJ_of(obj, v1d, v2d);
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
        if constexpr (SO) {
            a1 -= e.x;
            a2 -= e.y;
        }
        const T vv2 = (T)0.5 * (v1 * v1 + v2 * v2);
        const T s1 = Ct0 + Ct1 * v1 + Ct2 * v2 + Ct3 * vv2;
        const T rden = recip(out + den0);
        T2 r;
        r.x = (a1 + VT * s1) * rden;
        r.y = (a2 + VT * Ct3) * rden;
        return r;
    };
    const AdjCell cq = {u1, u2, hth, thw2, S0x, S0y, wl, obj};
    auto accumulate = [&](int a, int b, int k, T2 r, T2 fs, T2 old) {
        const double v1d = sm.vx[a], v2d = sm.vy[b];
        const double wt = sm.wx[a] * sm.wy[b];
        const double p1 = (double)r.x, p2 = (double)r.y;
        const double g1 = (double)(gc * sm.ex[w][a] * sm.ey[w][b]);
        const double g2 = (double)(th2 * (T)g1);
        adjoint_terms(A0, A1, A2, A3, A4, R, Pw, cq, v1d, v2d, wt, g1, g2, p1, p2, (double)fs.x, (double)fs.y, gM, k);
        const double e1 = p1 - (double)old.x, e2 = p2 - (double)old.y;
        dn = fma(wt, fma(e1, e1, e2 * e2), dn);
        dd = fma(wt, fma(p1, p1, p2 * p2), dd);
    };
    if constexpr (XCH) {
        int a = lane % n1, b = lane / n1;
        const int da = kWave % n1, db = kWave / n1;
        const int nstep = (nv + kWave - 1) / kWave;
        T2 own_n = {0, 0}, fs_n = {0, 0}, e_n = {0, 0}, dwn_n[4] = {};
        if (act) {
            const int k = min(lane, nv - 1);
            own_n = pin[row + k];
            fs_n = ntload2(&fst[row + k]);
            if constexpr (SO) e_n = ntload2(&eterm[row + k]);
#pragma unroll
            for (int q = 0; q < 4; q++) dwn_n[q] = dsrc[q][k];
        }
        for (int t = 0; t < nstep; t++) {
            const int buf = t & 1;
            const int k = t * kWave + lane;
            // every wave publishes its own values of this step, then the
            // next step's loads go out before this step's arithmetic
            sm.xch[buf][w][lane] = own_n;
            const T2 old = own_n, fs = fs_n, e = e_n;
            T2 dwn[4];
#pragma unroll
            for (int q = 0; q < 4; q++) dwn[q] = dwn_n[q];
            __syncthreads();
            if (act && t + 1 < nstep) {
                const int kn = min(k + kWave, nv - 1);
                own_n = pin[row + kn];
                fs_n = ntload2(&fst[row + kn]);
                if constexpr (SO) e_n = ntload2(&eterm[row + kn]);
#pragma unroll
                for (int q = 0; q < 4; q++) dwn_n[q] = dsrc[q][kn];
            }
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (slot[q] >= 0) dwn[q] = sm.xch[buf][slot[q]][lane];
            if (act && k < nv) {
                const T2 r = update(a, b, dwn, e);
                __builtin_nontemporal_store(r.x, &pout[row + k].x);
                __builtin_nontemporal_store(r.y, &pout[row + k].y);
                accumulate(a, b, k, r, fs, old);
            }
            a += da;
            b += db;
            if (a >= n1) {
                a -= n1;
                b++;
            }
        }
    } else if (pair_velocities<T>(n1)) {
        int a = (2 * lane) % n1, b = (2 * lane) / n1;
        const int da = (2 * kWave) % n1, db = (2 * kWave) / n1;
        const int nstep = (nv + 2 * kWave - 1) / (2 * kWave);
        for (int t = 0; t < nstep; t++) {
            const int k = 2 * (t * kWave + lane);
            if (act && k < nv) {
                const f4 o4 = *reinterpret_cast<const f4 *>(pin + row + k);
                const f4 s4 = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(fst + row + k));
                f4 d4[4];
#pragma unroll
                for (int q = 0; q < 4; q++) d4[q] = *reinterpret_cast<const f4 *>(dsrc[q] + k);
                T2 d0[4], d1[4], e0 = {0, 0}, e1 = {0, 0};
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    d0[q].x = d4[q].x;
                    d0[q].y = d4[q].y;
                    d1[q].x = d4[q].z;
                    d1[q].y = d4[q].w;
                }
                if constexpr (SO) {
                    const f4 e4 = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(eterm + row + k));
                    e0.x = e4.x;
                    e0.y = e4.y;
                    e1.x = e4.z;
                    e1.y = e4.w;
                }
                const T2 r0 = update(a, b, d0, e0), r1 = update(a + 1, b, d1, e1);
                const f4 r4 = {(float)r0.x, (float)r0.y, (float)r1.x, (float)r1.y};
                __builtin_nontemporal_store(r4, reinterpret_cast<f4 *>(pout + row + k));
                T2 fs0, fs1, old0, old1;
                fs0.x = s4.x;
                fs0.y = s4.y;
                fs1.x = s4.z;
                fs1.y = s4.w;
                old0.x = o4.x;
                old0.y = o4.y;
                old1.x = o4.z;
                old1.y = o4.w;
                accumulate(a, b, k, r0, fs0, old0);
                accumulate(a + 1, b, k + 1, r1, fs1, old1);
            }
            a += da;
            b += db;
            if (a >= n1) {
                a -= n1;
                b++;
            }
        }
    } else {
        int a = lane % n1, b = lane / n1;
        const int da = kWave % n1, db = kWave / n1;
        const int nstep = (nv + kWave - 1) / kWave;
        for (int t = 0; t < nstep; t++) {
            const int k = t * kWave + lane;
            if (act && k < nv) {
                const T2 old = pin[row + k], fs = ntload2(&fst[row + k]);
                T2 dwn[4], e = {0, 0};
#pragma unroll
                for (int q = 0; q < 4; q++) dwn[q] = dsrc[q][k];
                if constexpr (SO) e = ntload2(&eterm[row + k]);
                const T2 r = update(a, b, dwn, e);
                __builtin_nontemporal_store(r.x, &pout[row + k].x);
                __builtin_nontemporal_store(r.y, &pout[row + k].y);
                accumulate(a, b, k, r, fs, old);
            }
            a += da;
            b += db;
            if (a >= n1) {
                a -= n1;
                b++;
            }
        }
    }
    double acc[9] = {A0, A1, A2, A3, A4, R, Pw, dn, dd};
    wave_sum<9>(acc);
    if (act && lane == 0) {
        adjoint_store(d, ac, wl, acc, d.aW[par ^ 1] + 8 * c, d.Phi[par ^ 1]);
        d.red[2 * c] = acc[7];
        d.red[2 * c + 1] = acc[8];
    }
}

// Adjoint moments What, rho_tau and wall multipliers Phi_l of phi[par] with
// no update (a loaded phi): the lane <-> velocity map, expressions and
// summation order of the adjoint sweep's epilogue, so the next sweep sees
// what a sweep that had produced this phi would have left.  CORR: phi is
// first corrected in place by the collision invariant -(z . Psi, z_3) of the
// adjoint prediction (z [nc][4]), and the moments are those of the result.
template <typename T, bool CORR = false>
__device__ __forceinline__ void adjoint_moments_patch(const DevSolve &d, int p, int par, const double *z = nullptr)
{
    using T2 = typename Vec2<T>::type;
    __shared__ PatchLds<T, false> sm;
    const int w = uni((int)(threadIdx.x / kWave)), lane = threadIdx.x % kWave;
    const int c0 = uni(d.patch[p]), cnt = uni(d.patch[p + 1]) - c0;
    const bool act = w < cnt;
    const int c = c0 + (act ? w : 0);
    const int nv = d.nv, n1 = d.n1;
    // read and (CORR) written in place: no restrict
    const T2 *pin = static_cast<const T2 *>(d.phi[par]);
    const T2 *__restrict__ fst = static_cast<const T2 *>(d.fstar);
    const T *__restrict__ gM = static_cast<const T *>(d.gM);
    const double *ac = d.acoef + kAcoef * c;
    const double u1 = uni(ac[1]), u2 = uni(ac[2]), th = uni(ac[3]);
    patch_tables<T, false>(d, sm, w, lane, u1, u2, 0.5 / th);
    const int l0 = uni(d.nbr[4 * c]);
    const int wl = l0 <= -2 ? -2 - l0 : -1;
    double S0x = 0, S0y = 0;
    if (wl >= 0) {
        S0x = uni(d.S[8 * c]);
        S0y = uni(d.S[8 * c + 1]);
    }
    const T gc = uni((T)ac[5]), th2 = uni((T)(0.5 * th));
    const AdjCell cq = {u1, u2, 0.5 * th, 0.5 * d.theta_w, S0x, S0y, wl, d.objective};
    const size_t row = (size_t)c * nv;
    __syncthreads();
    double A0 = 0, A1 = 0, A2 = 0, A3 = 0, A4 = 0, R = 0, Pw = 0;
    T2 *pio = static_cast<T2 *>(d.phi[par]);
    double zc[4] = {0, 0, 0, 0};
    if (CORR) {
#pragma unroll
        for (int i = 0; i < 4; i++) zc[i] = uni(z[4 * c + i]);
    }
    // one velocity: (CORR) the corrected value, returned for the store, and
    // its share of the sums
    auto accumulate = [&](int a, int b, int k, T2 r, T2 fs) {
        const double v1d = sm.vx[a], v2d = sm.vy[b];
        if (CORR) {
            const double s1 = ((zc[0] + zc[1] * v1d) + zc[2] * v2d) + zc[3] * (0.5 * (v1d * v1d + v2d * v2d));
            r.x = (T)((double)r.x - s1);
            r.y = (T)((double)r.y - zc[3]);
        }
        const double wt = sm.wx[a] * sm.wy[b];
        const double g1 = (double)(gc * sm.ex[w][a] * sm.ey[w][b]);
        const double g2 = (double)(th2 * (T)g1);
        adjoint_terms(A0, A1, A2, A3, A4, R, Pw, cq, v1d, v2d, wt, g1, g2, (double)r.x, (double)r.y, (double)fs.x,
                      (double)fs.y, gM, k);
        return r;
    };
    // streaming access as in the sweeps: the frozen f and the corrected row
    // are not read again here (non-temporal), FP32 pairs move 16 bytes
    if (act) {
        if (pair_velocities<T>(n1)) {
            int a = (2 * lane) % n1, b = (2 * lane) / n1;
            const int da = (2 * kWave) % n1, db = (2 * kWave) / n1;
            for (int k = 2 * lane; k < nv; k += 2 * kWave) {
                const f4 p4 = *reinterpret_cast<const f4 *>(pin + row + k);
                const f4 s4 = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(fst + row + k));
                T2 r0, r1, fs0, fs1;
                r0.x = p4.x;
                r0.y = p4.y;
                r1.x = p4.z;
                r1.y = p4.w;
                fs0.x = s4.x;
                fs0.y = s4.y;
                fs1.x = s4.z;
                fs1.y = s4.w;
                r0 = accumulate(a, b, k, r0, fs0);
                r1 = accumulate(a + 1, b, k + 1, r1, fs1);
                if (CORR) {
                    const f4 o4 = {(float)r0.x, (float)r0.y, (float)r1.x, (float)r1.y};
                    __builtin_nontemporal_store(o4, reinterpret_cast<f4 *>(pio + row + k));
                }
                a += da;
                b += db;
                if (a >= n1) {
                    a -= n1;
                    b++;
                }
            }
        } else {
            int a = lane % n1, b = lane / n1;
            const int da = kWave % n1, db = kWave / n1;
            for (int k = lane; k < nv; k += kWave) {
                const T2 r = accumulate(a, b, k, pin[row + k], ntload2(&fst[row + k]));
                if (CORR) {
                    __builtin_nontemporal_store(r.x, &pio[row + k].x);
                    __builtin_nontemporal_store(r.y, &pio[row + k].y);
                }
                a += da;
                b += db;
                if (a >= n1) {
                    a -= n1;
                    b++;
                }
            }
        }
    }
    double acc[7] = {A0, A1, A2, A3, A4, R, Pw};
    wave_sum<7>(acc);
    if (act && lane == 0) adjoint_store(d, ac, wl, acc, d.aW[par] + 8 * c, d.Phi[par]);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
constexpr int kPatchBlock = kPatchCells * kWave;   // threads of a patch workgroup
static_assert(kPatchCells >= 4, "the velocity tables are loaded by the first 256 threads");

template <typename T, bool SO>
__global__ __launch_bounds__(kPatchBlock) void k_primal_sweep(DevSolve d, int par)
{
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;
    primal_patch<T, SO>(d, p, par);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments(DevSolve d, int par)
{
    const int c = blockIdx.x * (kBlock / kWave) + (int)(threadIdx.x / kWave);
    if (c < d.nc) moments_wave<T>(d, c, par);
}

template <typename T, bool SO>
__global__ __launch_bounds__(kPatchBlock) void k_adjoint_sweep(DevSolve d, int par)
{
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;
    adjoint_patch<T, kAdjointExchange<T>, SO>(d, p, par);
}

template <typename T>
__global__ __launch_bounds__(kPatchBlock) void k_adjoint_moments(DevSolve d, int par)
{
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;
    adjoint_moments_patch<T>(d, p, par);
}

template <typename T>
__global__ __launch_bounds__(kPatchBlock) void k_adjoint_correct_moments(DevSolve d, int par, const double *z)
{
    const int p = xcd_item(d.np, blockIdx.x);
    if (p < 0) return;
    adjoint_moments_patch<T, true>(d, p, par, z);
}

// one sweep of the primal-phase (or adjoint-phase) members of a batch that
// run one scheme (SO: second order, the held corrections evaluated before
// the launch); a workgroup owns one (solve, patch).  Phases and schemes are
// separate kernels so that each gets the occupancy of its own registers.
template <typename T, bool SO>
__global__ __launch_bounds__(kPatchBlock) void k_batch_primal(const DevSolve *__restrict__ tab,
                                                              const int32_t *__restrict__ blk_solve,
                                                              const int32_t *__restrict__ blk_patch,
                                                              const int32_t *__restrict__ par0, int step)
{
    const int s = blk_solve[blockIdx.x];
    if (s < 0) return;
    primal_patch<T, SO>(tab[s], blk_patch[blockIdx.x], (par0[s] + step) & 1);
}

template <typename T, bool SO>
__global__ __launch_bounds__(kPatchBlock) void k_batch_adjoint(const DevSolve *__restrict__ tab,
                                                               const int32_t *__restrict__ blk_solve,
                                                               const int32_t *__restrict__ blk_patch,
                                                               const int32_t *__restrict__ par0, int step)
{
    const int s = blk_solve[blockIdx.x];
    if (s < 0) return;
    adjoint_patch<T, kAdjointExchange<T>, SO>(tab[s], blk_patch[blockIdx.x], (par0[s] + step) & 1);
}

// Block tables of a batch on the device (the allocation-free batch): block
// b of group g runs on XCD x = b % 8 and is the (b / 8)-th slot of that
// XCD's column, which holds, member after member of the group in table
// order, the x-th eighth of each member's patches (ceil(np / 8) of them, the
// last eighth possibly shorter); slots past the last member are padding (-1).
// The same map as the host-built one of dvm_batch_create.
struct BatchGroups {
    int nb[4];
};

__global__ __launch_bounds__(kBlock) void k_batch_tables(const DevSolve *__restrict__ tab,
                                                         const int32_t *__restrict__ phase, int n, BatchGroups grp,
                                                         int32_t *__restrict__ blk_solve,
                                                         int32_t *__restrict__ blk_patch)
{
    const int total = grp.nb[0] + grp.nb[1] + grp.nb[2] + grp.nb[3];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= total) return;
    int g = 0, local = b;
    while (local >= grp.nb[g]) {
        local -= grp.nb[g];
        g++;
    }
    const int x = local & 7;
    int slot = local >> 3, solve = -1, patch = 0;
    for (int i = 0; i < n; i++) {
        if (2 * phase[i] + (tab[i].order == 2 ? 1 : 0) != g) continue;
        const int np = tab[i].np, per = (np + 7) / 8;
        const int p0 = x * per, cnt = max(0, min(np, p0 + per) - p0);
        if (slot < cnt) {
            solve = i;
            patch = p0 + slot;
            break;
        }
        slot -= cnt;
    }
    blk_solve[b] = solve;
    blk_patch[b] = solve >= 0 ? patch : 0;
}

// The fixed device array of the allocation-free batch (one per GPU the
// library runs on; held until the process ends).  Host code reaches it only
// through the address static_batch_scratch looks up for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticBatchBytes];

hipError_t static_batch_scratch(char **out)
{
    constexpr int kMaxDevices = 64;
    static char *addr[kMaxDevices] = {};
    static std::mutex mu;
    int dev = 0;
    if (hipError_t e = hipGetDevice(&dev)) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) return e;
        addr[dev] = static_cast<char *>(p);
    }
    *out = addr[dev];
    return hipSuccess;
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

// per-cell adjoint coefficients from the frozen moments, one wave per cell:
// ac[0..3] the equilibrium's (rho, u1, u2, theta), ac[4] 1/tau (the cell's
// own rho, theta), ac[5] rho/(2 pi theta) of the equilibrium, ac[6..9]
// (1/tau) dtau/dW, ac[16..31] dP/dW (row = parameter, column = moment)
__global__ __launch_bounds__(kBlock) void k_adjoint_coef(DevSolve d, const double *Wst)
{
    const int c = blockIdx.x * (kBlock / kWave) + (int)(threadIdx.x / kWave);
    if (c >= d.nc) return;                      // whole waves; the kernel has no block barrier
    const double *W = Wst + 4 * c;
    const double rho = W[0], u1 = W[1] / rho, u2 = W[2] / rho, E = W[3] / rho;
    const double th = (2.0 / 3.0) * (E - 0.5 * (u1 * u1 + u2 * u2));
    const double itau = d.inv_tau_inf * rho * sqrt(2.0 * th);
    const double ir = 1.0 / rho, k23 = 2.0 / 3.0;
    // d theta / dW of the cell's own primitive variables
    const double dth0 = k23 * (u1 * u1 + u2 * u2 - E) * ir, dth1 = -k23 * u1 * ir, dth2 = -k23 * u2 * ir,
                 dth3 = k23 * ir;
    double P[4] = {rho, u1, u2, th}, M[16];
    if (d.equil) {
        const double Wv[4] = {W[0], W[1], W[2], W[3]};
        eq_conservative(d, Wv, P, M);
    } else {
        const double J[16] = {1.0, 0.0, 0.0, 0.0, -u1 * ir, ir, 0.0, 0.0, -u2 * ir, 0.0, ir, 0.0,
                              dth0, dth1, dth2, dth3};
#pragma unroll
        for (int q = 0; q < 16; q++) M[q] = J[q];
    }
    if (threadIdx.x % kWave != 0) return;
    double *ac = d.acoef + kAcoef * c;
    ac[0] = P[0];
    ac[1] = P[1];
    ac[2] = P[2];
    ac[3] = P[3];
    ac[4] = itau;
    ac[5] = P[0] / (2.0 * kPi * P[3]);
    // (1/tau) dtau/dW, tau ~ 1 / (rho sqrt(theta)) (hard sphere)
    const double h = 0.5 / th;
    ac[6] = -ir - h * dth0;
    ac[7] = -h * dth1;
    ac[8] = -h * dth2;
    ac[9] = -h * dth3;
    ac[10] = E;
    for (int q = 11; q < 16; q++) ac[q] = 0.0;
    for (int q = 0; q < 16; q++) ac[16 + q] = M[q];
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
// launchers
// ---------------------------------------------------------------------------
static inline int ew_grid(size_t n) { return (int)std::min<size_t>((n + kBlock - 1) / kBlock, 8192); }

hipError_t launch_primal_init(const DevSolve &d, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_fill_fd<T>, dim3(ew_grid((size_t)d.nc * d.nv)), dim3(kBlock), 0, st, d, 0));
    if (hipError_t e = hipGetLastError()) return e;
    return launch_moments(d, 0, st);
}

hipError_t launch_moments(const DevSolve &d, int par, hipStream_t st)
{
    constexpr int per_block = kBlock / kWave;
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_moments<T>, dim3((d.nc + per_block - 1) / per_block), dim3(kBlock), 0,
                                             st, d, par));
    return hipGetLastError();
}

hipError_t launch_primal_sweep(const DevSolve &d, int par, hipStream_t st)
{
    if (d.order == 2)
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_primal_sweep<T, true>), dim3(xcd_grid(d.np)), dim3(kPatchBlock), 0,
                                                 st, d, par));
    else
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_primal_sweep<T, false>), dim3(xcd_grid(d.np)), dim3(kPatchBlock), 0,
                                                 st, d, par));
    return hipGetLastError();
}

hipError_t launch_residual(const DevSolve &d, int adjoint, hipStream_t st)
{
    hipLaunchKernelGGL(k_residual, dim3(1), dim3(kBlock), 0, st, d.red, d.nc, d.out + (adjoint ? 4 : 2));
    return hipGetLastError();
}

hipError_t launch_objective(const DevSolve &d, int par, hipStream_t st)
{
    if (d.order == 2) {
        if (hipError_t e = launch_so_objective_elem(d, par, st)) return e;
    } else {
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_objective_elem<T>, dim3(d.nw), dim3(kBlock), 0, st, d, par));
        if (hipError_t e = hipGetLastError()) return e;
    }
    hipLaunchKernelGGL(k_objective_sum, dim3(1), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_adjoint_init(const DevSolve &d, int fpar, hipStream_t st)
{
    constexpr int per_block = kBlock / kWave;
    hipLaunchKernelGGL(k_adjoint_coef, dim3((d.nc + per_block - 1) / per_block), dim3(kBlock), 0, st, d, d.W[fpar]);
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

// Discrete-conservative equilibrium parameters P'(W[par]) of every cell
// (and dP'/dW if with_M) into mstate: kEqGroup lanes per cell, so one wave
// serves several cells and the Newton steps' reductions span a few lanes.
// On the 256x128 grid with 64x64 velocities: 1, 2, 4, 8, 16 and 32 lanes
// per cell take 113, 79, 78, 100, 149 and 243 us.
constexpr int kEqGroup = 4;

__device__ __forceinline__ void eq_params_cell(const DevSolve &d, int c, int par, int with_M)
{
    const double *Wc = d.W[par] + 4 * c;
    const double W[4] = {Wc[0], Wc[1], Wc[2], Wc[3]};
    const double rho = W[0], u1 = W[1] / rho, u2 = W[2] / rho;
    const double th = (2.0 / 3.0) * (W[3] / rho - 0.5 * (u1 * u1 + u2 * u2));
    double P[4] = {rho, u1, u2, th}, M[16];
    eq_conservative<kEqGroup>(d, W, P, with_M ? M : nullptr);
    if (threadIdx.x % kEqGroup != 0) return;
    double *o = d.mstate + kEqState * c;
#pragma unroll
    for (int a = 0; a < 4; a++) o[a] = P[a];
    if (with_M) {
#pragma unroll
        for (int q = 0; q < 16; q++) o[4 + q] = M[q];
    }
}

__global__ __launch_bounds__(kBlock) void k_eq_params(DevSolve d, int par, int with_M)
{
    const int c = blockIdx.x * (kBlock / kEqGroup) + (int)(threadIdx.x / kEqGroup);
    if (c >= d.nc) return;                      // whole groups; shuffles stay inside a group
    eq_params_cell(d, c, par, with_M);
}

// the same for a group of batch members (member a: tab[idx[a]], state in
// buffer par[a]), bitwise the single-solve kernel's results
__global__ __launch_bounds__(kBlock) void k_eq_params_group(const DevSolve *__restrict__ tab, MacroGroup g,
                                                            int with_M)
{
    const int i = blockIdx.x * (kBlock / kEqGroup) + (int)(threadIdx.x / kEqGroup);
    if (i >= g.pre[g.n]) return;                // whole lane groups
    const int a = group_member(g, i);
    eq_params_cell(tab[g.idx[a]], i - g.pre[a], g.par[a], with_M);
}

hipError_t launch_eq_params(const DevSolve &d, int par, int with_M, hipStream_t st)
{
    if (!d.mstate || !d.equil) return hipErrorInvalidValue;
    constexpr int per_block = kBlock / kEqGroup;
    hipLaunchKernelGGL(k_eq_params, dim3((d.nc + per_block - 1) / per_block), dim3(kBlock), 0, st, d, par, with_M);
    return hipGetLastError();
}

hipError_t launch_eq_params_group(const DevSolve *tab, const MacroGroup &g, int with_M, hipStream_t st)
{
    if (g.n <= 0) return hipSuccess;
    constexpr int per_block = kBlock / kEqGroup;
    hipLaunchKernelGGL(k_eq_params_group, dim3((g.pre[g.n] + per_block - 1) / per_block), dim3(kBlock), 0, st, tab, g,
                       with_M);
    return hipGetLastError();
}

hipError_t launch_adjoint_correct_moments(const DevSolve &d, int par, const double *z, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_adjoint_correct_moments<T>, dim3(xcd_grid(d.np)), dim3(kPatchBlock), 0,
                                             st, d, par, z));
    return hipGetLastError();
}

hipError_t launch_adjoint_moments(const DevSolve &d, int par, hipStream_t st)
{
    DVM_DISPATCH(d.mixed, hipLaunchKernelGGL(k_adjoint_moments<T>, dim3(xcd_grid(d.np)), dim3(kPatchBlock), 0, st, d,
                                             par));
    return hipGetLastError();
}

hipError_t launch_adjoint_sweep(const DevSolve &d, int par, hipStream_t st)
{
    if (d.order == 2)
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_adjoint_sweep<T, true>), dim3(xcd_grid(d.np)), dim3(kPatchBlock), 0,
                                                 st, d, par));
    else
        DVM_DISPATCH(d.mixed, hipLaunchKernelGGL((k_adjoint_sweep<T, false>), dim3(xcd_grid(d.np)), dim3(kPatchBlock), 0,
                                                 st, d, par));
    return hipGetLastError();
}

hipError_t launch_batch(const DevSolve *tab, const int32_t *blk_solve, const int32_t *blk_patch,
                        const int32_t *par0, int step, int nblocks, int mixed, int adjoint, int so, hipStream_t st)
{
    if (nblocks <= 0) return hipSuccess;
    if (adjoint && so)
        DVM_DISPATCH(mixed, hipLaunchKernelGGL((k_batch_adjoint<T, true>), dim3(nblocks), dim3(kPatchBlock), 0, st,
                                               tab, blk_solve, blk_patch, par0, step));
    else if (adjoint)
        DVM_DISPATCH(mixed, hipLaunchKernelGGL((k_batch_adjoint<T, false>), dim3(nblocks), dim3(kPatchBlock), 0, st,
                                               tab, blk_solve, blk_patch, par0, step));
    else if (so)
        DVM_DISPATCH(mixed, hipLaunchKernelGGL((k_batch_primal<T, true>), dim3(nblocks), dim3(kPatchBlock), 0, st,
                                               tab, blk_solve, blk_patch, par0, step));
    else
        DVM_DISPATCH(mixed, hipLaunchKernelGGL((k_batch_primal<T, false>), dim3(nblocks), dim3(kPatchBlock), 0, st,
                                               tab, blk_solve, blk_patch, par0, step));
    return hipGetLastError();
}

hipError_t launch_batch_tables(const DevSolve *tab, const int32_t *phase, int n, const int *nb_group,
                               int32_t *blk_solve, int32_t *blk_patch, hipStream_t st)
{
    BatchGroups grp;
    int total = 0;
    for (int g = 0; g < 4; g++) {
        grp.nb[g] = nb_group[g];
        total += nb_group[g];
    }
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_tables, dim3((total + kBlock - 1) / kBlock), dim3(kBlock), 0, st, tab, phase, n, grp,
                       blk_solve, blk_patch);
    return hipGetLastError();
}

hipError_t launch_batch_residual(const DevSolve *tab, int n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_residual, dim3(n), dim3(kBlock), 0, st, tab, out);
    return hipGetLastError();
}

}  // namespace dvm
