/*
 * ORACLE -- test infrastructure only.
 *
 * A plain, slow, FP64 CPU implementation of the discrete-velocity BGK
 * primal and adjoint solvers and the wall shape sensitivity of Yuan & Wu,
 * "Adjoint shape optimization from the continuum to free-molecular gas
 * flows" (arXiv 2501.00923).  It exists to check the GPU library; only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no source with the GPU library.
 *
 * What each part follows (sections / equations of the paper):
 *   conservative moments W = sum_k w_k Psi_k . f_k     Sec. 2.2, eq. (macint_reduce)
 *   reduced Maxwellian g1, g2 = RT/2 g1               Sec. 2.2, eq. (maxwell_reduce)
 *   relaxation time tau = mu/p, hard sphere           Sec. 2.1
 *   Kn -> tau_inf                                     Sec. 2.1, eq. (kndefine)
 *   far-field Dirichlet inflow                        Sec. 2.3, eq. (bc_drlt)
 *   diffuse wall, F_rho_w and normalised g_w          Sec. 2.3 / 3.2, eqs. (formula_bgk_fdw), (barg)
 *   objective J (drag m_J = v1, heat m_J = v^2/2)     Sec. 2.4, eq. (formula_opt); Sec. 3.2 eq. (numer_J)
 *   primal finite-volume DVM balance                  Sec. 3.1, eq. (numerpr_gov)
 *   adjoint equation, collision terms, wall BC        Sec. 2.5, eqs. (formula_adjointbgk),
 *                                                     (adjoint_eqdefines), (adjoint_macdefines);
 *                                                     Sec. 3.1, eq. (numerad_gov)
 *   wall-element derivatives of J and B_w             Sec. 3.2, eqs. (sens_J_itf), (gaussgrad), (sens_B_itf)
 *   element -> node transform                         Sec. 3.2, eq. (sens_nod)
 *   second-order spatial reconstruction               Sec. 3.1 (readings in its section below)
 *
 * Readings where the paper is silent (the paper omits its solver scheme,
 * Sec. 3.1):
 *   - first-order upwind face values, Jacobi point-implicit iteration
 *     f^{n+1} = (inflow + V g^n / tau^n) / (outflow + V / tau^n), every
 *     per-cell quantity (W, tau, g, wall flux F) taken from f^n;
 *   - nondimensional units rho_inf = 1, theta = RT with theta_inf = 1/2
 *     (velocity unit sqrt(2 R T_inf)), gamma = 5/3 (three translational
 *     degrees of freedom, as the reduction from 3-D velocity implies),
 *     u_inf = Ma sqrt(gamma theta_inf) along x;
 *   - tau_inf = (5 sqrt(pi) / 8) Kn l_ref with l_ref = 1;
 *   - velocities with v.n = 0 count as incoming (Xi^-); every flux carries
 *     the factor v.n so the choice is immaterial;
 *   - the adjoint is the exact transpose of the discrete primal map under
 *     the inner product sum_k w_k (.); with first-order upwinding it
 *     coincides term by term with the upwind discretisation of the paper's
 *     continuous adjoint equation and its wall condition;
 *   - eq. (sens_B_itf) for dB/dn carries the element length A_l like the
 *     other two lines; the inner sums run over a separate dummy index;
 *   - the surface-element value of f on Xi^+ is the wall cell's value (first
 *     order), on Xi^- it is F_l * gbar (the discrete diffuse condition).
 *
 * Pins (tests/test_oracle_*.py): velocity quadrature exactness and symmetry;
 * Maxwellian moments against closed forms; dg/dW and dtau/dW by complex
 * step; zero wall mass flux; a uniform Maxwellian at rest is stationary;
 * free-molecular drag against the closed form; dot-product identity of the
 * adjoint operator against a complex-step linearisation of the primal
 * residual; adjoint dJ/dp against central finite differences for Kn, Ma
 * and T_w; wall-element derivatives against finite differences of the
 * discrete J and B_w expressions; node transform against finite
 * differences of the element geometry; mirror symmetry of the
 * sensitivities.  The end-to-end shape derivative of the paper is its
 * wall-only approximation (Sec. 2.5: volume-mesh motion is not
 * differentiated); its agreement with finite differences is a
 * discretisation-level trend, not an identity (parity unpinned beyond the
 * element-level pins above).  The exact discrete shape derivative
 * (or_mesh_sensitivity, the Lagrangian differentiated in every node
 * coordinate by complex step) is pinned by translation invariance and by
 * central differences of the re-converged drag under shape change, for the
 * first-order scheme and for the second-order one (limiter factors of f held
 * fixed; exact with the limiter off, a percent-level approximation with it).
 * Second-order scheme (tests/test_oracle_second_order.py): exact slopes and
 * face values for linear fields on equal parallelograms; the limiter's
 * overshoot bound and smoothness; the defect-correction fixed point solves R2 = 0 independently of
 * the correction interval; drag converges at second order under O-grid
 * refinement (first order for the first-order scheme); dot-product identity
 * of the frozen-limiter adjoint against the complex twin of R2 and J;
 * unlimited adjoint dJ/dp against central differences.  The wall and mesh
 * sensitivities are first-order only.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_VK_KAPPA 1e-3   /* Venkatakrishnan limiter: e = OR_VK_KAPPA |f_c| */

/* face order per cell: 0 = j-, 1 = i+, 2 = j+, 3 = i- ; neighbour code:
 * >= 0 interior cell, -1 far field, -2 - l wall element l */

typedef struct {
    int topo, ni, nj, nwake, nc, nw;
    int *nbr;          /* [nc][4] */
    double *S;         /* [nc][4][2]  A n, outward of the cell */
    double *vol;       /* [nc] */
    double *cen;       /* [nc][2] */
    int *wall_cell;    /* [nw] */
    int *wall_face;    /* [nw] face slot of the wall cell */
    double *wA, *wn, *wx;   /* [nw], [nw][2], [nw][2] */
    double *wa, *wb;   /* element end nodes x_{l,1}, x_{l,2} [nw][2] */

    int n1, n2, nv;
    double *v;         /* [nv][2] */
    double *w;         /* [nv] */

    double Kn, Ma, Tw, inv_tau_inf, theta_inf, theta_w, u_inf;
    int objective;
    double *fd;        /* [nv][2] far-field Maxwellian */
    double *gM;        /* [nv] g_M1(1, 0, T_w) */
    double *D;         /* [nw] normalisation of eq. (barg) */
    double *mJ;        /* [nv] */

    double *f, *fn;    /* [nc][nv][2] */
    double *W;         /* [nc][4] moments of f */
    double *F;         /* [nw] wall incoming mass flux of f */
    double *phi, *phin;
    double *cellred;   /* [nc][2] residual partials */
    double *nodes;     /* [(nj+1)(ni+1)][2] mesh node coordinates */
    int nthreads;

    /* second-order scheme (order 2; see "second-order reconstruction") */
    int order, limiter, kcorr;
    double *fm;        /* [nc][4][2] face midpoints */
    double *corr;      /* [nc][nv][2] held second-order flux correction */
    double *dF;        /* [nw] held wall-flux correction */
    int corr_ok, since;
    double *psi;       /* [nc][nv][2] limiter of the frozen f (adjoint) */
    double *acorr;     /* [nc][nv][2] held adjoint reconstruction term */
    int acorr_ok, asince;

    /* equilibrium: 0 pointwise Maxwellian of the cell's primitive variables,
     * 1 discrete-conservative (see "discrete-conservative equilibrium") */
    int equilibrium;
    double *eqP;       /* [nc][4] (rho', u1', u2', theta') of the current W */
    double *eqM;       /* [nc][4][4] d(rho', u1', u2', theta')/dW */
    int eq_ok;         /* eqP, eqM hold the current W */

    /* prediction acceleration (primal, first order; see "macroscopic
     * prediction"): every acc_every sweeps, acc_inner red-black block
     * Gauss-Seidel steps on the macroscopic system */
    int acc_every, acc_inner, acc_sweeps;
    double acc_alpha;
    /* adjoint prediction: the primal macroscopic system at the frozen f,
     * sweeps of the adjoint phase */
    double *aDinv, *aO;
    int acc_asweeps;
} or_problem;

/* ------------------------------------------------------------------ */
/* velocity grids                                                      */
/* ------------------------------------------------------------------ */

/* 1-D rules on [-vmax, vmax]. kind 0: n midpoint cells; kind 1: n-point
 * composite Newton-Cotes (Simpson on both sides of one centred 3/8 panel,
 * n divisible by 4); kind 2: x = vmax sinh(b s)/sinh(b), s at the n cell
 * midpoints of (-1, 1), weight = width of the mapped cell. Returns 0 or -1. */
int or_vgrid_1d(int kind, int n, double vmax, double param, double *x, double *w)
{
    if (n < 2 || vmax <= 0) return -1;
    if (kind == 0) {
        double h = 2.0 * vmax / n;
        for (int a = 0; a < n; a++) { x[a] = -vmax + (a + 0.5) * h; w[a] = h; }
        return 0;
    }
    if (kind == 1) {
        if (n % 4 != 0) return -1;
        int m = n - 1;               /* intervals */
        int ms = (m - 3) / 2;        /* Simpson intervals on each side (even) */
        double h = 2.0 * vmax / m;
        for (int a = 0; a < n; a++) { x[a] = -vmax + a * h; w[a] = 0.0; }
        for (int a = 0; a < ms; a += 2) {            /* left Simpson panels */
            w[a] += h / 3.0; w[a + 1] += 4.0 * h / 3.0; w[a + 2] += h / 3.0;
        }
        w[ms] += 3.0 * h / 8.0; w[ms + 1] += 9.0 * h / 8.0;
        w[ms + 2] += 9.0 * h / 8.0; w[ms + 3] += 3.0 * h / 8.0;
        for (int a = ms + 3; a < m; a += 2) {        /* right Simpson panels */
            w[a] += h / 3.0; w[a + 1] += 4.0 * h / 3.0; w[a + 2] += h / 3.0;
        }
        return 0;
    }
    if (kind == 2) {
        double b = param > 0 ? param : 2.0;
        double sb = sinh(b);
        for (int a = 0; a < n; a++) {
            double s = -1.0 + (a + 0.5) * 2.0 / n;
            double sl = -1.0 + a * 2.0 / n, sr = -1.0 + (a + 1) * 2.0 / n;
            x[a] = vmax * sinh(b * s) / sb;
            w[a] = vmax * (sinh(b * sr) - sinh(b * sl)) / sb;   /* mapped cell width */
        }
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------ */
/* Maxwellian and moments                                              */
/* ------------------------------------------------------------------ */

/* reduced Maxwellian, eq. (maxwell_reduce), theta = RT */
static double maxwell1(double rho, double u1, double u2, double th, double v1, double v2)
{
    double c1 = v1 - u1, c2 = v2 - u2;
    return rho / (2.0 * OR_PI * th) * exp(-(c1 * c1 + c2 * c2) / (2.0 * th));
}

/* primitive variables from W = (rho, rho u1, rho u2, rho E), Sec. 2.1 with
 * 1/(gamma-1) = 3/2 */
static void prim(const double *W, double *rho, double *u1, double *u2, double *th)
{
    *rho = W[0];
    *u1 = W[1] / W[0];
    *u2 = W[2] / W[0];
    *th = (2.0 / 3.0) * (W[3] / W[0] - 0.5 * ((*u1) * (*u1) + (*u2) * (*u2)));
}

void or_maxwell(double rho, double u1, double u2, double th, int nv, const double *v, double *g)
{
    for (int k = 0; k < nv; k++) {
        double g1 = maxwell1(rho, u1, u2, th, v[2 * k], v[2 * k + 1]);
        g[2 * k] = g1;
        g[2 * k + 1] = 0.5 * th * g1;
    }
}

/* W = sum_k w_k Psi_k . f_k with Psi = [[1,0],[v,0],[v^2/2,1]] */
void or_moments(int nv, const double *v, const double *w, const double *f, double *W)
{
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int k = 0; k < nv; k++) {
        double v1 = v[2 * k], v2 = v[2 * k + 1];
        double f1 = f[2 * k], f2 = f[2 * k + 1];
        s0 += w[k] * f1;
        s1 += w[k] * v1 * f1;
        s2 += w[k] * v2 * f1;
        s3 += w[k] * (0.5 * (v1 * v1 + v2 * v2) * f1 + f2);
    }
    W[0] = s0; W[1] = s1; W[2] = s2; W[3] = s3;
}

/* 1/tau for a cell: tau = tau_inf * (rho_inf sqrt(theta_inf)) / (rho sqrt(theta)),
 * rho_inf = 1, theta_inf = 1/2 */
static double inv_tau_of(const or_problem *p, double rho, double th)
{
    return p->inv_tau_inf * rho * sqrt(2.0 * th);
}

/* d g_c / d W (2 x 4) for a cell state W at velocity v; chain rule through
 * (rho, u1, u2, theta).  Also returns (1/tau) d tau / d W. */
static void dg_dW(double rho, double u1, double u2, double th, double E,
                  double v1, double v2, double dg[2][4], double dtau_over_tau[4])
{
    double g1 = maxwell1(rho, u1, u2, th, v1, v2);
    double c1 = v1 - u1, c2 = v2 - u2, cc = c1 * c1 + c2 * c2;
    /* d g1 / d(rho, u1, u2, theta) */
    double dP[4] = { g1 / rho, g1 * c1 / th, g1 * c2 / th, g1 * (cc / (2 * th * th) - 1.0 / th) };
    /* d g2 / d(prim) = th/2 dg1 + g1/2 on theta */
    double dP2[4] = { 0.5 * th * dP[0], 0.5 * th * dP[1], 0.5 * th * dP[2], 0.5 * th * dP[3] + 0.5 * g1 };
    /* d prim / d W */
    double J[4][4] = {
        { 1.0, 0.0, 0.0, 0.0 },
        { -u1 / rho, 1.0 / rho, 0.0, 0.0 },
        { -u2 / rho, 0.0, 1.0 / rho, 0.0 },
        { (2.0 / 3.0) * (u1 * u1 + u2 * u2 - E) / rho, -(2.0 / 3.0) * u1 / rho,
          -(2.0 / 3.0) * u2 / rho, (2.0 / 3.0) / rho } };
    for (int m = 0; m < 4; m++) {
        double a = 0, b = 0;
        for (int q = 0; q < 4; q++) { a += dP[q] * J[q][m]; b += dP2[q] * J[q][m]; }
        dg[0][m] = a; dg[1][m] = b;
        /* tau ~ 1 / (rho sqrt(theta)) */
        dtau_over_tau[m] = -J[0][m] / rho - 0.5 * J[3][m] / th;
    }
}

void or_dg_dW(double rho, double u1, double u2, double th, double v1, double v2,
              double *dg /*[2][4]*/, double *dtt /*[4]*/)
{
    double E = 0.5 * (u1 * u1 + u2 * u2) + 1.5 * th;
    double a[2][4], b[4];
    dg_dW(rho, u1, u2, th, E, v1, v2, a, b);
    memcpy(dg, a, sizeof(a));
    memcpy(dtt, b, sizeof(b));
}

/* ------------------------------------------------------------------ */
/* discrete-conservative equilibrium                                   */
/* ------------------------------------------------------------------ */
/* A reading of the equilibrium on a discrete velocity grid, taken as an
 * option (the pointwise Maxwellian of the cell's primitive variables stays
 * the default): the equilibrium of a cell is the reduced Maxwellian
 * g(P') whose moments on the grid equal the cell's moments,
 *     sum_k w_k Psi_k g_k(P') = W,
 * with P' = (rho', u1', u2', theta') found by Newton's method from the
 * primitive variables of W (on a grid that integrates the Maxwellian
 * exactly, P' = P(W)).  The discrete BGK collision term then conserves mass,
 * momentum and energy, as the continuous one does (Sec. 2.1); tau keeps the
 * cell's own rho and theta.  Newton runs a fixed number of steps (the
 * quadrature error of a usable grid is at most a few percent, and each step
 * squares the relative error). */
#define OR_EQ_NEWTON 6

/* moments m = sum_k w Psi g(P) and their Jacobian dm/dP at P */
static void eq_moments_jac(const or_problem *p, const double P[4], double m[4], double J[4][4])
{
    const double rho = P[0], u1 = P[1], u2 = P[2], th = P[3];
    for (int a = 0; a < 4; a++) { m[a] = 0; for (int b = 0; b < 4; b++) J[a][b] = 0; }
    for (int k = 0; k < p->nv; k++) {
        double v1 = p->v[2 * k], v2 = p->v[2 * k + 1], w = p->w[k];
        double g1 = maxwell1(rho, u1, u2, th, v1, v2), g2 = 0.5 * th * g1;
        double c1 = v1 - u1, c2 = v2 - u2, cc = c1 * c1 + c2 * c2;
        double d1[4] = { g1 / rho, g1 * c1 / th, g1 * c2 / th, g1 * (cc / (2 * th * th) - 1.0 / th) };
        double d2[4] = { 0.5 * th * d1[0], 0.5 * th * d1[1], 0.5 * th * d1[2], 0.5 * th * d1[3] + 0.5 * g1 };
        double psi[4] = { 1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2) };
        for (int a = 0; a < 4; a++) {
            m[a] += w * (psi[a] * g1 + (a == 3 ? g2 : 0.0));
            for (int b = 0; b < 4; b++) J[a][b] += w * (psi[a] * d1[b] + (a == 3 ? d2[b] : 0.0));
        }
    }
}

/* x = A^{-1} b by Gaussian elimination with partial pivoting (A, b copied) */
static void solve4(const double A_in[4][4], const double b_in[4], double x[4])
{
    double A[4][5];
    for (int a = 0; a < 4; a++) { for (int b = 0; b < 4; b++) A[a][b] = A_in[a][b]; A[a][4] = b_in[a]; }
    for (int col = 0; col < 4; col++) {
        int piv = col;
        for (int r = col + 1; r < 4; r++) if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (piv != col) for (int b = 0; b < 5; b++) { double t = A[col][b]; A[col][b] = A[piv][b]; A[piv][b] = t; }
        for (int r = col + 1; r < 4; r++) {
            double fct = A[r][col] / A[col][col];
            for (int b = col; b < 5; b++) A[r][b] -= fct * A[col][b];
        }
    }
    for (int r = 3; r >= 0; r--) {
        double acc = A[r][4];
        for (int b = r + 1; b < 4; b++) acc -= A[r][b] * x[b];
        x[r] = acc / A[r][r];
    }
}

/* equilibrium parameters P' of moments W; M (may be NULL) receives
 * dP'/dW = (dm/dP')^{-1} at P' (pointwise: d(rho, u, theta)/dW) */
static void eq_params(const or_problem *p, const double *W, double P[4], double M[4][4])
{
    prim(W, &P[0], &P[1], &P[2], &P[3]);
    int conservative = p->equilibrium == 1;
    if (conservative) {
        for (int it = 0; it < OR_EQ_NEWTON; it++) {
            double m[4], J[4][4], r[4], dP[4];
            eq_moments_jac(p, P, m, J);
            for (int a = 0; a < 4; a++) r[a] = W[a] - m[a];
            solve4(J, r, dP);
            for (int a = 0; a < 4; a++) P[a] += dP[a];
        }
        /* a grid too coarse for the state (a Maxwellian much narrower than
         * the velocity spacing) can leave Newton without a usable root: the
         * cell then keeps the pointwise Maxwellian of its primitive variables */
        if (!(P[0] > 0) || !(P[3] > 0) || !isfinite(P[1]) || !isfinite(P[2])) {
            prim(W, &P[0], &P[1], &P[2], &P[3]);
            conservative = 0;
        }
    }
    if (!M) return;
    if (conservative) {
        double m[4], J[4][4];
        eq_moments_jac(p, P, m, J);
        for (int b = 0; b < 4; b++) {
            double e[4] = { 0, 0, 0, 0 }, col[4];
            e[b] = 1.0;
            solve4(J, e, col);
            for (int a = 0; a < 4; a++) M[a][b] = col[a];
        }
    } else {
        const double rho = P[0], u1 = P[1], u2 = P[2], E = W[3] / W[0];
        double J[4][4] = {
            { 1.0, 0.0, 0.0, 0.0 },
            { -u1 / rho, 1.0 / rho, 0.0, 0.0 },
            { -u2 / rho, 0.0, 1.0 / rho, 0.0 },
            { (2.0 / 3.0) * (u1 * u1 + u2 * u2 - E) / rho, -(2.0 / 3.0) * u1 / rho,
              -(2.0 / 3.0) * u2 / rho, (2.0 / 3.0) / rho } };
        memcpy(M, J, sizeof J);
    }
}

/* eqP, eqM of the current W (every cell) */
static void eq_cache(or_problem *p)
{
    if (p->eq_ok) return;
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
    for (int c = 0; c < p->nc; c++) {
        double M[4][4];
        eq_params(p, p->W + 4 * c, p->eqP + 4 * c, M);
        memcpy(p->eqM + 16 * c, M, sizeof M);
    }
    p->eq_ok = 1;
}

/* d g_c / d W (2 x 4) at velocity k of cell c for the current W, through
 * the equilibrium parameters, and (1/tau) d tau / d W (tau from the cell's
 * own rho, theta) */
static void dg_dW_cell(or_problem *p, int c, int k, double dg[2][4], double dtt[4])
{
    eq_cache(p);
    const double *P = p->eqP + 4 * c, *M = p->eqM + 16 * c;
    double rho, u1, u2, th;
    prim(p->W + 4 * c, &rho, &u1, &u2, &th);
    double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
    double g1 = maxwell1(P[0], P[1], P[2], P[3], v1, v2);
    double c1 = v1 - P[1], c2 = v2 - P[2], cc = c1 * c1 + c2 * c2, t = P[3];
    double d1[4] = { g1 / P[0], g1 * c1 / t, g1 * c2 / t, g1 * (cc / (2 * t * t) - 1.0 / t) };
    double d2[4] = { 0.5 * t * d1[0], 0.5 * t * d1[1], 0.5 * t * d1[2], 0.5 * t * d1[3] + 0.5 * g1 };
    /* d(rho, theta)/dW of the cell's own primitive variables for tau */
    const double E = p->W[4 * c + 3] / p->W[4 * c];
    const double drho[4] = { 1.0, 0.0, 0.0, 0.0 };
    const double dth[4] = { (2.0 / 3.0) * (u1 * u1 + u2 * u2 - E) / rho, -(2.0 / 3.0) * u1 / rho,
                            -(2.0 / 3.0) * u2 / rho, (2.0 / 3.0) / rho };
    for (int m = 0; m < 4; m++) {
        double a = 0, b = 0;
        for (int q = 0; q < 4; q++) { a += d1[q] * M[4 * q + m]; b += d2[q] * M[4 * q + m]; }
        dg[0][m] = a; dg[1][m] = b;
        dtt[m] = -drho[m] / rho - 0.5 * dth[m] / th;
    }
}

/* equilibrium (g1, g2) of cell c at velocity k for the current W */
static void eq_cell_g(or_problem *p, int c, int k, double *g1, double *g2)
{
    eq_cache(p);
    const double *P = p->eqP + 4 * c;
    *g1 = maxwell1(P[0], P[1], P[2], P[3], p->v[2 * k], p->v[2 * k + 1]);
    *g2 = 0.5 * P[3] * (*g1);
}

/* complex twin of eq_params (complex-step pins): the same Newton steps */
static void eq_params_z(const or_problem *p, const double complex *W, double complex P[4])
{
    P[0] = W[0]; P[1] = W[1] / W[0]; P[2] = W[2] / W[0];
    P[3] = (2.0 / 3.0) * (W[3] / W[0] - 0.5 * (P[1] * P[1] + P[2] * P[2]));
    if (p->equilibrium != 1) return;
    double complex P0[4] = { P[0], P[1], P[2], P[3] };
    for (int it = 0; it < OR_EQ_NEWTON; it++) {
        double complex m[4] = { 0, 0, 0, 0 }, A[4][5];
        for (int a = 0; a < 4; a++) for (int b = 0; b < 5; b++) A[a][b] = 0;
        for (int k = 0; k < p->nv; k++) {
            double v1 = p->v[2 * k], v2 = p->v[2 * k + 1], w = p->w[k];
            double complex c1 = v1 - P[1], c2 = v2 - P[2], cc = c1 * c1 + c2 * c2, t = P[3];
            double complex g1 = P[0] / (2 * OR_PI * t) * cexp(-cc / (2 * t)), g2 = 0.5 * t * g1;
            double complex d1[4] = { g1 / P[0], g1 * c1 / t, g1 * c2 / t, g1 * (cc / (2 * t * t) - 1.0 / t) };
            double complex d2[4] = { 0.5 * t * d1[0], 0.5 * t * d1[1], 0.5 * t * d1[2], 0.5 * t * d1[3] + 0.5 * g1 };
            double psi[4] = { 1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2) };
            for (int a = 0; a < 4; a++) {
                m[a] += w * (psi[a] * g1 + (a == 3 ? g2 : 0.0));
                for (int b = 0; b < 4; b++) A[a][b] += w * (psi[a] * d1[b] + (a == 3 ? d2[b] : 0.0));
            }
        }
        for (int a = 0; a < 4; a++) A[a][4] = W[a] - m[a];
        for (int col = 0; col < 4; col++) {
            int piv = col;
            for (int r = col + 1; r < 4; r++) if (fabs(creal(A[r][col])) > fabs(creal(A[piv][col]))) piv = r;
            if (piv != col) for (int b = 0; b < 5; b++) { double complex tt = A[col][b]; A[col][b] = A[piv][b]; A[piv][b] = tt; }
            for (int r = col + 1; r < 4; r++) {
                double complex fct = A[r][col] / A[col][col];
                for (int b = col; b < 5; b++) A[r][b] -= fct * A[col][b];
            }
        }
        double complex x[4];
        for (int r = 3; r >= 0; r--) {
            double complex acc = A[r][4];
            for (int b = r + 1; b < 4; b++) acc -= A[r][b] * x[b];
            x[r] = acc / A[r][r];
        }
        for (int a = 0; a < 4; a++) P[a] += x[a];
    }
    if (!(creal(P[0]) > 0) || !(creal(P[3]) > 0) || !isfinite(creal(P[1])) || !isfinite(creal(P[2])))
        for (int a = 0; a < 4; a++) P[a] = P0[a];
}

int or_set_equilibrium(or_problem *p, int kind)
{
    if (kind != 0 && kind != 1) return -1;
    if (kind != 1 && p->acc_every > 0) return -1;
    p->equilibrium = kind;
    p->eq_ok = 0;
    return 0;
}

/* equilibrium parameters of a moment vector (pins): P[4], M[4][4] = dP/dW */
void or_eq_params(or_problem *p, const double *W, double *P, double *M)
{
    double Mm[4][4];
    eq_params(p, W, P, Mm);
    if (M) memcpy(M, Mm, sizeof Mm);
}

/* ------------------------------------------------------------------ */
/* mesh                                                                */
/* ------------------------------------------------------------------ */

static int node_id(const or_problem *p, int i, int j) { return i + (p->ni + 1) * j; }

static int build_mesh(or_problem *p, const double *nodes)
{
    int ni = p->ni, nj = p->nj;
    p->nc = ni * nj;
    p->nw = ni - 2 * p->nwake;
    p->nbr = malloc(sizeof(int) * 4 * p->nc);
    p->S = malloc(sizeof(double) * 8 * p->nc);
    p->vol = malloc(sizeof(double) * p->nc);
    p->cen = malloc(sizeof(double) * 2 * p->nc);
    p->fm = malloc(sizeof(double) * 8 * p->nc);
    p->wall_cell = malloc(sizeof(int) * p->nw);
    p->wall_face = malloc(sizeof(int) * p->nw);
    p->wA = malloc(sizeof(double) * p->nw);
    p->wn = malloc(sizeof(double) * 2 * p->nw);
    p->wx = malloc(sizeof(double) * 2 * p->nw);
    p->wa = malloc(sizeof(double) * 2 * p->nw);
    p->wb = malloc(sizeof(double) * 2 * p->nw);
    for (int j = 0; j < nj; j++) {
        for (int i = 0; i < ni; i++) {
            int c = i + ni * j;
            /* counter-clockwise corners */
            int cid[4] = { node_id(p, i, j), node_id(p, i + 1, j), node_id(p, i + 1, j + 1), node_id(p, i, j + 1) };
            double X[4], Y[4];
            for (int q = 0; q < 4; q++) { X[q] = nodes[2 * cid[q]]; Y[q] = nodes[2 * cid[q] + 1]; }
            /* shoelace area and centroid, in coordinates relative to the first
             * corner (thin wall cells far from the origin would otherwise
             * lose digits to cancellation) */
            double X0 = X[0], Y0 = Y[0], Xr[4], Yr[4];
            for (int q = 0; q < 4; q++) { Xr[q] = X[q] - X0; Yr[q] = Y[q] - Y0; }
            double A2 = 0, cx = 0, cy = 0;
            for (int q = 0; q < 4; q++) {
                int r = (q + 1) % 4;
                double cr = Xr[q] * Yr[r] - Xr[r] * Yr[q];
                A2 += cr;
                cx += (Xr[q] + Xr[r]) * cr;
                cy += (Yr[q] + Yr[r]) * cr;
            }
            if (!(A2 > 0)) return -1;
            p->vol[c] = 0.5 * A2;
            p->cen[2 * c] = X0 + cx / (3.0 * A2);
            p->cen[2 * c + 1] = Y0 + cy / (3.0 * A2);
            /* face q is the edge corner q -> corner q+1; outward normal
             * (dy, -dx) for a counter-clockwise walk */
            for (int q = 0; q < 4; q++) {
                int r = (q + 1) % 4;
                p->S[8 * c + 2 * q] = Y[r] - Y[q];
                p->S[8 * c + 2 * q + 1] = -(X[r] - X[q]);
                p->fm[8 * c + 2 * q] = 0.5 * (X[q] + X[r]);
                p->fm[8 * c + 2 * q + 1] = 0.5 * (Y[q] + Y[r]);
            }
            /* neighbours */
            int *nb = p->nbr + 4 * c;
            /* j- */
            if (j > 0) nb[0] = i + ni * (j - 1);
            else if (p->topo == 1 && (i < p->nwake || i >= ni - p->nwake)) nb[0] = (ni - 1 - i);
            else nb[0] = -2 - (i - p->nwake);
            /* i+ */
            if (i < ni - 1) nb[1] = c + 1;
            else nb[1] = (p->topo == 0) ? ni * j : -1;
            /* j+ */
            nb[2] = (j < nj - 1) ? c + ni : -1;
            /* i- */
            if (i > 0) nb[3] = c - 1;
            else nb[3] = (p->topo == 0) ? (ni - 1) + ni * j : -1;
        }
    }
    for (int l = 0; l < p->nw; l++) {
        int i = l + p->nwake;
        int c = i;                       /* j = 0 */
        p->wall_cell[l] = c;
        p->wall_face[l] = 0;
        double Sx = p->S[8 * c], Sy = p->S[8 * c + 1];
        double A = sqrt(Sx * Sx + Sy * Sy);
        p->wA[l] = A;
        p->wn[2 * l] = Sx / A;
        p->wn[2 * l + 1] = Sy / A;
        int na = node_id(p, i, 0), nb = node_id(p, i + 1, 0);
        p->wa[2 * l] = nodes[2 * na]; p->wa[2 * l + 1] = nodes[2 * na + 1];
        p->wb[2 * l] = nodes[2 * nb]; p->wb[2 * l + 1] = nodes[2 * nb + 1];
        p->wx[2 * l] = 0.5 * (p->wa[2 * l] + p->wb[2 * l]);
        p->wx[2 * l + 1] = 0.5 * (p->wa[2 * l + 1] + p->wb[2 * l + 1]);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* setup                                                               */
/* ------------------------------------------------------------------ */

static void setup_flow(or_problem *p)
{
    const int nv = p->nv;
    p->theta_inf = 0.5;
    p->theta_w = 0.5 * p->Tw;             /* T_w in units of T_inf */
    p->u_inf = p->Ma * sqrt((5.0 / 3.0) * p->theta_inf);
    /* eq. (kndefine) with theta_inf = 1/2, l_ref = 1 */
    double tau_inf = 5.0 * sqrt(OR_PI) / 8.0 * p->Kn;
    p->inv_tau_inf = isinf(p->Kn) ? 0.0 : 1.0 / tau_inf;
    for (int k = 0; k < nv; k++) {
        double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
        double g1 = maxwell1(1.0, p->u_inf, 0.0, p->theta_inf, v1, v2);
        p->fd[2 * k] = g1;
        p->fd[2 * k + 1] = 0.5 * p->theta_inf * g1;
        p->gM[k] = maxwell1(1.0, 0.0, 0.0, p->theta_w, v1, v2);
        p->mJ[k] = (p->objective == 0) ? v1 : 0.5 * (v1 * v1 + v2 * v2);
    }
    for (int l = 0; l < p->nw; l++) {
        double n1 = p->wn[2 * l], n2 = p->wn[2 * l + 1], d = 0;
        for (int k = 0; k < nv; k++) {
            double vn = p->v[2 * k] * n1 + p->v[2 * k + 1] * n2;
            if (vn <= 0) d -= p->w[k] * vn * p->gM[k];
        }
        p->D[l] = d;
    }
}

or_problem *or_create(int topo, int ni, int nj, int nwake, const double *nodes,
                      int vkind, int n1, int n2, double vmax, double vparam,
                      double Kn, double Ma, double Tw, int objective, int nthreads)
{
    if (ni < 2 || nj < 1 || (topo != 0 && topo != 1)) return NULL;
    if (topo == 0 && nwake != 0) return NULL;
    if (topo == 1 && (nwake < 1 || 2 * nwake >= ni)) return NULL;
    or_problem *p = calloc(1, sizeof(or_problem));
    p->topo = topo; p->ni = ni; p->nj = nj; p->nwake = nwake;
    p->nthreads = nthreads > 0 ? nthreads : 1;
    if (build_mesh(p, nodes) != 0) { free(p); return NULL; }
    p->nodes = malloc(sizeof(double) * 2 * (size_t)(ni + 1) * (nj + 1));
    memcpy(p->nodes, nodes, sizeof(double) * 2 * (size_t)(ni + 1) * (nj + 1));
    p->n1 = n1; p->n2 = n2; p->nv = n1 * n2;
    double *x1 = malloc(sizeof(double) * n1), *w1 = malloc(sizeof(double) * n1);
    double *x2 = malloc(sizeof(double) * n2), *w2 = malloc(sizeof(double) * n2);
    if (or_vgrid_1d(vkind, n1, vmax, vparam, x1, w1) || or_vgrid_1d(vkind, n2, vmax, vparam, x2, w2)) {
        free(x1); free(w1); free(x2); free(w2); free(p); return NULL;
    }
    p->v = malloc(sizeof(double) * 2 * p->nv);
    p->w = malloc(sizeof(double) * p->nv);
    for (int b = 0; b < n2; b++)
        for (int a = 0; a < n1; a++) {
            int k = a + n1 * b;
            p->v[2 * k] = x1[a]; p->v[2 * k + 1] = x2[b];
            p->w[k] = w1[a] * w2[b];
        }
    free(x1); free(w1); free(x2); free(w2);
    p->Kn = Kn; p->Ma = Ma; p->Tw = Tw; p->objective = objective;
    p->fd = malloc(sizeof(double) * 2 * p->nv);
    p->gM = malloc(sizeof(double) * p->nv);
    p->mJ = malloc(sizeof(double) * p->nv);
    p->D = malloc(sizeof(double) * p->nw);
    setup_flow(p);
    size_t n = (size_t)p->nc * p->nv * 2;
    p->f = malloc(sizeof(double) * n);
    p->fn = malloc(sizeof(double) * n);
    p->phi = calloc(n, sizeof(double));
    p->phin = calloc(n, sizeof(double));
    p->W = malloc(sizeof(double) * 4 * p->nc);
    p->F = malloc(sizeof(double) * p->nw);
    p->cellred = malloc(sizeof(double) * 2 * p->nc);
    p->order = 1; p->limiter = 1; p->kcorr = 40;
    p->equilibrium = 0; p->eq_ok = 0;
    p->eqP = malloc(sizeof(double) * 4 * p->nc);
    p->eqM = malloc(sizeof(double) * 16 * p->nc);
    if (!p->f || !p->fn || !p->phi || !p->phin) return NULL;
    return p;
}

void or_destroy(or_problem *p)
{
    if (!p) return;
    free(p->nbr); free(p->S); free(p->vol); free(p->cen); free(p->wall_cell); free(p->wall_face);
    free(p->wA); free(p->wn); free(p->wx); free(p->wa); free(p->wb);
    free(p->v); free(p->w); free(p->fd); free(p->gM); free(p->D); free(p->mJ);
    free(p->f); free(p->fn); free(p->W); free(p->F); free(p->phi); free(p->phin); free(p->cellred);
    free(p->nodes);
    free(p->fm); free(p->corr); free(p->dF); free(p->psi); free(p->acorr); free(p->eqP); free(p->eqM);
    free(p->aDinv); free(p->aO);
    free(p);
}

void or_sizes(const or_problem *p, int64_t *out)
{
    out[0] = p->nc; out[1] = p->nw; out[2] = p->nv; out[3] = p->n1; out[4] = p->n2;
    out[5] = p->ni; out[6] = p->nj; out[7] = p->nwake;
}

void or_export_mesh(const or_problem *p, int32_t *nbr, int32_t *wall_cell, double *S, double *vol,
                    double *wA, double *wn, double *wx, double *cen)
{
    for (int c = 0; c < 4 * p->nc; c++) nbr[c] = p->nbr[c];
    for (int l = 0; l < p->nw; l++) wall_cell[l] = p->wall_cell[l];
    memcpy(S, p->S, sizeof(double) * 8 * p->nc);
    memcpy(vol, p->vol, sizeof(double) * p->nc);
    memcpy(wA, p->wA, sizeof(double) * p->nw);
    memcpy(wn, p->wn, sizeof(double) * 2 * p->nw);
    memcpy(wx, p->wx, sizeof(double) * 2 * p->nw);
    memcpy(cen, p->cen, sizeof(double) * 2 * p->nc);
}

void or_export_vgrid(const or_problem *p, double *v, double *w)
{
    memcpy(v, p->v, sizeof(double) * 2 * p->nv);
    memcpy(w, p->w, sizeof(double) * p->nv);
}

void or_export_flow(const or_problem *p, double *out /* tau_inf_inv, u_inf, theta_w, fd..., gM..., D... */)
{
    out[0] = p->inv_tau_inf; out[1] = p->u_inf; out[2] = p->theta_w;
}

void or_export_wall(const or_problem *p, double *D, double *F)
{
    memcpy(D, p->D, sizeof(double) * p->nw);
    memcpy(F, p->F, sizeof(double) * p->nw);
}

/* ------------------------------------------------------------------ */
/* primal                                                              */
/* ------------------------------------------------------------------ */

/* W and wall flux F_l = sum_{v.n > 0} w (v.n) f1 (eq. formula_bgk_fdw,
 * discrete form of Sec. 3.2) for the current f */
static void update_W_F(or_problem *p, const double *f)
{
    const int nv = p->nv;
    p->eq_ok = 0;
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
    for (int c = 0; c < p->nc; c++)
        or_moments(nv, p->v, p->w, f + (size_t)c * nv * 2, p->W + 4 * c);
    for (int l = 0; l < p->nw; l++) {
        const double *fc = f + (size_t)p->wall_cell[l] * nv * 2;
        double n1 = p->wn[2 * l], n2 = p->wn[2 * l + 1], s = 0;
        for (int k = 0; k < nv; k++) {
            double vn = p->v[2 * k] * n1 + p->v[2 * k + 1] * n2;
            if (vn > 0) s += p->w[k] * vn * fc[2 * k];
        }
        p->F[l] = s;
    }
}

void or_primal_init(or_problem *p)
{
    size_t nv = p->nv;
    for (int c = 0; c < p->nc; c++)
        memcpy(p->f + (size_t)c * nv * 2, p->fd, sizeof(double) * 2 * nv);
    update_W_F(p, p->f);
    p->corr_ok = 0;
    p->acc_sweeps = 0;
}

/* value of f carried into cell c through face q at velocity k (s <= 0);
 * Fw: the wall fluxes F_l of the diffuse wall value */
static void inflow_value(const or_problem *p, const double *f, const double *Fw, int c, int q, int k,
                         double *o1, double *o2)
{
    int nb = p->nbr[4 * c + q];
    if (nb >= 0) {
        const double *fj = f + ((size_t)nb * p->nv + k) * 2;
        *o1 = fj[0]; *o2 = fj[1];
    } else if (nb == -1) {
        *o1 = p->fd[2 * k]; *o2 = p->fd[2 * k + 1];
    } else {
        int l = -2 - nb;
        double gb1 = p->gM[k] / p->D[l];           /* eq. (barg) */
        *o1 = Fw[l] * gb1;
        *o2 = Fw[l] * 0.5 * p->theta_w * gb1;
    }
}

/* ------------------------------------------------------------------ */
/* second-order reconstruction                                         */
/* ------------------------------------------------------------------ */
/* Sec. 3.1 states second-order accuracy in physical space for both the
 * primal and the adjoint balance and leaves the scheme to its references.
 * Readings taken here (order 2):
 *   - a cell value sits at the cell's area centroid x_c; the gradient is
 *     Green-Gauss, grad f_c = (1/V_c) sum_q fbar_q S_cq, with fbar the mean
 *     of the two cell values on an interior face and f_c on a boundary face;
 *   - Venkatakrishnan limiter, per cell, velocity and component (so_limit),
 *     with its smoothing e = 1e-3 |f_c| relative to the cell value, so that
 *     it acts alike on the Maxwellian's core and on its tail values many
 *     decades smaller; smooth, it lets the defect-correction iteration
 *     converge to rounding and keeps the frozen factors of the adjoint
 *     well-conditioned (Barth-Jespersen, the non-smooth alternative, stalls
 *     the iteration and makes psi jump where f is flat);
 *   - the value of a face is reconstructed on its upwind side,
 *     f_u + psi_u grad f_u . (m_q - x_u); inflow from the far field stays
 *     f_d, inflow from the wall stays F_l gbar, with F_l summed over the
 *     reconstructed outgoing wall values; the drag uses the same wall values;
 *   - iteration by defect correction: every K sweeps the difference c
 *     between the second- and first-order face fluxes of each cell, and the
 *     difference dF of the wall fluxes, are evaluated from the current f
 *     and held; each sweep is the first-order Jacobi sweep with -c in its
 *     numerator and F + dF as wall flux.  A fixed point solves the
 *     second-order balance R2(f) = 0.  (Applying the correction in every
 *     sweep, K = 1, is a forward-Euler pseudo-time step of the second-order
 *     operator and diverges where transport dominates.)
 *   - adjoint: the limiter factors psi of the converged f are frozen; the
 *     adjoint is the exact transpose of the frozen-limiter linearisation of
 *     R2 and J, iterated the same way: its reconstruction term E is
 *     re-evaluated every K sweeps. */

/* Green-Gauss gradient g[component][direction] of f at cell c, velocity k */
static void so_grad(const or_problem *p, const double *f, int c, int k, double g[2][2])
{
    const int nv = p->nv;
    const double *fc = f + ((size_t)c * nv + k) * 2;
    g[0][0] = g[0][1] = g[1][0] = g[1][1] = 0;
    for (int q = 0; q < 4; q++) {
        int nb = p->nbr[4 * c + q];
        double b1 = fc[0], b2 = fc[1];
        if (nb >= 0) {
            const double *fj = f + ((size_t)nb * nv + k) * 2;
            b1 = 0.5 * (fc[0] + fj[0]);
            b2 = 0.5 * (fc[1] + fj[1]);
        }
        double Sx = p->S[8 * c + 2 * q], Sy = p->S[8 * c + 2 * q + 1];
        g[0][0] += b1 * Sx; g[0][1] += b1 * Sy;
        g[1][0] += b2 * Sx; g[1][1] += b2 * Sy;
    }
    for (int m = 0; m < 2; m++) { g[m][0] /= p->vol[c]; g[m][1] /= p->vol[c]; }
}

/* Venkatakrishnan limiter factor of each component for the gradient g: per
 * face q, with d the unlimited increment g . (m_q - x_c), D = hi - f_c for
 * d > 0 and lo - f_c otherwise (hi, lo: max and min over the cell and its
 * interior neighbours) and e = kappa |f_c|,
 *   phi_q = (D^2 + e^2 + 2 d D) / (D^2 + 2 d^2 + d D + e^2),
 * psi = min(1, min_q phi_q).  A smooth function of the cell values: flat
 * regions (|d|, |D| << e) give psi -> 1 and a face value overshoots
 * [lo, hi] by at most e / (2 sqrt 2). */
static void so_limit(const or_problem *p, const double *f, int c, int k, const double g[2][2], double psi[2])
{
    const int nv = p->nv;
    psi[0] = psi[1] = 1.0;
    if (!p->limiter) return;
    const double *fc = f + ((size_t)c * nv + k) * 2;
    for (int m = 0; m < 2; m++) {
        double lo = fc[m], hi = fc[m];
        for (int q = 0; q < 4; q++) {
            int nb = p->nbr[4 * c + q];
            if (nb < 0) continue;
            double v = f[((size_t)nb * nv + k) * 2 + m];
            if (v < lo) lo = v;
            if (v > hi) hi = v;
        }
        const double e2 = (OR_VK_KAPPA * fc[m]) * (OR_VK_KAPPA * fc[m]);
        for (int q = 0; q < 4; q++) {
            double rx = p->fm[8 * c + 2 * q] - p->cen[2 * c], ry = p->fm[8 * c + 2 * q + 1] - p->cen[2 * c + 1];
            double d = g[m][0] * rx + g[m][1] * ry;
            double D = d > 0 ? hi - fc[m] : lo - fc[m];
            double den = D * D + 2.0 * d * d + d * D + e2;
            double r = den > 0 ? (D * D + e2 + 2.0 * d * D) / den : 1.0;
            if (r < psi[m]) psi[m] = r;
        }
    }
}

/* limited slopes G = psi grad f, [nc][nv][2 components][2 directions], and
 * optionally the factors psi [nc][nv][2] */
static void so_slopes(const or_problem *p, const double *f, double *G, double *psi)
{
    const int nv = p->nv;
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
    for (int c = 0; c < p->nc; c++)
        for (int k = 0; k < nv; k++) {
            double g[2][2], ps[2];
            so_grad(p, f, c, k, g);
            so_limit(p, f, c, k, g, ps);
            double *o = G + ((size_t)c * nv + k) * 4;
            o[0] = ps[0] * g[0][0]; o[1] = ps[0] * g[0][1];
            o[2] = ps[1] * g[1][0]; o[3] = ps[1] * g[1][1];
            if (psi) { psi[((size_t)c * nv + k) * 2] = ps[0]; psi[((size_t)c * nv + k) * 2 + 1] = ps[1]; }
        }
}

/* reconstruction increment of face q of cell c at velocity k, component m,
 * from the face's upwind side (s = v.S_cq): the cell itself (s > 0), the
 * interior neighbour (s <= 0), none for inflow through a boundary */
static double so_delta(const or_problem *p, const double *G, int c, int q, int k, int m, double s)
{
    int u = c;
    if (!(s > 0)) {
        u = p->nbr[4 * c + q];
        if (u < 0) return 0.0;
    }
    const double *g = G + ((size_t)u * p->nv + k) * 4 + 2 * m;
    double rx = p->fm[8 * c + 2 * q] - p->cen[2 * u], ry = p->fm[8 * c + 2 * q + 1] - p->cen[2 * u + 1];
    return g[0] * rx + g[1] * ry;
}

/* dF_l = sum_{v.n > 0} w (v.n) (reconstructed - cell value of f1) at the wall */
static void so_wall_dF(const or_problem *p, const double *G, double *dF)
{
    for (int l = 0; l < p->nw; l++) {
        int c = p->wall_cell[l];
        double n1 = p->wn[2 * l], n2 = p->wn[2 * l + 1], acc = 0;
        for (int k = 0; k < p->nv; k++) {
            double vn = p->v[2 * k] * n1 + p->v[2 * k + 1] * n2;
            if (vn > 0) acc += p->w[k] * vn * so_delta(p, G, c, p->wall_face[l], k, 0, 1.0);
        }
        dF[l] = acc;
    }
}

/* c = sum_q (v.S_q)(second-order - first-order face value) and dF of f */
static void so_correction(or_problem *p, const double *f)
{
    const int nv = p->nv;
    double *G = malloc(sizeof(double) * 4 * (size_t)p->nc * nv);
    so_slopes(p, f, G, NULL);
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
    for (int c = 0; c < p->nc; c++)
        for (int k = 0; k < nv; k++) {
            double v1 = p->v[2 * k], v2 = p->v[2 * k + 1], c1 = 0, c2 = 0;
            for (int q = 0; q < 4; q++) {
                double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1];
                c1 += s * so_delta(p, G, c, q, k, 0, s);
                c2 += s * so_delta(p, G, c, q, k, 1, s);
            }
            p->corr[((size_t)c * nv + k) * 2] = c1;
            p->corr[((size_t)c * nv + k) * 2 + 1] = c2;
        }
    so_wall_dF(p, G, p->dF);
    free(G);
}

static void so_alloc(or_problem *p)
{
    size_t n = (size_t)p->nc * p->nv * 2;
    if (!p->corr) p->corr = calloc(n, sizeof(double));
    if (!p->dF) p->dF = calloc(p->nw, sizeof(double));
    if (!p->psi) p->psi = calloc(n, sizeof(double));
    if (!p->acorr) p->acorr = calloc(n, sizeof(double));
}

/* order 1 or 2; limiter 0 (none) or 1 (Venkatakrishnan); K >= 1 sweeps
 * between evaluations of the held correction.  Returns 0, or -1 for an
 * invalid setting. */
int or_set_scheme(or_problem *p, int order, int limiter, int kcorr)
{
    if ((order != 1 && order != 2) || (limiter != 0 && limiter != 1) || kcorr < 1) return -1;
    p->order = order; p->limiter = limiter; p->kcorr = kcorr;
    if (order == 2) so_alloc(p);
    p->corr_ok = p->acorr_ok = 0;
    return 0;
}

/* limited slopes and limiter factors of f (pins) */
void or_so_slopes(or_problem *p, const double *f, double *G, double *psi) { so_slopes(p, f, G, psi); }

/* the face values R2 uses: for every cell c, face q and velocity k the
 * value on the face's upwind side, out [nc][4][nv][2] */
void or_so_faces(or_problem *p, const double *f, double *out)
{
    const int nv = p->nv;
    double *G = malloc(sizeof(double) * 4 * (size_t)p->nc * nv), *F2 = malloc(sizeof(double) * p->nw);
    double *Ws = malloc(sizeof(double) * 4 * p->nc), *Fs = malloc(sizeof(double) * p->nw);
    memcpy(Ws, p->W, sizeof(double) * 4 * p->nc); memcpy(Fs, p->F, sizeof(double) * p->nw);
    update_W_F(p, f);
    so_slopes(p, f, G, NULL);
    so_wall_dF(p, G, F2);
    for (int l = 0; l < p->nw; l++) F2[l] += p->F[l];
    for (int c = 0; c < p->nc; c++)
        for (int q = 0; q < 4; q++)
            for (int k = 0; k < nv; k++) {
                double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
                double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1], a1, a2;
                if (s > 0) { a1 = f[((size_t)c * nv + k) * 2]; a2 = f[((size_t)c * nv + k) * 2 + 1]; }
                else inflow_value(p, f, F2, c, q, k, &a1, &a2);
                double *o = out + (((size_t)c * 4 + q) * nv + k) * 2;
                o[0] = a1 + so_delta(p, G, c, q, k, 0, s);
                o[1] = a2 + so_delta(p, G, c, q, k, 1, s);
            }
    memcpy(p->W, Ws, sizeof(double) * 4 * p->nc); memcpy(p->F, Fs, sizeof(double) * p->nw);
    p->eq_ok = 0;
    free(G); free(F2); free(Ws); free(Fs);
}

/* ------------------------------------------------------------------ */
/* macroscopic prediction                                              */
/* ------------------------------------------------------------------ */
/* Sec. 3.1 accelerates the primal (and adjoint) kinetic iterations with
 * "prediction" solutions of approximate macroscopic equations taken from the
 * continuum limit and defers the scheme to its references.  The reading
 * taken here is a synthetic-acceleration step in the spirit of the implicit
 * gas-kinetic schemes' macroscopic prediction (Zhu, Zhong & Xu, J. Comput.
 * Phys. 2016) and of the general synthetic iterative scheme (Su, Zhu & Wu,
 * J. Comput. Phys. 2020): every K sweeps,
 *   1. r_c = sum_k w Psi_k R_c,k, the moments of the kinetic residual R of
 *      eq. (numerpr_gov) at the current f (zero at the discrete solution:
 *      the step cannot move the fixed point);
 *   2. A dW = -r, with A the moments of the upwind transport of Maxwellian
 *      perturbations, A dW = sum_k w Psi_k sum_q (v_k . S_q) dg_face,k: the
 *      outflow faces carry the cell's own dg/dW dW_c, the inflow faces the
 *      neighbour's, nothing from the far field, and the wall face the
 *      diffuse value's response gbar_k dF_l (dF_l = sum_{v.n>0} w (v.n)
 *      dg1/dW dW_c) -- the exact linearisation of the transport of the
 *      discrete scheme restricted to local equilibria (a kinetic
 *      flux-vector-split Euler operator), with the pseudo-time term
 *      V_c/dt_c = (|u_c| + c_c) sum_q |S_q| / CFL on its diagonal (c the
 *      sound speed, CFL = 1000: an implicit step with a very large local
 *      time step, which keeps the near-singular modes of the steady
 *      operator -- a slow wake behind a trailing edge, a sonic region --
 *      from being amplified), solved approximately by red-black block
 *      Gauss-Seidel steps from dW = 0;
 *   3. each cell's correction is limited so that rho and theta change by
 *      at most a fraction alpha (0.2) in one step;
 *   4. the predicted moments W + dW replace W as the state the next sweep
 *      relaxes towards (g and tau of that sweep).  The sweep weights the
 *      prediction per velocity by its collision share V/tau / (V/tau +
 *      sum_out v.S): it takes hold where collisions dominate and fades in
 *      cells thinner than a mean free path, where the kinetic sweep itself
 *      is the right solver and the inviscid macroscopic operator is not.
 * A fixed point of the accelerated iteration has r = 0, i.e. solves the
 * discrete equations, and the plain iteration's solution has r = 0, dW = 0:
 * both iterations share their solutions.  The step needs the conservative
 * equilibrium: the macroscopic equations are conservation laws, and only
 * then does an equilibrium perturbation dg/dW dW carry the moments dW (the
 * collision term's moments then vanish identically). */

#define OR_MACRO_CFL 1000.0

/* the pseudo-time term V_c/dt_c of cell c at the current W */
static double macro_shift(const or_problem *p, int c)
{
    double rho, u1, u2, th, sS = 0;
    prim(p->W + 4 * c, &rho, &u1, &u2, &th);
    for (int q = 0; q < 4; q++) sS += hypot(p->S[8 * c + 2 * q], p->S[8 * c + 2 * q + 1]);
    return (sqrt(u1 * u1 + u2 * u2) + sqrt(5.0 / 3.0 * th)) * sS / OR_MACRO_CFL;
}

/* the macroscopic system of the current f (first order): r [nc][4], Dinv
 * [nc][16] (inverse of the cell's own block, pseudo-time term included), O
 * [nc][4][16] (blocks of the four face neighbours; zero for boundary faces) */
static void macro_assemble(or_problem *p, double *r, double *Dinv, double *O)
{
    const int nv = p->nv;
    eq_cache(p);
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
    for (int c = 0; c < p->nc; c++) {
        double rho, u1, u2, th;
        prim(p->W + 4 * c, &rho, &u1, &u2, &th);
        const double itau = inv_tau_of(p, rho, th), V = p->vol[c];
        double rc[4] = { 0, 0, 0, 0 }, Dc[4][4] = { { 0 } }, Oc[4][4][4] = { { { 0 } } };
        int wl = -1;
        for (int q = 0; q < 4; q++) if (p->nbr[4 * c + q] <= -2) wl = -2 - p->nbr[4 * c + q];
        double dF[4] = { 0, 0, 0, 0 }, wall1[4] = { 0, 0, 0, 0 };
        for (int k = 0; k < nv; k++) {
            const double v1 = p->v[2 * k], v2 = p->v[2 * k + 1], wk = p->w[k];
            const double psi[4] = { 1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2) };
            const double *fc = p->f + ((size_t)c * nv + k) * 2;
            double dgc[2][4], dtt[4], g1, g2;
            dg_dW_cell(p, c, k, dgc, dtt);
            eq_cell_g(p, c, k, &g1, &g2);
            /* collision part of the residual (zero for the conservative equilibrium) */
            const double e1 = V * itau * (fc[0] - g1), e2 = V * itau * (fc[1] - g2);
            for (int a = 0; a < 4; a++) rc[a] += wk * (psi[a] * e1 + (a == 3 ? e2 : 0.0));
            for (int q = 0; q < 4; q++) {
                const double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1];
                double a1, a2;
                if (s > 0) {
                    a1 = fc[0]; a2 = fc[1];
                    for (int a = 0; a < 4; a++)
                        for (int b = 0; b < 4; b++) Dc[a][b] += wk * s * (psi[a] * dgc[0][b] + (a == 3 ? dgc[1][b] : 0.0));
                } else {
                    inflow_value(p, p->f, p->F, c, q, k, &a1, &a2);
                    const int nb = p->nbr[4 * c + q];
                    if (nb >= 0) {
                        double dgn[2][4], dttn[4];
                        dg_dW_cell(p, nb, k, dgn, dttn);
                        for (int a = 0; a < 4; a++)
                            for (int b = 0; b < 4; b++)
                                Oc[q][a][b] += wk * s * (psi[a] * dgn[0][b] + (a == 3 ? dgn[1][b] : 0.0));
                    } else if (nb <= -2) {
                        const double gb1 = p->gM[k] / p->D[wl], gb2 = 0.5 * p->theta_w * gb1;
                        for (int a = 0; a < 4; a++) wall1[a] += wk * s * (psi[a] * gb1 + (a == 3 ? gb2 : 0.0));
                    }
                }
                for (int a = 0; a < 4; a++) rc[a] += wk * s * (psi[a] * a1 + (a == 3 ? a2 : 0.0));
            }
            if (wl >= 0) {
                const double vn = v1 * p->wn[2 * wl] + v2 * p->wn[2 * wl + 1];
                if (vn > 0) for (int b = 0; b < 4; b++) dF[b] += wk * vn * dgc[0][b];
            }
        }
        for (int a = 0; a < 4; a++) for (int b = 0; b < 4; b++) Dc[a][b] += wall1[a] * dF[b];
        const double lam = macro_shift(p, c);
        for (int a = 0; a < 4; a++) Dc[a][a] += lam;
        for (int b = 0; b < 4; b++) {
            double e[4] = { 0, 0, 0, 0 }, col[4];
            e[b] = 1.0;
            solve4(Dc, e, col);
            for (int a = 0; a < 4; a++) Dinv[16 * c + 4 * a + b] = col[a];
        }
        for (int q = 0; q < 4; q++)
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) O[64 * c + 16 * q + 4 * a + b] = Oc[q][a][b];
        for (int a = 0; a < 4; a++) r[4 * c + a] = rc[a];
    }
}

/* red-black block Gauss-Seidel from x = 0: colour (i + j) % 2 in mesh
 * numbering, red (0) first; each half step reads the other array */
static void macro_solve(or_problem *p, const double *r, const double *Dinv, const double *O, double *x)
{
    const int nc = p->nc;
    double *y = calloc(4 * (size_t)nc, sizeof(double));
    memset(x, 0, sizeof(double) * 4 * nc);
    for (int it = 0; it < p->acc_inner; it++) {
        for (int col = 0; col < 2; col++) {
            const double *src = col == 0 ? x : y;
            double *dst = col == 0 ? y : x;
            for (int c = 0; c < nc; c++) {
                const int i = c % p->ni, j = c / p->ni;
                if ((i + j) % 2 != col) { for (int a = 0; a < 4; a++) dst[4 * c + a] = src[4 * c + a]; continue; }
                double b[4];
                for (int a = 0; a < 4; a++) b[a] = -r[4 * c + a];
                for (int q = 0; q < 4; q++) {
                    const int nb = p->nbr[4 * c + q];
                    if (nb < 0) continue;
                    for (int a = 0; a < 4; a++)
                        for (int e = 0; e < 4; e++) b[a] -= O[64 * c + 16 * q + 4 * a + e] * src[4 * nb + e];
                }
                for (int a = 0; a < 4; a++) {
                    double acc = 0;
                    for (int e = 0; e < 4; e++) acc += Dinv[16 * c + 4 * a + e] * b[e];
                    dst[4 * c + a] = acc;
                }
            }
        }
    }
    free(y);
}

/* theta of a moment vector */
static double theta_of(const double *W)
{
    double rho, u1, u2, th;
    prim(W, &rho, &u1, &u2, &th);
    return th;
}

static void macro_predict(or_problem *p)
{
    const int nc = p->nc;
    double *r = malloc(sizeof(double) * 4 * nc), *Dinv = malloc(sizeof(double) * 16 * nc);
    double *O = malloc(sizeof(double) * 64 * (size_t)nc);
    double *x = malloc(sizeof(double) * 4 * nc);
    macro_assemble(p, r, Dinv, O);
    macro_solve(p, r, Dinv, O, x);
    for (int c = 0; c < nc; c++) {
        double *W = p->W + 4 * c, Wt[4];
        for (int a = 0; a < 4; a++) Wt[a] = W[a] + x[4 * c + a];
        const double th0 = theta_of(W), th1 = theta_of(Wt);
        const double ch = fmax(fabs(x[4 * c]) / W[0], fabs(th1 - th0) / th0);
        double fac = 0.0;
        if (Wt[0] > 0 && th1 > 0 && isfinite(ch)) fac = ch > p->acc_alpha ? p->acc_alpha / ch : 1.0;
        for (int a = 0; a < 4; a++) W[a] += fac * x[4 * c + a];
    }
    p->eq_ok = 0;
    free(r); free(Dinv); free(O); free(x);
}

/* ---- adjoint prediction ----
 * The adjoint iteration is accelerated by the transpose of the primal's
 * accelerated sweep (Sec. 3.1 accelerates the adjoint system the same way),
 * so that the two iterations share their convergence factors.  Linearised
 * at the converged f, a primal sweep is f' = f + D^-1 R'(f) with D the
 * diagonal sum_out v.S + V/tau; the sweep after a prediction relaxes towards
 * W + dW, dW = L r with r = -M R the residual's moments (M the moments,
 * L the linear map of the Gauss-Seidel steps) and W + dW entering through
 * g and tau: f' = f + D^-1 Q R' with Q = I - H L M, H = dg/dW V/tau +
 * (g - f) d(V/tau)/dW.  The same step for the adjoint equation R'^T lam +
 * dJ/df = 0, transposed under sum_k w_k, is
 *   lam' = lam + Q^T D^-1 R*(lam) = lam_s - Psi L^T (H^T (lam_s - lam)),
 * lam_s the plain sweep's result: every K-th adjoint sweep corrects its
 * result by the collision invariant Psi z, z = L^T y, y_c = V_c [ What_c /
 * tau_c - (1/tau dtau/dW)_c rho_tau,c ] of the sweep's change lam_s - lam
 * (What and rho_tau the adjoint moments of eq. adjoint_macdefines).  The
 * correction vanishes with the plain sweep's change, so the adjoint
 * solution is unchanged; the accelerated adjoint cycle equals R'^-T times
 * the transposed primal cycle times R'^T, i.e. has the primal cycle's
 * eigenvalues. */

/* L^T: the transpose of the linear map r -> x of macro_solve, its half steps
 * transposed in reverse order */
static void macro_solve_adj(or_problem *p, const double *s, const double *Dinv, const double *O, double *rbar)
{
    const int nc = p->nc;
    double *xb = malloc(sizeof(double) * 4 * nc), *yb = malloc(sizeof(double) * 4 * nc);
    memcpy(xb, s, sizeof(double) * 4 * nc);
    memset(rbar, 0, sizeof(double) * 4 * nc);
    for (int it = p->acc_inner - 1; it >= 0; it--) {
        for (int col = 1; col >= 0; col--) {
            /* half step col wrote dst_fwd from src_fwd: its adjoint reads the
             * output's adjoint (ob) and writes the input's (ib) */
            const double *ob = col == 1 ? xb : yb;
            double *ib = col == 1 ? yb : xb;
            memset(ib, 0, sizeof(double) * 4 * nc);
            for (int c = 0; c < nc; c++) {
                const int i = c % p->ni, j = c / p->ni;
                if ((i + j) % 2 != col) { for (int a = 0; a < 4; a++) ib[4 * c + a] += ob[4 * c + a]; continue; }
                /* x_c = Dinv_c (-r_c - sum_q O_cq src_nb): t = -Dinv_c^T ob_c */
                double t[4];
                for (int a = 0; a < 4; a++) {
                    double acc = 0;
                    for (int e = 0; e < 4; e++) acc += Dinv[16 * c + 4 * e + a] * ob[4 * c + e];
                    t[a] = -acc;
                }
                for (int a = 0; a < 4; a++) rbar[4 * c + a] += t[a];
                for (int q = 0; q < 4; q++) {
                    const int nb = p->nbr[4 * c + q];
                    if (nb < 0) continue;
                    for (int e = 0; e < 4; e++) {
                        double acc = 0;
                        for (int a = 0; a < 4; a++) acc += O[64 * c + 16 * q + 4 * a + e] * t[a];
                        ib[4 * nb + e] += acc;
                    }
                }
            }
        }
    }
    free(xb); free(yb);
}

/* the correction of an accelerated adjoint sweep: phin (the plain sweep's
 * result from phi) -= Psi z */
static void macro_adjoint_correct(or_problem *p, const double *phi, double *phin)
{
    const int nc = p->nc, nv = p->nv;
    double *y = malloc(sizeof(double) * 4 * nc), *z = malloc(sizeof(double) * 4 * nc);
    eq_cache(p);
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
    for (int c = 0; c < nc; c++) {
        double rho, u1, u2, th;
        prim(p->W + 4 * c, &rho, &u1, &u2, &th);
        const double itau = inv_tau_of(p, rho, th), V = p->vol[c];
        double wh[4] = { 0, 0, 0, 0 }, rt = 0, dtt[4] = { 0, 0, 0, 0 };
        for (int k = 0; k < nv; k++) {
            double dg[2][4], g1, g2;
            dg_dW_cell(p, c, k, dg, dtt);
            eq_cell_g(p, c, k, &g1, &g2);
            const size_t o = ((size_t)c * nv + k) * 2;
            const double d0 = phin[o] - phi[o], d1 = phin[o + 1] - phi[o + 1];
            for (int m = 0; m < 4; m++) wh[m] += p->w[k] * (d0 * dg[0][m] + d1 * dg[1][m]);
            rt += p->w[k] * (d0 * (g1 - p->f[o]) + d1 * (g2 - p->f[o + 1])) * itau;
        }
        for (int m = 0; m < 4; m++) y[4 * c + m] = V * (itau * wh[m] - dtt[m] * rt);
    }
    macro_solve_adj(p, y, p->aDinv, p->aO, z);
    for (int c = 0; c < nc; c++)
        for (int k = 0; k < nv; k++) {
            const double v1 = p->v[2 * k], v2 = p->v[2 * k + 1], *zc = z + 4 * c;
            const size_t o = ((size_t)c * nv + k) * 2;
            phin[o] -= zc[0] + zc[1] * v1 + zc[2] * v2 + zc[3] * 0.5 * (v1 * v1 + v2 * v2);
            phin[o + 1] -= zc[3];
        }
    free(y); free(z);
}

int or_set_acceleration(or_problem *p, int every, int inner)
{
    /* the macroscopic equations are conservation laws: the conservative
     * equilibrium, first order */
    if (every < 0 || inner < 0 || (every > 0 && p->equilibrium != 1)) return -1;
    p->acc_every = every;
    p->acc_inner = inner;
    p->acc_alpha = 0.2;
    return 0;
}

/* the Gauss-Seidel map L of the adjoint's frozen system and its transpose
 * (pins; after or_adjoint_init with the prediction on) */
int or_macro_gs(or_problem *p, const double *r, double *x)
{
    if (!p->aDinv) return -1;
    macro_solve(p, r, p->aDinv, p->aO, x);
    return 0;
}

int or_macro_gs_adj(or_problem *p, const double *s, double *rbar)
{
    if (!p->aDinv) return -1;
    macro_solve_adj(p, s, p->aDinv, p->aO, rbar);
    return 0;
}

/* the macroscopic system of the current state (pins): r [nc][4], D^-1
 * [nc][4][4] (pseudo-time term included), O [nc][4][4][4], and the
 * pseudo-time term lam [nc] */
void or_macro_system(or_problem *p, double *r, double *Dinv, double *O, double *lam)
{
    macro_assemble(p, r, Dinv, O);
    for (int c = 0; c < p->nc; c++) lam[c] = macro_shift(p, c);
}

/* One Jacobi sweep of eq. (numerpr_gov), every cell from f^n.  Returns the
 * relative change of W in the 2-norm. */
double or_primal_iterate(or_problem *p, int niter)
{
    const int nv = p->nv;
    double r = 0;
    double *Fw = malloc(sizeof(double) * (p->nw > 0 ? p->nw : 1));
    for (int it = 0; it < niter; it++) {
        const int so = p->order == 2;
        if (so && (!p->corr_ok || p->since == p->kcorr)) {
            so_correction(p, p->f);
            p->corr_ok = 1;
            p->since = 0;
        }
        for (int l = 0; l < p->nw; l++) Fw[l] = p->F[l] + (so ? p->dF[l] : 0.0);
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
        for (int c = 0; c < p->nc; c++) {
            double rho, u1, u2, th, P[4];
            prim(p->W + 4 * c, &rho, &u1, &u2, &th);
            eq_params(p, p->W + 4 * c, P, NULL);
            double itau = inv_tau_of(p, rho, th);
            double V = p->vol[c];
            for (int k = 0; k < nv; k++) {
                double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
                double in1 = 0, in2 = 0, out = 0;
                for (int q = 0; q < 4; q++) {
                    double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1];
                    if (s > 0) out += s;
                    else {
                        double a1, a2;
                        inflow_value(p, p->f, Fw, c, q, k, &a1, &a2);
                        in1 -= s * a1; in2 -= s * a2;
                    }
                }
                if (so) {
                    in1 -= p->corr[((size_t)c * nv + k) * 2];
                    in2 -= p->corr[((size_t)c * nv + k) * 2 + 1];
                }
                double g1 = maxwell1(P[0], P[1], P[2], P[3], v1, v2), g2 = 0.5 * P[3] * g1;
                double den = out + V * itau;
                double *fo = p->fn + ((size_t)c * nv + k) * 2;
                fo[0] = (in1 + V * itau * g1) / den;
                fo[1] = (in2 + V * itau * g2) / den;
            }
        }
        if (so) p->since++;
        /* residual on W */
        double *Wold = malloc(sizeof(double) * 4 * p->nc);
        memcpy(Wold, p->W, sizeof(double) * 4 * p->nc);
        double *t = p->f; p->f = p->fn; p->fn = t;
        update_W_F(p, p->f);
        double num = 0, den = 0;
        for (int c = 0; c < 4 * p->nc; c++) {
            double d = p->W[c] - Wold[c];
            num += d * d;
            den += Wold[c] * Wold[c];
        }
        free(Wold);
        r = sqrt(num / den);
        p->acc_sweeps++;
        if (p->acc_every > 0 && p->order == 1 && p->acc_sweeps % p->acc_every == 0) macro_predict(p);
    }
    free(Fw);
    return r;
}

void or_get_f(const or_problem *p, double *out) { memcpy(out, p->f, sizeof(double) * (size_t)p->nc * p->nv * 2); }
void or_set_f(or_problem *p, const double *in) { memcpy(p->f, in, sizeof(double) * (size_t)p->nc * p->nv * 2); update_W_F(p, p->f); p->corr_ok = 0; p->acc_sweeps = 0; }
void or_get_W(const or_problem *p, double *out) { memcpy(out, p->W, sizeof(double) * 4 * p->nc); }
void or_get_phi(const or_problem *p, double *out) { memcpy(out, p->phi, sizeof(double) * (size_t)p->nc * p->nv * 2); }
void or_set_phi(or_problem *p, const double *in) { memcpy(p->phi, in, sizeof(double) * (size_t)p->nc * p->nv * 2); p->acorr_ok = 0; p->acc_asweeps = 0; }

/* wall value f1_{l,k}: cell value on Xi^+, F_l gbar1 on Xi^- (Sec. 3.2) */
static double wall_f1(const or_problem *p, const double *f, int l, int k)
{
    double vn = p->v[2 * k] * p->wn[2 * l] + p->v[2 * k + 1] * p->wn[2 * l + 1];
    if (vn > 0) return f[((size_t)p->wall_cell[l] * p->nv + k) * 2];
    return p->F[l] * p->gM[k] / p->D[l];
}

/* J = sum_l A_l sum_k w m_J (v.n) f1_{l,k}, eq. (numer_J); per element into Jl.
 * Order 2: the outgoing wall values are reconstructed from the current f and
 * the incoming ones use the matching F_l + dF_l. */
double or_objective(const or_problem *p, double *Jl)
{
    double J = 0;
    double *G = NULL;
    if (p->order == 2) {
        G = malloc(sizeof(double) * 4 * (size_t)p->nc * p->nv);
        so_slopes(p, p->f, G, NULL);
    }
    for (int l = 0; l < p->nw; l++) {
        double s = 0, F2 = p->F[l];
        int c = p->wall_cell[l], q0 = p->wall_face[l];
        if (G) {
            for (int k = 0; k < p->nv; k++) {
                double vn = p->v[2 * k] * p->wn[2 * l] + p->v[2 * k + 1] * p->wn[2 * l + 1];
                if (vn > 0) F2 += p->w[k] * vn * so_delta(p, G, c, q0, k, 0, 1.0);
            }
        }
        for (int k = 0; k < p->nv; k++) {
            double vn = p->v[2 * k] * p->wn[2 * l] + p->v[2 * k + 1] * p->wn[2 * l + 1];
            double f1 = wall_f1(p, p->f, l, k);
            if (G) f1 = vn > 0 ? f1 + so_delta(p, G, c, q0, k, 0, 1.0) : F2 * p->gM[k] / p->D[l];
            s += p->w[k] * p->mJ[k] * vn * f1;
        }
        if (Jl) Jl[l] = p->wA[l] * s;
        J += p->wA[l] * s;
    }
    free(G);
    return J;
}

double or_cd_scale(const or_problem *p)
{
    /* C_d = J / (rho_inf |u_inf|^2 / 2 * L); L = chord (1) or circle diameter (2) */
    double L = (p->topo == 0) ? 2.0 : 1.0;
    return 0.5 * p->u_inf * p->u_inf * L;
}

/* discrete residual R(f) of eq. (numerpr_gov), moved to one side:
 * R = sum_q (v.S_q) f_q + V (f - g(W(f))) / tau(W(f)); W and F of the
 * argument f are used.  out [nc][nv][2]. */
void or_primal_residual(or_problem *p, const double *f, double *out)
{
    const int nv = p->nv;
    if (p->order == 2) {
        /* R2 = sum_q (v.S_q) f_q (second-order face values) + V (f - g) / tau */
        double *fq = malloc(sizeof(double) * 8 * (size_t)p->nc * nv);
        or_so_faces(p, f, fq);
        double *Wsave = malloc(sizeof(double) * 4 * p->nc);
        memcpy(Wsave, p->W, sizeof(double) * 4 * p->nc);
        for (int c = 0; c < p->nc; c++) or_moments(nv, p->v, p->w, f + (size_t)c * nv * 2, p->W + 4 * c);
        p->eq_ok = 0;
        for (int c = 0; c < p->nc; c++) {
            double rho, u1, u2, th;
            prim(p->W + 4 * c, &rho, &u1, &u2, &th);
            double itau = inv_tau_of(p, rho, th), V = p->vol[c];
            for (int k = 0; k < nv; k++) {
                double v1 = p->v[2 * k], v2 = p->v[2 * k + 1], r1 = 0, r2 = 0;
                for (int q = 0; q < 4; q++) {
                    double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1];
                    const double *a = fq + (((size_t)c * 4 + q) * nv + k) * 2;
                    r1 += s * a[0]; r2 += s * a[1];
                }
                const double *fc = f + ((size_t)c * nv + k) * 2;
                double g1, g2;
                eq_cell_g(p, c, k, &g1, &g2);
                out[((size_t)c * nv + k) * 2] = r1 + V * itau * (fc[0] - g1);
                out[((size_t)c * nv + k) * 2 + 1] = r2 + V * itau * (fc[1] - g2);
            }
        }
        memcpy(p->W, Wsave, sizeof(double) * 4 * p->nc);
        p->eq_ok = 0;
        free(Wsave); free(fq);
        return;
    }
    double *Wsave = malloc(sizeof(double) * 4 * p->nc), *Fsave = malloc(sizeof(double) * p->nw);
    memcpy(Wsave, p->W, sizeof(double) * 4 * p->nc);
    memcpy(Fsave, p->F, sizeof(double) * p->nw);
    update_W_F(p, f);
    for (int c = 0; c < p->nc; c++) {
        double rho, u1, u2, th;
        prim(p->W + 4 * c, &rho, &u1, &u2, &th);
        double itau = inv_tau_of(p, rho, th), V = p->vol[c];
        for (int k = 0; k < nv; k++) {
            double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
            const double *fc = f + ((size_t)c * nv + k) * 2;
            double r1 = 0, r2 = 0;
            for (int q = 0; q < 4; q++) {
                double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1];
                if (s > 0) { r1 += s * fc[0]; r2 += s * fc[1]; }
                else { double a1, a2; inflow_value(p, f, p->F, c, q, k, &a1, &a2); r1 += s * a1; r2 += s * a2; }
            }
            double g1, g2;
            eq_cell_g(p, c, k, &g1, &g2);
            out[((size_t)c * nv + k) * 2] = r1 + V * itau * (fc[0] - g1);
            out[((size_t)c * nv + k) * 2 + 1] = r2 + V * itau * (fc[1] - g2);
        }
    }
    memcpy(p->W, Wsave, sizeof(double) * 4 * p->nc);
    memcpy(p->F, Fsave, sizeof(double) * p->nw);
    p->eq_ok = 0;
    free(Wsave); free(Fsave);
}

/* ------------------------------------------------------------------ */
/* complex-step twin of the residual and of J (pins only)              */
/* ------------------------------------------------------------------ */

/* Evaluates R and J with f -> f + i h u and one parameter shifted by i h
 * (which: 0 none, 1 Kn, 2 Ma, 3 Tw); returns Im(.)/h in dR (may be NULL)
 * and *dJ.  Written independently of the real-valued solver above. */
void or_complex_step(or_problem *p, const double *u, double h, int which, double *dR, double *dJ)
{
    const int nv = p->nv, nc = p->nc, nw = p->nw;
    double complex Kn = p->Kn + (which == 1 ? I * h : 0);
    double complex Ma = p->Ma + (which == 2 ? I * h : 0);
    double complex Tw = p->Tw + (which == 3 ? I * h : 0);
    double complex thw = 0.5 * Tw, thinf = 0.5;
    double complex uinf = Ma * csqrt((5.0 / 3.0) * thinf);
    double complex itinf = isinf(p->Kn) ? 0 : 1.0 / (5.0 * sqrt(OR_PI) / 8.0 * Kn);
    double complex *fz = malloc(sizeof(double complex) * (size_t)nc * nv * 2);
    for (size_t q = 0; q < (size_t)nc * nv * 2; q++) fz[q] = p->f[q] + (u ? I * h * u[q] : 0);
    double complex *fdz = malloc(sizeof(double complex) * nv * 2), *gMz = malloc(sizeof(double complex) * nv);
    for (int k = 0; k < nv; k++) {
        double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
        double complex c1 = v1 - uinf;
        double complex g = 1.0 / (2 * OR_PI * thinf) * cexp(-(c1 * c1 + v2 * v2) / (2 * thinf));
        fdz[2 * k] = g; fdz[2 * k + 1] = 0.5 * thinf * g;
        gMz[k] = 1.0 / (2 * OR_PI * thw) * cexp(-(v1 * v1 + v2 * v2) / (2 * thw));
    }
    /* order 2: slopes of the perturbed f with the limiter factors of the
     * real f held (the frozen-limiter linearisation) */
    double complex *Gz = NULL;
    if (p->order == 2) {
        double *Gr = malloc(sizeof(double) * 4 * (size_t)nc * nv), *ps = malloc(sizeof(double) * 2 * (size_t)nc * nv);
        so_slopes(p, p->f, Gr, ps);
        free(Gr);
        Gz = malloc(sizeof(double complex) * 4 * (size_t)nc * nv);
        for (int c = 0; c < nc; c++)
            for (int k = 0; k < nv; k++) {
                const double complex *fc = fz + ((size_t)c * nv + k) * 2;
                double complex g[2][2] = { { 0, 0 }, { 0, 0 } };
                for (int q = 0; q < 4; q++) {
                    int nb = p->nbr[4 * c + q];
                    double complex b1 = fc[0], b2 = fc[1];
                    if (nb >= 0) {
                        const double complex *fj = fz + ((size_t)nb * nv + k) * 2;
                        b1 = 0.5 * (fc[0] + fj[0]); b2 = 0.5 * (fc[1] + fj[1]);
                    }
                    g[0][0] += b1 * p->S[8 * c + 2 * q]; g[0][1] += b1 * p->S[8 * c + 2 * q + 1];
                    g[1][0] += b2 * p->S[8 * c + 2 * q]; g[1][1] += b2 * p->S[8 * c + 2 * q + 1];
                }
                double complex *o = Gz + ((size_t)c * nv + k) * 4;
                const double *pk = ps + ((size_t)c * nv + k) * 2;
                o[0] = pk[0] * g[0][0] / p->vol[c]; o[1] = pk[0] * g[0][1] / p->vol[c];
                o[2] = pk[1] * g[1][0] / p->vol[c]; o[3] = pk[1] * g[1][1] / p->vol[c];
            }
        free(ps);
    }
    /* reconstruction increment of face q of cell c, component m, upwind side */
#define ZDELTA(c_, q_, k_, m_, up_)                                                                   \
    (Gz == NULL || (up_) < 0 ? (double complex)0                                                     \
     : Gz[((size_t)(up_) * nv + (k_)) * 4 + 2 * (m_)] * (p->fm[8 * (c_) + 2 * (q_)] - p->cen[2 * (up_)]) + \
       Gz[((size_t)(up_) * nv + (k_)) * 4 + 2 * (m_) + 1] * (p->fm[8 * (c_) + 2 * (q_) + 1] - p->cen[2 * (up_) + 1]))
    double complex *Dz = malloc(sizeof(double complex) * nw), *Fz = malloc(sizeof(double complex) * nw);
    for (int l = 0; l < nw; l++) {
        const int cw = p->wall_cell[l], qw = p->wall_face[l];
        const double complex *fc = fz + (size_t)cw * nv * 2;
        double complex d = 0, F = 0;
        for (int k = 0; k < nv; k++) {
            double vn = p->v[2 * k] * p->wn[2 * l] + p->v[2 * k + 1] * p->wn[2 * l + 1];
            if (vn > 0) F += p->w[k] * vn * (fc[2 * k] + ZDELTA(cw, qw, k, 0, cw));
            else d -= p->w[k] * vn * gMz[k];
        }
        Dz[l] = d; Fz[l] = F;
    }
    /* J */
    double complex J = 0;
    for (int l = 0; l < nw; l++) {
        const int cw = p->wall_cell[l], qw = p->wall_face[l];
        const double complex *fc = fz + (size_t)cw * nv * 2;
        for (int k = 0; k < nv; k++) {
            double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
            double vn = v1 * p->wn[2 * l] + v2 * p->wn[2 * l + 1];
            double complex f1 = vn > 0 ? fc[2 * k] + ZDELTA(cw, qw, k, 0, cw) : Fz[l] * gMz[k] / Dz[l];
            double mj = p->objective == 0 ? v1 : 0.5 * (v1 * v1 + v2 * v2);
            J += p->wA[l] * p->w[k] * mj * vn * f1;
        }
    }
    *dJ = cimag(J) / h;
    if (dR) {
        for (int c = 0; c < nc; c++) {
            const double complex *fc = fz + (size_t)c * nv * 2;
            double complex W0 = 0, W1 = 0, W2 = 0, W3 = 0;
            for (int k = 0; k < nv; k++) {
                double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
                W0 += p->w[k] * fc[2 * k];
                W1 += p->w[k] * v1 * fc[2 * k];
                W2 += p->w[k] * v2 * fc[2 * k];
                W3 += p->w[k] * (0.5 * (v1 * v1 + v2 * v2) * fc[2 * k] + fc[2 * k + 1]);
            }
            double complex rho = W0, u1 = W1 / W0, u2 = W2 / W0;
            double complex th = (2.0 / 3.0) * (W3 / W0 - 0.5 * (u1 * u1 + u2 * u2));
            double complex itau = itinf * rho * csqrt(2.0 * th);
            double complex Wz[4] = { W0, W1, W2, W3 }, Pz[4];
            eq_params_z(p, Wz, Pz);
            double V = p->vol[c];
            for (int k = 0; k < nv; k++) {
                double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
                double complex r1 = 0, r2 = 0;
                for (int q = 0; q < 4; q++) {
                    double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1];
                    double complex a1, a2;
                    if (s > 0) {
                        a1 = fc[2 * k] + ZDELTA(c, q, k, 0, c);
                        a2 = fc[2 * k + 1] + ZDELTA(c, q, k, 1, c);
                    } else {
                        int nb = p->nbr[4 * c + q];
                        if (nb >= 0) {
                            a1 = fz[((size_t)nb * nv + k) * 2] + ZDELTA(c, q, k, 0, nb);
                            a2 = fz[((size_t)nb * nv + k) * 2 + 1] + ZDELTA(c, q, k, 1, nb);
                        }
                        else if (nb == -1) { a1 = fdz[2 * k]; a2 = fdz[2 * k + 1]; }
                        else { int l = -2 - nb; a1 = Fz[l] * gMz[k] / Dz[l]; a2 = 0.5 * thw * a1; }
                    }
                    r1 += s * a1; r2 += s * a2;
                }
                double complex c1 = v1 - Pz[1], c2 = v2 - Pz[2];
                double complex g1 = Pz[0] / (2 * OR_PI * Pz[3]) * cexp(-(c1 * c1 + c2 * c2) / (2 * Pz[3]));
                r1 += V * itau * (fc[2 * k] - g1);
                r2 += V * itau * (fc[2 * k + 1] - 0.5 * Pz[3] * g1);
                dR[((size_t)c * nv + k) * 2] = cimag(r1) / h;
                dR[((size_t)c * nv + k) * 2 + 1] = cimag(r2) / h;
            }
        }
    }
#undef ZDELTA
    free(fz); free(fdz); free(gMz); free(Dz); free(Fz); free(Gz);
}

/* ------------------------------------------------------------------ */
/* adjoint                                                             */
/* ------------------------------------------------------------------ */

/* per-cell adjoint moments of eq. (adjoint_macdefines):
 * What = sum_k w phi . dg/dW (4), rho_tau = sum_k w phi . (g - f) / tau;
 * and per wall element the multiplier of eq. (formula_adjointbgk),
 * Phi_l = int_{Xi^-} varphi_w . dg_w/dF = -sum_{v.n<=0} w (v.n)[(phi1 + m_J) gbar1 + phi2 gbar2]. */
static void adjoint_moments(or_problem *p, const double *phi, double *What, double *rtau, double *Phi)
{
    const int nv = p->nv;
    eq_cache(p);
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
    for (int c = 0; c < p->nc; c++) {
        double rho, u1, u2, th;
        const double *W = p->W + 4 * c;
        prim(W, &rho, &u1, &u2, &th);
        double itau = inv_tau_of(p, rho, th);
        double acc[4] = { 0, 0, 0, 0 }, rt = 0;
        for (int k = 0; k < nv; k++) {
            double dg[2][4], dtt[4];
            dg_dW_cell(p, c, k, dg, dtt);
            const double *ph = phi + ((size_t)c * nv + k) * 2;
            const double *fc = p->f + ((size_t)c * nv + k) * 2;
            for (int m = 0; m < 4; m++) acc[m] += p->w[k] * (ph[0] * dg[0][m] + ph[1] * dg[1][m]);
            double g1, g2;
            eq_cell_g(p, c, k, &g1, &g2);
            rt += p->w[k] * (ph[0] * (g1 - fc[0]) + ph[1] * (g2 - fc[1])) * itau;
        }
        for (int m = 0; m < 4; m++) What[4 * c + m] = acc[m];
        rtau[c] = rt;
    }
    for (int l = 0; l < p->nw; l++) {
        const double *ph = phi + (size_t)p->wall_cell[l] * nv * 2;
        double s = 0;
        for (int k = 0; k < nv; k++) {
            double vn = p->v[2 * k] * p->wn[2 * l] + p->v[2 * k + 1] * p->wn[2 * l + 1];
            if (vn <= 0) {
                double gb1 = p->gM[k] / p->D[l], gb2 = 0.5 * p->theta_w * gb1;
                s -= p->w[k] * vn * ((ph[2 * k] + p->mJ[k]) * gb1 + ph[2 * k + 1] * gb2);
            }
        }
        Phi[l] = s;
    }
}

/* source terms phi_eq / tau + phi_tau of eq. (numerad_gov) at cell c,
 * velocity k (eq. adjoint_eqdefines) */
static void adjoint_source(const or_problem *p, int c, int k, const double *What, const double *rtau,
                           double *s1, double *s2, double *itau_out)
{
    double rho, u1, u2, th;
    const double *W = p->W + 4 * c;
    prim(W, &rho, &u1, &u2, &th);
    double itau = inv_tau_of(p, rho, th);
    double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
    double dg[2][4], dtt[4];
    dg_dW_cell((or_problem *)p, c, k, dg, dtt);
    const double *Wh = What + 4 * c;
    double psi1[4] = { 1.0, v1, v2, 0.5 * (v1 * v1 + v2 * v2) };  /* first column of Psi */
    double eq1 = 0, tt1 = 0;
    for (int m = 0; m < 4; m++) { eq1 += Wh[m] * psi1[m]; tt1 += dtt[m] * psi1[m]; }
    double eq2 = Wh[3], tt2 = dtt[3];               /* second column (0,0,0,1) */
    /* phi_tau = -rho_tau (1/tau) dtau/dW . Psi, with dtt = (1/tau) dtau/dW */
    *s1 = eq1 * itau - rtau[c] * tt1;
    *s2 = eq2 * itau - rtau[c] * tt2;
    *itau_out = itau;
}

/* adjoint value carried into cell c from the downstream side of face q
 * (s > 0): neighbour, far field 0, wall (Phi_l - m_J, 0) */
static void outflow_adjoint(const or_problem *p, const double *phi, const double *Phi, int c, int q, int k,
                            int with_source, double *o1, double *o2)
{
    int nb = p->nbr[4 * c + q];
    if (nb >= 0) { const double *pj = phi + ((size_t)nb * p->nv + k) * 2; *o1 = pj[0]; *o2 = pj[1]; }
    else if (nb == -1) { *o1 = 0; *o2 = 0; }
    else { int l = -2 - nb; *o1 = Phi[l] - (with_source ? p->mJ[k] : 0.0); *o2 = 0; }
}

/* Reconstruction term of the order-2 adjoint: E = (d r2 / d f)^T a, where
 * r2 collects psi_u grad f_u . (m_q - x_u) over the faces q an upwind cell u
 * feeds (psi frozen) and a_q = s (phi_u - phi_down) is the weight of face
 * q's value in the Lagrangian J + sum_k w phi . R (phi_down of the
 * first-order adjoint: neighbour, 0 at the far field, (Phi_l - m_J, 0) at the
 * wall).  Written as the transpose of the Green-Gauss sum: B_u = psi_u sum_q
 * a_q (m_q - x_u) is scattered back to f_u and to its interior neighbours
 * with the weights fbar_q = (f_u + f_nb)/2 or f_u gives them.  Phi holds the
 * wall multipliers of phi; the objective's m_J enters through p->mJ. */
static void so_adjoint_term(const or_problem *p, const double *phi, const double *Phi, double *E)
{
    const int nv = p->nv;
    memset(E, 0, sizeof(double) * 2 * (size_t)p->nc * nv);
    for (int u = 0; u < p->nc; u++) {
        const double V = p->vol[u];
        for (int k = 0; k < nv; k++) {
            double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
            const double *pu = phi + ((size_t)u * nv + k) * 2;
            double B[2][2] = { { 0, 0 }, { 0, 0 } };
            for (int q = 0; q < 4; q++) {
                double s = v1 * p->S[8 * u + 2 * q] + v2 * p->S[8 * u + 2 * q + 1];
                if (!(s > 0)) continue;
                double d1, d2;
                outflow_adjoint(p, phi, Phi, u, q, k, 1, &d1, &d2);
                double rx = p->fm[8 * u + 2 * q] - p->cen[2 * u], ry = p->fm[8 * u + 2 * q + 1] - p->cen[2 * u + 1];
                double a1 = s * (pu[0] - d1), a2 = s * (pu[1] - d2);
                B[0][0] += a1 * rx; B[0][1] += a1 * ry;
                B[1][0] += a2 * rx; B[1][1] += a2 * ry;
            }
            const double *ps = p->psi + ((size_t)u * nv + k) * 2;
            for (int m = 0; m < 2; m++) { B[m][0] *= ps[m]; B[m][1] *= ps[m]; }
            for (int q = 0; q < 4; q++) {
                int nb = p->nbr[4 * u + q];
                double Sx = p->S[8 * u + 2 * q], Sy = p->S[8 * u + 2 * q + 1];
                for (int m = 0; m < 2; m++) {
                    double t = (B[m][0] * Sx + B[m][1] * Sy) / V;
                    if (nb >= 0) {
                        E[((size_t)u * nv + k) * 2 + m] += 0.5 * t;
                        E[((size_t)nb * nv + k) * 2 + m] += 0.5 * t;
                    } else {
                        E[((size_t)u * nv + k) * 2 + m] += t;
                    }
                }
            }
        }
    }
}

void or_adjoint_init(or_problem *p)
{
    /* a primal prediction may have left the predicted moments in W for the
     * next sweep: the adjoint is taken at the moments of f */
    if (p->acc_every > 0) update_W_F(p, p->f);
    memset(p->phi, 0, sizeof(double) * (size_t)p->nc * p->nv * 2);
    p->acc_asweeps = 0;
    if (p->acc_every > 0 && p->order == 1) {
        /* the primal macroscopic system at the frozen f */
        const size_t nc = p->nc;
        double *r = malloc(sizeof(double) * 4 * nc);
        free(p->aDinv); free(p->aO);
        p->aDinv = malloc(sizeof(double) * 16 * nc);
        p->aO = malloc(sizeof(double) * 64 * nc);
        macro_assemble(p, r, p->aDinv, p->aO);
        free(r);
    }
    if (p->order == 2) {
        /* limiter factors of the converged f, frozen for the adjoint */
        double *G = malloc(sizeof(double) * 4 * (size_t)p->nc * p->nv);
        so_slopes(p, p->f, G, p->psi);
        free(G);
        p->acorr_ok = 0;
    }
}

/* Jacobi sweeps of eq. (numerad_gov) with the converged f frozen.  Returns
 * the relative weighted change of phi in the last sweep. */
double or_adjoint_iterate(or_problem *p, int niter)
{
    const int nv = p->nv;
    double *What = malloc(sizeof(double) * 4 * p->nc), *rtau = malloc(sizeof(double) * p->nc);
    double *Phi = malloc(sizeof(double) * p->nw);
    double r = 0;
    for (int it = 0; it < niter; it++) {
        adjoint_moments(p, p->phi, What, rtau, Phi);
        const int so = p->order == 2;
        if (so && (!p->acorr_ok || p->asince == p->kcorr)) {
            so_adjoint_term(p, p->phi, Phi, p->acorr);
            p->acorr_ok = 1;
            p->asince = 0;
        }
#pragma omp parallel for schedule(static) num_threads(p->nthreads)
        for (int c = 0; c < p->nc; c++) {
            double V = p->vol[c];
            double dn = 0, dd = 0;
            for (int k = 0; k < nv; k++) {
                double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
                double a1 = 0, a2 = 0, out = 0;
                for (int q = 0; q < 4; q++) {
                    double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1];
                    if (s > 0) {
                        double b1, b2;
                        outflow_adjoint(p, p->phi, Phi, c, q, k, 1, &b1, &b2);
                        a1 += s * b1; a2 += s * b2; out += s;
                    }
                }
                if (so) {
                    a1 -= p->acorr[((size_t)c * nv + k) * 2];
                    a2 -= p->acorr[((size_t)c * nv + k) * 2 + 1];
                }
                double s1, s2, itau;
                adjoint_source(p, c, k, What, rtau, &s1, &s2, &itau);
                double den = out + V * itau;
                double *po = p->phin + ((size_t)c * nv + k) * 2;
                const double *pi = p->phi + ((size_t)c * nv + k) * 2;
                po[0] = (a1 + V * s1) / den;
                po[1] = (a2 + V * s2) / den;
                double d0 = po[0] - pi[0], d1 = po[1] - pi[1];
                dn += p->w[k] * (d0 * d0 + d1 * d1);
                dd += p->w[k] * (po[0] * po[0] + po[1] * po[1]);
            }
            p->cellred[2 * c] = dn;
            p->cellred[2 * c + 1] = dd;
        }
        double num = 0, den = 0;
        for (int c = 0; c < p->nc; c++) { num += p->cellred[2 * c]; den += p->cellred[2 * c + 1]; }
        r = den > 0 ? sqrt(num / den) : 0.0;
        /* every K-th sweep: the transposed prediction's correction (the
         * residual above is the plain sweep's change) */
        if (p->acc_every > 0 && p->aDinv && !so && (p->acc_asweeps + 1) % p->acc_every == 0)
            macro_adjoint_correct(p, p->phi, p->phin);
        double *t = p->phi; p->phi = p->phin; p->phin = t;
        if (so) p->asince++;
        p->acc_asweeps++;
    }
    free(What); free(rtau); free(Phi);
    return r;
}

/* The adjoint operator A*(phi) = sum_{s>0} s (phi - phi_down) + V (phi - phi_eq)/tau - V phi_tau
 * (with_source = 1 includes the objective's m_J terms at the wall; 0 gives
 * the homogeneous operator, the transpose of dR/df under sum_k w_k). */
void or_adjoint_operator(or_problem *p, const double *phi, int with_source, double *out)
{
    const int nv = p->nv;
    double *What = malloc(sizeof(double) * 4 * p->nc), *rtau = malloc(sizeof(double) * p->nc);
    double *Phi = malloc(sizeof(double) * p->nw);
    double *mJsave = NULL;
    if (!with_source) { mJsave = p->mJ; p->mJ = calloc(nv, sizeof(double)); }
    adjoint_moments(p, phi, What, rtau, Phi);
    double *E = NULL;
    if (p->order == 2) {
        E = malloc(sizeof(double) * 2 * (size_t)p->nc * nv);
        so_adjoint_term(p, phi, Phi, E);
    }
    for (int c = 0; c < p->nc; c++) {
        double V = p->vol[c];
        for (int k = 0; k < nv; k++) {
            double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
            const double *pi = phi + ((size_t)c * nv + k) * 2;
            double r1 = 0, r2 = 0;
            for (int q = 0; q < 4; q++) {
                double s = v1 * p->S[8 * c + 2 * q] + v2 * p->S[8 * c + 2 * q + 1];
                if (s > 0) {
                    double b1, b2;
                    outflow_adjoint(p, phi, Phi, c, q, k, 1, &b1, &b2);
                    r1 += s * (pi[0] - b1); r2 += s * (pi[1] - b2);
                }
            }
            double s1, s2, itau;
            adjoint_source(p, c, k, What, rtau, &s1, &s2, &itau);
            if (E) { r1 += E[((size_t)c * nv + k) * 2]; r2 += E[((size_t)c * nv + k) * 2 + 1]; }
            out[((size_t)c * nv + k) * 2] = r1 + V * (pi[0] * itau - s1);
            out[((size_t)c * nv + k) * 2 + 1] = r2 + V * (pi[1] * itau - s2);
        }
    }
    free(E);
    if (!with_source) { free(p->mJ); p->mJ = mJsave; }
    free(What); free(rtau); free(Phi);
}

/* dJ/dp = dJ/dp|_f + sum_{i,k,c} w_k phi . dR/dp (Lagrangian of Sec. 2.5 in
 * discrete form) for p = Kn (1), Ma (2), T_w (3); the partials come from
 * the complex-step twin. */
double or_adjoint_dJdp(or_problem *p, int which)
{
    const int nv = p->nv;
    size_t n = (size_t)p->nc * nv * 2;
    double *dR = malloc(sizeof(double) * n), dJ;
    or_complex_step(p, NULL, 1e-30, which, dR, &dJ);
    double s = dJ;
    for (int c = 0; c < p->nc; c++)
        for (int k = 0; k < nv; k++) {
            size_t q = ((size_t)c * nv + k) * 2;
            s += p->w[k] * (p->phi[q] * dR[q] + p->phi[q + 1] * dR[q + 1]);
        }
    free(dR);
    return s;
}

/* ------------------------------------------------------------------ */
/* exact discrete shape derivative: complex step in the node coordinates */
/* ------------------------------------------------------------------ */

/* Face vectors (dy, -dx) of the edges corner q -> q+1 and the shoelace area
 * of cell c, with coordinate d of node m shifted by i h. */
static void cell_geometry_z(const or_problem *p, int c, int m, int d, double h, double complex S[4][2],
                            double complex *V)
{
    int i = c % p->ni, j = c / p->ni;
    int cid[4] = { node_id(p, i, j), node_id(p, i + 1, j), node_id(p, i + 1, j + 1), node_id(p, i, j + 1) };
    double complex X[4], Y[4];
    for (int q = 0; q < 4; q++) {
        X[q] = p->nodes[2 * cid[q]] + ((cid[q] == m && d == 0) ? I * h : 0);
        Y[q] = p->nodes[2 * cid[q] + 1] + ((cid[q] == m && d == 1) ? I * h : 0);
    }
    double complex A2 = 0;
    for (int q = 0; q < 4; q++) {
        int r = (q + 1) % 4;
        A2 += (X[q] - X[0]) * (Y[r] - Y[0]) - (X[r] - X[0]) * (Y[q] - Y[0]);
        S[q][0] = Y[r] - Y[q];
        S[q][1] = -(X[r] - X[q]);
    }
    *V = 0.5 * A2;
}

/* Second-order scheme: complex geometry of cell c with node coordinate
 * (m, d) shifted by i h -- face vectors, volume, area centroid and face
 * midpoints, by the formulas the mesh set-up uses. */
static void cell_geometry2_z(const or_problem *p, int c, int m, int d, double h, double complex S[4][2],
                             double complex *V, double complex cen[2], double complex fm[4][2])
{
    int i = c % p->ni, j = c / p->ni;
    int cid[4] = { node_id(p, i, j), node_id(p, i + 1, j), node_id(p, i + 1, j + 1), node_id(p, i, j + 1) };
    double complex X[4], Y[4];
    for (int q = 0; q < 4; q++) {
        X[q] = p->nodes[2 * cid[q]] + ((cid[q] == m && d == 0) ? I * h : 0);
        Y[q] = p->nodes[2 * cid[q] + 1] + ((cid[q] == m && d == 1) ? I * h : 0);
    }
    double complex Xr[4], Yr[4], A2 = 0, cx = 0, cy = 0;
    for (int q = 0; q < 4; q++) { Xr[q] = X[q] - X[0]; Yr[q] = Y[q] - Y[0]; }
    for (int q = 0; q < 4; q++) {
        int r = (q + 1) % 4;
        double complex cr = Xr[q] * Yr[r] - Xr[r] * Yr[q];
        A2 += cr;
        cx += (Xr[q] + Xr[r]) * cr;
        cy += (Yr[q] + Yr[r]) * cr;
        S[q][0] = Y[r] - Y[q];
        S[q][1] = -(X[r] - X[q]);
        fm[q][0] = 0.5 * (X[q] + X[r]);
        fm[q][1] = 0.5 * (Y[q] + Y[r]);
    }
    *V = 0.5 * A2;
    cen[0] = X[0] + cx / (3.0 * A2);
    cen[1] = Y[0] + cy / (3.0 * A2);
}

/* geometry of one cell for the second-order Lagrangian: complex when the
 * shifted node is one of its corners, else the mesh's own values */
typedef struct { int c; double complex S[4][2], V, cen[2], fm[4][2]; } so_geo;

static void so_geo_real(const or_problem *p, int c, so_geo *g)
{
    g->c = c;
    for (int q = 0; q < 4; q++) {
        g->S[q][0] = p->S[8 * c + 2 * q]; g->S[q][1] = p->S[8 * c + 2 * q + 1];
        g->fm[q][0] = p->fm[8 * c + 2 * q]; g->fm[q][1] = p->fm[8 * c + 2 * q + 1];
    }
    g->V = p->vol[c];
    g->cen[0] = p->cen[2 * c]; g->cen[1] = p->cen[2 * c + 1];
}

/* limited slopes of cell u at velocity k with the frozen factors psi:
 * psi_m (1/V) sum_q fbar_q S_q, over the geometry g (complex or real) */
static void so_grad_z(const or_problem *p, const double *psi, const so_geo *g, int k, double complex G[2][2])
{
    const int u = g->c, nv = p->nv;
    const double *fc = p->f + ((size_t)u * nv + k) * 2;
    G[0][0] = G[0][1] = G[1][0] = G[1][1] = 0;
    for (int q = 0; q < 4; q++) {
        int nb = p->nbr[4 * u + q];
        double b1 = fc[0], b2 = fc[1];
        if (nb >= 0) {
            const double *fj = p->f + ((size_t)nb * nv + k) * 2;
            b1 = 0.5 * (fc[0] + fj[0]);
            b2 = 0.5 * (fc[1] + fj[1]);
        }
        G[0][0] += b1 * g->S[q][0]; G[0][1] += b1 * g->S[q][1];
        G[1][0] += b2 * g->S[q][0]; G[1][1] += b2 * g->S[q][1];
    }
    const double *ps = psi + ((size_t)u * nv + k) * 2;
    for (int m = 0; m < 2; m++) { G[m][0] *= ps[m] / g->V; G[m][1] *= ps[m] / g->V; }
}

/* The second-order Lagrangian differentiated in every node coordinate, with
 * f, phi and the limiter factors psi of f held fixed.  A node moves the
 * geometry (face vectors, volume, centroid, face midpoints) of the cells it
 * is a corner of; through their slopes and centroids it also moves the
 * reconstructed values their neighbours receive, so the residuals of those
 * cells and of their neighbours change, and the wall terms (F_l + dF_l, D_l,
 * J_l) of a wall cell among the first. */
static void mesh_sensitivity_so(or_problem *p, double h, double *out)
{
    const int ni = p->ni, nj = p->nj, nv = p->nv, nc = p->nc, nn = (ni + 1) * (nj + 1);
    double *G = malloc(sizeof(double) * 4 * (size_t)nc * nv);
    double *psi = malloc(sizeof(double) * 2 * (size_t)nc * nv);
    double *dF = malloc(sizeof(double) * (p->nw > 0 ? p->nw : 1));
    so_slopes(p, p->f, G, psi);
    so_wall_dF(p, G, dF);
    eq_cache(p);
#pragma omp parallel for schedule(dynamic, 4) num_threads(p->nthreads)
    for (int m = 0; m < nn; m++) {
        const int im = m % (ni + 1), jm = m / (ni + 1);
        int adj[4], na = 0, aff[20], nf = 0;
        for (int jc = jm - 1; jc <= jm; jc++)
            for (int ic = im - 1; ic <= im; ic++)
                if (ic >= 0 && ic < ni && jc >= 0 && jc < nj) adj[na++] = ic + ni * jc;
        for (int a = 0; a < na; a++) {
            int cands[5] = { adj[a], p->nbr[4 * adj[a]], p->nbr[4 * adj[a] + 1], p->nbr[4 * adj[a] + 2],
                             p->nbr[4 * adj[a] + 3] };
            for (int t = 0; t < 5; t++) {
                int c = cands[t], seen = 0;
                if (c < 0) continue;
                for (int e = 0; e < nf; e++) seen |= aff[e] == c;
                if (!seen) aff[nf++] = c;
            }
        }
        for (int d = 0; d < 2; d++) {
            so_geo ga[4];
            for (int a = 0; a < na; a++) {
                ga[a].c = adj[a];
                cell_geometry2_z(p, adj[a], m, d, h, ga[a].S, &ga[a].V, ga[a].cen, ga[a].fm);
            }
            double complex L = 0;
            for (int e = 0; e < nf; e++) {
                const int c = aff[e];
                so_geo gr, *gc = NULL;
                for (int a = 0; a < na; a++) if (adj[a] == c) gc = &ga[a];
                if (!gc) { so_geo_real(p, c, &gr); gc = &gr; }
                /* geometry of each upwind neighbour */
                so_geo gn_real[4];
                const so_geo *gn[4] = { NULL, NULL, NULL, NULL };
                for (int q = 0; q < 4; q++) {
                    int nb = p->nbr[4 * c + q];
                    if (nb < 0) continue;
                    for (int a = 0; a < na; a++) if (adj[a] == nb) gn[q] = &ga[a];
                    if (!gn[q]) { so_geo_real(p, nb, &gn_real[q]); gn[q] = &gn_real[q]; }
                }
                const double *fc = p->f + (size_t)c * nv * 2;
                const double *pc = p->phi + (size_t)c * nv * 2;
                const int nb0 = p->nbr[4 * c];
                const int l = nb0 <= -2 ? -2 - nb0 : -1;
                /* wall: F_l + dF_l, D_l with this cell's normal; J_l */
                double complex Fw = 0, Dw = 0, A = 0, n1 = 0, n2 = 0;
                if (l >= 0) {
                    A = csqrt(gc->S[0][0] * gc->S[0][0] + gc->S[0][1] * gc->S[0][1]);
                    n1 = gc->S[0][0] / A;
                    n2 = gc->S[0][1] / A;
                    for (int k = 0; k < nv; k++) {
                        double complex vn = p->v[2 * k] * n1 + p->v[2 * k + 1] * n2;
                        if (creal(vn) > 0) {
                            double complex Gk[2][2];
                            so_grad_z(p, psi, gc, k, Gk);
                            double complex f1 = fc[2 * k] + Gk[0][0] * (gc->fm[0][0] - gc->cen[0])
                                                          + Gk[0][1] * (gc->fm[0][1] - gc->cen[1]);
                            Fw += p->w[k] * vn * f1;
                        } else {
                            Dw -= p->w[k] * vn * p->gM[k];
                        }
                    }
                    for (int k = 0; k < nv; k++) {
                        double complex vn = p->v[2 * k] * n1 + p->v[2 * k + 1] * n2, f1;
                        if (creal(vn) > 0) {
                            double complex Gk[2][2];
                            so_grad_z(p, psi, gc, k, Gk);
                            f1 = fc[2 * k] + Gk[0][0] * (gc->fm[0][0] - gc->cen[0]) + Gk[0][1] * (gc->fm[0][1] - gc->cen[1]);
                        } else {
                            f1 = Fw * p->gM[k] / Dw;
                        }
                        L += A * p->w[k] * p->mJ[k] * vn * f1;
                    }
                }
                double rho, u1, u2, th;
                prim(p->W + 4 * c, &rho, &u1, &u2, &th);
                const double itau = inv_tau_of(p, rho, th);
                for (int k = 0; k < nv; k++) {
                    const double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
                    double complex Gc[2][2];
                    so_grad_z(p, psi, gc, k, Gc);
                    double complex r1 = 0, r2 = 0;
                    for (int q = 0; q < 4; q++) {
                        double complex sq = v1 * gc->S[q][0] + v2 * gc->S[q][1];
                        double complex a1, a2;
                        int nb = p->nbr[4 * c + q];
                        if (creal(sq) > 0) {
                            double complex rx = gc->fm[q][0] - gc->cen[0], ry = gc->fm[q][1] - gc->cen[1];
                            a1 = fc[2 * k] + Gc[0][0] * rx + Gc[0][1] * ry;
                            a2 = fc[2 * k + 1] + Gc[1][0] * rx + Gc[1][1] * ry;
                        } else if (nb >= 0) {
                            double complex Gn[2][2];
                            so_grad_z(p, psi, gn[q], k, Gn);
                            double complex rx = gc->fm[q][0] - gn[q]->cen[0], ry = gc->fm[q][1] - gn[q]->cen[1];
                            const double *fj = p->f + ((size_t)nb * nv + k) * 2;
                            a1 = fj[0] + Gn[0][0] * rx + Gn[0][1] * ry;
                            a2 = fj[1] + Gn[1][0] * rx + Gn[1][1] * ry;
                        } else if (nb == -1) {
                            a1 = p->fd[2 * k];
                            a2 = p->fd[2 * k + 1];
                        } else {
                            a1 = (l >= 0 && gc != &gr ? Fw / Dw : (p->F[l] + dF[l]) / p->D[l]) * p->gM[k];
                            a2 = 0.5 * p->theta_w * a1;
                        }
                        r1 += sq * a1;
                        r2 += sq * a2;
                    }
                    double g1, g2;
                    eq_cell_g(p, c, k, &g1, &g2);
                    r1 += gc->V * itau * (fc[2 * k] - g1);
                    r2 += gc->V * itau * (fc[2 * k + 1] - g2);
                    L += p->w[k] * (pc[2 * k] * r1 + pc[2 * k + 1] * r2);
                }
            }
            out[2 * m + d] = cimag(L) / h;
        }
    }
    free(G);
    free(psi);
    free(dF);
}

/* d/dx of the discrete Lagrangian L = J + sum_{c,k} w_k phi_{c,k} . R_{c,k}
 * (as in or_adjoint_dJdp) for every node coordinate x, with f and phi held
 * fixed.  When f solves the primal equations and phi the adjoint equations
 * this is dJ/dx of the discrete problem under mesh motion (the volume-mesh
 * terms that the paper's wall-only derivative of Sec. 2.5 leaves out
 * included).  Each coordinate in turn is shifted by i h; only the residuals
 * of the cells with that node as a corner change (face vectors, volume and,
 * for a wall cell, the element's normal and length through F_l, D_l and the
 * diffuse wall value), and J only through those elements.  out has
 * [(nj+1)(ni+1)][2] entries in the node numbering of the mesh. */
void or_mesh_sensitivity(or_problem *p, double h, double *out)
{
    if (p->order == 2) {
        mesh_sensitivity_so(p, h, out);
        return;
    }
    const int ni = p->ni, nj = p->nj, nv = p->nv, nn = (ni + 1) * (nj + 1);
    eq_cache(p);
#pragma omp parallel for schedule(dynamic, 4) num_threads(p->nthreads)
    for (int m = 0; m < nn; m++) {
        const int im = m % (ni + 1), jm = m / (ni + 1);
        for (int d = 0; d < 2; d++) {
            double complex L = 0;
            for (int jc = jm - 1; jc <= jm; jc++) {
                for (int ic = im - 1; ic <= im; ic++) {
                    if (ic < 0 || ic >= ni || jc < 0 || jc >= nj) continue;
                    const int c = ic + ni * jc;
                    double complex S[4][2], V;
                    cell_geometry_z(p, c, m, d, h, S, &V);
                    const double *fc = p->f + (size_t)c * nv * 2;
                    const double *pc = p->phi + (size_t)c * nv * 2;
                    /* diffuse wall of this cell's j- face */
                    const int nb0 = p->nbr[4 * c];
                    const int l = nb0 <= -2 ? -2 - nb0 : -1;
                    double complex A = 0, n1 = 0, n2 = 0, Fz = 0, Dz = 0;
                    if (l >= 0) {
                        A = csqrt(S[0][0] * S[0][0] + S[0][1] * S[0][1]);
                        n1 = S[0][0] / A;
                        n2 = S[0][1] / A;
                        for (int k = 0; k < nv; k++) {
                            double complex vn = p->v[2 * k] * n1 + p->v[2 * k + 1] * n2;
                            if (creal(vn) > 0) Fz += p->w[k] * vn * fc[2 * k];
                            else Dz -= p->w[k] * vn * p->gM[k];
                        }
                        /* J_l, eq. (numer_J) */
                        for (int k = 0; k < nv; k++) {
                            double complex vn = p->v[2 * k] * n1 + p->v[2 * k + 1] * n2;
                            double complex f1 = creal(vn) > 0 ? fc[2 * k] : Fz * p->gM[k] / Dz;
                            L += A * p->w[k] * p->mJ[k] * vn * f1;
                        }
                    }
                    double rho, u1, u2, th;
                    prim(p->W + 4 * c, &rho, &u1, &u2, &th);
                    const double itau = inv_tau_of(p, rho, th);
                    for (int k = 0; k < nv; k++) {
                        const double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
                        double complex r1 = 0, r2 = 0;
                        for (int q = 0; q < 4; q++) {
                            double complex sq = v1 * S[q][0] + v2 * S[q][1];
                            double complex a1, a2;
                            if (creal(sq) > 0) { a1 = fc[2 * k]; a2 = fc[2 * k + 1]; }
                            else {
                                int nb = p->nbr[4 * c + q];
                                if (nb >= 0) { a1 = p->f[((size_t)nb * nv + k) * 2]; a2 = p->f[((size_t)nb * nv + k) * 2 + 1]; }
                                else if (nb == -1) { a1 = p->fd[2 * k]; a2 = p->fd[2 * k + 1]; }
                                else { a1 = Fz * p->gM[k] / Dz; a2 = 0.5 * p->theta_w * a1; }
                            }
                            r1 += sq * a1;
                            r2 += sq * a2;
                        }
                        double g1, g2;
                        eq_cell_g(p, c, k, &g1, &g2);
                        r1 += V * itau * (fc[2 * k] - g1);
                        r2 += V * itau * (fc[2 * k + 1] - g2);
                        L += p->w[k] * (pc[2 * k] * r1 + pc[2 * k + 1] * r2);
                    }
                }
            }
            out[2 * m + d] = cimag(L) / h;
        }
    }
}

/* ------------------------------------------------------------------ */
/* wall sensitivity                                                    */
/* ------------------------------------------------------------------ */

/* The scheme's values the sensitivity formulas read: order 1 takes the
 * upwind cell values and the wall flux F_l; order 2 the reconstructed
 * values (slopes G of f) and F_l + dF_l.  The paper evaluates its formulas
 * with the values of its (second-order) scheme. */
typedef struct { double *G; double *Fw; } wall_ctx;

static wall_ctx wall_ctx_make(const or_problem *p)
{
    wall_ctx w = { NULL, malloc(sizeof(double) * (p->nw > 0 ? p->nw : 1)) };
    if (p->order == 2) {
        w.G = malloc(sizeof(double) * 4 * (size_t)p->nc * p->nv);
        so_slopes(p, p->f, w.G, NULL);
        so_wall_dF(p, w.G, w.Fw);
        for (int l = 0; l < p->nw; l++) w.Fw[l] += p->F[l];
    } else {
        for (int l = 0; l < p->nw; l++) w.Fw[l] = p->F[l];
    }
    return w;
}

static void wall_ctx_free(wall_ctx *w) { free(w->G); free(w->Fw); }

/* wall value of component m at element l, velocity k: the wall cell's
 * (reconstructed) value on Xi^+, the diffuse value on Xi^- */
static double wall_fx(const or_problem *p, const wall_ctx *w, int l, int k, int m)
{
    int c = p->wall_cell[l];
    double vn = p->v[2 * k] * p->wn[2 * l] + p->v[2 * k + 1] * p->wn[2 * l + 1];
    if (vn > 0)
        return p->f[((size_t)c * p->nv + k) * 2 + m] + (w->G ? so_delta(p, w->G, c, p->wall_face[l], k, m, 1.0) : 0.0);
    double g1 = w->Fw[l] * p->gM[k] / p->D[l];
    return m == 0 ? g1 : 0.5 * p->theta_w * g1;
}

/* Green-Gauss gradient of eq. (gaussgrad) at cell c, velocity k, with the
 * scheme's face values (upwind side; reconstructed at order 2) */
static void gauss_grad(const or_problem *p, const wall_ctx *w, int c, int k, double g[2][2])
{
    double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
    const double *fc = p->f + ((size_t)c * p->nv + k) * 2;
    double V = p->vol[c];
    g[0][0] = g[0][1] = g[1][0] = g[1][1] = 0;
    for (int q = 0; q < 4; q++) {
        double Sx = p->S[8 * c + 2 * q], Sy = p->S[8 * c + 2 * q + 1];
        double s = v1 * Sx + v2 * Sy, a1, a2;
        if (s > 0) { a1 = fc[0]; a2 = fc[1]; }
        else inflow_value(p, p->f, w->Fw, c, q, k, &a1, &a2);
        if (w->G) { a1 += so_delta(p, w->G, c, q, k, 0, s); a2 += so_delta(p, w->G, c, q, k, 1, s); }
        g[0][0] += a1 * Sx; g[0][1] += a1 * Sy;
        g[1][0] += a2 * Sx; g[1][1] += a2 * Sy;
    }
    for (int a = 0; a < 2; a++) for (int b = 0; b < 2; b++) g[a][b] /= V;
}

/* The Green-Gauss gradient of eq. (gaussgrad) at cell c for every velocity,
 * out[k][component][direction], with the current f and wall fluxes (access
 * for the tests that pin it on fields whose upwind differences have closed
 * forms). */
void or_gauss_grad(or_problem *p, int c, double *out)
{
    wall_ctx wc = wall_ctx_make(p);
    for (int k = 0; k < p->nv; k++) {
        double g[2][2];
        gauss_grad(p, &wc, c, k, g);
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) out[4 * k + 2 * a + b] = g[a][b];
    }
    wall_ctx_free(&wc);
}

/* Element derivatives dL/dA_l, dL/dx_l, dL/dn_l (eqs. sens_J_itf, sens_B_itf)
 * and their transform to the wall nodes (eq. sens_nod).  Wall node m is
 * x_{l,1} of element l = m and x_{l,2} of element m - 1 (closed loop). */
void or_wall_sensitivity(or_problem *p, double *SA, double *Sx, double *Sn, double *dJdnodes)
{
    const int nv = p->nv, nw = p->nw;
    wall_ctx wc = wall_ctx_make(p);
    for (int l = 0; l < nw; l++) {
        int c = p->wall_cell[l];
        double n1 = p->wn[2 * l], n2 = p->wn[2 * l + 1], A = p->wA[l];
        const double *ph = p->phi + (size_t)c * nv * 2;
        double sa = 0, jx[2] = { 0, 0 }, bx[2] = { 0, 0 }, G[2] = { 0, 0 }, M[2] = { 0, 0 };
        double Phi = 0, jn[2] = { 0, 0 };
        for (int k = 0; k < nv; k++) {
            double v1 = p->v[2 * k], v2 = p->v[2 * k + 1], vn = v1 * n1 + v2 * n2, wk = p->w[k];
            double f1 = wall_fx(p, &wc, l, k, 0);
            double gr[2][2];
            gauss_grad(p, &wc, c, k, gr);
            sa += wk * p->mJ[k] * vn * f1;
            jx[0] += wk * p->mJ[k] * vn * gr[0][0];
            jx[1] += wk * p->mJ[k] * vn * gr[0][1];
            jn[0] += wk * p->mJ[k] * v1 * f1;
            jn[1] += wk * p->mJ[k] * v2 * f1;
            M[0] += wk * v1 * f1;
            M[1] += wk * v2 * f1;
            if (vn > 0) {
                G[0] += wk * vn * gr[0][0];
                G[1] += wk * vn * gr[0][1];
            } else {
                double pw1 = -vn * (ph[2 * k] + p->mJ[k]), pw2 = -vn * ph[2 * k + 1];
                double gb1 = p->gM[k] / p->D[l], gb2 = 0.5 * p->theta_w * gb1;
                bx[0] += wk * (pw1 * gr[0][0] + pw2 * gr[1][0]);
                bx[1] += wk * (pw1 * gr[0][1] + pw2 * gr[1][1]);
                Phi += wk * (pw1 * gb1 + pw2 * gb2);
            }
        }
        SA[l] = sa;
        Sx[2 * l] = A * (jx[0] + bx[0] - Phi * G[0]);
        Sx[2 * l + 1] = A * (jx[1] + bx[1] - Phi * G[1]);
        Sn[2 * l] = A * (jn[0] - Phi * M[0]);
        Sn[2 * l + 1] = A * (jn[1] - Phi * M[1]);
    }
    wall_ctx_free(&wc);
    if (!dJdnodes) return;
    for (int m = 0; m < 2 * nw; m++) dJdnodes[m] = 0;
    for (int l = 0; l < nw; l++) {
        double ax = p->wa[2 * l], ay = p->wa[2 * l + 1], bxn = p->wb[2 * l], byn = p->wb[2 * l + 1];
        double A = p->wA[l], n1 = p->wn[2 * l], n2 = p->wn[2 * l + 1];
        double dAa[2] = { (ax - bxn) / A, (ay - byn) / A };
        double cross = (ax - bxn) * n2 - (ay - byn) * n1;
        double sg = cross > 0 ? 1.0 : -1.0;
        /* dn/da: rows = components of n, columns = coordinates of a */
        double Na[2][2] = { { -n1 * n2 * sg / A, -n2 * n2 * sg / A }, { n1 * n1 * sg / A, n1 * n2 * sg / A } };
        double ga[2], gb[2];
        for (int d = 0; d < 2; d++) {
            double tn = Sn[2 * l] * Na[0][d] + Sn[2 * l + 1] * Na[1][d];
            ga[d] = SA[l] * dAa[d] + 0.5 * Sx[2 * l + d] + tn;
            gb[d] = -SA[l] * dAa[d] + 0.5 * Sx[2 * l + d] - tn;
        }
        int ma = l, mb = (l + 1) % nw;
        dJdnodes[2 * ma] += ga[0]; dJdnodes[2 * ma + 1] += ga[1];
        dJdnodes[2 * mb] += gb[0]; dJdnodes[2 * mb + 1] += gb[1];
    }
}

/* Discrete J_l + B_w,l of eqs. (numer_J), (numer_B) for element l at
 * perturbed element attributes (A, x, n) with f and phi frozen: f on the
 * element follows the linear reconstruction f_l + grad f . (x - x_l); the
 * integration ranges stay those of the unperturbed normal (Sec. 3.2).
 * Pins the element derivatives. */
double or_wall_JB(or_problem *p, int l, double A, double x1, double x2, double n1, double n2)
{
    const int nv = p->nv;
    int c = p->wall_cell[l];
    double on1 = p->wn[2 * l], on2 = p->wn[2 * l + 1];
    double dx1 = x1 - p->wx[2 * l], dx2 = x2 - p->wx[2 * l + 1];
    const double *ph = p->phi + (size_t)c * nv * 2;
    wall_ctx wc = wall_ctx_make(p);
    /* F and D at (x, n) */
    double F = 0, D = 0;
    for (int k = 0; k < nv; k++) {
        double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
        double vn0 = v1 * on1 + v2 * on2, vn = v1 * n1 + v2 * n2;
        double gr[2][2];
        gauss_grad(p, &wc, c, k, gr);
        if (vn0 > 0) F += p->w[k] * vn * (wall_fx(p, &wc, l, k, 0) + gr[0][0] * dx1 + gr[0][1] * dx2);
        else D -= p->w[k] * vn * p->gM[k];
    }
    double J = 0, B = 0;
    for (int k = 0; k < nv; k++) {
        double v1 = p->v[2 * k], v2 = p->v[2 * k + 1];
        double vn0 = v1 * on1 + v2 * on2, vn = v1 * n1 + v2 * n2;
        double gr[2][2];
        gauss_grad(p, &wc, c, k, gr);
        double f1l = wall_fx(p, &wc, l, k, 0);
        double f2l = wall_fx(p, &wc, l, k, 1);
        double f1x = f1l + gr[0][0] * dx1 + gr[0][1] * dx2;
        double f2x = f2l + gr[1][0] * dx1 + gr[1][1] * dx2;
        J += p->w[k] * p->mJ[k] * vn * f1x;
        if (vn0 <= 0) {
            double pw1 = -vn0 * (ph[2 * k] + p->mJ[k]), pw2 = -vn0 * ph[2 * k + 1];
            double gb1 = p->gM[k] / D, gb2 = 0.5 * p->theta_w * gb1;
            B += p->w[k] * (pw1 * (f1x - F * gb1) + pw2 * (f2x - F * gb2));
        }
    }
    wall_ctx_free(&wc);
    return A * (J + B);
}
