// Host side of the optimisation's outer loop: the CST parameterisation and
// its least-squares initial design (Sec. 3.3), the volume constraint (Sec.
// 2.4, Sec. 3.2), and the set-up and small dense steps of the
// radial-basis-function mesh deformation (Sec. 3.4, Step 2) whose per-node
// sums run in dvm_rbf.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <thread>
#include <vector>

#include "../../include/dvm.h"
#include "dvm_internal.h"

using dvm::set_error;

namespace {

#define HIP_OK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return set_error(DVM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kMaxCentres = 8192;   // dense host factor: 8192^2 doubles = 512 MiB

// f(r) for r in [lo, hi) on nt host threads, r going to thread r mod nt.
// Each entry of a result is computed by one thread in a fixed order, so the
// result does not depend on the thread count.
template <class F>
void parallel_rows(int lo, int hi, int nt, F &&f)
{
    nt = std::max(1, std::min(nt, hi - lo));
    if (nt == 1) {
        for (int r = lo; r < hi; r++) f(r);
        return;
    }
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; t++)
        th.emplace_back([=, &f] {
            for (int r = lo + t; r < hi; r += nt) f(r);
        });
    for (auto &x : th) x.join();
}

// In-place Cholesky factorisation A = L L^T of a symmetric n x n matrix
// (row-major, lower triangle used); false if A is not positive definite.
// Right-looking by column blocks of kCholBlock: factor the diagonal block,
// solve the panel below it row by row, then subtract the panel's products
// from the trailing lower triangle.  Every inner loop runs over contiguous
// row segments of at most kCholBlock entries, which stay in cache.
constexpr int kCholBlock = 64;

bool cholesky(std::vector<double> &A, int n)
{
    double *a = A.data();
    auto at = [=](int i, int j) -> double & { return a[(size_t)i * n + j]; };
    // up to 16 host threads for the large RBF systems, none for small ones
    const int nt = n < 256 ? 1 : (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
    for (int k0 = 0; k0 < n; k0 += kCholBlock) {
        const int k1 = std::min(n, k0 + kCholBlock);
        for (int j = k0; j < k1; j++) {
            double d = at(j, j);
            for (int k = k0; k < j; k++) d -= at(j, k) * at(j, k);
            if (!(d > 0.0)) return false;
            const double ljj = std::sqrt(d);
            at(j, j) = ljj;
            for (int i = j + 1; i < k1; i++) {
                double s = at(i, j);
                for (int k = k0; k < j; k++) s -= at(i, k) * at(j, k);
                at(i, j) = s / ljj;
            }
        }
        if (k1 == n) break;
        // panel: row i's entries in columns [k0, k1) by forward substitution
        parallel_rows(k1, n, nt, [&](int i) {
            for (int j = k0; j < k1; j++) {
                double s = at(i, j);
                for (int k = k0; k < j; k++) s -= at(i, k) * at(j, k);
                at(i, j) = s / at(j, j);
            }
        });
        // trailing update A(i, j) -= sum_k L(i, k) L(j, k), k1 <= j <= i, by
        // tiles of kCholBlock x kCholBlock (one task each, the two panel
        // slices it reads stay in cache), inside them 4 x 4 register tiles
        // in which every loaded panel entry serves four products
        const int kw = k1 - k0;
        const int nb = (n - k1 + kCholBlock - 1) / kCholBlock;
        parallel_rows(0, nb * (nb + 1) / 2, nt, [&](int task) {
            int bi = 0;
            while ((bi + 1) * (bi + 2) / 2 <= task) bi++;
            const int bj = task - bi * (bi + 1) / 2;
            const int i0 = k1 + bi * kCholBlock, i1 = std::min(n, i0 + kCholBlock);
            const int j0 = k1 + bj * kCholBlock, j1 = std::min(n, j0 + kCholBlock);
            for (int i = i0; i < i1; i += 4)
                for (int j = j0; j < j1 && j <= i + 3; j += 4) {
                    if (i + 4 <= i1 && j + 4 <= j1 && j + 3 <= i) {
                        const double *r0 = a + (size_t)i * n + k0, *r1 = r0 + n, *r2 = r1 + n, *r3 = r2 + n;
                        const double *c0 = a + (size_t)j * n + k0, *c1 = c0 + n, *c2 = c1 + n, *c3 = c2 + n;
                        double acc[4][4] = {};
                        for (int k = 0; k < kw; k++) {
                            const double x[4] = {r0[k], r1[k], r2[k], r3[k]};
                            const double y[4] = {c0[k], c1[k], c2[k], c3[k]};
                            for (int u = 0; u < 4; u++)
                                for (int v = 0; v < 4; v++) acc[u][v] += x[u] * y[v];
                        }
                        for (int u = 0; u < 4; u++)
                            for (int v = 0; v < 4; v++) at(i + u, j + v) -= acc[u][v];
                    } else {          // tiles on the diagonal or the ragged edge
                        for (int u = i; u < std::min(i + 4, i1); u++)
                            for (int v = j; v < std::min(j + 4, j1) && v <= u; v++) {
                                double acc = 0.0;
                                for (int k = k0; k < k1; k++) acc += at(u, k) * at(v, k);
                                at(u, v) -= acc;
                            }
                    }
                }
        });
    }
    return true;
}

// Solve L L^T x = b in place for nrhs right-hand sides stored b[i*nrhs + r].
// Both substitutions read L by rows: forward, row i against the solved
// entries above it; backward (L^T x = y), each solved x_i is subtracted,
// times row i of L, from the entries before it.
void cholesky_solve(const std::vector<double> &L, int n, double *b, int nrhs)
{
    for (int i = 0; i < n; i++) {
        const double *li = L.data() + (size_t)i * n;
        for (int r = 0; r < nrhs; r++) {
            double s = b[(size_t)i * nrhs + r];
            for (int k = 0; k < i; k++) s -= li[k] * b[(size_t)k * nrhs + r];
            b[(size_t)i * nrhs + r] = s / li[i];
        }
    }
    for (int i = n - 1; i >= 0; i--) {
        const double *li = L.data() + (size_t)i * n;
        for (int r = 0; r < nrhs; r++) {
            const double x = b[(size_t)i * nrhs + r] / li[i];
            b[(size_t)i * nrhs + r] = x;
            for (int k = 0; k < i; k++) b[(size_t)k * nrhs + r] -= li[k] * x;
        }
    }
}

// ---------------------------------------------------------------------------
// CST (Sec. 3.3)
// ---------------------------------------------------------------------------

struct Cst {
    int nb;
    double binom[DVM_CST_MAX_NB + 1];
    explicit Cst(int nb_) : nb(nb_)
    {
        binom[0] = 1.0;
        for (int b = 1; b <= nb; b++) binom[b] = binom[b - 1] * (nb - b + 1) / b;
    }
    int np() const { return 2 * nb + 6; }
    // eta at one station and (if row != NULL) its row of d eta / d alpha
    double eval(const double *a, double xi, bool up, double *row) const
    {
        const double x = xi, y = 1.0 - xi;
        double bern[DVM_CST_MAX_NB + 1];
        // S_b = binom(nb, b) x^b y^(nb - b)
        double xp = 1.0;
        for (int b = 0; b <= nb; b++) {
            bern[b] = binom[b] * xp;
            xp *= x;
        }
        double yp = 1.0;
        for (int b = nb; b >= 0; b--) {
            bern[b] *= yp;
            yp *= y;
        }
        const double *A = up ? a + 2 : a + nb + 3;
        double S = 0.0;
        for (int b = 0; b <= nb; b++) S += A[b] * bern[b];
        const double C = std::pow(x, a[0]) * std::pow(y, a[1]);
        const double T = up ? a[2 * nb + 4] : a[2 * nb + 5];
        if (row) {
            std::fill(row, row + np(), 0.0);
            row[0] = x > 0.0 ? C * std::log(x) * S : 0.0;
            row[1] = y > 0.0 ? C * std::log(y) * S : 0.0;
            double *dA = up ? row + 2 : row + nb + 3;
            for (int b = 0; b <= nb; b++) dA[b] = C * bern[b];
            row[up ? 2 * nb + 4 : 2 * nb + 5] = x;
        }
        return C * S + x * T;
    }
};

int check_cst(int nb, const double *alpha, int n, const double *xi, const int32_t *upper)
{
    if (nb < 1 || nb > DVM_CST_MAX_NB) return set_error(DVM_EINVAL, "CST order %d outside [1, %d]", nb, DVM_CST_MAX_NB);
    if (n < 0 || (n > 0 && (!xi || !upper)) || !alpha) return set_error(DVM_EINVAL, "null or negative-size argument");
    if (!(alpha[0] > 0.0) || !(alpha[1] > 0.0))
        return set_error(DVM_EINVAL, "class exponents must be positive (N1 %g, N2 %g)", alpha[0], alpha[1]);
    for (int m = 0; m < n; m++)
        if (!(xi[m] >= 0.0 && xi[m] <= 1.0)) return set_error(DVM_EINVAL, "station %d: xi %g outside [0, 1]", m, xi[m]);
    return DVM_OK;
}

}  // namespace

int dvm_cst_eval(int nb, const double *alpha, int n, const double *xi, const int32_t *upper, double *eta,
                 double *jac)
{
    if (int e = check_cst(nb, alpha, n, xi, upper)) return e;
    if (n > 0 && !eta) return set_error(DVM_EINVAL, "null eta");
    const Cst cst(nb);
    for (int m = 0; m < n; m++)
        eta[m] = cst.eval(alpha, xi[m], upper[m] != 0, jac ? jac + (size_t)m * cst.np() : nullptr);
    return DVM_OK;
}

int dvm_cst_fit(int nb, int n, const double *xi, const int32_t *upper, const double *eta, const int32_t *fixed,
                double *alpha, double *rms)
{
    if (!alpha || (n > 0 && !eta)) return set_error(DVM_EINVAL, "null argument");
    if (nb < 1 || nb > DVM_CST_MAX_NB) return set_error(DVM_EINVAL, "CST order %d outside [1, %d]", nb, DVM_CST_MAX_NB);
    try {
        const Cst cst(nb);
        const int np = cst.np();
        std::vector<int> fr;
        for (int p = 0; p < np; p++) {
            const bool fx = fixed ? fixed[p] != 0 : p >= 2 * nb + 4;
            if (!fx) fr.push_back(p);
        }
        std::vector<double> a(alpha, alpha + np);
        if (!fixed || !fixed[0]) a[0] = 0.5;
        if (!fixed || !fixed[1]) a[1] = 1.0;
        if (int e = check_cst(nb, a.data(), n, xi, upper)) return e;
        const int nf = (int)fr.size();
        std::vector<double> row(np), r(n), Jf((size_t)n * nf), H, g(nf), trial(np);
        auto residual = [&](const std::vector<double> &al, bool jac) {
            double c = 0.0;
            for (int m = 0; m < n; m++) {
                r[m] = eta[m] - cst.eval(al.data(), xi[m], upper[m] != 0, jac ? row.data() : nullptr);
                c += r[m] * r[m];
                if (jac)
                    for (int k = 0; k < nf; k++) Jf[(size_t)m * nf + k] = row[fr[k]];
            }
            return c;
        };
        auto normal = [&](const std::vector<int> &cols, std::vector<double> &Hm, std::vector<double> &gv) {
            const int k = (int)cols.size();
            Hm.assign((size_t)k * k, 0.0);
            gv.assign(k, 0.0);
            for (int m = 0; m < n; m++)
                for (int i = 0; i < k; i++) {
                    const double ji = Jf[(size_t)m * nf + cols[i]];
                    gv[i] += ji * r[m];
                    for (int j = 0; j <= i; j++) Hm[(size_t)i * k + j] += ji * Jf[(size_t)m * nf + cols[j]];
                }
            for (int i = 0; i < k; i++)
                for (int j = 0; j < i; j++) Hm[(size_t)j * k + i] = Hm[(size_t)i * k + j];
        };
        // the free shape coefficients and offsets enter linearly: fit them
        // at the starting class first
        double c = residual(a, true);
        {
            std::vector<int> lin;
            for (int k = 0; k < nf; k++)
                if (fr[k] >= 2) lin.push_back(k);
            std::vector<double> Hl, gl;
            normal(lin, Hl, gl);
            if (!lin.empty()) {
                if (!cholesky(Hl, (int)lin.size()))
                    return set_error(DVM_EINVAL, "the %d stations do not determine the %zu linear CST variables", n,
                                     lin.size());
                cholesky_solve(Hl, (int)lin.size(), gl.data(), 1);
                for (size_t k = 0; k < lin.size(); k++) a[fr[lin[k]]] += gl[k];
            }
        }
        // damped Gauss-Newton (Marquardt scaling) over all free variables
        std::vector<int> all(nf);
        for (int k = 0; k < nf; k++) all[k] = k;
        double lam = 1e-3;
        c = residual(a, true);
        for (int it = 0; it < 200 && nf > 0; it++) {
            normal(all, H, g);
            bool improved = false;
            for (int tr = 0; tr < 30; tr++) {
                std::vector<double> Hd(H);
                for (int k = 0; k < nf; k++) Hd[(size_t)k * nf + k] += lam * H[(size_t)k * nf + k];
                std::vector<double> step(g);
                if (!cholesky(Hd, nf)) {
                    lam *= 10.0;
                    continue;
                }
                cholesky_solve(Hd, nf, step.data(), 1);
                trial = a;
                for (int k = 0; k < nf; k++) trial[fr[k]] += step[k];
                if (!(trial[0] > 0.0) || !(trial[1] > 0.0)) {
                    lam *= 10.0;
                    continue;
                }
                const double ct = residual(trial, false);
                if (ct <= c) {
                    improved = c - ct > 1e-15 * c;
                    a = trial;
                    c = ct;
                    lam = std::max(lam / 10.0, 1e-12);
                    break;
                }
                lam *= 10.0;
            }
            if (!improved) break;
            c = residual(a, true);
        }
        std::copy(a.begin(), a.end(), alpha);
        if (rms) *rms = n > 0 ? std::sqrt(c / n) : 0.0;
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(DVM_ENOMEM, "out of host memory");
    }
}

int dvm_volume_constraint(int nw, const double *wall_xy, double v_min, double *Q, double *dQ_dx)
{
    if (nw < 3 || !wall_xy || !Q) return set_error(DVM_EINVAL, "need a closed loop of >= 3 wall nodes and Q");
    double q = 0.0;
    for (int l = 0; l < nw; l++) {
        const double *a = wall_xy + 2 * l, *b = wall_xy + 2 * ((l + 1) % nw);
        // A n into the solid = (dy, -dx) for a clockwise wall; midpoint (a + b) / 2
        q += 0.5 * ((b[1] - a[1]) * (0.5 * (a[0] + b[0])) - (b[0] - a[0]) * (0.5 * (a[1] + b[1])));
    }
    *Q = q + v_min;
    if (dQ_dx) {
        for (int m = 0; m < nw; m++) {
            const double *p = wall_xy + 2 * ((m + nw - 1) % nw), *x = wall_xy + 2 * m,
                         *nx = wall_xy + 2 * ((m + 1) % nw);
            // elements (p, x) and (x, nx): sum of A n is (nx_y - p_y, p_x - nx_x)
            dQ_dx[2 * m] = 0.5 * ((x[1] - p[1]) + (nx[1] - x[1]));
            dQ_dx[2 * m + 1] = 0.5 * ((p[0] - x[0]) + (x[0] - nx[0]));
        }
    }
    return DVM_OK;
}

// ---------------------------------------------------------------------------
// RBF deformation (Sec. 3.4, Step 2)
// ---------------------------------------------------------------------------

struct dvm_deform {
    int nn = 0, nw = 0, nchunk = 0;
    double radius = 0.0;
    std::vector<double> x0;        // [nn][2] reference nodes
    std::vector<int32_t> widx;     // [nn] wall node of each node, or -1
    std::vector<double> c;         // [nw][2] centres
    std::vector<double> L;         // Cholesky factor of M, [nw][nw]
    // device
    char *base = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    size_t o_x0 = 0, o_widx = 0, o_c = 0, o_gam = 0, o_wall = 0, o_out = 0, o_g = 0, o_part = 0, o_h = 0, total = 0;
};

int dvm_deform_create(const dvm_mesh *m, double radius, dvm_deform **out)
{
    if (!m || !out) return set_error(DVM_EINVAL, "null argument");
    *out = nullptr;
    if (!(radius > 0.0) || !std::isfinite(radius)) return set_error(DVM_EINVAL, "support radius %g must be > 0", radius);
    try {
        const dvm::MeshNodes mn = dvm::mesh_nodes(m);
        if (mn.nw > kMaxCentres)
            return set_error(DVM_EINVAL, "%d wall nodes: the dense RBF system takes at most %d", mn.nw, kMaxCentres);
        auto *d = new dvm_deform;
        d->nn = (mn.ni + 1) * (mn.nj + 1);
        d->nw = mn.nw;
        d->radius = radius;
        d->x0.assign(mn.nodes, mn.nodes + 2 * (size_t)d->nn);
        d->widx.assign(d->nn, -1);
        d->c.assign(2 * (size_t)d->nw, 0.0);
        for (int i = mn.nwake; i <= mn.nwake + mn.nw; i++) d->widx[i] = (i - mn.nwake) % mn.nw;
        for (int l = 0; l < d->nw; l++) {
            d->c[2 * l] = d->x0[2 * (size_t)(mn.nwake + l)];
            d->c[2 * l + 1] = d->x0[2 * (size_t)(mn.nwake + l) + 1];
        }
        const int nw = d->nw;
        d->L.assign((size_t)nw * nw, 0.0);
        for (int i = 0; i < nw; i++)
            for (int j = 0; j < nw; j++) {
                const double dx = d->c[2 * i] - d->c[2 * j], dy = d->c[2 * i + 1] - d->c[2 * j + 1];
                const double r = std::sqrt(dx * dx + dy * dy) / radius;
                d->L[(size_t)i * nw + j] = r < 1.0 ? (1.0 - r) * (1.0 - r) : 0.0;
            }
        if (!cholesky(d->L, nw)) {
            delete d;
            return set_error(DVM_EINVAL, "RBF interpolation matrix is not positive definite (coincident wall nodes?)");
        }
        d->nchunk = dvm::rbf_chunks(d->nn);
        size_t o = 0;
        auto take = [&](size_t b) {
            const size_t at = o;
            o = align_up(o + b);
            return at;
        };
        d->o_x0 = take(16 * (size_t)d->nn);
        d->o_widx = take(4 * (size_t)d->nn);
        d->o_c = take(16 * (size_t)nw);
        d->o_gam = take(16 * (size_t)nw);
        d->o_wall = take(16 * (size_t)nw);
        d->o_out = take(16 * (size_t)d->nn);
        d->o_g = take(16 * (size_t)d->nn);
        d->o_part = take(16 * (size_t)nw * d->nchunk);
        d->o_h = take(16 * (size_t)nw);
        d->total = o;
        *out = d;
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(DVM_ENOMEM, "out of host memory");
    }
}

size_t dvm_deform_workspace_bytes(const dvm_deform *d) { return d ? d->total : 0; }

int dvm_deform_bind(dvm_deform *d, void *dev_ptr, size_t bytes, void *hip_stream)
{
    if (!d || !dev_ptr) return set_error(DVM_EINVAL, "null argument");
    if ((uintptr_t)dev_ptr % kAlign) return set_error(DVM_EINVAL, "device buffer not 256-byte aligned");
    if (bytes < d->total) return set_error(DVM_ENOMEM, "device buffer %zu bytes < %zu needed", bytes, d->total);
    d->base = (char *)dev_ptr;
    d->bytes = bytes;
    d->stream = (hipStream_t)hip_stream;
    HIP_OK(hipMemcpyAsync(d->base + d->o_x0, d->x0.data(), 16 * (size_t)d->nn, hipMemcpyHostToDevice, d->stream));
    HIP_OK(hipMemcpyAsync(d->base + d->o_widx, d->widx.data(), 4 * (size_t)d->nn, hipMemcpyHostToDevice, d->stream));
    HIP_OK(hipMemcpyAsync(d->base + d->o_c, d->c.data(), 16 * (size_t)d->nw, hipMemcpyHostToDevice, d->stream));
    HIP_OK(hipStreamSynchronize(d->stream));
    return DVM_OK;
}

int dvm_deform_apply(dvm_deform *d, const double *wall_xy, double *nodes_xy)
{
    if (!d || !wall_xy || !nodes_xy) return set_error(DVM_EINVAL, "null argument");
    if (!d->base) return set_error(DVM_ESTATE, "deformer not bound to a device buffer");
    try {
        const int nw = d->nw;
        std::vector<double> gam(2 * (size_t)nw);
        for (size_t k = 0; k < gam.size(); k++) {
            if (!std::isfinite(wall_xy[k])) return set_error(DVM_EINVAL, "non-finite wall position");
            gam[k] = wall_xy[k] - d->c[k];
        }
        cholesky_solve(d->L, nw, gam.data(), 2);
        HIP_OK(hipMemcpyAsync(d->base + d->o_gam, gam.data(), 16 * (size_t)nw, hipMemcpyHostToDevice, d->stream));
        HIP_OK(hipMemcpyAsync(d->base + d->o_wall, wall_xy, 16 * (size_t)nw, hipMemcpyHostToDevice, d->stream));
        HIP_OK(dvm::launch_rbf_apply((const double *)(d->base + d->o_x0), (const int32_t *)(d->base + d->o_widx), d->nn,
                                     (const double *)(d->base + d->o_c), (const double *)(d->base + d->o_gam),
                                     (const double *)(d->base + d->o_wall), nw, 1.0 / d->radius,
                                     (double *)(d->base + d->o_out), d->stream));
        HIP_OK(hipMemcpyAsync(nodes_xy, d->base + d->o_out, 16 * (size_t)d->nn, hipMemcpyDeviceToHost, d->stream));
        HIP_OK(hipStreamSynchronize(d->stream));
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(DVM_ENOMEM, "out of host memory");
    }
}

int dvm_deform_chain(dvm_deform *d, const double *dJ_dx, double *dJ_dwall)
{
    if (!d || !dJ_dx || !dJ_dwall) return set_error(DVM_EINVAL, "null argument");
    if (!d->base) return set_error(DVM_ESTATE, "deformer not bound to a device buffer");
    try {
        const int nw = d->nw;
        HIP_OK(hipMemcpyAsync(d->base + d->o_g, dJ_dx, 16 * (size_t)d->nn, hipMemcpyHostToDevice, d->stream));
        HIP_OK(dvm::launch_rbf_chain((const double *)(d->base + d->o_x0), (const int32_t *)(d->base + d->o_widx),
                                     (const double *)(d->base + d->o_g), d->nn, (const double *)(d->base + d->o_c),
                                     nw, 1.0 / d->radius, (double *)(d->base + d->o_part),
                                     (double *)(d->base + d->o_h), d->stream));
        std::vector<double> h(2 * (size_t)nw);
        HIP_OK(hipMemcpyAsync(h.data(), d->base + d->o_h, 16 * (size_t)nw, hipMemcpyDeviceToHost, d->stream));
        HIP_OK(hipStreamSynchronize(d->stream));
        cholesky_solve(d->L, nw, h.data(), 2);       // M is symmetric: M^-T h = M^-1 h
        std::copy(h.begin(), h.end(), dJ_dwall);
        for (int n = 0; n < d->nn; n++) {
            const int l = d->widx[n];
            if (l >= 0) {
                dJ_dwall[2 * l] += dJ_dx[2 * (size_t)n];
                dJ_dwall[2 * l + 1] += dJ_dx[2 * (size_t)n + 1];
            }
        }
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return set_error(DVM_ENOMEM, "out of host memory");
    }
}

void dvm_deform_destroy(dvm_deform *d) { delete d; }
