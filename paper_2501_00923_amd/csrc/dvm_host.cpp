// Host side of libdvm: structured-grid connectivity and geometry, velocity
// quadrature, flow constants, the device workspace layout, the solve state
// machine and the C ABI declared in include/dvm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <mutex>
#include <vector>

#include "../../include/dvm.h"
#include "dvm_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(DVM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

// ---------------------------------------------------------------------------
// mesh
// ---------------------------------------------------------------------------
struct dvm_mesh {
    int topo = 0, ni = 0, nj = 0, nwake = 0, nc = 0, nw = 0;
    std::vector<double> nodes;       // [(nj+1)(ni+1)][2]
    std::vector<int32_t> nbr;        // [nc][4]
    std::vector<int32_t> wall_cell;  // [nw]
    std::vector<double> S;           // [nc][4][2]
    std::vector<double> vol;         // [nc]
    std::vector<double> cen;         // [nc][2] area centroids
    std::vector<double> fm;          // [nc][4][2] face midpoints
    std::vector<double> wA, wn, wx, wa, wb;
    std::vector<int32_t> perm;       // [nc] device (storage) number of each cell
    std::vector<int32_t> pstart;     // [np + 1] first device cell of each patch
};

namespace {

using P2 = std::array<double, 2>;

// Sweep and storage order: strips of kTileI columns, each walked outward in
// tiles of kTileI x kTileJ cells; a tile is cut into patches of kPatchI x
// kPatchJ cells (one workgroup of a sweep each) taken row by row, and a
// patch's cells are numbered row by row.  Neighbour rows that a patch reads
// from outside itself belong to patches processed shortly before or after
// it on the same XCD (in its L2, else in the MALL), and the rows of the
// workgroups in flight are contiguous in memory.
void build_patches(dvm_mesh &m)
{
    using dvm::kPatchI;
    using dvm::kPatchJ;
    using dvm::kTileI;
    using dvm::kTileJ;
    m.perm.assign(m.nc, -1);
    m.pstart.clear();
    int32_t next = 0;
    for (int i0 = 0; i0 < m.ni; i0 += kTileI) {
        const int i1 = std::min(i0 + kTileI, m.ni);
        for (int j0 = 0; j0 < m.nj; j0 += kTileJ) {
            const int j1 = std::min(j0 + kTileJ, m.nj);
            for (int pj = j0; pj < j1; pj += kPatchJ)
                for (int pi = i0; pi < i1; pi += kPatchI) {
                    m.pstart.push_back(next);
                    for (int j = pj; j < std::min(pj + kPatchJ, j1); j++)
                        for (int i = pi; i < std::min(pi + kPatchI, i1); i++) m.perm[i + m.ni * j] = next++;
                }
        }
    }
    m.pstart.push_back(next);
}

int build_mesh(dvm_mesh &m)
{
    const int ni = m.ni, nj = m.nj;
    auto node = [&](int i, int j) -> P2 {
        const double *p = &m.nodes[2 * ((size_t)j * (ni + 1) + i)];
        return {p[0], p[1]};
    };
    auto cell = [&](int i, int j) { return i + ni * j; };
    const bool cgrid = m.topo == DVM_TOPO_C;
    m.nc = ni * nj;
    m.nw = ni - 2 * m.nwake;
    m.nbr.assign((size_t)4 * m.nc, 0);
    m.S.assign((size_t)8 * m.nc, 0.0);
    m.vol.assign(m.nc, 0.0);
    m.cen.assign((size_t)2 * m.nc, 0.0);
    m.fm.assign((size_t)8 * m.nc, 0.0);
    for (int j = 0; j < nj; j++) {
        for (int i = 0; i < ni; i++) {
            const int c = cell(i, j);
            const P2 q[4] = {node(i, j), node(i + 1, j), node(i + 1, j + 1), node(i, j + 1)};
            // planar quadrilateral area = half the cross product of its diagonals
            const double d1x = q[2][0] - q[0][0], d1y = q[2][1] - q[0][1];
            const double d2x = q[3][0] - q[1][0], d2y = q[3][1] - q[1][1];
            const double area = 0.5 * (d1x * d2y - d1y * d2x);
            if (!(area > 0.0)) return fail(DVM_EINVAL, "cell (%d,%d) has non-positive area %g", i, j, area);
            m.vol[c] = area;
            // centroid: the two triangles (q0 q1 q2), (q0 q2 q3), relative to q0
            {
                const double r1x = q[1][0] - q[0][0], r1y = q[1][1] - q[0][1];
                const double r2x = q[2][0] - q[0][0], r2y = q[2][1] - q[0][1];
                const double r3x = q[3][0] - q[0][0], r3y = q[3][1] - q[0][1];
                const double a1 = r1x * r2y - r1y * r2x, a2 = r2x * r3y - r2y * r3x;
                m.cen[2 * c] = q[0][0] + (a1 * (r1x + r2x) + a2 * (r2x + r3x)) / (3.0 * (a1 + a2));
                m.cen[2 * c + 1] = q[0][1] + (a1 * (r1y + r2y) + a2 * (r2y + r3y)) / (3.0 * (a1 + a2));
            }
            for (int e = 0; e < 4; e++) {
                const P2 &s = q[e], &t = q[(e + 1) & 3];
                m.S[8 * c + 2 * e] = t[1] - s[1];       // (dy, -dx): outward for a CCW walk
                m.S[8 * c + 2 * e + 1] = s[0] - t[0];
                m.fm[8 * c + 2 * e] = 0.5 * (s[0] + t[0]);
                m.fm[8 * c + 2 * e + 1] = 0.5 * (s[1] + t[1]);
            }
            int32_t *nb = &m.nbr[4 * c];
            // face 0: j-   (wall, wake cut or interior)
            if (j > 0)
                nb[0] = cell(i, j - 1);
            else if (cgrid && (i < m.nwake || i >= ni - m.nwake))
                nb[0] = cell(ni - 1 - i, 0);
            else
                nb[0] = -2 - (i - m.nwake);
            // face 1: i+
            nb[1] = (i + 1 < ni) ? cell(i + 1, j) : (cgrid ? -1 : cell(0, j));
            // face 2: j+
            nb[2] = (j + 1 < nj) ? cell(i, j + 1) : -1;
            // face 3: i-
            nb[3] = (i > 0) ? cell(i - 1, j) : (cgrid ? -1 : cell(ni - 1, j));
        }
    }
    m.wall_cell.resize(m.nw);
    m.wA.resize(m.nw);
    m.wn.resize(2 * m.nw);
    m.wx.resize(2 * m.nw);
    m.wa.resize(2 * m.nw);
    m.wb.resize(2 * m.nw);
    for (int l = 0; l < m.nw; l++) {
        const int i = m.nwake + l;
        const int c = cell(i, 0);
        m.wall_cell[l] = c;
        const P2 a = node(i, 0), b = node(i + 1, 0);
        const double sx = m.S[8 * c], sy = m.S[8 * c + 1];
        const double A = std::sqrt(sx * sx + sy * sy);
        m.wA[l] = A;
        m.wn[2 * l] = sx / A;
        m.wn[2 * l + 1] = sy / A;
        m.wa[2 * l] = a[0];
        m.wa[2 * l + 1] = a[1];
        m.wb[2 * l] = b[0];
        m.wb[2 * l + 1] = b[1];
        m.wx[2 * l] = 0.5 * (a[0] + b[0]);
        m.wx[2 * l + 1] = 0.5 * (a[1] + b[1]);
    }
    build_patches(m);
    return DVM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// velocity grid
// ---------------------------------------------------------------------------
struct dvm_vgrid {
    int kind = 0, n1 = 0, n2 = 0;
    double vmax = 0, param = 0;
    std::vector<double> x1, w1, x2, w2;
};

namespace {

int rule_1d(int kind, int n, double vmax, double param, std::vector<double> &x, std::vector<double> &w)
{
    if (n < 2 || n > dvm::kMaxN1D) return fail(DVM_EINVAL, "velocity nodes per direction must be in [2, %d]", dvm::kMaxN1D);
    if (!(vmax > 0)) return fail(DVM_EINVAL, "vmax must be positive");
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    switch (kind) {
    case DVM_VG_MIDPOINT: {
        const double h = 2.0 * vmax / n;
        for (int a = 0; a < n; a++) {
            x[a] = -vmax + (a + 0.5) * h;
            w[a] = h;
        }
        return DVM_OK;
    }
    case DVM_VG_NEWTON_COTES: {
        if (n % 4) return fail(DVM_EINVAL, "Newton-Cotes grid needs n divisible by 4 (got %d)", n);
        const int m = n - 1;                  // intervals
        const double h = 2.0 * vmax / m;
        for (int a = 0; a < n; a++) x[a] = -vmax + a * h;
        const int left = (m - 3) / 2;         // Simpson intervals left of the 3/8 panel
        auto simpson = [&](int from, int to) {
            for (int p = from; p < to; p += 2) {
                w[p] += h / 3.0;
                w[p + 1] += 4.0 * h / 3.0;
                w[p + 2] += h / 3.0;
            }
        };
        simpson(0, left);
        const double e = 3.0 * h / 8.0;
        const double mid[4] = {e, 3.0 * e, 3.0 * e, e};
        for (int t = 0; t < 4; t++) w[left + t] += mid[t];
        simpson(left + 3, m);
        return DVM_OK;
    }
    case DVM_VG_SINH: {
        const double p = param > 0 ? param : 2.0;
        const double sp = std::sinh(p);
        auto map = [&](double s) { return vmax * std::sinh(p * s) / sp; };
        for (int a = 0; a < n; a++) {
            const double s0 = -1.0 + a * 2.0 / n, s1 = -1.0 + (a + 1) * 2.0 / n;
            x[a] = map(-1.0 + (a + 0.5) * 2.0 / n);
            w[a] = map(s1) - map(s0);
        }
        return DVM_OK;
    }
    default:
        return fail(DVM_EINVAL, "unknown velocity grid kind %d", kind);
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------
struct dvm_solver {
    // problem
    int topo, ni, nj, nc, nw, np, n1, n2, nv, mixed, want_adjoint, objective;
    // mesh in device numbering (cell c of the mesh is device cell perm[c],
    // device cell d is mesh cell cell_of[d])
    std::vector<int32_t> nbr, wall_cell, perm, cell_of, pstart;
    std::vector<double> S, vol, wA, wn, wa, wb, D;
    std::vector<double> rf, rn;   // [nc][4][2] face midpoint - own / neighbour centroid (order 2)
    std::vector<double> x1, w1, x2, w2;
    std::vector<double> fd;   // [nv][2]
    std::vector<double> gM;   // [nv]
    std::vector<double> gw2;  // [nv][2]
    double inv_tau_inf, u_inf, theta_w, cd_scale;
    // spatial scheme: order 1, or 2 with limiter and K sweeps between corrections
    int order = 1, limiter = DVM_LIMITER_VENKAT, kcorr = 40;
    int equil = DVM_EQ_POINTWISE;
    // macroscopic prediction every acc_every primal sweeps (0: off) with
    // acc_inner red-black steps; acc_count = primal sweeps since the state began
    int acc_every = 0, acc_inner = 0, acc_count = 0, acc_acount = 0;
    // workspace
    struct {
        size_t nbr, patch, cell_of, S, vol, wall_cell, wA, wn, wa, wb, D, vx, vy, wx, wy, fd, gM, gw2;
        size_t f[2], W[2], F[2], red, phi[2], aW[2], Phi[2], acoef, Jl, sens, dJdn, jac, dJda, msens, dJdx, out;
        size_t mstate, mr, mDinv, mO, mx[2];
        size_t rf, rn, G, corr, psi, dF, total;
    } off;
    char *base = nullptr;
    hipStream_t stream = nullptr;
    dvm::DevSolve dev{};
    // state
    int phase = -1;   // -1 none, 0 primal, 1 adjoint
    int fpar = 0, ppar = 0, frozen_fpar = 0;
    int iters[2] = {0, 0};
    int in_batch = 0;
    // order 2: is a held correction valid, and sweeps since it was evaluated
    int corr_ok[2] = {0, 0}, since[2] = {0, 0};
};

namespace {

size_t elt_bytes(const dvm_solver &s) { return s.mixed ? sizeof(float) : sizeof(double); }

void layout(dvm_solver &s)
{
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        const size_t o = cur;
        cur = align_up(cur + bytes);
        return o;
    };
    const size_t nc = s.nc, nw = s.nw, nv = s.nv, e = elt_bytes(s);
    auto &o = s.off;
    o.nbr = take(4 * nc * sizeof(int32_t));
    o.patch = take((s.np + 1) * sizeof(int32_t));
    o.cell_of = take(nc * sizeof(int32_t));
    o.S = take(8 * nc * sizeof(double));
    o.vol = take(nc * sizeof(double));
    o.wall_cell = take(nw * sizeof(int32_t));
    o.wA = take(nw * sizeof(double));
    o.wn = take(2 * nw * sizeof(double));
    o.wa = take(2 * nw * sizeof(double));
    o.wb = take(2 * nw * sizeof(double));
    o.D = take(nw * sizeof(double));
    o.vx = take(s.n1 * sizeof(double));
    o.vy = take(s.n2 * sizeof(double));
    o.wx = take(s.n1 * sizeof(double));
    o.wy = take(s.n2 * sizeof(double));
    o.fd = take(2 * nv * e);
    o.gM = take(nv * e);
    o.gw2 = take(2 * nv * e);
    for (int p = 0; p < 2; p++) {
        o.f[p] = take(2 * nc * nv * e);
        o.W[p] = take(4 * nc * sizeof(double));
        o.F[p] = take(nw * sizeof(double));
    }
    o.red = take(2 * nc * sizeof(double));
    if (s.want_adjoint) {
        for (int p = 0; p < 2; p++) {
            o.phi[p] = take(2 * nc * nv * e);
            o.aW[p] = take(8 * nc * sizeof(double));
            o.Phi[p] = take(nw * sizeof(double));
        }
        o.acoef = take(dvm::kAcoef * nc * sizeof(double));
        o.sens = take(5 * nw * sizeof(double));
        o.dJdn = take(2 * nw * sizeof(double));
        o.jac = take(2 * nw * dvm::kMaxParams * sizeof(double));
        o.dJda = take(dvm::kMaxParams * sizeof(double));
        o.msens = take(8 * nc * sizeof(double));
        o.dJdx = take(2 * (size_t)(s.ni + 1) * (s.nj + 1) * sizeof(double));
    } else {
        o.phi[0] = o.phi[1] = o.aW[0] = o.aW[1] = o.Phi[0] = o.Phi[1] = o.acoef = o.sens = o.dJdn = o.jac =
            o.dJda = o.msens = o.dJdx = (size_t)-1;
    }
    o.Jl = take(nw * sizeof(double));
    o.out = take(16 * sizeof(double));
    if (s.order == 2) {
        o.rf = take(8 * nc * sizeof(double));
        o.rn = take(8 * nc * sizeof(double));
        o.G = take(4 * nc * nv * e);
        o.corr = take(2 * nc * nv * e);
        o.dF = take(nw * sizeof(double));
        o.psi = s.want_adjoint ? take(2 * nc * nv * e) : (size_t)-1;
    } else {
        o.rf = o.rn = o.G = o.corr = o.dF = o.psi = (size_t)-1;
    }
    o.mstate = s.equil == DVM_EQ_CONSERVATIVE ? take(dvm::kEqState * nc * sizeof(double)) : (size_t)-1;
    if (s.acc_every > 0) {
        o.mr = take(4 * nc * sizeof(double));
        o.mDinv = take(16 * nc * sizeof(double));
        o.mO = take(64 * nc * sizeof(double));
        o.mx[0] = take(4 * nc * sizeof(double));
        o.mx[1] = take(4 * nc * sizeof(double));
    } else {
        o.mr = o.mDinv = o.mO = o.mx[0] = o.mx[1] = (size_t)-1;
    }
    o.total = cur;
}

template <typename P>
P *at(const dvm_solver &s, size_t off)
{
    return off == (size_t)-1 ? nullptr : reinterpret_cast<P *>(s.base + off);
}

void fill_dev(dvm_solver &s)
{
    dvm::DevSolve &d = s.dev;
    d.nc = s.nc;
    d.nw = s.nw;
    d.nv = s.nv;
    d.n1 = s.n1;
    d.n2 = s.n2;
    d.np = s.np;
    d.ni = s.ni;
    d.nj = s.nj;
    d.topo = s.topo;
    d.objective = s.objective;
    d.mixed = s.mixed;
    d.order = s.order;
    d.limiter = s.limiter;
    d.equil = s.equil;
    d.nbr = at<int32_t>(s, s.off.nbr);
    d.patch = at<int32_t>(s, s.off.patch);
    d.cell_of = at<int32_t>(s, s.off.cell_of);
    d.S = at<double>(s, s.off.S);
    d.vol = at<double>(s, s.off.vol);
    d.wall_cell = at<int32_t>(s, s.off.wall_cell);
    d.wall_A = at<double>(s, s.off.wA);
    d.wall_n = at<double>(s, s.off.wn);
    d.wall_a = at<double>(s, s.off.wa);
    d.wall_b = at<double>(s, s.off.wb);
    d.D = at<double>(s, s.off.D);
    d.vx = at<double>(s, s.off.vx);
    d.vy = at<double>(s, s.off.vy);
    d.wx = at<double>(s, s.off.wx);
    d.wy = at<double>(s, s.off.wy);
    d.fd = at<void>(s, s.off.fd);
    d.gM = at<void>(s, s.off.gM);
    d.gw2 = at<void>(s, s.off.gw2);
    d.inv_tau_inf = s.inv_tau_inf;
    d.u_inf = s.u_inf;
    d.theta_w = s.theta_w;
    d.cd_scale = s.cd_scale;
    for (int p = 0; p < 2; p++) {
        d.f[p] = at<void>(s, s.off.f[p]);
        d.W[p] = at<double>(s, s.off.W[p]);
        d.F[p] = at<double>(s, s.off.F[p]);
        d.phi[p] = at<void>(s, s.off.phi[p]);
        d.aW[p] = at<double>(s, s.off.aW[p]);
        d.Phi[p] = at<double>(s, s.off.Phi[p]);
    }
    d.red = at<double>(s, s.off.red);
    d.fstar = d.f[s.frozen_fpar];
    d.acoef = at<double>(s, s.off.acoef);
    d.Jl = at<double>(s, s.off.Jl);
    d.sens = at<double>(s, s.off.sens);
    d.dJdn = at<double>(s, s.off.dJdn);
    d.jac = at<double>(s, s.off.jac);
    d.dJda = at<double>(s, s.off.dJda);
    d.msens = at<double>(s, s.off.msens);
    d.dJdx = at<double>(s, s.off.dJdx);
    d.out = at<double>(s, s.off.out);
    d.rf = at<double>(s, s.off.rf);
    d.rn = at<double>(s, s.off.rn);
    d.G = at<void>(s, s.off.G);
    d.corr = at<void>(s, s.off.corr);
    d.psi = at<void>(s, s.off.psi);
    d.dF = at<double>(s, s.off.dF);
    d.mstate = at<double>(s, s.off.mstate);
    d.mr = at<double>(s, s.off.mr);
    d.mDinv = at<double>(s, s.off.mDinv);
    d.mO = at<double>(s, s.off.mO);
    d.mx[0] = at<double>(s, s.off.mx[0]);
    d.mx[1] = at<double>(s, s.off.mx[1]);
}

int upload(dvm_solver &s, size_t off, const void *src, size_t bytes)
{
    HIP_OK(hipMemcpyAsync(s.base + off, src, bytes, hipMemcpyHostToDevice, s.stream));
    return DVM_OK;
}

int read_back(dvm_solver &s, const double *dev_src, double *dst, size_t n)
{
    HIP_OK(hipMemcpyAsync(dst, dev_src, n * sizeof(double), hipMemcpyDeviceToHost, s.stream));
    HIP_OK(hipStreamSynchronize(s.stream));
    return DVM_OK;
}

// Per-cell rows of `bytes` bytes between device numbering and mesh numbering.
void rows_to_mesh(const dvm_solver &s, const char *dev_rows, char *mesh_rows, size_t bytes)
{
    for (int c = 0; c < s.nc; c++) std::memcpy(mesh_rows + (size_t)c * bytes, dev_rows + (size_t)s.perm[c] * bytes, bytes);
}

void rows_to_dev(const dvm_solver &s, const char *mesh_rows, char *dev_rows, size_t bytes)
{
    for (int c = 0; c < s.nc; c++) std::memcpy(dev_rows + (size_t)s.perm[c] * bytes, mesh_rows + (size_t)c * bytes, bytes);
}

double rel_norm(double num, double den)
{
    if (!(den > 0)) return num == 0 ? 0.0 : INFINITY;
    return std::sqrt(num / den);
}

int read_residual(dvm_solver &s, int adjoint, double *r)
{
    HIP_OK(dvm::launch_residual(s.dev, adjoint, s.stream));
    double v[2];
    if (int e = read_back(s, s.dev.out + (adjoint ? 4 : 2), v, 2)) return e;
    *r = rel_norm(v[0], v[1]);
    return DVM_OK;
}

int check_bound(const dvm_solver *s)
{
    if (!s) return fail(DVM_EINVAL, "null solver");
    if (!s->base) return fail(DVM_ESTATE, "solver is not bound to a device buffer");
    if (s->in_batch) return fail(DVM_ESTATE, "solver is a member of a live batch");
    return DVM_OK;
}

// Order 2 (defect correction): before a sweep, re-evaluate the held
// correction from the current state when there is none or K sweeps have
// used it.
int sweeps(dvm_solver &s, int adjoint, int n)
{
    for (int i = 0; i < n; i++) {
        if (s.order == 2 && (!s.corr_ok[adjoint] || s.since[adjoint] == s.kcorr)) {
            if (adjoint)
                HIP_OK(dvm::launch_so_adjoint_term(s.dev, s.ppar, s.stream));
            else
                HIP_OK(dvm::launch_so_correction(s.dev, s.fpar, s.stream));
            s.corr_ok[adjoint] = 1;
            s.since[adjoint] = 0;
        }
        if (adjoint) {
            HIP_OK(dvm::launch_adjoint_sweep(s.dev, s.ppar, s.stream));
            s.ppar ^= 1;
            if (s.acc_every > 0 && ++s.acc_acount % s.acc_every == 0)
                HIP_OK(dvm::launch_macro_adjoint_predict(s.dev, s.ppar, s.acc_inner, s.stream));
        } else {
            if (s.equil == DVM_EQ_CONSERVATIVE) {
                if (!s.dev.mstate) return fail(DVM_ESTATE, "no equilibrium parameter buffer");
                HIP_OK(dvm::launch_eq_params(s.dev, s.fpar, 0, s.stream));
            }
            HIP_OK(dvm::launch_primal_sweep(s.dev, s.fpar, s.stream));
            s.fpar ^= 1;
            if (s.acc_every > 0 && ++s.acc_count % s.acc_every == 0)
                HIP_OK(dvm::launch_macro_predict(s.dev, s.fpar, s.acc_inner, s.stream));
        }
        s.since[adjoint]++;
    }
    s.iters[adjoint] += n;
    return DVM_OK;
}

int iterate(dvm_solver &s, int adjoint, int max_iter, double tol, int check_every, int *iters, double *resid)
{
    if (max_iter < 0) return fail(DVM_EINVAL, "max_iter < 0");
    if (check_every <= 0) check_every = max_iter > 0 ? max_iter : 1;
    int done = 0;
    double r = NAN;
    while (done < max_iter) {
        const int m = std::min(check_every, max_iter - done);
        if (int e = sweeps(s, adjoint, m)) return e;
        done += m;
        if (tol > 0 || done == max_iter) {
            if (int e = read_residual(s, adjoint, &r)) return e;
            if (!std::isfinite(r)) {
                if (iters) *iters = done;
                if (resid) *resid = r;
                return fail(DVM_ENAN, "%s residual is not finite after %d sweeps", adjoint ? "adjoint" : "primal",
                            done);
            }
            if (tol > 0 && r < tol) break;
        }
    }
    if (iters) *iters = done;
    if (resid) *resid = r;
    if (tol > 0 && !(r < tol))
        return fail(DVM_ENOTCONV, "%s residual %.3e above tolerance %.3e after %d sweeps",
                    adjoint ? "adjoint" : "primal", r, tol, done);
    return DVM_OK;
}

int setup_flow(dvm_solver &s, const dvm_flow &fl)
{
    if (!(fl.Tw > 0) || !(fl.Ma >= 0) || !(fl.Kn > 0) || std::isnan(fl.Kn))
        return fail(DVM_EINVAL, "flow state needs Kn > 0, Ma >= 0, Tw > 0");
    if (fl.objective != DVM_OBJ_DRAG && fl.objective != DVM_OBJ_HEAT) return fail(DVM_EINVAL, "unknown objective");
    const double th_inf = 0.5;                        // theta = RT, velocity unit sqrt(2 R T_inf)
    s.theta_w = th_inf * fl.Tw;
    s.u_inf = fl.Ma * std::sqrt(5.0 / 3.0 * th_inf);  // gamma = 5/3
    // Kn = (16/5) (tau / l_ref) sqrt(RT / (2 pi)), l_ref = 1, theta_inf = 1/2
    s.inv_tau_inf = std::isinf(fl.Kn) ? 0.0 : 1.0 / (0.625 * std::sqrt(kPi) * fl.Kn);
    s.cd_scale = 0.5 * s.u_inf * s.u_inf * (s.topo == DVM_TOPO_O ? 2.0 : 1.0);
    s.objective = fl.objective;
    s.fd.resize(2 * s.nv);
    s.gM.resize(s.nv);
    s.gw2.resize(2 * s.nv);
    for (int b = 0; b < s.n2; b++) {
        for (int a = 0; a < s.n1; a++) {
            const int k = a + s.n1 * b;
            const double c1 = s.x1[a] - s.u_inf, c2 = s.x2[b];
            const double g = std::exp(-(c1 * c1 + c2 * c2) / (2.0 * th_inf)) / (2.0 * kPi * th_inf);
            s.fd[2 * k] = g;
            s.fd[2 * k + 1] = 0.5 * th_inf * g;
            const double r2 = s.x1[a] * s.x1[a] + s.x2[b] * s.x2[b];
            s.gM[k] = std::exp(-r2 / (2.0 * s.theta_w)) / (2.0 * kPi * s.theta_w);
            s.gw2[2 * k] = s.gM[k];
            s.gw2[2 * k + 1] = 0.5 * s.theta_w * s.gM[k];
        }
    }
    // eq. (barg): D_l = -sum_{v.n <= 0} w (v.n) g_M1(1, 0, T_w)
    s.D.assign(s.nw, 0.0);
    for (int l = 0; l < s.nw; l++) {
        double acc = 0;
        for (int b = 0; b < s.n2; b++)
            for (int a = 0; a < s.n1; a++) {
                const double vn = s.x1[a] * s.wn[2 * l] + s.x2[b] * s.wn[2 * l + 1];
                if (vn <= 0) acc -= s.w1[a] * s.w2[b] * vn * s.gM[a + s.n1 * b];
            }
        if (!(acc > 0)) return fail(DVM_EINVAL, "wall element %d has no incoming velocities", l);
        s.D[l] = acc;
    }
    return DVM_OK;
}

template <typename T>
std::vector<T> convert(const std::vector<double> &v)
{
    return std::vector<T>(v.begin(), v.end());
}

}  // namespace

// ---------------------------------------------------------------------------
// batch
// ---------------------------------------------------------------------------
struct dvm_batch {
    std::vector<dvm_solver *> owned;     // member list of a dvm_batch_create batch
    dvm_solver *fixed[dvm::kStaticBatchMaxMembers] = {};   // member list of an allocation-free batch
    dvm_solver **members = nullptr;
    int n = 0;
    int static_dev = -1;                 // >= 0: the allocation-free batch of this device
    char *work = nullptr;
    hipStream_t stream = nullptr;
    int nblocks = 0, mixed = 0;
    int nb_group[4] = {0, 0, 0, 0};      // blocks of group 2 * phase + (order == 2), in that order
    int step = 0;
    size_t off_tab = 0, off_par = 0, off_phase = 0, off_bs = 0, off_bc = 0, off_out = 0;
};

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace dvm {

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

MeshNodes mesh_nodes(const dvm_mesh *m)
{
    return {m->topo, m->ni, m->nj, m->nwake, m->nw, m->nodes.data()};
}

}  // namespace dvm

extern "C" {

const char *dvm_last_error(void) { return g_err.c_str(); }

int dvm_mesh_create(int topology, int ni, int nj, int n_wake, const double *nodes_xy, dvm_mesh **out)
{
    if (!out || !nodes_xy) return fail(DVM_EINVAL, "null argument");
    *out = nullptr;
    if (topology != DVM_TOPO_O && topology != DVM_TOPO_C) return fail(DVM_EINVAL, "unknown topology %d", topology);
    if (ni < 3 || nj < 1) return fail(DVM_EINVAL, "grid too small (ni=%d, nj=%d)", ni, nj);
    if (topology == DVM_TOPO_O && n_wake != 0) return fail(DVM_EINVAL, "O-grid takes n_wake = 0");
    if (topology == DVM_TOPO_C && (n_wake < 1 || 2 * n_wake >= ni - 1))
        return fail(DVM_EINVAL, "C-grid needs 1 <= n_wake and 2 n_wake < ni - 1");
    if ((int64_t)ni * nj > (int64_t)1 << 30) return fail(DVM_EINVAL, "grid too large");
    try {
        auto *m = new dvm_mesh;
        m->topo = topology;
        m->ni = ni;
        m->nj = nj;
        m->nwake = n_wake;
        m->nodes.assign(nodes_xy, nodes_xy + 2 * (size_t)(ni + 1) * (nj + 1));
        if (int e = build_mesh(*m)) {
            delete m;
            return e;
        }
        *out = m;
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return fail(DVM_ENOMEM, "out of host memory");
    }
}

int dvm_mesh_info(const dvm_mesh *m, int32_t *n_cells, int32_t *n_wall)
{
    if (!m) return fail(DVM_EINVAL, "null mesh");
    if (n_cells) *n_cells = m->nc;
    if (n_wall) *n_wall = m->nw;
    return DVM_OK;
}

int dvm_mesh_export(const dvm_mesh *m, int32_t *nbr, int32_t *wall_cell, double *S, double *vol, double *wall_A,
                    double *wall_n, double *wall_x)
{
    if (!m) return fail(DVM_EINVAL, "null mesh");
    if (nbr) std::copy(m->nbr.begin(), m->nbr.end(), nbr);
    if (wall_cell) std::copy(m->wall_cell.begin(), m->wall_cell.end(), wall_cell);
    if (S) std::copy(m->S.begin(), m->S.end(), S);
    if (vol) std::copy(m->vol.begin(), m->vol.end(), vol);
    if (wall_A) std::copy(m->wA.begin(), m->wA.end(), wall_A);
    if (wall_n) std::copy(m->wn.begin(), m->wn.end(), wall_n);
    if (wall_x) std::copy(m->wx.begin(), m->wx.end(), wall_x);
    return DVM_OK;
}

void dvm_mesh_destroy(dvm_mesh *m) { delete m; }

int dvm_vgrid_create(int kind, int n1, int n2, double vmax, double param, dvm_vgrid **out)
{
    if (!out) return fail(DVM_EINVAL, "null argument");
    *out = nullptr;
    try {
        auto *g = new dvm_vgrid;
        g->kind = kind;
        g->n1 = n1;
        g->n2 = n2;
        g->vmax = vmax;
        g->param = param;
        if (int e = rule_1d(kind, n1, vmax, param, g->x1, g->w1)) {
            delete g;
            return e;
        }
        if (int e = rule_1d(kind, n2, vmax, param, g->x2, g->w2)) {
            delete g;
            return e;
        }
        *out = g;
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return fail(DVM_ENOMEM, "out of host memory");
    }
}

int dvm_vgrid_info(const dvm_vgrid *g, int32_t *nv)
{
    if (!g) return fail(DVM_EINVAL, "null velocity grid");
    if (nv) *nv = g->n1 * g->n2;
    return DVM_OK;
}

int dvm_vgrid_export(const dvm_vgrid *g, double *v, double *w)
{
    if (!g) return fail(DVM_EINVAL, "null velocity grid");
    for (int b = 0; b < g->n2; b++)
        for (int a = 0; a < g->n1; a++) {
            const int k = a + g->n1 * b;
            if (v) {
                v[2 * k] = g->x1[a];
                v[2 * k + 1] = g->x2[b];
            }
            if (w) w[k] = g->w1[a] * g->w2[b];
        }
    return DVM_OK;
}

void dvm_vgrid_destroy(dvm_vgrid *g) { delete g; }

int dvm_solver_create(const dvm_mesh *m, const dvm_vgrid *g, const dvm_flow *flow, int precision, int want_adjoint,
                      dvm_solver **out)
{
    if (!out || !m || !g || !flow) return fail(DVM_EINVAL, "null argument");
    *out = nullptr;
    if (precision != DVM_FP64 && precision != DVM_MIXED) return fail(DVM_EINVAL, "unknown precision %d", precision);
    try {
        auto *s = new dvm_solver;
        s->topo = m->topo;
        s->nc = m->nc;
        s->nw = m->nw;
        s->n1 = g->n1;
        s->n2 = g->n2;
        s->nv = g->n1 * g->n2;
        s->mixed = precision == DVM_MIXED;
        s->want_adjoint = want_adjoint ? 1 : 0;
        s->np = (int)m->pstart.size() - 1;
        s->ni = m->ni;
        s->nj = m->nj;
        s->perm = m->perm;
        s->cell_of.resize(m->nc);
        for (int c = 0; c < m->nc; c++) s->cell_of[m->perm[c]] = c;
        s->pstart = m->pstart;
        s->nbr.resize(m->nbr.size());
        s->S.resize(m->S.size());
        s->vol.resize(m->vol.size());
        for (int c = 0; c < m->nc; c++) {
            const int32_t dc = m->perm[c];
            for (int q = 0; q < 4; q++) {
                const int32_t n = m->nbr[4 * c + q];
                s->nbr[4 * dc + q] = n >= 0 ? m->perm[n] : n;
            }
            for (int e = 0; e < 8; e++) s->S[8 * dc + e] = m->S[8 * c + e];
            s->vol[dc] = m->vol[c];
        }
        s->rf.assign((size_t)8 * m->nc, 0.0);
        s->rn.assign((size_t)8 * m->nc, 0.0);
        for (int c = 0; c < m->nc; c++) {
            const int32_t dc = m->perm[c];
            for (int q = 0; q < 4; q++)
                for (int x = 0; x < 2; x++) {
                    const double mid = m->fm[8 * c + 2 * q + x];
                    const int32_t n = m->nbr[4 * c + q];
                    s->rf[8 * dc + 2 * q + x] = mid - m->cen[2 * c + x];
                    if (n >= 0) s->rn[8 * dc + 2 * q + x] = mid - m->cen[2 * n + x];
                }
        }
        s->wall_cell.resize(m->nw);
        for (int l = 0; l < m->nw; l++) s->wall_cell[l] = m->perm[m->wall_cell[l]];
        s->wA = m->wA;
        s->wn = m->wn;
        s->wa = m->wa;
        s->wb = m->wb;
        s->x1 = g->x1;
        s->w1 = g->w1;
        s->x2 = g->x2;
        s->w2 = g->w2;
        if (int e = setup_flow(*s, *flow)) {
            delete s;
            return e;
        }
        layout(*s);
        *out = s;
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return fail(DVM_ENOMEM, "out of host memory");
    }
}

size_t dvm_solver_workspace_bytes(const dvm_solver *s) { return s ? s->off.total : 0; }

int dvm_solver_set_scheme(dvm_solver *s, int order, int limiter, int correction_interval)
{
    if (!s) return fail(DVM_EINVAL, "null solver");
    if (s->base) return fail(DVM_ESTATE, "the scheme is set before dvm_solver_bind");
    if (order != 1 && order != 2) return fail(DVM_EINVAL, "order must be 1 or 2 (got %d)", order);
    if (limiter != DVM_LIMITER_NONE && limiter != DVM_LIMITER_VENKAT) return fail(DVM_EINVAL, "unknown limiter %d", limiter);
    if (correction_interval < 1) return fail(DVM_EINVAL, "correction interval must be >= 1");
    if (order == 2 && s->acc_every > 0) return fail(DVM_EINVAL, "the macroscopic prediction is first-order only");
    s->order = order;
    s->limiter = limiter;
    s->kcorr = correction_interval;
    layout(*s);
    return DVM_OK;
}

int dvm_solver_set_equilibrium(dvm_solver *s, int kind)
{
    if (!s) return fail(DVM_EINVAL, "null solver");
    if (s->base) return fail(DVM_ESTATE, "the equilibrium is set before dvm_solver_bind");
    if (kind != DVM_EQ_POINTWISE && kind != DVM_EQ_CONSERVATIVE) return fail(DVM_EINVAL, "unknown equilibrium %d", kind);
    if (kind != DVM_EQ_CONSERVATIVE && s->acc_every > 0)
        return fail(DVM_EINVAL, "the macroscopic prediction needs the conservative equilibrium");
    s->equil = kind;
    layout(*s);             // the conservative equilibrium keeps its parameters per cell
    return DVM_OK;
}

int dvm_solver_set_acceleration(dvm_solver *s, int every, int inner)
{
    if (!s) return fail(DVM_EINVAL, "null solver");
    if (s->base) return fail(DVM_ESTATE, "the acceleration is set before dvm_solver_bind");
    if (every < 0 || inner < 0 || inner > 100000) return fail(DVM_EINVAL, "every >= 0 and 0 <= inner <= 100000");
    if (every > 0 && s->order != 1) return fail(DVM_EINVAL, "the macroscopic prediction is first-order only");
    if (every > 0 && s->equil != DVM_EQ_CONSERVATIVE)
        return fail(DVM_EINVAL, "the macroscopic prediction needs the conservative equilibrium");
    s->acc_every = every;
    s->acc_inner = inner;
    layout(*s);
    return DVM_OK;
}

int dvm_solver_bind(dvm_solver *s, void *dev_ptr, size_t bytes, void *hip_stream)
{
    if (!s || !dev_ptr) return fail(DVM_EINVAL, "null argument");
    if (s->in_batch) return fail(DVM_ESTATE, "solver is a member of a live batch");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % kAlign) return fail(DVM_EINVAL, "device buffer not 256-byte aligned");
    if (bytes < s->off.total)
        return fail(DVM_ENOMEM, "device buffer of %zu bytes < workspace %zu bytes", bytes, s->off.total);
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dev_ptr) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(DVM_EINVAL, "buffer is not device memory");
    }
    s->base = static_cast<char *>(dev_ptr);
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->phase = -1;
    s->fpar = s->ppar = s->frozen_fpar = 0;
    s->iters[0] = s->iters[1] = 0;
    s->corr_ok[0] = s->corr_ok[1] = 0;
    fill_dev(*s);
    const auto &o = s->off;
    int e = 0;
    e = e ? e : upload(*s, o.nbr, s->nbr.data(), s->nbr.size() * sizeof(int32_t));
    e = e ? e : upload(*s, o.patch, s->pstart.data(), s->pstart.size() * sizeof(int32_t));
    e = e ? e : upload(*s, o.cell_of, s->cell_of.data(), s->cell_of.size() * sizeof(int32_t));
    e = e ? e : upload(*s, o.S, s->S.data(), s->S.size() * sizeof(double));
    e = e ? e : upload(*s, o.vol, s->vol.data(), s->vol.size() * sizeof(double));
    e = e ? e : upload(*s, o.wall_cell, s->wall_cell.data(), s->wall_cell.size() * sizeof(int32_t));
    e = e ? e : upload(*s, o.wA, s->wA.data(), s->wA.size() * sizeof(double));
    e = e ? e : upload(*s, o.wn, s->wn.data(), s->wn.size() * sizeof(double));
    e = e ? e : upload(*s, o.wa, s->wa.data(), s->wa.size() * sizeof(double));
    e = e ? e : upload(*s, o.wb, s->wb.data(), s->wb.size() * sizeof(double));
    e = e ? e : upload(*s, o.D, s->D.data(), s->D.size() * sizeof(double));
    e = e ? e : upload(*s, o.vx, s->x1.data(), s->x1.size() * sizeof(double));
    e = e ? e : upload(*s, o.vy, s->x2.data(), s->x2.size() * sizeof(double));
    e = e ? e : upload(*s, o.wx, s->w1.data(), s->w1.size() * sizeof(double));
    e = e ? e : upload(*s, o.wy, s->w2.data(), s->w2.size() * sizeof(double));
    if (s->order == 2) {
        e = e ? e : upload(*s, o.rf, s->rf.data(), s->rf.size() * sizeof(double));
        e = e ? e : upload(*s, o.rn, s->rn.data(), s->rn.size() * sizeof(double));
    }
    std::vector<float> fdf, gMf, gw2f;
    if (s->mixed) {
        fdf = convert<float>(s->fd);
        gMf = convert<float>(s->gM);
        gw2f = convert<float>(s->gw2);
        e = e ? e : upload(*s, o.fd, fdf.data(), fdf.size() * sizeof(float));
        e = e ? e : upload(*s, o.gM, gMf.data(), gMf.size() * sizeof(float));
        e = e ? e : upload(*s, o.gw2, gw2f.data(), gw2f.size() * sizeof(float));
    } else {
        e = e ? e : upload(*s, o.fd, s->fd.data(), s->fd.size() * sizeof(double));
        e = e ? e : upload(*s, o.gM, s->gM.data(), s->gM.size() * sizeof(double));
        e = e ? e : upload(*s, o.gw2, s->gw2.data(), s->gw2.size() * sizeof(double));
    }
    if (e) {
        s->base = nullptr;
        return e;
    }
    HIP_OK(hipStreamSynchronize(s->stream));
    return DVM_OK;
}

int dvm_solver_set_stream(dvm_solver *s, void *hip_stream)
{
    if (!s) return fail(DVM_EINVAL, "null solver");
    s->stream = static_cast<hipStream_t>(hip_stream);
    return DVM_OK;
}

int dvm_primal_init(dvm_solver *s)
{
    if (int e = check_bound(s)) return e;
    HIP_OK(dvm::launch_primal_init(s->dev, s->stream));
    s->fpar = 0;
    s->acc_count = 0;
    s->phase = 0;
    s->iters[0] = s->iters[1] = 0;
    s->corr_ok[0] = 0;
    return DVM_OK;
}

int dvm_primal_iterate(dvm_solver *s, int max_iter, double tol, int check_every, int *iters, double *resid)
{
    if (int e = check_bound(s)) return e;
    if (s->phase != 0) return fail(DVM_ESTATE, "no primal phase (call dvm_primal_init)");
    return iterate(*s, 0, max_iter, tol, check_every, iters, resid);
}

int dvm_primal_sweeps(dvm_solver *s, int n)
{
    if (int e = check_bound(s)) return e;
    if (s->phase != 0) return fail(DVM_ESTATE, "no primal phase (call dvm_primal_init)");
    if (n < 0) return fail(DVM_EINVAL, "n < 0");
    return sweeps(*s, 0, n);
}

int dvm_objective(dvm_solver *s, double *J, double *Cd)
{
    if (int e = check_bound(s)) return e;
    if (s->phase < 0) return fail(DVM_ESTATE, "no primal state");
    const int par = s->phase == 1 ? s->frozen_fpar : s->fpar;
    HIP_OK(dvm::launch_objective(s->dev, par, s->stream));
    double v[2];
    if (int e = read_back(*s, s->dev.out, v, 2)) return e;
    if (J) *J = v[0];
    if (Cd) *Cd = v[1];
    return DVM_OK;
}

int dvm_read_moments(dvm_solver *s, double *W)
{
    if (int e = check_bound(s)) return e;
    if (s->phase < 0) return fail(DVM_ESTATE, "no primal state");
    if (!W) return fail(DVM_EINVAL, "null output");
    const int par = s->phase == 1 ? s->frozen_fpar : s->fpar;
    try {
        std::vector<double> dev((size_t)4 * s->nc);
        if (int e = read_back(*s, s->dev.W[par], dev.data(), dev.size())) return e;
        rows_to_mesh(*s, reinterpret_cast<const char *>(dev.data()), reinterpret_cast<char *>(W), 4 * sizeof(double));
    } catch (const std::bad_alloc &) {
        return fail(DVM_ENOMEM, "out of host memory");
    }
    return DVM_OK;
}

int dvm_adjoint_init(dvm_solver *s)
{
    if (int e = check_bound(s)) return e;
    if (!s->want_adjoint) return fail(DVM_ESTATE, "solver was created without adjoint buffers");
    if (s->phase < 0) return fail(DVM_ESTATE, "no primal state to linearise about");
    if (s->phase == 0) s->frozen_fpar = s->fpar;
    fill_dev(*s);
    // a primal prediction may have left the predicted moments in W for the
    // next sweep: the adjoint is taken at the moments of f
    if (s->acc_every > 0) HIP_OK(dvm::launch_moments(s->dev, s->frozen_fpar, s->stream));
    HIP_OK(dvm::launch_adjoint_init(s->dev, s->frozen_fpar, s->stream));
    if (s->order == 2) HIP_OK(dvm::launch_so_freeze(s->dev, s->frozen_fpar, s->stream));
    if (s->acc_every > 0) HIP_OK(dvm::launch_macro_adjoint_setup(s->dev, s->frozen_fpar, s->stream));
    s->acc_acount = 0;
    s->ppar = 0;
    s->phase = 1;
    s->iters[1] = 0;
    s->corr_ok[1] = 0;
    return DVM_OK;
}

int dvm_adjoint_iterate(dvm_solver *s, int max_iter, double tol, int check_every, int *iters, double *resid)
{
    if (int e = check_bound(s)) return e;
    if (s->phase != 1) return fail(DVM_ESTATE, "no adjoint phase (call dvm_adjoint_init)");
    return iterate(*s, 1, max_iter, tol, check_every, iters, resid);
}

int dvm_adjoint_sweeps(dvm_solver *s, int n)
{
    if (int e = check_bound(s)) return e;
    if (s->phase != 1) return fail(DVM_ESTATE, "no adjoint phase (call dvm_adjoint_init)");
    if (n < 0) return fail(DVM_EINVAL, "n < 0");
    return sweeps(*s, 1, n);
}

static int run_sens(dvm_solver *s, int n_params)
{
    HIP_OK(dvm::launch_wall_sens(s->dev, s->frozen_fpar, s->ppar, n_params, s->stream));
    return DVM_OK;
}

int dvm_wall_sensitivity(dvm_solver *s, double *S_A, double *S_x, double *S_n, double *dJ_dnodes)
{
    if (int e = check_bound(s)) return e;
    if (s->phase != 1) return fail(DVM_ESTATE, "no adjoint state");
    if (int e = run_sens(s, 0)) return e;
    std::vector<double> sens(5 * (size_t)s->nw), dn(2 * (size_t)s->nw);
    if (int e = read_back(*s, s->dev.sens, sens.data(), sens.size())) return e;
    if (int e = read_back(*s, s->dev.dJdn, dn.data(), dn.size())) return e;
    for (int l = 0; l < s->nw; l++) {
        if (S_A) S_A[l] = sens[5 * l];
        if (S_x) {
            S_x[2 * l] = sens[5 * l + 1];
            S_x[2 * l + 1] = sens[5 * l + 2];
        }
        if (S_n) {
            S_n[2 * l] = sens[5 * l + 3];
            S_n[2 * l + 1] = sens[5 * l + 4];
        }
    }
    if (dJ_dnodes) std::copy(dn.begin(), dn.end(), dJ_dnodes);
    return DVM_OK;
}

int dvm_param_sensitivity(dvm_solver *s, int n_params, const double *wall_jac, double *dJ_dalpha)
{
    if (int e = check_bound(s)) return e;
    if (s->phase != 1) return fail(DVM_ESTATE, "no adjoint state");
    if (n_params < 0 || n_params > dvm::kMaxParams) return fail(DVM_EINVAL, "n_params must be in [0, %d]", dvm::kMaxParams);
    if (n_params > 0 && (!wall_jac || !dJ_dalpha)) return fail(DVM_EINVAL, "null argument");
    std::vector<double> jac((size_t)2 * s->nw * dvm::kMaxParams, 0.0);
    for (int r = 0; r < 2 * s->nw; r++)
        for (int p = 0; p < n_params; p++) jac[(size_t)r * dvm::kMaxParams + p] = wall_jac[(size_t)r * n_params + p];
    if (int e = upload(*s, s->off.jac, jac.data(), jac.size() * sizeof(double))) return e;
    if (int e = run_sens(s, n_params)) return e;
    if (n_params == 0) {
        HIP_OK(hipStreamSynchronize(s->stream));   // jac must outlive its upload
        return DVM_OK;
    }
    return read_back(*s, s->dev.dJda, dJ_dalpha, n_params);
}

int dvm_mesh_sensitivity(dvm_solver *s, double *dJ_dx)
{
    if (int e = check_bound(s)) return e;
    if (s->phase != 1) return fail(DVM_ESTATE, "no adjoint state");
    if (!dJ_dx) return fail(DVM_EINVAL, "null output");
    HIP_OK(dvm::launch_mesh_sens(s->dev, s->frozen_fpar, s->ppar, s->stream));
    return read_back(*s, s->dev.dJdx, dJ_dx, 2 * (size_t)(s->ni + 1) * (s->nj + 1));
}

size_t dvm_state_bytes(const dvm_solver *s, int which)
{
    if (!s) return 0;
    const size_t row = (size_t)s->nc * s->nv * 2 * elt_bytes(*s);
    if (which == DVM_STATE_F) return row;
    if (which == DVM_STATE_PHI && s->want_adjoint)
        return row + (size_t)8 * s->nc * sizeof(double) + (size_t)s->nw * sizeof(double);
    if (which == DVM_STATE_PHI_ROWS && s->want_adjoint) return row;
    return 0;
}

int dvm_state_save(dvm_solver *s, int which, void *host_dst, size_t bytes)
{
    if (int e = check_bound(s)) return e;
    const size_t need = dvm_state_bytes(s, which);
    if (!need || !host_dst || bytes < need) return fail(DVM_EINVAL, "bad state kind or buffer size");
    if (which == DVM_STATE_F && s->phase < 0) return fail(DVM_ESTATE, "no primal state");
    if (which != DVM_STATE_F && s->phase != 1) return fail(DVM_ESTATE, "no adjoint state");
    char *dst = static_cast<char *>(host_dst);
    const size_t rowb = (size_t)s->nv * 2 * elt_bytes(*s), all = rowb * s->nc, awb = 8 * sizeof(double);
    try {
        std::vector<char> tmp(all + (which == DVM_STATE_PHI ? awb * s->nc : 0));
        if (which == DVM_STATE_F) {
            const int par = s->phase == 1 ? s->frozen_fpar : s->fpar;
            HIP_OK(hipMemcpyAsync(tmp.data(), s->dev.f[par], all, hipMemcpyDeviceToHost, s->stream));
        } else if (which == DVM_STATE_PHI_ROWS) {
            HIP_OK(hipMemcpyAsync(tmp.data(), s->dev.phi[s->ppar], all, hipMemcpyDeviceToHost, s->stream));
        } else {
            HIP_OK(hipMemcpyAsync(tmp.data(), s->dev.phi[s->ppar], all, hipMemcpyDeviceToHost, s->stream));
            HIP_OK(hipMemcpyAsync(tmp.data() + all, s->dev.aW[s->ppar], awb * s->nc, hipMemcpyDeviceToHost, s->stream));
            HIP_OK(hipMemcpyAsync(dst + all + awb * s->nc, s->dev.Phi[s->ppar], (size_t)s->nw * sizeof(double),
                                  hipMemcpyDeviceToHost, s->stream));
        }
        HIP_OK(hipStreamSynchronize(s->stream));
        rows_to_mesh(*s, tmp.data(), dst, rowb);
        if (which == DVM_STATE_PHI) rows_to_mesh(*s, tmp.data() + all, dst + all, awb);
    } catch (const std::bad_alloc &) {
        return fail(DVM_ENOMEM, "out of host memory");
    }
    return DVM_OK;
}

int dvm_state_load(dvm_solver *s, int which, const void *host_src, size_t bytes)
{
    if (int e = check_bound(s)) return e;
    const size_t need = dvm_state_bytes(s, which);
    if (!need || !host_src || bytes < need) return fail(DVM_EINVAL, "bad state kind or buffer size");
    if (which != DVM_STATE_F && s->phase != 1)
        return fail(DVM_ESTATE, "no adjoint phase to load into (call dvm_adjoint_init)");
    const char *src = static_cast<const char *>(host_src);
    const size_t rowb = (size_t)s->nv * 2 * elt_bytes(*s), all = rowb * s->nc, awb = 8 * sizeof(double);
    try {
        std::vector<char> tmp(all + (which == DVM_STATE_PHI ? awb * s->nc : 0));
        rows_to_dev(*s, src, tmp.data(), rowb);
        if (which == DVM_STATE_F) {
            s->fpar = 0;
            s->acc_count = 0;
            HIP_OK(hipMemcpyAsync(s->dev.f[0], tmp.data(), all, hipMemcpyHostToDevice, s->stream));
            HIP_OK(dvm::launch_moments(s->dev, 0, s->stream));
            s->phase = 0;
            s->iters[0] = s->iters[1] = 0;
            s->corr_ok[0] = 0;
        } else if (which == DVM_STATE_PHI_ROWS) {
            HIP_OK(hipMemcpyAsync(s->dev.phi[s->ppar], tmp.data(), all, hipMemcpyHostToDevice, s->stream));
            HIP_OK(dvm::launch_adjoint_moments(s->dev, s->ppar, s->stream));
            s->corr_ok[1] = 0;
            s->acc_acount = 0;
        } else {
            rows_to_dev(*s, src + all, tmp.data() + all, awb);
            HIP_OK(hipMemcpyAsync(s->dev.phi[s->ppar], tmp.data(), all, hipMemcpyHostToDevice, s->stream));
            HIP_OK(hipMemcpyAsync(s->dev.aW[s->ppar], tmp.data() + all, awb * s->nc, hipMemcpyHostToDevice, s->stream));
            HIP_OK(hipMemcpyAsync(s->dev.Phi[s->ppar], src + all + awb * s->nc, (size_t)s->nw * sizeof(double),
                                  hipMemcpyHostToDevice, s->stream));
            s->corr_ok[1] = 0;
        }
        HIP_OK(hipStreamSynchronize(s->stream));   // tmp must outlive the copies
    } catch (const std::bad_alloc &) {
        return fail(DVM_ENOMEM, "out of host memory");
    }
    return DVM_OK;
}

int dvm_state_copy(dvm_solver *dst, const dvm_solver *src, int which)
{
    if (int e = check_bound(dst)) return e;
    if (int e = check_bound(src)) return e;
    if (dst == src) return fail(DVM_EINVAL, "source and destination are the same solver");
    if (dst->topo != src->topo || dst->ni != src->ni || dst->nj != src->nj || dst->nv != src->nv ||
        dst->nw != src->nw || dst->mixed != src->mixed || dst->perm != src->perm)
        return fail(DVM_EINVAL, "solvers differ in grid size, topology, velocity count or precision");
    if (which != DVM_STATE_F && which != DVM_STATE_PHI) return fail(DVM_EINVAL, "bad state kind %d", which);
    if (which == DVM_STATE_F && src->phase < 0) return fail(DVM_ESTATE, "source has no primal state");
    if (which == DVM_STATE_PHI && (src->phase != 1 || dst->phase != 1))
        return fail(DVM_ESTATE, "copying phi needs both solvers in the adjoint phase");
    const size_t all = (size_t)dst->nv * 2 * elt_bytes(*dst) * dst->nc;
    HIP_OK(hipStreamSynchronize(src->stream));
    if (which == DVM_STATE_F) {
        const int par = src->phase == 1 ? src->frozen_fpar : src->fpar;
        dst->fpar = 0;
        dst->acc_count = 0;
        HIP_OK(hipMemcpyAsync(dst->dev.f[0], src->dev.f[par], all, hipMemcpyDeviceToDevice, dst->stream));
        HIP_OK(dvm::launch_moments(dst->dev, 0, dst->stream));
        dst->phase = 0;
        dst->iters[0] = dst->iters[1] = 0;
        dst->corr_ok[0] = 0;
    } else {
        HIP_OK(hipMemcpyAsync(dst->dev.phi[dst->ppar], src->dev.phi[src->ppar], all, hipMemcpyDeviceToDevice,
                              dst->stream));
        HIP_OK(hipMemcpyAsync(dst->dev.aW[dst->ppar], src->dev.aW[src->ppar], 8 * sizeof(double) * dst->nc,
                              hipMemcpyDeviceToDevice, dst->stream));
        HIP_OK(hipMemcpyAsync(dst->dev.Phi[dst->ppar], src->dev.Phi[src->ppar], sizeof(double) * dst->nw,
                              hipMemcpyDeviceToDevice, dst->stream));
        dst->corr_ok[1] = 0;
    }
    HIP_OK(hipStreamSynchronize(dst->stream));
    return DVM_OK;
}

int dvm_solver_iterations(const dvm_solver *s, int phase)
{
    if (!s || phase < 0 || phase > 1) return -1;
    return s->iters[phase];
}

int dvm_solver_phase(const dvm_solver *s) { return s ? s->phase : -1; }

void dvm_solver_destroy(dvm_solver *s) { delete s; }

// ---- batch ----------------------------------------------------------------

static int batch_group(const dvm_solver *s) { return 2 * s->phase + (s->order == 2 ? 1 : 0); }

static void batch_layout(int n, int64_t nblocks, dvm_batch *b, size_t *total)
{
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        const size_t o = cur;
        cur = align_up(cur + bytes);
        return o;
    };
    const size_t ot = take((size_t)n * sizeof(dvm::DevSolve));
    const size_t op = take((size_t)n * sizeof(int32_t));
    const size_t oph = take((size_t)n * sizeof(int32_t));
    const size_t obs = take((size_t)nblocks * sizeof(int32_t));
    const size_t obc = take((size_t)nblocks * sizeof(int32_t));
    const size_t oo = take((size_t)2 * n * sizeof(double));
    if (b) {
        b->off_tab = ot;
        b->off_par = op;
        b->off_phase = oph;
        b->off_bs = obs;
        b->off_bc = obc;
        b->off_out = oo;
    }
    *total = cur;
}

size_t dvm_batch_work_bytes(int n, int64_t total_cells)
{
    if (n <= 0 || total_cells < 0) return 0;
    size_t t;
    // one workgroup per patch (at most one per cell), each member split
    // into 8 pieces of ceil(patches/8): at most 7 padding workgroups per member
    batch_layout(n, total_cells + 7 * (int64_t)n, nullptr, &t);
    return t;
}

// Members of one precision, each bound, in a phase and listed once; the
// workgroups of the four launch groups (primal first- and second-order
// members, adjoint first- and second-order members).
static int batch_check(dvm_solver *const *solvers, int n, int *mixed_out, int64_t per_group[4])
{
    int mixed = -1;
    for (int i = 0; i < n; i++) {
        const dvm_solver *s = solvers[i];
        if (int e = check_bound(s)) return e;
        for (int j = 0; j < i; j++)
            if (solvers[j] == s) return fail(DVM_EINVAL, "solver listed twice");
        if (s->phase < 0) return fail(DVM_ESTATE, "member %d has no primal or adjoint phase", i);
        if (mixed < 0) mixed = s->mixed;
        if (mixed != s->mixed) return fail(DVM_EINVAL, "batch members must share one precision");
    }
    // four groups of workgroups -- primal-phase first-order members, primal
    // second-order, adjoint first-order, adjoint second-order (one kernel
    // launch each) -- one workgroup per (member, patch). Workgroup b of a
    // group runs on XCD b % 8, so within a group XCD x takes the x-th eighth
    // (in sweep order) of every member's patches: each XCD gets the same
    // share of every member's work, whatever the mix of mesh and
    // velocity-grid sizes, and its L2 sees contiguous tiles as in a
    // single-solve sweep.
    for (int g = 0; g < 4; g++) per_group[g] = 0;
    for (int i = 0; i < n; i++) per_group[batch_group(solvers[i])] += (solvers[i]->np + 7) / 8;
    if (8 * (per_group[0] + per_group[1] + per_group[2] + per_group[3]) > INT32_MAX)
        return fail(DVM_EINVAL, "batch too large");
    *mixed_out = mixed;
    return DVM_OK;
}

int dvm_batch_create(dvm_solver *const *solvers, int n, void *work_dev, size_t work_bytes, void *hip_stream,
                     dvm_batch **out)
{
    if (!out || !solvers || n <= 0 || !work_dev) return fail(DVM_EINVAL, "null argument or empty batch");
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(work_dev) % kAlign) return fail(DVM_EINVAL, "work buffer not 256-byte aligned");
    int mixed = -1;
    int64_t per_group[4];
    if (int e = batch_check(solvers, n, &mixed, per_group)) return e;
    const int64_t nblocks = 8 * (per_group[0] + per_group[1] + per_group[2] + per_group[3]);
    size_t need;
    try {
        auto *b = new dvm_batch;
        batch_layout(n, nblocks, b, &need);
        if (work_bytes < need) {
            delete b;
            return fail(DVM_ENOMEM, "batch work buffer of %zu bytes < %zu bytes", work_bytes, need);
        }
        b->owned.assign(solvers, solvers + n);
        b->members = b->owned.data();
        b->n = n;
        b->work = static_cast<char *>(work_dev);
        b->stream = static_cast<hipStream_t>(hip_stream);
        b->nblocks = (int)nblocks;
        for (int g = 0; g < 4; g++) b->nb_group[g] = (int)(8 * per_group[g]);
        b->mixed = mixed;
        std::vector<dvm::DevSolve> tab(n);
        std::vector<int32_t> par(n), phase(n);
        for (int i = 0; i < n; i++) {
            tab[i] = solvers[i]->dev;
            phase[i] = solvers[i]->phase;
            par[i] = phase[i] == 0 ? solvers[i]->fpar : solvers[i]->ppar;
        }
        std::vector<int32_t> bs(nblocks, -1), bc(nblocks, 0);
        int64_t base = 0;
        for (int gr = 0; gr < 4; gr++) {
            std::vector<int64_t> pos(8, 0);   // next slot of each XCD
            for (int i = 0; i < n; i++) {
                const dvm_solver *s = solvers[i];
                if (batch_group(s) != gr) continue;
                const int64_t per = (s->np + 7) / 8;
                for (int x = 0; x < 8; x++) {
                    const int64_t p0 = x * per, p1 = std::min<int64_t>(s->np, p0 + per);
                    for (int64_t p = p0; p < p1; p++, pos[x]++) {
                        const int64_t blk = base + 8 * pos[x] + x;
                        bs[blk] = i;
                        bc[blk] = (int32_t)p;
                    }
                }
            }
            base += 8 * per_group[gr];
        }
        char *w = b->work;
        hipStream_t st = b->stream;
        auto up = [&](size_t off, const void *src, size_t bytes) {
            return hipMemcpyAsync(w + off, src, bytes, hipMemcpyHostToDevice, st);
        };
        hipError_t e = up(b->off_tab, tab.data(), tab.size() * sizeof(dvm::DevSolve));
        if (!e) e = up(b->off_par, par.data(), par.size() * sizeof(int32_t));
        if (!e) e = up(b->off_phase, phase.data(), phase.size() * sizeof(int32_t));
        if (!e) e = up(b->off_bs, bs.data(), bs.size() * sizeof(int32_t));
        if (!e) e = up(b->off_bc, bc.data(), bc.size() * sizeof(int32_t));
        if (!e) e = hipStreamSynchronize(st);
        if (e) {
            delete b;
            return fail(DVM_EHIP, "batch table upload: %s", hipGetErrorString(e));
        }
        for (int i = 0; i < n; i++) solvers[i]->in_batch = 1;
        *out = b;
        return DVM_OK;
    } catch (const std::bad_alloc &) {
        return fail(DVM_ENOMEM, "out of host memory");
    }
}

// The allocation-free batch: at most one per device at a time, its handle
// and member list in static host storage, its tables in the device's fixed
// scratch array (built there by a kernel).
namespace {
constexpr int kStaticDevices = 64;
dvm_batch g_static_batch[kStaticDevices];
bool g_static_live[kStaticDevices] = {};
std::mutex g_static_mu;
}  // namespace

int dvm_batch_create_static(dvm_solver *const *solvers, int n, void *hip_stream, dvm_batch **out)
{
    if (!out || !solvers || n <= 0) return fail(DVM_EINVAL, "null argument or empty batch");
    *out = nullptr;
    if (n > dvm::kStaticBatchMaxMembers)
        return fail(DVM_EINVAL, "%d members: the allocation-free batch takes at most %d", n,
                    dvm::kStaticBatchMaxMembers);
    int mixed = -1;
    int64_t per_group[4];
    if (int e = batch_check(solvers, n, &mixed, per_group)) return e;
    const int64_t nblocks = 8 * (per_group[0] + per_group[1] + per_group[2] + per_group[3]);
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticDevices) return fail(DVM_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (g_static_live[dev])
        return fail(DVM_ESTATE, "an allocation-free batch already exists on device %d (destroy it first)", dev);
    dvm_batch *b = &g_static_batch[dev];
    size_t need;
    batch_layout(n, nblocks, b, &need);
    if (need > dvm::kStaticBatchBytes)
        return fail(DVM_EINVAL, "the batch's tables need %zu bytes; the allocation-free batch holds %zu", need,
                    dvm::kStaticBatchBytes);
    char *w = nullptr;
    HIP_OK(dvm::static_batch_scratch(&w));
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int32_t par[dvm::kStaticBatchMaxMembers], phase[dvm::kStaticBatchMaxMembers];
    for (int i = 0; i < n; i++) {
        phase[i] = solvers[i]->phase;
        par[i] = phase[i] == 0 ? solvers[i]->fpar : solvers[i]->ppar;
        HIP_OK(hipMemcpyAsync(w + b->off_tab + i * sizeof(dvm::DevSolve), &solvers[i]->dev, sizeof(dvm::DevSolve),
                              hipMemcpyHostToDevice, st));
    }
    HIP_OK(hipMemcpyAsync(w + b->off_par, par, n * sizeof(int32_t), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(w + b->off_phase, phase, n * sizeof(int32_t), hipMemcpyHostToDevice, st));
    int nbg[4];
    for (int g = 0; g < 4; g++) nbg[g] = (int)(8 * per_group[g]);
    HIP_OK(dvm::launch_batch_tables(reinterpret_cast<const dvm::DevSolve *>(w + b->off_tab),
                                    reinterpret_cast<const int32_t *>(w + b->off_phase), n, nbg,
                                    reinterpret_cast<int32_t *>(w + b->off_bs), reinterpret_cast<int32_t *>(w + b->off_bc),
                                    st));
    HIP_OK(hipStreamSynchronize(st));   // par, phase and the solver structs must outlive their copies
    for (int i = 0; i < n; i++) b->fixed[i] = solvers[i];
    b->members = b->fixed;
    b->n = n;
    b->static_dev = dev;
    b->work = w;
    b->stream = st;
    b->nblocks = (int)nblocks;
    for (int g = 0; g < 4; g++) b->nb_group[g] = nbg[g];
    b->mixed = mixed;
    b->step = 0;
    for (int i = 0; i < n; i++) solvers[i]->in_batch = 1;
    g_static_live[dev] = true;
    *out = b;
    return DVM_OK;
}

// append member m (nc cells, state buffer par) to a launch group
static void group_add(dvm::MacroGroup &g, int m, int nc, int par)
{
    g.idx[g.n] = m;
    g.par[g.n] = par;
    g.pre[g.n + 1] = g.pre[g.n] + nc;
    g.n++;
}

int dvm_batch_run(dvm_batch *b, int iters)
{
    if (!b) return fail(DVM_EINVAL, "null batch");
    if (iters < 0) return fail(DVM_EINVAL, "iters < 0");
    char *w = b->work;
    const auto *tab = reinterpret_cast<const dvm::DevSolve *>(w + b->off_tab);
    const auto *bs = reinterpret_cast<const int32_t *>(w + b->off_bs);
    const auto *bc = reinterpret_cast<const int32_t *>(w + b->off_bc);
    const auto *par = reinterpret_cast<const int32_t *>(w + b->off_par);
    std::vector<int> due[2];
    for (int it = 0; it < iters; it++) {
        // second-order members: the held correction of the current state,
        // on the same cadence as a single solve's
        for (int m = 0; m < b->n; m++) {
            dvm_solver *s = b->members[m];
            if (s->order != 2) continue;
            const int ph = s->phase;
            if (!s->corr_ok[ph] || s->since[ph] == s->kcorr) {
                const int cur = (ph == 0 ? s->fpar : s->ppar) ^ (it & 1);
                if (ph == 0)
                    HIP_OK(dvm::launch_so_correction(s->dev, cur, b->stream));
                else
                    HIP_OK(dvm::launch_so_adjoint_term(s->dev, cur, b->stream));
                s->corr_ok[ph] = 1;
                s->since[ph] = 0;
            }
            s->since[ph]++;
        }
        // primal members with the conservative equilibrium: its parameters
        // of the current state, which their sweep reads (one launch per
        // group of members)
        {
            dvm::MacroGroup g;
            g.n = 0;
            g.pre[0] = 0;
            for (int m = 0; m < b->n; m++) {
                dvm_solver *s = b->members[m];
                if (s->phase != 0 || s->equil != DVM_EQ_CONSERVATIVE) continue;
                if (!s->dev.mstate) return fail(DVM_ESTATE, "no equilibrium parameter buffer");
                group_add(g, m, s->nc, s->fpar ^ (it & 1));
                if (g.n == dvm::kMacroGroup) {
                    HIP_OK(dvm::launch_eq_params_group(tab, g, 0, b->stream));
                    g.n = 0;
                }
            }
            HIP_OK(dvm::launch_eq_params_group(tab, g, 0, b->stream));
        }
        int off = 0;
        for (int g = 0; g < 4; g++) {
            HIP_OK(dvm::launch_batch(tab, bs + off, bc + off, par, b->step + it, b->nb_group[g], b->mixed, g >> 1,
                                     g & 1, b->stream));
            off += b->nb_group[g];
        }
        // members with the macroscopic prediction, on their own cadence (the
        // state after this sweep sits in buffer par ^ ((it + 1) & 1)): each
        // member's own set-up and finishing kernels, and the Gauss-Seidel
        // steps of all members due with the same inner count in shared
        // launches (the per-cell arithmetic is the single solve's)
        due[0].clear();
        due[1].clear();
        for (int m = 0; m < b->n; m++) {
            dvm_solver *s = b->members[m];
            if (s->acc_every <= 0) continue;
            if (s->phase == 0 && ++s->acc_count % s->acc_every == 0) due[0].push_back(m);
            if (s->phase == 1 && ++s->acc_acount % s->acc_every == 0) due[1].push_back(m);
        }
        for (int adj = 0; adj < 2; adj++) {
            if (due[adj].empty()) continue;
            for (int m : due[adj]) {
                dvm_solver *s = b->members[m];
                const int par = (adj ? s->ppar : s->fpar) ^ ((it + 1) & 1);
                HIP_OK(adj ? dvm::launch_macro_adjoint_begin(s->dev, par, b->stream)
                           : dvm::launch_macro_predict_begin(s->dev, par, b->stream));
            }
            std::vector<int> inners;
            for (int m : due[adj])
                if (std::find(inners.begin(), inners.end(), b->members[m]->acc_inner) == inners.end())
                    inners.push_back(b->members[m]->acc_inner);
            for (int inner : inners) {
                dvm::MacroGroup g;
                g.n = 0;
                g.pre[0] = 0;
                for (int m : due[adj]) {
                    dvm_solver *s = b->members[m];
                    if (s->acc_inner != inner) continue;
                    group_add(g, m, s->nc, 0);
                    if (g.n == dvm::kMacroGroup) {
                        HIP_OK(dvm::launch_macro_gs_group(tab, g, inner, adj, b->stream));
                        g.n = 0;
                    }
                }
                HIP_OK(dvm::launch_macro_gs_group(tab, g, inner, adj, b->stream));
            }
            for (int m : due[adj]) {
                dvm_solver *s = b->members[m];
                const int par = (adj ? s->ppar : s->fpar) ^ ((it + 1) & 1);
                HIP_OK(adj ? dvm::launch_macro_adjoint_end(s->dev, par, b->stream)
                           : dvm::launch_macro_predict_end(s->dev, par, b->stream));
            }
        }
    }
    b->step += iters;
    for (int m = 0; m < b->n; m++) {
        dvm_solver *s = b->members[m];
        if (s->phase == 0)
            s->fpar ^= (iters & 1);
        else
            s->ppar ^= (iters & 1);
        s->iters[s->phase] += iters;
    }
    return DVM_OK;
}

int dvm_batch_residual(dvm_batch *b, double *resid)
{
    if (!b || !resid) return fail(DVM_EINVAL, "null argument");
    const int n = b->n;
    double *out = reinterpret_cast<double *>(b->work + b->off_out);
    HIP_OK(dvm::launch_batch_residual(reinterpret_cast<const dvm::DevSolve *>(b->work + b->off_tab), n, out,
                                      b->stream));
    double small[2 * dvm::kStaticBatchMaxMembers];
    std::vector<double> big;
    if (n > dvm::kStaticBatchMaxMembers) {
        try {
            big.resize(2 * (size_t)n);
        } catch (const std::bad_alloc &) {
            return fail(DVM_ENOMEM, "out of host memory");
        }
    }
    double *v = n > dvm::kStaticBatchMaxMembers ? big.data() : small;
    HIP_OK(hipMemcpyAsync(v, out, 2 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIP_OK(hipStreamSynchronize(b->stream));
    for (int i = 0; i < n; i++) resid[i] = rel_norm(v[2 * i], v[2 * i + 1]);
    return DVM_OK;
}

void dvm_batch_destroy(dvm_batch *b)
{
    if (!b) return;
    for (int m = 0; m < b->n; m++) b->members[m]->in_batch = 0;
    if (b->static_dev >= 0) {
        std::lock_guard<std::mutex> lock(g_static_mu);
        g_static_live[b->static_dev] = false;
        b->n = 0;
        b->members = nullptr;
        return;
    }
    delete b;
}

}  // extern "C"
