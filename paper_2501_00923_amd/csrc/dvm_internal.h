// Internal interface between the host side of libdvm and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct dvm_mesh;

namespace dvm {

constexpr int kBlock = 256;        // threads per workgroup of the per-cell and per-element kernels
constexpr int kWave = 64;          // wavefront width
constexpr int kMaxN1D = 128;       // max velocity nodes per direction
constexpr int kMaxParams = 64;
constexpr int kAcoef = 32;         // doubles per cell of the adjoint coefficients
constexpr int kEqState = 20;       // doubles per cell of mstate: P' (4), dP'/dW (16, row = parameter)

// The sweeps give each workgroup a patch of kPatchI x kPatchJ cells, one
// wave per cell; patches tile kTileI x kTileJ tiles, which follow each
// other along strips of kTileI columns.  Cells are stored (and numbered on
// the device) in that order, patch after patch.  Measured on the 256x128
// C-grid with 2304 velocities (FP64 adjoint sweep): strips of 8, 16, 32 and
// 64 columns take 775, 755, 735 and 745 us.
constexpr int kPatchI = 2, kPatchJ = 2, kPatchCells = kPatchI * kPatchJ;
constexpr int kTileI = 32, kTileJ = 16;

// Everything a kernel needs about one solve, passed by value (single solve)
// or read from a device table (batched).  Pointers are device pointers into
// the solver's workspace.  Storage type of f / phi / fd / gM is float in
// mixed mode and double in FP64 mode.
struct DevSolve {
    int nc, nw, nv, n1, n2;
    int np;                  // patches
    int ni, nj;              // structured grid size (cells along the wall, cells outward)
    int topo;
    int objective;
    int mixed;
    int order;               // spatial order of the scheme: 1, or 2 (reconstructed face values)
    int equil;               // equilibrium: 0 pointwise Maxwellian, 1 discrete-conservative
    int limiter;             // order 2: 0 none, 1 Venkatakrishnan
    // mesh
    const int32_t *nbr;      // [nc][4] (device cell numbering)
    const int32_t *patch;    // [np + 1] first cell of each patch; patch p = cells [patch[p], patch[p+1])
    const int32_t *cell_of;  // [nc] mesh cell number (i + ni*j) of each device cell
    const double *S;         // [nc][4][2]
    const double *vol;       // [nc]
    const int32_t *wall_cell;// [nw]
    const double *wall_A;    // [nw]
    const double *wall_n;    // [nw][2]
    const double *wall_a;    // [nw][2]
    const double *wall_b;    // [nw][2]
    const double *D;         // [nw] eq. (barg) normaliser
    // velocity grid (1-D factors)
    const double *vx, *vy, *wx, *wy;
    const void *fd;          // [nv][2] far-field values (storage type)
    const void *gM;          // [nv]    g_M1(1, 0, theta_w) (storage type)
    const void *gw2;         // [nv][2] (g_M1, theta_w/2 g_M1)(1, 0, theta_w) (storage type)
    // flow
    double inv_tau_inf, u_inf, theta_w, cd_scale;
    // primal state (ping-pong)
    void *f[2];
    double *W[2];            // [nc][4]
    double *F[2];            // [nw]
    double *red;             // [nc][2] per-cell residual partials of the last sweep
    // adjoint state
    void *phi[2];
    double *aW[2];           // [nc][8]: What (4), rho_tau, pad
    double *Phi[2];          // [nw]
    const void *fstar;       // frozen primal f (= f[primal parity at adjoint init])
    double *acoef;           // [nc][kAcoef] per-cell adjoint coefficients (see k_adjoint_coef)
    // sensitivity / objective
    double *Jl;              // [nw]
    double *sens;            // [nw][5]: S_A, S_x(2), S_n(2)
    double *dJdn;            // [nw][2]
    double *jac;             // [nw][2][kMaxParams]
    double *dJda;            // [kMaxParams]
    double *msens;           // [nc][4][2] per mesh cell: dL/d(corner coordinates)
    double *dJdx;            // [(nj+1)(ni+1)][2] dL/d(node coordinates), mesh node numbering
    double *out;             // [16] small scalar outputs
    // second-order scheme (order 2 only; null otherwise)
    const double *rf;        // [nc][4][2] face midpoint minus the cell's centroid
    const double *rn;        // [nc][4][2] face midpoint minus the neighbour's centroid (interior faces)
    void *G;                 // [nc][nv][4] limited slopes (f1x, f1y, f2x, f2y); adjoint: B (storage type)
    void *corr;              // [nc][nv][2] held flux correction c; adjoint: held term E (storage type)
    void *psi;               // [nc][nv][2] limiter factors of the frozen f (storage type)
    double *dF;              // [nw] held wall-flux correction
    // macroscopic prediction (primal acceleration; null when off)
    double *mstate;          // [nc][kEqState] equilibrium parameters P' and dP'/dW (conservative equilibrium)
    double *mr;              // [nc][4] moments of the kinetic residual
    double *mDinv;           // [nc][16] inverse of the cell's own block
    double *mO;              // [nc][4][16] outflow block of each face (dg/dW form)
    double *mx[2];           // [nc][4] red-black iterates
};

// launches (all on `st`); par = index of the current f / phi buffer
hipError_t launch_primal_init(const DevSolve &d, hipStream_t st);
hipError_t launch_primal_sweep(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_moments(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_residual(const DevSolve &d, int adjoint, hipStream_t st);
hipError_t launch_objective(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_adjoint_init(const DevSolve &d, int fpar, hipStream_t st);
hipError_t launch_adjoint_sweep(const DevSolve &d, int par, hipStream_t st);
// adjoint moments (What, rho_tau) and wall multipliers of phi[par] (a loaded phi)
hipError_t launch_adjoint_moments(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_adjoint_correct_moments(const DevSolve &d, int par, const double *z, hipStream_t st);
hipError_t launch_eq_params(const DevSolve &d, int par, int with_M, hipStream_t st);
hipError_t launch_wall_sens(const DevSolve &d, int fpar, int ppar, int n_params, hipStream_t st);
hipError_t launch_mesh_sens(const DevSolve &d, int fpar, int ppar, hipStream_t st);
// macroscopic prediction of the moments W[par] of f[par] (first-order
// scheme): assembly, `inner` red-black block Gauss-Seidel steps, limited
// update of W[par]
hipError_t launch_macro_predict(const DevSolve &d, int par, int inner, hipStream_t st);
// adjoint prediction: the system at the frozen f[fpar] and its transpose
// (at the adjoint's start); every K adjoint sweeps, A^T dl = -r* and What of
// phi[ppar] += dl
hipError_t launch_macro_adjoint_setup(const DevSolve &d, int fpar, hipStream_t st);
hipError_t launch_macro_adjoint_predict(const DevSolve &d, int ppar, int inner, hipStream_t st);
// A group of batch members for one launch of a per-cell kernel: member a is
// tab[idx[a]], owns cells pre[a] .. pre[a+1]-1 of the launch and its state
// is in buffer par[a].
constexpr int kMacroGroup = 64;
struct MacroGroup {
    int n;
    int idx[kMacroGroup];
    int par[kMacroGroup];
    int pre[kMacroGroup + 1];
};
hipError_t launch_macro_predict_begin(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_macro_predict_end(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_macro_adjoint_begin(const DevSolve &d, int pnew, hipStream_t st);
hipError_t launch_macro_adjoint_end(const DevSolve &d, int pnew, hipStream_t st);
hipError_t launch_macro_gs_group(const DevSolve *tab, const MacroGroup &g, int inner, int adjoint, hipStream_t st);
hipError_t launch_eq_params_group(const DevSolve *tab, const MacroGroup &g, int with_M, hipStream_t st);

// second-order scheme: the slopes G and dF of f[par]; the held primal
// correction c (with G and dF) from f[par]; the
// limiter factors psi of f[fpar] for the adjoint; the held adjoint term E
// from phi[par]; the drag with reconstructed wall values (per element)
hipError_t launch_so_slopes(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_so_correction(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_so_freeze(const DevSolve &d, int fpar, hipStream_t st);
hipError_t launch_so_adjoint_term(const DevSolve &d, int par, hipStream_t st);
hipError_t launch_so_objective_elem(const DevSolve &d, int par, hipStream_t st);

// batched: table of DevSolve on the device, per-block (solve, patch) map,
// per-solve buffer parity at batch creation; step = sweeps done since batch
// creation; adjoint selects the kernel of that phase, so the scheme (the
// blocks of one launch are members of one phase and one scheme)
hipError_t launch_batch(const DevSolve *tab, const int32_t *blk_solve, const int32_t *blk_patch,
                        const int32_t *par0, int step, int nblocks, int mixed, int adjoint, int so, hipStream_t st);
hipError_t launch_batch_residual(const DevSolve *tab, int n, double *out, hipStream_t st);

// The allocation-free batch (dvm_batch_create_static) keeps its launch
// tables in one fixed device array per GPU, of kStaticBatchBytes, for at
// most kStaticBatchMaxMembers members.  static_batch_scratch gives the
// current device's copy of the array (its address is looked up once per
// device); launch_batch_tables writes the per-workgroup (member, patch) map
// of the four groups (group g = 2 * phase + (order == 2), nb_group[g]
// workgroups each, in that order) from the member table and phases, in the
// layout dvm_batch_create builds on the host.
constexpr size_t kStaticBatchBytes = size_t(8) << 20;
constexpr int kStaticBatchMaxMembers = 64;
hipError_t static_batch_scratch(char **out);
hipError_t launch_batch_tables(const DevSolve *tab, const int32_t *phase, int n, const int *nb_group,
                               int32_t *blk_solve, int32_t *blk_patch, hipStream_t st);


// radial-basis-function mesh motion (Wendland C0, support 1/inv_r):
// apply: out[n] = wall[widx[n]] for wall nodes, else x0[n] + sum_w gamma[w]
// phi(|x0[n] - c[w]| inv_r); chain: h[w] = sum over non-wall nodes n of
// phi(|x0[n] - c[w]| inv_r) g[n], via per-chunk partials part[chunk][nw]
// summed in chunk order.  Points are double2 = (x, y).
constexpr int kRbfChainNodes = 256;    // nodes per workgroup of the chain kernel
constexpr int kRbfTile = 64;           // centres per workgroup of the chain kernel
inline int rbf_chunks(int nn) { return (nn + kRbfChainNodes - 1) / kRbfChainNodes; }
hipError_t launch_rbf_apply(const double *x0, const int32_t *widx, int nn, const double *c,
                            const double *gamma, const double *wall, int nw, double inv_r, double *out,
                            hipStream_t st);
hipError_t launch_rbf_chain(const double *x0, const int32_t *widx, const double *g, int nn, const double *c,
                            int nw, double inv_r, double *part, double *h, hipStream_t st);

// for host sources other than dvm_host.cpp: set the thread's error message
// (returns code), and the node grid of a mesh
int set_error(int code, const char *fmt, ...);
struct MeshNodes {
    int topo, ni, nj, nwake, nw;
    const double *nodes;     // [(nj+1)(ni+1)][2]
};
MeshNodes mesh_nodes(const dvm_mesh *m);

}  // namespace dvm
