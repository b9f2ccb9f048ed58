// Radial-basis-function bulk-mesh motion (Sec. 3.4, Step 2) with the
// Wendland C0 function phi(r) = (1 - r)^2 on r < 1 (r = distance / support).
//
// Per node the work is a sum over all wall centres of a few FP64 operations
// and a square root; the centre tables (or node chunk) sit in LDS and the
// lanes of a wave read at most four distinct entries at a time (LDS
// broadcasts).  Every sum runs in a fixed order, so results do not depend
// on timing.
#include <hip/hip_runtime.h>

#include "dvm_internal.h"

namespace dvm {
namespace {

constexpr int kApplyBlock = 256;
constexpr int kChainBlock = 256;   // 4 waves, each over a quarter of the chunk

// phi(|d| / R) added, times (gx, gy), to (ax, ay); pairs farther apart than
// the support (d^2 >= R^2) skip the square root
__device__ __forceinline__ void wendland_c0_acc(double dx, double dy, double inv_r, double r2, double gx, double gy,
                                                double &ax, double &ay)
{
    const double d2 = dx * dx + dy * dy;
    if (d2 < r2) {
        const double s = 1.0 - sqrt(d2) * inv_r;
        const double ph = s * s;
        ax += ph * gx;
        ay += ph * gy;
    }
}

// Four lanes per mesh node (64 nodes per workgroup), each summing every
// fourth centre; centres and weights are staged through LDS in blocks of
// kApplyBlock and the four partial sums are combined by a fixed butterfly.
constexpr int kApplyNodes = kApplyBlock / 4;

__global__ __launch_bounds__(kApplyBlock) void k_rbf_apply(const double2 *__restrict__ x0,
                                                            const int32_t *__restrict__ widx, int nn,
                                                            const double2 *__restrict__ c,
                                                            const double2 *__restrict__ gam,
                                                            const double2 *__restrict__ wall, int nw,
                                                            double inv_r, double2 *__restrict__ out)
{
    __shared__ double2 sc[kApplyBlock], sg[kApplyBlock];
    const int n = blockIdx.x * kApplyNodes + (threadIdx.x >> 2);
    const int part = threadIdx.x & 3;
    const double2 p = n < nn ? x0[n] : make_double2(0.0, 0.0);
    const double r2 = 1.0 / (inv_r * inv_r);
    double ax = 0.0, ay = 0.0;
    for (int w0 = 0; w0 < nw; w0 += kApplyBlock) {
        const int w = w0 + threadIdx.x;
        if (w < nw) {
            sc[threadIdx.x] = c[w];
            sg[threadIdx.x] = gam[w];
        }
        __syncthreads();
        const int m = min(kApplyBlock, nw - w0);
        for (int k = part; k < m; k += 4)
            wendland_c0_acc(p.x - sc[k].x, p.y - sc[k].y, inv_r, r2, sg[k].x, sg[k].y, ax, ay);
        __syncthreads();
    }
    ax += __shfl_xor(ax, 1, 64);
    ay += __shfl_xor(ay, 1, 64);
    ax += __shfl_xor(ax, 2, 64);
    ay += __shfl_xor(ay, 2, 64);
    if (n < nn && part == 0) {
        const int l = widx[n];
        out[n] = l >= 0 ? wall[l] : make_double2(p.x + ax, p.y + ay);
    }
}

// Workgroup (chunk, tile): centres tile*64 + lane, nodes of the chunk
// (kRbfChainNodes) staged in LDS; wave q takes the q-th quarter of them and
// the four partial sums are added in wave order.  Wall nodes carry no
// interpolated term (their derivative is taken directly on the host).
__global__ __launch_bounds__(kChainBlock) void k_rbf_chain_part(const double2 *__restrict__ x0,
                                                                 const int32_t *__restrict__ widx,
                                                                 const double2 *__restrict__ g, int nn,
                                                                 const double2 *__restrict__ c, int nw,
                                                                 double inv_r, double2 *__restrict__ part)
{
    __shared__ double2 sx[kRbfChainNodes], sg[kRbfChainNodes];
    __shared__ double2 red[kChainBlock];
    const int chunk = blockIdx.x;
    const int n0 = chunk * kRbfChainNodes;
    const int cnt = min(kRbfChainNodes, nn - n0);
    for (int t = threadIdx.x; t < kRbfChainNodes; t += kChainBlock) {
        double2 xv = make_double2(0.0, 0.0), gv = make_double2(0.0, 0.0);
        if (t < cnt) {
            xv = x0[n0 + t];
            if (widx[n0 + t] < 0) gv = g[n0 + t];
        }
        sx[t] = xv;
        sg[t] = gv;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int w = blockIdx.y * kRbfTile + lane;
    const bool valid = w < nw;
    const double2 cw = valid ? c[w] : make_double2(0.0, 0.0);
    constexpr int per = kRbfChainNodes / (kChainBlock / 64);
    const int k1 = min(cnt, (q + 1) * per);
    const double r2 = 1.0 / (inv_r * inv_r);
    double hx = 0.0, hy = 0.0;
    for (int k = q * per; k < k1; k++) wendland_c0_acc(sx[k].x - cw.x, sx[k].y - cw.y, inv_r, r2, sg[k].x, sg[k].y, hx, hy);
    red[threadIdx.x] = make_double2(hx, hy);
    __syncthreads();
    if (q == 0 && valid) {
        const double2 a = red[lane], b = red[64 + lane], e = red[128 + lane], f = red[192 + lane];
        part[(size_t)chunk * nw + w] = make_double2(((a.x + b.x) + e.x) + f.x, ((a.y + b.y) + e.y) + f.y);
    }
}

// One wave per centre: lane k adds chunks k, k + 64, ...; the lanes'
// sums are combined by a fixed butterfly.
__global__ __launch_bounds__(kApplyBlock) void k_rbf_chain_sum(const double2 *__restrict__ part, int nchunk,
                                                                int nw, double2 *__restrict__ h)
{
    const int w = blockIdx.x * (kApplyBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    double hx = 0.0, hy = 0.0;
    if (w < nw) {
        for (int k = lane; k < nchunk; k += 64) {
            const double2 v = part[(size_t)k * nw + w];
            hx += v.x;
            hy += v.y;
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        hx += __shfl_xor(hx, off, 64);
        hy += __shfl_xor(hy, off, 64);
    }
    if (w < nw && lane == 0) h[w] = make_double2(hx, hy);
}

}  // namespace

hipError_t launch_rbf_apply(const double *x0, const int32_t *widx, int nn, const double *c, const double *gamma,
                            const double *wall, int nw, double inv_r, double *out, hipStream_t st)
{
    if (nn <= 0) return hipSuccess;
    const int nb = (nn + kApplyNodes - 1) / kApplyNodes;
    hipLaunchKernelGGL(k_rbf_apply, dim3(nb), dim3(kApplyBlock), 0, st, (const double2 *)x0, widx, nn,
                       (const double2 *)c, (const double2 *)gamma, (const double2 *)wall, nw, inv_r,
                       (double2 *)out);
    return hipGetLastError();
}

hipError_t launch_rbf_chain(const double *x0, const int32_t *widx, const double *g, int nn, const double *c,
                            int nw, double inv_r, double *part, double *h, hipStream_t st)
{
    if (nn <= 0 || nw <= 0) return hipSuccess;
    const int nchunk = rbf_chunks(nn);
    const dim3 grid(nchunk, (nw + kRbfTile - 1) / kRbfTile);
    hipLaunchKernelGGL(k_rbf_chain_part, grid, dim3(kChainBlock), 0, st, (const double2 *)x0, widx,
                       (const double2 *)g, nn, (const double2 *)c, nw, inv_r, (double2 *)part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    constexpr int waves = kApplyBlock / 64;
    hipLaunchKernelGGL(k_rbf_chain_sum, dim3((nw + waves - 1) / waves), dim3(kApplyBlock), 0, st,
                       (const double2 *)part, nchunk, nw, (double2 *)h);
    return hipGetLastError();
}

}  // namespace dvm
