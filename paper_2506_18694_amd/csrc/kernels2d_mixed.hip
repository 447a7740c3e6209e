// Kernels of the mixed formulation ([DG0]^2 x P1 on the right-diagonal
// mesh; Sec. 2 and the mixed shifted-HSS preconditioner).
//
// A mixed vector of one column is [u | sigma]: u at the N = (n+1)^2 nodes
// (lexicographic), then sigma on the 2 n^2 triangles, triangle
// e = t n^2 + (p + n q) of cell (p, q) with t = 0 for
// {(p,q), (p+1,q), (p+1,q+1)} and t = 1 for {(p,q), (p+1,q+1), (p,q+1)},
// its x and y components at 2e and 2e + 1 (complex FP64, or FP32 in the
// preconditioner of the FP32 multigrid mode).
//
// Per triangle (area h^2/2) the P1 gradient is a difference of two nodal
// values over h; the discrete divergence G^T f at a node sums, over the six
// triangles around it, area * f_T . grad(phi_node)|_T = +-(h/2) f_x or f_y.
#include "helm_common.h"
#include "stencil_rows.h"
#include "launch.h"

namespace helm {
namespace {

constexpr int BS = 256;

inline unsigned blocks(long long N) { return (unsigned)((N + BS - 1) / BS); }

// grad u on triangle (t, p, q), scaled by n = 1/h (u read in TI, result in T)
template <typename T, typename TI>
__device__ __forceinline__ void tri_grad(const cx<TI>* u, int n, int t, int p, int q, cx<T>& gx,
                                         cx<T>& gy) {
    const long long np = n + 1;
    const long long a = p + np * q;  // node (p, q)
    const T s = (T)n;
    if (t == 0) {  // (p,q), (p+1,q), (p+1,q+1)
        const cx<T> uA = cvt<T>(u[a]), uB = cvt<T>(u[a + 1]), uC = cvt<T>(u[a + np + 1]);
        gx = s * (uB - uA);
        gy = s * (uC - uB);
    } else {       // (p,q), (p+1,q+1), (p,q+1)
        const cx<T> uA = cvt<T>(u[a]), uC = cvt<T>(u[a + np + 1]), uD = cvt<T>(u[a + np]);
        gx = s * (uC - uD);
        gy = s * (uD - uA);
    }
}

// y = sb B + Op u + G^T (sa sigma + sg g) at every node (B, g nullable);
// X (u and sigma) in TI, everything else in T.
template <typename T, typename TI>
__global__ __launch_bounds__(BS) void k_mixed_nodes(Op2<T> op, cx<T> sb, cx<T> sa, cx<T> sg,
                                                    Vec<const cx<TI>> X, Vec<const cx<T>> B,
                                                    Vec<const cx<T>> Gv, Vec<cx<T>> Y, long long N,
                                                    unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long v = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    if (v >= N) return;
    const int n = op.n;
    const long long np = n + 1, nn = (long long)n * n;
    const int j = (int)(v / np), i = (int)(v - (long long)j * np);
    const cx<TI>* u = X.at(slot);
    const cx<TI>* sig = u + N;
    const cx<T>* g = Gv.base ? Gv.at(slot) : nullptr;
    const Row7<T> r = row_weights(op, i, j);
    cx<T> acc = r.w[0] * cvt<T>(u[v]);
    if (i < n) acc = cfma(r.w[1], cvt<T>(u[v + 1]), acc);
    if (i > 0) acc = cfma(r.w[2], cvt<T>(u[v - 1]), acc);
    if (j < n) acc = cfma(r.w[3], cvt<T>(u[v + np]), acc);
    if (j > 0) acc = cfma(r.w[4], cvt<T>(u[v - np]), acc);
    if (i < n && j < n) acc = cfma(r.w[5], cvt<T>(u[v + np + 1]), acc);
    if (i > 0 && j > 0) acc = cfma(r.w[6], cvt<T>(u[v - np - 1]), acc);
    // f = sa sigma + sg g on triangle e, component c
    auto f = [&](long long e, int c) {
        cx<T> val = sa * cvt<T>(sig[2 * e + c]);
        if (g) val = cfma(sg, g[2 * e + c], val);
        return val;
    };
    cx<T> div = mk((T)0, (T)0);
    if (i < n && j < n) {            // cell (i, j): both triangles have the node as vertex A
        const long long cell = i + (long long)n * j;
        div = div - f(cell, 0) - f(nn + cell, 1);
    }
    if (i > 0 && j < n) {            // cell (i-1, j): t = 0, vertex B, grad = (1, -1)/h
        const long long cell = (i - 1) + (long long)n * j;
        div = div + f(cell, 0) - f(cell, 1);
    }
    if (i < n && j > 0) {            // cell (i, j-1): t = 1, vertex D, grad = (-1, 1)/h
        const long long cell = i + (long long)n * (j - 1);
        div = div - f(nn + cell, 0) + f(nn + cell, 1);
    }
    if (i > 0 && j > 0) {            // cell (i-1, j-1): vertex C of both triangles
        const long long cell = (i - 1) + (long long)n * (j - 1);
        div = div + f(cell, 1) + f(nn + cell, 0);
    }
    const T hh = (T)(0.5 / n);       // area * |grad phi| = (h^2/2)(1/h)
    acc = cfma(mk(hh, (T)0), div, acc);
    if (B.base) acc = cfma(sb, B.at(slot)[v], acc);
    Y.at(slot)[v] = acc;
}

// sigma rows of the mixed system: y = area (s sigma - grad u)  (APPLY) or
// y = B - area (s sigma - grad u)  (RESID), written after the u part of Y
template <typename T, typename TI, int MODE>
__global__ __launch_bounds__(BS) void k_mixed_tris(int n, cx<T> s, Vec<const cx<TI>> X,
                                                   Vec<const cx<T>> B, Vec<cx<T>> Y, long long N,
                                                   unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long e = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    const long long nn = (long long)n * n;
    if (e >= 2 * nn) return;
    const int t = (int)(e / nn);
    const long long cell = e - t * nn;
    const int q = (int)(cell / n), p = (int)(cell - (long long)q * n);
    const cx<TI>* u = X.at(slot);
    const cx<TI>* sig = u + N;
    cx<T> gxv, gyv;
    tri_grad<T, TI>(u, n, t, p, q, gxv, gyv);
    const T area = (T)(0.5 / ((double)n * n));
    cx<T> yx = area * (s * cvt<T>(sig[2 * e]) - gxv), yy = area * (s * cvt<T>(sig[2 * e + 1]) - gyv);
    if (MODE == MODE_RESID) {
        const cx<T>* b = B.at(slot) + N;
        yx = b[2 * e] - yx;
        yy = b[2 * e + 1] - yy;
    }
    cx<T>* y = Y.at(slot) + N;
    y[2 * e] = yx;
    y[2 * e + 1] = yy;
}

// g = nukp sigma + nu grad u + c R_sigma / area   (one HSS step's sigma data)
template <typename T>
__global__ __launch_bounds__(BS) void k_mixed_g(int n, cx<T> nukp, T nu, T c, Vec<const cx<T>> X,
                                                Vec<const cx<T>> R, Vec<cx<T>> G, long long N,
                                                unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long e = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    const long long nn = (long long)n * n;
    if (e >= 2 * nn) return;
    const int t = (int)(e / nn);
    const long long cell = e - t * nn;
    const int q = (int)(cell / n), p = (int)(cell - (long long)q * n);
    const cx<T>* u = X.at(slot);
    const cx<T>* sig = u + N;
    const cx<T>* rs = R.at(slot) + N;
    cx<T> gxv, gyv;
    tri_grad<T, T>(u, n, t, p, q, gxv, gyv);
    const T ia = (T)(2.0 * (double)n * n);  // 1 / area
    cx<T>* g = G.at(slot);
    g[2 * e] = nukp * sig[2 * e] + nu * gxv + (c * ia) * rs[2 * e];
    g[2 * e + 1] = nukp * sig[2 * e + 1] + nu * gyv + (c * ia) * rs[2 * e + 1];
}

// sigma = inv (grad u + g), written into the sigma part of Y
template <typename T>
__global__ __launch_bounds__(BS) void k_mixed_sigma(int n, cx<T> inv, Vec<const cx<T>> X,
                                                    Vec<const cx<T>> G, Vec<cx<T>> Y, long long N,
                                                    unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long e = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    const long long nn = (long long)n * n;
    if (e >= 2 * nn) return;
    const int t = (int)(e / nn);
    const long long cell = e - t * nn;
    const int q = (int)(cell / n), p = (int)(cell - (long long)q * n);
    cx<T> gxv, gyv;
    tri_grad<T, T>(X.at(slot), n, t, p, q, gxv, gyv);
    const cx<T>* g = G.at(slot);
    cx<T>* y = Y.at(slot) + N;
    y[2 * e] = inv * (gxv + g[2 * e]);
    y[2 * e + 1] = inv * (gyv + g[2 * e + 1]);
}

}  // namespace

template <typename T, typename TI>
void mixed_nodes(hipStream_t st, const Op2<T>& op, cx<T> sb, cx<T> sa, cx<T> sg,
                 Vec<const cx<TI>> X, Vec<const cx<T>> B, Vec<const cx<T>> G, Vec<cx<T>> Y,
                 int nslots) {
    const long long N = (long long)(op.n + 1) * (op.n + 1);
    const unsigned gx = blocks(N);
    k_mixed_nodes<T, TI><<<gx * nslots, BS, 0, st>>>(op, sb, sa, sg, X, B, G, Y, N, gx);
}

template <typename T, typename TI>
void mixed_tris(hipStream_t st, int n, int mode, cx<T> s, Vec<const cx<TI>> X, Vec<const cx<T>> B,
                Vec<cx<T>> Y, int nslots) {
    const long long N = (long long)(n + 1) * (n + 1);
    const unsigned gx = blocks(2LL * n * n);
    if (mode == MODE_RESID)
        k_mixed_tris<T, TI, MODE_RESID><<<gx * nslots, BS, 0, st>>>(n, s, X, B, Y, N, gx);
    else
        k_mixed_tris<T, TI, MODE_APPLY><<<gx * nslots, BS, 0, st>>>(n, s, X, B, Y, N, gx);
}

template <typename T>
void mixed_g(hipStream_t st, int n, cx<T> nukp, T nu, T c, Vec<const cx<T>> X, Vec<const cx<T>> R,
             Vec<cx<T>> G, int nslots) {
    const long long N = (long long)(n + 1) * (n + 1);
    const unsigned gx = blocks(2LL * n * n);
    k_mixed_g<T><<<gx * nslots, BS, 0, st>>>(n, nukp, nu, c, X, R, G, N, gx);
}

template <typename T>
void mixed_sigma(hipStream_t st, int n, cx<T> inv, Vec<const cx<T>> X, Vec<const cx<T>> G,
                 Vec<cx<T>> Y, int nslots) {
    const long long N = (long long)(n + 1) * (n + 1);
    const unsigned gx = blocks(2LL * n * n);
    k_mixed_sigma<T><<<gx * nslots, BS, 0, st>>>(n, inv, X, G, Y, N, gx);
}

template void mixed_nodes<double, double>(hipStream_t, const Op2<double>&, cxd, cxd, cxd,
                                          Vec<const cxd>, Vec<const cxd>, Vec<const cxd>, Vec<cxd>, int);
template void mixed_nodes<double, float>(hipStream_t, const Op2<double>&, cxd, cxd, cxd,
                                         Vec<const cxf>, Vec<const cxd>, Vec<const cxd>, Vec<cxd>, int);
template void mixed_nodes<float, float>(hipStream_t, const Op2<float>&, cxf, cxf, cxf,
                                        Vec<const cxf>, Vec<const cxf>, Vec<const cxf>, Vec<cxf>, int);
template void mixed_tris<double, double>(hipStream_t, int, int, cxd, Vec<const cxd>, Vec<const cxd>,
                                         Vec<cxd>, int);
template void mixed_tris<double, float>(hipStream_t, int, int, cxd, Vec<const cxf>, Vec<const cxd>,
                                        Vec<cxd>, int);
template void mixed_tris<float, float>(hipStream_t, int, int, cxf, Vec<const cxf>, Vec<const cxf>,
                                       Vec<cxf>, int);
template void mixed_g<double>(hipStream_t, int, cxd, double, double, Vec<const cxd>, Vec<const cxd>,
                              Vec<cxd>, int);
template void mixed_g<float>(hipStream_t, int, cxf, float, float, Vec<const cxf>, Vec<const cxf>,
                             Vec<cxf>, int);
template void mixed_sigma<double>(hipStream_t, int, cxd, Vec<const cxd>, Vec<const cxd>, Vec<cxd>, int);
template void mixed_sigma<float>(hipStream_t, int, cxf, Vec<const cxf>, Vec<const cxf>, Vec<cxf>, int);

}  // namespace helm
