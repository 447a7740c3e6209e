// Kernels of the mixed formulation ([DG0]^2 x P1 on the right-diagonal
// mesh; Sec. 2 and the mixed shifted-HSS preconditioner).
//
// A mixed vector of one column is [u | sigma]: u at the N = (n+1)^2 nodes
// (lexicographic), then sigma on the 2 n^2 triangles, triangle
// e = t n^2 + (p + n q) of cell (p, q) with t = 0 for
// {(p,q), (p+1,q), (p+1,q+1)} and t = 1 for {(p,q), (p+1,q+1), (p,q+1)},
// its x and y components at 2e and 2e + 1 (complex FP64 each).
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

// grad u on triangle (t, p, q), scaled by n = 1/h
__device__ __forceinline__ void tri_grad(const cxd* u, int n, int t, int p, int q, cxd& gx, cxd& gy) {
    const long long np = n + 1;
    const long long a = p + np * q;  // node (p, q)
    const double s = (double)n;
    if (t == 0) {  // (p,q), (p+1,q), (p+1,q+1)
        const cxd uA = u[a], uB = u[a + 1], uC = u[a + np + 1];
        gx = s * (uB - uA);
        gy = s * (uC - uB);
    } else {       // (p,q), (p+1,q+1), (p,q+1)
        const cxd uA = u[a], uC = u[a + np + 1], uD = u[a + np];
        gx = s * (uC - uD);
        gy = s * (uD - uA);
    }
}

// y = sb B + Op u + G^T (sa sigma + sg g) at every node (B, g nullable).
__global__ __launch_bounds__(BS) void k_mixed_nodes(Op2<double> op, cxd sb, cxd sa, cxd sg,
                                                    Vec<const cxd> X, Vec<const cxd> B,
                                                    Vec<const cxd> Gv, Vec<cxd> Y, long long N,
                                                    unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long v = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    if (v >= N) return;
    const int n = op.n;
    const long long np = n + 1, nn = (long long)n * n;
    const int j = (int)(v / np), i = (int)(v - (long long)j * np);
    const cxd* u = X.at(slot);
    const cxd* sig = u + N;
    const cxd* g = Gv.base ? Gv.at(slot) : nullptr;
    const Row7<double> r = row_weights(op, i, j);
    cxd acc = r.w[0] * u[v];
    if (i < n) acc = cfma(r.w[1], u[v + 1], acc);
    if (i > 0) acc = cfma(r.w[2], u[v - 1], acc);
    if (j < n) acc = cfma(r.w[3], u[v + np], acc);
    if (j > 0) acc = cfma(r.w[4], u[v - np], acc);
    if (i < n && j < n) acc = cfma(r.w[5], u[v + np + 1], acc);
    if (i > 0 && j > 0) acc = cfma(r.w[6], u[v - np - 1], acc);
    // f = sa sigma + sg g on triangle e, component c
    auto f = [&](long long e, int c) {
        cxd val = sa * sig[2 * e + c];
        if (g) val = cfma(sg, g[2 * e + c], val);
        return val;
    };
    cxd div = mk(0.0, 0.0);
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
    const double hh = 0.5 / n;       // area * |grad phi| = (h^2/2)(1/h)
    acc = cfma(mk(hh, 0.0), div, acc);
    if (B.base) acc = cfma(sb, B.at(slot)[v], acc);
    Y.at(slot)[v] = acc;
}

// sigma rows of the mixed system: y = area (s sigma - grad u)  (APPLY) or
// y = B - area (s sigma - grad u)  (RESID), written after the u part of Y
template <int MODE>
__global__ __launch_bounds__(BS) void k_mixed_tris(int n, cxd s, Vec<const cxd> X, Vec<const cxd> B,
                                                   Vec<cxd> Y, long long N, unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long e = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    const long long nn = (long long)n * n;
    if (e >= 2 * nn) return;
    const int t = (int)(e / nn);
    const long long cell = e - t * nn;
    const int q = (int)(cell / n), p = (int)(cell - (long long)q * n);
    const cxd* u = X.at(slot);
    const cxd* sig = u + N;
    cxd gxv, gyv;
    tri_grad(u, n, t, p, q, gxv, gyv);
    const double area = 0.5 / ((double)n * n);
    cxd yx = area * (s * sig[2 * e] - gxv), yy = area * (s * sig[2 * e + 1] - gyv);
    if (MODE == MODE_RESID) {
        const cxd* b = B.at(slot) + N;
        yx = b[2 * e] - yx;
        yy = b[2 * e + 1] - yy;
    }
    cxd* y = Y.at(slot) + N;
    y[2 * e] = yx;
    y[2 * e + 1] = yy;
}

// g = nukp sigma + nu grad u + c R_sigma / area   (one HSS step's sigma data)
__global__ __launch_bounds__(BS) void k_mixed_g(int n, cxd nukp, double nu, double c,
                                                Vec<const cxd> X, Vec<const cxd> R, Vec<cxd> G,
                                                long long N, unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long e = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    const long long nn = (long long)n * n;
    if (e >= 2 * nn) return;
    const int t = (int)(e / nn);
    const long long cell = e - t * nn;
    const int q = (int)(cell / n), p = (int)(cell - (long long)q * n);
    const cxd* u = X.at(slot);
    const cxd* sig = u + N;
    const cxd* rs = R.at(slot) + N;
    cxd gxv, gyv;
    tri_grad(u, n, t, p, q, gxv, gyv);
    const double ia = 2.0 * (double)n * n;  // 1 / area
    cxd* g = G.at(slot);
    g[2 * e] = nukp * sig[2 * e] + nu * gxv + (c * ia) * rs[2 * e];
    g[2 * e + 1] = nukp * sig[2 * e + 1] + nu * gyv + (c * ia) * rs[2 * e + 1];
}

// sigma = inv (grad u + g), written into the sigma part of Y
__global__ __launch_bounds__(BS) void k_mixed_sigma(int n, cxd inv, Vec<const cxd> X,
                                                    Vec<const cxd> G, Vec<cxd> Y, long long N,
                                                    unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long e = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    const long long nn = (long long)n * n;
    if (e >= 2 * nn) return;
    const int t = (int)(e / nn);
    const long long cell = e - t * nn;
    const int q = (int)(cell / n), p = (int)(cell - (long long)q * n);
    cxd gxv, gyv;
    tri_grad(X.at(slot), n, t, p, q, gxv, gyv);
    const cxd* g = G.at(slot);
    cxd* y = Y.at(slot) + N;
    y[2 * e] = inv * (gxv + g[2 * e]);
    y[2 * e + 1] = inv * (gyv + g[2 * e + 1]);
}

}  // namespace

void mixed_nodes(hipStream_t st, const Op2<double>& op, cxd sb, cxd sa, cxd sg, Vec<const cxd> X,
                 Vec<const cxd> B, Vec<const cxd> G, Vec<cxd> Y, int nslots) {
    const long long N = (long long)(op.n + 1) * (op.n + 1);
    const unsigned gx = blocks(N);
    k_mixed_nodes<<<gx * nslots, BS, 0, st>>>(op, sb, sa, sg, X, B, G, Y, N, gx);
}

void mixed_tris(hipStream_t st, int n, int mode, cxd s, Vec<const cxd> X, Vec<const cxd> B,
                Vec<cxd> Y, int nslots) {
    const long long N = (long long)(n + 1) * (n + 1);
    const unsigned gx = blocks(2LL * n * n);
    if (mode == MODE_RESID)
        k_mixed_tris<MODE_RESID><<<gx * nslots, BS, 0, st>>>(n, s, X, B, Y, N, gx);
    else
        k_mixed_tris<MODE_APPLY><<<gx * nslots, BS, 0, st>>>(n, s, X, B, Y, N, gx);
}

void mixed_g(hipStream_t st, int n, cxd nukp, double nu, double c, Vec<const cxd> X,
             Vec<const cxd> R, Vec<cxd> G, int nslots) {
    const long long N = (long long)(n + 1) * (n + 1);
    const unsigned gx = blocks(2LL * n * n);
    k_mixed_g<<<gx * nslots, BS, 0, st>>>(n, nukp, nu, c, X, R, G, N, gx);
}

void mixed_sigma(hipStream_t st, int n, cxd inv, Vec<const cxd> X, Vec<const cxd> G, Vec<cxd> Y,
                 int nslots) {
    const long long N = (long long)(n + 1) * (n + 1);
    const unsigned gx = blocks(2LL * n * n);
    k_mixed_sigma<<<gx * nslots, BS, 0, st>>>(n, inv, X, G, Y, N, gx);
}

}  // namespace helm
