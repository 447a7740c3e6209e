// 2D P1 kernels on the right-diagonal mesh: matrix-free operator apply,
// scaled-Jacobi sweeps, HSS residual, residual restriction and prolongation.
//
// Stencil.  On the mesh whose cells are split along the diagonal from
// (x_i, y_j) to (x_i+1, y_j+1), node (i, j) couples to E, W, N, S and the two
// diagonal neighbours NE (i+1, j+1) and SW (i-1, j-1).  Summing the P1
// element matrices of the (up to six) triangles at a node gives, with
// flags c_pq = 1 when the cell with corner offset (p-1, q-1) is inside the
// square:
//   K : centre c00+c10+c01+c11, E -(c11+c10)/2, W -(c01+c00)/2,
//       N -(c11+c01)/2, S -(c00+c10)/2, diagonals 0;
//   M : (h^2/24) x [centre 2(2c11+c01+2c00+c10), E c11+c10, W c01+c00,
//       N c11+c01, S c00+c10, NE 2c11, SW 2c00];
//   M_Gamma : (h/6) x [1 per boundary edge to each edge neighbour,
//       centre 2 per boundary edge at the node].
// Interior nodes therefore use the constant weights 4a + b h^2/2 (centre),
// -a + b h^2/12 (axis) and b h^2/12 (diagonal); boundary nodes take the
// flagged general form.  Transfers are P1 interpolation between the nested
// n/2 and n meshes (the paper's "standard transfer operators") and its
// transpose.
#include "launch.h"
#include "stencil_rows.h"

namespace helm {

namespace {

constexpr int BS = 256;

template <typename T, typename TI>
__device__ __forceinline__ cx<T> ld(const cx<TI>* p, long long t) {
    return cvt<T>(p[t]);
}

// (Op x) at node (i, j) = t; general form valid for every node.
template <typename T, typename TI>
__device__ __forceinline__ cx<T> apply_general(const Op2<T>& op, const cx<TI>* x, int i, int j,
                                               long long t, cx<T>* diag) {
    const int n = op.n;
    const long long np = n + 1;
    Row7<T> r = row_weights(op, i, j);
    cx<T> acc = r.w[0] * ld<T>(x, t);
    if (i < n) acc = cfma(r.w[1], ld<T>(x, t + 1), acc);
    if (i > 0) acc = cfma(r.w[2], ld<T>(x, t - 1), acc);
    if (j < n) acc = cfma(r.w[3], ld<T>(x, t + np), acc);
    if (j > 0) acc = cfma(r.w[4], ld<T>(x, t - np), acc);
    if (i < n && j < n) acc = cfma(r.w[5], ld<T>(x, t + np + 1), acc);
    if (i > 0 && j > 0) acc = cfma(r.w[6], ld<T>(x, t - np - 1), acc);
    if (diag) *diag = r.w[0];
    return acc;
}

template <typename T, typename TI>
__device__ __forceinline__ cx<T> apply_interior(const Op2<T>& op, const cx<TI>* x, long long t,
                                                long long np) {
    cx<T> c = ld<T>(x, t);
    cx<T> sa = (ld<T>(x, t + 1) + ld<T>(x, t - 1)) + (ld<T>(x, t + np) + ld<T>(x, t - np));
    cx<T> sd = ld<T>(x, t + np + 1) + ld<T>(x, t - np - 1);
    return cfma(op.wDg, sd, cfma(op.wAx, sa, op.wC * c));
}

template <typename T, typename TI, int MODE>
__global__ __launch_bounds__(BS) void k_stencil2d(Op2<T> op, T s, Vec<const cx<TI>> X,
                                                  Vec<const cx<T>> B, Vec<cx<T>> Y,
                                                  long long N, unsigned gx) {
    const unsigned total = gridDim.x;
    const unsigned lin = xcd_remap(blockIdx.x, total);
    const int slot = lin / gx;
    const long long t = (long long)(lin % gx) * BS + threadIdx.x;
    if (t >= N) return;
    const int n = op.n;
    const long long np = n + 1;
    const int j = (int)(t / np);
    const int i = (int)(t - (long long)j * np);
    const bool interior = (i > 0) & (i < n) & (j > 0) & (j < n);
    cx<T>* y = Y.at(slot);
    if (MODE == MODE_JACOBI0 || (MODE == MODE_PRES && !X.base)) {
        const cx<T>* b = B.at(slot);
        const cx<T> f = interior ? op.odC : jacobi_factor(op, i, j);
        y[t] = f * b[t];
        return;
    }
    const cx<TI>* x = X.at(slot);
    cx<T> lx, d;
    if (interior) {
        lx = apply_interior<T, TI>(op, x, t, np);
    } else {
        lx = apply_general<T, TI>(op, x, i, j, t, &d);
    }
    if (MODE == MODE_APPLY) {
        y[t] = lx;
    } else if (MODE == MODE_RESID) {
        const cx<T>* b = B.at(slot);
        y[t] = s * (b[t] - lx);
    } else if (MODE == MODE_PRES) {
        const cx<T>* b = B.at(slot);
        y[t] = (interior ? op.odC : jacobi_factor(op, i, j)) * (b[t] - lx);
    } else if (MODE == MODE_PAPPLY) {
        y[t] = (interior ? op.odC : jacobi_factor(op, i, j)) * lx;
    } else {  // MODE_JACOBI
        const cx<T>* b = B.at(slot);
        cx<T> r = b[t] - lx;
        const cx<T> f = interior ? op.odC : jacobi_factor(op, i, j);
        y[t] = cfma(f, r, ld<T>(x, t));
    }
}

// b_c(I, J) = sum over fine nodes f of P(f, (I,J)) r(f): weight 1 at
// (2I, 2J) and 1/2 at the six fine neighbours along the mesh edges.
template <typename T>
__global__ __launch_bounds__(BS) void k_restrict2d(int n, Vec<const cx<T>> R, Vec<cx<T>> Bc,
                                                   long long Nc, unsigned gx) {
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = lin / gx;
    const long long tc = (long long)(lin % gx) * BS + threadIdx.x;
    if (tc >= Nc) return;
    const int nc = n / 2;
    const long long npc = nc + 1, np = n + 1;
    const int J = (int)(tc / npc), I = (int)(tc - (long long)J * npc);
    const int i = 2 * I, j = 2 * J;
    const long long t = (long long)j * np + i;
    const cx<T>* r = R.at(slot);
    cx<T> acc = mk((T)0, (T)0);
    if (i < n) acc = acc + r[t + 1];
    if (i > 0) acc = acc + r[t - 1];
    if (j < n) acc = acc + r[t + np];
    if (j > 0) acc = acc + r[t - np];
    if (i < n && j < n) acc = acc + r[t + np + 1];
    if (i > 0 && j > 0) acc = acc + r[t - np - 1];
    Bc.at(slot)[tc] = r[t] + (T)0.5 * acc;
}

// Fused residual + restriction: the fine residual at the seven fine nodes
// of each coarse basis function is formed on the fly.
template <typename T>
__global__ __launch_bounds__(BS) void k_resid_restrict2d(Op2<T> op, Vec<const cx<T>> X,
                                                         Vec<const cx<T>> B, Vec<cx<T>> Bc,
                                                         long long Nc, unsigned gx) {
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = lin / gx;
    const long long tc = (long long)(lin % gx) * BS + threadIdx.x;
    if (tc >= Nc) return;
    const int n = op.n, nc = n / 2;
    const long long npc = nc + 1, np = n + 1;
    const int J = (int)(tc / npc), I = (int)(tc - (long long)J * npc);
    const int i0 = 2 * I, j0 = 2 * J;
    const cx<T>* x = X.at(slot);
    const cx<T>* b = B.at(slot);
    const int di[7] = {0, 1, -1, 0, 0, 1, -1};
    const int dj[7] = {0, 0, 0, 1, -1, 1, -1};
    cx<T> acc = mk((T)0, (T)0);
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const int i = i0 + di[q], j = j0 + dj[q];
        if (i < 0 || i > n || j < 0 || j > n) continue;
        const long long t = (long long)j * np + i;
        const bool interior = (i > 0) & (i < n) & (j > 0) & (j < n);
        cx<T> lx = interior ? apply_interior<T, T>(op, x, t, np)
                            : apply_general<T, T>(op, x, i, j, t, nullptr);
        cx<T> r = b[t] - lx;
        acc = acc + (q == 0 ? r : (T)0.5 * r);
    }
    Bc.at(slot)[tc] = acc;
}

// x(i, j) += (P e)(i, j): coarse values at even-even nodes, averages of the
// two coarse endpoints of the coarse edge through every other fine node.
template <typename T>
__global__ __launch_bounds__(BS) void k_prolong2d(int n, Vec<const cx<T>> E, Vec<cx<T>> X,
                                                  long long N, unsigned gx) {
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = lin / gx;
    const long long t = (long long)(lin % gx) * BS + threadIdx.x;
    if (t >= N) return;
    const long long np = n + 1, npc = n / 2 + 1;
    const int j = (int)(t / np), i = (int)(t - (long long)j * np);
    const int I = i >> 1, J = j >> 1;
    const cx<T>* e = E.at(slot);
    const long long c = (long long)J * npc + I;
    cx<T> v = e[c];
    const int oi = i & 1, oj = j & 1;
    if (oi | oj) {
        const long long c2 = c + oi + (long long)oj * npc;  // other endpoint
        v = (T)0.5 * (v + e[c2]);
    }
    cx<T>* x = X.at(slot);
    x[t] = x[t] + v;
}

inline unsigned blocks(long long N) { return (unsigned)((N + BS - 1) / BS); }

}  // namespace

template <typename T, typename TI>
void stencil2d(hipStream_t st, const Op2<T>& op, int mode, T s, Vec<const cx<TI>> X,
               Vec<const cx<T>> B, Vec<cx<T>> Y, int nslots) {
    const long long N = (long long)(op.n + 1) * (op.n + 1);
    const unsigned gx = blocks(N);
    dim3 grid(gx * nslots);
    switch (mode) {
        case MODE_APPLY:
            k_stencil2d<T, TI, MODE_APPLY><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_RESID:
            k_stencil2d<T, TI, MODE_RESID><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_JACOBI:
            k_stencil2d<T, TI, MODE_JACOBI><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_JACOBI0:
            k_stencil2d<T, TI, MODE_JACOBI0><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_PRES:
            k_stencil2d<T, TI, MODE_PRES><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_PAPPLY:
            k_stencil2d<T, TI, MODE_PAPPLY><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
    }
}

template <typename T>
void restrict2d(hipStream_t st, int n, Vec<const cx<T>> R, Vec<cx<T>> Bc, int nslots) {
    const long long Nc = (long long)(n / 2 + 1) * (n / 2 + 1);
    const unsigned gx = blocks(Nc);
    k_restrict2d<T><<<gx * nslots, BS, 0, st>>>(n, R, Bc, Nc, gx);
}

template <typename T>
void resid_restrict2d(hipStream_t st, const Op2<T>& op, Vec<const cx<T>> X, Vec<const cx<T>> B,
                      Vec<cx<T>> Bc, int nslots) {
    const long long Nc = (long long)(op.n / 2 + 1) * (op.n / 2 + 1);
    const unsigned gx = blocks(Nc);
    k_resid_restrict2d<T><<<gx * nslots, BS, 0, st>>>(op, X, B, Bc, Nc, gx);
}

template <typename T>
void prolong2d(hipStream_t st, int n, Vec<const cx<T>> E, Vec<cx<T>> X, int nslots) {
    const long long N = (long long)(n + 1) * (n + 1);
    const unsigned gx = blocks(N);
    k_prolong2d<T><<<gx * nslots, BS, 0, st>>>(n, E, X, N, gx);
}

template void stencil2d<double, double>(hipStream_t, const Op2<double>&, int, double,
                                        Vec<const cxd>, Vec<const cxd>, Vec<cxd>, int);
template void stencil2d<double, float>(hipStream_t, const Op2<double>&, int, double,
                                       Vec<const cxf>, Vec<const cxd>, Vec<cxd>, int);
template void stencil2d<float, float>(hipStream_t, const Op2<float>&, int, float,
                                      Vec<const cxf>, Vec<const cxf>, Vec<cxf>, int);
template void restrict2d<double>(hipStream_t, int, Vec<const cxd>, Vec<cxd>, int);
template void restrict2d<float>(hipStream_t, int, Vec<const cxf>, Vec<cxf>, int);
template void resid_restrict2d<double>(hipStream_t, const Op2<double>&, Vec<const cxd>,
                                       Vec<const cxd>, Vec<cxd>, int);
template void resid_restrict2d<float>(hipStream_t, const Op2<float>&, Vec<const cxf>,
                                      Vec<const cxf>, Vec<cxf>, int);
template void prolong2d<double>(hipStream_t, int, Vec<const cxd>, Vec<cxd>, int);
template void prolong2d<float>(hipStream_t, int, Vec<const cxf>, Vec<cxf>, int);

}  // namespace helm
