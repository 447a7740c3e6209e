// 3D Q1 kernels on the uniform hexahedral mesh: matrix-free 27-point
// operator apply / Jacobi / residual, and trilinear transfers.
//
// The Q1 element matrices on a uniform mesh are tensor products of the 1D
// linear-element matrices, so the assembled K, M and M_Gamma are
//   K = K1 (x) M1 (x) M1 + M1 (x) K1 (x) M1 + M1 (x) M1 (x) K1,
//   M = M1 (x) M1 (x) M1,
//   M_Gamma = E (x) M1 (x) M1 + M1 (x) E (x) M1 + M1 (x) M1 (x) E,
// with the 1D rows of line_factors() (boundary rows halve the interior
// centre; E = 1 on the end nodes).  Interior nodes use four weights, one
// per neighbour class (centre, 6 faces, 12 edges, 8 corners); nodes on the
// boundary evaluate the tensor-product weight of each neighbour.
#include "launch.h"
#include "stencil_rows.h"

namespace helm {

namespace {

constexpr int BS = 256;

template <typename T, typename TI>
__device__ __forceinline__ cx<T> ld3(const cx<TI>* p, long long t) {
    return cvt<T>(p[t]);
}

template <typename T, typename TI>
__device__ __forceinline__ cx<T> apply3_interior(const Op3<T>& op, const cx<TI>* x, long long t,
                                                 long long sy, long long sz) {
    cx<T> c = ld3<T>(x, t);
    cx<T> f = mk((T)0, (T)0), e = mk((T)0, (T)0), k = mk((T)0, (T)0);
    f = f + ld3<T>(x, t - 1) + ld3<T>(x, t + 1) + ld3<T>(x, t - sy) + ld3<T>(x, t + sy) +
        ld3<T>(x, t - sz) + ld3<T>(x, t + sz);
#pragma unroll
    for (int dz = -1; dz <= 1; dz += 2) {
#pragma unroll
        for (int dy = -1; dy <= 1; dy += 2) {
            const long long b = t + dz * sz + dy * sy;
            e = e + ld3<T>(x, t + dz * sz + dy * sy);  // yz edges
            k = k + ld3<T>(x, b - 1) + ld3<T>(x, b + 1);
        }
#pragma unroll
        for (int dx = -1; dx <= 1; dx += 2) e = e + ld3<T>(x, t + dz * sz + dx);  // xz edges
    }
#pragma unroll
    for (int dy = -1; dy <= 1; dy += 2)
#pragma unroll
        for (int dx = -1; dx <= 1; dx += 2) e = e + ld3<T>(x, t + dy * sy + dx);  // xy edges
    return cfma(op.wInt[3], k, cfma(op.wInt[2], e, cfma(op.wInt[1], f, op.wInt[0] * c)));
}

template <typename T, typename TI>
__device__ __forceinline__ cx<T> apply3_general(const Op3<T>& op, const cx<TI>* x, int i, int j,
                                                int l, long long t, long long sy, long long sz,
                                                cx<T>* diag) {
    const int n = op.n;
    const Line3<T> fx = line_factors<T>(i, n, op.h);
    const Line3<T> fy = line_factors<T>(j, n, op.h);
    const Line3<T> fz = line_factors<T>(l, n, op.h);
    cx<T> acc = mk((T)0, (T)0);
    for (int dz = -1; dz <= 1; ++dz) {
        if (l + dz < 0 || l + dz > n) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            if (j + dy < 0 || j + dy > n) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                if (i + dx < 0 || i + dx > n) continue;
                const cx<T> w = weight3(op, fx, fy, fz, dx, dy, dz);
                acc = cfma(w, ld3<T>(x, t + dz * sz + dy * sy + dx), acc);
            }
        }
    }
    if (diag) *diag = weight3(op, fx, fy, fz, 0, 0, 0);
    return acc;
}

template <typename T, typename TI, int MODE>
__global__ __launch_bounds__(BS) void k_stencil3d(Op3<T> op, T s, Vec<const cx<TI>> X,
                                                  Vec<const cx<T>> B, Vec<cx<T>> Y, long long N,
                                                  unsigned gx) {
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = lin / gx;
    const long long t = (long long)(lin % gx) * BS + threadIdx.x;
    if (t >= N) return;
    const int n = op.n;
    const long long sy = n + 1, sz = sy * sy;
    const int l = (int)(t / sz);
    const long long rem = t - (long long)l * sz;
    const int j = (int)(rem / sy);
    const int i = (int)(rem - (long long)j * sy);
    const bool interior = (i > 0) & (i < n) & (j > 0) & (j < n) & (l > 0) & (l < n);
    cx<T>* y = Y.at(slot);
    if (MODE == MODE_JACOBI0) {
        cx<T> f;
        if (interior) {
            f = op.odC;
        } else {
            const Line3<T> fx = line_factors<T>(i, n, op.h);
            const Line3<T> fy = line_factors<T>(j, n, op.h);
            const Line3<T> fz = line_factors<T>(l, n, op.h);
            f = cdiv(mk(op.omega, (T)0), weight3(op, fx, fy, fz, 0, 0, 0));
        }
        y[t] = f * B.at(slot)[t];
        return;
    }
    const cx<TI>* x = X.at(slot);
    cx<T> lx, d;
    if (interior) lx = apply3_interior<T, TI>(op, x, t, sy, sz);
    else lx = apply3_general<T, TI>(op, x, i, j, l, t, sy, sz, &d);
    if (MODE == MODE_APPLY) {
        y[t] = lx;
    } else if (MODE == MODE_RESID) {
        y[t] = s * (B.at(slot)[t] - lx);
    } else {
        cx<T> r = B.at(slot)[t] - lx;
        cx<T> f = interior ? op.odC : cdiv(mk(op.omega, (T)0), d);
        y[t] = cfma(f, r, ld3<T>(x, t));
    }
}

// b_c = P^T r for trilinear P: weights 1 (even offset) or 1/2 (odd) per axis.
template <typename T>
__global__ __launch_bounds__(BS) void k_restrict3d(int n, Vec<const cx<T>> R, Vec<cx<T>> Bc,
                                                   long long Nc, unsigned gx) {
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = lin / gx;
    const long long tc = (long long)(lin % gx) * BS + threadIdx.x;
    if (tc >= Nc) return;
    const int nc = n / 2;
    const long long syc = nc + 1, szc = syc * syc, sy = n + 1, sz = sy * sy;
    const int L = (int)(tc / szc);
    const long long rem = tc - (long long)L * szc;
    const int J = (int)(rem / syc), I = (int)(rem - (long long)J * syc);
    const cx<T>* r = R.at(slot);
    cx<T> acc = mk((T)0, (T)0);
    for (int dz = -1; dz <= 1; ++dz) {
        const int l = 2 * L + dz;
        if (l < 0 || l > n) continue;
        const T wz = dz ? (T)0.5 : (T)1;
        for (int dy = -1; dy <= 1; ++dy) {
            const int j = 2 * J + dy;
            if (j < 0 || j > n) continue;
            const T wy = dy ? (T)0.5 : (T)1;
            for (int dx = -1; dx <= 1; ++dx) {
                const int i = 2 * I + dx;
                if (i < 0 || i > n) continue;
                const T wx = dx ? (T)0.5 : (T)1;
                acc = acc + (wx * wy * wz) * r[(long long)l * sz + (long long)j * sy + i];
            }
        }
    }
    Bc.at(slot)[tc] = acc;
}

// x += P e (trilinear interpolation from the n/2 mesh)
template <typename T>
__global__ __launch_bounds__(BS) void k_prolong3d(int n, Vec<const cx<T>> E, Vec<cx<T>> X,
                                                  long long N, unsigned gx) {
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = lin / gx;
    const long long t = (long long)(lin % gx) * BS + threadIdx.x;
    if (t >= N) return;
    const long long sy = n + 1, sz = sy * sy;
    const int nc = n / 2;
    const long long syc = nc + 1, szc = syc * syc;
    const int l = (int)(t / sz);
    const long long rem = t - (long long)l * sz;
    const int j = (int)(rem / sy), i = (int)(rem - (long long)j * sy);
    const int I = i >> 1, J = j >> 1, L = l >> 1;
    const int oi = i & 1, oj = j & 1, ol = l & 1;
    const cx<T>* e = E.at(slot);
    cx<T> v = mk((T)0, (T)0);
    for (int cz = 0; cz <= ol; ++cz)
        for (int cy = 0; cy <= oj; ++cy)
            for (int cx_ = 0; cx_ <= oi; ++cx_)
                v = v + e[(long long)(L + cz) * szc + (long long)(J + cy) * syc + (I + cx_)];
    const T w = (T)1 / (T)(1 << (oi + oj + ol));
    cx<T>* x = X.at(slot);
    x[t] = x[t] + w * v;
}

inline unsigned blocks(long long N) { return (unsigned)((N + BS - 1) / BS); }

}  // namespace

template <typename T, typename TI>
void stencil3d(hipStream_t st, const Op3<T>& op, int mode, T s, Vec<const cx<TI>> X,
               Vec<const cx<T>> B, Vec<cx<T>> Y, int nslots) {
    const long long N = (long long)(op.n + 1) * (op.n + 1) * (op.n + 1);
    const unsigned gx = blocks(N);
    dim3 grid(gx * nslots);
    switch (mode) {
        case MODE_APPLY:
            k_stencil3d<T, TI, MODE_APPLY><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_RESID:
            k_stencil3d<T, TI, MODE_RESID><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_JACOBI:
            k_stencil3d<T, TI, MODE_JACOBI><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_JACOBI0:
            k_stencil3d<T, TI, MODE_JACOBI0><<<grid, BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
    }
}

template <typename T>
void restrict3d(hipStream_t st, int n, Vec<const cx<T>> R, Vec<cx<T>> Bc, int nslots) {
    const long long Nc = (long long)(n / 2 + 1) * (n / 2 + 1) * (n / 2 + 1);
    const unsigned gx = blocks(Nc);
    k_restrict3d<T><<<gx * nslots, BS, 0, st>>>(n, R, Bc, Nc, gx);
}

template <typename T>
void prolong3d(hipStream_t st, int n, Vec<const cx<T>> E, Vec<cx<T>> X, int nslots) {
    const long long N = (long long)(n + 1) * (n + 1) * (n + 1);
    const unsigned gx = blocks(N);
    k_prolong3d<T><<<gx * nslots, BS, 0, st>>>(n, E, X, N, gx);
}

template void stencil3d<double, double>(hipStream_t, const Op3<double>&, int, double,
                                        Vec<const cxd>, Vec<const cxd>, Vec<cxd>, int);
template void stencil3d<double, float>(hipStream_t, const Op3<double>&, int, double,
                                       Vec<const cxf>, Vec<const cxd>, Vec<cxd>, int);
template void stencil3d<float, float>(hipStream_t, const Op3<float>&, int, float, Vec<const cxf>,
                                      Vec<const cxf>, Vec<cxf>, int);
template void restrict3d<double>(hipStream_t, int, Vec<const cxd>, Vec<cxd>, int);
template void restrict3d<float>(hipStream_t, int, Vec<const cxf>, Vec<cxf>, int);
template void prolong3d<double>(hipStream_t, int, Vec<const cxd>, Vec<cxd>, int);
template void prolong3d<float>(hipStream_t, int, Vec<const cxf>, Vec<cxf>, int);

}  // namespace helm
