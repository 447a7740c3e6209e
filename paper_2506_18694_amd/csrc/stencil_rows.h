// Per-node stencil rows shared by the kernels and the host code that forms
// the dense coarsest-mesh matrix (so the coarse solve inverts exactly the
// operator the smoothers see).
#pragma once

#include "helm_common.h"

namespace helm {

template <typename T>
struct Row7 {
    cx<T> w[7];  // C, E, W, N, S, NE, SW
};

// 2D P1 right-diagonal mesh: row of a K + b M + c M_Gamma at node (i, j),
// from the element matrices of the triangles present around the node.
template <typename T>
__host__ __device__ __forceinline__ Row7<T> row_weights(const Op2<T>& op, int i, int j) {
    const int n = op.n;
    const T c00 = (i > 0 && j > 0), c10 = (i < n && j > 0);
    const T c01 = (i > 0 && j < n), c11 = (i < n && j < n);
    const T hor = (T)((j == 0) + (j == n)), ver = (T)((i == 0) + (i == n));
    const T gE = hor * (T)(i < n), gW = hor * (T)(i > 0);
    const T gN = ver * (T)(j < n), gS = ver * (T)(j > 0);
    const T kC = c00 + c10 + c01 + c11;
    const T kE = -(c11 + c10) * (T)0.5, kW = -(c01 + c00) * (T)0.5;
    const T kN = -(c11 + c01) * (T)0.5, kS = -(c00 + c10) * (T)0.5;
    const T mC = (T)2 * ((T)2 * c11 + c01 + (T)2 * c00 + c10);
    const T mE = c11 + c10, mW = c01 + c00, mN = c11 + c01, mS = c00 + c10;
    const T gC = (T)2 * (gE + gW + gN + gS);
    Row7<T> r;
    r.w[0] = kC * op.A + mC * op.Bm + gC * op.Cg;
    r.w[1] = kE * op.A + mE * op.Bm + gE * op.Cg;
    r.w[2] = kW * op.A + mW * op.Bm + gW * op.Cg;
    r.w[3] = kN * op.A + mN * op.Bm + gN * op.Cg;
    r.w[4] = kS * op.A + mS * op.Bm + gS * op.Cg;
    r.w[5] = ((T)2 * c11) * op.Bm;
    r.w[6] = ((T)2 * c00) * op.Bm;
    return r;
}

// 3D Q1: 1D factors of node index i on a line of n cells.
//   K1 row: (1/h) {-1, 2, -1} interior, {., 1, -1} at i = 0, {-1, 1, .} at i = n
//   M1 row: (h/6) {1, 4, 1} interior, {., 2, 1} / {1, 2, .} at the ends
//   E  row: 1 on the centre at i = 0 or i = n, else 0
// The 27 weights are a (K1 M1 M1 + M1 K1 M1 + M1 M1 K1)
// + b (M1 M1 M1) + c (E M1 M1 + M1 E M1 + M1 M1 E).
template <typename T>
struct Line3 {
    T k[3], m[3], e;  // offsets -1, 0, +1 (0 where the neighbour is absent)
};

template <typename T>
__host__ __device__ __forceinline__ Line3<T> line_factors(int i, int n, T h) {
    Line3<T> f;
    const T ih = (T)1 / h, h6 = h / (T)6;
    const bool lo = (i == 0), hi = (i == n);
    f.k[0] = lo ? (T)0 : -ih;
    f.k[2] = hi ? (T)0 : -ih;
    f.k[1] = (lo || hi) ? ih : (T)2 * ih;
    f.m[0] = lo ? (T)0 : h6;
    f.m[2] = hi ? (T)0 : h6;
    f.m[1] = (lo || hi) ? (T)2 * h6 : (T)4 * h6;
    f.e = (lo || hi) ? (T)1 : (T)0;
    return f;
}

// weight of neighbour (dx, dy, dz) in {-1,0,1}^3 of node with factors fx, fy, fz
template <typename T>
__host__ __device__ __forceinline__ cx<T> weight3(const Op3<T>& op, const Line3<T>& fx,
                                                  const Line3<T>& fy, const Line3<T>& fz, int dx,
                                                  int dy, int dz) {
    const T kx = fx.k[dx + 1], ky = fy.k[dy + 1], kz = fz.k[dz + 1];
    const T mx = fx.m[dx + 1], my = fy.m[dy + 1], mz = fz.m[dz + 1];
    const T ex = dx == 0 ? fx.e : (T)0, ey = dy == 0 ? fy.e : (T)0, ez = dz == 0 ? fz.e : (T)0;
    const T kk = kx * my * mz + mx * ky * mz + mx * my * kz;
    const T mm = mx * my * mz;
    const T gg = ex * my * mz + mx * ey * mz + mx * my * ez;
    return kk * op.a + mm * op.b + gg * op.c;
}

}  // namespace helm
