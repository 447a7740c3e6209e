// Internal types shared by the HIP kernels and the host driver.
//
// Complex values are interleaved (re, im) pairs aligned to their full size
// so that a double complex moves as one 16-byte load and a float complex as
// one 8-byte load.  Every operator of the method is a K + b M + c M_Gamma
// with complex (a, b, c) (the primal form of Sec. 2 and the HSS operators
// of eq. (HSSpc primal)), so one stencil record per (operator, level)
// describes it completely: the kernels assemble nothing.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace helm {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;  // real, imaginary
};

using cxd = cx<double>;
using cxf = cx<float>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T re, T im) { cx<T> r; r.x = re; r.y = im; return r; }
__host__ __device__ __forceinline__ float fmat(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmat(double a, double b, double c) { return fma(a, b, c); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return mk(fmat(a.x, b.x, -(a.y * b.y)), fmat(a.x, b.y, a.y * b.x));
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk(s * a.x, s * a.y); }
// a * b + c
template <typename T>
__host__ __device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
    return mk(fmat(a.x, b.x, fmat(-a.y, b.y, c.x)), fmat(a.x, b.y, fmat(a.y, b.x, c.y)));
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cjmul(cx<T> a, cx<T> b) {
    return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cdiv(cx<T> a, cx<T> b) {
    T d = b.x * b.x + b.y * b.y;
    return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
template <typename T, typename U>
__host__ __device__ __forceinline__ cx<T> cvt(cx<U> a) { return mk((T)a.x, (T)a.y); }

// A batch of equally sized vectors ("slots"): slot s lives at
// base + (cols ? cols[s] : s) * cstride + off elements.  This lets one
// launch address the s-th right-hand side of a contiguous work buffer and
// the j-th Krylov vector of column cols[s] alike.
template <typename V>
struct Vec {
    V* base;
    long long cstride;
    long long off;
    const int* cols;
    __device__ __forceinline__ V* at(int s) const {
        long long c = cols ? (long long)cols[s] : (long long)s;
        return base + c * cstride + off;
    }
};

template <typename V>
inline Vec<V> contiguous(V* p, long long n) { return Vec<V>{p, n, 0, nullptr}; }

// Stencil record of a a K + b M + c M_Gamma operator on one 2D P1 level.
// A = a, Bm = b h^2 / 24, Cg = c h / 6 (the natural units of the P1 element
// and edge matrices); wC/wAx/wDg are the interior weights of the centre,
// the four axis neighbours and the two "/" diagonal neighbours;
// odC = omega / wC is the interior Jacobi factor.
// The diagonal takes four values: interior, edge (any side), and the two
// corner types of the right-diagonal mesh ((0,0)/(n,n) touch two triangles,
// (n,0)/(0,n) one), so the Jacobi factors omega / D are precomputed:
// odC interior, odE edge, odA corners (0,0)/(n,n), odB corners (n,0)/(0,n).
// Boundary nodes: with the values outside the mesh taken as zero, the
// interior stencil at a node on one mesh edge misses the element row by
// dC on the centre and dN on each of the two neighbours along the edge; at a
// corner, after both edges' corrections, by kA (corners (0,0) and (n,n)) or
// kB (corners (n,0) and (0,n)) on the centre.
template <typename T>
struct Op2 {
    cx<T> A, Bm, Cg;
    cx<T> wC, wAx, wDg;
    cx<T> odC, odE, odA, odB;
    cx<T> dC, dN, kA, kB;
    T omega;
    int n;
    unsigned dir;  // Dirichlet faces (x0=1, x1=2, y0=4, y1=8) for the streaming kernels
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> jacobi_factor(const Op2<T>& op, int i, int j) {
    const int n = op.n;
    const bool ei = (i == 0) | (i == n), ej = (j == 0) | (j == n);
    if (!(ei | ej)) return op.odC;
    if (!(ei & ej)) return op.odE;
    return ((i == 0) == (j == 0)) ? op.odA : op.odB;
}

// Stencil record on one 3D Q1 level: 1D factors of the tensor-product
// element matrices.  K1 = (1/h)[-1 2 -1], M1 = (h/6)[1 4 1], boundary rows
// halve the centre; E marks boundary nodes (M_Gamma = sum of E x M1 x M1).
template <typename T>
struct Op3 {
    cx<T> a, b, c;   // operator = a K + b M + c M_Gamma
    T h;
    T omega;
    cx<T> wInt[4];   // interior weights by neighbour class (0: centre,
                     // 1: face, 2: edge, 3: corner neighbours)
    cx<T> odC;       // omega / interior diagonal
    int n;
};

enum StencilMode : int {
    MODE_APPLY = 0,    // y = Op x
    MODE_RESID = 1,    // y = s (b - Op x)
    MODE_JACOBI = 2,   // y = x + omega D^{-1} (b - Op x)
    MODE_JACOBI0 = 3,  // y = omega D^{-1} b          (zero initial guess)
    MODE_PRES = 4,     // y = omega D^{-1} (b - Op x)  (X null: x = 0)
    MODE_PAPPLY = 5,   // y = omega D^{-1} Op x
};

// Remap a linear workgroup id so that each of the 8 XCDs (which receive
// workgroups round-robin) owns one contiguous range of tiles; neighbouring
// tiles then share halo rows in the same L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned lin, unsigned total) {
    const unsigned nx = 8;
    unsigned xcd = lin % nx, idx = lin / nx;
    unsigned q = total / nx, r = total % nx;
    unsigned start = xcd * q + (xcd < r ? xcd : r);
    return start + idx;
}

}  // namespace helm
