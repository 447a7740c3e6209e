// One V-cycle over the small 2D levels in a single workgroup per right-hand
// side, with every level's vectors resident in LDS.
//
// The coarse levels of the hierarchy have too few nodes to fill the GPU;
// launched one kernel per smoothing / transfer pass, each costs a fixed few
// microseconds of latency regardless of its size.  This kernel runs the
// whole zero-guess V(2,2) cycle below a given level - pre-smoothing,
// residual restriction, the dense FP64 coarsest solve, prolongation and
// post-smoothing on every small level - in one launch, one workgroup per
// right-hand side, synchronising with workgroup barriers instead.  The
// arithmetic per node is that of the per-level kernels.
#include "launch.h"
#include "stencil_rows.h"

namespace helm {

namespace {

constexpr int NTS = 1024;
constexpr int WAVE = 64;

template <typename T>
__device__ __forceinline__ cx<T> zero_c() { return mk((T)0, (T)0); }

// (Op x)(i, j) for an LDS vector of the whole level (width n + 1)
template <typename T>
__device__ __forceinline__ cx<T> apply_level(const Op2<T>& op, const cx<T>* s, int i, int j,
                                             cx<T>* diag) {
    const int n = op.n, W = n + 1, p = j * W + i;
    if (i > 0 && i < n && j > 0 && j < n) {
        if (diag) *diag = op.wC;
        cx<T> sa = (s[p + 1] + s[p - 1]) + (s[p + W] + s[p - W]);
        cx<T> sd = s[p + W + 1] + s[p - W - 1];
        return cfma(op.wDg, sd, cfma(op.wAx, sa, op.wC * s[p]));
    }
    Row7<T> r = row_weights(op, i, j);
    if (diag) *diag = r.w[0];
    cx<T> acc = r.w[0] * s[p];
    if (i < n) acc = cfma(r.w[1], s[p + 1], acc);
    if (i > 0) acc = cfma(r.w[2], s[p - 1], acc);
    if (j < n) acc = cfma(r.w[3], s[p + W], acc);
    if (j > 0) acc = cfma(r.w[4], s[p - W], acc);
    if (i < n && j < n) acc = cfma(r.w[5], s[p + W + 1], acc);
    if (i > 0 && j > 0) acc = cfma(r.w[6], s[p - W - 1], acc);
    return acc;
}

template <typename T>
__device__ __forceinline__ cx<T> jfac(const Op2<T>& op, int i, int j) {
    return jacobi_factor(op, i, j);
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_vcycle_small(SmallCycle<T> sc, const cxd* __restrict__ Ainv,
                                                      int nc, Vec<const cx<T>> Bin, Vec<cx<T>> Xout) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(lds_raw);
    const int slot = blockIdx.x;
    const int tid = threadIdx.x;
    const int L = sc.nlev;
    {
        const cx<T>* b = Bin.at(slot);
        cx<T>* B0 = lds + sc.off_b[0];
        const int N0 = (sc.n[0] + 1) * (sc.n[0] + 1);
        for (int q = tid; q < N0; q += NTS) B0[q] = b[q];
    }
    __syncthreads();
    // down: pre-smooth twice from zero, restrict the residual
    for (int l = 0; l < L - 1; ++l) {
        const Op2<T>& op = sc.op[l];
        const int n = op.n, W = n + 1, N = W * W;
        cx<T>* B = lds + sc.off_b[l];
        cx<T>* X = lds + sc.off_x[l];
        cx<T>* Tt = lds + sc.off_t[l];
        for (int q = tid; q < N; q += NTS) Tt[q] = jfac(op, q % W, q / W) * B[q];
        __syncthreads();
        for (int q = tid; q < N; q += NTS) {
            const int i = q % W, j = q / W;
            cx<T> d;
            const cx<T> lt = apply_level(op, Tt, i, j, &d);
            X[q] = cfma(jfac(op, i, j), B[q] - lt, Tt[q]);
        }
        __syncthreads();
        for (int q = tid; q < N; q += NTS) Tt[q] = B[q] - apply_level(op, X, q % W, q / W, (cx<T>*)nullptr);
        __syncthreads();
        const int m = n / 2, Wc = m + 1, Nc = Wc * Wc;
        cx<T>* Bc = lds + sc.off_b[l + 1];
        for (int q = tid; q < Nc; q += NTS) {
            const int I = q % Wc, J = q / Wc, i = 2 * I, j = 2 * J, p = j * W + i;
            cx<T> acc = zero_c<T>();
            if (i < n) acc = acc + Tt[p + 1];
            if (i > 0) acc = acc + Tt[p - 1];
            if (j < n) acc = acc + Tt[p + W];
            if (j > 0) acc = acc + Tt[p - W];
            if (i < n && j < n) acc = acc + Tt[p + W + 1];
            if (i > 0 && j > 0) acc = acc + Tt[p - W - 1];
            Bc[q] = Tt[p] + (T)0.5 * acc;
        }
        __syncthreads();
    }
    // coarsest: x = Ainv b in FP64.  Thread (r, g) forms the partial sum of
    // row r over the columns g, g + G, ...; its loads are issued in batches
    // of eight so that they are in flight together.  Partials meet in the
    // scratch area (at least NTS FP64 complex values), then one thread per
    // row adds its G partials in a fixed order.
    {
        const cx<T>* B = lds + sc.off_b[L - 1];
        cx<T>* X = lds + sc.off_x[L - 1];
        cxd* part = reinterpret_cast<cxd*>(lds + sc.off_t[0]);
        const int G = nc < NTS ? NTS / nc : 1;
        const int r = tid / G, g = tid % G;
        if (r < nc) {
            const cxd* a = Ainv + (long long)r * nc;
            double re = 0.0, im = 0.0;
            for (int c0 = g; c0 < nc; c0 += 8 * G) {
                cxd av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int cc = c0 + u * G;
                    av[u] = cc < nc ? a[cc] : mk(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int cc = c0 + u * G;
                    if (cc < nc) {
                        const cxd bv = cvt<double>(B[cc]);
                        re = fma(av[u].x, bv.x, fma(-av[u].y, bv.y, re));
                        im = fma(av[u].x, bv.y, fma(av[u].y, bv.x, im));
                    }
                }
            }
            part[tid] = mk(re, im);
        }
        __syncthreads();
        if (tid < nc) {
            double re = 0.0, im = 0.0;
            for (int q = 0; q < G; ++q) {
                re += part[tid * G + q].x;
                im += part[tid * G + q].y;
            }
            X[tid] = mk((T)re, (T)im);
        }
    }
    __syncthreads();
    // up: prolongate and correct, post-smooth twice
    for (int l = L - 2; l >= 0; --l) {
        const Op2<T>& op = sc.op[l];
        const int n = op.n, W = n + 1, N = W * W, Wc = n / 2 + 1;
        cx<T>* B = lds + sc.off_b[l];
        cx<T>* X = lds + sc.off_x[l];
        cx<T>* Tt = lds + sc.off_t[l];
        const cx<T>* E = lds + sc.off_x[l + 1];
        for (int q = tid; q < N; q += NTS) {
            const int i = q % W, j = q / W;
            const int c = (j >> 1) * Wc + (i >> 1);
            const int oi = i & 1, oj = j & 1;
            cx<T> v = E[c];
            if (oi | oj) v = (T)0.5 * (v + E[c + oi + oj * Wc]);
            X[q] = X[q] + v;
        }
        __syncthreads();
        for (int q = tid; q < N; q += NTS) {
            const int i = q % W, j = q / W;
            Tt[q] = cfma(jfac(op, i, j), B[q] - apply_level(op, X, i, j, (cx<T>*)nullptr), X[q]);
        }
        __syncthreads();
        for (int q = tid; q < N; q += NTS) {
            const int i = q % W, j = q / W;
            X[q] = cfma(jfac(op, i, j), B[q] - apply_level(op, Tt, i, j, (cx<T>*)nullptr), Tt[q]);
        }
        __syncthreads();
    }
    {
        cx<T>* x = Xout.at(slot);
        const cx<T>* X0 = lds + sc.off_x[0];
        const int N0 = (sc.n[0] + 1) * (sc.n[0] + 1);
        for (int q = tid; q < N0; q += NTS) x[q] = X0[q];
    }
}

}  // namespace

template <typename T>
void vcycle_small(hipStream_t st, const SmallCycle<T>& sc, size_t lds_bytes, const cxd* Ainv,
                  int nc, Vec<const cx<T>> B, Vec<cx<T>> X, int ns) {
    k_vcycle_small<T><<<ns, NTS, lds_bytes, st>>>(sc, Ainv, nc, B, X);
}

template void vcycle_small<double>(hipStream_t, const SmallCycle<double>&, size_t, const cxd*,
                                   int, Vec<const cxd>, Vec<cxd>, int);
template void vcycle_small<float>(hipStream_t, const SmallCycle<float>&, size_t, const cxd*, int,
                                  Vec<const cxf>, Vec<cxf>, int);

}  // namespace helm
