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

template <typename T>
__device__ __forceinline__ cx<T> sel(bool c, cx<T> a, cx<T> b) { return c ? a : b; }

// a + s t for a real s
template <typename T>
__device__ __forceinline__ cx<T> axpy_real(T sc, cx<T> t, cx<T> a) {
    return mk(fmat(sc, t.x, a.x), fmat(sc, t.y, a.y));
}

// Node q of a level with W = n + 1 nodes per row: (i, j) = (q mod W, q div W)
// by a multiply with md = ceil(2^20 / W), exact while q W <= 2^20.
struct Node {
    int i, j, p;
};
__device__ __forceinline__ Node node_of(int q, int W, int md) {
    Node nd;
    nd.j = (int)(((unsigned)q * (unsigned)md) >> 20);
    nd.i = q - nd.j * W;
    nd.p = q;
    return nd;
}

// (Op s)(i, j) for an LDS vector of the whole level.  Values outside the
// mesh are taken as zero: the interior stencil then needs, on a boundary
// column, the along-column neighbours and centre corrected (dN, dC), on a
// boundary row the along-row ones, and at a corner the remaining centre
// term (kA at (0,0) and (n,n), kB at (n,0) and (0,n)).  Every node runs the
// same instructions; the out-of-mesh neighbours are read at the centre's
// address and replaced by zero.
template <typename T>
__device__ __forceinline__ cx<T> apply_level(const Op2<T>& op, const cx<T>* s, const Node& nd) {
    const int n = op.n, W = n + 1, p = nd.p;
    const bool hE = nd.i < n, hW = nd.i > 0, hN = nd.j < n, hS = nd.j > 0;
    const cx<T> z = zero_c<T>();
    const cx<T> c = s[p];
    const cx<T> e = sel(hE, s[hE ? p + 1 : p], z), w = sel(hW, s[hW ? p - 1 : p], z);
    const cx<T> nn = sel(hN, s[hN ? p + W : p], z), ss = sel(hS, s[hS ? p - W : p], z);
    const bool hNE = hE & hN, hSW = hW & hS;
    const cx<T> ne = sel(hNE, s[hNE ? p + W + 1 : p], z), sw = sel(hSW, s[hSW ? p - W - 1 : p], z);
    cx<T> acc = cfma(op.wDg, ne + sw, cfma(op.wAx, (e + w) + (nn + ss), op.wC * c));
    const T cb = (hE & hW) ? (T)0 : (T)1, rb = (hN & hS) ? (T)0 : (T)1;
    acc = axpy_real(cb, cfma(op.dN, nn + ss, op.dC * c), acc);
    acc = axpy_real(rb, cfma(op.dN, e + w, op.dC * c), acc);
    const bool lo = (nd.i == 0) == (nd.j == 0);
    return axpy_real(cb * rb, sel(lo, op.kA, op.kB) * c, acc);
}

// Jacobi factor omega / diag at a node: interior, edge, or one of the two
// corner classes
template <typename T>
__device__ __forceinline__ cx<T> jfac(const Op2<T>& op, const Node& nd) {
    const int n = op.n;
    const bool ei = (nd.i == 0) | (nd.i == n), ej = (nd.j == 0) | (nd.j == n);
    const bool lo = (nd.i == 0) == (nd.j == 0);
    return sel(ei & ej, sel(lo, op.odA, op.odB), sel(ei | ej, op.odE, op.odC));
}

// b_c = P^T r at coarse node (I, J): the fine residual at (2I, 2J) plus half
// of it at the six neighbours present in the mesh
template <typename T>
__device__ __forceinline__ cx<T> restrict_at(const cx<T>* r, int n, int I, int J) {
    const int W = n + 1, i = 2 * I, j = 2 * J, p = j * W + i;
    const bool hE = i < n, hW = i > 0, hN = j < n, hS = j > 0;
    const bool hNE = hE & hN, hSW = hW & hS;
    const cx<T> z = zero_c<T>();
    const cx<T> e = sel(hE, r[hE ? p + 1 : p], z), w = sel(hW, r[hW ? p - 1 : p], z);
    const cx<T> nn = sel(hN, r[hN ? p + W : p], z), ss = sel(hS, r[hS ? p - W : p], z);
    const cx<T> ne = sel(hNE, r[hNE ? p + W + 1 : p], z), sw = sel(hSW, r[hSW ? p - W - 1 : p], z);
    const cx<T> sum = ((e + w) + (nn + ss)) + (ne + sw);
    return cfma(mk((T)0.5, (T)0), sum, r[p]);
}

template <typename T>
__global__ __launch_bounds__(NTS) void k_vcycle_small(SmallCycle<T> sc, const cxd* __restrict__ Ainv,
                                                      int nc, Vec<const cx<T>> Bin, Vec<cx<T>> Xout) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(lds_raw);
    const int slot = blockIdx.x;
    const int tid = threadIdx.x;
    const int L = sc.nlev;
    // coarsest solve x = Ainv b in FP64: thread (r, g) forms the partial sum
    // of row r over the columns g, g + G, ...; its first CW entries of Ainv
    // are loaded now so that their latency is hidden behind the descent
    constexpr int CW = 8;
    const int G = nc < NTS ? NTS / nc : 1;
    const int cr = tid / G, cg = tid % G;
    const bool crow = cr < nc;
    cxd av[CW];
#pragma unroll
    for (int u = 0; u < CW; ++u) {
        const int cc = cg + u * G;
        av[u] = (crow && cc < nc) ? Ainv[(long long)cr * nc + cc] : mk(0.0, 0.0);
    }
    // level 0: load b and form the first pre-smoothing iterate t = jf b
    {
        const Op2<T>& op = sc.op[0];
        const int W = op.n + 1, N = W * W, md = sc.mdiv[0];
        const cx<T>* b = Bin.at(slot);
        cx<T>* B = lds + sc.off_b[0];
        cx<T>* Tt = lds + sc.off_t[0];
        for (int q = tid; q < N; q += NTS) {
            const cx<T> v = b[q];
            B[q] = v;
            Tt[q] = jfac(op, node_of(q, W, md)) * v;
        }
    }
    __syncthreads();
    // down: first pre-smoothing iterate (level 0: formed with the load),
    // second sweep, residual, restriction
    for (int l = 0; l < L - 1; ++l) {
        const Op2<T>& op = sc.op[l];
        const int n = op.n, W = n + 1, N = W * W, md = sc.mdiv[l];
        const cx<T>* B = lds + sc.off_b[l];
        cx<T>* X = lds + sc.off_x[l];
        cx<T>* Tt = lds + sc.off_t[l];
        if (l > 0) {
            for (int q = tid; q < N; q += NTS) Tt[q] = jfac(op, node_of(q, W, md)) * B[q];
            __syncthreads();
        }
        for (int q = tid; q < N; q += NTS) {
            const Node nd = node_of(q, W, md);
            X[q] = cfma(jfac(op, nd), B[q] - apply_level(op, Tt, nd), Tt[q]);
        }
        __syncthreads();
        for (int q = tid; q < N; q += NTS) Tt[q] = B[q] - apply_level(op, X, node_of(q, W, md));
        __syncthreads();
        const int Wc = n / 2 + 1, Nc = Wc * Wc, mdc = sc.mdiv[l + 1];
        cx<T>* Bc = lds + sc.off_b[l + 1];
        for (int q = tid; q < Nc; q += NTS) {
            const Node ndc = node_of(q, Wc, mdc);
            Bc[q] = restrict_at(Tt, n, ndc.i, ndc.j);
        }
        __syncthreads();
    }
    // coarsest: partials meet in the scratch area (at least NTS FP64 complex
    // values), then one thread per row adds its G partials in a fixed order
    {
        const cx<T>* B = lds + sc.off_b[L - 1];
        cx<T>* X = lds + sc.off_x[L - 1];
        cxd* part = reinterpret_cast<cxd*>(lds + sc.off_part);
        if (crow) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int u = 0; u < CW; ++u) {
                const int cc = cg + u * G;
                if (cc < nc) {
                    const cxd bv = cvt<double>(B[cc]);
                    re = fma(av[u].x, bv.x, fma(-av[u].y, bv.y, re));
                    im = fma(av[u].x, bv.y, fma(av[u].y, bv.x, im));
                }
            }
            for (int cc = cg + CW * G; cc < nc; cc += G) {
                const cxd a = Ainv[(long long)cr * nc + cc];
                const cxd bv = cvt<double>(B[cc]);
                re = fma(a.x, bv.x, fma(-a.y, bv.y, re));
                im = fma(a.x, bv.y, fma(a.y, bv.x, im));
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
        const int n = op.n, W = n + 1, N = W * W, Wc = n / 2 + 1, md = sc.mdiv[l];
        const cx<T>* B = lds + sc.off_b[l];
        cx<T>* X = lds + sc.off_x[l];
        cx<T>* Tt = lds + sc.off_t[l];
        const cx<T>* E = lds + sc.off_x[l + 1];
        for (int q = tid; q < N; q += NTS) {
            const Node nd = node_of(q, W, md);
            const int c = (nd.j >> 1) * Wc + (nd.i >> 1);
            const int oi = nd.i & 1, oj = nd.j & 1;
            cx<T> v = E[c];
            if (oi | oj) v = (T)0.5 * (v + E[c + oi + oj * Wc]);
            X[q] = X[q] + v;
        }
        __syncthreads();
        for (int q = tid; q < N; q += NTS) {
            const Node nd = node_of(q, W, md);
            Tt[q] = cfma(jfac(op, nd), B[q] - apply_level(op, X, nd), X[q]);
        }
        __syncthreads();
        if (l > 0) {
            for (int q = tid; q < N; q += NTS) {
                const Node nd = node_of(q, W, md);
                X[q] = cfma(jfac(op, nd), B[q] - apply_level(op, Tt, nd), Tt[q]);
            }
            __syncthreads();
        } else {
            // the finest small level's last sweep goes straight to memory
            cx<T>* x = Xout.at(slot);
            for (int q = tid; q < N; q += NTS) {
                const Node nd = node_of(q, W, md);
                x[q] = cfma(jfac(op, nd), B[q] - apply_level(op, Tt, nd), Tt[q]);
            }
        }
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
