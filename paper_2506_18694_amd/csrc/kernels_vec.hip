// Vector kernels of the outer FP64 flexible GMRES and of the preconditioner
// boundary: Arnoldi inner products (deterministic two-stage reductions with
// wavefront shuffles), basis updates, norms, precision casts, and the dense
// FP64 coarsest-mesh solve.
#include "launch.h"
#include "faces.h"

namespace helm {

namespace {

constexpr int BS = 256;
constexpr int WAVE = 64;
constexpr int NPT = 4;       // nodes per thread in reductions
constexpr int GROUP = 4;     // Krylov vectors per reduction pass

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
}

// Sum `cnt` doubles per thread over the block; result valid in thread 0's
// out[] (others unspecified).  lds holds (BS / WAVE) * cnt doubles.
template <int CNT>
__device__ __forceinline__ void block_sum(double (&v)[CNT], double* lds) {
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
#pragma unroll
    for (int c = 0; c < CNT; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < CNT; ++c) lds[wv * CNT + c] = v[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < CNT; ++c) {
            double s = 0.0;
            for (int w = 0; w < BS / WAVE; ++w) s += lds[w * CNT + c];
            v[c] = s;
        }
    }
    __syncthreads();
}

// ---- coarse solve ---------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BS) void k_coarse(const cxd* __restrict__ A, int nc,
                                               Vec<const cx<T>> B, Vec<cx<T>> X, unsigned gx) {
    const int slot = blockIdx.x / gx;
    const int row = (blockIdx.x % gx) * (BS / WAVE) + threadIdx.x / WAVE;
    const int lane = threadIdx.x % WAVE;
    if (row >= nc) return;
    const cx<T>* b = B.at(slot);
    const cxd* a = A + (long long)row * nc;
    double re = 0.0, im = 0.0;
    for (int c = lane; c < nc; c += WAVE) {
        cxd bv = cvt<double>(b[c]);
        cxd av = a[c];
        re = fma(av.x, bv.x, fma(-av.y, bv.y, re));
        im = fma(av.x, bv.y, fma(av.y, bv.x, im));
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) X.at(slot)[row] = mk((T)re, (T)im);
}

// ---- elementwise ------------------------------------------------------------
template <typename TO, typename TI>
__global__ __launch_bounds__(BS) void k_copy_cast(long long N, Vec<const cx<TI>> X,
                                                  Vec<cx<TO>> Y, unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long t = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    if (t >= N) return;
    Y.at(slot)[t] = cvt<TO>(X.at(slot)[t]);
}

// Zero the nodes of the Dirichlet faces (bit f of mask: face f = 2 axis + side,
// x0 x1 y0 y1 z0 z1).  Block row y is the face, z the slot; x runs over the
// (n+1)^(dim-1) nodes of the face.
template <typename T>
__global__ __launch_bounds__(BS) void k_mask_faces(int dim, int n, unsigned mask, Vec<cx<T>> Y) {
    const int f = (int)blockIdx.y;
    if (!((mask >> f) & 1u)) return;
    const long long n1 = n + 1;
    const long long m = (long long)blockIdx.x * BS + threadIdx.x;
    if (m >= (dim == 2 ? n1 : n1 * n1)) return;
    const int axis = f >> 1;
    const long long fixed = (f & 1) ? n : 0, a = m % n1, b = m / n1;
    const long long i = axis == 0 ? fixed : a;
    const long long j = axis == 1 ? fixed : (axis == 0 ? a : b);
    const long long l = axis == 2 ? fixed : b;
    Y.at((int)blockIdx.z)[i + n1 * (j + n1 * l)] = mk((T)0, (T)0);
}

template <typename T>
__global__ __launch_bounds__(BS) void k_axpy1(long long N, T alpha, Vec<const cx<T>> X,
                                              Vec<cx<T>> Y, unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long t = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    if (t >= N) return;
    cx<T>* y = Y.at(slot);
    y[t] = y[t] + alpha * X.at(slot)[t];
}

__global__ __launch_bounds__(BS) void k_scale_inv(long long N, Vec<const cxd> X, Vec<cxd> Y,
                                                  const double* div, int dstride, unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long t = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    if (t >= N) return;
    const double d = div[slot * dstride];
    const double s = d != 0.0 ? 1.0 / d : 0.0;
    Y.at(slot)[t] = s * X.at(slot)[t];
}

__global__ __launch_bounds__(BS) void k_real_to_complex(long long N, const double* f, cxd* b,
                                                        unsigned gx) {
    const int slot = blockIdx.x / gx;
    const long long t = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    if (t >= N) return;
    b[slot * N + t] = mk(f[slot * N + t], 0.0);
}

// ---- Arnoldi reductions -------------------------------------------------------
// part[(slot * m + i) * nblk + blk] = sum over the block's nodes of conj(V_i) w;
// with wpart, also wpart[slot * nblk + blk] = the block's sum of |w|^2; with
// flag, slots whose flag is 0 are skipped
__global__ __launch_bounds__(BS) void k_multidot(long long N, int m, const int* mlen,
                                                 Vec<const cxd> V, Vec<const cxd> W, cxd* part,
                                                 unsigned nblk, double* wpart, const int* flag) {
    __shared__ double lds[(BS / WAVE) * 2 * GROUP];
    const int slot = blockIdx.x / nblk;
    const unsigned blk = blockIdx.x % nblk;
    if (flag && !flag[slot]) return;  // uniform over the block
    const long long base = (long long)blk * BS * NPT + threadIdx.x;
    const cxd* w = W.at(slot);
    const cxd* v0 = V.at(slot);
    cxd wv[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        long long t = base + (long long)q * BS;
        wv[q] = t < N ? w[t] : mk(0.0, 0.0);
    }
    const int ms = mlen ? mlen[slot] : m;  // this slot's vector count (<= m)
    for (int i0 = 0; i0 < ms; i0 += GROUP) {
        double acc[2 * GROUP];
#pragma unroll
        for (int c = 0; c < 2 * GROUP; ++c) acc[c] = 0.0;
#pragma unroll
        for (int u = 0; u < GROUP; ++u) {
            if (i0 + u < ms) {
                const cxd* v = v0 + (long long)(i0 + u) * N;
#pragma unroll
                for (int q = 0; q < NPT; ++q) {
                    long long t = base + (long long)q * BS;
                    if (t < N) {
                        cxd p = cjmul(v[t], wv[q]);
                        acc[2 * u] += p.x;
                        acc[2 * u + 1] += p.y;
                    }
                }
            }
        }
        block_sum<2 * GROUP>(acc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int u = 0; u < GROUP; ++u)
                if (i0 + u < ms)
                    part[((long long)slot * m + i0 + u) * nblk + blk] = mk(acc[2 * u], acc[2 * u + 1]);
        }
    }
    if (wpart) {
        double acc[1] = {0.0};
#pragma unroll
        for (int q = 0; q < NPT; ++q) acc[0] += wv[q].x * wv[q].x + wv[q].y * wv[q].y;
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) wpart[(long long)slot * nblk + blk] = acc[0];
    }
}

// Second classical Gram-Schmidt pass needed?  With h = V^H w from the first
// pass and V orthonormal, |w - V h|^2 = |w|^2 - |h|^2.  One pass leaves w'
// orthogonal to V up to about eps |w| / |w'| (the "twice is enough"
// argument of Kahan and Parlett), so the pass is repeated when |w'| < eta |w|
// with eta^2 = REORTH_ETA2 (eta ~ 1/7: at most ~7 eps after one pass), and
// also when the sums are not finite.
constexpr double REORTH_ETA2 = 0.02;
__global__ __launch_bounds__(BS) void k_reorth_flag(int m, const int* mlen, int nblk,
                                                    const double* wpart, const cxd* h, int hstride,
                                                    int* flag) {
    __shared__ double lds[(BS / WAVE) * 2];
    const int slot = blockIdx.x;
    const int ms = mlen ? mlen[slot] : m;
    double acc[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += BS) acc[0] += wpart[(long long)slot * nblk + b];
    for (int i = threadIdx.x; i < ms; i += BS) {
        const cxd v = h[(long long)slot * hstride + i];
        acc[1] += v.x * v.x + v.y * v.y;
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) flag[slot] = (acc[1] <= (1.0 - REORTH_ETA2) * acc[0]) ? 0 : 1;
}

// one block per (slot, i): out = sum over blocks, fixed order; with flag,
// slots whose flag is 0 get out = 0 (or keep out when accumulating)
__global__ __launch_bounds__(BS) void k_reduce_parts(int m, const int* mlen, int nblk,
                                                     const cxd* part, cxd* out, int ostride,
                                                     int accumulate, const int* flag) {
    __shared__ double lds[(BS / WAVE) * 2];
    const int slot = blockIdx.x / m, i = blockIdx.x % m;
    if (mlen && i >= mlen[slot]) return;  // uniform over the block
    if (flag && !flag[slot]) {
        if (threadIdx.x == 0 && !accumulate) out[(long long)slot * ostride + i] = mk(0.0, 0.0);
        return;
    }
    const cxd* p = part + ((long long)slot * m + i) * nblk;
    double acc[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nblk; b += BS) {
        acc[0] += p[b].x;
        acc[1] += p[b].y;
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        cxd* o = out + (long long)slot * ostride + i;
        cxd r = mk(acc[0], acc[1]);
        *o = accumulate ? (*o + r) : r;
    }
}

__global__ __launch_bounds__(BS) void k_norm2(long long N, Vec<const cxd> W, double* part,
                                              unsigned nblk) {
    __shared__ double lds[BS / WAVE];
    const int slot = blockIdx.x / nblk;
    const unsigned blk = blockIdx.x % nblk;
    const long long base = (long long)blk * BS * NPT + threadIdx.x;
    const cxd* w = W.at(slot);
    double acc[1] = {0.0};
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        long long t = base + (long long)q * BS;
        if (t < N) {
            cxd v = w[t];
            acc[0] += v.x * v.x + v.y * v.y;
        }
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[(long long)slot * nblk + blk] = acc[0];
}

__global__ __launch_bounds__(BS) void k_norm2_final(int nblk, const double* part, double* out,
                                                    int ostride) {
    __shared__ double lds[BS / WAVE];
    const int slot = blockIdx.x;
    double acc[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += BS) acc[0] += part[(long long)slot * nblk + b];
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) out[(long long)slot * ostride] = sqrt(acc[0]);
}

// w -= sum_i h_i V_i   (h from device memory, staged in LDS); with flag,
// slots whose flag is 0 are skipped
__global__ __launch_bounds__(BS) void k_multi_axpy(long long N, int m, const int* mlen,
                                                   Vec<const cxd> V, const cxd* h, int hstride,
                                                   Vec<cxd> W, unsigned gx, const int* flag) {
    extern __shared__ cxd hs[];
    const int slot = blockIdx.x / gx;
    if (flag && !flag[slot]) return;  // uniform over the block
    const int ms = mlen ? mlen[slot] : m;
    for (int i = threadIdx.x; i < ms; i += BS) hs[i] = h[(long long)slot * hstride + i];
    __syncthreads();
    const long long t = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    if (t >= N) return;
    const cxd* v = V.at(slot);
    cxd acc = mk(0.0, 0.0);
    for (int i = 0; i < ms; ++i) acc = cfma(hs[i], v[(long long)i * N + t], acc);
    cxd* w = W.at(slot);
    w[t] = w[t] - acc;
}

template <typename TZ>
__global__ __launch_bounds__(BS) void k_update_solution(long long N, int m, const int* mlen,
                                                        Vec<const cx<TZ>> Z, const cxd* y,
                                                        int ystride, Vec<cxd> X, unsigned gx) {
    extern __shared__ cxd ys[];
    const int slot = blockIdx.x / gx;
    const int ms = mlen ? mlen[slot] : m;
    for (int i = threadIdx.x; i < ms; i += BS) ys[i] = y[(long long)slot * ystride + i];
    __syncthreads();
    const long long t = (long long)(blockIdx.x % gx) * BS + threadIdx.x;
    if (t >= N) return;
    const cx<TZ>* z = Z.at(slot);
    cxd acc = mk(0.0, 0.0);
    for (int i = 0; i < ms; ++i) acc = cfma(ys[i], cvt<double>(z[(long long)i * N + t]), acc);
    cxd* x = X.at(slot);
    x[t] = x[t] + acc;
}

// The small least-squares problem of m-step GMRES, one thread per slot:
// minimise |beta e_1 - H y| over y in C^m for the (m+1) x m upper
// Hessenberg H whose column j holds rows 0..j at hu[slot*hs + j*(m+1) + i]
// (complex) and the subdiagonal h_{j+1,j} = hn[slot*(m+1) + j + 1] (real),
// beta = hn[slot*(m+1)].  Givens rotations reduce H to upper triangular
// form in place; back substitution gives y[slot*m + i].  A zero pivot (an
// invariant Krylov space, or beta = 0) gives y_i = 0 for that column.
constexpr int LSQ_MAX = 20;
__global__ __launch_bounds__(WAVE) void k_gmres_lsq(int m, cxd* hu, int hs, const double* hn,
                                                    cxd* y, int nslots) {
    const int slot = blockIdx.x * WAVE + threadIdx.x;
    if (slot >= nslots) return;
    cxd* H = hu + (long long)slot * hs;
    const double* sub = hn + (long long)slot * (m + 1);
    cxd g[LSQ_MAX + 1], cs[LSQ_MAX], sn[LSQ_MAX];
    g[0] = mk(sub[0], 0.0);
    for (int j = 0; j < m; ++j) {
        cxd* col = H + (long long)j * (m + 1);
        for (int i = 0; i < j; ++i) {
            const cxd a = col[i], b = col[i + 1];
            col[i] = cs[i] * a + sn[i] * b;
            col[i + 1] = mk(-sn[i].x, sn[i].y) * a + mk(cs[i].x, -cs[i].y) * b;
        }
        const cxd a = col[j];
        const double b = sub[j + 1];
        const double den = sqrt(a.x * a.x + a.y * a.y + b * b);
        if (den == 0.0) {
            cs[j] = mk(1.0, 0.0);
            sn[j] = mk(0.0, 0.0);
        } else {
            cs[j] = mk(a.x / den, -a.y / den);
            sn[j] = mk(b / den, 0.0);
            col[j] = mk(den, 0.0);
        }
        g[j + 1] = mk(-sn[j].x, sn[j].y) * g[j];
        g[j] = cs[j] * g[j];
    }
    cxd* ys = y + (long long)slot * m;
    for (int i = m - 1; i >= 0; --i) {
        cxd s = g[i];
        for (int q = i + 1; q < m; ++q) s = s - H[(long long)q * (m + 1) + i] * ys[q];
        const cxd d = H[(long long)i * (m + 1) + i];
        ys[i] = (d.x == 0.0 && d.y == 0.0) ? mk(0.0, 0.0) : cdiv(s, d);
    }
}

inline unsigned blocks(long long N) { return (unsigned)((N + BS - 1) / BS); }

}  // namespace

int multidot_blocks(long long N) { return (int)((N + (long long)BS * NPT - 1) / ((long long)BS * NPT)); }

template <typename T>
void coarse_apply(hipStream_t st, const cxd* Ainv, int nc, Vec<const cx<T>> B, Vec<cx<T>> X,
                  int nslots) {
    const unsigned gx = (nc + BS / WAVE - 1) / (BS / WAVE);
    k_coarse<T><<<gx * nslots, BS, 0, st>>>(Ainv, nc, B, X, gx);
}

template <typename TO, typename TI>
void copy_cast(hipStream_t st, long long N, Vec<const cx<TI>> X, Vec<cx<TO>> Y, int nslots) {
    const unsigned gx = blocks(N);
    k_copy_cast<TO, TI><<<gx * nslots, BS, 0, st>>>(N, X, Y, gx);
}

template <typename T>
void mask_faces(hipStream_t st, int dim, int n, unsigned mask, Vec<cx<T>> Y, int nslots) {
    if (mask == 0 || nslots < 1) return;
    const long long per = dim == 2 ? (long long)(n + 1) : (long long)(n + 1) * (n + 1);
    const dim3 grid(blocks(per), 2 * dim, nslots);
    k_mask_faces<T><<<grid, BS, 0, st>>>(dim, n, mask, Y);
}

template <typename T>
void axpy1(hipStream_t st, long long N, T alpha, Vec<const cx<T>> X, Vec<cx<T>> Y, int nslots) {
    const unsigned gx = blocks(N);
    k_axpy1<T><<<gx * nslots, BS, 0, st>>>(N, alpha, X, Y, gx);
}

void scale_inv(hipStream_t st, long long N, Vec<const cxd> X, Vec<cxd> Y, const double* div,
               int div_stride, int nslots) {
    const unsigned gx = blocks(N);
    k_scale_inv<<<gx * nslots, BS, 0, st>>>(N, X, Y, div, div_stride, gx);
}

void gmres_lsq(hipStream_t st, int m, cxd* hu, int hs, const double* hn, cxd* y, int nslots) {
    k_gmres_lsq<<<(unsigned)((nslots + WAVE - 1) / WAVE), WAVE, 0, st>>>(m, hu, hs, hn, y, nslots);
}

void real_to_complex(hipStream_t st, long long N, const double* f, cxd* b, int nslots) {
    const unsigned gx = blocks(N);
    k_real_to_complex<<<gx * nslots, BS, 0, st>>>(N, f, b, gx);
}

void multidot(hipStream_t st, long long N, int m, const int* mlen, Vec<const cxd> V,
              Vec<const cxd> W, cxd* part, int nslots, double* wpart, const int* flag) {
    const unsigned nblk = multidot_blocks(N);
    k_multidot<<<nblk * nslots, BS, 0, st>>>(N, m, mlen, V, W, part, nblk, wpart, flag);
}

void reduce_parts(hipStream_t st, int m, const int* mlen, int nblk, const cxd* part, cxd* out,
                  int ostride, int accumulate, int nslots, const int* flag) {
    k_reduce_parts<<<m * nslots, BS, 0, st>>>(m, mlen, nblk, part, out, ostride, accumulate, flag);
}

void reorth_flag(hipStream_t st, int m, const int* mlen, int nblk, const double* wpart,
                 const cxd* h, int hstride, int* flag, int nslots) {
    k_reorth_flag<<<nslots, BS, 0, st>>>(m, mlen, nblk, wpart, h, hstride, flag);
}

void multi_axpy(hipStream_t st, long long N, int m, const int* mlen, Vec<const cxd> V,
                const cxd* h, int hstride, Vec<cxd> W, int nslots, const int* flag) {
    const unsigned gx = blocks(N);
    k_multi_axpy<<<gx * nslots, BS, sizeof(cxd) * m, st>>>(N, m, mlen, V, h, hstride, W, gx, flag);
}

void norm2(hipStream_t st, long long N, Vec<const cxd> W, double* part, double* out, int ostride,
           int nslots) {
    const unsigned nblk = multidot_blocks(N);
    k_norm2<<<nblk * nslots, BS, 0, st>>>(N, W, part, nblk);
    k_norm2_final<<<nslots, BS, 0, st>>>(nblk, part, out, ostride);
}

template <typename TZ>
void update_solution(hipStream_t st, long long N, int m, const int* mlen, Vec<const cx<TZ>> Z,
                     const cxd* y, int ystride, Vec<cxd> X, int nslots) {
    const unsigned gx = blocks(N);
    k_update_solution<TZ><<<gx * nslots, BS, sizeof(cxd) * m, st>>>(N, m, mlen, Z, y, ystride, X,
                                                                     gx);
}

template void coarse_apply<double>(hipStream_t, const cxd*, int, Vec<const cxd>, Vec<cxd>, int);
template void coarse_apply<float>(hipStream_t, const cxd*, int, Vec<const cxf>, Vec<cxf>, int);
template void copy_cast<double, double>(hipStream_t, long long, Vec<const cxd>, Vec<cxd>, int);
template void copy_cast<float, double>(hipStream_t, long long, Vec<const cxd>, Vec<cxf>, int);
template void copy_cast<double, float>(hipStream_t, long long, Vec<const cxf>, Vec<cxd>, int);
template void copy_cast<float, float>(hipStream_t, long long, Vec<const cxf>, Vec<cxf>, int);
template void mask_faces<double>(hipStream_t, int, int, unsigned, Vec<cxd>, int);
template void mask_faces<float>(hipStream_t, int, int, unsigned, Vec<cxf>, int);
template void axpy1<double>(hipStream_t, long long, double, Vec<const cxd>, Vec<cxd>, int);
template void axpy1<float>(hipStream_t, long long, float, Vec<const cxf>, Vec<cxf>, int);
template void update_solution<double>(hipStream_t, long long, int, const int*, Vec<const cxd>,
                                      const cxd*, int, Vec<cxd>, int);
template void update_solution<float>(hipStream_t, long long, int, const int*, Vec<const cxf>,
                                     const cxd*, int, Vec<cxd>, int);

}  // namespace helm
