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

// Every neighbour is loaded first (an absent one at the centre's address),
// so that the 27 loads are in flight together; the 1D factors of an absent
// neighbour are zero, so its weight vanishes.
template <typename T, typename TI>
__device__ __forceinline__ cx<T> apply3_general(const Op3<T>& op, const cx<TI>* x, int i, int j,
                                                int l, long long t, long long sy, long long sz,
                                                cx<T>* diag) {
    const int n = op.n;
    cx<T> v[27];
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const bool in = (l + dz >= 0) & (l + dz <= n) & (j + dy >= 0) & (j + dy <= n) &
                                (i + dx >= 0) & (i + dx <= n);
                v[(dz + 1) * 9 + (dy + 1) * 3 + dx + 1] = ld3<T>(x, in ? t + dz * sz + dy * sy + dx : t);
            }
    const Line3<T> fx = line_factors<T>(i, n, op.h);
    const Line3<T> fy = line_factors<T>(j, n, op.h);
    const Line3<T> fz = line_factors<T>(l, n, op.h);
    cx<T> acc = mk((T)0, (T)0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
                acc = cfma(weight3(op, fx, fy, fz, dx, dy, dz), v[(dz + 1) * 9 + (dy + 1) * 3 + dx + 1], acc);
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
    if (MODE == MODE_JACOBI0 || (MODE == MODE_PRES && !X.base)) {
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
    } else if (MODE == MODE_PRES || MODE == MODE_PAPPLY) {
        const cx<T> f = interior ? op.odC : cdiv(mk(op.omega, (T)0), d);
        y[t] = f * (MODE == MODE_PRES ? B.at(slot)[t] - lx : lx);
    } else {
        cx<T> r = B.at(slot)[t] - lx;
        cx<T> f = interior ? op.odC : cdiv(mk(op.omega, (T)0), d);
        y[t] = cfma(f, r, ld3<T>(x, t));
    }
}

// The same operator passes as k_stencil3d (APPLY, RESID, JACOBI) on the
// interior nodes of a large level, marching along z through a 64 x 4
// column tile of the mesh (one thread per (i, j), a segment of TZ output
// planes per workgroup).  Each plane of x is read once into a
// double-buffered LDS plane with a one-node halo (the next plane requested
// from memory while this one is used) and reduced per column to three
// in-plane sums: the node, its 4 edge-adjacent and its 4 diagonal
// neighbours.  A sliding window of these sums over three planes gives the
// 27-point apply as centre (plane l), faces (plane l's edge sum + the nodes
// of planes l +- 1), edges (plane l's diagonal sum + the edge sums of planes
// l +- 1) and corners (the diagonal sums of planes l +- 1).  The boundary
// nodes are left to k_stencil3d_bnd.
constexpr int TX = 64, TY = 4, TZ = 32;  // columns per tile (x by y) and planes per segment
constexpr int TILE_MIN_N = 128;  // smallest level run with the column-tile kernel

template <typename T, typename TI, int MODE, int TX = helm::TX, int TY = helm::TY, int TZ = helm::TZ>
__global__ __launch_bounds__(BS) void k_stencil3d_tile(Op3<T> op, T s, Vec<const cx<TI>> X,
                                                       Vec<const cx<T>> B, Vec<cx<T>> Y,
                                                       int tiles_x, int tiles_y, int segs) {
    constexpr int PW = TX + 2, PH = TY + 2, PN = PW * PH;
    static_assert(TX * TY == BS, "one thread per column of the tile");
    static_assert(PN <= 2 * BS, "two staged values per thread cover a plane");
    __shared__ cx<T> pl[2][PH][PW];
    unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const unsigned per_slot = (unsigned)(tiles_x * tiles_y * segs);
    const int slot = (int)(b / per_slot);
    b %= per_slot;
    const int seg = (int)(b % (unsigned)segs);
    b /= (unsigned)segs;
    const int ty = (int)(b % (unsigned)tiles_y), tx = (int)(b / (unsigned)tiles_y);
    const int n = op.n;
    const long long sy = n + 1, sz = sy * sy;
    const int li = threadIdx.x % TX, lj = threadIdx.x / TX;
    const int i = tx * TX + li, j = ty * TY + lj;
    // output planes [l0, l1): the interior planes of this segment
    const int l0 = max(seg * TZ, 1), l1 = min(seg * TZ + TZ, n);
    const cx<TI>* x = X.at(slot);
    const cx<T>* bv = B.at(slot);
    cx<T>* y = Y.at(slot);
    // the two halo values this thread stages per plane (clamped into the
    // mesh; interior nodes see only mesh nodes)
    long long off[2];
    int hi[2], hj[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int q = min((int)threadIdx.x + u * BS, PN - 1);
        hi[u] = q % PW;
        hj[u] = q / PW;
        const int gi = min(max(tx * TX + hi[u] - 1, 0), n), gj = min(max(ty * TY + hj[u] - 1, 0), n);
        off[u] = (long long)gj * sy + gi;
    }
    const bool second = (int)threadIdx.x + BS < PN;
    const bool inner = (i > 0) & (i < n) & (j > 0) & (j < n);
    const long long col = (long long)min(j, n) * sy + min(i, n);  // this thread's column (clamped)
    const bool needb = MODE != MODE_APPLY;
    const cx<T> z = mk((T)0, (T)0);
    cx<T> v0 = z, v1 = z, bn = z;
    auto fetch = [&](int p) {  // plane p of x, and b at (i, j, p - 1)
        const long long base = (long long)min(max(p, 0), n) * sz;
        v0 = cvt<T>(x[base + off[0]]);
        if (second) v1 = cvt<T>(x[base + off[1]]);
        if (needb) bn = bv[(long long)min(max(p - 1, 0), n) * sz + col];
    };
    fetch(l0 - 1);
    pl[0][hj[0]][hi[0]] = v0;
    if (second) pl[0][hj[1]][hi[1]] = v1;
    fetch(l0);
    cx<T> a0m = z, a1m = z, a2m = z, a0c = z, a1c = z, a2c = z;  // sums of planes p-2, p-1
    cx<T> bc = z;                                                 // b at the output node
    int k = 0;
    for (int p = l0 - 1; p <= l1; ++p) {
        __syncthreads();
        // stage plane p + 1 (requested one step ago) into the other buffer
        // after this step's reads of it have been fenced by the barrier
        const cx<T> s0 = v0, s1 = v1, bnext = bn;
        if (p + 2 <= l1) fetch(p + 2);
        const cx<T>(*pc)[PW] = pl[k];
        const cx<T> a0 = pc[lj + 1][li + 1];
        const cx<T> a1 = (pc[lj + 1][li] + pc[lj + 1][li + 2]) + (pc[lj][li + 1] + pc[lj + 2][li + 1]);
        const cx<T> a2 = (pc[lj][li] + pc[lj][li + 2]) + (pc[lj + 2][li] + pc[lj + 2][li + 2]);
        const int l = p - 1;  // output plane: window p-2, p-1, p
        if (inner && l >= l0 && l < l1) {
            const long long t = (long long)l * sz + col;
            const cx<T> f = a1c + (a0m + a0);
            const cx<T> e = a2c + (a1m + a1);
            const cx<T> c3 = a2m + a2;
            const cx<T> lx = cfma(op.wInt[3], c3, cfma(op.wInt[2], e, cfma(op.wInt[1], f, op.wInt[0] * a0c)));
            if (MODE == MODE_APPLY) y[t] = lx;
            else if (MODE == MODE_RESID) y[t] = s * (bc - lx);
            else y[t] = cfma(op.odC, bc - lx, a0c);
        }
        a0m = a0c;
        a1m = a1c;
        a2m = a2c;
        a0c = a0;
        a1c = a1;
        a2c = a2;
        bc = bnext;
        if (p + 1 <= l1) {
            pl[k ^ 1][hj[0]][hi[0]] = s0;
            if (second) pl[k ^ 1][hj[1]][hi[1]] = s1;
        }
        k ^= 1;
    }
}

// The boundary nodes of a level (the planes l = 0 and l = n, then the ring
// i in {0, n} or j in {0, n} of every other plane), one thread each, with
// the general tensor-product row.
template <typename T, typename TI, int MODE>
__global__ __launch_bounds__(BS) void k_stencil3d_bnd(Op3<T> op, T s, Vec<const cx<TI>> X,
                                                      Vec<const cx<T>> B, Vec<cx<T>> Y,
                                                      long long NB, unsigned gx) {
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    const int slot = lin / gx;
    const long long q = (long long)(lin % gx) * BS + threadIdx.x;
    if (q >= NB) return;
    const int n = op.n, W = n + 1;
    const long long sy = W, sz = sy * sy, plane = (long long)W * W, ring = 4LL * W - 4;
    int i, j, l;
    if (q < 2 * plane) {
        l = q < plane ? 0 : n;
        const long long r = q < plane ? q : q - plane;
        j = (int)(r / W);
        i = (int)(r - (long long)j * W);
    } else {
        const long long r = q - 2 * plane;
        l = 1 + (int)(r / ring);
        const int e = (int)(r - (long long)(l - 1) * ring);
        if (e < W) {
            j = 0;
            i = e;
        } else if (e < 2 * W) {
            j = n;
            i = e - W;
        } else if (e < 3 * W - 2) {
            i = 0;
            j = e - 2 * W + 1;
        } else {
            i = n;
            j = e - (3 * W - 2) + 1;
        }
    }
    const long long t = (long long)l * sz + (long long)j * sy + i;
    cx<T> d;
    const cx<T> lx = apply3_general<T, TI>(op, X.at(slot), i, j, l, t, sy, sz, &d);
    cx<T>* y = Y.at(slot);
    if (MODE == MODE_APPLY) {
        y[t] = lx;
    } else if (MODE == MODE_RESID) {
        y[t] = s * (B.at(slot)[t] - lx);
    } else {
        y[t] = cfma(cdiv(mk(op.omega, (T)0), d), B.at(slot)[t] - lx, ld3<T>(X.at(slot), t));
    }
}

// Transfers run one thread per node of a plane: blockIdx.y is the plane
// (and slot), blockIdx.x * BS + threadIdx.x the node within the plane, so
// no thread divides a 64-bit index.

// b_c = P^T r for trilinear P: weights 1 (even offset) or 1/2 (odd) per
// axis.  The 27 fine values are requested together (absent ones at the
// centre's address, weight zero).
template <typename T>
__global__ __launch_bounds__(BS) void k_restrict3d(int n, Vec<const cx<T>> R, Vec<cx<T>> Bc) {
    const int nc = n / 2, Wc = nc + 1, W = n + 1;
    const int slot = blockIdx.y / Wc, L = blockIdx.y % Wc;
    const int q = blockIdx.x * BS + threadIdx.x;
    if (q >= Wc * Wc) return;
    const int J = q / Wc, I = q - J * Wc;
    const long long sy = W, sz = (long long)W * W;
    const long long tc = (long long)(2 * L) * sz + (long long)(2 * J) * sy + 2 * I;
    const cx<T>* r = R.at(slot);
    cx<T> v[27];
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const bool in = (2 * L + dz >= 0) & (2 * L + dz <= n) & (2 * J + dy >= 0) &
                                (2 * J + dy <= n) & (2 * I + dx >= 0) & (2 * I + dx <= n);
                v[(dz + 1) * 9 + (dy + 1) * 3 + dx + 1] = r[in ? tc + dz * sz + dy * sy + dx : tc];
            }
    cx<T> acc = mk((T)0, (T)0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                const bool in = (2 * L + dz >= 0) & (2 * L + dz <= n) & (2 * J + dy >= 0) &
                                (2 * J + dy <= n) & (2 * I + dx >= 0) & (2 * I + dx <= n);
                const T w = in ? (dx ? (T)0.5 : (T)1) * (dy ? (T)0.5 : (T)1) * (dz ? (T)0.5 : (T)1) : (T)0;
                acc = acc + w * v[(dz + 1) * 9 + (dy + 1) * 3 + dx + 1];
            }
    Bc.at(slot)[(long long)L * Wc * Wc + q] = acc;
}

// x += P e (trilinear interpolation from the n/2 mesh)
template <typename T>
__global__ __launch_bounds__(BS) void k_prolong3d(int n, Vec<const cx<T>> E, Vec<cx<T>> X) {
    const int W = n + 1, nc = n / 2, Wc = nc + 1;
    const int slot = blockIdx.y / W, l = blockIdx.y % W;
    const int q = blockIdx.x * BS + threadIdx.x;
    if (q >= W * W) return;
    const int j = q / W, i = q - j * W;
    const int I = i >> 1, J = j >> 1, L = l >> 1;
    const int oi = i & 1, oj = j & 1, ol = l & 1;
    const long long syc = Wc, szc = (long long)Wc * Wc;
    const cx<T>* e = E.at(slot);
    // the (up to eight) coarse corners of the cell holding the node; an odd
    // offset on an axis takes both ends of that axis with weight one half
    const long long c0 = (long long)L * szc + (long long)J * syc + I;
    const long long dxo = oi, dyo = oj * syc, dzo = ol * szc;
    const cx<T> v000 = e[c0], v100 = e[c0 + dxo], v010 = e[c0 + dyo], v110 = e[c0 + dxo + dyo];
    const cx<T> v001 = e[c0 + dzo], v101 = e[c0 + dxo + dzo], v011 = e[c0 + dyo + dzo],
                v111 = e[c0 + dxo + dyo + dzo];
    const cx<T> sum = ((v000 + v100) + (v010 + v110)) + ((v001 + v101) + (v011 + v111));
    // each distinct corner appears 8 / 2^(oi+oj+ol) times in the sum, so
    // sum / 8 is their mean (the scalings by powers of two are exact)
    cx<T>* x = X.at(slot);
    const long long t = (long long)l * W * W + q;
    x[t] = x[t] + (T)0.125 * sum;
}

inline unsigned blocks(long long N) { return (unsigned)((N + BS - 1) / BS); }

}  // namespace

template <typename T, typename TI>
void stencil3d(hipStream_t st, const Op3<T>& op, int mode, T s, Vec<const cx<TI>> X,
               Vec<const cx<T>> B, Vec<cx<T>> Y, int nslots, bool tiled_ok) {
    const long long N = (long long)(op.n + 1) * (op.n + 1) * (op.n + 1);
    const unsigned gx = blocks(N);
    const int tiles_x = (op.n + 1 + TX - 1) / TX, tiles_y = (op.n + 1 + TY - 1) / TY;
    const int segs = (op.n + 1 + TZ - 1) / TZ;
    const dim3 tgrid((unsigned)(tiles_x * tiles_y * segs * nslots));
    const long long W = op.n + 1, NB = 2 * W * W + (W - 2) * (4 * W - 4);
    const unsigned gb = blocks(NB);
    // the column-tile kernel on levels large enough to fill the chip with
    // tiles; below that, one thread per node
    const bool tiled = tiled_ok && op.n >= TILE_MIN_N;
#define HELM_S3(M)                                                                                  \
    do {                                                                                            \
        if (tiled) {                                                                                \
            k_stencil3d_tile<T, TI, M><<<tgrid, BS, 0, st>>>(op, s, X, B, Y, tiles_x, tiles_y, segs);   \
            k_stencil3d_bnd<T, TI, M><<<gb * nslots, BS, 0, st>>>(op, s, X, B, Y, NB, gb);          \
        } else {                                                                                    \
            k_stencil3d<T, TI, M><<<dim3(gx * nslots), BS, 0, st>>>(op, s, X, B, Y, N, gx);         \
        }                                                                                           \
    } while (0)
    switch (mode) {
        case MODE_APPLY: HELM_S3(MODE_APPLY); break;
        case MODE_RESID: HELM_S3(MODE_RESID); break;
        case MODE_JACOBI: HELM_S3(MODE_JACOBI); break;
        case MODE_JACOBI0:
            k_stencil3d<T, TI, MODE_JACOBI0><<<dim3(gx * nslots), BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        // the preconditioned forms (GMRES smoothing) run one thread per node
        case MODE_PRES:
            k_stencil3d<T, TI, MODE_PRES><<<dim3(gx * nslots), BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
        case MODE_PAPPLY:
            k_stencil3d<T, TI, MODE_PAPPLY><<<dim3(gx * nslots), BS, 0, st>>>(op, s, X, B, Y, N, gx);
            break;
    }
#undef HELM_S3
}

template <typename T>
void restrict3d(hipStream_t st, int n, Vec<const cx<T>> R, Vec<cx<T>> Bc, int nslots) {
    const int Wc = n / 2 + 1;
    const dim3 grid((unsigned)((Wc * Wc + BS - 1) / BS), (unsigned)(Wc * nslots));
    k_restrict3d<T><<<grid, BS, 0, st>>>(n, R, Bc);
}

template <typename T>
void prolong3d(hipStream_t st, int n, Vec<const cx<T>> E, Vec<cx<T>> X, int nslots) {
    const int W = n + 1;
    const dim3 grid((unsigned)((W * W + BS - 1) / BS), (unsigned)(W * nslots));
    k_prolong3d<T><<<grid, BS, 0, st>>>(n, E, X);
}

template void stencil3d<double, double>(hipStream_t, const Op3<double>&, int, double,
                                        Vec<const cxd>, Vec<const cxd>, Vec<cxd>, int, bool);
template void stencil3d<double, float>(hipStream_t, const Op3<double>&, int, double,
                                       Vec<const cxf>, Vec<const cxd>, Vec<cxd>, int, bool);
template void stencil3d<float, float>(hipStream_t, const Op3<float>&, int, float, Vec<const cxf>,
                                      Vec<const cxf>, Vec<cxf>, int, bool);
template void restrict3d<double>(hipStream_t, int, Vec<const cxd>, Vec<cxd>, int);
template void restrict3d<float>(hipStream_t, int, Vec<const cxf>, Vec<cxf>, int);
template void prolong3d<double>(hipStream_t, int, Vec<const cxd>, Vec<cxd>, int);
template void prolong3d<float>(hipStream_t, int, Vec<const cxf>, Vec<cxf>, int);

}  // namespace helm
