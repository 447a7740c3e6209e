// Fused z-marching passes for the 3D Q1 levels.
//
// Every operator a K + b M + c M_Gamma on the uniform hexahedral mesh is a
// sum of tensor products of the 1D linear-element rows (K1 = (1/h)[-1 2 -1],
// M1 = (h/6)[1 4 1]; a boundary row halves the centre; E = 1 on the end
// nodes):
//   K = K1 M1 M1 + M1 K1 M1 + M1 M1 K1,  M = M1 M1 M1,
//   M_Gamma = E M1 M1 + M1 E M1 + M1 M1 E.
// With the values outside the mesh taken as zero, the row of node (i, j, l)
// splits into in-plane parts and one 1D pass along z.  Per plane p of the
// node's column the in-plane sums
//   a0 = x(i, j),  H = x(i-1, j) + x(i+1, j),  V = x(i, j-1) + x(i, j+1),
//   a2 = the four diagonal neighbours
// give, with the node's x and y factors (halved centres on a boundary
// line),
//   PMM = (M1 M1) x,  PK = (K1 M1 + M1 K1) x,  PG = (E M1 + M1 E) x,
// and the row is
//   L x (l) = T1(l-1) + T1(l+1) + T0(l)                (interior plane l)
//   L x (l) = T1(l-1) + T1(l+1) + T0(l)/2 + c PMM(l)   (l = 0 or n)
// with T1 = (h/6)(a PK + b PMM + c PG) - (a/h) PMM and
// T0 = 4 (h/6)(a PK + b PMM + c PG) + 2 (a/h) PMM.  Interior, face, edge and
// corner nodes run the same code; no separate boundary kernel is needed.
//
// One workgroup owns a tile of mesh columns and a segment of planes and
// marches up the segment.  Each plane of the input passes once through a
// double-buffered LDS plane with a one-node halo (the plane after the next
// already requested), and every dependent pass is a pipeline stage behind
// the previous one: the first stage's output plane reaches the second stage
// through a second double-buffered LDS plane, read at the next step, so that
// one barrier per step orders every plane exchange.  Passes:
//   k3_pass  one or two operator stages: apply, scaled residual, Jacobi
//            sweeps (from a guess, from the guess plus the prolonged coarse
//            correction, or from zero), the shifted-HSS residual
//            rho = c (R - B u) with the first zero-guess sweep, both
//            zero-guess sweeps in one stencil stage, and the HSS update
//            u += x or u = x on the last output
//   k3_rr    residual restriction b_c = P^T (b - L x): stage 1 forms the
//            residual plane, stage 2 applies the transpose of trilinear
//            interpolation (in-plane weights 1, 1/2, 1/4; across planes
//            1/2, 1, 1/2) on the coarse columns of the tile
#include <algorithm>
#include <type_traits>

#include "launch.h"

namespace helm {

namespace {

// A workgroup of LW x H threads stages one LW x H region of an input plane
// (one value per thread); the first stage runs on its interior
// (LW - 2) x (H - 2) columns, the second stage on the (LW - 4) x (H - 4)
// inside that.
// Tile rows by precision and level: FP64 tiles on the fine levels are
// 32 x 32 (1024 threads; those passes are bound by HBM, so the smallest
// halo share wins), FP32 tiles 32 x 16 (512 threads: its passes are bound
// by issue and the barrier per plane, and two 512-thread workgroups per CU
// overlap each other's barriers).
#ifndef HELM_K3_LH_FP64
#define HELM_K3_LH_FP64 32
#endif
#ifndef HELM_K3_LH_FP32
#define HELM_K3_LH_FP32 16
#endif
// The latency-bound coarse FP64 levels use 32 x 16 tiles as well: twice the
// workgroups, two per CU.
#ifndef HELM_K3_LH_FP64_COARSE
#define HELM_K3_LH_FP64_COARSE 16
#endif
// levels with at least this many cells per side use the full-height tile
#ifndef HELM_K3_TALL_N
#define HELM_K3_TALL_N 192
#endif
constexpr int LW = 32;            // tile columns (x)
constexpr int RC = (LW - 4) / 2;  // coarse columns per tile in the restriction
template <int LH>
struct Tile {
    static constexpr int H = LH;                // tile rows (y)
    static constexpr int FT = LW * H;           // threads per workgroup
    static constexpr int RCH = (H - 4) / 2;     // coarse rows per tile in the restriction
    static constexpr int CWH = H / 2 + 1;       // coarse rows under a tile (prolongation)
};
// tile rows of a level of n cells per side
template <typename T>
constexpr int tall_rows() { return sizeof(T) == 4 ? HELM_K3_LH_FP32 : HELM_K3_LH_FP64; }
template <typename T>
constexpr int short_rows() { return sizeof(T) == 4 ? HELM_K3_LH_FP32 : HELM_K3_LH_FP64_COARSE; }
#ifndef HELM_K3_PF
#define HELM_K3_PF 2
#endif
#ifndef HELM_K3_SPLIT
#define HELM_K3_SPLIT 1
#endif
constexpr int PF = HELM_K3_PF;  // input planes requested ahead of the one in LDS (>= 1)

// Complex values move as one vector load or store (a struct copy could be
// split in two, and a select between a load and a local zero turns into a
// load through a select of addresses, putting the zero in scratch memory).
template <typename T>
struct Vec2T;
template <>
struct Vec2T<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2T<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <typename T>
__device__ __forceinline__ cx<T> ldv(const cx<T>* p) {
    const typename Vec2T<T>::type v = *reinterpret_cast<const typename Vec2T<T>::type*>(p);
    return mk(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void stv(cx<T>* p, cx<T> a) {
    typename Vec2T<T>::type v;
    v.x = a.x;
    v.y = a.y;
    *reinterpret_cast<typename Vec2T<T>::type*>(p) = v;
}

// Selection between two complex values, one component at a time (a select
// of whole values can be turned into a load through a select of addresses
// of stack copies).
template <typename T>
__device__ __forceinline__ cx<T> csel(bool c, cx<T> a, cx<T> b) {
    return mk(c ? a.x : b.x, c ? a.y : b.y);
}

// A value at byte offset off of a plane: the plane's address is the same
// on every lane (scalar registers), off the lane's column (one 32-bit
// register), so the loads and stores take the scalar-base form.
template <typename V>
__device__ __forceinline__ cx<V> ldo(const cx<V>* plane, unsigned off) {
    return ldv(reinterpret_cast<const cx<V>*>(reinterpret_cast<const char*>(plane) + off));
}
template <typename V>
__device__ __forceinline__ void sto(cx<V>* plane, unsigned off, cx<V> a) {
    stv(reinterpret_cast<cx<V>*>(reinterpret_cast<char*>(plane) + off), a);
}

template <typename T>
__device__ __forceinline__ cx<T> c3(const cx<T>* w, cx<T> a0, cx<T> s1, cx<T> a2) {
    return cfma(w[0], a0, cfma(w[1], s1, w[2] * a2));
}

// T1, T0 of one plane (see top): the interior coefficients on (a0, H + V,
// a2), and on waves holding a boundary column the change of the 1D factors
// there (bx, by: the column lies on a boundary line),
// (A nb + C bx by) a0 + B (bx V + by H) with nb = bx + by.  On the first and
// last plane (bz, the same on every lane) T0 becomes T0 / 2 + c PMM: the
// difference is added in a branch of its own.
template <typename T>
__device__ __forceinline__ void plane_terms(const Op3F<T>& op, bool edge_wave, cx<T> a0, cx<T> H,
                                            cx<T> V, cx<T> a2, bool bx, bool by, bool bz, cx<T>& T1,
                                            cx<T>& T0) {
    const cx<T> s1 = H + V;
#if HELM_K3_SPLIT
    // real weights on (a0, s1, a2), plus i k times the mass pattern
    // 16 a0 + 4 s1 + a2 (the imaginary part of every weight is that of its
    // mass term): 20 operations instead of 24 for T1 and T0
    const T mx = fmat((T)16, a0.x, fmat((T)4, s1.x, a2.x));
    const T my = fmat((T)16, a0.y, fmat((T)4, s1.y, a2.y));
    T1 = mk(fmat(op.r1[0], a0.x, fmat(op.r1[1], s1.x, fmat(op.r1[2], a2.x, -op.k1 * my))),
            fmat(op.r1[0], a0.y, fmat(op.r1[1], s1.y, fmat(op.r1[2], a2.y, op.k1 * mx))));
    T0 = mk(fmat(op.r0[0], a0.x, fmat(op.r0[1], s1.x, fmat(op.r0[2], a2.x, -op.k0 * my))),
            fmat(op.r0[0], a0.y, fmat(op.r0[1], s1.y, fmat(op.r0[2], a2.y, op.k0 * mx))));
    if (bz)
        T0 = mk(fmat(op.rj[0], a0.x, fmat(op.rj[1], s1.x, fmat(op.rj[2], a2.x, fmat(-op.kj, my, T0.x)))),
                fmat(op.rj[0], a0.y, fmat(op.rj[1], s1.y, fmat(op.rj[2], a2.y, fmat(op.kj, mx, T0.y)))));
#else
    T1 = c3(op.i1, a0, s1, a2);
    T0 = c3(op.i0, a0, s1, a2);
    if (bz) T0 = T0 + c3(op.j0, a0, s1, a2);
#endif
    if (!edge_wave) return;
    const T nb = (T)((int)bx + (int)by), bxy = (bx && by) ? (T)1 : (T)0;
    const cx<T> w = mk((bx ? V.x : (T)0) + (by ? H.x : (T)0), (bx ? V.y : (T)0) + (by ? H.y : (T)0));
    T1 = cfma(nb * op.e1[0] + bxy * op.e1[2], a0, cfma(op.e1[1], w, T1));
    T0 = cfma(nb * op.e0[0] + bxy * op.e0[2], a0, cfma(op.e0[1], w, T0));
    if (bz) T0 = cfma(nb * op.f0[0] + bxy * op.f0[2], a0, cfma(op.f0[1], w, T0));
}

// in-plane sums at (row r, column q) of an LDS plane of LW columns
template <typename T>
__device__ __forceinline__ void plane_sums(const cx<T> (*pl)[LW], int r, int q, cx<T>& a0, cx<T>& H,
                                           cx<T>& V, cx<T>& a2) {
    a0 = pl[r][q];
    H = pl[r][q - 1] + pl[r][q + 1];
    V = pl[r - 1][q] + pl[r + 1][q];
    a2 = (pl[r - 1][q - 1] + pl[r - 1][q + 1]) + (pl[r + 1][q - 1] + pl[r + 1][q + 1]);
}

// work unit -> (slot, tile x, tile y, segment); the tiles of one segment are
// consecutive, so neighbouring tiles run on one XCD and share halo lines
__device__ __forceinline__ void unit_of(const Grid3F& g, int& slot, int& tx, int& ty, int& seg) {
    unsigned b = xcd_remap(blockIdx.x, gridDim.x);
    const unsigned tiles = (unsigned)(g.tiles_x * g.tiles_y);
    const unsigned per = tiles * (unsigned)g.segs;
    slot = (int)(b / per);
    b %= per;
    seg = (int)(b / tiles);
    b %= tiles;
    ty = (int)(b / (unsigned)g.tiles_x);
    tx = (int)(b % (unsigned)g.tiles_x);
}

// ---------------------------------------------------------------- k3_pass --
// The march is unrolled UNR steps at a time so that every ring slot is a
// fixed register: the load of a plane goes into the slot of the plane that
// the same step consumed, and no value is moved between slots.  Every load
// of the unrolled body is issued unconditionally (plane and column indices
// clamped into the mesh, the value masked where it is consumed), so the
// count of requests in flight is the same on every path.  (Moving a
// register whose load is still in flight, or merging paths that issued
// different numbers of requests, makes the step wait for every request
// outstanding, and memory returns in order, so it would wait for the
// prefetches it has just issued.)  UNR is a multiple of the ring depth and
// of the two LDS buffers; the last partial block runs guarded steps.
constexpr int UNR = 6;
static_assert(UNR % PF == 0 && UNR % 2 == 0, "unroll must cover the rings and the LDS buffers");
constexpr int CW = LW / 2 + 1;  // coarse columns under a tile (prolongation)

template <int U>
using IC = std::integral_constant<int, U>;

// FIRST (the first stage, its output lagging the input by one plane when
// it is a stencil, in step with it when pointwise):
//   F_APPLY  y = L x                             (NS = 1)
//   F_RESID  y = s (b - L x)                     (NS = 1)
//   F_JAC    x1 = x + w/D (b - L x)   (x + P e_c when PRO)
//   F_HSS    rho = s (R - B u) (written to Rho), x1 = w/D rho; B the
//            second operator, R in Bv, u in X
//   F_HSS0   rho = s R (written), x1 = w/D rho   (u = 0; pointwise)
//   F_PRE0   x1 = w/D b                          (pointwise)
//   F_JAC0   x1 = x0 + w/D (b - L x0) with x0 = w/D b: the two zero-guess
//            sweeps, the first formed on each input plane as it is staged
// NS = 2 adds x2 = x1 + w/D (b - L x1) (b = rho for the HSS forms).
// UPD: 0 y = result, 1 y += result (the HSS update u += e with u in Y).
//
// Prolongation (PRO): (P e)(i, j, l) is trilinear interpolation from the n/2
// mesh.  Each coarse plane C the tile needs is staged once in LDS (the
// CW x CW coarse columns under the tile) and interpolated in-plane to every
// fine column, ce(C) = sum of the four coarse corners of the column (with
// repeats where a coordinate is even); a fine plane 2C takes ce(C) / 4 and
// 2C + 1 takes (ce(C) + ce(C + 1)) / 8 (exact powers of two).  The coarse
// plane for fine step p is written to LDS one step ahead and requested two
// steps ahead of that; the march then starts on an even plane.
template <typename T, typename TI, int FIRST, int NS, bool PRO, int UPD, int TH, bool DIR>
__global__ __launch_bounds__(Tile<TH>::FT) void k3_pass(Op3F<T> L, Op3F<T> B, T s, Vec<const cx<TI>> X,
                                              Vec<const cx<T>> Bv, Vec<const cx<T>> Ec,
                                              Vec<cx<T>> Rho, Vec<cx<T>> Y, Grid3F g) {
    constexpr bool PW = FIRST == F_HSS0 || FIRST == F_PRE0;
    constexpr bool HSS = FIRST == F_HSS || FIRST == F_HSS0;
    constexpr int LH = Tile<TH>::H, CWH = Tile<TH>::CWH;
    constexpr int OWN = LW - 2 * NS, OWNH = LH - 2 * NS;  // owned columns and rows of a tile
    static_assert(!(PRO && PW), "the prolongation feeds a stencil first stage");
    __shared__ cx<T> pin[2][LH][LW];
    __shared__ cx<T> pmid[NS == 2 ? 2 : 1][LH][LW];
    __shared__ cx<T> cpl[PRO ? 2 : 1][PRO ? CWH : 1][PRO ? CW : 1];
    int slot, tx, ty, seg;
    unit_of(g, slot, tx, ty, seg);
    const int n = L.n;
    const long long sy = n + 1, sz = sy * sy;
    const int lx = (int)threadIdx.x % LW, ly = (int)threadIdx.x / LW;
    const int i0 = tx * OWN - NS, j0 = ty * OWNH - NS;  // first column of the tile
    const int i = i0 + lx, j = j0 + ly;                 // this thread's column
    const bool inmesh = (i >= 0) & (i <= n) & (j >= 0) & (j <= n);
    const bool st1 = (lx >= 1) & (lx < LW - 1) & (ly >= 1) & (ly < LH - 1);
    const bool st2 = (lx >= 2) & (lx < LW - 2) & (ly >= 2) & (ly < LH - 2);
    const bool owned = inmesh & (NS == 2 ? st2 : st1);
    const bool bx = (i == 0) | (i == n), by = (j == 0) | (j == n);
    const bool edge_wave = __any((int)(inmesh & (bx | by)));
    const int cxy = (int)bx + (int)by;  // boundary coordinates in x and y
    // DIR: outputs on the nodes of Dirichlet faces are zero (the column lies
    // on an x or y Dirichlet face, or the plane is a z Dirichlet face)
    const unsigned dm = DIR ? L.dir : 0u;
    const bool dcol = DIR && (((dm & 1u) && i == 0) || ((dm & 2u) && i == n) ||
                              ((dm & 4u) && j == 0) || ((dm & 8u) && j == n));
    auto dfix = [&](int l) { return dcol || ((dm & 16u) && l == 0) || ((dm & 32u) && l == n); };
    // the Jacobi factor w/D of this column on plane l, indexed by the number
    // of boundary coordinates (the same on every lane of an interior wave)
    auto odf = [&](int l) {
        const bool e = (l == 0) | (l == n);
        if (!edge_wave) return csel(e, L.od[1], L.od[0]);
        const int ix = cxy + (int)e;
        return csel(ix < 2, csel(ix == 0, L.od[0], L.od[1]), csel(ix == 2, L.od[2], L.od[3]));
    };
    const long long col = inmesh ? (long long)j * sy + i : 0;
    const unsigned ox = (unsigned)col * (unsigned)sizeof(cx<TI>), ob = (unsigned)col * (unsigned)sizeof(cx<T>);
    const int z0 = seg * g.tz, z1 = min(z0 + g.tz, n + 1);  // output planes [z0, z1)
    // vector bases (plane l at + l sz)
    constexpr bool J0 = FIRST == F_JAC0;
    const cx<TI>* xs = J0 ? reinterpret_cast<const cx<TI>*>(Bv.at(slot)) : (X.base ? X.at(slot) : nullptr);
    const cx<T>* bs = Bv.base ? Bv.at(slot) : nullptr;
    cx<T>* rs = HSS ? Rho.at(slot) : nullptr;
    cx<T>* ys = Y.at(slot);
    const cx<T> z = mk((T)0, (T)0);

    // unconditional loads at this thread's column (column 0 outside the
    // mesh), plane l clamped into [0, min(hi, n)]; masked where consumed
    auto pl = [&](int l, int hi) { return (long long)max(0, min(l, min(hi, n))) * sz; };
    auto ldx = [&](int l, int hi) { return ldo(xs + pl(l, hi), ox); };
    auto ldcol = [&](const cx<T>* p, int l, int hi) { return ldo(p + pl(l, hi), ob); };
    auto lok = [&](int l) { return inmesh && l >= 0 && l <= n; };
    // prolongation: this thread's coarse corner in the tile's LDS coarse
    // plane, and the coarse value it stages (threads 0 .. CW CWH - 1)
    const int nc = n / 2;
    const long long syc = nc + 1, szc = syc * syc;
    const int cI0 = i0 >> 1, cJ0 = j0 >> 1;  // floor: i0 may be negative
    const int ci = (i >> 1) - cI0, cj = (j >> 1) - cJ0, cdx = i & 1, cdy = j & 1;
    const int ca = (int)threadIdx.x % CW, cb = (int)threadIdx.x / CW;
    const bool cld = PRO && (int)threadIdx.x < CW * CWH;
    const bool cin = cld && cI0 + ca >= 0 && cI0 + ca <= nc && cJ0 + cb >= 0 && cJ0 + cb <= nc;
    const cx<T>* ecs = PRO ? Ec.at(slot) : nullptr;
    const unsigned oc = cin ? (unsigned)((cJ0 + cb) * syc + (cI0 + ca)) * (unsigned)sizeof(cx<T>) : 0u;
    auto ldc = [&](int C) {  // coarse values outside the coarse mesh only reach masked nodes
        return ldo(ecs + (long long)max(0, min(C, nc)) * szc, oc);
    };
    auto interp = [&](int buf) {
        return (cpl[buf][cj][ci] + cpl[buf][cj][ci + cdx]) +
               (cpl[buf][cj + cdy][ci] + cpl[buf][cj + cdy][ci + cdx]);
    };

    // the first stage outputs planes [o0, o1); a stencil first stage reads
    // input planes [o0 - 1, o1], a pointwise one [o0, o1 - 1]
    const int o0 = z0 - (NS - 1), o1 = z1 + (NS - 1);
    int p0 = PW ? o0 : o0 - 1;
    if (PRO) p0 -= p0 & 1;  // an even first plane (its output is not stored)
    // the second stage runs two planes behind the first (it reads the
    // middle plane the first stage wrote at the previous step), so the
    // march takes one step more
    const int p1 = (PW ? o1 - 1 : o1) + (NS == 2 ? 1 : 0);
    const int qb = PW ? p0 : p0 - 1;  // plane the first stage outputs at step p0
    const int qy = NS == 1 ? qb : qb - 2;  // plane the last stage outputs at step p0
    // rings: x at planes p + 1 .. p + PF, b at q1 .. q1 + PF - 1 and y at the
    // output planes of steps p .. p + PF - 1 (step p0 + u uses slot u % PF)
    cx<TI> xr[PF];
    cx<T> br[PF], yr[PF];
    cx<T> cA = z, cB = z, cr = z;  // ce of coarse planes C - 1, C; staged coarse value
    if (PRO) {
        const int m = p0 >> 1;
        if (cld) {
            cpl[m & 1][cb][ca] = ldc(m);
            cpl[(m + 1) & 1][cb][ca] = ldc(m + 1);
        }
        __syncthreads();
        cB = interp(m & 1);
        cr = ldc(m + 2);
    }
    if (!PW) {
        cx<T> v = cvt<T>(ldx(p0, p1));
        if (J0) v = odf(p0) * v;
        if (PRO) v = v + (T)0.25 * cB;
        pin[0][ly][lx] = csel(lok(p0), v, z);
    }
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        if (!PW) xr[u] = ldx(p0 + 1 + u, p1);
        if (FIRST != F_APPLY) br[u] = ldcol(bs, qb + u, o1 - 1);
        if (UPD == 1) yr[u] = ldcol(ys, qy + u, z1 - 1);
    }
    // stage 1: acc1 = T1(q - 1) + T0(q) for the next output plane q, T1p = T1(q);
    // xc: input centre of q.  Stage 2 likewise, with b2 its right-hand side.
    cx<T> acc1 = z, T1p = z, xc = z;
    cx<T> acc2 = z, U1p = z, xc2 = z, b2 = z, b2n = z;

    auto step = [&](auto uc, int p) __attribute__((always_inline)) {
        constexpr int u = decltype(uc)::value;
        constexpr int kb = u & 1;   // LDS buffer of input plane p
        constexpr int sl = u % PF;  // ring slot of this step
        const int q1 = PW ? p : p - 1;  // plane the first stage outputs at this step
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        if (!PW) {
            // input plane p + 1 into the buffer of plane p - 1 (free since the
            // barrier; past the last plane it is written and never read)
            cx<T> v = cvt<T>(xr[sl]);
            if (J0) v = odf(p + 1) * v;
            if (PRO) {
                if (kb == 0) {  // p + 1 = 2C - 1
                    cA = cB;
                    cB = interp(((p + 2) >> 1) & 1);
                    v = v + (T)0.125 * (cA + cB);
                } else {  // p + 1 = 2C
                    v = v + (T)0.25 * cB;
                }
            }
            pin[kb ^ 1][ly][lx] = csel(lok(p + 1), v, z);
            xr[sl] = ldx(p + 1 + PF, p1);
            if (PRO && kb == 1) {  // coarse plane (p + 3) / 2, needed at step p + 1
                if (cld) cpl[((p + 3) >> 1) & 1][cb][ca] = cr;
                cr = ldc((p + 5) >> 1);
            }
        }
        const cx<T> bcur = br[sl];
        if (FIRST != F_APPLY) br[sl] = ldcol(bs, q1 + PF, o1 - 1);
        const bool q1ok = inmesh && q1 >= 0 && q1 <= n && q1 >= o0;
        const cx<T> od1 = odf(q1);
        cx<T> x1 = z, bq = z;
        if (PW) {
            if (q1ok) {
                if (FIRST == F_HSS0) {
                    cx<T> r = s * bcur;
                    if (DIR) r = csel(dfix(q1), z, r);
                    if (owned && q1 >= z0 && q1 < z1) sto(rs + (long long)q1 * sz, ob, r);
                    x1 = od1 * r;
                    bq = r;
                } else {
                    x1 = od1 * bcur;
                    if (DIR) x1 = csel(dfix(q1), z, x1);
                    bq = bcur;
                }
            }
        } else {
            const Op3F<T>& A = FIRST == F_HSS ? B : L;
            cx<T> t1 = z, t0 = z, a0 = z;
            if (st1) {
                cx<T> H, V, a2;
                plane_sums<T>(pin[kb], ly, lx, a0, H, V, a2);
                plane_terms<T>(A, edge_wave, a0, H, V, a2, bx, by, (p == 0) | (p == n), t1, t0);
                if (p < 0 || p > n) t1 = t0 = z;
            }
            const cx<T> ax = acc1 + t1;  // A x at plane q1
            if (q1ok && st1) {
                if (FIRST == F_APPLY) {
                    x1 = ax;
                    if (DIR) x1 = csel(dfix(q1), z, x1);
                } else if (FIRST == F_RESID) {
                    x1 = s * (bcur - ax);
                    if (DIR) x1 = csel(dfix(q1), z, x1);
                } else if (FIRST == F_JAC || J0) {
                    x1 = cfma(od1, bcur - ax, xc);
                    if (DIR) x1 = csel(dfix(q1), z, x1);
                    bq = bcur;
                } else {  // F_HSS
                    cx<T> r = s * (bcur - ax);
                    if (DIR) r = csel(dfix(q1), z, r);
                    if (owned && q1 >= z0 && q1 < z1) sto(rs + (long long)q1 * sz, ob, r);
                    x1 = od1 * r;
                    bq = r;
                }
            }
            acc1 = T1p + t0;
            T1p = t1;
            xc = a0;
        }
        if (NS == 1) {
            if (UPD == 1) {
                const cx<T> yo = yr[sl];
                yr[sl] = ldcol(ys, q1 + PF, z1 - 1);
                if (owned && q1ok && q1 < z1) sto(ys + (long long)q1 * sz, ob, yo + x1);
            } else if (owned && q1ok && q1 < z1) {
                sto(ys + (long long)q1 * sz, ob, x1);
            }
            return;
        }
        // second stage: x1 of plane q1 - 1, written to the middle plane at
        // the previous step (ordered by this step's barrier); output q1 - 2.
        // x1 of plane q1 goes to the other middle buffer, read at the next
        // step, so one barrier per step orders both.
        pmid[kb][ly][lx] = x1;
        const int qm = q1 - 1, q2 = q1 - 2;
        cx<T> yo = z;
        if (UPD == 1) {
            yo = yr[sl];
            yr[sl] = ldcol(ys, q2 + PF, z1 - 1);
        }
        if (st2) {
            cx<T> a0, H, V, a2, u1 = z, u0 = z;
            plane_sums<T>(pmid[kb ^ 1], ly, lx, a0, H, V, a2);
            if (qm >= 0 && qm <= n)
                plane_terms<T>(L, edge_wave, a0, H, V, a2, bx, by, (qm == 0) | (qm == n), u1, u0);
            if (owned && q2 >= z0 && q2 < z1) {
                const cx<T> od2 = odf(q2);
                cx<T> x2 = cfma(od2, b2 - (acc2 + u1), xc2);
                if (DIR) x2 = csel(dfix(q2), z, x2);
                sto(ys + (long long)q2 * sz, ob, UPD == 1 ? yo + x2 : x2);
            }
            acc2 = U1p + u0;
            U1p = u1;
            xc2 = a0;
        }
        b2 = b2n;
        b2n = bq;
    };
    int pb = p0;
    for (; pb + UNR - 1 <= p1; pb += UNR) {
        step(IC<0>{}, pb);
        step(IC<1>{}, pb + 1);
        step(IC<2>{}, pb + 2);
        step(IC<3>{}, pb + 3);
        step(IC<4>{}, pb + 4);
        step(IC<5>{}, pb + 5);
    }
    if (pb <= p1) step(IC<0>{}, pb);
    if (pb + 1 <= p1) step(IC<1>{}, pb + 1);
    if (pb + 2 <= p1) step(IC<2>{}, pb + 2);
    if (pb + 3 <= p1) step(IC<3>{}, pb + 3);
    if (pb + 4 <= p1) step(IC<4>{}, pb + 4);
}

// ------------------------------------------------------------------ k3_rr --
// b_c = P^T (b - L x) from the n mesh to the n/2 mesh.  A tile owns RC x RC
// coarse columns; its first stage forms the residual on the fine columns
// 2 I - 1 .. 2 I + 1 around them, the second stage restricts each residual
// plane in-plane on the coarse columns and accumulates it into the coarse
// planes (weight 1 on plane 2 L, 1/2 on 2 L +- 1).  Segments own coarse
// planes [Z0, Z0 + tz).  The march starts on an even plane and is unrolled
// as in k3_pass.
template <typename T, int TH, bool DIR>
__global__ __launch_bounds__(Tile<TH>::FT) void k3_rr(Op3F<T> L, Vec<const cx<T>> X, Vec<const cx<T>> Bv,
                                                     Vec<cx<T>> Bc, Grid3F g) {
    constexpr int LH = Tile<TH>::H, RCH = Tile<TH>::RCH;
    __shared__ cx<T> pin[2][LH][LW];
    // residual plane with the even and odd columns of a row stored apart, so
    // that the coarse columns of the second stage read consecutive words
    __shared__ cx<T> pres[2][LH][2][LW / 2];
    int slot, tx, ty, seg;
    unit_of(g, slot, tx, ty, seg);
    const int n = L.n, nc = n / 2;
    const long long sy = n + 1, sz = sy * sy, syc = nc + 1, szc = syc * syc;
    const int lx = (int)threadIdx.x % LW, ly = (int)threadIdx.x / LW;
    // staged column; the residual is formed on the region's interior, whose
    // first column 2 RC tx - 1 is the fine neighbour left of coarse column RC tx
    const int i = 2 * RC * tx - 2 + lx, j = 2 * RCH * ty - 2 + ly;
    const bool inmesh = (i >= 0) & (i <= n) & (j >= 0) & (j <= n);
    const bool st1 = (lx >= 1) & (lx < LW - 1) & (ly >= 1) & (ly < LH - 1);
    const bool bx = (i == 0) | (i == n), by = (j == 0) | (j == n);
    const bool edge_wave = __any((int)(inmesh & (bx | by)));
    const long long col = inmesh ? (long long)j * sy + i : 0;
    const unsigned ob = (unsigned)col * (unsigned)sizeof(cx<T>);
    const int Z0 = seg * g.tz, Z1 = min(Z0 + g.tz, nc + 1);
    const cx<T>* xs = X.at(slot);
    const cx<T>* bs = Bv.at(slot);
    cx<T>* bc = Bc.at(slot);
    const cx<T> z = mk((T)0, (T)0);
    // coarse column of the second stage (threads 0 .. RC^2 - 1); its fine
    // centre (2 I, 2 J) is staged at (2 ci + 2, 2 cj + 2)
    const bool cst = (int)threadIdx.x < RC * RCH;
    const int ci = (int)threadIdx.x % RC, cj = (int)threadIdx.x / RC;
    const int I = RC * tx + ci, J = RCH * ty + cj;
    const bool cown = cst & (I <= nc) & (J <= nc);
    // DIR: the residual is cleared on the fine nodes of Dirichlet faces and
    // the restricted value on the coarse ones
    const unsigned dm = DIR ? L.dir : 0u;
    const bool dcol = DIR && (((dm & 1u) && i == 0) || ((dm & 2u) && i == n) ||
                              ((dm & 4u) && j == 0) || ((dm & 8u) && j == n));
    const bool ccol = DIR && (((dm & 1u) && I == 0) || ((dm & 2u) && I == nc) ||
                              ((dm & 4u) && J == 0) || ((dm & 8u) && J == nc));
    const unsigned occ = cown ? (unsigned)(J * syc + I) * (unsigned)sizeof(cx<T>) : 0u;

    // unconditional loads (see k3_pass), masked where consumed
    auto ldcol = [&](const cx<T>* p, int l, int hi) {
        return ldo(p + (long long)max(0, min(l, min(hi, n))) * sz, ob);
    };
    auto lok = [&](int l) { return inmesh && l >= 0 && l <= n; };
    // residual planes [2 Z0 - 1, 2 Z1 - 1] are formed at steps p = q + 1;
    // the input starts one plane below the first of them (p0 is even)
    const int p0 = 2 * Z0 - 2, p1 = 2 * Z1;
    {
        const cx<T> v = ldcol(xs, p0, p1);
        pin[0][ly][lx] = csel(lok(p0), v, z);
    }
    cx<T> xr[PF], br[PF];  // x at planes p + 1 .. p + PF; b at q .. q + PF - 1
#pragma unroll
    for (int u = 0; u < PF; ++u) {
        xr[u] = ldcol(xs, p0 + 1 + u, p1);
        br[u] = ldcol(bs, p0 - 1 + u, p1 - 1);
    }
    cx<T> acc = z, T1p = z;
    cx<T> cur = z, half = z;  // coarse accumulators of the second stage

    auto step = [&](auto uc, int p) __attribute__((always_inline)) {
        constexpr int u = decltype(uc)::value;
        constexpr int kb = u & 1;
        constexpr int sl = u % PF;
        const int q = p - 1;  // residual plane formed at this step (odd when u is even)
        __syncthreads();
        pin[kb ^ 1][ly][lx] = csel(lok(p + 1), xr[sl], z);
        xr[sl] = ldcol(xs, p + 1 + PF, p1);
        const cx<T> bcur = br[sl];
        br[sl] = ldcol(bs, q + PF, p1 - 1);
        cx<T> t1 = z, t0 = z;
        if (st1) {
            cx<T> a0, H, V, a2;
            plane_sums<T>(pin[kb], ly, lx, a0, H, V, a2);
            plane_terms<T>(L, edge_wave, a0, H, V, a2, bx, by, (p == 0) | (p == n), t1, t0);
            if (p < 0 || p > n) t1 = t0 = z;
        }
        cx<T> r = z;
        if (st1 && inmesh && q >= 0 && q <= n) r = bcur - (acc + t1);
        if (DIR) r = csel(dcol || ((dm & 16u) && q == 0) || ((dm & 32u) && q == n), z, r);
        acc = T1p + t0;
        T1p = t1;
        pres[kb][ly][lx & 1][lx >> 1] = r;
        // second stage on the residual plane q - 1, written at the previous
        // step into the other buffer (ordered by this step's barrier)
        if (cst) {
            const cx<T>(*pr)[2][LW / 2] = pres[kb ^ 1];
            cx<T> c0, cH, cV, c2;
            // fine centre (2 cj + 2, 2 ci + 2): even column ci + 1, its
            // neighbours the odd columns ci and ci + 1 of the same rows
            const int r0 = 2 * cj + 2;
            c0 = pr[r0][0][ci + 1];
            cH = pr[r0][1][ci] + pr[r0][1][ci + 1];
            cV = pr[r0 - 1][0][ci + 1] + pr[r0 + 1][0][ci + 1];
            c2 = (pr[r0 - 1][1][ci] + pr[r0 - 1][1][ci + 1]) + (pr[r0 + 1][1][ci] + pr[r0 + 1][1][ci + 1]);
            const cx<T> r2 = c0 + (T)0.5 * (cH + cV) + (T)0.25 * c2;
            const int q2 = q - 1;  // same parity as p
            if (kb == 1) {  // q2 odd
                const int Lc = (q2 - 1) >> 1;  // coarse plane completed by this odd plane
                cx<T> v = cur + (T)0.5 * r2;
                if (DIR) v = csel(ccol || ((dm & 16u) && Lc == 0) || ((dm & 32u) && Lc == nc), z, v);
                if (cown && Lc >= Z0 && Lc < Z1) sto(bc + (long long)Lc * szc, occ, v);
                half = (T)0.5 * r2;
            } else {
                cur = half + r2;
            }
        }
    };
    // the restriction of the last residual plane (2 Z1 - 1) runs one step
    // after it is formed
    const int pe = p1 + 1;
    int pb = p0;
    for (; pb + UNR - 1 <= pe; pb += UNR) {
        step(IC<0>{}, pb);
        step(IC<1>{}, pb + 1);
        step(IC<2>{}, pb + 2);
        step(IC<3>{}, pb + 3);
        step(IC<4>{}, pb + 4);
        step(IC<5>{}, pb + 5);
    }
    if (pb <= pe) step(IC<0>{}, pb);
    if (pb + 1 <= pe) step(IC<1>{}, pb + 1);
    if (pb + 2 <= pe) step(IC<2>{}, pb + 2);
    if (pb + 3 <= pe) step(IC<3>{}, pb + 3);
    if (pb + 4 <= pe) step(IC<4>{}, pb + 4);
}

// Workgroups of a kernel that the device holds at once (its occupancy per
// CU, from its register and LDS use, times the CUs), asked once per kernel.
template <auto K, int FT>
int resident_units() {
    static const int units = [] {
        int nb = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, K, FT, 0) != hipSuccess || nb < 1) nb = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        return nb * cus;
    }();
    return units;
}

// Segment height: output planes per workgroup.  A launch takes
// ceil(units / resident) rounds, each as long as one segment's march (its
// planes plus a pipeline head of about HEAD planes); the height minimises
// rounds x (planes + HEAD), at least MINTZ planes unless one segment
// covers the level.
#ifndef HELM_K3_MINTZ
#define HELM_K3_MINTZ 1
#endif
#ifndef HELM_K3_HEAD
#define HELM_K3_HEAD 4
#endif
int seg_planes(int planes, int tiles, int nslots, int resident) {
#ifdef HELM_K3_SEGS
    return (planes + HELM_K3_SEGS - 1) / HELM_K3_SEGS;
#endif
    const long long cus = resident;
    int best = planes;
    long long best_cost = -1;
    for (int segs = 1; segs <= planes; ++segs) {
        const int tz = (planes + segs - 1) / segs;
        if (tz < HELM_K3_MINTZ && segs > 1) break;
        const long long units = (long long)tiles * segs * nslots;
        const long long rounds = (units + cus - 1) / cus;
        const long long cost = rounds * (tz + HELM_K3_HEAD);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = tz;
        }
    }
    return best;
}

// The same for the restriction, whose segments own coarse planes and march
// two fine planes per coarse one (plus a head of about HEAD + 2).
int seg_planes_rr(int cplanes, int tiles, int nslots, int resident) {
    int best = cplanes;
    long long best_cost = -1;
    for (int tz = cplanes; tz >= 1; --tz) {
        const int segs = (cplanes + tz - 1) / tz;
        if (tz < HELM_K3_MINTZ && segs > 1) break;
        const long long units = (long long)tiles * segs * nslots;
        const long long rounds = (units + resident - 1) / resident;
        const long long cost = rounds * (2LL * tz + HELM_K3_HEAD + 2);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = tz;
        }
    }
    return best;
}

template <typename T, typename TI, int F, int NS, bool PRO, int UPD, int TH, bool DIR>
void launch_pass_h(hipStream_t st, const Op3F<T>& L, const Op3F<T>& B, T s, Vec<const cx<TI>> X,
                   Vec<const cx<T>> Bv, Vec<const cx<T>> Ec, Vec<cx<T>> Rho, Vec<cx<T>> Y, int nslots,
                   int tz) {
    const int n = L.n, own = LW - 2 * NS, ownh = Tile<TH>::H - 2 * NS;
    Grid3F g;
    g.tiles_x = (n + 1 + own - 1) / own;
    g.tiles_y = (n + 1 + ownh - 1) / ownh;
    g.tz = tz > 0 ? tz
                  : seg_planes(n + 1, g.tiles_x * g.tiles_y, nslots,
                               resident_units<k3_pass<T, TI, F, NS, PRO, UPD, TH, DIR>, Tile<TH>::FT>());
    g.segs = (n + 1 + g.tz - 1) / g.tz;
    const dim3 grid((unsigned)(g.tiles_x * g.tiles_y * g.segs * nslots));
    k3_pass<T, TI, F, NS, PRO, UPD, TH, DIR><<<grid, Tile<TH>::FT, 0, st>>>(L, B, s, X, Bv, Ec, Rho, Y, g);
}

template <typename T, typename TI, int F, int NS, bool PRO, int UPD, int TH>
void launch_pass_d(hipStream_t st, const Op3F<T>& L, const Op3F<T>& B, T s, Vec<const cx<TI>> X,
                   Vec<const cx<T>> Bv, Vec<const cx<T>> Ec, Vec<cx<T>> Rho, Vec<cx<T>> Y, int nslots,
                   int tz) {
    if (L.dir) launch_pass_h<T, TI, F, NS, PRO, UPD, TH, true>(st, L, B, s, X, Bv, Ec, Rho, Y, nslots, tz);
    else launch_pass_h<T, TI, F, NS, PRO, UPD, TH, false>(st, L, B, s, X, Bv, Ec, Rho, Y, nslots, tz);
}

template <typename T, typename TI, int F, int NS, bool PRO, int UPD>
void launch_pass(hipStream_t st, const Op3F<T>& L, const Op3F<T>& B, T s, Vec<const cx<TI>> X,
                 Vec<const cx<T>> Bv, Vec<const cx<T>> Ec, Vec<cx<T>> Rho, Vec<cx<T>> Y, int nslots,
                 int tz) {
    if constexpr (short_rows<T>() != tall_rows<T>()) {
        if (L.n < HELM_K3_TALL_N) {
            launch_pass_d<T, TI, F, NS, PRO, UPD, short_rows<T>()>(st, L, B, s, X, Bv, Ec, Rho, Y, nslots, tz);
            return;
        }
    }
    launch_pass_d<T, TI, F, NS, PRO, UPD, tall_rows<T>()>(st, L, B, s, X, Bv, Ec, Rho, Y, nslots, tz);
}

template <typename T, int TH, bool DIR>
void rr3d_h(hipStream_t st, const Op3F<T>& L, Vec<const cx<T>> X, Vec<const cx<T>> Bv, Vec<cx<T>> Bc,
            int nslots, int tz) {
    const int nc = L.n / 2;
    Grid3F g;
    g.tiles_x = (nc + 1 + RC - 1) / RC;
    g.tiles_y = (nc + 1 + Tile<TH>::RCH - 1) / Tile<TH>::RCH;
    g.tz = tz > 0 ? tz
                  : seg_planes_rr(nc + 1, g.tiles_x * g.tiles_y, nslots,
                                  resident_units<k3_rr<T, TH, DIR>, Tile<TH>::FT>());
    g.segs = (nc + 1 + g.tz - 1) / g.tz;
    const dim3 grid((unsigned)(g.tiles_x * g.tiles_y * g.segs * nslots));
    k3_rr<T, TH, DIR><<<grid, Tile<TH>::FT, 0, st>>>(L, X, Bv, Bc, g);
}

template <typename T, int TH>
void rr3d_d(hipStream_t st, const Op3F<T>& L, Vec<const cx<T>> X, Vec<const cx<T>> Bv, Vec<cx<T>> Bc,
            int nslots, int tz) {
    if (L.dir) rr3d_h<T, TH, true>(st, L, X, Bv, Bc, nslots, tz);
    else rr3d_h<T, TH, false>(st, L, X, Bv, Bc, nslots, tz);
}

}  // namespace

template <typename T, typename TI>
bool pass3d(hipStream_t st, const Op3F<T>& L, const Op3F<T>& B, int first, int ns, bool pro, int upd,
            T s, Vec<const cx<TI>> X, Vec<const cx<T>> Bv, Vec<const cx<T>> Ec, Vec<cx<T>> Rho,
            Vec<cx<T>> Y, int nslots, int tz) {
#define HELM_P3(F, NS_, PRO_, UPD_)                                                              \
    do {                                                                                         \
        launch_pass<T, TI, F, NS_, PRO_, UPD_>(st, L, B, s, X, Bv, Ec, Rho, Y, nslots, tz);     \
        return true;                                                                             \
    } while (0)
    if (ns == 1 && !pro && upd == 0) {
        if (first == F_APPLY) HELM_P3(F_APPLY, 1, false, 0);
        if (first == F_RESID) HELM_P3(F_RESID, 1, false, 0);
        if (first == F_JAC) HELM_P3(F_JAC, 1, false, 0);
        if (first == F_PRE0) HELM_P3(F_PRE0, 1, false, 0);
    }
    if constexpr (std::is_same<T, TI>::value) {
        if (ns == 1) {
            if (first == F_JAC && pro && upd == 0) HELM_P3(F_JAC, 1, true, 0);
            if (first == F_JAC && !pro && upd == 1) HELM_P3(F_JAC, 1, false, 1);
            if (first == F_HSS && !pro && upd == 0) HELM_P3(F_HSS, 1, false, 0);
            if (first == F_HSS0 && !pro && upd == 0) HELM_P3(F_HSS0, 1, false, 0);
            if (first == F_JAC0 && !pro && upd == 0) HELM_P3(F_JAC0, 1, false, 0);
        }
        if (ns == 2) {
            if (first == F_JAC && !pro && upd == 0) HELM_P3(F_JAC, 2, false, 0);
            if (first == F_JAC && pro && upd == 0) HELM_P3(F_JAC, 2, true, 0);
            if (first == F_JAC && pro && upd == 1) HELM_P3(F_JAC, 2, true, 1);
            if (first == F_HSS && !pro && upd == 0) HELM_P3(F_HSS, 2, false, 0);
            if (first == F_HSS0 && !pro && upd == 0) HELM_P3(F_HSS0, 2, false, 0);
            if (first == F_PRE0 && !pro && upd == 0) HELM_P3(F_PRE0, 2, false, 0);
        }
    }
#undef HELM_P3
    return false;
}

template <typename T>
void rr3d(hipStream_t st, const Op3F<T>& L, Vec<const cx<T>> X, Vec<const cx<T>> Bv, Vec<cx<T>> Bc,
          int nslots, int tz) {
    if constexpr (short_rows<T>() != tall_rows<T>()) {
        if (L.n < HELM_K3_TALL_N) {
            rr3d_d<T, short_rows<T>()>(st, L, X, Bv, Bc, nslots, tz);
            return;
        }
    }
    rr3d_d<T, tall_rows<T>()>(st, L, X, Bv, Bc, nslots, tz);
}

template bool pass3d<double, double>(hipStream_t, const Op3F<double>&, const Op3F<double>&, int, int,
                                     bool, int, double, Vec<const cxd>, Vec<const cxd>,
                                     Vec<const cxd>, Vec<cxd>, Vec<cxd>, int, int);
template bool pass3d<double, float>(hipStream_t, const Op3F<double>&, const Op3F<double>&, int, int,
                                    bool, int, double, Vec<const cxf>, Vec<const cxd>,
                                    Vec<const cxd>, Vec<cxd>, Vec<cxd>, int, int);
template bool pass3d<float, float>(hipStream_t, const Op3F<float>&, const Op3F<float>&, int, int, bool,
                                   int, float, Vec<const cxf>, Vec<const cxf>, Vec<const cxf>,
                                   Vec<cxf>, Vec<cxf>, int, int);
template void rr3d<double>(hipStream_t, const Op3F<double>&, Vec<const cxd>, Vec<const cxd>, Vec<cxd>,
                           int, int);
template void rr3d<float>(hipStream_t, const Op3F<float>&, Vec<const cxf>, Vec<const cxf>, Vec<cxf>,
                          int, int);

}  // namespace helm
