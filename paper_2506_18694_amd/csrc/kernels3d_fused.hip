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
// already requested), and every dependent pass is a pipeline stage one
// plane behind the previous one: the first stage's output plane reaches the
// second stage through a second LDS plane.  Passes:
//   k3_pass  one or two operator stages: apply, scaled residual, Jacobi
//            sweeps (from a guess, from the guess plus the prolonged coarse
//            correction, or from zero), the shifted-HSS residual
//            rho = c (R - B u) with the first zero-guess sweep, and the HSS
//            update u += x or u = x on the last output
//   k3_rr    residual restriction b_c = P^T (b - L x): stage 1 forms the
//            residual plane, stage 2 applies the transpose of trilinear
//            interpolation (in-plane weights 1, 1/2, 1/4; across planes
//            1/2, 1, 1/2) on the coarse columns of the tile
#include <algorithm>
#include <type_traits>

#include "launch.h"

namespace helm {

namespace {

// A workgroup of LW x LW threads stages one LW x LW region of an input plane
// (one value per thread); the first stage runs on its interior
// (LW - 2)^2 columns, the second stage on the (LW - 4)^2 inside that.
constexpr int LW = 32;
constexpr int FT = LW * LW;  // threads per workgroup
constexpr int RC = 14;       // coarse columns per tile side in the restriction
#ifndef HELM_K3_PF
#define HELM_K3_PF 3
#endif
constexpr int PF = HELM_K3_PF;  // input planes requested ahead of the one in LDS (>= 1)

template <typename T>
__device__ __forceinline__ cx<T> c3(const cx<T>* w, cx<T> a0, cx<T> s1, cx<T> a2) {
    return cfma(w[0], a0, cfma(w[1], s1, w[2] * a2));
}

// T1, T0 of one plane (see top).  Waves without a column on a boundary
// line in x or y take the interior coefficients; the others evaluate the
// factors of each column (bx, by: the column lies on a boundary line; bz:
// the plane is the first or last).
template <typename T>
__device__ __forceinline__ void plane_terms(const Op3F<T>& op, bool edge_wave, cx<T> a0, cx<T> H,
                                            cx<T> V, cx<T> a2, bool bx, bool by, bool bz, cx<T>& T1,
                                            cx<T>& T0) {
    if (!edge_wave) {
        const cx<T> s1 = H + V;
        T1 = c3(op.i1, a0, s1, a2);
        T0 = bz ? c3(op.j0, a0, s1, a2) : c3(op.i0, a0, s1, a2);
        return;
    }
    const T h6 = op.h6, ih = op.ih;
    const T mx = bx ? 2 * h6 : 4 * h6, kx = bx ? ih : 2 * ih;
    const T my = by ? 2 * h6 : 4 * h6, ky = by ? ih : 2 * ih;
    const T ex = bx ? (T)1 : (T)0, ey = by ? (T)1 : (T)0;
    // PMM = mx my a0 + mx h6 V + my h6 H + h6^2 a2
    const cx<T> pmm = (mx * my) * a0 + (mx * h6) * V + (my * h6) * H + (h6 * h6) * a2;
    // PK = (kx my + mx ky) a0 + (kx h6 - mx ih) V + (ky h6 - my ih) H - (1/3) a2
    const cx<T> pk = (kx * my + mx * ky) * a0 + (kx * h6 - mx * ih) * V + (ky * h6 - my * ih) * H +
                     op.third * a2;
    // PG = ex (my a0 + h6 V) + ey (mx a0 + h6 H)
    const cx<T> pg = (ex * my + ey * mx) * a0 + (ex * h6) * V + (ey * h6) * H;
    T1 = cfma(op.uK, pk, cfma(op.uM, pmm, op.uG * pg));
    const cx<T> t0 = cfma(op.vK, pk, cfma(op.vM, pmm, op.vG * pg));
    T0 = bz ? cfma(op.c, pmm, (T)0.5 * t0) : t0;
}

// in-plane sums at (row r, column q) of an LW x LW LDS plane
template <typename T>
__device__ __forceinline__ void plane_sums(const cx<T> (*pl)[LW], int r, int q, cx<T>& a0, cx<T>& H,
                                           cx<T>& V, cx<T>& a2) {
    a0 = pl[r][q];
    H = pl[r][q - 1] + pl[r][q + 1];
    V = pl[r - 1][q] + pl[r + 1][q];
    a2 = (pl[r - 1][q - 1] + pl[r - 1][q + 1]) + (pl[r + 1][q - 1] + pl[r + 1][q + 1]);
}

// (P e)(i, j, l), trilinear interpolation from the n/2 mesh: the eight
// corners of the smallest coarse cell holding the node, with repeats where
// an offset is even, summed and scaled by 1/8 (exact powers of two)
template <typename T>
__device__ __forceinline__ cx<T> prolong_at(const cx<T>* e, int nc, int i, int j, int l) {
    const long long syc = nc + 1, szc = syc * syc;
    const long long c0 = (long long)(l >> 1) * szc + (long long)(j >> 1) * syc + (i >> 1);
    const long long dx = i & 1, dy = (long long)(j & 1) * syc, dz = (long long)(l & 1) * szc;
    const cx<T> v000 = e[c0], v100 = e[c0 + dx], v010 = e[c0 + dy], v110 = e[c0 + dx + dy];
    const cx<T> v001 = e[c0 + dz], v101 = e[c0 + dx + dz], v011 = e[c0 + dy + dz],
                v111 = e[c0 + dx + dy + dz];
    const cx<T> s = ((v000 + v100) + (v010 + v110)) + ((v001 + v101) + (v011 + v111));
    return (T)0.125 * s;
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
// FIRST (the first stage, its output lagging the input by one plane when
// it is a stencil, in step with it when pointwise):
//   F_APPLY  y = L x                             (NS = 1)
//   F_RESID  y = s (b - L x)                     (NS = 1)
//   F_JAC    x1 = x + w/D (b - L x)   (x + P e_c when PRO)
//   F_HSS    rho = s (R - B u) (written to Rho), x1 = w/D rho; B the
//            second operator, R in Bv, u in X
//   F_HSS0   rho = s R (written), x1 = w/D rho   (u = 0; pointwise)
//   F_PRE0   x1 = w/D b                          (pointwise)
// NS = 2 adds x2 = x1 + w/D (b - L x1) (b = rho for the HSS forms).
// UPD: 0 y = result, 1 y += result (the HSS update u += e with u in Y).
template <typename T, typename TI, int FIRST, int NS, bool PRO, int UPD>
__global__ __launch_bounds__(FT) void k3_pass(Op3F<T> L, Op3F<T> B, T s, Vec<const cx<TI>> X,
                                              Vec<const cx<T>> Bv, Vec<const cx<T>> Ec,
                                              Vec<cx<T>> Rho, Vec<cx<T>> Y, Grid3F g) {
    constexpr bool PW = FIRST == F_HSS0 || FIRST == F_PRE0;
    constexpr bool HSS = FIRST == F_HSS || FIRST == F_HSS0;
    constexpr int OWN = LW - 2 * NS;  // owned columns per tile side
    __shared__ cx<T> pin[2][LW][LW];
    __shared__ cx<T> pmid[LW][LW];
    int slot, tx, ty, seg;
    unit_of(g, slot, tx, ty, seg);
    const int n = L.n;
    const long long sy = n + 1, sz = sy * sy;
    const int lx = (int)threadIdx.x % LW, ly = (int)threadIdx.x / LW;
    const int i = tx * OWN - NS + lx, j = ty * OWN - NS + ly;  // this thread's column
    const bool inmesh = (i >= 0) & (i <= n) & (j >= 0) & (j <= n);
    const bool st1 = (lx >= 1) & (lx < LW - 1) & (ly >= 1) & (ly < LW - 1);
    const bool st2 = (lx >= 2) & (lx < LW - 2) & (ly >= 2) & (ly < LW - 2);
    const bool owned = inmesh & (NS == 2 ? st2 : st1);
    const bool bx = (i == 0) | (i == n), by = (j == 0) | (j == n);
    const bool edge_wave = __any((int)(inmesh & (bx | by)));
    const int cxy = (int)bx + (int)by;  // boundary coordinates in x and y
    const long long col = inmesh ? (long long)j * sy + i : 0;
    const int z0 = seg * g.tz, z1 = min(z0 + g.tz, n + 1);  // output planes [z0, z1)
    const cx<TI>* x = X.base ? X.at(slot) : nullptr;
    const cx<T>* bv = Bv.base ? Bv.at(slot) : nullptr;
    const cx<T>* ec = PRO ? Ec.at(slot) : nullptr;
    cx<T>* rho = HSS ? Rho.at(slot) : nullptr;
    cx<T>* y = Y.at(slot);
    const cx<T> z = mk((T)0, (T)0);

    // the value this thread stages from input plane p (zero outside the mesh)
    auto stage = [&](int p) {
        cx<T> v = z;
        if (inmesh && p >= 0 && p <= n) {
            v = cvt<T>(x[(long long)p * sz + col]);
            if (PRO) v = v + prolong_at<T>(ec, n / 2, i, j, p);
        }
        return v;
    };
    auto ldcol = [&](const cx<T>* p, int l) {  // value at this thread's column, plane l
        return (inmesh && l >= 0 && l <= n) ? p[(long long)l * sz + col] : z;
    };

    // the first stage outputs planes [o0, o1); a stencil first stage reads
    // input planes [o0 - 1, o1], a pointwise one [o0, o1 - 1]
    const int o0 = z0 - (NS - 1), o1 = z1 + (NS - 1);
    const int p0 = PW ? o0 : o0 - 1, p1 = PW ? o1 - 1 : o1;
    cx<T> ring[PF];  // input planes p + 1 .. p + PF (stencil first stage)
#pragma unroll
    for (int u = 0; u < PF; ++u) ring[u] = z;
    if (!PW) {
        pin[0][ly][lx] = stage(p0);
#pragma unroll
        for (int u = 0; u < PF; ++u)
            if (p0 + 1 + u <= p1) ring[u] = stage(p0 + 1 + u);
    }
    // stage 1: acc1 = T1(q - 1) + T0(q) for the next output plane q, T1p = T1(q);
    // xc: input centre of q.  Stage 2 likewise, with b2 its right-hand side.
    cx<T> acc1 = z, T1p = z, xc = z;
    cx<T> acc2 = z, U1p = z, xc2 = z, b2 = z, bq = z;
    cx<T> bnext = FIRST != F_APPLY ? ldcol(bv, PW ? p0 : p0 - 1) : z;
    int k = 0;
    for (int p = p0; p <= p1; ++p) {
        const int q1 = PW ? p : p - 1;  // plane the first stage outputs at this step
        __syncthreads();
        cx<T> vn = z;
        if (!PW && p + PF + 1 <= p1) vn = stage(p + PF + 1);
        const cx<T> bcur = bnext;
        if (FIRST != F_APPLY && q1 + 1 < o1) bnext = ldcol(bv, q1 + 1);
        const bool q1ok = inmesh && q1 >= 0 && q1 <= n && q1 >= o0;
        const int cls = cxy + (int)((q1 == 0) | (q1 == n));
        cx<T> x1 = z;
        if (PW) {
            if (q1ok) {
                if (FIRST == F_HSS0) {
                    const cx<T> r = s * bcur;
                    if (owned && q1 >= z0 && q1 < z1) rho[(long long)q1 * sz + col] = r;
                    x1 = L.od[cls] * r;
                    bq = r;
                } else {
                    x1 = L.od[cls] * bcur;
                    bq = bcur;
                }
            }
        } else {
            const Op3F<T>& A = FIRST == F_HSS ? B : L;
            cx<T> t1 = z, t0 = z, a0 = z;
            if (st1) {
                cx<T> H, V, a2;
                plane_sums<T>(pin[k], ly, lx, a0, H, V, a2);
                plane_terms<T>(A, edge_wave, a0, H, V, a2, bx, by, (p == 0) | (p == n), t1, t0);
                if (p < 0 || p > n) t1 = t0 = z;
            }
            const cx<T> ax = acc1 + t1;  // A x at plane q1
            if (q1ok && st1) {
                if (FIRST == F_APPLY) {
                    x1 = ax;
                } else if (FIRST == F_RESID) {
                    x1 = s * (bcur - ax);
                } else if (FIRST == F_JAC) {
                    x1 = cfma(L.od[cls], bcur - ax, xc);
                    bq = bcur;
                } else {  // F_HSS
                    const cx<T> r = s * (bcur - ax);
                    if (owned && q1 >= z0 && q1 < z1) rho[(long long)q1 * sz + col] = r;
                    x1 = L.od[cls] * r;
                    bq = r;
                }
            }
            acc1 = T1p + t0;
            T1p = t1;
            xc = a0;
            if (p + 1 <= p1) pin[k ^ 1][ly][lx] = ring[0];
#pragma unroll
            for (int u = 0; u + 1 < PF; ++u) ring[u] = ring[u + 1];
            ring[PF - 1] = vn;
            k ^= 1;
        }
        if (NS == 1) {
            if (owned && q1ok && q1 < z1) {
                const long long t = (long long)q1 * sz + col;
                y[t] = UPD == 1 ? y[t] + x1 : x1;
            }
            continue;
        }
        // second stage: x1 of plane q1 through the middle plane; output q1 - 1
        pmid[ly][lx] = x1;
        __syncthreads();
        if (st2) {
            cx<T> a0, H, V, a2, u1 = z, u0 = z;
            plane_sums<T>(pmid, ly, lx, a0, H, V, a2);
            if (q1 >= 0 && q1 <= n)
                plane_terms<T>(L, edge_wave, a0, H, V, a2, bx, by, (q1 == 0) | (q1 == n), u1, u0);
            const int q2 = q1 - 1;
            if (owned && q2 >= z0 && q2 < z1) {
                const int cls2 = cxy + (int)((q2 == 0) | (q2 == n));
                const cx<T> x2 = cfma(L.od[cls2], b2 - (acc2 + u1), xc2);
                const long long t = (long long)q2 * sz + col;
                y[t] = UPD == 1 ? y[t] + x2 : x2;
            }
            acc2 = U1p + u0;
            U1p = u1;
            xc2 = a0;
            b2 = bq;
        }
    }
}

// ------------------------------------------------------------------ k3_rr --
// b_c = P^T (b - L x) from the n mesh to the n/2 mesh.  A tile owns RC x RC
// coarse columns; its first stage forms the residual on the fine columns
// 2 I - 1 .. 2 I + 1 around them, the second stage restricts each residual
// plane in-plane on the coarse columns and accumulates it into the coarse
// planes (weight 1 on plane 2 L, 1/2 on 2 L +- 1).  Segments own coarse
// planes [Z0, Z0 + tz).
template <typename T>
__global__ __launch_bounds__(FT) void k3_rr(Op3F<T> L, Vec<const cx<T>> X, Vec<const cx<T>> Bv,
                                            Vec<cx<T>> Bc, Grid3F g) {
    __shared__ cx<T> pin[2][LW][LW];
    __shared__ cx<T> pres[LW][LW];
    int slot, tx, ty, seg;
    unit_of(g, slot, tx, ty, seg);
    const int n = L.n, nc = n / 2;
    const long long sy = n + 1, sz = sy * sy, syc = nc + 1, szc = syc * syc;
    const int lx = (int)threadIdx.x % LW, ly = (int)threadIdx.x / LW;
    // staged column; the residual is formed on the region's interior, whose
    // first column 2 RC tx - 1 is the fine neighbour left of coarse column RC tx
    const int i = 2 * RC * tx - 2 + lx, j = 2 * RC * ty - 2 + ly;
    const bool inmesh = (i >= 0) & (i <= n) & (j >= 0) & (j <= n);
    const bool st1 = (lx >= 1) & (lx < LW - 1) & (ly >= 1) & (ly < LW - 1);
    const bool bx = (i == 0) | (i == n), by = (j == 0) | (j == n);
    const bool edge_wave = __any((int)(inmesh & (bx | by)));
    const long long col = inmesh ? (long long)j * sy + i : 0;
    const int Z0 = seg * g.tz, Z1 = min(Z0 + g.tz, nc + 1);
    const cx<T>* x = X.at(slot);
    const cx<T>* bv = Bv.at(slot);
    cx<T>* bc = Bc.at(slot);
    const cx<T> z = mk((T)0, (T)0);
    // coarse column of the second stage (threads 0 .. RC^2 - 1); its fine
    // centre (2 I, 2 J) is staged at (2 ci + 2, 2 cj + 2)
    const bool cst = (int)threadIdx.x < RC * RC;
    const int ci = (int)threadIdx.x % RC, cj = (int)threadIdx.x / RC;
    const int I = RC * tx + ci, J = RC * ty + cj;
    const bool cown = cst & (I <= nc) & (J <= nc);
    const long long ccol = cown ? (long long)J * syc + I : 0;

    auto stage = [&](int p) {
        return (inmesh && p >= 0 && p <= n) ? x[(long long)p * sz + col] : z;
    };
    auto ldb = [&](int l) { return (inmesh && l >= 0 && l <= n) ? bv[(long long)l * sz + col] : z; };
    // residual planes [2 Z0 - 1, 2 Z1 - 1] are formed at steps p = q + 1;
    // the input starts one plane below the first of them
    const int p0 = 2 * Z0 - 2, p1 = 2 * Z1;
    pin[0][ly][lx] = stage(p0);
    cx<T> ring[PF];
#pragma unroll
    for (int u = 0; u < PF; ++u) ring[u] = p0 + 1 + u <= p1 ? stage(p0 + 1 + u) : z;
    cx<T> acc = z, T1p = z, bnext = ldb(p0 - 1);
    cx<T> cur = z, half = z;  // coarse accumulators of the second stage
    int k = 0;
    for (int p = p0; p <= p1; ++p) {
        const int q = p - 1;  // residual plane formed at this step
        __syncthreads();
        cx<T> vn = z;
        if (p + PF + 1 <= p1) vn = stage(p + PF + 1);
        const cx<T> bcur = bnext;
        bnext = ldb(q + 1);
        cx<T> t1 = z, t0 = z;
        if (st1) {
            cx<T> a0, H, V, a2;
            plane_sums<T>(pin[k], ly, lx, a0, H, V, a2);
            plane_terms<T>(L, edge_wave, a0, H, V, a2, bx, by, (p == 0) | (p == n), t1, t0);
            if (p < 0 || p > n) t1 = t0 = z;
        }
        cx<T> r = z;
        if (st1 && inmesh && q >= 0 && q <= n) r = bcur - (acc + t1);
        acc = T1p + t0;
        T1p = t1;
        if (p + 1 <= p1) pin[k ^ 1][ly][lx] = ring[0];
#pragma unroll
        for (int u = 0; u + 1 < PF; ++u) ring[u] = ring[u + 1];
        ring[PF - 1] = vn;
        k ^= 1;
        pres[ly][lx] = r;
        __syncthreads();
        if (cst) {
            cx<T> c0, cH, cV, c2;
            plane_sums<T>(pres, 2 * cj + 2, 2 * ci + 2, c0, cH, cV, c2);
            const cx<T> r2 = c0 + (T)0.5 * (cH + cV) + (T)0.25 * c2;
            if (q & 1) {
                const int Lc = (q - 1) >> 1;  // coarse plane completed by this odd plane
                if (cown && Lc >= Z0 && Lc < Z1) bc[(long long)Lc * szc + ccol] = cur + (T)0.5 * r2;
                half = (T)0.5 * r2;
            } else {
                cur = half + r2;
            }
        }
    }
}

// Segment height: output planes per workgroup.  One 1024-thread workgroup
// runs per CU, so a launch takes ceil(units / 256) rounds, each as long as
// one segment's march (its planes plus a pipeline head of about four); the
// height minimises rounds x (planes + 4), at least 8 planes unless one
// segment covers the level.
int seg_planes(int planes, int tiles, int nslots) {
#ifdef HELM_K3_SEGS
    return (planes + HELM_K3_SEGS - 1) / HELM_K3_SEGS;
#endif
    const long long cus = 256;
    int best = planes;
    long long best_cost = -1;
    for (int segs = 1; segs <= planes; ++segs) {
        const int tz = (planes + segs - 1) / segs;
        if (tz < 8 && segs > 1) break;
        const long long units = (long long)tiles * segs * nslots;
        const long long rounds = (units + cus - 1) / cus;
        const long long cost = rounds * (tz + 4);
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = tz;
        }
    }
    return best;
}

}  // namespace

template <typename T, typename TI>
bool pass3d(hipStream_t st, const Op3F<T>& L, const Op3F<T>& B, int first, int ns, bool pro, int upd,
            T s, Vec<const cx<TI>> X, Vec<const cx<T>> Bv, Vec<const cx<T>> Ec, Vec<cx<T>> Rho,
            Vec<cx<T>> Y, int nslots, int tz) {
    const int n = L.n;
    const int own = LW - 2 * ns;
    Grid3F g;
    g.tiles_x = (n + 1 + own - 1) / own;
    g.tiles_y = (n + 1 + own - 1) / own;
    g.tz = tz > 0 ? tz : seg_planes(n + 1, g.tiles_x * g.tiles_y, nslots);
    g.segs = (n + 1 + g.tz - 1) / g.tz;
    const dim3 grid((unsigned)(g.tiles_x * g.tiles_y * g.segs * nslots));
#define HELM_P3(F, NS_, PRO_, UPD_)                                                               \
    do {                                                                                          \
        k3_pass<T, TI, F, NS_, PRO_, UPD_><<<grid, FT, 0, st>>>(L, B, s, X, Bv, Ec, Rho, Y, g); \
        return true;                                                                              \
    } while (0)
    if (ns == 1 && !pro && upd == 0) {
        if (first == F_APPLY) HELM_P3(F_APPLY, 1, false, 0);
        if (first == F_RESID) HELM_P3(F_RESID, 1, false, 0);
        if (first == F_JAC) HELM_P3(F_JAC, 1, false, 0);
        if (first == F_PRE0) HELM_P3(F_PRE0, 1, false, 0);
    }
    if constexpr (std::is_same<T, TI>::value) {
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
    const int nc = L.n / 2;
    Grid3F g;
    g.tiles_x = (nc + 1 + RC - 1) / RC;
    g.tiles_y = g.tiles_x;
    g.tz = tz > 0 ? tz : std::max(4, seg_planes(2 * nc + 1, g.tiles_x * g.tiles_y, nslots) / 2);
    g.segs = (nc + 1 + g.tz - 1) / g.tz;
    const dim3 grid((unsigned)(g.tiles_x * g.tiles_y * g.segs * nslots));
    k3_rr<T><<<grid, FT, 0, st>>>(L, X, Bv, Bc, g);
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
