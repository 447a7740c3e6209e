// Host-side launchers of the HIP kernels (internal to libhelm).
#pragma once

#include "helm_common.h"

namespace helm {

// ---- 2D P1 stencils (kernels2d.hip) ---------------------------------------
// mode: StencilMode; s: scale for MODE_RESID.  X may be null for JACOBI0,
// B null for APPLY.
template <typename T, typename TI>
void stencil2d(hipStream_t st, const Op2<T>& op, int mode, T s, Vec<const cx<TI>> X,
               Vec<const cx<T>> B, Vec<cx<T>> Y, int nslots);

// b_c = P^T r  (fine level with n cells -> n/2)
template <typename T>
void restrict2d(hipStream_t st, int n, Vec<const cx<T>> R, Vec<cx<T>> Bc, int nslots);

// b_c = P^T (b - L x), residual formed on the fly
template <typename T>
void resid_restrict2d(hipStream_t st, const Op2<T>& op, Vec<const cx<T>> X, Vec<const cx<T>> B,
                      Vec<cx<T>> Bc, int nslots);

// x += P e  (coarse level with n/2 cells -> fine n)
template <typename T>
void prolong2d(hipStream_t st, int n, Vec<const cx<T>> E, Vec<cx<T>> X, int nslots);

// ---- fused 2D multigrid kernels (kernels2d_fused.hip) ----------------------
// x = two Jacobi sweeps for L x = b from x = 0
template <typename T>
void pre0_2d(hipStream_t st, const Op2<T>& L, Vec<const cx<T>> B, Vec<cx<T>> X, int ns);
// rho = c (R - B_shift u) (u = 0 when U.base is null), written; then x as
// in pre0_2d with b = rho
template <typename T>
void hss_pre0_2d(hipStream_t st, const Op2<T>& L, const Op2<T>& Bs, T c, Vec<const cx<T>> U,
                 Vec<const cx<T>> R, Vec<cx<T>> Rho, Vec<cx<T>> X, int ns);
// x_out = S Jacobi sweeps from x_in (+ P e_c when Ec.base is set); with
// update, x_out += result instead.  S in {1, 2, 4}.
template <typename T>
void sweeps_2d(hipStream_t st, const Op2<T>& L, int S, Vec<const cx<T>> Xin, Vec<const cx<T>> Ec,
               Vec<const cx<T>> B, Vec<cx<T>> Xout, bool update, int ns);

// as pre0_2d / hss_pre0_2d, and also b_c = P^T (b - L x) on the n/2 mesh
template <typename T>
void pre0r_2d(hipStream_t st, const Op2<T>& L, Vec<const cx<T>> B, Vec<cx<T>> X, Vec<cx<T>> Bc,
              int ns);
template <typename T>
void hss_pre0r_2d(hipStream_t st, const Op2<T>& L, const Op2<T>& Bs, T c, Vec<const cx<T>> U,
                  Vec<const cx<T>> R, Vec<cx<T>> Rho, Vec<cx<T>> X, Vec<cx<T>> Bc, int ns);

// ---- register-streaming 2D kernels (kernels2d_stream.hip) -----------------
// Work split: strips of 64 columns (one per lane) x segments of H rows x
// slots; one wavefront per unit.  The units on the mesh boundary (first and
// last strip or segment) form the first `eblocks` workgroups.
struct StreamGrid {
    int H;
    unsigned strips, segs, units;
    unsigned edge_units, eblocks;
};
StreamGrid stream_grid(int n, int halo, int ns, int H);
// x_out = S Jacobi sweeps from x_in (+ P e_c when Ec.base is set); with
// update, x_out += result; when Bc.base is set, also b_c = P^T (b - L x_out)
// on the n/2 mesh.  Supported: (S, prolong, restrict, update) in
// {(4,1,1,0), (2,1,0,1), (2,1,0,0), (2,0,1,0), (4,1,0,0), (1,0,0,0)};
// returns false (and launches nothing) for any other.
template <typename T>
bool stream_sweeps_2d(hipStream_t st, const Op2<T>& L, int S, Vec<const cx<T>> Xin,
                      Vec<const cx<T>> Ec, Vec<const cx<T>> B, Vec<cx<T>> Xout, Vec<cx<T>> Bc,
                      bool update, int ns);
// Measuring segment heights on first use (on by default) for the calling
// thread; returns the previous setting.  Off: heights not measured yet come
// from the model, and no timing launch or event is made.
bool stream_tuning(bool on);
// two zero-guess pre-smoothing sweeps x for L x = b and b_c = P^T (b - L x);
// b given (B.base set), or b = rho = c (R - B_shift u) (U.base set) or
// rho = c R (neither), rho then written.
template <typename T>
void stream_pre_2d(hipStream_t st, const Op2<T>& L, const Op2<T>& Bs, T c, Vec<const cx<T>> U,
                   Vec<const cx<T>> R, Vec<cx<T>> Rho, Vec<const cx<T>> B, Vec<cx<T>> X,
                   Vec<cx<T>> Bc, int ns);

// ---- small-level V-cycle in LDS (kernels2d_small.hip) ---------------------
// Levels 0..nlev-1 of this record are consecutive mesh levels; the last is
// the coarsest (solved with the dense FP64 inverse).  Offsets are in
// complex elements of the dynamic LDS arena; t is shared by all levels and
// also holds the coarse solve's FP64 partial sums (off_part).  mdiv[l] =
// ceil(2^20 / (n[l] + 1)) turns a node index into its row by a multiply.
constexpr int MAX_SMALL = 8;
template <typename T>
struct SmallCycle {
    int nlev;
    int n[MAX_SMALL];
    Op2<T> op[MAX_SMALL];
    int off_b[MAX_SMALL], off_x[MAX_SMALL], off_t[MAX_SMALL];
    int mdiv[MAX_SMALL];
    int off_part;
};
template <typename T>
void vcycle_small(hipStream_t st, const SmallCycle<T>& sc, size_t lds_bytes, const cxd* Ainv,
                  int nc, Vec<const cx<T>> B, Vec<cx<T>> X, int ns);

// ---- 3D Q1 stencils (kernels3d.hip) ---------------------------------------
// tiled: levels n >= 128 run the z-marching column-tile kernel for the
// interior nodes and a boundary-node kernel; otherwise (and for
// MODE_JACOBI0) one thread per node
template <typename T, typename TI>
void stencil3d(hipStream_t st, const Op3<T>& op, int mode, T s, Vec<const cx<TI>> X,
               Vec<const cx<T>> B, Vec<cx<T>> Y, int nslots, bool tiled = true);
template <typename T>
void restrict3d(hipStream_t st, int n, Vec<const cx<T>> R, Vec<cx<T>> Bc, int nslots);
template <typename T>
void prolong3d(hipStream_t st, int n, Vec<const cx<T>> E, Vec<cx<T>> X, int nslots);

// ---- fused z-marching 3D Q1 passes (kernels3d_fused.hip) ------------------
// Operator record of a K + b M + c M_Gamma on one 3D level for the fused
// passes: the coefficients of the per-plane terms T1 = uK PK + uM PMM +
// uG PG and T0 = vK PK + vM PMM + vG PG (uK = (h/6) a, uM = (h/6) b - a/h,
// uG = (h/6) c, vK = 4 (h/6) a, vM = 4 (h/6) b + 2 a/h, vG = 4 (h/6) c),
// c for the end planes, and omega / D by the number of coordinates of the
// node on the mesh boundary (0 interior, 1 face, 2 edge, 3 corner; the
// diagonal is symmetric in the three axes).
// Interior columns (no boundary line in x or y) use T1 = i1[0] a0 +
// i1[1] (H + V) + i1[2] a2 and T0 = i0[.] likewise, and on the first and
// last plane T0/2 + c PMM = j0[.] likewise.
template <typename T>
struct Op3F {
    cx<T> i1[3], i0[3], j0[3];  // T1, T0, and T0 of an end plane minus T0, on interior columns
    // the same weights split (the K factor a is real): real parts, and the
    // imaginary parts as k * (16, 4, 1) (the in-plane mass pattern)
    T r1[3], r0[3], rj[3];
    T k1, k0, kj;
    cx<T> e1[3], e0[3], f0[3];  // their changes on a boundary column (see kernels3d_fused.hip)
    cx<T> od[4];
    int n;
    unsigned dir;  // Dirichlet faces (x0=1 .. z1=32): every pass writes zero on their nodes
};
struct Grid3F {
    int tiles_x, tiles_y, segs, tz;  // tiles per side, plane segments, planes per segment
};
// first stage of a fused pass
enum Pass3First : int {
    F_APPLY = 0,  // y = L x
    F_RESID = 1,  // y = s (b - L x)
    F_JAC = 2,    // x1 = x + w/D (b - L x)   (x + P e_c with the prolongation)
    F_HSS = 3,    // rho = s (R - B u), x1 = w/D rho
    F_HSS0 = 4,   // rho = s R, x1 = w/D rho
    F_PRE0 = 5,   // x1 = w/D b
    F_JAC0 = 6,   // x1 = x0 + w/D (b - L x0), x0 = w/D b: both zero-guess sweeps
};
// One fused pass: the first stage, and with ns = 2 a Jacobi sweep on its
// output (b = rho for the HSS forms).  Supported: ns = 1 with F_APPLY,
// F_RESID, F_JAC, F_PRE0 (any TI), and (TI = T) F_JAC with pro (the input
// is X + P Ec) or upd = 1 (Y += result), F_HSS, F_HSS0, F_JAC0 (X unused:
// the input planes are w/D b, formed from Bv); ns = 2 (TI = T)
// with F_JAC (pro, upd as before), F_HSS, F_HSS0, F_PRE0.  X, Bv,
// Ec, Rho, Y as the form needs; Y must not alias X.  tz: planes per
// segment (0 = from the launch shape).  Returns false (and launches
// nothing) for an unsupported combination.
template <typename T, typename TI>
bool pass3d(hipStream_t st, const Op3F<T>& L, const Op3F<T>& B, int first, int ns, bool pro, int upd,
            T s, Vec<const cx<TI>> X, Vec<const cx<T>> Bv, Vec<const cx<T>> Ec, Vec<cx<T>> Rho,
            Vec<cx<T>> Y, int nslots, int tz = 0);
// b_c = P^T (b - L x), the n mesh to the n/2 mesh, in one pass
template <typename T>
void rr3d(hipStream_t st, const Op3F<T>& L, Vec<const cx<T>> X, Vec<const cx<T>> Bv, Vec<cx<T>> Bc,
          int nslots, int tz = 0);

// ---- mixed [DG0]^2 x P1 formulation (kernels2d_mixed.hip) ------------------
// X, B, Y of mixed vectors [u | sigma] (sigma after the N = (n+1)^2 nodes).
// y = sb B_u + Op u + G^T (sa sigma + sg g) at the nodes (B, G nullable; G
// holds 4 n^2 triangle values per slot); Y addresses node vectors.
template <typename T, typename TI>
void mixed_nodes(hipStream_t st, const Op2<T>& op, cx<T> sb, cx<T> sa, cx<T> sg,
                 Vec<const cx<TI>> X, Vec<const cx<T>> B, Vec<const cx<T>> G, Vec<cx<T>> Y,
                 int nslots);
// sigma rows: y = area (s sigma - grad u)  or  B - area (s sigma - grad u)
template <typename T, typename TI>
void mixed_tris(hipStream_t st, int n, int mode, cx<T> s, Vec<const cx<TI>> X, Vec<const cx<T>> B,
                Vec<cx<T>> Y, int nslots);
// g = nukp sigma + nu grad u + c R_sigma / area
template <typename T>
void mixed_g(hipStream_t st, int n, cx<T> nukp, T nu, T c, Vec<const cx<T>> X, Vec<const cx<T>> R,
             Vec<cx<T>> G, int nslots);
// sigma = inv (grad u + g)
template <typename T>
void mixed_sigma(hipStream_t st, int n, cx<T> inv, Vec<const cx<T>> X, Vec<const cx<T>> G,
                 Vec<cx<T>> Y, int nslots);

// ---- vector kernels (kernels_vec.hip) ----------------------------------------
// x = Ainv b on the coarsest mesh, Ainv dense complex FP64 (nc x nc, row-major)
template <typename T>
void coarse_apply(hipStream_t st, const cxd* Ainv, int nc, Vec<const cx<T>> B, Vec<cx<T>> X,
                  int nslots);
// y = x (type conversion allowed)
template <typename TO, typename TI>
void copy_cast(hipStream_t st, long long N, Vec<const cx<TI>> X, Vec<cx<TO>> Y, int nslots);
// y += alpha x
template <typename T>
void axpy1(hipStream_t st, long long N, T alpha, Vec<const cx<T>> X, Vec<cx<T>> Y, int nslots);
// y = alpha x, alpha real per slot: y = x / div[slot]  (div read on device)
void scale_inv(hipStream_t st, long long N, Vec<const cxd> X, Vec<cxd> Y, const double* div,
               int div_stride, int nslots);
// partial dot products: part[slot][i][blk] = sum_{n in blk} conj(V_i[n]) w[n], i < m
// V_i at Vb.at(slot) + i*N
int multidot_blocks(long long N);
// mlen (nullable, device): per-slot vector count <= m; m sets the layout.
// wpart (nullable): also wpart[slot][blk] = sum_{n in blk} |w[n]|^2.
// flag (nullable, device): slots with flag[slot] == 0 are skipped.
void multidot(hipStream_t st, long long N, int m, const int* mlen, Vec<const cxd> V,
              Vec<const cxd> W, cxd* part, int nslots, double* wpart = nullptr,
              const int* flag = nullptr);
// reduce part over blocks: out[slot*ostride + i] (+)= sum_blk part[slot][i][blk];
// slots with flag[slot] == 0 get 0 (or keep out when accumulating)
void reduce_parts(hipStream_t st, int m, const int* mlen, int nblk, const cxd* part, cxd* out,
                  int ostride, int accumulate, int nslots, const int* flag = nullptr);
// flag[slot] = 1 when |w|^2 - |h|^2 < |w|^2 / 2 (|w|^2 from multidot's wpart,
// h the first Gram-Schmidt pass's coefficients), else 0
void reorth_flag(hipStream_t st, int m, const int* mlen, int nblk, const double* wpart,
                 const cxd* h, int hstride, int* flag, int nslots);
// w -= sum_{i<m} h[slot*hstride + i] V_i; slots with flag[slot] == 0 skipped
void multi_axpy(hipStream_t st, long long N, int m, const int* mlen, Vec<const cxd> V,
                const cxd* h, int hstride, Vec<cxd> W, int nslots, const int* flag = nullptr);
// squared norm partials: part[slot][blk] = sum |w|^2 ; reduced into out[slot*ostride]
void norm2(hipStream_t st, long long N, Vec<const cxd> W, double* part, double* out, int ostride,
           int nslots);
// x += sum_{i<m} y[slot*ystride + i] Z_i  (Z in FP64 or FP32)
template <typename TZ>
void update_solution(hipStream_t st, long long N, int m, const int* mlen, Vec<const cx<TZ>> Z,
                     const cxd* y, int ystride, Vec<cxd> X, int nslots);
// m-step GMRES least squares per slot (Hessenberg hu, norms hn, see
// kernels_vec.hip); y[slot*m + i]; m <= 20
void gmres_lsq(hipStream_t st, int m, cxd* hu, int hs, const double* hn, cxd* y, int nslots);
// b = f (real -> complex)
void real_to_complex(hipStream_t st, long long N, const double* f, cxd* b, int nslots);

}  // namespace helm
