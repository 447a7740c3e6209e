// Fused 2D P1 multigrid kernels with LDS tiles and temporal blocking.
//
// A workgroup owns a TX x TY tile of output nodes.  It stages its inputs in
// LDS with a halo as wide as the number of dependent stencil passes it
// performs, runs those passes in LDS on shrinking regions (each pass needs
// one more ring of neighbours than the next), and writes only the tile.
// Values are identical to running the passes one launch at a time (same
// arithmetic per node); the halo rings are recomputed by neighbouring tiles.
//
//   k_pre0<HSS>:  [rho = c (R - B u) on the tile + 1 ring; write rho]
//                 t = omega D^{-1} b,  x = t + omega D^{-1} (b - L t)
//                 = the two pre-smoothing sweeps from a zero initial guess
//                 (b = rho when HSS).
//   k_sweeps<S>:  x <- x_in [+ P e_c]; then S sweeps x <- x + omega D^{-1}
//                 (b - L x); write x_out, or u += x when updating the HSS
//                 iterate.  S = 2 is the post-smoothing of a cycle; S = 4
//                 merges it with the pre-smoothing of the next cycle, which
//                 starts from this cycle's result.
#include "launch.h"
#include "stencil_rows.h"

namespace helm {

namespace {

template <typename T>
__device__ __forceinline__ cx<T> czero() { return mk((T)0, (T)0); }

// Jacobi factor omega / D at node (i, j)
template <typename T>
__device__ __forceinline__ cx<T> jac_factor(const Op2<T>& op, int i, int j, bool interior) {
    return interior ? op.odC : jacobi_factor(op, i, j);
}

// (Op x) at node (i, j) with x read from an LDS region of width W whose
// element for node (i, j) is at p (neighbours at p +- 1, p +- W).
template <typename T>
__device__ __forceinline__ cx<T> apply_lds(const Op2<T>& op, const cx<T>* s, int p, int W, int i,
                                           int j, bool interior) {
    if (interior) {
        cx<T> sa = (s[p + 1] + s[p - 1]) + (s[p + W] + s[p - W]);
        cx<T> sd = s[p + W + 1] + s[p - W - 1];
        return cfma(op.wDg, sd, cfma(op.wAx, sa, op.wC * s[p]));
    }
    const int n = op.n;
    Row7<T> r = row_weights(op, i, j);
    cx<T> acc = r.w[0] * s[p];
    if (i < n) acc = cfma(r.w[1], s[p + 1], acc);
    if (i > 0) acc = cfma(r.w[2], s[p - 1], acc);
    if (j < n) acc = cfma(r.w[3], s[p + W], acc);
    if (j > 0) acc = cfma(r.w[4], s[p - W], acc);
    if (i < n && j < n) acc = cfma(r.w[5], s[p + W + 1], acc);
    if (i > 0 && j > 0) acc = cfma(r.w[6], s[p - W - 1], acc);
    return acc;
}

struct TileInfo {
    int slot, x0, y0;
};

template <int TX, int TY>
__device__ __forceinline__ TileInfo tile_info(int n, unsigned tiles_x, unsigned tiles_per_slot) {
    const unsigned lin = xcd_remap(blockIdx.x, gridDim.x);
    TileInfo ti;
    ti.slot = lin / tiles_per_slot;
    const unsigned r = lin % tiles_per_slot;
    ti.x0 = (int)(r % tiles_x) * TX;
    ti.y0 = (int)(r / tiles_x) * TY;
    return ti;
}

// Load the region of radius RAD around the tile into LDS (zeros outside the
// mesh).  Region element (a, b) is node (x0 - RAD + a, y0 - RAD + b).
// All of a thread's global loads are issued before any LDS store so that
// they are in flight together (one memory latency per staging, not one per
// element).
template <typename T, int TX, int TY, int RAD, int NT>
__device__ __forceinline__ void load_region(cx<T>* dst, const cx<T>* src, int n, int x0, int y0) {
    constexpr int W = TX + 2 * RAD, H = TY + 2 * RAD, CNT = W * H;
    constexpr int IT = (CNT + NT - 1) / NT;
    const long long np = n + 1;
    cx<T> v[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int q = threadIdx.x + k * NT;
        const int a = q % W, b = q / W;
        const int i = x0 - RAD + a, j = y0 - RAD + b;
        v[k] = czero<T>();
        if (q < CNT && i >= 0 && i <= n && j >= 0 && j <= n) v[k] = src[(long long)j * np + i];
    }
#pragma unroll
    for (int k = 0; k < IT; ++k) {
        const int q = threadIdx.x + k * NT;
        if (q < CNT) dst[q] = v[k];
    }
}

// ---- k_pre0 ---------------------------------------------------------------
// HSS = 0: b given (radius 1 staged).  HSS = 1: b = rho = c (R - B u) formed
// on radius 1 from u (radius 2 staged) and R; rho written on the tile.
// HSS = 2: first HSS step, u = 0: rho = c R.
template <typename T, int TX, int TY, int HSS, int NT>
__global__ __launch_bounds__(NT) void k_pre0(Op2<T> L, Op2<T> Bs, T c, Vec<const cx<T>> U,
                                             Vec<const cx<T>> Rv, Vec<cx<T>> Rho,
                                             Vec<const cx<T>> Bv, Vec<cx<T>> X, unsigned tiles_x,
                                             unsigned tiles_per_slot) {
    constexpr int W1 = TX + 2, H1 = TY + 2;
    constexpr int W2 = TX + 4, H2 = TY + 4;
    __shared__ cx<T> sb[W1 * H1];
    __shared__ cx<T> st[W1 * H1];
    __shared__ cx<T> su[HSS == 1 ? W2 * H2 : 1];
    const int n = L.n;
    const long long np = n + 1;
    const TileInfo ti = tile_info<TX, TY>(n, tiles_x, tiles_per_slot);
    if (HSS == 0) {
        load_region<T, TX, TY, 1, NT>(sb, Bv.at(ti.slot), n, ti.x0, ti.y0);
        __syncthreads();
    } else {
        const cx<T>* R = Rv.at(ti.slot);
        constexpr int CNT = W1 * H1, IT = (CNT + NT - 1) / NT;
        cx<T> rv[IT];
#pragma unroll
        for (int k = 0; k < IT; ++k) {  // R on radius 1, all loads in flight
            const int q = threadIdx.x + k * NT;
            const int a = q % W1, b = q / W1;
            const int i = ti.x0 - 1 + a, j = ti.y0 - 1 + b;
            rv[k] = czero<T>();
            if (q < CNT && i >= 0 && i <= n && j >= 0 && j <= n) rv[k] = R[(long long)j * np + i];
        }
        if (HSS == 1) load_region<T, TX, TY, 2, NT>(su, U.at(ti.slot), n, ti.x0, ti.y0);
        __syncthreads();
        cx<T>* rho = Rho.at(ti.slot);
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int q = threadIdx.x + k * NT;
            if (q >= CNT) continue;
            const int a = q % W1, b = q / W1;
            const int i = ti.x0 - 1 + a, j = ti.y0 - 1 + b;
            cx<T> v = czero<T>();
            if (i >= 0 && i <= n && j >= 0 && j <= n) {
                if (HSS == 1) {
                    const bool in = (i > 0) & (i < n) & (j > 0) & (j < n);
                    const cx<T> bu = apply_lds(Bs, su, (b + 1) * W2 + (a + 1), W2, i, j, in);
                    v = c * (rv[k] - bu);
                } else {
                    v = c * rv[k];
                }
                if (a >= 1 && a <= TX && b >= 1 && b <= TY) rho[(long long)j * np + i] = v;
            }
            sb[q] = v;
        }
        __syncthreads();
    }
    // t = omega D^{-1} b on radius 1
    for (int q = threadIdx.x; q < W1 * H1; q += NT) {
        const int a = q % W1, b = q / W1;
        const int i = ti.x0 - 1 + a, j = ti.y0 - 1 + b;
        cx<T> v = czero<T>();
        if (i >= 0 && i <= n && j >= 0 && j <= n) {
            const bool in = (i > 0) & (i < n) & (j > 0) & (j < n);
            v = jac_factor(L, i, j, in) * sb[q];
        }
        st[q] = v;
    }
    __syncthreads();
    // x = t + omega D^{-1} (b - L t) on the tile
    cx<T>* x = X.at(ti.slot);
    for (int q = threadIdx.x; q < TX * TY; q += NT) {
        const int a = q % TX, b = q / TX;
        const int i = ti.x0 + a, j = ti.y0 + b;
        if (i > n || j > n) continue;
        const int p = (b + 1) * W1 + (a + 1);
        const bool in = (i > 0) & (i < n) & (j > 0) & (j < n);
        const cx<T> lt = apply_lds(L, st, p, W1, i, j, in);
        x[(long long)j * np + i] = cfma(jac_factor(L, i, j, in), sb[p] - lt, st[p]);
    }
}

// ---- k_pre0r --------------------------------------------------------------
// k_pre0 followed by the residual restriction, in one pass: the two
// zero-guess pre-smoothing sweeps are formed on the tile plus one ring, the
// residual r = b - L x on the tile plus one ring, and every coarse node
// (I, J) whose fine node (2I, 2J) lies in the tile gets
// b_c(I, J) = r(2I, 2J) + (1/2) sum of r over its six fine edge neighbours.
// HSS = 1/2 form b = rho = c (R - B u) first (u = 0 for HSS = 2), writing rho.
template <typename T, int TX, int TY, int HSS, int NT>
__global__ __launch_bounds__(NT) void k_pre0r(Op2<T> L, Op2<T> Bs, T c, Vec<const cx<T>> U,
                                              Vec<const cx<T>> Rv, Vec<cx<T>> Rho,
                                              Vec<const cx<T>> Bv, Vec<cx<T>> X, Vec<cx<T>> Bc,
                                              unsigned tiles_x, unsigned tiles_per_slot) {
    constexpr int W4 = TX + 8, H4 = TY + 8;
    constexpr int W3 = TX + 6, H3 = TY + 6;
    constexpr int W2 = TX + 4, H2 = TY + 4;
    constexpr int W1 = TX + 2, H1 = TY + 2;
    __shared__ cx<T> sb[W3 * H3];   // b (radius 3)
    __shared__ cx<T> st[W3 * H3];   // t = omega D^{-1} b (radius 3), then r (radius 1)
    __shared__ cx<T> sx[W2 * H2];   // x (radius 2)
    __shared__ cx<T> su[HSS == 1 ? W4 * H4 : 1];
    const int n = L.n;
    const long long np = n + 1;
    const TileInfo ti = tile_info<TX, TY>(n, tiles_x, tiles_per_slot);
    if (HSS == 0) {
        load_region<T, TX, TY, 3, NT>(sb, Bv.at(ti.slot), n, ti.x0, ti.y0);
        __syncthreads();
    } else {
        const cx<T>* R = Rv.at(ti.slot);
        constexpr int CNT = W3 * H3, IT = (CNT + NT - 1) / NT;
        cx<T> rv[IT];
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int q = threadIdx.x + k * NT;
            const int a = q % W3, b = q / W3;
            const int i = ti.x0 - 3 + a, j = ti.y0 - 3 + b;
            rv[k] = czero<T>();
            if (q < CNT && i >= 0 && i <= n && j >= 0 && j <= n) rv[k] = R[(long long)j * np + i];
        }
        if (HSS == 1) load_region<T, TX, TY, 4, NT>(su, U.at(ti.slot), n, ti.x0, ti.y0);
        __syncthreads();
        cx<T>* rho = Rho.at(ti.slot);
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int q = threadIdx.x + k * NT;
            if (q >= CNT) continue;
            const int a = q % W3, b = q / W3;
            const int i = ti.x0 - 3 + a, j = ti.y0 - 3 + b;
            cx<T> v = czero<T>();
            if (i >= 0 && i <= n && j >= 0 && j <= n) {
                if (HSS == 1) {
                    const bool in = (i > 0) & (i < n) & (j > 0) & (j < n);
                    v = c * (rv[k] - apply_lds(Bs, su, (b + 1) * W4 + (a + 1), W4, i, j, in));
                } else {
                    v = c * rv[k];
                }
                if (a >= 3 && a < 3 + TX && b >= 3 && b < 3 + TY) rho[(long long)j * np + i] = v;
            }
            sb[q] = v;
        }
        __syncthreads();
    }
    // t = omega D^{-1} b on radius 3
    for (int q = threadIdx.x; q < W3 * H3; q += NT) {
        const int a = q % W3, b = q / W3;
        const int i = ti.x0 - 3 + a, j = ti.y0 - 3 + b;
        cx<T> v = czero<T>();
        if (i >= 0 && i <= n && j >= 0 && j <= n) {
            const bool in = (i > 0) & (i < n) & (j > 0) & (j < n);
            v = jac_factor(L, i, j, in) * sb[q];
        }
        st[q] = v;
    }
    __syncthreads();
    // x = t + omega D^{-1} (b - L t) on radius 2; the tile is written out
    cx<T>* x = X.at(ti.slot);
    for (int q = threadIdx.x; q < W2 * H2; q += NT) {
        const int a = q % W2, b = q / W2;
        const int i = ti.x0 - 2 + a, j = ti.y0 - 2 + b;
        const int p3 = (b + 1) * W3 + (a + 1);
        cx<T> v = czero<T>();
        if (i >= 0 && i <= n && j >= 0 && j <= n) {
            const bool in = (i > 0) & (i < n) & (j > 0) & (j < n);
            const cx<T> lt = apply_lds(L, st, p3, W3, i, j, in);
            v = cfma(jac_factor(L, i, j, in), sb[p3] - lt, st[p3]);
            if (a >= 2 && a < 2 + TX && b >= 2 && b < 2 + TY) x[(long long)j * np + i] = v;
        }
        sx[q] = v;
    }
    __syncthreads();
    // r = b - L x on radius 1 (stored in st, width W1)
    for (int q = threadIdx.x; q < W1 * H1; q += NT) {
        const int a = q % W1, b = q / W1;
        const int i = ti.x0 - 1 + a, j = ti.y0 - 1 + b;
        cx<T> v = czero<T>();
        if (i >= 0 && i <= n && j >= 0 && j <= n) {
            const bool in = (i > 0) & (i < n) & (j > 0) & (j < n);
            v = sb[(b + 2) * W3 + (a + 2)] - apply_lds(L, sx, (b + 1) * W2 + (a + 1), W2, i, j, in);
        }
        st[q] = v;
    }
    __syncthreads();
    // restriction to the coarse nodes owned by this tile
    const int nc = n / 2;
    const long long npc = nc + 1;
    cx<T>* bc = Bc.at(ti.slot);
    for (int q = threadIdx.x; q < (TX / 2) * (TY / 2); q += NT) {
        const int A = q % (TX / 2), B = q / (TX / 2);
        const int I = ti.x0 / 2 + A, J = ti.y0 / 2 + B;
        if (I > nc || J > nc) continue;
        const int p = (2 * B + 1) * W1 + (2 * A + 1);  // fine (2I, 2J) in the radius-1 array
        const cx<T> s6 = (st[p + 1] + st[p - 1]) + (st[p + W1] + st[p - W1]) +
                         (st[p + W1 + 1] + st[p - W1 - 1]);
        bc[(long long)J * npc + I] = st[p] + (T)0.5 * s6;
    }
}

// ---- k_sweeps -------------------------------------------------------------
template <typename T, int TX, int TY, int S, bool PROLONG, bool UPDATE, int NT>
__global__ __launch_bounds__(NT) void k_sweeps(Op2<T> L, Vec<const cx<T>> Xin, Vec<const cx<T>> Ec,
                                               Vec<const cx<T>> Bv, Vec<cx<T>> Xout,
                                               unsigned tiles_x, unsigned tiles_per_slot) {
    constexpr int WS = TX + 2 * S, HS = TY + 2 * S;           // x, radius S
    constexpr int WB = TX + 2 * (S - 1), HB = TY + 2 * (S - 1);  // b, radius S-1
    __shared__ cx<T> sa[WS * HS];
    __shared__ cx<T> sc[WS * HS];
    __shared__ cx<T> sb[WB * HB];
    const int n = L.n;
    const long long np = n + 1;
    const TileInfo ti = tile_info<TX, TY>(n, tiles_x, tiles_per_slot);
    // stage x (+ P e_c) on radius S and b on radius S-1
    {
        const cx<T>* xin = Xin.at(ti.slot);
        const cx<T>* e = PROLONG ? Ec.at(ti.slot) : nullptr;
        const long long npc = n / 2 + 1;
        constexpr int CNT = WS * HS, IT = (CNT + NT - 1) / NT;
        cx<T> xv[IT], e0[PROLONG ? IT : 1], e1[PROLONG ? IT : 1];
        // issue every load first (x, and the one or two coarse values of P e_c)
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int q = threadIdx.x + k * NT;
            const int a = q % WS, b = q / WS;
            const int i = ti.x0 - S + a, j = ti.y0 - S + b;
            xv[k] = czero<T>();
            if (PROLONG) e0[k] = e1[k] = czero<T>();
            if (q < CNT && i >= 0 && i <= n && j >= 0 && j <= n) {
                xv[k] = xin[(long long)j * np + i];
                if (PROLONG) {
                    const long long cidx = (long long)(j >> 1) * npc + (i >> 1);
                    const int oi = i & 1, oj = j & 1;
                    e0[k] = e[cidx];
                    e1[k] = e[cidx + oi + (long long)oj * npc];  // = e0 at even-even nodes
                }
            }
        }
        load_region<T, TX, TY, S - 1, NT>(sb, Bv.at(ti.slot), n, ti.x0, ti.y0);
#pragma unroll
        for (int k = 0; k < IT; ++k) {
            const int q = threadIdx.x + k * NT;
            if (q < CNT) sa[q] = PROLONG ? xv[k] + (T)0.5 * (e0[k] + e1[k]) : xv[k];
        }
    }
    __syncthreads();
    cx<T>* cur = sa;
    cx<T>* nxt = sc;
#pragma unroll
    for (int s = 1; s <= S; ++s) {
        const int r = S - s;  // radius of this pass's region
        const int Wr = TX + 2 * r, Hr = TY + 2 * r;
        for (int q = threadIdx.x; q < Wr * Hr; q += NT) {
            const int a = q % Wr, b = q / Wr;
            const int i = ti.x0 - r + a, j = ti.y0 - r + b;
            // position in the radius-S array and in the b array
            const int p = (b + s) * WS + (a + s);
            const int pb = (b + s - 1) * WB + (a + s - 1);
            cx<T> v = czero<T>();
            if (i >= 0 && i <= n && j >= 0 && j <= n) {
                const bool in = (i > 0) & (i < n) & (j > 0) & (j < n);
                const cx<T> lx = apply_lds(L, cur, p, WS, i, j, in);
                v = cfma(jac_factor(L, i, j, in), sb[pb] - lx, cur[p]);
            }
            if (s < S) {
                nxt[p] = v;
            } else if (i <= n && j <= n) {
                cx<T>* out = Xout.at(ti.slot);
                const long long g = (long long)j * np + i;
                if (UPDATE) out[g] = out[g] + v;
                else out[g] = v;
            }
        }
        if (s < S) {
            __syncthreads();
            cx<T>* tmp = cur;
            cur = nxt;
            nxt = tmp;
        }
    }
}

template <int TX, int TY>
inline void grid_dims(int n, int ns, unsigned& tiles_x, unsigned& per_slot, unsigned& total) {
    tiles_x = (unsigned)((n + 1 + TX - 1) / TX);
    const unsigned tiles_y = (unsigned)((n + 1 + TY - 1) / TY);
    per_slot = tiles_x * tiles_y;
    total = per_slot * (unsigned)ns;
}

}  // namespace

// tile shape and workgroup size of the fused kernels
constexpr int FX = 64, FY = 8, FNT = 256;

template <typename T>
void pre0_2d(hipStream_t st, const Op2<T>& L, Vec<const cx<T>> B, Vec<cx<T>> X, int ns) {
    unsigned tx, ps, tot;
    grid_dims<FX, FY>(L.n, ns, tx, ps, tot);
    k_pre0<T, FX, FY, 0, FNT><<<tot, FNT, 0, st>>>(L, L, (T)0, Vec<const cx<T>>{}, Vec<const cx<T>>{},
                                             Vec<cx<T>>{}, B, X, tx, ps);
}

template <typename T>
void hss_pre0_2d(hipStream_t st, const Op2<T>& L, const Op2<T>& Bs, T c, Vec<const cx<T>> U,
                 Vec<const cx<T>> R, Vec<cx<T>> Rho, Vec<cx<T>> X, int ns) {
    unsigned tx, ps, tot;
    grid_dims<FX, FY>(L.n, ns, tx, ps, tot);
    if (U.base)
        k_pre0<T, FX, FY, 1, FNT><<<tot, FNT, 0, st>>>(L, Bs, c, U, R, Rho, Vec<const cx<T>>{}, X, tx, ps);
    else
        k_pre0<T, FX, FY, 2, FNT><<<tot, FNT, 0, st>>>(L, Bs, c, U, R, Rho, Vec<const cx<T>>{}, X, tx, ps);
}

template <typename T>
void pre0r_2d(hipStream_t st, const Op2<T>& L, Vec<const cx<T>> B, Vec<cx<T>> X, Vec<cx<T>> Bc,
              int ns) {
    unsigned tx, ps, tot;
    grid_dims<FX, FY>(L.n, ns, tx, ps, tot);
    k_pre0r<T, FX, FY, 0, FNT><<<tot, FNT, 0, st>>>(L, L, (T)0, Vec<const cx<T>>{},
                                                    Vec<const cx<T>>{}, Vec<cx<T>>{}, B, X, Bc, tx, ps);
}

template <typename T>
void hss_pre0r_2d(hipStream_t st, const Op2<T>& L, const Op2<T>& Bs, T c, Vec<const cx<T>> U,
                  Vec<const cx<T>> R, Vec<cx<T>> Rho, Vec<cx<T>> X, Vec<cx<T>> Bc, int ns) {
    unsigned tx, ps, tot;
    grid_dims<FX, FY>(L.n, ns, tx, ps, tot);
    if (U.base)
        k_pre0r<T, FX, FY, 1, FNT><<<tot, FNT, 0, st>>>(L, Bs, c, U, R, Rho, Vec<const cx<T>>{}, X, Bc,
                                                        tx, ps);
    else
        k_pre0r<T, FX, FY, 2, FNT><<<tot, FNT, 0, st>>>(L, Bs, c, U, R, Rho, Vec<const cx<T>>{}, X, Bc,
                                                        tx, ps);
}

template <typename T>
void sweeps_2d(hipStream_t st, const Op2<T>& L, int S, Vec<const cx<T>> Xin, Vec<const cx<T>> Ec,
               Vec<const cx<T>> B, Vec<cx<T>> Xout, bool update, int ns) {
    unsigned tx, ps, tot;
    grid_dims<FX, FY>(L.n, ns, tx, ps, tot);
    const bool pro = Ec.base != nullptr;
#define HELM_SWEEPS(SS, PP, UU) \
    k_sweeps<T, FX, FY, SS, PP, UU, FNT><<<tot, FNT, 0, st>>>(L, Xin, Ec, B, Xout, tx, ps)
    if (S == 2) {
        if (pro) { if (update) HELM_SWEEPS(2, true, true); else HELM_SWEEPS(2, true, false); }
        else { if (update) HELM_SWEEPS(2, false, true); else HELM_SWEEPS(2, false, false); }
    } else if (S == 4) {
        if (pro) HELM_SWEEPS(4, true, false);
        else HELM_SWEEPS(4, false, false);
    } else if (S == 1) {
        HELM_SWEEPS(1, false, false);
    }
#undef HELM_SWEEPS
}

template void pre0_2d<double>(hipStream_t, const Op2<double>&, Vec<const cxd>, Vec<cxd>, int);
template void pre0_2d<float>(hipStream_t, const Op2<float>&, Vec<const cxf>, Vec<cxf>, int);
template void hss_pre0_2d<double>(hipStream_t, const Op2<double>&, const Op2<double>&, double,
                                  Vec<const cxd>, Vec<const cxd>, Vec<cxd>, Vec<cxd>, int);
template void hss_pre0_2d<float>(hipStream_t, const Op2<float>&, const Op2<float>&, float,
                                 Vec<const cxf>, Vec<const cxf>, Vec<cxf>, Vec<cxf>, int);
template void pre0r_2d<double>(hipStream_t, const Op2<double>&, Vec<const cxd>, Vec<cxd>, Vec<cxd>,
                               int);
template void pre0r_2d<float>(hipStream_t, const Op2<float>&, Vec<const cxf>, Vec<cxf>, Vec<cxf>,
                              int);
template void hss_pre0r_2d<double>(hipStream_t, const Op2<double>&, const Op2<double>&, double,
                                   Vec<const cxd>, Vec<const cxd>, Vec<cxd>, Vec<cxd>, Vec<cxd>, int);
template void hss_pre0r_2d<float>(hipStream_t, const Op2<float>&, const Op2<float>&, float,
                                  Vec<const cxf>, Vec<const cxf>, Vec<cxf>, Vec<cxf>, Vec<cxf>, int);
template void sweeps_2d<double>(hipStream_t, const Op2<double>&, int, Vec<const cxd>,
                                Vec<const cxd>, Vec<const cxd>, Vec<cxd>, bool, int);
template void sweeps_2d<float>(hipStream_t, const Op2<float>&, int, Vec<const cxf>,
                               Vec<const cxf>, Vec<const cxf>, Vec<cxf>, bool, int);

}  // namespace helm
