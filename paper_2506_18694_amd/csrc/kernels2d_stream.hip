// Register-streaming 2D P1 multigrid kernels (wavefront temporal blocking).
//
// One wavefront owns a strip of 64 mesh columns (one column per lane) and a
// segment of H rows, and marches upward through the segment one row per
// step.  Every dependent pass (Jacobi sweep, residual, restriction) is a
// pipeline stage that lags the previous one by one row: at step t the input
// row t is loaded, sweep s produces row t - s, and so on.  Each stage keeps
// the last three rows it produced in registers; the north and south
// neighbours of a node are in the same lane, the east/west (and the two
// diagonal "/" neighbours) come from the adjacent lanes through wave-wide
// DPP lane shifts.  Nothing is staged in LDS and there are no barriers.
//
// Each stage loses one lane of validity on each side, so a strip computes 64
// columns and owns the 64 - 2R in the middle (R = number of neighbour
// stages); a segment starts its march R rows below its first owned row.
// The arithmetic per node is the same as in the one-pass kernels.
//
// A wavefront whose unit lies away from the mesh boundary applies the
// interior stencil everywhere; lanes and rows outside the mesh then carry
// finite garbage (loads read a clamped, valid address) that no mesh node
// depends on.  A unit that touches a boundary row or column zeroes every
// value outside the mesh and adds to the interior stencil the boundary
// corrections of the operator record (dC, dN, kA, kB), which together give
// the element rows of the edge and corner nodes.  Only owned nodes are
// written.
//
// The march runs in unrolled blocks of steps: within a block the three-row
// rings, the queue of right-hand-side rows and three input buffers rotate
// by renaming registers (the block length is a multiple of every period),
// and the input row t + 2 is loaded while step t computes.  A segment's
// step count is rounded up to whole blocks; the extra steps compute rows
// past the segment, which are never written.
#include <algorithm>
#include <type_traits>

#include "launch.h"
#include "stencil_rows.h"

namespace helm {

namespace {

constexpr int WAVE = 64;
constexpr int SW = 4;     // independent wavefronts per workgroup

template <int V>
using Int = std::integral_constant<int, V>;
template <bool V>
using Bool = std::integral_constant<bool, V>;

template <typename T>
__device__ __forceinline__ cx<T> zero_cx() { return mk((T)0, (T)0); }

// wave-wide lane shifts: lane l receives the value of lane l + 1 (east) or
// lane l - 1 (west); the lanes at the wave ends receive 0 (bound_ctrl, so no
// old value is needed).
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL,
                                                                 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double x) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, true);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane l <- lane l + 1
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane l <- lane l - 1

template <typename T>
__device__ __forceinline__ cx<T> from_east(cx<T> v) {
    return mk(dpp_shift<DPP_WAVE_SHL1>(v.x), dpp_shift<DPP_WAVE_SHL1>(v.y));
}
template <typename T>
__device__ __forceinline__ cx<T> from_west(cx<T> v) {
    return mk(dpp_shift<DPP_WAVE_SHR1>(v.x), dpp_shift<DPP_WAVE_SHR1>(v.y));
}

// Marks a rarely taken branch (boundary rows, boundary columns) as having a
// side effect, so that the compiler keeps it a branch: speculating it would
// evaluate the boundary formulas for every node of every step.
__device__ __forceinline__ void keep_branch() { asm volatile(""); }

// A wave-uniform value re-materialised through readfirstlane, so that
// per-lane selects between such values stay selects of registers (a select
// between two fields of the operator record would otherwise become a
// per-lane load from a stack copy of it).  Only for uniform values.
__device__ __forceinline__ float settle(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double settle(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ cx<T> settle(cx<T> v) { return mk(settle(v.x), settle(v.y)); }
template <typename T>
__device__ __forceinline__ cx<T> sel(bool c, cx<T> a, cx<T> b) {
    return mk(c ? a.x : b.x, c ? a.y : b.y);
}

// Lane and wave facts shared by the stages.
template <typename T>
struct Lanes {
    int i;          // mesh column of this lane (may lie outside 0..n)
    int ic;         // i clamped to 0..n (an address that is always valid)
    bool inx;       // 0 <= i <= n
    bool colb;      // i == 0 or i == n
    bool lo;        // i == 0
    T colbf;        // 1 on a boundary column, else 0
    bool any_colb;  // some lane of the wave is a boundary column (uniform)
    cx<T> jf;       // omega / D in the interior rows: boundary column or not
    cx<T> odC, odE, odA, odB;  // settled factors: interior, boundary rows
};

template <typename T>
__device__ __forceinline__ Lanes<T> lanes_of(const Op2<T>& L, int strip, int owned, int halo) {
    const int n = L.n;
    Lanes<T> ln;
    const int i0 = strip * owned - halo;
    ln.i = i0 + (int)(threadIdx.x % WAVE);
    ln.ic = min(max(ln.i, 0), n);
    ln.inx = ln.i == ln.ic;
    ln.colb = ln.i == 0 || ln.i == n;
    ln.lo = ln.i == 0;
    ln.colbf = ln.colb ? (T)1 : (T)0;
    ln.any_colb = (i0 <= 0 && 0 <= i0 + WAVE - 1) || (i0 <= n && n <= i0 + WAVE - 1);
    ln.odE = settle(L.odE);
    ln.odA = settle(L.odA);
    ln.odB = settle(L.odB);
    ln.odC = settle(L.odC);
    ln.jf = sel(ln.colb, ln.odE, ln.odC);
    return ln;
}

// The last three rows of one stage with the lane-shifted copies the stencil
// needs, in slots that rotate with the phase P of the step: before a step of
// phase P the oldest row is in slot P % 3, the centre in (P + 1) % 3 and the
// newest in (P + 2) % 3; the step's new row replaces the oldest.
template <typename T>
struct Ring {
    cx<T> v[3];  // rows
    cx<T> e[3];  // east neighbours (valid for the centre and the newest)
    cx<T> w[3];  // west neighbours (valid for the oldest and the centre)
};
template <int P>
struct Slots {
    static constexpr int N = P % 3, C = (P + 2) % 3, O = (P + 1) % 3;  // after the push
};

template <typename T>
__device__ __forceinline__ void ring_clear(Ring<T>& g) {
#pragma unroll
    for (int k = 0; k < 3; ++k) g.v[k] = g.e[k] = g.w[k] = zero_cx<T>();
}

template <int P, typename T>
__device__ __forceinline__ void ring_push(Ring<T>& g, cx<T> nv) {
    using Q = Slots<P>;
    g.v[Q::N] = nv;
    g.e[Q::N] = from_east(nv);
    g.w[Q::C] = from_west(g.v[Q::C]);
}

// a + s t for a real s
template <typename T>
__device__ __forceinline__ cx<T> axpy_real(T sc, cx<T> t, cx<T> a) {
    return mk(fmat(sc, t.x, a.x), fmat(sc, t.y, a.y));
}

// (Op v) at the centre row r of g (r uniform across the wave).  EDGE: the
// wavefront's unit touches a boundary row or column and holds zeros outside
// the mesh; otherwise every node it computes is an interior node.
template <int P, bool EDGE, typename T>
__device__ __forceinline__ cx<T> ring_apply(const Op2<T>& op, const Ring<T>& g, const Lanes<T>& ln,
                                            int r) {
    using Q = Slots<P>;
    const cx<T> c = g.v[Q::C], nn = g.v[Q::N], ss = g.v[Q::O];
    const cx<T> ee = g.e[Q::C], ww = g.w[Q::C], ne = g.e[Q::N], sw = g.w[Q::O];
    cx<T> acc = cfma(op.wDg, ne + sw, cfma(op.wAx, (ee + ww) + (nn + ss), op.wC * c));
    if (EDGE) {
        // boundary column: the two neighbours along it and the centre
        acc = axpy_real(ln.colbf, cfma(op.dN, nn + ss, op.dC * c), acc);
        if (r == 0 || r == op.n) {
            keep_branch();
            // boundary row, and at its two corners the remaining centre term
            acc = acc + cfma(op.dN, ee + ww, op.dC * c);
            acc = axpy_real(ln.colbf, sel(ln.lo == (r == 0), op.kA, op.kB) * c, acc);
        }
    }
    return acc;
}

// omega / D at row r
template <bool EDGE, typename T>
__device__ __forceinline__ cx<T> ring_jf(const Lanes<T>& ln, int r, int n) {
    if (!EDGE) return ln.odC;
    if (r == 0 || r == n) {
        keep_branch();
        return sel(ln.colb, sel(ln.lo == (r == 0), ln.odA, ln.odB), ln.odE);
    }
    return ln.jf;
}

// P^T r at the fine node (2I, 2J) = centre row rr of g:
// r(2I, 2J) + (1/2) (sum over its six fine edge neighbours; those outside
// the mesh hold zero in a boundary unit)
template <int P, typename T>
__device__ __forceinline__ cx<T> ring_restrict(const Ring<T>& g) {
    using Q = Slots<P>;
    const cx<T> s6 = ((g.e[Q::C] + g.w[Q::C]) + (g.v[Q::N] + g.v[Q::O])) + (g.e[Q::N] + g.w[Q::O]);
    return cfma(mk((T)0.5, (T)0), s6, g.v[Q::C]);
}

// in a boundary unit: zero outside the mesh (row r uniform)
template <bool EDGE, typename T>
__device__ __forceinline__ cx<T> clip(cx<T> v, const Lanes<T>& ln, int r, int n) {
    if (!EDGE) return v;
    return sel(ln.inx && r >= 0 && r <= n, v, zero_cx<T>());
}

struct Unit {
    int slot, strip, seg;
};

__device__ __forceinline__ bool unit_of(const StreamGrid& gr, Unit& u) {
    const unsigned blk = xcd_remap(blockIdx.x, gridDim.x);
    // the wavefront's index within the workgroup, made visibly uniform so
    // that the unit, the rows and every branch on them stay scalar
    const unsigned wid = (unsigned)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const unsigned id = blk * SW + wid;
    if (id >= gr.units) return false;
    const unsigned per_slot = gr.strips * gr.segs;
    u.slot = (int)(id / per_slot);
    const unsigned r = id % per_slot;
    u.seg = (int)(r / gr.strips);
    u.strip = (int)(r % gr.strips);
    return true;
}

// Loads are issued unconditionally from a clamped (always valid) address,
// so that every step issues the same number of loads and the next rows'
// loads stay in flight while this row computes.
template <typename T>
__device__ __forceinline__ cx<T> load_raw(const cx<T>* p, int ic, int r, int n) {
    const int rc = min(max(r, 0), n);
    return p[(long long)rc * (n + 1) + ic];
}

// slot of the queue entry k steps old at phase p (queue depth D)
template <int D>
__device__ __forceinline__ constexpr int qslot(int p, int k) {
    return ((p - k) % D + D) % D;
}

// ---- k_stream_sweeps --------------------------------------------------------
// x <- x_in [+ P e_c]; S Jacobi sweeps x <- x + omega D^{-1} (b - L x);
// write x, or u += x (UPDATE); with RESID also b_c = P^T (b - L x) on the
// n/2 mesh from the final x.
template <typename T, bool PROLONG, bool UPDATE>
struct SweepIn {
    cx<T> x, b, e0, e1, u;
};

template <typename T, int S, bool PROLONG, bool RESID, bool UPDATE>
__global__ __launch_bounds__(WAVE * SW) __attribute__((amdgpu_waves_per_eu(2))) void k_stream_sweeps(
    Op2<T> L, Vec<const cx<T>> Xin, Vec<const cx<T>> Ec, Vec<const cx<T>> Bv, Vec<cx<T>> Xout,
    Vec<cx<T>> Bc, StreamGrid gr) {
    constexpr int DEPTH = S + (RESID ? 2 : 0);  // lag of the deepest stage
    constexpr int HALO = DEPTH;
    constexpr int OWN = WAVE - 2 * HALO;
    constexpr int NR = S + (RESID ? 2 : 0);
    constexpr int NB = (S + (RESID ? 2 : 1) <= 3) ? 3 : 6;  // queue of b rows
    constexpr int CHUNK = NB;  // steps per block: a multiple of 3 and of NB
    Unit un;
    if (!unit_of(gr, un)) return;
    const int n = L.n;
    const Lanes<T> ln = lanes_of(L, un.strip, OWN, HALO);
    const int lane = (int)(threadIdx.x % WAVE);
    const bool own = lane >= HALO && lane < HALO + OWN && ln.i <= n;
    const int y0 = un.seg * gr.H;
    const int y1 = min(y0 + gr.H, n + 1);  // owned rows [y0, y1)
    const int jl = (y1 - 1) & ~1;          // last even owned row
    const int tb = y0 - HALO;
    const int te = RESID ? jl + S + 2 : y1 - 1 + S;

    const cx<T>* xin = Xin.at(un.slot);
    const cx<T>* e = PROLONG ? Ec.at(un.slot) : nullptr;
    const cx<T>* b = Bv.at(un.slot);
    cx<T>* xo = Xout.at(un.slot);
    cx<T>* bc = RESID ? Bc.at(un.slot) : nullptr;
    const long long np = n + 1, npc = n / 2 + 1;

    Ring<T> rg[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) ring_clear(rg[k]);
    cx<T> bq[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) bq[k] = zero_cx<T>();

    auto load = [&](SweepIn<T, PROLONG, UPDATE>& in, int t) {
        in.x = load_raw(xin, ln.ic, t, n);
        in.b = load_raw(b, ln.ic, t, n);
        if (PROLONG) {
            // P e_c at fine node (i, t): the mean of the coarse values at the
            // two ends of the coarse edge through it (the same coarse node at
            // an even-even fine node)
            const int tc = min(max(t, 0), n);
            const long long c0 = (long long)(tc >> 1) * npc + (ln.ic >> 1);
            in.e0 = e[c0];
            in.e1 = e[c0 + (ln.ic & 1) + (long long)(tc & 1) * npc];
        }
        if (UPDATE) in.u = load_raw((const cx<T>*)xo, ln.ic, t - S, n);
    };

    // one step of phase P: input row t, every stage one row on
    auto step = [&](auto pc, auto ec, const SweepIn<T, PROLONG, UPDATE>& in, int t) {
        constexpr int P = decltype(pc)::value;
        constexpr bool EDGE = decltype(ec)::value;
        using Q = Slots<P>;
        cx<T> x0 = in.x;
        if (PROLONG) x0 = cfma(mk((T)0.5, (T)0), in.e0 + in.e1, x0);
        ring_push<P>(rg[0], clip<EDGE>(x0, ln, t, n));
        bq[P % NB] = in.b;
#pragma unroll
        for (int s = 1; s <= S; ++s) {
            const int r = t - s;
            const Ring<T>& g = rg[s - 1];
            const cx<T> br = bq[qslot<NB>(P, s)];
            const cx<T> v = clip<EDGE>(
                cfma(ring_jf<EDGE>(ln, r, n), br - ring_apply<P, EDGE>(L, g, ln, r), g.v[Q::C]), ln,
                r, n);
            if (s < S) {
                ring_push<P>(rg[s], v);
            } else {
                if (own && r >= y0 && r < y1) {
                    const long long gi = (long long)r * np + ln.i;
                    if (UPDATE) xo[gi] = in.u + v;
                    else xo[gi] = v;
                }
                if (RESID) ring_push<P>(rg[S], v);
            }
        }
        if (RESID) {
            // residual of the final iterate, row t - S - 1
            const int r = t - S - 1;
            const cx<T> rv = bq[qslot<NB>(P, S + 1)] - ring_apply<P, EDGE>(L, rg[S], ln, r);
            ring_push<P>(rg[S + 1], clip<EDGE>(rv, ln, r, n));
            // restriction at the fine row t - S - 2 when it is even
            const int rr = t - S - 2;
            if (!(rr & 1) && rr >= y0 && rr < y1) {
                const cx<T> v = ring_restrict<P>(rg[S + 1]);
                if (own && !(ln.i & 1)) bc[(long long)(rr >> 1) * npc + (ln.i >> 1)] = v;
            }
        }
    };

    SweepIn<T, PROLONG, UPDATE> buf[3];
    load(buf[0], tb);
    load(buf[1], tb + 1);
    auto march = [&](auto ec) {
        auto block = [&](auto pc, int t) {
            constexpr int P = decltype(pc)::value;
            load(buf[(P + 2) % 3], t + P + 2);
            step(pc, ec, buf[P % 3], t + P);
        };
        for (int t = tb; t <= te; t += CHUNK) {
            block(Int<0>{}, t);
            block(Int<1>{}, t);
            block(Int<2>{}, t);
            if constexpr (CHUNK == 6) {
                block(Int<3>{}, t);
                block(Int<4>{}, t);
                block(Int<5>{}, t);
            }
        }
    };
    // a unit whose stencil rows (tb - DEPTH .. its last step) or columns
    // include a mesh boundary runs the boundary-aware code
    const int rlo = tb - DEPTH, rhi = tb + ((te - tb) / CHUNK + 1) * CHUNK - 1;
    if (ln.any_colb || (rlo <= 0 && 0 <= rhi) || (rlo <= n && n <= rhi)) march(Bool<true>{});
    else march(Bool<false>{});
}

// ---- k_stream_pre -----------------------------------------------------------
// The two pre-smoothing sweeps from a zero initial guess, x = t + omega D^{-1}
// (b - L t) with t = omega D^{-1} b, written; then b_c = P^T (b - L x).
// HSS = 0: b given.  HSS = 1: b = rho = c (R - B u), written.  HSS = 2: the
// first HSS step (u = 0): b = rho = c R, written.
template <typename T>
struct PreIn {
    cx<T> s, u;  // b or R, and u
};

template <typename T, int HSS>
__global__ __launch_bounds__(WAVE * SW) __attribute__((amdgpu_waves_per_eu(2))) void k_stream_pre(
    Op2<T> L, Op2<T> Bs, T c, Vec<const cx<T>> U, Vec<const cx<T>> Rv, Vec<cx<T>> Rho,
    Vec<const cx<T>> Bv, Vec<cx<T>> X, Vec<cx<T>> Bc, StreamGrid gr) {
    constexpr int DB = HSS == 1 ? 1 : 0;  // rows by which b lags the input
    constexpr int DEPTH = 3 + DB;
    constexpr int HALO = DEPTH;
    constexpr int OWN = WAVE - 2 * HALO;
    Unit un;
    if (!unit_of(gr, un)) return;
    const int n = L.n;
    const Lanes<T> ln = lanes_of(L, un.strip, OWN, HALO);
    const int lane = (int)(threadIdx.x % WAVE);
    const bool own = lane >= HALO && lane < HALO + OWN && ln.i <= n;
    const int y0 = un.seg * gr.H;
    const int y1 = min(y0 + gr.H, n + 1);
    const int jl = (y1 - 1) & ~1;
    const int tb = y0 - HALO;
    const int te = jl + 3 + DB;

    const cx<T>* src = HSS == 0 ? Bv.at(un.slot) : Rv.at(un.slot);
    const cx<T>* u = HSS == 1 ? U.at(un.slot) : nullptr;
    cx<T>* rho = HSS != 0 ? Rho.at(un.slot) : nullptr;
    cx<T>* x = X.at(un.slot);
    cx<T>* bc = Bc.at(un.slot);
    const long long np = n + 1, npc = n / 2 + 1;

    Ring<T> gu, g1, g2, gr3;
    ring_clear(gu);
    ring_clear(g1);
    ring_clear(g2);
    ring_clear(gr3);
    cx<T> rq[2];  // R rows: R(t) in slot P % 2, R(t - 1) in the other
    rq[0] = rq[1] = zero_cx<T>();
    cx<T> bq[3];  // b rows: b(rb - k) in slot (P - k) mod 3
#pragma unroll
    for (int k = 0; k < 3; ++k) bq[k] = zero_cx<T>();

    auto load = [&](PreIn<T>& in, int t) {
        in.s = load_raw(src, ln.ic, t, n);
        if (HSS == 1) in.u = load_raw(u, ln.ic, t, n);
    };

    auto step = [&](auto pc, auto ec, const PreIn<T>& in, int t) {
        constexpr int P = decltype(pc)::value;
        constexpr bool EDGE = decltype(ec)::value;
        using Q = Slots<P>;
        cx<T> bnew;
        int rb;  // row of bnew
        if (HSS == 1) {
            ring_push<P>(gu, clip<EDGE>(in.u, ln, t, n));
            rb = t - 1;
            bnew = c * (rq[(P + 1) % 2] - ring_apply<P, EDGE>(Bs, gu, ln, rb));
            rq[P % 2] = in.s;
        } else if (HSS == 2) {
            rb = t;
            bnew = c * in.s;
        } else {
            rb = t;
            bnew = in.s;
        }
        if (HSS != 0 && own && rb >= y0 && rb < y1) rho[(long long)rb * np + ln.i] = bnew;
        bq[P % 3] = bnew;
        // first sweep (pointwise): row rb
        ring_push<P>(g1, clip<EDGE>(ring_jf<EDGE>(ln, rb, n) * bnew, ln, rb, n));
        // second sweep: row rb - 1, written
        {
            const int r = rb - 1;
            const cx<T> v =
                cfma(ring_jf<EDGE>(ln, r, n), bq[qslot<3>(P, 1)] - ring_apply<P, EDGE>(L, g1, ln, r),
                     g1.v[Q::C]);
            if (own && r >= y0 && r < y1) x[(long long)r * np + ln.i] = v;
            ring_push<P>(g2, clip<EDGE>(v, ln, r, n));
        }
        // residual: row rb - 2
        {
            const int r = rb - 2;
            ring_push<P>(gr3, clip<EDGE>(bq[qslot<3>(P, 2)] - ring_apply<P, EDGE>(L, g2, ln, r), ln, r, n));
        }
        // restriction at the fine row rb - 3 when even
        {
            const int rr = rb - 3;
            if (!(rr & 1) && rr >= y0 && rr < y1) {
                const cx<T> v = ring_restrict<P>(gr3);
                if (own && !(ln.i & 1)) bc[(long long)(rr >> 1) * npc + (ln.i >> 1)] = v;
            }
        }
    };

    constexpr int CHUNK = HSS == 1 ? 6 : 3;  // a multiple of 3 and of the R queue's 2
    PreIn<T> buf[3];
    load(buf[0], tb);
    load(buf[1], tb + 1);
    auto march = [&](auto ec) {
        auto block = [&](auto pc, int t) {
            constexpr int P = decltype(pc)::value;
            load(buf[(P + 2) % 3], t + P + 2);
            step(pc, ec, buf[P % 3], t + P);
        };
        for (int t = tb; t <= te; t += CHUNK) {
            block(Int<0>{}, t);
            block(Int<1>{}, t);
            block(Int<2>{}, t);
            if constexpr (CHUNK == 6) {
                block(Int<3>{}, t);
                block(Int<4>{}, t);
                block(Int<5>{}, t);
            }
        }
    };
    // a unit whose stencil rows (tb - DEPTH .. its last step) or columns
    // include a mesh boundary runs the boundary-aware code
    const int rlo = tb - DEPTH, rhi = tb + ((te - tb) / CHUNK + 1) * CHUNK - 1;
    if (ln.any_colb || (rlo <= 0 && 0 <= rhi) || (rlo <= n && n <= rhi)) march(Bool<true>{});
    else march(Bool<false>{});
}

}  // namespace

StreamGrid stream_grid(int n, int halo, int ns, int H) {
    StreamGrid g;
    const int own = WAVE - 2 * halo;
    g.H = H;
    g.strips = (unsigned)((n + 1 + own - 1) / own);
    g.segs = (unsigned)((n + 1 + H - 1) / H);
    g.units = g.strips * g.segs * (unsigned)ns;
    return g;
}

// Segment height.  A segment of H rows costs about H + 2 halo + 1 steps of
// one wavefront; the kernel takes at least as long as one wavefront's chain
// of steps (about 1.2 us per step) and as long as all wavefronts' steps at
// the chip's throughput (about 1400 wavefront-steps per microsecond).  The
// height minimising the larger of the two is used.
static int stream_rows(int n, int halo, int ns) {
    int best = 64;
    double tbest = 1e30;
    for (int H = 4; H <= 128; H *= 2) {
        const StreamGrid g = stream_grid(n, halo, ns, H);
        const double steps = H + 2.0 * halo + 1.0;
        const double t = std::max(g.units * steps / 1400.0, steps * 1.2);
        if (t < tbest) {
            tbest = t;
            best = H;
        }
    }
    return best;
}

static unsigned stream_blocks(const StreamGrid& g) { return (g.units + SW - 1) / SW; }

template <typename T>
void stream_sweeps_2d(hipStream_t st, const Op2<T>& L, int S, Vec<const cx<T>> Xin,
                      Vec<const cx<T>> Ec, Vec<const cx<T>> B, Vec<cx<T>> Xout, Vec<cx<T>> Bc,
                      bool update, int ns) {
    const bool pro = Ec.base != nullptr, resid = Bc.base != nullptr;
    const int halo = S + (resid ? 2 : 0);
    const StreamGrid g = stream_grid(L.n, halo, ns, stream_rows(L.n, halo, ns));
    const unsigned nb = stream_blocks(g);
#define HELM_STREAM(SS, PP, RR, UU) \
    k_stream_sweeps<T, SS, PP, RR, UU><<<nb, WAVE * SW, 0, st>>>(L, Xin, Ec, B, Xout, Bc, g)
    if (S == 4 && pro && resid && !update) HELM_STREAM(4, true, true, false);
    else if (S == 2 && pro && !resid && update) HELM_STREAM(2, true, false, true);
    else if (S == 2 && pro && !resid && !update) HELM_STREAM(2, true, false, false);
    else if (S == 2 && !pro && resid && !update) HELM_STREAM(2, false, true, false);
    else if (S == 4 && pro && !resid && !update) HELM_STREAM(4, true, false, false);
    else if (S == 1 && !pro && !resid && !update) HELM_STREAM(1, false, false, false);
#undef HELM_STREAM
}

template <typename T>
void stream_pre_2d(hipStream_t st, const Op2<T>& L, const Op2<T>& Bs, T c, Vec<const cx<T>> U,
                   Vec<const cx<T>> R, Vec<cx<T>> Rho, Vec<const cx<T>> B, Vec<cx<T>> X,
                   Vec<cx<T>> Bc, int ns) {
    const int hss = B.base ? 0 : (U.base ? 1 : 2);
    const int halo = 3 + (hss == 1 ? 1 : 0);
    const StreamGrid g = stream_grid(L.n, halo, ns, stream_rows(L.n, halo, ns));
    const unsigned nb = stream_blocks(g);
    if (hss == 0)
        k_stream_pre<T, 0><<<nb, WAVE * SW, 0, st>>>(L, Bs, c, U, R, Rho, B, X, Bc, g);
    else if (hss == 1)
        k_stream_pre<T, 1><<<nb, WAVE * SW, 0, st>>>(L, Bs, c, U, R, Rho, B, X, Bc, g);
    else
        k_stream_pre<T, 2><<<nb, WAVE * SW, 0, st>>>(L, Bs, c, U, R, Rho, B, X, Bc, g);
}

template void stream_sweeps_2d<double>(hipStream_t, const Op2<double>&, int, Vec<const cxd>,
                                       Vec<const cxd>, Vec<const cxd>, Vec<cxd>, Vec<cxd>, bool, int);
template void stream_sweeps_2d<float>(hipStream_t, const Op2<float>&, int, Vec<const cxf>,
                                      Vec<const cxf>, Vec<const cxf>, Vec<cxf>, Vec<cxf>, bool, int);
template void stream_pre_2d<double>(hipStream_t, const Op2<double>&, const Op2<double>&, double,
                                    Vec<const cxd>, Vec<const cxd>, Vec<cxd>, Vec<const cxd>,
                                    Vec<cxd>, Vec<cxd>, int);
template void stream_pre_2d<float>(hipStream_t, const Op2<float>&, const Op2<float>&, float,
                                   Vec<const cxf>, Vec<const cxf>, Vec<cxf>, Vec<const cxf>,
                                   Vec<cxf>, Vec<cxf>, int);

}  // namespace helm
