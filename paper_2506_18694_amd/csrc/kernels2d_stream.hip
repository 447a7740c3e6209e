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
// Each stage loses one lane of validity on each side that borders another
// strip, so a middle strip computes 64 columns and owns the 64 - 2R in the
// middle (R = number of neighbour stages).  The first strip starts at column
// 0 and the last ends at column n in lane 63: there the lane shift fills the
// missing neighbour with zero, nothing is lost, and the strip owns up to the
// boundary.  A segment starts its march R rows below its first owned row.
//
// Values outside the mesh are zero where a stencil can see them: beyond the
// first and last column through the lane shift, below row 0 and above row n
// by clearing the stage outputs of those rows (only in the first and last
// blocks of steps of a segment that reaches them), and, when a single strip
// is wider than the mesh, in its lanes past column n.  The interior stencil
// plus the boundary corrections of the operator record (dC, dN, kA, kB) then
// gives the element rows of the edge and corner nodes.  Only owned nodes are
// written.  With Dirichlet faces (the DIR instantiations) every stage output,
// the HSS residual and the restricted values are also cleared on the nodes
// of those faces, which are not unknowns.
//
// The march runs in unrolled blocks of steps: within a block the three-row
// rings, the queue of right-hand-side rows and the input buffers rotate by
// renaming registers (the block length is a multiple of every period), and
// the input row t + 2 is loaded while step t computes.  A segment's step
// count is rounded up to whole blocks; the extra steps compute rows past
// the segment, which are never written.
//
// The rows next to a segment's ends run through code with the boundary
// handling compiled in, the others through code without it, and where
// those ends fall depends on the segment height, which is chosen by
// timing.  So that every node gets the same roundings whatever the
// height, nothing in this file lets the compiler fuse a product into a
// following sum on its own: every fused multiply-add is written out.
#pragma clang fp contract(off)
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
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
    int lo_own, hi_own;  // owned columns [lo_own, hi_own)
    cx<T> jf;       // omega / D in the interior rows: boundary column or not
    cx<T> odC, odE, odA, odB;  // settled factors: interior, boundary rows
};

// Strip geometry (see the top of the file): owned widths of the first and of
// the middle strips, both even so that every coarse column has one owner.
__host__ __device__ inline int strip_first(int halo) { return (WAVE - halo) & ~1; }
__host__ __device__ inline int strip_mid(int halo) { return (WAVE - 2 * halo) & ~1; }
__host__ __device__ inline int strip_count(int n, int halo) {
    if (n + 1 <= WAVE) return 1;
    // columns left after the first strip and a last strip of full width
    const int rest = n + 1 - strip_first(halo) - (WAVE - halo);
    return 2 + (rest > 0 ? (rest + strip_mid(halo) - 1) / strip_mid(halo) : 0);
}

template <typename T>
__device__ __forceinline__ Lanes<T> lanes_of(const Op2<T>& L, int strip, int strips, int halo) {
    const int n = L.n;
    Lanes<T> ln;
    int i0;
    if (strips == 1) {
        i0 = 0;
        ln.lo_own = 0;
        ln.hi_own = n + 1;
    } else if (strip == 0) {
        i0 = 0;
        ln.lo_own = 0;
        ln.hi_own = strip_first(halo);
    } else if (strip == strips - 1) {
        i0 = n - (WAVE - 1);
        ln.lo_own = strip_first(halo) + (strips - 2) * strip_mid(halo);
        ln.hi_own = n + 1;
    } else {
        ln.lo_own = strip_first(halo) + (strip - 1) * strip_mid(halo);
        ln.hi_own = ln.lo_own + strip_mid(halo);
        i0 = ln.lo_own - halo;
    }
    ln.i = i0 + (int)(threadIdx.x % WAVE);
    ln.ic = min(max(ln.i, 0), n);
    ln.inx = ln.i == ln.ic;
    ln.colb = ln.i == 0 || ln.i == n;
    ln.lo = ln.i == 0;
    ln.colbf = ln.colb ? (T)1 : (T)0;
    ln.any_colb = strips == 1 || strip == 0 || strip == strips - 1;
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

// What a wavefront's unit touches: boundary columns (0 or n among its
// lanes) and/or boundary rows (0 or n among its stencil rows).  A unit that
// touches a boundary holds zeros outside the mesh and adds the boundary
// corrections; an interior unit applies the interior stencil everywhere.
constexpr int TOUCH_COL = 1, TOUCH_ROW = 2, CLIP_LANES = 4;

// (Op v) at the centre row r of g (r uniform across the wave)
template <int P, int MODE, typename T>
__device__ __forceinline__ cx<T> ring_apply(const Op2<T>& op, const Ring<T>& g, const Lanes<T>& ln,
                                            int r) {
    using Q = Slots<P>;
    const cx<T> c = g.v[Q::C], nn = g.v[Q::N], ss = g.v[Q::O];
    const cx<T> ee = g.e[Q::C], ww = g.w[Q::C], ne = g.e[Q::N], sw = g.w[Q::O];
    cx<T> acc = cfma(op.wDg, ne + sw, cfma(op.wAx, (ee + ww) + (nn + ss), op.wC * c));
    if (MODE & TOUCH_COL) {
        // boundary column: the two neighbours along it and the centre
        acc = axpy_real(ln.colbf, cfma(op.dN, nn + ss, op.dC * c), acc);
    }
    if (MODE & TOUCH_ROW) {
        if (r == 0 || r == op.n) {
            keep_branch();
            // boundary row, and at its two corners the remaining centre term
            acc = acc + cfma(op.dN, ee + ww, op.dC * c);
            if (MODE & TOUCH_COL)
                acc = axpy_real(ln.colbf, sel(ln.lo == (r == 0), op.kA, op.kB) * c, acc);
        }
    }
    return acc;
}

// omega / D at row r
template <int MODE, typename T>
__device__ __forceinline__ cx<T> ring_jf(const Lanes<T>& ln, int r, int n) {
    if (MODE & TOUCH_ROW) {
        if (r == 0 || r == n) {
            keep_branch();
            return sel(ln.colb, sel(ln.lo == (r == 0), ln.odA, ln.odB), ln.odE);
        }
    }
    return (MODE & TOUCH_COL) ? ln.jf : ln.odC;
}

// P^T r at the fine node (2I, 2J) = centre row rr of g:
// r(2I, 2J) + (1/2) (sum over its six fine edge neighbours; those outside
// the mesh hold zero in a boundary unit)
template <int P, typename T>
__device__ __forceinline__ cx<T> ring_restrict(const Ring<T>& g) {
    using Q = Slots<P>;
    const cx<T> s6 = ((g.e[Q::C] + g.w[Q::C]) + (g.v[Q::N] + g.v[Q::O])) + (g.e[Q::N] + g.w[Q::O]);
    return axpy_real((T)0.5, s6, g.v[Q::C]);
}

// in a boundary unit: zero outside the mesh (row r uniform)
template <int MODE, typename T>
__device__ __forceinline__ cx<T> clip(cx<T> v, const Lanes<T>& ln, int r, int n) {
    if (MODE & CLIP_LANES) v = sel(ln.inx, v, zero_cx<T>());
    if (MODE & TOUCH_ROW) {
        if (r < 0 || r > n) {
            keep_branch();
            v = zero_cx<T>();
        }
    }
    return v;
}

// Dirichlet faces (DIR): zero on the nodes of the faces set in L.dir, for
// this lane's column and row r (uniform across the wave)
template <bool DIR, typename T>
__device__ __forceinline__ cx<T> dclip(cx<T> v, const Op2<T>& L, const Lanes<T>& ln, int r) {
    if constexpr (!DIR) {
        return v;
    } else {
        const unsigned d = L.dir;
        const bool f = ((d & 1u) && ln.i == 0) || ((d & 2u) && ln.i == L.n) || ((d & 4u) && r == 0) ||
                       ((d & 8u) && r == L.n);
        return sel(f, zero_cx<T>(), v);
    }
}

struct Unit {
    int slot, strip, seg;
};

// Units that touch the mesh boundary (first and last strip, first and last
// segment) run the slower boundary code; they are dispatched first, spread
// over all XCDs, so that they do not finish last.  The interior units follow,
// each XCD taking a contiguous range of them (neighbouring strips and
// segments share halo rows in one L2).
__device__ __forceinline__ bool unit_of(const StreamGrid& gr, Unit& u) {
    // the wavefront's index within the workgroup, made visibly uniform so
    // that the unit, the rows and every branch on them stay scalar
    const unsigned wid = (unsigned)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
    const unsigned S = gr.strips, G = gr.segs;
    const bool split = S > 2 && G > 2;
    const unsigned I = split ? (S - 2) * (G - 2) : 0;  // interior units per slot
    const unsigned E = S * G - I;                      // boundary units per slot
    if (blockIdx.x < gr.eblocks) {
        const unsigned id = blockIdx.x * SW + wid;
        if (id >= gr.edge_units) return false;
        u.slot = (int)(id / E);
        const unsigned e = id % E;
        if (!split) {
            u.seg = (int)(e / S);
            u.strip = (int)(e % S);
        } else if (e < 2 * S) {
            u.seg = e < S ? 0 : (int)G - 1;
            u.strip = (int)(e % S);
        } else {
            const unsigned k = e - 2 * S;
            u.seg = 1 + (int)(k / 2);
            u.strip = (k & 1) ? (int)S - 1 : 0;
        }
        return true;
    }
    const unsigned blk = xcd_remap(blockIdx.x - gr.eblocks, gridDim.x - gr.eblocks);
    const unsigned id = blk * SW + wid;
    if (id >= gr.units - gr.edge_units) return false;
    u.slot = (int)(id / I);
    const unsigned r = id % I;
    u.seg = 1 + (int)(r / (S - 2));
    u.strip = 1 + (int)(r % (S - 2));
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

template <typename T, int S, bool PROLONG, bool RESID, bool UPDATE, bool DIR>
__global__ __launch_bounds__(WAVE * SW) __attribute__((amdgpu_waves_per_eu(2))) void k_stream_sweeps(
    Op2<T> L, Vec<const cx<T>> Xin, Vec<const cx<T>> Ec, Vec<const cx<T>> Bv, Vec<cx<T>> Xout,
    Vec<cx<T>> Bc, StreamGrid gr) {
    constexpr int DEPTH = S + (RESID ? 2 : 0);  // lag of the deepest stage
    constexpr int HALO = DEPTH;
    constexpr int NR = S + (RESID ? 2 : 0);
    constexpr int NB = (S + (RESID ? 2 : 1) <= 3) ? 3 : 6;  // queue of b rows
    constexpr int NBUF = 3;    // input rows in flight
    constexpr int CHUNK = NB;  // steps per block: a multiple of 3, NB and NBUF
    Unit un;
    if (!unit_of(gr, un)) return;
    const int n = L.n;
    const Lanes<T> ln = lanes_of(L, un.strip, (int)gr.strips, HALO);
    const bool own = ln.i >= ln.lo_own && ln.i < ln.hi_own;
    [[maybe_unused]] const bool own_even = own & !(ln.i & 1);  // owned even column (coarse node)
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
        constexpr int MODE = decltype(ec)::value;
        using Q = Slots<P>;
        cx<T> x0 = in.x;
        if (PROLONG) x0 = axpy_real((T)0.5, in.e0 + in.e1, x0);
        ring_push<P>(rg[0], dclip<DIR>(clip<MODE>(x0, ln, t, n), L, ln, t));
        bq[P % NB] = in.b;
#pragma unroll
        for (int s = 1; s <= S; ++s) {
            const int r = t - s;
            const Ring<T>& g = rg[s - 1];
            const cx<T> br = bq[qslot<NB>(P, s)];
            const cx<T> v = dclip<DIR>(
                clip<MODE>(cfma(ring_jf<MODE>(ln, r, n), br - ring_apply<P, MODE>(L, g, ln, r), g.v[Q::C]),
                           ln, r, n),
                L, ln, r);
            if (s < S) {
                ring_push<P>(rg[s], v);
            } else {
                if (own & (r >= y0) & (r < y1)) xo[(long long)r * np + ln.i] = UPDATE ? in.u + v : v;
                if constexpr (RESID) ring_push<P>(rg[S], v);
            }
        }
        if constexpr (RESID) {
            // residual of the final iterate, row t - S - 1
            const int r = t - S - 1;
            const cx<T> rv = bq[qslot<NB>(P, S + 1)] - ring_apply<P, MODE>(L, rg[S], ln, r);
            ring_push<P>(rg[S + 1], dclip<DIR>(clip<MODE>(rv, ln, r, n), L, ln, r));
            // restriction at the fine row t - S - 2 when it is even (a coarse
            // node on a Dirichlet face sits on a fine one)
            const int rr = t - S - 2;
            if (!(rr & 1) & (rr >= y0) & (rr < y1)) {
                const cx<T> v = dclip<DIR>(ring_restrict<P>(rg[S + 1]), L, ln, rr);
                if (own_even) bc[(long long)(rr >> 1) * npc + (ln.i >> 1)] = v;
            }
        }
    };

    SweepIn<T, PROLONG, UPDATE> buf[NBUF];
#pragma unroll
    for (int k = 0; k < NBUF - 1; ++k) load(buf[k], tb + k);
    // blocks of CHUNK steps in mode MODE; the blocks whose stencil rows,
    // t - DEPTH .. t + CHUNK - 1, reach row 0 or row n run with the row mode
    // added, in loops of their own before and after the main loop
    auto march = [&](auto mc) {
        constexpr int MODE = decltype(mc)::value;
        auto chunk = [&](auto ec, int t) {
            auto block = [&](auto pc) {
                constexpr int P = decltype(pc)::value;
                load(buf[(P + NBUF - 1) % NBUF], t + P + NBUF - 1);
                step(pc, ec, buf[P % NBUF], t + P);
            };
            block(Int<0>{});
            block(Int<1>{});
            block(Int<2>{});
            if constexpr (CHUNK == 6) {
                block(Int<3>{});
                block(Int<4>{});
                block(Int<5>{});
            }
        };
        int t = tb;
        for (; t <= te && t - DEPTH <= 0; t += CHUNK) chunk(Int<MODE | TOUCH_ROW>{}, t);
        for (; t <= te && t + CHUNK - 1 < n; t += CHUNK) chunk(Int<MODE>{}, t);
        for (; t <= te; t += CHUNK) chunk(Int<MODE | TOUCH_ROW>{}, t);
    };
    // boundary columns are a property of the strip; boundary rows (and the
    // rows outside the mesh) only concern the first and last blocks of steps
    // of a segment that reaches them
    if (ln.any_colb) {
        if (n + 1 < WAVE) march(Int<TOUCH_COL | CLIP_LANES>{});
        else march(Int<TOUCH_COL>{});
    } else {
        march(Int<0>{});
    }
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

template <typename T, int HSS, bool DIR>
__global__ __launch_bounds__(WAVE * SW) __attribute__((amdgpu_waves_per_eu(2))) void k_stream_pre(
    Op2<T> L, Op2<T> Bs, T c, Vec<const cx<T>> U, Vec<const cx<T>> Rv, Vec<cx<T>> Rho,
    Vec<const cx<T>> Bv, Vec<cx<T>> X, Vec<cx<T>> Bc, StreamGrid gr) {
    constexpr int DB = HSS == 1 ? 1 : 0;  // rows by which b lags the input
    constexpr int DEPTH = 3 + DB;
    constexpr int HALO = DEPTH;
    Unit un;
    if (!unit_of(gr, un)) return;
    const int n = L.n;
    const Lanes<T> ln = lanes_of(L, un.strip, (int)gr.strips, HALO);
    const bool own = ln.i >= ln.lo_own && ln.i < ln.hi_own;
    [[maybe_unused]] const bool own_even = own & !(ln.i & 1);  // owned even column (coarse node)
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
        constexpr int MODE = decltype(ec)::value;
        using Q = Slots<P>;
        cx<T> bnew;
        int rb;  // row of bnew
        if (HSS == 1) {
            ring_push<P>(gu, clip<MODE>(in.u, ln, t, n));
            rb = t - 1;
            bnew = c * (rq[(P + 1) % 2] - ring_apply<P, MODE>(Bs, gu, ln, rb));
            rq[P % 2] = in.s;
        } else if (HSS == 2) {
            rb = t;
            bnew = c * in.s;
        } else {
            rb = t;
            bnew = in.s;
        }
        bnew = dclip<DIR>(bnew, L, ln, rb);
        if (HSS != 0 && (own & (rb >= y0) & (rb < y1))) rho[(long long)rb * np + ln.i] = bnew;
        bq[P % 3] = bnew;
        // first sweep (pointwise): row rb
        ring_push<P>(g1, clip<MODE>(ring_jf<MODE>(ln, rb, n) * bnew, ln, rb, n));
        // second sweep: row rb - 1, written
        {
            const int r = rb - 1;
            const cx<T> v = dclip<DIR>(
                cfma(ring_jf<MODE>(ln, r, n), bq[qslot<3>(P, 1)] - ring_apply<P, MODE>(L, g1, ln, r),
                     g1.v[Q::C]),
                L, ln, r);
            if (own & (r >= y0) & (r < y1)) x[(long long)r * np + ln.i] = v;
            ring_push<P>(g2, clip<MODE>(v, ln, r, n));
        }
        // residual: row rb - 2
        {
            const int r = rb - 2;
            ring_push<P>(gr3, dclip<DIR>(clip<MODE>(bq[qslot<3>(P, 2)] - ring_apply<P, MODE>(L, g2, ln, r), ln, r, n),
                                         L, ln, r));
        }
        // restriction at the fine row rb - 3 when even
        {
            const int rr = rb - 3;
            if (!(rr & 1) & (rr >= y0) & (rr < y1)) {
                const cx<T> v = dclip<DIR>(ring_restrict<P>(gr3), L, ln, rr);
                if (own_even) bc[(long long)(rr >> 1) * npc + (ln.i >> 1)] = v;
            }
        }
    };

    constexpr int NBUF = 3;                  // input rows in flight
    constexpr int CHUNK = HSS == 1 ? 6 : 3;  // a multiple of 3, NBUF and the R queue's 2
    PreIn<T> buf[NBUF];
#pragma unroll
    for (int k = 0; k < NBUF - 1; ++k) load(buf[k], tb + k);
    // blocks of CHUNK steps in mode MODE; the blocks whose stencil rows,
    // t - DEPTH .. t + CHUNK - 1, reach row 0 or row n run with the row mode
    // added, in loops of their own before and after the main loop
    auto march = [&](auto mc) {
        constexpr int MODE = decltype(mc)::value;
        auto chunk = [&](auto ec, int t) {
            auto block = [&](auto pc) {
                constexpr int P = decltype(pc)::value;
                load(buf[(P + NBUF - 1) % NBUF], t + P + NBUF - 1);
                step(pc, ec, buf[P % NBUF], t + P);
            };
            block(Int<0>{});
            block(Int<1>{});
            block(Int<2>{});
            if constexpr (CHUNK == 6) {
                block(Int<3>{});
                block(Int<4>{});
                block(Int<5>{});
            }
        };
        int t = tb;
        for (; t <= te && t - DEPTH <= 0; t += CHUNK) chunk(Int<MODE | TOUCH_ROW>{}, t);
        for (; t <= te && t + CHUNK - 1 < n; t += CHUNK) chunk(Int<MODE>{}, t);
        for (; t <= te; t += CHUNK) chunk(Int<MODE | TOUCH_ROW>{}, t);
    };
    // boundary columns are a property of the strip; boundary rows (and the
    // rows outside the mesh) only concern the first and last blocks of steps
    // of a segment that reaches them
    if (ln.any_colb) {
        if (n + 1 < WAVE) march(Int<TOUCH_COL | CLIP_LANES>{});
        else march(Int<TOUCH_COL>{});
    } else {
        march(Int<0>{});
    }
}

}  // namespace

StreamGrid stream_grid(int n, int halo, int ns, int H) {
    StreamGrid g;
    g.H = H;
    g.strips = (unsigned)strip_count(n, halo);
    g.segs = (unsigned)((n + 1 + H - 1) / H);
    g.units = g.strips * g.segs * (unsigned)ns;
    const unsigned I = (g.strips > 2 && g.segs > 2) ? (g.strips - 2) * (g.segs - 2) : 0;
    g.edge_units = (g.strips * g.segs - I) * (unsigned)ns;
    // boundary workgroups, rounded up to whole rounds over the 8 XCDs
    g.eblocks = (g.edge_units + SW - 1) / SW;
    g.eblocks = (g.eblocks + 7) / 8 * 8;
    return g;
}

// Segment height.  The kernel's time depends on the chain of steps of one
// wavefront (H + 2 halo + 1), on how the units fill the wavefront slots and
// on the slower boundary units; the best height is measured.  The first
// time a configuration (kernel, mesh size, slot count, precision) is launched
// on a stream that is not being captured, every candidate height is timed
// on the real operands (all the kernels timed this way recompute the same
// outputs from unchanged inputs) and the fastest is kept for the process.
// Until then, and under capture, a model picks the height: the larger of one
// wavefront's chain (about 1.2 us per step) and all wavefronts' steps at the
// chip's throughput (about 1400 wavefront-steps per microsecond).
static int stream_rows_model(int n, int halo, int ns) {
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

static unsigned stream_blocks(const StreamGrid& g) {
    return g.eblocks + (g.units - g.edge_units + SW - 1) / SW;
}

enum StreamKind : int { SK_S4R = 0, SK_S2P, SK_S2R, SK_S4P, SK_S1, SK_PRE0, SK_PRE1, SK_PRE2, SK_DIR = 16 };

struct RowsKey {
    int kind, n, ns, bytes;
    bool operator<(const RowsKey& o) const {
        return std::tie(kind, n, ns, bytes) < std::tie(o.kind, o.n, o.ns, o.bytes);
    }
};
static std::mutex g_rows_mu;
static std::map<RowsKey, int> g_rows;
// per-thread switch: when off, a height not measured yet comes from the model
// (no timing launches, no events created)
static thread_local bool g_rows_tuning = true;

bool stream_tuning(bool on) {
    const bool was = g_rows_tuning;
    g_rows_tuning = on;
    return was;
}

// Height for a launch of `kind`; `launch(H)` enqueues the kernel with height
// H.  tune = false: only look up (the kernel is not safe to repeat).
template <typename F>
static int stream_rows(hipStream_t st, RowsKey key, int halo, bool tune, F launch) {
    {
        std::lock_guard<std::mutex> lk(g_rows_mu);
        auto it = g_rows.find(key);
        if (it != g_rows.end()) return it->second;
    }
    const int model = stream_rows_model(key.n, halo, key.ns);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (!tune || !g_rows_tuning || hipStreamIsCapturing(st, &cs) != hipSuccess ||
        cs != hipStreamCaptureStatusNone)
        return model;
    static const int cand[] = {2, 3, 4, 6, 8, 12, 16, 20, 24, 28, 32, 36, 40, 42, 48, 56, 64, 96, 128};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return model;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return model;
    }
    int best = model;
    float tbest = 1e30f;
    for (int H : cand) {
        if (H > key.n + 1 && H != 4) break;
        launch(H);  // warm
        (void)hipEventRecord(e0, st);
        launch(H);
        launch(H);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms < tbest) {
            tbest = ms;
            best = H;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_rows_mu);
    g_rows[key] = best;
    return best;
}

template <typename T>
bool stream_sweeps_2d(hipStream_t st, const Op2<T>& L, int S, Vec<const cx<T>> Xin,
                      Vec<const cx<T>> Ec, Vec<const cx<T>> B, Vec<cx<T>> Xout, Vec<cx<T>> Bc,
                      bool update, int ns) {
    const bool pro = Ec.base != nullptr, resid = Bc.base != nullptr;
    const int halo = S + (resid ? 2 : 0);
    int kind = -1;
    if (S == 4 && pro && resid && !update) kind = SK_S4R;
    else if (S == 2 && pro && !resid) kind = SK_S2P;  // the update variant shares its height
    else if (S == 2 && !pro && resid && !update) kind = SK_S2R;
    else if (S == 4 && pro && !resid && !update) kind = SK_S4P;
    else if (S == 1 && !pro && !resid && !update) kind = SK_S1;
    if (kind < 0) return false;
    const bool dir = L.dir != 0u;
    auto launch = [&](int H) {
        const StreamGrid g = stream_grid(L.n, halo, ns, H);
        const unsigned nb = stream_blocks(g);
#define HELM_STREAM(SS, PP, RR, UU)                                                                      \
    do {                                                                                                 \
        if (dir) k_stream_sweeps<T, SS, PP, RR, UU, true><<<nb, WAVE * SW, 0, st>>>(L, Xin, Ec, B, Xout, Bc, g); \
        else k_stream_sweeps<T, SS, PP, RR, UU, false><<<nb, WAVE * SW, 0, st>>>(L, Xin, Ec, B, Xout, Bc, g); \
    } while (0)
        if (kind == SK_S4R) HELM_STREAM(4, true, true, false);
        else if (kind == SK_S2P && update) HELM_STREAM(2, true, false, true);
        else if (kind == SK_S2P) HELM_STREAM(2, true, false, false);
        else if (kind == SK_S2R) HELM_STREAM(2, false, true, false);
        else if (kind == SK_S4P) HELM_STREAM(4, true, false, false);
        else HELM_STREAM(1, false, false, false);
#undef HELM_STREAM
    };
    // u += x is not safe to repeat: the update launch only looks up
    launch(stream_rows(st, RowsKey{kind + (dir ? SK_DIR : 0), L.n, ns, (int)sizeof(T)}, halo, !update, launch));
    return true;
}

template <typename T>
void stream_pre_2d(hipStream_t st, const Op2<T>& L, const Op2<T>& Bs, T c, Vec<const cx<T>> U,
                   Vec<const cx<T>> R, Vec<cx<T>> Rho, Vec<const cx<T>> B, Vec<cx<T>> X,
                   Vec<cx<T>> Bc, int ns) {
    const int hss = B.base ? 0 : (U.base ? 1 : 2);
    const int halo = 3 + (hss == 1 ? 1 : 0);
    const bool dir = L.dir != 0u;
    auto launch = [&](int H) {
        const StreamGrid g = stream_grid(L.n, halo, ns, H);
        const unsigned nb = stream_blocks(g);
#define HELM_PRE(HH)                                                                          \
    do {                                                                                      \
        if (dir) k_stream_pre<T, HH, true><<<nb, WAVE * SW, 0, st>>>(L, Bs, c, U, R, Rho, B, X, Bc, g); \
        else k_stream_pre<T, HH, false><<<nb, WAVE * SW, 0, st>>>(L, Bs, c, U, R, Rho, B, X, Bc, g); \
    } while (0)
        if (hss == 0) HELM_PRE(0);
        else if (hss == 1) HELM_PRE(1);
        else HELM_PRE(2);
#undef HELM_PRE
    };
    launch(stream_rows(st, RowsKey{SK_PRE0 + hss + (dir ? SK_DIR : 0), L.n, ns, (int)sizeof(T)}, halo, true,
                       launch));
}

template bool stream_sweeps_2d<double>(hipStream_t, const Op2<double>&, int, Vec<const cxd>,
                                       Vec<const cxd>, Vec<const cxd>, Vec<cxd>, Vec<cxd>, bool, int);
template bool stream_sweeps_2d<float>(hipStream_t, const Op2<float>&, int, Vec<const cxf>,
                                      Vec<const cxf>, Vec<const cxf>, Vec<cxf>, Vec<cxf>, bool, int);
template void stream_pre_2d<double>(hipStream_t, const Op2<double>&, const Op2<double>&, double,
                                    Vec<const cxd>, Vec<const cxd>, Vec<cxd>, Vec<const cxd>,
                                    Vec<cxd>, Vec<cxd>, int);
template void stream_pre_2d<float>(hipStream_t, const Op2<float>&, const Op2<float>&, float,
                                   Vec<const cxf>, Vec<const cxf>, Vec<cxf>, Vec<const cxf>,
                                   Vec<cxf>, Vec<cxf>, int);

}  // namespace helm
