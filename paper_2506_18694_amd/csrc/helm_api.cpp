// libhelm: host driver and C ABI (include/helm.h).
//
// The solve is right-preconditioned flexible GMRES on B_0 in complex FP64
// (Saad's FGMRES; the paper's outer Krylov method, Sec. 5.1) with classical
// Gram-Schmidt applied twice for the Arnoldi step and Givens rotations on
// the host.  The preconditioner is the shifted-HSS iteration of Sec. 4
// (Definition "Shifted HSS iteration for the primal system") in correction
// form
//     u_{s+1} = u_s + V( (2k/(k+1)) (R - B_dh u_s) ),   u_0 = 0,
// s = 0 .. m ceil(k) - 1, where V is q V(2,2) cycles (each after the first
// starting from the previous result) for
//     L = K + (dh^2 - k^2 - 2i dh k^2) M + (dh - i k^2) M_Gamma
// (the left-hand side of eq. (HSSpc primal)); with exact inner solves this
// equals the literal two-term form of the definition.  The cycle uses
// omega-scaled Jacobi (D = diag L), FE interpolation P and P^T between
// nested meshes (n_l = n / 2^l), and a dense FP64 inverse of L on the
// coarsest mesh.  In HELM_FP32_MG mode the HSS iterate, the cycle and its
// smoothers run in complex FP32; the preconditioned directions are stored
// in FP32 and promoted exactly when FGMRES uses them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/helm.h"
#include "faces.h"
#include "launch.h"
#include "stencil_rows.h"

using namespace helm;
using zd = std::complex<double>;

namespace {

thread_local std::string g_last_error;

struct DevErr {
    hipError_t e;
};

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) {                                                        \
            g_last_error = std::string(#expr) + ": " + hipGetErrorString(_e);          \
            throw DevErr{_e};                                                          \
        }                                                                              \
    } while (0)

// a streaming pass this build has no kernel for is an internal error
#define STREAMCHK(expr)                                                                \
    do {                                                                               \
        if (!(expr)) {                                                                 \
            g_last_error = std::string("unsupported streaming pass: ") + #expr;        \
            throw DevErr{hipErrorInvalidValue};                                        \
        }                                                                              \
    } while (0)

struct Coef {
    zd a, b, c;  // operator = a K + b M + c M_Gamma
};

// (a, b, c) of the named operators (HELM_OP_*).  B_delta from the primal
// form of Sec. 2: (-delta + ik)^2 M - (-delta + ik) M_Gamma; L and N from
// eq. (HSSpc primal); H from the H_primal inner product of Sec. 3.1.
Coef op_coef(int op, double k, double delta, double dh) {
    const zd I(0.0, 1.0);
    auto bdelta = [&](double d) {
        zd s = -d + I * k;
        return Coef{1.0, s * s, -s};
    };
    switch (op) {
        case HELM_OP_B0: return bdelta(0.0);
        case HELM_OP_BDELTA: return bdelta(delta);
        case HELM_OP_BSHIFT: return bdelta(dh);
        case HELM_OP_L: return Coef{1.0, dh * dh - k * k - 2.0 * I * dh * k * k, dh - I * k * k};
        case HELM_OP_N: return Coef{-1.0, k * k - dh * dh - 2.0 * I * dh * k * k, -dh - I * k * k};
        case HELM_OP_H: return Coef{0.0, 2.0 * dh * k, k};
        case HELM_OP_M: return Coef{0.0, 1.0, 0.0};
    }
    return Coef{0.0, 0.0, 0.0};
}

template <typename T>
cx<T> tocx(zd z) { return mk((T)z.real(), (T)z.imag()); }

template <typename T>
Op2<T> make_op2(const Coef& cf, int n, double omega, unsigned dir = 0) {
    const double h = 1.0 / n;
    const zd A = cf.a, Bm = cf.b * (h * h / 24.0), Cg = cf.c * (h / 6.0);
    const zd wC = 4.0 * A + 12.0 * Bm, wAx = -A + 2.0 * Bm, wDg = 2.0 * Bm;
    Op2<T> o;
    o.dir = dir;
    o.A = tocx<T>(A);
    o.Bm = tocx<T>(Bm);
    o.Cg = tocx<T>(Cg);
    o.wC = tocx<T>(wC);
    o.wAx = tocx<T>(wAx);
    o.wDg = tocx<T>(wDg);
    o.odC = tocx<T>(omega / wC);
    // edge, corner (0,0)/(n,n) and corner (n,0)/(0,n) diagonals (see Op2)
    o.odE = tocx<T>(omega / (2.0 * A + 6.0 * Bm + 4.0 * Cg));
    o.odA = tocx<T>(omega / (A + 4.0 * Bm + 4.0 * Cg));
    o.odB = tocx<T>(omega / (A + 2.0 * Bm + 4.0 * Cg));
    // boundary corrections of the interior stencil (zero values outside):
    // edge centre and along-edge weights minus the interior ones, and the
    // corners' remaining centre terms
    o.dC = tocx<T>(-2.0 * A - 6.0 * Bm + 4.0 * Cg);
    o.dN = tocx<T>(0.5 * A - Bm + Cg);
    o.kA = tocx<T>(A + 4.0 * Bm - 4.0 * Cg);
    o.kB = tocx<T>(A + 2.0 * Bm - 4.0 * Cg);
    o.omega = (T)omega;
    o.n = n;
    return o;
}

template <typename T>
Op3<T> make_op3(const Coef& cf, int n, double omega) {
    const double h = 1.0 / n;
    Op3<T> o;
    o.a = tocx<T>(cf.a);
    o.b = tocx<T>(cf.b);
    o.c = tocx<T>(cf.c);
    o.h = (T)h;
    o.omega = (T)omega;
    o.n = n;
    // interior weights by neighbour class (number of nonzero offsets)
    Op3<double> od;
    od.a = tocx<double>(cf.a);
    od.b = tocx<double>(cf.b);
    od.c = tocx<double>(cf.c);
    od.h = h;
    od.n = n;
    Line3<double> f = line_factors<double>(1, 2, h);
    for (int cls = 0; cls < 4; ++cls) {
        int dx = cls >= 1 ? 1 : 0, dy = cls >= 2 ? 1 : 0, dz = cls >= 3 ? 1 : 0;
        cxd w = weight3(od, f, f, f, dx, dy, dz);
        o.wInt[cls] = mk((T)w.x, (T)w.y);
    }
    cxd wc = weight3(od, f, f, f, 0, 0, 0);
    zd dC(wc.x, wc.y);
    o.odC = tocx<T>(omega / dC);
    return o;
}

// Operator record of the fused 3D passes (kernels3d_fused.hip): the
// coefficients of the per-plane terms T1, T0 built from the 1D element rows
// K1 = (1/h)[-1 2 -1], M1 = (h/6)[1 4 1] (boundary rows halve the centre)
// and the Jacobi factors omega / D by the number of boundary coordinates.
template <typename T>
Op3F<T> make_op3f(const Coef& cf, int n, double omega, unsigned dir = 0) {
    const double h = 1.0 / n, h6 = h / 6.0, ih = 1.0 / h;
    const zd a = cf.a, b = cf.b, c = cf.c;
    // T1 = uK PK + uM PMM + uG PG and T0 = vK PK + vM PMM + vG PG
    const zd uK = h6 * a, uM = h6 * b - a * ih, uG = h6 * c;
    const zd vK = 4.0 * h6 * a, vM = 4.0 * h6 * b + 2.0 * a * ih, vG = 4.0 * h6 * c;
    Op3F<T> o;
    o.dir = dir;
    // interior columns: PK = (16 a0 - 2 (H + V) - 2 a2) / 6 and
    // PMM = (h/6)^2 (16 a0 + 4 (H + V) + a2), PG = 0
    const double pk[3] = {16.0 / 6.0, -2.0 / 6.0, -2.0 / 6.0};
    const double pm[3] = {16.0 * h6 * h6, 4.0 * h6 * h6, h6 * h6};
    for (int q = 0; q < 3; ++q) {
        const zd t1 = uK * pk[q] + uM * pm[q];
        const zd t0 = vK * pk[q] + vM * pm[q];
        const zd tj = -0.5 * t0 + c * pm[q];
        o.i1[q] = tocx<T>(t1);
        o.i0[q] = tocx<T>(t0);
        o.j0[q] = tocx<T>(tj);  // end plane: T0 / 2 + c PMM
        o.r1[q] = (T)t1.real();
        o.r0[q] = (T)t0.real();
        o.rj[q] = (T)tj.real();
    }
    // every operator of the primal form has a real stiffness factor a (1, -1
    // or 0), so the imaginary parts are those of the PMM terms:
    // Im(t)[q] = k (h/6)^2 (16, 4, 1)[q]
    o.k1 = (T)(uM.imag() * h6 * h6);
    o.k0 = (T)(vM.imag() * h6 * h6);
    o.kj = (T)((-0.5 * vM.imag() + c.imag()) * h6 * h6);
    // a column on bx + by boundary lines (bx, by in {0, 1}) halves the centre
    // of the 1D factors in those directions and adds E = 1:
    //   PMM += (-8 h6^2 nb + 4 h6^2 bx by) a0 - 2 h6^2 w
    //   PK  += (-8/6 nb + 4/6 bx by) a0 + w / 6
    //   PG  += (4 h6 nb - 4 h6 bx by) a0 + h6 w
    // with nb = bx + by and w = bx V + by H; so each of T1, T0 changes by
    // (A nb + C bx by) a0 + B w with (A, B, C) below, and the end-plane
    // difference (c PMM - T0 / 2) by c times the PMM change minus half of T0's
    const double dm[3] = {-8.0 * h6 * h6, -2.0 * h6 * h6, 4.0 * h6 * h6};
    const double dk[3] = {-8.0 / 6.0, 1.0 / 6.0, 4.0 / 6.0};
    const double dg[3] = {4.0 * h6, h6, -4.0 * h6};
    for (int q = 0; q < 3; ++q) {
        const zd d1 = uK * dk[q] + uM * dm[q] + uG * dg[q];
        const zd d0 = vK * dk[q] + vM * dm[q] + vG * dg[q];
        o.e1[q] = tocx<T>(d1);
        o.e0[q] = tocx<T>(d0);
        o.f0[q] = tocx<T>(-0.5 * d0 + c * dm[q]);
    }
    // diagonal with nb coordinates on the boundary (factors halved there, E = 1)
    for (int nb = 0; nb < 4; ++nb) {
        double m[3], k[3], e[3];
        for (int ax = 0; ax < 3; ++ax) {
            const bool bnd = ax < nb;
            m[ax] = bnd ? 2.0 * h6 : 4.0 * h6;
            k[ax] = bnd ? ih : 2.0 * ih;
            e[ax] = bnd ? 1.0 : 0.0;
        }
        const zd D = a * (k[0] * m[1] * m[2] + m[0] * k[1] * m[2] + m[0] * m[1] * k[2]) +
                     b * (m[0] * m[1] * m[2]) +
                     c * (e[0] * m[1] * m[2] + m[0] * e[1] * m[2] + m[0] * m[1] * e[2]);
        o.od[nb] = tocx<T>(omega / D);
    }
    o.n = n;
    return o;
}

// In-place inverse of a dense complex matrix by Gauss-Jordan elimination
// with partial pivoting.  Returns false if singular.
bool invert_dense(std::vector<zd>& A, int n) {
    std::vector<zd> inv((size_t)n * n, zd(0.0));
    for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = std::abs(A[(size_t)col * n + col]);
        for (int r = col + 1; r < n; ++r) {
            double v = std::abs(A[(size_t)r * n + col]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return false;
        if (piv != col) {
            for (int c = 0; c < n; ++c) {
                std::swap(A[(size_t)piv * n + c], A[(size_t)col * n + c]);
                std::swap(inv[(size_t)piv * n + c], inv[(size_t)col * n + c]);
            }
        }
        const zd d = 1.0 / A[(size_t)col * n + col];
        for (int c = 0; c < n; ++c) {
            A[(size_t)col * n + c] *= d;
            inv[(size_t)col * n + c] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const zd f = A[(size_t)r * n + col];
            if (f == 0.0) continue;
            for (int c = 0; c < n; ++c) {
                A[(size_t)r * n + c] -= f * A[(size_t)col * n + c];
                inv[(size_t)r * n + c] -= f * inv[(size_t)col * n + c];
            }
        }
    }
    A.swap(inv);
    return true;
}

}  // namespace

// ------------------------------------------------------------------ handle --
struct helm_s {
    int dim = 2, elem = HELM_P1_TRI_RIGHT, n = 0, levels = 1;
    double k = 0, delta = 0, dh = 0;
    helm_opts opts{};
    hipStream_t stream = nullptr;
    int device = 0;
    int hss_steps = 0, restart = 0, max_outer = 0;
    std::vector<int> nl;
    std::vector<long long> Nl;
    cxd* d_cinv = nullptr;  // coarsest-mesh inverse of L, FP64
    int nc = 0;             // coarsest-mesh node count
    int prec = HELM_FP64;
    double omega = 2.0 / 3.0;
    int cycles = 2;           // V-cycles per inner HSS solve
    int smooth_its = 5;       // GMRES iterations per smoothing (W variant)
    bool cycles_auto = true;  // choose `cycles` from the measured cycle rate
    double vrate = 0.0;       // measured V-cycle contraction (0 = not yet)

    // captured HIP graphs of the preconditioner's HSS loop, per workspace,
    // slot count, precision and cycle count; captured on cap_stream
    // the loop is captured as a head graph (step 0 and the remainder steps)
    // and a body graph of `block` steps replayed `reps` times, so that no
    // graph holds more than ~20000 launches
    // (keyed by the workspace address and the column count its layout was
    // made for: a new workspace of another size can reuse an old address)
    struct GraphEntry {
        void* ws;
        int cap, s0, ns, tag, cycles;
        hipGraphExec_t head, body;
        int reps;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;
    // second stream (and fork/join events) for the second group of slots
    hipStream_t aux_stream = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;

    // optional HIP-event timing of the finest-level smoothing passes of
    // every PROF_EVERY-th HSS step (an event record on each side of a launch
    // costs a few microseconds of queue time, so only a sample is timed)
    static constexpr int PROF_EVERY = 10;
    bool prof_on = false;
    bool prof_step = true;  // the current 3D HSS step is a timed one
    std::vector<hipEvent_t> prof_ev;
    size_t prof_used = 0;
    double prof_ms = 0.0, prof_bytes = 0.0, prof_pending_bytes = 0.0;
    long long prof_launches = 0;

    // mixed [DG0]^2 x P1 formulation (2D): the HSS inner operator becomes
    // K + k^2 (dh - i)^2 M + k^2 (dh - i) M_Gamma (sigma eliminated)
    bool mixed = false;
    long long nv = 0;  // unknowns per column: N, or N + 4 n^2 (mixed)

    // Dirichlet faces (u = 0; bit f: x0 x1 y0 y1 z0 z1).  Their nodes are
    // not unknowns: every vector the library produces is zero there, and
    // the operators' rows on the other nodes are those of the Sommerfeld
    // operator (whose couplings to the face nodes meet zeros).  The 3D
    // z-marching passes and the 2D streaming kernels clear the face nodes
    // of every stage output themselves; the other paths (2D levels below
    // the streaming ones, fused kernels switched off) run one pass per
    // launch with the faces cleared after every pass.
    unsigned dir = 0;

    Coef coef(int op) const {
        if (mixed && op == HELM_OP_L) {
            const zd s(dh, -1.0);
            return Coef{1.0, k * k * s * s, k * k * s};
        }
        return op_coef(op, k, delta, dh);
    }

    void prof_mark() {
        if (prof_used == prof_ev.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            prof_ev.push_back(e);
        }
        (void)hipEventRecord(prof_ev[prof_used++], stream);
    }
    // called after the streams have been synchronised
    void prof_collect() {
        for (size_t q = 0; q + 1 < prof_used; q += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, prof_ev[q], prof_ev[q + 1]) != hipSuccess) continue;
            prof_ms += ms;
            ++prof_launches;
        }
        prof_bytes += prof_pending_bytes;
        prof_pending_bytes = 0.0;
        prof_used = 0;
    }
};

namespace {

constexpr size_t ALIGN = 256;
inline size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Device workspace for up to `nrhs` columns.  Per column c: the load
// vector B[c] and iterate X[c] (FP64), the Krylov basis V[c][0..R] (FP64)
// and the preconditioned directions Z[c][0..R-1] (the preconditioner's
// storage precision); per slot: the multigrid level vectors and the HSS
// buffers R and u; plus small reduction and index arrays.
constexpr int NMAPS = 8;
struct Layout {
    size_t mg_b[32], mg_x[32], mg_t[32];
    size_t R, u;
    size_t V, Z, Bw, Xw;
    size_t dh, dh2, dnorm, part, npart, dy, cols, maps, flag;
    // W variant: per level the GMRES smoother's Krylov basis (m+1 vectors
    // per slot), its Hessenberg columns (two passes), norms, coefficients
    // and reduction partials
    size_t gk[32], ghu, ghu2, gn, gy, gpart, gnpart;
    size_t mg;  // mixed: the per-step triangle data g of every slot
    size_t total;
    int cap;    // columns the layout was made for (its offsets depend on it)
};

Layout layout(const helm_t* h, int nrhs) {
    Layout L{};
    L.cap = nrhs;
    size_t off = 0;
    const size_t smg = h->prec == HELM_FP64 ? sizeof(cxd) : sizeof(cxf);
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += up(bytes);
        return o;
    };
    const int R = h->restart;
    const long long N = h->Nl[0];
    // reductions run over whole columns (h->nv values: the mixed element's
    // triangle data included), so their partials are sized for that length
    const int nblk = multidot_blocks(h->nv);
    L.cols = take(sizeof(int) * nrhs);
    L.maps = take(sizeof(int) * NMAPS * nrhs);
    L.flag = take(sizeof(int) * nrhs);
    L.dh = take(sizeof(cxd) * nrhs * (R + 1));
    L.dh2 = take(sizeof(cxd) * nrhs * (R + 1));
    L.dnorm = take(sizeof(double) * 3 * nrhs);
    L.dy = take(sizeof(cxd) * nrhs * R);
    L.part = take(sizeof(cxd) * (size_t)nrhs * (R + 1) * nblk);
    L.npart = take(sizeof(double) * (size_t)nrhs * nblk);
    for (int l = 0; l < h->levels; ++l) {
        L.mg_b[l] = take(smg * nrhs * h->Nl[l]);
        L.mg_x[l] = take(smg * nrhs * h->Nl[l]);
        L.mg_t[l] = take(smg * nrhs * h->Nl[l]);
    }
    // column vectors: N unknowns, or N + 4 n^2 for the mixed formulation
    const long long Nv = h->nv;
    L.R = take(smg * nrhs * Nv);
    L.u = take(smg * nrhs * Nv);
    L.V = take(sizeof(cxd) * (size_t)nrhs * (R + 1) * Nv);
    L.Z = take(smg * (size_t)nrhs * R * Nv);
    L.Bw = take(sizeof(cxd) * (size_t)nrhs * Nv);
    L.Xw = take(sizeof(cxd) * (size_t)nrhs * Nv);
    L.mg = h->mixed ? take(sizeof(cxd) * (size_t)nrhs * (Nv - N)) : 0;
    if (h->opts.cycle == HELM_CYCLE_W_GMRES) {
        const int m = h->smooth_its;
        for (int l = 0; l < h->levels; ++l) L.gk[l] = take(sizeof(cxd) * (size_t)nrhs * (m + 1) * h->Nl[l]);
        L.ghu = take(sizeof(cxd) * (size_t)nrhs * m * (m + 1));
        L.ghu2 = take(sizeof(cxd) * (size_t)nrhs * (m + 1));
        L.gn = take(sizeof(double) * (size_t)nrhs * (m + 1));
        L.gy = take(sizeof(cxd) * (size_t)nrhs * m);
        L.gpart = take(sizeof(cxd) * (size_t)nrhs * (m + 1) * nblk);
        L.gnpart = take(sizeof(double) * (size_t)nrhs * nblk);
    }
    L.total = off;
    return L;
}

template <typename V>
Vec<V> at_ws(void* ws, size_t off, long long cstride) {
    return Vec<V>{reinterpret_cast<V*>(static_cast<char*>(ws) + off), cstride, 0, nullptr};
}

template <typename V>
Vec<const V> cst(Vec<V> v) {
    return Vec<const V>{v.base, v.cstride, v.off, v.cols};
}

// 3D levels run the fused z-marching passes (kernels3d_fused.hip) unless
// switched off (no_stream: one thread per node and the column-tile kernel)
inline bool fused3d(const helm_t* h) { return h->dim == 3 && !h->opts.no_stream; }

// Clear the Dirichlet faces of level l in Y (no launch without Dirichlet faces).
template <typename T>
void dir_mask(const helm_t* h, hipStream_t st, int l, Vec<cx<T>> Y, int ns) {
    if (h->dir) mask_faces<T>(st, h->dim, h->nl[l], h->dir, Y, ns);
}

// Op x (MODE_APPLY), s (b - Op x) (MODE_RESID), a Jacobi sweep (MODE_JACOBI)
// or the zero-guess sweep (MODE_JACOBI0) on 3D level l, for operator cf
template <typename T, typename TI>
void op3d(helm_t* h, hipStream_t st, const Coef& cf, int l, int mode, T s, Vec<const cx<TI>> X,
          Vec<const cx<T>> B, Vec<cx<T>> Y, int ns) {
    if (fused3d(h) && (mode == MODE_APPLY || mode == MODE_RESID || mode == MODE_JACOBI ||
                       mode == MODE_JACOBI0)) {
        const Op3F<T> o = make_op3f<T>(cf, h->nl[l], h->omega, h->dir);
        const int first = mode == MODE_APPLY ? F_APPLY
                          : mode == MODE_RESID ? F_RESID
                          : mode == MODE_JACOBI ? F_JAC
                                                : F_PRE0;
        STREAMCHK((pass3d<T, TI>(st, o, o, first, 1, false, 0, s, X, B, Vec<const cx<T>>{},
                                 Vec<cx<T>>{}, Y, ns)));
        return;
    }
    stencil3d<T, TI>(st, make_op3<T>(cf, h->nl[l], h->omega), mode, s, X, B, Y, ns, !h->opts.no_stream);
}

// ---------------------------------------------------------------- levels --
template <typename T>
void apply_mode(helm_t* h, int op, int l, int mode, T s, Vec<const cx<T>> X, Vec<const cx<T>> B,
                Vec<cx<T>> Y, int ns) {
    const Coef cf = h->coef(op);
    if (h->dim == 2) {
        stencil2d<T, T>(h->stream, make_op2<T>(cf, h->nl[l], h->omega), mode, s, X, B, Y, ns);
    } else {
        op3d<T, T>(h, h->stream, cf, l, mode, s, X, B, Y, ns);
    }
    dir_mask<T>(h, h->stream, l, Y, ns);
}

template <typename T>
void resid_restrict(helm_t* h, int l, Vec<const cx<T>> X, Vec<const cx<T>> B, Vec<cx<T>> Bc,
                    Vec<cx<T>> tmp, int ns) {
    const Coef cf = h->coef(HELM_OP_L);
    if (fused3d(h)) {
        // Dirichlet faces are cleared inside the pass
        rr3d<T>(h->stream, make_op3f<T>(cf, h->nl[l], h->omega, h->dir), X, B, Bc, ns);
    } else if (h->dir) {
        // the residual on the face nodes is not part of the system: cleared
        // before it is restricted, and the coarse face nodes after
        apply_mode<T>(h, HELM_OP_L, l, MODE_RESID, (T)1, X, B, tmp, ns);
        if (h->dim == 2) restrict2d<T>(h->stream, h->nl[l], cst(tmp), Bc, ns);
        else restrict3d<T>(h->stream, h->nl[l], cst(tmp), Bc, ns);
        dir_mask<T>(h, h->stream, l + 1, Bc, ns);
    } else if (h->dim == 2) {
        resid_restrict2d<T>(h->stream, make_op2<T>(cf, h->nl[l], h->omega), X, B, Bc, ns);
    } else {
        stencil3d<T, T>(h->stream, make_op3<T>(cf, h->nl[l], h->omega), MODE_RESID, (T)1, X, B,
                        tmp, ns, !h->opts.no_stream);
        restrict3d<T>(h->stream, h->nl[l], cst(tmp), Bc, ns);
    }
}

template <typename T>
void prolong(helm_t* h, int l, Vec<const cx<T>> E, Vec<cx<T>> X, int ns) {
    if (h->dim == 2) prolong2d<T>(h->stream, h->nl[l], E, X, ns);
    else prolong3d<T>(h->stream, h->nl[l], E, X, ns);
    dir_mask<T>(h, h->stream, l, X, ns);
}

// One V(2,2) cycle on level l for L x = b, starting from x = 0 or (guess)
// from the x passed in; the result is left in x.  Level buffers b, x, t of
// levels > l come from ws.  Starting from x0 gives x0 + V(b - L x0).
template <typename T>
void vcycle(helm_t* h, const Layout& Lw, void* ws, int l, Vec<const cx<T>> b, Vec<cx<T>> x,
            Vec<cx<T>> t, int ns, bool guess = false) {
    if (l == h->levels - 1) {
        coarse_apply<T>(h->stream, h->d_cinv, h->nc, b, x, ns);
        return;
    }
    const T one = (T)1;
    const bool prof = h->prof_on && h->prof_step && l == 0;
    auto sweep = [&](Vec<const cx<T>> xin, Vec<cx<T>> xout) {
        if (prof) h->prof_mark();
        apply_mode<T>(h, HELM_OP_L, l, MODE_JACOBI, one, xin, b, xout, ns);
        if (prof) {
            h->prof_mark();
            h->prof_pending_bytes += 3.0 * sizeof(cx<T>) * (double)h->Nl[0] * ns;
        }
    };
    // pre-smoothing: t = omega D^{-1} b (or t = J(x)), x = t + omega D^{-1} (b - L t)
    if (guess) sweep(cst(x), t);
    else apply_mode<T>(h, HELM_OP_L, l, MODE_JACOBI0, one, Vec<const cx<T>>{}, b, t, ns);
    sweep(cst(t), x);
    const long long Nc = h->Nl[l + 1];
    Vec<cx<T>> bc = at_ws<cx<T>>(ws, Lw.mg_b[l + 1], Nc);
    Vec<cx<T>> xc = at_ws<cx<T>>(ws, Lw.mg_x[l + 1], Nc);
    Vec<cx<T>> tc = at_ws<cx<T>>(ws, Lw.mg_t[l + 1], Nc);
    resid_restrict<T>(h, l, cst(x), b, bc, t, ns);
    vcycle<T>(h, Lw, ws, l + 1, cst(bc), xc, tc, ns);
    prolong<T>(h, l, cst(xc), x, ns);
    // post-smoothing: t = J(x), x = J(t)
    sweep(cst(x), t);
    sweep(cst(t), x);
}

template <typename T>
__global__ void k_zero(cx<T>* p, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = mk((T)0, (T)0);
}

template <typename T>
void zero(hipStream_t st, cx<T>* p, long long n) {
    if (n <= 0) return;
    k_zero<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, n);
}

// First level handled by the LDS-resident small-level cycle (-1: none).  The
// levels from there down to the coarsest must fit one workgroup's LDS
// (64 KB: b and x per level plus one shared scratch vector) and the
// coarsest mesh must be small enough for one workgroup to apply its dense
// inverse (at most 289 nodes).
template <typename T>
int small_start(const helm_t* h) {
    if (h->dim != 2 || h->levels < 2 || h->nc > 289 || h->opts.no_small || h->dir) return -1;
    for (int l = 1; l < h->levels - 1; ++l) {
        // shared scratch sized for level l and the coarse-solve partials
        size_t elems = std::max((size_t)h->Nl[l], 1024 * sizeof(cxd) / sizeof(cx<T>)) + 1;
        for (int m = l; m < h->levels; ++m) elems += 2 * (size_t)h->Nl[m];
        if (elems * sizeof(cx<T>) <= 65536 && h->levels - l <= MAX_SMALL) return l;
    }
    return -1;
}

template <typename T>
void run_small(helm_t* h, int l0, Vec<const cx<T>> b, Vec<cx<T>> x, int ns) {
    SmallCycle<T> sc{};
    sc.nlev = h->levels - l0;
    int off = 0;
    for (int m = 0; m < sc.nlev; ++m) {
        const int lev = l0 + m;
        sc.n[m] = h->nl[lev];
        sc.op[m] = make_op2<T>(h->coef(HELM_OP_L), h->nl[lev], h->omega);
        sc.off_b[m] = off;
        off += (int)h->Nl[lev];
        sc.off_x[m] = off;
        off += (int)h->Nl[lev];
    }
    // shared scratch: the largest level's vector, and room for 1024 FP64
    // complex partial sums of the coarse solve; 16-byte aligned
    off += off & 1;
    for (int m = 0; m < sc.nlev; ++m) {
        sc.off_t[m] = off;
        sc.mdiv[m] = ((1 << 20) + h->nl[l0 + m]) / (h->nl[l0 + m] + 1);
    }
    sc.off_part = off;
    off += std::max((int)h->Nl[l0], 1024 * (int)(sizeof(cxd) / sizeof(cx<T>)));
    vcycle_small<T>(h->stream, sc, sizeof(cx<T>) * (size_t)off, h->d_cinv, h->nc, b, x, ns);
}

// Levels that run with the register-streaming kernels: every 2D level
// above the small-level kernel, unless switched off.
inline bool use_stream(const helm_t* h, int l) {
    return h->dim == 2 && !h->opts.no_stream && h->nl[l] >= 16;
}

// 2D handles that run the fused HSS step (with Dirichlet faces only where
// the finest level streams: the streaming kernels clear the faces
// themselves, the LDS-tiled ones do not)
inline bool fused2d(const helm_t* h) {
    return h->dim == 2 && (!h->dir || (use_stream(h, 0) && h->levels > 1));
}

// Fused 2D cycle from a zero initial guess on level l (l >= 1 inside the HSS
// loop, or l = 0 for a stand-alone cycle).  b is read, x and t are this
// level's work buffers; returns the buffer holding the result (x or t).
// Per level: one kernel for the zero-guess pre-smoothing and the residual
// restriction, the coarser levels, one kernel for prolongation and the
// post-smoothing; the small levels run as one LDS-resident kernel.
template <typename T>
Vec<cx<T>> vcycle2d_zero(helm_t* h, const Layout& Lw, void* ws, int l, Vec<const cx<T>> b,
                         Vec<cx<T>> x, Vec<cx<T>> t, int ns) {
    if (l == h->levels - 1) {
        coarse_apply<T>(h->stream, h->d_cinv, h->nc, b, x, ns);
        return x;
    }
    if (l == small_start<T>(h)) {
        run_small<T>(h, l, b, x, ns);
        return x;
    }
    if (h->dir && !use_stream(h, l)) {
        // Dirichlet faces below the streaming levels: one pass per launch
        vcycle<T>(h, Lw, ws, l, b, x, t, ns);
        return x;
    }
    const Op2<T> L = make_op2<T>(h->coef(HELM_OP_L), h->nl[l], h->omega, h->dir);
    const long long Nc = h->Nl[l + 1];
    Vec<cx<T>> bc = at_ws<cx<T>>(ws, Lw.mg_b[l + 1], Nc);
    Vec<cx<T>> xc = at_ws<cx<T>>(ws, Lw.mg_x[l + 1], Nc);
    Vec<cx<T>> tc = at_ws<cx<T>>(ws, Lw.mg_t[l + 1], Nc);
    if (use_stream(h, l)) {
        stream_pre_2d<T>(h->stream, L, L, (T)0, Vec<const cx<T>>{}, Vec<const cx<T>>{},
                         Vec<cx<T>>{}, b, x, bc, ns);
        Vec<cx<T>> ec = vcycle2d_zero<T>(h, Lw, ws, l + 1, cst(bc), xc, tc, ns);
        STREAMCHK(stream_sweeps_2d<T>(h->stream, L, 2, cst(x), cst(ec), b, t, Vec<cx<T>>{}, false, ns));
        return t;
    }
    pre0r_2d<T>(h->stream, L, b, x, bc, ns);
    Vec<cx<T>> ec = vcycle2d_zero<T>(h, Lw, ws, l + 1, cst(bc), xc, tc, ns);
    sweeps_2d<T>(h->stream, L, 2, cst(x), cst(ec), b, t, false, ns);
    return t;
}

// One shifted-HSS step s with fused 2D kernels: the residual
// rho = c (R - B u) is formed together with the first cycle's
// pre-smoothing and residual restriction; cycle q's post-smoothing and
// cycle q+1's pre-smoothing run as one four-sweep pass; the last
// post-smoothing adds its result into u (writes it at step 0, u = 0).
template <typename T>
void hss_step2d(helm_t* h, const Layout& Lw, void* ws, int ns, int s) {
    const long long N = h->Nl[0];
    Vec<cx<T>> R = at_ws<cx<T>>(ws, Lw.R, N);
    Vec<cx<T>> u = at_ws<cx<T>>(ws, Lw.u, N);
    Vec<cx<T>> rho = at_ws<cx<T>>(ws, Lw.mg_b[0], N);
    Vec<cx<T>> xa = at_ws<cx<T>>(ws, Lw.mg_x[0], N);
    Vec<cx<T>> xb = at_ws<cx<T>>(ws, Lw.mg_t[0], N);
    const T c = (T)(2.0 * h->k / (h->k + 1.0));
    const Op2<T> L = make_op2<T>(h->coef(HELM_OP_L), h->nl[0], h->omega, h->dir);
    const Op2<T> Bs = make_op2<T>(h->coef(HELM_OP_BSHIFT), h->nl[0], h->omega, h->dir);
    Vec<const cx<T>> uin = s == 0 ? Vec<const cx<T>>{} : cst(u);
    if (h->levels == 1) {
        // single level: every cycle is the exact coarse solve
        if (s == 0) zero<T>(h->stream, u.base, N * ns);
        hss_pre0_2d<T>(h->stream, L, Bs, c, uin, cst(R), rho, xa, ns);
        coarse_apply<T>(h->stream, h->d_cinv, h->nc, cst(rho), xb, ns);
        axpy1<T>(h->stream, N, (T)1, cst(xb), u, ns);
        return;
    }
    const long long N1 = h->Nl[1];
    Vec<cx<T>> b1 = at_ws<cx<T>>(ws, Lw.mg_b[1], N1);
    Vec<cx<T>> x1 = at_ws<cx<T>>(ws, Lw.mg_x[1], N1);
    Vec<cx<T>> t1 = at_ws<cx<T>>(ws, Lw.mg_t[1], N1);
    const bool streaming = use_stream(h, 0);
    if (streaming) stream_pre_2d<T>(h->stream, L, Bs, c, uin, cst(R), rho, Vec<const cx<T>>{}, xa, b1, ns);
    else hss_pre0r_2d<T>(h->stream, L, Bs, c, uin, cst(R), rho, xa, b1, ns);
    Vec<cx<T>> x = xa, t = xb;
    for (int q = 0; q < h->cycles; ++q) {
        if (q > 0 && !streaming) resid_restrict2d<T>(h->stream, L, cst(x), cst(rho), b1, ns);
        Vec<const cx<T>> ec = cst(vcycle2d_zero<T>(h, Lw, ws, 1, cst(b1), x1, t1, ns));
        const bool last = q == h->cycles - 1;
        // the profiled kernel is the four-sweep pass (the single two-sweep
        // update pass when only one cycle is used)
        const bool prof = h->prof_on && (h->cycles == 1 || !last) && s % helm_s::PROF_EVERY == 0;
        if (prof) h->prof_mark();
        if (last) {
            if (streaming) STREAMCHK(stream_sweeps_2d<T>(h->stream, L, 2, cst(x), ec, cst(rho), u, Vec<cx<T>>{}, s > 0, ns));
            else sweeps_2d<T>(h->stream, L, 2, cst(x), ec, cst(rho), u, s > 0, ns);
        } else {
            if (streaming) STREAMCHK(stream_sweeps_2d<T>(h->stream, L, 4, cst(x), ec, cst(rho), t, b1, false, ns));
            else sweeps_2d<T>(h->stream, L, 4, cst(x), ec, cst(rho), t, false, ns);
            std::swap(x, t);
        }
        if (prof) {
            h->prof_mark();
            // algorithmic bytes: x, b and e_c (a quarter vector) read, x'
            // written, and with the streaming pass b_c (a quarter vector)
            // written; the update pass reads and writes u instead
            const double passes = last ? (s > 0 ? 4.25 : 3.25) : (streaming ? 3.5 : 3.25);
            h->prof_pending_bytes += sizeof(cx<T>) * (double)N * ns * passes;
        }
    }
}

// One shifted-HSS step s with one pass per launch (3D without the fused
// passes, and every mesh with Dirichlet faces): rho = c (R - B u), q V-cycles,
// u += e.
template <typename T>
void hss_step_generic(helm_t* h, const Layout& Lw, void* ws, int ns, int s) {
    const long long N = h->Nl[0];
    Vec<cx<T>> R = at_ws<cx<T>>(ws, Lw.R, N);
    Vec<cx<T>> u = at_ws<cx<T>>(ws, Lw.u, N);
    Vec<cx<T>> rho = at_ws<cx<T>>(ws, Lw.mg_b[0], N);
    Vec<cx<T>> e = at_ws<cx<T>>(ws, Lw.mg_x[0], N);
    Vec<cx<T>> t = at_ws<cx<T>>(ws, Lw.mg_t[0], N);
    const T c = (T)(2.0 * h->k / (h->k + 1.0));
    if (s == 0) zero<T>(h->stream, u.base, N * ns);
    apply_mode<T>(h, HELM_OP_BSHIFT, 0, MODE_RESID, c, cst(u), cst(R), rho, ns);
    h->prof_step = s % helm_s::PROF_EVERY == 0;
    vcycle<T>(h, Lw, ws, 0, cst(rho), e, t, ns);
    for (int q = 1; q < h->cycles; ++q) vcycle<T>(h, Lw, ws, 0, cst(rho), e, t, ns, true);
    h->prof_step = true;
    axpy1<T>(h->stream, N, (T)1, cst(e), u, ns);
}

// Two Jacobi sweeps on a 3D level through the fused passes, the first of
// them replaced as `first` says (the zero-guess sweep, the HSS residual with
// the zero-guess sweep, or a sweep from X, plus P Ec when pro); the second
// sweep's right-hand side is rho for the HSS forms, else Bv.  upd = 1 adds
// the result into Y.  In FP32 one pass runs both sweeps as pipeline stages;
// in FP64 the two-stage pass does not fit the registers of a 1024-thread
// workgroup, so two one-stage passes run with T in between.
// prof: bracket the first launch with timing events (the two-stage pass,
// or the first one-stage pass) and count its algorithmic bytes per column,
// `bytes` vectors of the level.
// The fused 3D sweeps in pairs (two stages per pass) in FP32, one per pass
// in FP64 (whose two-stage kernels exceed the register budget; also on the
// coarser levels, where halving the launches is worth less than the spills).
#ifndef HELM_K3_TWO_STAGE_FP32
#define HELM_K3_TWO_STAGE_FP32 1
#endif
#ifndef HELM_K3_TWO_STAGE_COARSE_FP64
#define HELM_K3_TWO_STAGE_COARSE_FP64 0
#endif
#ifndef HELM_K3_TWO_STAGE_FP64
#define HELM_K3_TWO_STAGE_FP64 0
#endif
#ifndef HELM_K3_PAIR_PRE_FP64
#define HELM_K3_PAIR_PRE_FP64 0
#endif
template <typename T>
constexpr bool two_stage3d(bool coarse) {
    return sizeof(T) == 4 ? HELM_K3_TWO_STAGE_FP32 != 0
                          : (HELM_K3_TWO_STAGE_FP64 != 0 || (coarse && HELM_K3_TWO_STAGE_COARSE_FP64 != 0));
}

template <typename T>
void sweeps3d(helm_t* h, const Op3F<T>& L, const Op3F<T>& B, int first, bool pro, int upd, T s,
              Vec<const cx<T>> X, Vec<const cx<T>> Bv, Vec<const cx<T>> Ec, Vec<cx<T>> Rho,
              Vec<cx<T>> Tmp, Vec<cx<T>> Y, int ns, bool two, bool prof = false, double bytes = 0.0) {
    if (prof) h->prof_mark();
    if (!two && first == F_PRE0 && !pro && upd == 0) {
        // both zero-guess sweeps in one stencil pass (the first formed on
        // the staged input planes)
        STREAMCHK((pass3d<T, T>(h->stream, L, L, F_JAC0, 1, false, 0, (T)1, Vec<const cx<T>>{}, Bv,
                                Vec<const cx<T>>{}, Vec<cx<T>>{}, Y, ns)));
        if (prof) {
            h->prof_mark();
            h->prof_pending_bytes += sizeof(cx<T>) * (double)ns * bytes;
        }
        return;
    }
    if (two) {
        STREAMCHK((pass3d<T, T>(h->stream, L, B, first, 2, pro, upd, s, X, Bv, Ec, Rho, Y, ns)));
    } else {
        STREAMCHK((pass3d<T, T>(h->stream, L, B, first, 1, pro, 0, s, X, Bv, Ec, Rho, Tmp, ns)));
    }
    if (prof) {
        h->prof_mark();
        h->prof_pending_bytes += sizeof(cx<T>) * (double)ns * bytes;
    }
    if (two) return;
    const bool hss = first == F_HSS || first == F_HSS0;
    STREAMCHK((pass3d<T, T>(h->stream, L, L, F_JAC, 1, false, upd, (T)1, cst(Tmp), hss ? cst(Rho) : Bv,
                            Vec<const cx<T>>{}, Vec<cx<T>>{}, Y, ns)));
}

// Fused 3D cycle from a zero initial guess on level l: the two
// pre-smoothing sweeps (the first from zero), one pass for the residual
// restriction, the coarser levels, and the prolongation with the two
// post-smoothing sweeps.  b is read, x and t are this level's work buffers;
// returns the buffer holding the result (x or t).
template <typename T>
Vec<cx<T>> vcycle3d_zero(helm_t* h, const Layout& Lw, void* ws, int l, Vec<const cx<T>> b,
                         Vec<cx<T>> x, Vec<cx<T>> t, int ns) {
    if (l == h->levels - 1) {
        coarse_apply<T>(h->stream, h->d_cinv, h->nc, b, x, ns);
        return x;
    }
    const Op3F<T> L = make_op3f<T>(h->coef(HELM_OP_L), h->nl[l], h->omega, h->dir);
    const long long Nc = h->Nl[l + 1];
    Vec<cx<T>> bc = at_ws<cx<T>>(ws, Lw.mg_b[l + 1], Nc);
    Vec<cx<T>> xc = at_ws<cx<T>>(ws, Lw.mg_x[l + 1], Nc);
    Vec<cx<T>> tc = at_ws<cx<T>>(ws, Lw.mg_t[l + 1], Nc);
    const Vec<const cx<T>> none{};
    const bool two = two_stage3d<T>(true);
    sweeps3d<T>(h, L, L, F_PRE0, false, 0, (T)1, none, b, none, Vec<cx<T>>{}, t, x, ns, two);
    rr3d<T>(h->stream, L, cst(x), b, bc, ns);
    Vec<cx<T>> ec = vcycle3d_zero<T>(h, Lw, ws, l + 1, cst(bc), xc, tc, ns);
    // the one-stage path ends in x (through t), the two-stage one in t
    Vec<cx<T>> out = two ? t : x;
    sweeps3d<T>(h, L, L, F_JAC, true, 0, (T)1, cst(x), b, cst(ec), Vec<cx<T>>{}, t, out, ns, two);
    return out;
}

// One shifted-HSS step s with the fused 3D passes: the residual
// rho = c (R - B_shift u) together with the first cycle's two pre-smoothing
// sweeps; per cycle the residual restriction, the coarser levels and the
// prolongation with two post-smoothing sweeps (cycles after the first start
// with two sweeps from the previous result); the last sweep adds its result
// into u (writes it at step 0, u = 0).
template <typename T>
void hss_step3d_fused(helm_t* h, const Layout& Lw, void* ws, int ns, int s) {
    const long long N = h->Nl[0];
    Vec<cx<T>> R = at_ws<cx<T>>(ws, Lw.R, N);
    Vec<cx<T>> u = at_ws<cx<T>>(ws, Lw.u, N);
    Vec<cx<T>> rho = at_ws<cx<T>>(ws, Lw.mg_b[0], N);
    Vec<cx<T>> x = at_ws<cx<T>>(ws, Lw.mg_x[0], N);
    Vec<cx<T>> t = at_ws<cx<T>>(ws, Lw.mg_t[0], N);
    const long long N1 = h->Nl[1];
    Vec<cx<T>> b1 = at_ws<cx<T>>(ws, Lw.mg_b[1], N1);
    Vec<cx<T>> x1 = at_ws<cx<T>>(ws, Lw.mg_x[1], N1);
    Vec<cx<T>> t1 = at_ws<cx<T>>(ws, Lw.mg_t[1], N1);
    const T c = (T)(2.0 * h->k / (h->k + 1.0));
    const Op3F<T> L = make_op3f<T>(h->coef(HELM_OP_L), h->nl[0], h->omega, h->dir);
    const Op3F<T> Bs = make_op3f<T>(h->coef(HELM_OP_BSHIFT), h->nl[0], h->omega, h->dir);
    const Vec<const cx<T>> none{};
    // the one-stage (FP64) sequence keeps the cycle's iterate in x, with t
    // between its two sweeps; the two-stage (FP32) one alternates x and t
    const bool two = two_stage3d<T>(false), one = !two;
    if (s == 0) {
        sweeps3d<T>(h, L, Bs, F_HSS0, false, 0, c, none, cst(R), none, rho, t, x, ns, two);
    } else if (one) {
        // rho = c (R - B u) in one pass, then both zero-guess sweeps on rho
        // in the next (five vectors moved instead of seven)
        STREAMCHK((pass3d<T, T>(h->stream, Bs, Bs, F_RESID, 1, false, 0, c, cst(u), cst(R), none,
                                Vec<cx<T>>{}, rho, ns)));
        sweeps3d<T>(h, L, L, F_PRE0, false, 0, (T)1, none, cst(rho), none, Vec<cx<T>>{}, t, x, ns, false);
    } else {
        sweeps3d<T>(h, L, Bs, F_HSS, false, 0, c, cst(u), cst(R), none, rho, t, x, ns, two);
    }
    for (int q = 0; q < h->cycles; ++q) {
        if (q > 0) {
            // the pre-smoothing pair from the previous result
            const bool pair = two || HELM_K3_PAIR_PRE_FP64 != 0;
            sweeps3d<T>(h, L, L, F_JAC, false, 0, (T)1, cst(x), cst(rho), none, Vec<cx<T>>{}, t,
                        pair ? t : x, ns, pair);
            if (pair) std::swap(x, t);
        }
        rr3d<T>(h->stream, L, cst(x), cst(rho), b1, ns);
        Vec<const cx<T>> ec = cst(vcycle3d_zero<T>(h, Lw, ws, 1, cst(b1), x1, t1, ns));
        const bool last = q == h->cycles - 1;
        // the profiled pass: the prolongation with the first (FP64) or both
        // (FP32) post-smoothing sweeps of the cycles before the last; x, rho
        // and e_c (an eighth vector) read, the result written
        const bool prof = h->prof_on && !last && s % helm_s::PROF_EVERY == 0;
        if (last) {
            sweeps3d<T>(h, L, L, F_JAC, true, s > 0 ? 1 : 0, (T)1, cst(x), cst(rho), ec, Vec<cx<T>>{},
                        t, u, ns, two);
        } else {
            sweeps3d<T>(h, L, L, F_JAC, true, 0, (T)1, cst(x), cst(rho), ec, Vec<cx<T>>{}, t,
                        one ? x : t, ns, two, prof, 3.125 * (double)N);
            if (!one) std::swap(x, t);
        }
    }
}

// ---- the paper's multigrid variant (Sec. 5.3): W-cycle, GMRES smoothing ----
#include "wcycle_impl.h"

// ---- the mixed formulation ([DG0]^2 x P1, 2D) ------------------------------
#include "mixed_impl.h"

// HSS step s of the handle's variant on the slot range described by L.
template <typename T>
void hss_step(helm_t* h, const Layout& L, void* ws, int ns, int s) {
    if (h->mixed) {
        hss_step_mixed<T>(h, L, ws, ns, s);
        return;
    }
    if constexpr (std::is_same<T, double>::value) {
        if (w_variant(h)) {
            hss_step_w(h, L, ws, ns, s);
            return;
        }
    }
    if (fused2d(h)) hss_step2d<T>(h, L, ws, ns, s);
    else if (fused3d(h) && h->levels > 1) hss_step3d_fused<T>(h, L, ws, ns, s);
    else hss_step_generic<T>(h, L, ws, ns, s);
}

// A range of slots that runs its HSS loop on a stream of its own: the
// layout's per-slot buffers start at the range's first slot.
struct SlotGroup {
    Layout L;
    int ns;
    hipStream_t st;
};

template <typename T>
Layout shift_slots(const helm_t* h, const Layout& Lw, int s0) {
    Layout g = Lw;
    const size_t e = sizeof(cx<T>);
    for (int l = 0; l < h->levels; ++l) {
        const size_t d = e * (size_t)s0 * (size_t)h->Nl[l];
        g.mg_b[l] += d;
        g.mg_x[l] += d;
        g.mg_t[l] += d;
    }
    g.R += e * (size_t)s0 * (size_t)h->Nl[0];
    g.u += e * (size_t)s0 * (size_t)h->Nl[0];
    return g;
}

// Shifted-HSS preconditioner on the slot-major buffers R -> u (precision T)
// for every group; the groups' steps are enqueued in turn so that the
// streams advance together and one group's finest-level passes overlap
// another's latency-bound coarse levels.
template <typename T>
void hss_loop(helm_t* h, void* ws, const SlotGroup* g, int ng, int s_begin = 0, int s_end = -1) {
    struct Restore {
        helm_t* h;
        hipStream_t st;
        ~Restore() { h->stream = st; }
    } restore{h, h->stream};
    if (s_end < 0) s_end = h->hss_steps;
    for (int s = s_begin; s < s_end; ++s) {
        for (int q = 0; q < ng; ++q) {
            h->stream = g[q].st;
            hss_step<T>(h, g[q].L, ws, g[q].ns, s);
        }
    }
}

// Number of V-cycles per inner HSS solve.  With exact inner solves the HSS
// error contracts by nu = (k-1)/(k+1) per step in the H-norm (the Cayley
// transform is H-unitary).  An inexact inner solve with cycle error E turns
// the step's error map T into T + E(I - T); as ||I - T|| <= 1 + nu, it stays
// a contraction when ||E|| (1 + nu) < 1 - nu, i.e. ||E|| < 1/k.  The V-cycle
// rate rho_V is measured once per handle by power iteration on the cycle's
// error map e <- e - V(L e) from a fixed pseudo-random start, and the
// smallest q with rho_V^q <= 1/k is used (at least 2, at most 8; 1/n for
// the mixed form, see below).
template <typename T>
void ensure_cycles(helm_t* h, const Layout& Lw, void* ws) {
    if (!h->cycles_auto || h->vrate > 0.0) return;
    const long long N = h->Nl[0];
    Vec<cx<T>> e = at_ws<cx<T>>(ws, Lw.R, N);
    Vec<cx<T>> r = at_ws<cx<T>>(ws, Lw.u, N);
    Vec<cx<T>> d = at_ws<cx<T>>(ws, Lw.mg_x[0], N);
    Vec<cx<T>> t = at_ws<cx<T>>(ws, Lw.mg_t[0], N);
    Vec<cxd> e64 = at_ws<cxd>(ws, Lw.V, N);
    double* d_norm = reinterpret_cast<double*>(static_cast<char*>(ws) + Lw.dnorm);
    double* d_npart = reinterpret_cast<double*>(static_cast<char*>(ws) + Lw.npart);
    std::vector<cx<T>> init(N);
    uint64_t state = 0x9E3779B97F4A7C15ull;
    for (long long q = 0; q < N; ++q) {  // xorshift64*, uniform in [-1, 1)
        auto next = [&]() {
            state ^= state >> 12;
            state ^= state << 25;
            state ^= state >> 27;
            return (double)((state * 0x2545F4914F6CDD1Dull) >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        };
        const double re = next(), im = next();
        init[q] = mk((T)re, (T)im);
    }
    HIPCHK(hipMemcpyAsync(e.base, init.data(), sizeof(cx<T>) * N, hipMemcpyHostToDevice, h->stream));
    dir_mask<T>(h, h->stream, 0, e, 1);
    const int iters = 8;
    std::vector<double> norms;
    for (int it = 0; it < iters; ++it) {
        apply_mode<T>(h, HELM_OP_L, 0, MODE_APPLY, (T)1, cst(e), Vec<const cx<T>>{}, r, 1);
        vcycle<T>(h, Lw, ws, 0, cst(r), d, t, 1);
        axpy1<T>(h->stream, N, (T)-1, cst(d), e, 1);
        copy_cast<double, T>(h->stream, N, cst(e), e64, 1);
        norm2(h->stream, N, cst(e64), d_npart, d_norm, 1, 1);
        double nv = 0.0;
        HIPCHK(hipMemcpyAsync(&nv, d_norm, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        norms.push_back(nv);
    }
    double rate = std::pow(norms[iters - 1] / norms[iters - 4], 1.0 / 3.0);
    if (!(rate > 0.0) || !std::isfinite(rate)) rate = 0.5;
    h->vrate = rate;
    // ||T + E (I - T)|| <= nu + rho^q (1 + nu) < 1  <=>  rho^q < (1 - nu)/(1 + nu) = 1/k.
    // Mixed form: sigma' = (grad u' + g) / (k (dh - i)) turns an error e in u
    // into one of size ~ |e| / (h k) in sigma, so the cycle error must be
    // smaller by h k: rho^q < h = 1/n.
    const double bound = h->mixed ? 1.0 / h->n : 1.0 / h->k;
    int q = 2;
    while (q < 8 && std::pow(rate, q) > bound) ++q;
    h->cycles = q;
}

// Capture HSS steps [s_begin, s_end) of one slot group on the capture
// stream.  Returns the graph (caller destroys it).
template <typename T>
hipGraph_t capture_steps(helm_t* h, void* ws, const SlotGroup& g, int s_begin, int s_end) {
    hipGraph_t graph = nullptr;
    SlotGroup cg = g;
    cg.st = h->cap_stream;
    HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        hss_loop<T>(h, ws, &cg, 1, s_begin, s_end);
    } catch (...) {
        (void)hipStreamEndCapture(h->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    HIPCHK(hipStreamEndCapture(h->cap_stream, &graph));
    return graph;
}

template <typename T>
hipGraphExec_t instantiate_steps(helm_t* h, void* ws, const SlotGroup& g, int s_begin, int s_end) {
    hipGraph_t graph = capture_steps<T>(h, ws, g, s_begin, s_end);
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(e);
    return ex;
}

// z = B~^{-1} v for ns slots: v and z addressed through Vec descriptors
// (FP64 v; z in the mode's storage type).
template <typename T>
void precondition(helm_t* h, const Layout& Lw, void* ws, Vec<const cxd> v, Vec<cx<T>> z, int ns) {
    const long long N = h->nv;  // column length (the mixed vectors included)
    copy_cast<T, double>(h->stream, N, v, at_ws<cx<T>>(ws, Lw.R, N), ns);
    // optionally two slot groups on two streams when there are several columns
    // (not with the W variant, whose smoother buffers are not per group)
    const int ng = (ns >= 2 && h->opts.split && !w_variant(h) && !h->mixed) ? 2 : 1;
    const int n0 = ng == 2 ? (ns + 1) / 2 : ns;
    SlotGroup grp[2] = {{Lw, n0, h->stream}, {shift_slots<T>(h, Lw, n0), ns - n0, h->aux_stream}};
    if (ng == 2) {
        HIPCHK(hipEventRecord(h->ev_fork, h->stream));
        HIPCHK(hipStreamWaitEvent(h->aux_stream, h->ev_fork, 0));
    }
    // timed runs stay eager: event timings are read between the launches;
    // the W variant (thousands of small launches per step) runs eagerly too
    if (h->prof_on || h->opts.no_graphs || w_variant(h)) {
        hss_loop<T>(h, ws, grp, ng);
    } else {
        // each group's HSS loop (all steps, cycles and levels) is replayed
        // from captured HIP graphs; it reads R and writes u at fixed
        // workspace addresses, so the graphs serve every outer iteration.
        // A loop of up to ~20000 launches is one graph; a longer one is a
        // head graph (step 0 and the remainder) and a body graph of a block
        // of steps replayed several times (steps s > 0 launch the same work)
        const int tag = (int)sizeof(T);
        for (int q = 0; q < ng; ++q) {
            const int s0 = q == 0 ? 0 : n0;
            const helm_s::GraphEntry* ge = nullptr;
            for (const auto& e : h->graphs)
                if (e.ws == ws && e.cap == Lw.cap && e.s0 == s0 && e.ns == grp[q].ns &&
                    e.tag == tag && e.cycles == h->cycles)
                    ge = &e;
            if (!ge) {
                // run the first two steps eagerly before capturing, so that
                // the launches that measure their best tiling do so (the
                // captured loop recomputes everything from step 0)
                {
                    struct Restore {
                        helm_t* h;
                        hipStream_t st;
                        ~Restore() { h->stream = st; }
                    } restore{h, h->stream};
                    h->stream = grp[q].st;
                    for (int s = 0; s < std::min(2, h->hss_steps); ++s) {
                        hss_step<T>(h, grp[q].L, ws, grp[q].ns, s);
                    }
                }
                const int S = h->hss_steps;
                int head = S, block = 0, reps = 0;
                if (S >= 2) {
                    // launches of one step s > 0
                    hipGraph_t one = capture_steps<T>(h, ws, grp[q], 1, 2);
                    size_t n1 = 0;
                    const hipError_t e = hipGraphGetNodes(one, nullptr, &n1);
                    (void)hipGraphDestroy(one);
                    HIPCHK(e);
                    const size_t limit = 20000;
                    block = (int)std::max<size_t>(1, limit / std::max<size_t>(1, n1));
                    if (S - 1 > block) {
                        const int r = (S - 1) % block;
                        head = 1 + r;
                        reps = (S - 1 - r) / block;
                    }
                }
                helm_s::GraphEntry ne{ws, Lw.cap, s0, grp[q].ns, tag, h->cycles, nullptr, nullptr, reps};
                ne.head = instantiate_steps<T>(h, ws, grp[q], 0, head);
                if (reps > 0) {
                    try {
                        ne.body = instantiate_steps<T>(h, ws, grp[q], head, head + block);
                    } catch (...) {
                        (void)hipGraphExecDestroy(ne.head);
                        throw;
                    }
                }
                h->graphs.push_back(ne);
                ge = &h->graphs.back();
            }
            HIPCHK(hipGraphLaunch(ge->head, grp[q].st));
            for (int r = 0; r < ge->reps; ++r) HIPCHK(hipGraphLaunch(ge->body, grp[q].st));
        }
    }
    if (ng == 2) {
        HIPCHK(hipEventRecord(h->ev_join, h->aux_stream));
        HIPCHK(hipStreamWaitEvent(h->stream, h->ev_join, 0));
    }
    copy_cast<T, T>(h->stream, N, cst(at_ws<cx<T>>(ws, Lw.u, N)), z, ns);
}

// One stand-alone cycle b -> x (zero initial guess) on level 0.
template <typename T>
void vcycle_entry(helm_t* h, const Layout& Lw, void* ws, const void* b, void* x, int ns) {
    const long long N = h->Nl[0];
    Vec<const cx<T>> bv{static_cast<const cx<T>*>(b), N, 0, nullptr};
    Vec<cx<T>> xv{static_cast<cx<T>*>(x), N, 0, nullptr};
    Vec<cx<T>> tv = at_ws<cx<T>>(ws, Lw.mg_t[0], N);
    if constexpr (std::is_same<T, double>::value) {
        if (w_variant(h)) {
            wcycle_gm(h, Lw, ws, 0, bv, xv, false, ns);
            return;
        }
    }
    if (fused2d(h) || fused3d(h)) {
        Vec<cx<T>> r = h->dim == 2 ? vcycle2d_zero<T>(h, Lw, ws, 0, bv, xv, tv, ns)
                                   : vcycle3d_zero<T>(h, Lw, ws, 0, bv, xv, tv, ns);
        if (r.base != xv.base) copy_cast<T, T>(h->stream, N, cst(r), xv, ns);
    } else {
        vcycle<T>(h, Lw, ws, 0, bv, xv, tv, ns);
    }
}

// ----------------------------------------------------------------- FGMRES --
#include "fgmres_engine.h"

// helm_solve: every column is admitted at once; steps run until all are done.
template <typename T>
int solve_columns(helm_t* h, const cxd* rhs, cxd* x, int nrhs, double tol, void* ws,
                  helm_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    const long long N = h->nv;
    Engine<T> E;
    struct Guard {
        Engine<T>& e;
        ~Guard() { e.release(); }
    } guard{E};
    E.init(h, ws, nrhs, tol);
    ensure_cycles<T>(h, E.Lw, ws);
    h->prof_on = h->opts.profile != 0;
    h->prof_used = 0;
    h->prof_ms = h->prof_bytes = h->prof_pending_bytes = 0.0;
    h->prof_launches = 0;
    for (int c = 0; c < nrhs; ++c)
        E.admit(c, rhs + (long long)c * N, h->opts.x0_given ? x + (long long)c * N : nullptr, tol);
    int steps = 0;
    while (E.enqueue()) {
        E.complete();
        if (steps++ == 0) {
            for (const auto& C : E.col)
                if (C.have_bnorm && !std::isfinite(C.bnorm)) {
                    g_last_error = "non-finite right-hand side";
                    h->prof_on = false;
                    return HELM_EINVAL;
                }
        }
        if (h->opts.verbose > 0 && steps % h->opts.verbose == 0) {
            double worst = 0.0;
            int active = 0;
            for (const auto& C : E.col)
                if (C.phase == COL_ACTIVE) {
                    worst = std::max(worst, C.est);
                    ++active;
                }
            fprintf(stderr, "[helm] step %d: max Arnoldi residual %.3e over %d active columns\n",
                    steps, worst, active);
            fflush(stderr);
        }
    }
    HIPCHK(hipMemcpyAsync(x, E.Xb(), sizeof(cxd) * N * nrhs, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    h->prof_on = false;
    bool ok = true;
    double worst = 0.0, worst_arn = 0.0, rate = 0.0;
    int maxits = 0, restarts = 0;
    for (const auto& C : E.col) {
        ok = ok && C.converged;
        worst = std::max(worst, C.true_rel);
        worst_arn = std::max(worst_arn, C.est);
        maxits = std::max(maxits, C.its);
        restarts = std::max(restarts, C.restarts);
        if (C.its > 0 && C.r0 > 0.0)
            rate = std::max(rate, std::pow(C.true_rel * C.bnorm / C.r0, 1.0 / C.its));
    }
    if (st) {
        st->outer_its = maxits;
        st->restarts = restarts;
        st->hss_steps = h->hss_steps;
        st->vcycles = E.vcycles;
        st->converged = ok ? 1 : 0;
        st->arnoldi_rel_residual = worst_arn;
        st->true_rel_residual = worst;
        st->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        st->precond_ms = E.precond_ms;
        st->sweep_ms = h->prof_ms;
        st->sweep_launches = h->prof_launches;
        st->sweep_bytes = h->prof_bytes;
        st->mg_cycles = h->cycles;
        st->vcycle_rate = h->vrate;
        st->reorth_passes = E.reorth;
        st->outer_rate = rate;
    }
    return ok ? HELM_OK : HELM_ENOCONV;
}

// Preconditioned Richardson, the stationary iteration of Sec. 4:
// x <- x + B~^{-1} (b - B x), per column until |b - B x| <= tol |b| or
// max_outer iterations.  Each iteration computes the true residual of every
// running column (one batched stencil pass and norm), reads the norms on
// the host, and applies the preconditioner to the residuals of the columns
// still running; a column that has converged keeps its iterate.
template <typename T>
int richardson_columns(helm_t* h, const cxd* rhs, cxd* x, int nrhs, double tol, void* ws,
                       helm_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    const long long N = h->nv;
    const Layout Lw = layout(h, nrhs);
    hipStream_t s = h->stream;
    char* w = static_cast<char*>(ws);
    int* d_cols = reinterpret_cast<int*>(w + Lw.maps);          // running column ids
    int* d_slot = d_cols + nrhs;                                // their residual slots
    double* d_norm = reinterpret_cast<double*>(w + Lw.dnorm);   // [0, n): |r|, [n, 2n): |b|
    double* d_npart = reinterpret_cast<double*>(w + Lw.npart);
    cxd* d_one = reinterpret_cast<cxd*>(w + Lw.dy);
    cxd* r = reinterpret_cast<cxd*>(w + Lw.V);                  // residual slots
    cx<T>* z = reinterpret_cast<cx<T>*>(w + Lw.Z);              // corrections
    int* hmap = nullptr;
    double* hn = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct Guard {
        int*& m;
        double*& n;
        hipEvent_t &a, &b;
        ~Guard() {
            if (m) (void)hipHostFree(m);
            if (n) (void)hipHostFree(n);
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } guard{hmap, hn, e0, e1};
    // pinned maps: [0, 2 nrhs) for the preconditioner pass, [2 nrhs, 3 nrhs)
    // for the residual pass (each region is rewritten only after the copy
    // that last read it has completed)
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hmap), sizeof(int) * 3 * nrhs, 0));
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hn), sizeof(double) * 2 * nrhs, 0));
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    ensure_cycles<T>(h, Lw, ws);
    h->prof_on = h->opts.profile != 0;
    h->prof_used = 0;
    h->prof_ms = h->prof_bytes = h->prof_pending_bytes = 0.0;
    h->prof_launches = 0;
    struct ProfOff {
        helm_t* h;
        ~ProfOff() { h->prof_on = false; }
    } prof_off{h};
    if (!h->opts.x0_given) zero<double>(s, x, N * nrhs);
    const cxd one = mk(1.0, 0.0);
    HIPCHK(hipMemcpyAsync(d_one, &one, sizeof(cxd), hipMemcpyHostToDevice, s));
    norm2(s, N, Vec<const cxd>{rhs, N, 0, nullptr}, d_npart, d_norm + nrhs, 1, nrhs);
    std::vector<double> bnorm(nrhs), rel(nrhs, 0.0), r0(nrhs, -1.0);
    std::vector<int> its(nrhs, 0), done(nrhs, 0);
    std::vector<int> run;
    for (int c = 0; c < nrhs; ++c) run.push_back(c);
    const Coef b0 = h->coef(h->delta == 0.0 ? HELM_OP_B0 : HELM_OP_BDELTA);
    double precond_ms = 0.0;
    long long vcycles = 0;
    bool first = true;
    while (!run.empty()) {
        const int nr = (int)run.size();
        int* hrun = hmap + 2 * nrhs;
        for (int q = 0; q < nr; ++q) hrun[q] = run[q];
        HIPCHK(hipMemcpyAsync(d_cols, hrun, sizeof(int) * nr, hipMemcpyHostToDevice, s));
        // r[q] = b[c] - B x[c] for the running columns c = run[q]
        const Vec<const cxd> Xr{x, N, 0, d_cols}, Br{rhs, N, 0, d_cols};
        const Vec<cxd> Rr{r, N, 0, nullptr};
        if (h->mixed)
            mixed_system<double>(h, h->delta, MODE_RESID, Xr, Br, Rr, nr);
        else if (h->dim == 2)
            stencil2d<double, double>(s, make_op2<double>(b0, h->n, h->omega), MODE_RESID, 1.0, Xr,
                                      Br, Rr, nr);
        else
            op3d<double, double>(h, s, b0, 0, MODE_RESID, 1.0, Xr, Br, Rr, nr);
        if (!h->mixed) dir_mask<double>(h, s, 0, Rr, nr);
        norm2(s, N, cst(Rr), d_npart, d_norm, 1, nr);
        HIPCHK(hipMemcpyAsync(hn, d_norm, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (first) {
            for (int c = 0; c < nrhs; ++c) {
                bnorm[c] = hn[nrhs + c];
                if (!std::isfinite(bnorm[c])) {
                    g_last_error = "non-finite right-hand side";
                    return HELM_EINVAL;
                }
            }
            first = false;
        }
        if (h->prof_on) h->prof_collect();
        float ms = 0.f;
        if (vcycles > 0 && hipEventElapsedTime(&ms, e0, e1) == hipSuccess) precond_ms += ms;
        std::vector<int> next, slot;
        for (int q = 0; q < nr; ++q) {
            const int c = run[q];
            const double rn = hn[q];
            if (r0[c] < 0.0) r0[c] = rn;
            if (bnorm[c] == 0.0) {  // zero column: x = 0
                zero<double>(s, x + (long long)c * N, N);
                rel[c] = 0.0;
                done[c] = 1;
                continue;
            }
            rel[c] = rn / bnorm[c];
            if (rel[c] <= tol) done[c] = 1;
            else if (its[c] >= h->max_outer || !std::isfinite(rn)) done[c] = 0;
            else {
                next.push_back(c);
                slot.push_back(q);
                continue;
            }
            run[q] = -1;
        }
        if (next.empty()) break;
        // z[s] = B~^{-1} r[slot[s]], then x[next[s]] += z[s]
        const int nn = (int)next.size();
        for (int q = 0; q < nn; ++q) {
            hmap[q] = next[q];
            hmap[nrhs + q] = slot[q];
        }
        HIPCHK(hipMemcpyAsync(d_cols, hmap, sizeof(int) * 2 * nrhs, hipMemcpyHostToDevice, s));
        HIPCHK(hipEventRecord(e0, s));
        precondition<T>(h, Lw, ws, Vec<const cxd>{r, N, 0, d_slot}, Vec<cx<T>>{z, N, 0, nullptr}, nn);
        HIPCHK(hipEventRecord(e1, s));
        vcycles += (long long)nn * h->hss_steps * h->cycles;
        update_solution<T>(s, N, 1, nullptr, Vec<const cx<T>>{z, N, 0, nullptr}, d_one, 0,
                           Vec<cxd>{x, N, 0, d_cols}, nn);
        for (int c : next) ++its[c];
        run = next;
    }
    HIPCHK(hipStreamSynchronize(s));
    if (h->prof_on) h->prof_collect();
    bool ok = true;
    double worst = 0.0, rate = 0.0;
    int maxits = 0;
    for (int c = 0; c < nrhs; ++c) {
        ok = ok && done[c];
        worst = std::max(worst, rel[c]);
        maxits = std::max(maxits, its[c]);
        if (its[c] > 0 && r0[c] > 0.0)
            rate = std::max(rate, std::pow(rel[c] * bnorm[c] / r0[c], 1.0 / its[c]));
    }
    if (st) {
        *st = helm_stats{};
        st->outer_its = maxits;
        st->restarts = 0;
        st->hss_steps = h->hss_steps;
        st->vcycles = vcycles;
        st->converged = ok ? 1 : 0;
        st->arnoldi_rel_residual = worst;
        st->true_rel_residual = worst;
        st->solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        st->precond_ms = precond_ms;
        st->sweep_ms = h->prof_ms;
        st->sweep_launches = h->prof_launches;
        st->sweep_bytes = h->prof_bytes;
        st->mg_cycles = h->cycles;
        st->vcycle_rate = h->vrate;
        st->reorth_passes = 0;
        st->outer_rate = rate;
    }
    return ok ? HELM_OK : HELM_ENOCONV;
}

// The preconditioner with the HSS residual |v - B_shift u_s| recorded after
// every step s (FP64 arithmetic; u_s promoted from the storage precision).
template <typename T>
void hss_history(helm_t* h, const Layout& Lw, void* ws, const cxd* v, Vec<cx<T>> z, int ns,
                 double* res) {
    const long long N = h->nv;
    hipStream_t s = h->stream;
    const int S = h->hss_steps;
    double* d_norm = reinterpret_cast<double*>(static_cast<char*>(ws) + Lw.dnorm);
    double* d_npart = reinterpret_cast<double*>(static_cast<char*>(ws) + Lw.npart);
    const Vec<cxd> rv = at_ws<cxd>(ws, Lw.V, N);
    const Vec<const cxd> vv{v, N, 0, nullptr};
    const Vec<const cx<T>> u = cst(at_ws<cx<T>>(ws, Lw.u, N));
    const Coef cb = h->coef(HELM_OP_BSHIFT);
    std::vector<double> hn(2 * (size_t)ns);
    if (h->dir && !h->mixed) {
        // v is taken as zero on the Dirichlet nodes, as the residuals below
        copy_cast<double, double>(s, N, vv, rv, ns);
        dir_mask<double>(h, s, 0, rv, ns);
        copy_cast<T, double>(s, N, cst(rv), at_ws<cx<T>>(ws, Lw.R, N), ns);
        norm2(s, N, cst(rv), d_npart, d_norm, 1, ns);
    } else {
        copy_cast<T, double>(s, N, vv, at_ws<cx<T>>(ws, Lw.R, N), ns);
        norm2(s, N, vv, d_npart, d_norm, 1, ns);
    }
    HIPCHK(hipMemcpyAsync(hn.data(), d_norm, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int c = 0; c < ns; ++c) res[(size_t)c * (S + 1)] = hn[c];
    SlotGroup g{Lw, ns, s};
    for (int step = 0; step < S; ++step) {
        hss_step<T>(h, g.L, ws, ns, step);
        if (h->mixed)
            mixed_system<T>(h, h->dh, MODE_RESID, u, vv, rv, ns);
        else if (h->dim == 2)
            stencil2d<double, T>(s, make_op2<double>(cb, h->n, h->omega), MODE_RESID, 1.0, u, vv, rv,
                                 ns);
        else
            op3d<double, T>(h, s, cb, 0, MODE_RESID, 1.0, u, vv, rv, ns);
        if (!h->mixed) dir_mask<double>(h, s, 0, rv, ns);
        norm2(s, N, cst(rv), d_npart, d_norm, 1, ns);
        HIPCHK(hipMemcpyAsync(hn.data(), d_norm, sizeof(double) * ns, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int c = 0; c < ns; ++c) res[(size_t)c * (S + 1) + step + 1] = hn[c];
    }
    copy_cast<T, T>(s, N, u, z, ns);
}

int status_from_exception() { return HELM_EDEVICE; }

}  // namespace

// =================================================================== C ABI ==
extern "C" {

void helm_opts_default(helm_opts* o) {
    if (!o) return;
    o->precision = HELM_FP64;
    o->nu1 = 2;
    o->nu2 = 2;
    o->omega = 2.0 / 3.0;
    o->hss_m = 1;
    o->hss_steps = 0;
    o->restart = 0;
    o->max_outer = 0;
    o->x0_given = 0;
    o->profile = 0;
    o->mg_cycles = 0;
    o->no_graphs = 0;
    o->no_small = 0;
    o->verbose = 0;
    o->no_stream = 0;
    o->full_reorth = 0;
    o->split = 0;
    o->outer = HELM_OUTER_FGMRES;
    o->cycle = HELM_CYCLE_V_JACOBI;
    o->smooth_its = 0;
}

const char* helm_strerror(int status) {
    switch (status) {
        case HELM_OK: return "ok";
        case HELM_EINVAL: return "invalid argument";
        case HELM_ENOMEM: return "out of memory";
        case HELM_EDEVICE: return "HIP device error";
        case HELM_ENOCONV: return "not converged within max_outer";
        case HELM_ENOTSUP: return "not supported by this build";
    }
    return "unknown status";
}

const char* helm_last_error(void) { return g_last_error.c_str(); }

// device objects owned by a handle (null-safe; used on every exit path)
static void release_handle_objects(helm_t* h) {
    if (h->d_cinv) (void)hipFree(h->d_cinv);
    h->d_cinv = nullptr;
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->aux_stream) (void)hipStreamDestroy(h->aux_stream);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    h->cap_stream = h->aux_stream = nullptr;
    h->ev_fork = h->ev_join = nullptr;
}

int helm_create(const helm_mesh* mesh, double k, double delta, double delta_hat,
                const helm_bc* bc, const helm_opts* opts, void* hip_stream, helm_t** out) {
    if (!out) return HELM_EINVAL;
    *out = nullptr;
    if (!mesh) return HELM_EINVAL;
    helm_opts o;
    if (opts) o = *opts; else helm_opts_default(&o);
    if (mesh->dim != 2 && mesh->dim != 3) return HELM_EINVAL;
    if ((mesh->dim == 2 && mesh->elem != HELM_P1_TRI_RIGHT && mesh->elem != HELM_MIXED_DG0_P1) ||
        (mesh->dim == 3 && mesh->elem != HELM_Q1_HEX))
        return HELM_EINVAL;
    const bool mixed = mesh->elem == HELM_MIXED_DG0_P1;
    if (mesh->n < 2 || mesh->levels < 1 || mesh->levels > 30) return HELM_EINVAL;
    if (mesh->n % (1 << (mesh->levels - 1)) != 0) return HELM_EINVAL;
    if (!(k > 0.0) || !std::isfinite(k)) return HELM_EINVAL;
    if (!(delta >= 0.0) || !std::isfinite(delta)) return HELM_EINVAL;
    if (!(delta_hat > delta) || !std::isfinite(delta_hat)) return HELM_EINVAL;
    if (o.hss_m < 1 || o.hss_steps < 0 || o.mg_cycles < 0 || o.mg_cycles > 16) return HELM_EINVAL;
    if (!(o.omega > 0.0 && o.omega < 2.0)) return HELM_EINVAL;
    if (o.precision != HELM_FP64 && o.precision != HELM_FP32_MG) return HELM_EINVAL;
    if (o.restart < 0 || o.max_outer < 0 || o.restart > 2000) return HELM_EINVAL;
    if (o.outer != HELM_OUTER_FGMRES && o.outer != HELM_OUTER_RICHARDSON) return HELM_EINVAL;
    if (o.cycle != HELM_CYCLE_V_JACOBI && o.cycle != HELM_CYCLE_W_GMRES) return HELM_EINVAL;
    if (o.smooth_its < 0 || o.smooth_its > 20) return HELM_EINVAL;
    const bool wvar = o.cycle == HELM_CYCLE_W_GMRES;
    const unsigned dirm = bc ? bc->dirichlet_faces : 0u;
    if (dirm & ~((1u << (2 * mesh->dim)) - 1u)) return HELM_EINVAL;
    // Dirichlet faces: primal form with V cycles only
    if (dirm && (mixed || wvar)) return HELM_ENOTSUP;
    if (!wvar && (o.nu1 != 2 || o.nu2 != 2)) return HELM_ENOTSUP;
    if (wvar && o.precision != HELM_FP64) return HELM_ENOTSUP;
    // the mixed formulation: V cycles
    if (mixed && wvar) return HELM_ENOTSUP;
    const int nc_side = mesh->n >> (mesh->levels - 1);
    long long ncoarse = 1;
    for (int d = 0; d < mesh->dim; ++d) ncoarse *= (nc_side + 1);
    if (!wvar && ncoarse > 4096) return HELM_EINVAL;

    helm_t* h = new (std::nothrow) helm_t;
    if (!h) return HELM_ENOMEM;
    try {
        h->dim = mesh->dim;
        h->elem = mesh->elem;
        h->n = mesh->n;
        h->levels = mesh->levels;
        h->k = k;
        h->delta = delta;
        h->dh = delta_hat;
        h->opts = o;
        h->prec = o.precision;
        h->omega = o.omega;
        h->stream = static_cast<hipStream_t>(hip_stream);
        HIPCHK(hipGetDevice(&h->device));
        h->hss_steps = o.hss_steps > 0 ? o.hss_steps : (int)(o.hss_m * std::ceil(k));
        h->cycles = o.mg_cycles > 0 ? o.mg_cycles : (wvar ? 1 : 2);
        h->cycles_auto = o.mg_cycles == 0 && !wvar;
        h->smooth_its = o.smooth_its > 0 ? o.smooth_its : 5;
        h->restart = o.restart > 0 ? o.restart : std::min(2000, 3 * (int)std::ceil(k) + 30);
        h->max_outer = o.max_outer > 0 ? o.max_outer : 4 * h->restart;
        // Richardson keeps one residual and one correction per column
        if (o.outer == HELM_OUTER_RICHARDSON) {
            h->max_outer = o.max_outer > 0 ? o.max_outer
                                           : 4 * std::min(2000, 3 * (int)std::ceil(k) + 30);
            h->restart = 1;
        }
        for (int l = 0; l < h->levels; ++l) {
            const int nl = h->n >> l;
            long long Nl = 1;
            for (int d = 0; d < h->dim; ++d) Nl *= (nl + 1);
            h->nl.push_back(nl);
            h->Nl.push_back(Nl);
        }
        h->mixed = mixed;
        h->dir = dirm;
        h->nv = h->Nl[0] + (mixed ? 4LL * h->n * h->n : 0);
        // coarsest-mesh dense L (from the same stencil rows the kernels use);
        // the W variant smooths on the coarsest mesh instead
        const int ncs = h->nl.back();
        const int nc = (int)h->Nl.back();
        h->nc = nc;
        if (!wvar) {
        std::vector<zd> A((size_t)nc * nc, zd(0.0));
        const Coef cf = h->coef(HELM_OP_L);
        if (h->dim == 2) {
            const Op2<double> op = make_op2<double>(cf, ncs, h->omega);
            const int np = ncs + 1;
            const int di[7] = {0, 1, -1, 0, 0, 1, -1}, dj[7] = {0, 0, 0, 1, -1, 1, -1};
            for (int j = 0; j <= ncs; ++j)
                for (int i = 0; i <= ncs; ++i) {
                    Row7<double> r = row_weights(op, i, j);
                    for (int q = 0; q < 7; ++q) {
                        const int ii = i + di[q], jj = j + dj[q];
                        if (ii < 0 || ii > ncs || jj < 0 || jj > ncs) continue;
                        A[(size_t)(i + np * j) * nc + (ii + np * jj)] += zd(r.w[q].x, r.w[q].y);
                    }
                }
        } else {
            const Op3<double> op = make_op3<double>(cf, ncs, h->omega);
            const int np = ncs + 1;
            for (int l = 0; l <= ncs; ++l)
                for (int j = 0; j <= ncs; ++j)
                    for (int i = 0; i <= ncs; ++i) {
                        const Line3<double> fx = line_factors<double>(i, ncs, op.h);
                        const Line3<double> fy = line_factors<double>(j, ncs, op.h);
                        const Line3<double> fz = line_factors<double>(l, ncs, op.h);
                        for (int dz = -1; dz <= 1; ++dz)
                            for (int dy = -1; dy <= 1; ++dy)
                                for (int dx = -1; dx <= 1; ++dx) {
                                    const int ii = i + dx, jj = j + dy, ll = l + dz;
                                    if (ii < 0 || ii > ncs || jj < 0 || jj > ncs || ll < 0 || ll > ncs)
                                        continue;
                                    const cxd w = weight3(op, fx, fy, fz, dx, dy, dz);
                                    A[(size_t)(i + np * (j + np * l)) * nc + (ii + np * (jj + np * ll))] +=
                                        zd(w.x, w.y);
                                }
                    }
        }
        // Dirichlet nodes: identity rows and columns (not unknowns)
        if (h->dir) {
            const int np = ncs + 1;
            for (int q = 0; q < nc; ++q) {
                const int c[3] = {q % np, (q / np) % np, q / (np * np)};
                bool on = false;
                for (int ax = 0; ax < h->dim; ++ax)
                    on = on || (c[ax] == 0 && ((h->dir >> (2 * ax)) & 1u)) ||
                         (c[ax] == ncs && ((h->dir >> (2 * ax + 1)) & 1u));
                if (!on) continue;
                for (int r = 0; r < nc; ++r) {
                    A[(size_t)q * nc + r] = zd(0.0);
                    A[(size_t)r * nc + q] = zd(0.0);
                }
                A[(size_t)q * nc + q] = zd(1.0);
            }
        }
        if (!invert_dense(A, nc)) {
            g_last_error = "singular coarsest-mesh operator";
            delete h;
            return HELM_EINVAL;
        }
        std::vector<cxd> Ah((size_t)nc * nc);
        for (size_t q = 0; q < Ah.size(); ++q) Ah[q] = mk(A[q].real(), A[q].imag());
        if (hipMalloc(&h->d_cinv, sizeof(cxd) * Ah.size()) != hipSuccess) {
            delete h;
            return HELM_ENOMEM;
        }
        HIPCHK(hipMemcpy(h->d_cinv, Ah.data(), sizeof(cxd) * Ah.size(), hipMemcpyHostToDevice));
        }
        // private stream used only to capture the preconditioner graph, and
        // the stream of the second slot group
        HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        HIPCHK(hipStreamCreateWithFlags(&h->aux_stream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
    } catch (const DevErr&) {
        release_handle_objects(h);
        delete h;
        return HELM_EDEVICE;
    } catch (const std::bad_alloc&) {
        release_handle_objects(h);
        delete h;
        return HELM_ENOMEM;
    }
    *out = h;
    return HELM_OK;
}

int helm_destroy(helm_t* h) {
    if (!h) return HELM_OK;
    int rc = HELM_OK;
    if (hipStreamSynchronize(h->stream) != hipSuccess) rc = HELM_EDEVICE;
    if (h->aux_stream && hipStreamSynchronize(h->aux_stream) != hipSuccess) rc = HELM_EDEVICE;
    if (h->d_cinv && hipFree(h->d_cinv) != hipSuccess) rc = HELM_EDEVICE;
    h->d_cinv = nullptr;
    for (hipEvent_t e : h->prof_ev) (void)hipEventDestroy(e);
    for (auto& g : h->graphs) {
        (void)hipGraphExecDestroy(g.head);
        if (g.body) (void)hipGraphExecDestroy(g.body);
    }
    release_handle_objects(h);
    delete h;
    return rc;
}

long long helm_vector_length(const helm_t* h) { return h ? h->nv : -1; }

long long helm_nodes(const helm_t* h, int level) {
    if (!h || level < 0 || level >= h->levels) return -1;
    return h->Nl[level];
}

int helm_workspace_bytes(const helm_t* h, int nrhs, size_t* bytes) {
    if (!h || !bytes || nrhs < 1) return HELM_EINVAL;
    *bytes = layout(h, nrhs).total;
    return HELM_OK;
}

int helm_solve(helm_t* h, const void* rhs, void* x, int nrhs, double tol, void* workspace,
               helm_stats* stats) {
    if (!h || !rhs || !x || !workspace || nrhs < 1) return HELM_EINVAL;
    if (!(tol > 0.0 && tol < 1.0)) return HELM_EINVAL;
    try {
        if (h->opts.outer == HELM_OUTER_RICHARDSON) {
            if (h->prec == HELM_FP64)
                return richardson_columns<double>(h, static_cast<const cxd*>(rhs),
                                                  static_cast<cxd*>(x), nrhs, tol, workspace, stats);
            return richardson_columns<float>(h, static_cast<const cxd*>(rhs), static_cast<cxd*>(x),
                                             nrhs, tol, workspace, stats);
        }
        if (h->prec == HELM_FP64)
            return solve_columns<double>(h, static_cast<const cxd*>(rhs), static_cast<cxd*>(x),
                                         nrhs, tol, workspace, stats);
        return solve_columns<float>(h, static_cast<const cxd*>(rhs), static_cast<cxd*>(x), nrhs,
                                    tol, workspace, stats);
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    } catch (const std::bad_alloc&) {
        return HELM_ENOMEM;
    }
}

int helm_load_nodal(helm_t* h, const double* f_nodal, void* b, int nrhs) {
    if (!h || !f_nodal || !b || nrhs < 1) return HELM_EINVAL;
    const long long N = h->Nl[0];
    cxd* tmp = nullptr;
    try {
        HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&tmp), sizeof(cxd) * N * nrhs, h->stream));
        real_to_complex(h->stream, N, f_nodal, tmp, nrhs);
        if (h->mixed) {
            // F_u = M f / (delta - ik), F_sigma = 0 (the mixed right-hand side of Sec. 2)
            const long long Nv = h->nv;
            cxd* bp = static_cast<cxd*>(b);
            const Coef cf{0.0, 1.0 / zd(h->delta, -h->k), 0.0};
            stencil2d<double, double>(h->stream, make_op2<double>(cf, h->n, h->omega), MODE_APPLY, 1.0,
                                      Vec<const cxd>{tmp, N, 0, nullptr}, Vec<const cxd>{},
                                      Vec<cxd>{bp, Nv, 0, nullptr}, nrhs);
            for (int c = 0; c < nrhs; ++c) zero<double>(h->stream, bp + (long long)c * Nv + N, Nv - N);
        } else
        apply_mode<double>(h, HELM_OP_M, 0, MODE_APPLY, 1.0, Vec<const cxd>{tmp, N, 0, nullptr},
                           Vec<const cxd>{}, Vec<cxd>{static_cast<cxd*>(b), N, 0, nullptr}, nrhs);
        HIPCHK(hipFreeAsync(tmp, h->stream));
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

#define PREC_DISPATCH(prec, CALL_D, CALL_F) \
    ((prec) == HELM_FP64 ? (CALL_D) : (CALL_F))

int helm_apply(helm_t* h, int op, int level, int prec, const void* x, void* y, int nrhs) {
    if (!h || !x || !y || nrhs < 1 || level < 0 || level >= h->levels) return HELM_EINVAL;
    if (op == HELM_OP_MIXED || op == HELM_OP_MIXED_SHIFT) {
        if (!h->mixed || level != 0 || prec != HELM_FP64) return HELM_EINVAL;
        const long long Nv = h->nv;
        try {
            mixed_system<double>(h, op == HELM_OP_MIXED ? h->delta : h->dh, MODE_APPLY,
                         Vec<const cxd>{static_cast<const cxd*>(x), Nv, 0, nullptr}, Vec<const cxd>{},
                         Vec<cxd>{static_cast<cxd*>(y), Nv, 0, nullptr}, nrhs);
            HIPCHK(hipGetLastError());
        } catch (const DevErr&) {
            return HELM_EDEVICE;
        }
        return HELM_OK;
    }
    if (op < HELM_OP_B0 || op > HELM_OP_M) return HELM_EINVAL;
    if (prec != HELM_FP64 && prec != HELM_FP32_MG) return HELM_EINVAL;
    const long long N = h->Nl[level];
    try {
        if (prec == HELM_FP64)
            apply_mode<double>(h, op, level, MODE_APPLY, 1.0,
                               Vec<const cxd>{static_cast<const cxd*>(x), N, 0, nullptr},
                               Vec<const cxd>{}, Vec<cxd>{static_cast<cxd*>(y), N, 0, nullptr}, nrhs);
        else
            apply_mode<float>(h, op, level, MODE_APPLY, 1.0f,
                              Vec<const cxf>{static_cast<const cxf*>(x), N, 0, nullptr},
                              Vec<const cxf>{}, Vec<cxf>{static_cast<cxf*>(y), N, 0, nullptr}, nrhs);
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

extern "C++" {
template <typename T>
static void hss_residual_t(helm_t* h, const void* R, const void* u, void* rho, int nrhs) {
    const long long N = h->Nl[0];
    const T c = (T)(2.0 * h->k / (h->k + 1.0));
    Vec<const cx<T>> Rv{static_cast<const cx<T>*>(R), N, 0, nullptr};
    Vec<cx<T>> out{static_cast<cx<T>*>(rho), N, 0, nullptr};
    if (u) {
        apply_mode<T>(h, HELM_OP_BSHIFT, 0, MODE_RESID, c,
                      Vec<const cx<T>>{static_cast<const cx<T>*>(u), N, 0, nullptr}, Rv, out, nrhs);
    } else {
        // u = 0: rho = c R, through the residual kernel on a zero vector
        cx<T>* tmp = nullptr;
        HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&tmp), sizeof(cx<T>) * N * nrhs, h->stream));
        zero<T>(h->stream, tmp, N * nrhs);
        apply_mode<T>(h, HELM_OP_BSHIFT, 0, MODE_RESID, c, Vec<const cx<T>>{tmp, N, 0, nullptr}, Rv,
                      out, nrhs);
        HIPCHK(hipFreeAsync(tmp, h->stream));
    }
}
}  // extern "C++"

int helm_hss_residual(helm_t* h, int prec, const void* R, const void* u, void* rho, int nrhs) {
    if (!h || !R || !rho || nrhs < 1) return HELM_EINVAL;
    if (prec != HELM_FP64 && prec != HELM_FP32_MG) return HELM_EINVAL;
    try {
        if (prec == HELM_FP64) hss_residual_t<double>(h, R, u, rho, nrhs);
        else hss_residual_t<float>(h, R, u, rho, nrhs);
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

int helm_jacobi(helm_t* h, int level, int prec, const void* x_in, const void* b, void* x_out,
                int nrhs) {
    if (!h || !b || !x_out || nrhs < 1 || level < 0 || level >= h->levels) return HELM_EINVAL;
    if (prec != HELM_FP64 && prec != HELM_FP32_MG) return HELM_EINVAL;
    if (x_out == x_in || x_out == b) return HELM_EINVAL;
    const long long N = h->Nl[level];
    const int mode = x_in ? MODE_JACOBI : MODE_JACOBI0;
    try {
        if (prec == HELM_FP64)
            apply_mode<double>(h, HELM_OP_L, level, mode, 1.0,
                               Vec<const cxd>{static_cast<const cxd*>(x_in), N, 0, nullptr},
                               Vec<const cxd>{static_cast<const cxd*>(b), N, 0, nullptr},
                               Vec<cxd>{static_cast<cxd*>(x_out), N, 0, nullptr}, nrhs);
        else
            apply_mode<float>(h, HELM_OP_L, level, mode, 1.0f,
                              Vec<const cxf>{static_cast<const cxf*>(x_in), N, 0, nullptr},
                              Vec<const cxf>{static_cast<const cxf*>(b), N, 0, nullptr},
                              Vec<cxf>{static_cast<cxf*>(x_out), N, 0, nullptr}, nrhs);
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

extern "C++" {
template <typename T>
static void restrict_t(helm_t* h, int level, const void* x, const void* b, void* bc, int nrhs) {
    const long long N = h->Nl[level], Nc = h->Nl[level + 1];
    cx<T>* tmp = nullptr;
    if (h->dim == 3 || h->dir)
        HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&tmp), sizeof(cx<T>) * N * nrhs, h->stream));
    resid_restrict<T>(h, level, Vec<const cx<T>>{static_cast<const cx<T>*>(x), N, 0, nullptr},
                      Vec<const cx<T>>{static_cast<const cx<T>*>(b), N, 0, nullptr},
                      Vec<cx<T>>{static_cast<cx<T>*>(bc), Nc, 0, nullptr},
                      Vec<cx<T>>{tmp, N, 0, nullptr}, nrhs);
    if (tmp) HIPCHK(hipFreeAsync(tmp, h->stream));
}
}  // extern "C++"

int helm_restrict_residual(helm_t* h, int level, int prec, const void* x, const void* b,
                           void* b_coarse, int nrhs) {
    if (!h || !x || !b || !b_coarse || nrhs < 1 || level < 0 || level >= h->levels - 1)
        return HELM_EINVAL;
    if (prec != HELM_FP64 && prec != HELM_FP32_MG) return HELM_EINVAL;
    try {
        if (prec == HELM_FP64) restrict_t<double>(h, level, x, b, b_coarse, nrhs);
        else restrict_t<float>(h, level, x, b, b_coarse, nrhs);
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

int helm_prolong_correct(helm_t* h, int level, int prec, const void* e_coarse, void* x, int nrhs) {
    if (!h || !e_coarse || !x || nrhs < 1 || level < 0 || level >= h->levels - 1) return HELM_EINVAL;
    if (prec != HELM_FP64 && prec != HELM_FP32_MG) return HELM_EINVAL;
    const long long N = h->Nl[level], Nc = h->Nl[level + 1];
    try {
        if (prec == HELM_FP64)
            prolong<double>(h, level, Vec<const cxd>{static_cast<const cxd*>(e_coarse), Nc, 0, nullptr},
                            Vec<cxd>{static_cast<cxd*>(x), N, 0, nullptr}, nrhs);
        else
            prolong<float>(h, level, Vec<const cxf>{static_cast<const cxf*>(e_coarse), Nc, 0, nullptr},
                           Vec<cxf>{static_cast<cxf*>(x), N, 0, nullptr}, nrhs);
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

int helm_coarse_solve(helm_t* h, int prec, const void* b, void* x, int nrhs) {
    if (!h || !b || !x || nrhs < 1) return HELM_EINVAL;
    if (prec != HELM_FP64 && prec != HELM_FP32_MG) return HELM_EINVAL;
    if (!h->d_cinv) return HELM_ENOTSUP;  // the W variant has no coarse factorisation
    const long long Nc = h->Nl.back();
    try {
        const int lc = h->levels - 1;
        if (prec == HELM_FP64) {
            Vec<cxd> xv{static_cast<cxd*>(x), Nc, 0, nullptr};
            coarse_apply<double>(h->stream, h->d_cinv, h->nc,
                                 Vec<const cxd>{static_cast<const cxd*>(b), Nc, 0, nullptr}, xv, nrhs);
            dir_mask<double>(h, h->stream, lc, xv, nrhs);
        } else {
            Vec<cxf> xv{static_cast<cxf*>(x), Nc, 0, nullptr};
            coarse_apply<float>(h->stream, h->d_cinv, h->nc,
                                Vec<const cxf>{static_cast<const cxf*>(b), Nc, 0, nullptr}, xv, nrhs);
            dir_mask<float>(h, h->stream, lc, xv, nrhs);
        }
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

int helm_vcycle(helm_t* h, int prec, const void* b, void* x, int nrhs, void* workspace) {
    if (!h || !b || !x || !workspace || nrhs < 1) return HELM_EINVAL;
    if (prec != HELM_FP64 && prec != HELM_FP32_MG) return HELM_EINVAL;
    if (prec != h->prec) return HELM_EINVAL;  // workspace is laid out for the handle's mode
    const long long N = h->Nl[0];
    const Layout Lw = layout(h, nrhs);
    try {
        (void)N;
        if (prec == HELM_FP64) vcycle_entry<double>(h, Lw, workspace, b, x, nrhs);
        else vcycle_entry<float>(h, Lw, workspace, b, x, nrhs);
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

int helm_precondition(helm_t* h, const void* v, void* z, int nrhs, void* workspace) {
    if (!h || !v || !z || !workspace || nrhs < 1) return HELM_EINVAL;
    const long long N = h->nv;
    const Layout Lw = layout(h, nrhs);
    try {
        Vec<const cxd> vv{static_cast<const cxd*>(v), N, 0, nullptr};
        if (h->prec == HELM_FP64) {
            ensure_cycles<double>(h, Lw, workspace);
            precondition<double>(h, Lw, workspace, vv, Vec<cxd>{static_cast<cxd*>(z), N, 0, nullptr},
                                 nrhs);
        } else {
            ensure_cycles<float>(h, Lw, workspace);
            precondition<float>(h, Lw, workspace, vv, at_ws<cxf>(workspace, Lw.Z, N), nrhs);
            copy_cast<double, float>(h->stream, N, cst(at_ws<cxf>(workspace, Lw.Z, N)),
                                     Vec<cxd>{static_cast<cxd*>(z), N, 0, nullptr}, nrhs);
        }
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

int helm_hss_history(helm_t* h, const void* v, void* z, int nrhs, void* workspace, double* res) {
    if (!h || !v || !z || !workspace || !res || nrhs < 1) return HELM_EINVAL;
    const long long N = h->nv;
    const Layout Lw = layout(h, nrhs);
    const cxd* vp = static_cast<const cxd*>(v);
    try {
        if (h->prec == HELM_FP64) {
            ensure_cycles<double>(h, Lw, workspace);
            hss_history<double>(h, Lw, workspace, vp, Vec<cxd>{static_cast<cxd*>(z), N, 0, nullptr},
                                nrhs, res);
        } else {
            ensure_cycles<float>(h, Lw, workspace);
            hss_history<float>(h, Lw, workspace, vp, at_ws<cxf>(workspace, Lw.Z, N), nrhs, res);
            copy_cast<double, float>(h->stream, N, cst(at_ws<cxf>(workspace, Lw.Z, N)),
                                     Vec<cxd>{static_cast<cxd*>(z), N, 0, nullptr}, nrhs);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->stream));
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

}  // extern "C"

// ------------------------------------------------- cycle without allocation --
// helm_vcycle_noalloc keeps the cycle's level vectors in this file-scope
// device array instead of a caller workspace.  Every device the call runs on
// holds its own copy, at its own address, until the process ends; in host
// code the name is only a stand-in, so the address is looked up once per
// device and that pointer is what the kernels receive.
static __device__ __align__(256) unsigned char scratch[HELM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_SCRATCH_DEVICES] = {};

// device address of `scratch` on device dev (current on the calling thread)
void* scratch_on(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// the level vectors one cycle on level 0 uses: level 0's second buffer t,
// then b, x and t of every coarser level (the same roles as in layout())
Layout layout_cycle(const helm_t* h, int nrhs) {
    Layout L{};
    L.cap = nrhs;
    size_t off = 0;
    const size_t smg = h->prec == HELM_FP64 ? sizeof(cxd) : sizeof(cxf);
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += up(bytes);
        return o;
    };
    L.mg_t[0] = take(smg * nrhs * h->Nl[0]);
    for (int l = 1; l < h->levels; ++l) {
        L.mg_b[l] = take(smg * nrhs * h->Nl[l]);
        L.mg_x[l] = take(smg * nrhs * h->Nl[l]);
        L.mg_t[l] = take(smg * nrhs * h->Nl[l]);
    }
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

int helm_vcycle_noalloc(helm_t* h, int prec, const void* b, void* x, int nrhs) {
    if (!h || !b || !x || nrhs < 1) return HELM_EINVAL;
    if (prec != HELM_FP64 && prec != HELM_FP32_MG) return HELM_EINVAL;
    if (prec != h->prec) return HELM_EINVAL;
    if (w_variant(h)) return HELM_ENOTSUP;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        g_last_error = "hipGetDevice failed";
        return HELM_EDEVICE;
    }
    if (dev != h->device) {
        g_last_error = "helm_vcycle_noalloc: the current device is not the handle's device";
        return HELM_EINVAL;
    }
    if (dev < 0 || dev >= MAX_SCRATCH_DEVICES) return HELM_ENOTSUP;
    const Layout Lw = layout_cycle(h, nrhs);
    if (Lw.total > HELM_NOALLOC_SCRATCH_BYTES) {
        g_last_error = "helm_vcycle_noalloc: " + std::to_string(nrhs) + " column(s) on this mesh need " +
                       std::to_string(Lw.total) + " bytes of scratch; the library holds " +
                       std::to_string((size_t)HELM_NOALLOC_SCRATCH_BYTES) + " per device";
        return HELM_EINVAL;
    }
    // no segment-height timing on this path (it would create events)
    struct Tuning {
        bool was;
        ~Tuning() { (void)stream_tuning(was); }
    } tuning{stream_tuning(false)};
    try {
        void* ws = scratch_on(dev);
        if (prec == HELM_FP64) vcycle_entry<double>(h, Lw, ws, b, x, nrhs);
        else vcycle_entry<float>(h, Lw, ws, b, x, nrhs);
        HIPCHK(hipGetLastError());
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    }
    return HELM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ serving --
#include "server_impl.h"
