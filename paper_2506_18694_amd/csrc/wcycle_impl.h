// The paper's multigrid variant (Sec. 5.3) on the host: Jacobi-preconditioned
// GMRES smoothing, the W-cycle and the HSS step that uses it (included by
// helm_api.cpp inside its internal namespace).
#pragma once

// y = D^{-1} (b - L x) (MODE_PRES; X null means x = 0) or y = D^{-1} L x
// (MODE_PAPPLY) on level l in FP64: the Jacobi factors with omega = 1.
void pmode(helm_t* h, int l, int mode, Vec<const cxd> X, Vec<const cxd> B, Vec<cxd> Y, int ns) {
    const Coef cf = h->coef(HELM_OP_L);
    if (h->dim == 2)
        stencil2d<double, double>(h->stream, make_op2<double>(cf, h->nl[l], 1.0), mode, 1.0, X, B, Y, ns);
    else
        stencil3d<double, double>(h->stream, make_op3<double>(cf, h->nl[l], 1.0), mode, 1.0, X, B, Y, ns,
                                  false);
}

// m = smooth_its iterations of Jacobi-left-preconditioned GMRES for
// L x = b on level l, from the current x (guess) or from x = 0: the
// Krylov basis of D^{-1} L from r = D^{-1}(b - L x) by Arnoldi with
// classical Gram-Schmidt applied twice, the (m+1) x m least-squares
// problem solved on the device, x += V y.  Every column works in its own
// slot; nothing is read back to the host.
void gmres_smooth(helm_t* h, const Layout& Lw, void* ws, int l, Vec<const cxd> b, Vec<cxd> x,
                  bool guess, int ns) {
    hipStream_t st = h->stream;
    const int m = h->smooth_its;
    const long long N = h->Nl[l];
    char* w = static_cast<char*>(ws);
    cxd* G = reinterpret_cast<cxd*>(w + Lw.gk[l]);
    cxd* hu = reinterpret_cast<cxd*>(w + Lw.ghu);
    cxd* hu2 = reinterpret_cast<cxd*>(w + Lw.ghu2);
    double* hn = reinterpret_cast<double*>(w + Lw.gn);
    cxd* gy = reinterpret_cast<cxd*>(w + Lw.gy);
    cxd* part = reinterpret_cast<cxd*>(w + Lw.gpart);
    double* npart = reinterpret_cast<double*>(w + Lw.gnpart);
    const long long cs = (long long)(m + 1) * N;  // slot stride of the basis
    const int hs = m * (m + 1);                    // slot stride of the Hessenberg
    const int nblk = multidot_blocks(N);
    auto basis = [&](int i) { return Vec<cxd>{G + (long long)i * N, cs, 0, nullptr}; };
    const Vec<const cxd> V{G, cs, 0, nullptr};
    if (!guess) zero<double>(st, x.base, N * ns);
    pmode(h, l, MODE_PRES, guess ? cst(x) : Vec<const cxd>{}, b, basis(0), ns);
    norm2(st, N, cst(basis(0)), npart, hn, m + 1, ns);
    scale_inv(st, N, cst(basis(0)), basis(0), hn, m + 1, ns);
    for (int j = 0; j < m; ++j) {
        const Vec<cxd> wv = basis(j + 1);
        cxd* hcol = hu + (long long)j * (m + 1);
        pmode(h, l, MODE_PAPPLY, cst(basis(j)), Vec<const cxd>{}, wv, ns);
        for (int pass = 0; pass < 2; ++pass) {
            multidot(st, N, j + 1, nullptr, V, cst(wv), part, ns);
            if (pass == 0) {
                reduce_parts(st, j + 1, nullptr, nblk, part, hcol, hs, 0, ns);
                multi_axpy(st, N, j + 1, nullptr, V, hcol, hs, wv, ns);
            } else {
                reduce_parts(st, j + 1, nullptr, nblk, part, hu2, m + 1, 0, ns);
                reduce_parts(st, j + 1, nullptr, nblk, part, hcol, hs, 1, ns);
                multi_axpy(st, N, j + 1, nullptr, V, hu2, m + 1, wv, ns);
            }
        }
        norm2(st, N, cst(wv), npart, hn + j + 1, m + 1, ns);
        scale_inv(st, N, cst(wv), wv, hn + j + 1, m + 1, ns);
    }
    gmres_lsq(st, m, hu, hs, hn, gy, ns);
    update_solution<double>(st, N, m, nullptr, V, gy, m, x, ns);
}

// One W-cycle for L_l x = b from x (guess) or 0: smoothing, residual
// restriction, two cycles on the coarse equation (the second from the
// first's result), prolongation and correction, smoothing; the coarsest
// level smooths once.
void wcycle_gm(helm_t* h, const Layout& Lw, void* ws, int l, Vec<const cxd> b, Vec<cxd> x, bool guess,
               int ns) {
    gmres_smooth(h, Lw, ws, l, b, x, guess, ns);
    if (l == h->levels - 1) return;
    const long long N1 = h->Nl[l + 1];
    Vec<cxd> bc = at_ws<cxd>(ws, Lw.mg_b[l + 1], N1);
    Vec<cxd> xc = at_ws<cxd>(ws, Lw.mg_x[l + 1], N1);
    resid_restrict<double>(h, l, cst(x), b, bc, at_ws<cxd>(ws, Lw.mg_t[l], h->Nl[l]), ns);
    wcycle_gm(h, Lw, ws, l + 1, cst(bc), xc, false, ns);
    wcycle_gm(h, Lw, ws, l + 1, cst(bc), xc, true, ns);
    prolong<double>(h, l, cst(xc), x, ns);
    gmres_smooth(h, Lw, ws, l, b, x, true, ns);
}

// One shifted-HSS step with the W variant: rho = c (R - B u), `cycles`
// W-cycles (each after the first from the previous iterate), u += e.
void hss_step_w(helm_t* h, const Layout& Lw, void* ws, int ns, int s) {
    const long long N = h->Nl[0];
    Vec<cxd> R = at_ws<cxd>(ws, Lw.R, N);
    Vec<cxd> u = at_ws<cxd>(ws, Lw.u, N);
    Vec<cxd> rho = at_ws<cxd>(ws, Lw.mg_b[0], N);
    Vec<cxd> e = at_ws<cxd>(ws, Lw.mg_x[0], N);
    const double c = 2.0 * h->k / (h->k + 1.0);
    if (s == 0) zero<double>(h->stream, u.base, N * ns);
    apply_mode<double>(h, HELM_OP_BSHIFT, 0, MODE_RESID, c, cst(u), cst(R), rho, ns);
    for (int q = 0; q < h->cycles; ++q) wcycle_gm(h, Lw, ws, 0, cst(rho), e, q > 0, ns);
    axpy1<double>(h->stream, N, 1.0, cst(e), u, ns);
}

inline bool w_variant(const helm_t* h) { return h->opts.cycle == HELM_CYCLE_W_GMRES; }
