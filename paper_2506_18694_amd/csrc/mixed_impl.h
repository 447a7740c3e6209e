// The mixed formulation ([DG0]^2 x P1, 2D) on the host: the mixed operator
// and the sigma-eliminated HSS step (included by helm_api.cpp inside its
// internal namespace).
#pragma once

// Y = A_delta X (MODE_APPLY) or Y = B - A_delta X (MODE_RESID) for mixed
// vectors [u | sigma]: u rows (delta - ik) M u + M_Gamma u + G^T sigma,
// sigma rows (delta - ik) M_s sigma - G u.  FP64 arithmetic; X in FP64 or
// in the preconditioner's FP32 storage.
template <typename TI>
void mixed_system(helm_t* h, double delta, int mode, Vec<const cx<TI>> X, Vec<const cxd> B,
                  Vec<cxd> Y, int ns) {
    const zd s(delta, -h->k);
    const double sg = mode == MODE_RESID ? -1.0 : 1.0;
    const Op2<double> op = make_op2<double>(Coef{0.0, sg * s, sg}, h->n, h->omega);
    mixed_nodes<double, TI>(h->stream, op, mk(1.0, 0.0), mk(sg, 0.0), mk(0.0, 0.0), X,
                            mode == MODE_RESID ? B : Vec<const cxd>{}, Vec<const cxd>{}, Y, ns);
    mixed_tris<double, TI>(h->stream, h->n, mode, mk(s.real(), s.imag()), X, B, Y, ns);
}

// One HSS step of the mixed shifted-HSS preconditioner with sigma
// eliminated (correction form for u): with nu = (k-1)/(k+1), c = 2k/(k+1),
// g = nu (k(dh+i) sigma + grad u) + c M_s^{-1} R_sigma (per triangle),
// rho = k(dh-i) [nu (k(dh+i) M u - G^T sigma + k M_Gamma u) + c R_u]
//       - G^T g - Lmix u,
// e = q V-cycles on Lmix e = rho (the streaming kernels of the primal
// form, whose operator differs only in its coefficients), u += e,
// sigma = (grad u + g) / (k(dh-i)).
template <typename T>
void hss_step_mixed(helm_t* h, const Layout& Lw, void* ws, int ns, int s) {
    const long long N = h->Nl[0], Nv = h->nv;
    const double k = h->k;
    Vec<cx<T>> U = at_ws<cx<T>>(ws, Lw.u, Nv);
    Vec<cx<T>> R = at_ws<cx<T>>(ws, Lw.R, Nv);
    Vec<cx<T>> G = at_ws<cx<T>>(ws, Lw.mg, Nv - N);
    Vec<cx<T>> rho = at_ws<cx<T>>(ws, Lw.mg_b[0], N);
    Vec<cx<T>> e = at_ws<cx<T>>(ws, Lw.mg_x[0], N);
    Vec<cx<T>> t = at_ws<cx<T>>(ws, Lw.mg_t[0], N);
    const double nu = (k - 1.0) / (k + 1.0), c = 2.0 * k / (k + 1.0);
    const zd kp = k * zd(h->dh, 1.0), km = k * zd(h->dh, -1.0);
    if (s == 0) zero<T>(h->stream, U.base, Nv * ns);
    mixed_g<T>(h->stream, h->n, tocx<T>(nu * kp), (T)nu, (T)c, cst(U), cst(R), G, ns);
    // k(dh-i) nu (k(dh+i) M + k M_Gamma) - Lmix as one stencil
    const Coef lm = h->coef(HELM_OP_L);
    const Coef comb{-lm.a, km * nu * kp - lm.b, km * nu * k - lm.c};
    const zd sa = -km * nu, sb = km * c;
    mixed_nodes<T, T>(h->stream, make_op2<T>(comb, h->n, h->omega), tocx<T>(sb), tocx<T>(sa),
                      mk((T)-1, (T)0), cst(U), cst(R), cst(G), rho, ns);
    // q cycles x <- x + V(rho - Lmix x) from x = 0, each added into u as it
    // comes: a zero-guess cycle with the streaming kernels on the current
    // residual, whose update rho - Lmix d is formed out of place; the
    // residual, the cycle's result and its scratch rotate through the three
    // level-0 buffers
    Vec<cx<T>> buf[3] = {rho, e, t};
    int ib = 0;  // the buffer holding the current residual
    for (int q = 0; q < h->cycles; ++q) {
        const int i1 = (ib + 1) % 3, i2 = (ib + 2) % 3;
        const Vec<cx<T>> d = vcycle2d_zero<T>(h, Lw, ws, 0, cst(buf[ib]), buf[i1], buf[i2], ns);
        axpy1<T>(h->stream, N, (T)1, cst(d), U, ns);
        if (q + 1 < h->cycles) {
            const int id = d.base == buf[i1].base ? i1 : i2;
            const int in = 3 - ib - id;
            apply_mode<T>(h, HELM_OP_L, 0, MODE_RESID, (T)1, cst(d), cst(buf[ib]), buf[in], ns);
            ib = in;
        }
    }
    mixed_sigma<T>(h->stream, h->n, tocx<T>(1.0 / km), cst(U), cst(G), U, ns);
}
