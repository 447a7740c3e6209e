// Column-wise flexible GMRES engine (included by helm_api.cpp only).
//
// Each right-hand side ("column") owns a workspace slot c with its own
// Krylov basis V[c], preconditioned directions Z[c], load vector B[c] and
// iterate X[c], and its own Krylov index j.  One step advances every active
// column by one FGMRES iteration (Saad's right-preconditioned flexible
// GMRES, Sec. 5.1's outer method), batching the device work of all columns
// into the same launches:
//   1. columns starting (or restarting) a cycle: r = b - B X, beta = |r|,
//      V[c][0] = r / beta; columns waiting for their final check: |b - B X|;
//   2. all iterating columns: z = B~^{-1} V[c][j] (the shifted-HSS
//      preconditioner, one batched launch sequence), w = B z, classical
//      Gram-Schmidt against V[c][0..j], repeated once for the columns whose
//      first pass cancelled most of w (Kahan's "twice is enough" test,
//      taken on the device), h_{j+1,j} = |w|, V[c][j+1] = w / h_{j+1,j};
//   3. one device->host copy of the new Hessenberg columns and norms.
// The host then applies the Givens rotations per column and decides:
// converged or out of iterations -> X[c] += Z[c] y and a true-residual
// check next step; basis full -> X[c] += Z[c] y and restart; else continue.
// Columns may be added between steps (continuous batching); a column's
// arithmetic does not depend on which other columns share its launches.
#pragma once

enum ColPhase { COL_FREE = 0, COL_FRESH, COL_ACTIVE, COL_CHECK, COL_DONE };

struct Column {
    int phase = COL_FREE;
    long long tag = -1;  // owner (request id) for the server, or the column index
    int j = 0, its = 0, restarts = 0;
    bool have_bnorm = false, converged = false;
    double bnorm = 0.0, beta = 0.0, est = 1.0, true_rel = -1.0;
    double r0 = -1.0;   // true residual norm before the first iteration
    double tol = 1e-8;  // relative residual target of this column
    std::vector<zd> H, cs, sn, g;  // Hessenberg (column-major, ld R+1), rotations, rhs
};

template <typename T>
struct Engine {
    helm_t* h = nullptr;
    char* ws = nullptr;
    Layout Lw{};
    int cap = 0, R = 0;
    long long N = 0;
    double tol = 1e-8;
    hipStream_t s = nullptr;
    std::vector<Column> col;
    // pinned host staging
    int* hmap = nullptr;     // NMAPS * cap (step maps)
    int* hfin = nullptr;     // NMAPS * cap (finishing maps)
    cxd* hh = nullptr;       // 2 * cap * (R + 1)
    double* hn = nullptr;    // 3 * cap
    int* hflag = nullptr;    // cap (second Gram-Schmidt pass taken)
    cxd* hy = nullptr;       // cap * R
    hipEvent_t ev = nullptr;
    // the last enqueued step
    std::vector<int> it_cols, chk_cols, fresh_cols;
    bool pending = false;
    double precond_ms = 0.0;
    long long vcycles = 0, reorth = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;

    // device views
    int* d_maps() const { return reinterpret_cast<int*>(ws + Lw.maps); }
    cxd* d_h() const { return reinterpret_cast<cxd*>(ws + Lw.dh); }
    cxd* d_h2() const { return reinterpret_cast<cxd*>(ws + Lw.dh2); }
    double* d_norm() const { return reinterpret_cast<double*>(ws + Lw.dnorm); }
    cxd* d_part() const { return reinterpret_cast<cxd*>(ws + Lw.part); }
    double* d_npart() const { return reinterpret_cast<double*>(ws + Lw.npart); }
    int* d_flag() const { return reinterpret_cast<int*>(ws + Lw.flag); }
    cxd* d_y() const { return reinterpret_cast<cxd*>(ws + Lw.dy); }
    cxd* Vb() const { return reinterpret_cast<cxd*>(ws + Lw.V); }
    cx<T>* Zb() const { return reinterpret_cast<cx<T>*>(ws + Lw.Z); }
    cxd* Bb() const { return reinterpret_cast<cxd*>(ws + Lw.Bw); }
    cxd* Xb() const { return reinterpret_cast<cxd*>(ws + Lw.Xw); }

    void init(helm_t* hh_, void* ws_, int cap_, double tol_) {
        h = hh_;
        ws = static_cast<char*>(ws_);
        cap = cap_;
        R = h->restart;
        N = h->nv;  // column length (nodes, or nodes + triangle data when mixed)
        tol = tol_;
        s = h->stream;
        Lw = layout(h, cap);
        col.assign(cap, Column{});
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hmap), sizeof(int) * NMAPS * cap, 0));
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hfin), sizeof(int) * NMAPS * cap, 0));
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hh), sizeof(cxd) * 2 * cap * (R + 1), 0));
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hn), sizeof(double) * 3 * cap, 0));
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hflag), sizeof(int) * cap, 0));
        HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&hy), sizeof(cxd) * (size_t)cap * R, 0));
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
    }
    void release() {
        if (hmap) (void)hipHostFree(hmap);
        if (hfin) (void)hipHostFree(hfin);
        if (hh) (void)hipHostFree(hh);
        if (hn) (void)hipHostFree(hn);
        if (hflag) (void)hipHostFree(hflag);
        if (hy) (void)hipHostFree(hy);
        if (ev) (void)hipEventDestroy(ev);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        hmap = hfin = nullptr;
        hh = hy = nullptr;
        hn = nullptr;
        ev = e0 = e1 = nullptr;
    }

    int free_slots() const {
        int f = 0;
        for (const auto& c : col) f += c.phase == COL_FREE;
        return f;
    }
    bool busy() const {
        for (const auto& c : col)
            if (c.phase == COL_FRESH || c.phase == COL_ACTIVE || c.phase == COL_CHECK) return true;
        return false;
    }

    // Take a free slot for a new column: B[c] = rhs, X[c] = x0 (or 0).
    int admit(long long tag, const cxd* rhs, const cxd* x0, double ctol) {
        int c = -1;
        for (int q = 0; q < cap; ++q)
            if (col[q].phase == COL_FREE) { c = q; break; }
        if (c < 0) return -1;
        Column& C = col[c];
        C = Column{};
        C.tag = tag;
        C.tol = ctol;
        C.phase = COL_FRESH;
        C.H.assign((size_t)(R + 1) * R, zd(0.0));
        C.cs.assign(R, zd(0.0));
        C.sn.assign(R, zd(0.0));
        C.g.assign(R + 1, zd(0.0));
        HIPCHK(hipMemcpyAsync(Bb() + (long long)c * N, rhs, sizeof(cxd) * N, hipMemcpyDeviceToDevice, s));
        if (x0)
            HIPCHK(hipMemcpyAsync(Xb() + (long long)c * N, x0, sizeof(cxd) * N, hipMemcpyDeviceToDevice, s));
        else
            zero<double>(s, Xb() + (long long)c * N, N);
        // Dirichlet nodes are not unknowns: the rhs and guess are zero there
        if (h->dir && !h->mixed) {
            dir_mask<double>(h, s, 0, Vec<cxd>{Bb() + (long long)c * N, N, 0, nullptr}, 1);
            dir_mask<double>(h, s, 0, Vec<cxd>{Xb() + (long long)c * N, N, 0, nullptr}, 1);
        }
        return c;
    }

    void apply_B(int mode, Vec<const cxd> X, Vec<const cxd> Bv, Vec<cxd> Y, int ns) {
        if (h->mixed) {
            mixed_system<double>(h, h->delta, mode, X, Bv, Y, ns);
            return;
        }
        const Coef b0 = h->coef(h->delta == 0.0 ? HELM_OP_B0 : HELM_OP_BDELTA);
        if (h->dim == 2)
            stencil2d<double, double>(s, make_op2<double>(b0, h->n, h->omega), mode, 1.0, X, Bv, Y, ns);
        else
            op3d<double, double>(h, s, b0, 0, mode, 1.0, X, Bv, Y, ns);
        dir_mask<double>(h, s, 0, Y, ns);
    }
    void apply_BZ(Vec<const cx<T>> Zv, Vec<cxd> Y, int ns) {
        if (h->mixed) {
            mixed_system<T>(h, h->delta, MODE_APPLY, Zv, Vec<const cxd>{}, Y, ns);
            return;
        }
        const Coef b0 = h->coef(h->delta == 0.0 ? HELM_OP_B0 : HELM_OP_BDELTA);
        if (h->dim == 2)
            stencil2d<double, T>(s, make_op2<double>(b0, h->n, h->omega), MODE_APPLY, 1.0, Zv,
                                 Vec<const cxd>{}, Y, ns);
        else
            op3d<double, T>(h, s, b0, 0, MODE_APPLY, 1.0, Zv, Vec<const cxd>{}, Y, ns);
        dir_mask<double>(h, s, 0, Y, ns);
    }

    // Enqueue one step's device work.  Returns false if nothing to do.
    bool enqueue() {
        fresh_cols.clear();
        chk_cols.clear();
        it_cols.clear();
        for (int c = 0; c < cap; ++c) {
            if (col[c].phase == COL_FRESH) fresh_cols.push_back(c);
            else if (col[c].phase == COL_CHECK) chk_cols.push_back(c);
        }
        // initial residuals (fresh) and final checks share one batch
        std::vector<int> rc = fresh_cols;
        rc.insert(rc.end(), chk_cols.begin(), chk_cols.end());
        for (int c = 0; c < cap; ++c)
            if (col[c].phase == COL_ACTIVE) it_cols.push_back(c);
        std::vector<int> itc = fresh_cols;  // fresh columns iterate this step too
        itc.insert(itc.end(), it_cols.begin(), it_cols.end());
        it_cols = itc;
        if (rc.empty() && it_cols.empty()) return false;
        // index maps (one upload): [0] column ids of rc, [1] V0 of rc,
        // [2] b-norm columns, then for the iterating set: [3] V[c][j], [4] V[c][j+1],
        // [5] V[c][0], [6] Z[c][j], [7] j+1
        const int nr = (int)rc.size(), ni = (int)it_cols.size();
        int* m = hmap;
        std::vector<int> bn;  // fresh columns without a b norm yet
        for (int q = 0; q < nr; ++q) {
            const int c = rc[q];
            m[0 * cap + q] = c;
            m[1 * cap + q] = c * (R + 1);
        }
        for (int c : fresh_cols)
            if (!col[c].have_bnorm) bn.push_back(c);
        for (int q = 0; q < (int)bn.size(); ++q) m[2 * cap + q] = bn[q];
        int jmax = 0;
        for (int q = 0; q < ni; ++q) {
            const int c = it_cols[q];
            const int j = col[c].phase == COL_FRESH ? 0 : col[c].j;
            m[3 * cap + q] = c * (R + 1) + j;
            m[4 * cap + q] = c * (R + 1) + j + 1;
            m[5 * cap + q] = c * (R + 1);
            m[6 * cap + q] = c * R + j;
            m[7 * cap + q] = j + 1;
            jmax = std::max(jmax, j + 1);
        }
        int* dm = d_maps();
        HIPCHK(hipMemcpyAsync(dm, m, sizeof(int) * NMAPS * cap, hipMemcpyHostToDevice, s));
        double* dn = d_norm();  // [0, cap): |w|, [cap, 2cap): |r|, [2cap, 3cap): |b|
        if (!bn.empty())
            norm2(s, N, Vec<const cxd>{Bb(), N, 0, dm + 2 * cap}, d_npart(), dn + 2 * cap, 1,
                  (int)bn.size());
        if (nr) {
            // r = b - B x into V[c][0]
            apply_B(MODE_RESID, Vec<const cxd>{Xb(), N, 0, dm}, Vec<const cxd>{Bb(), N, 0, dm},
                    Vec<cxd>{Vb(), N, 0, dm + cap}, nr);
            norm2(s, N, Vec<const cxd>{Vb(), N, 0, dm + cap}, d_npart(), dn + cap, 1, nr);
            if (!fresh_cols.empty())  // fresh columns come first in rc
                scale_inv(s, N, Vec<const cxd>{Vb(), N, 0, dm + cap}, Vec<cxd>{Vb(), N, 0, dm + cap},
                          dn + cap, 1, (int)fresh_cols.size());
        }
        if (ni) {
            HIPCHK(hipEventRecord(e0, s));
            precondition<T>(h, Lw, ws, Vec<const cxd>{Vb(), N, 0, dm + 3 * cap},
                            Vec<cx<T>>{Zb(), N, 0, dm + 6 * cap}, ni);
            HIPCHK(hipEventRecord(e1, s));
            vcycles += (long long)ni * h->hss_steps * h->cycles;
            apply_BZ(Vec<const cx<T>>{Zb(), N, 0, dm + 6 * cap}, Vec<cxd>{Vb(), N, 0, dm + 4 * cap}, ni);
            const Vec<const cxd> V0{Vb(), N, 0, dm + 5 * cap};
            const Vec<cxd> W{Vb(), N, 0, dm + 4 * cap};
            const int nblk = multidot_blocks(N);
            // classical Gram-Schmidt; the second pass runs for the columns
            // whose first pass kept less than ~0.14 of w's norm (every
            // column with full_reorth), decided on the device
            const bool sel = !h->opts.full_reorth;
            const int* flag2 = sel ? d_flag() : nullptr;
            for (int pass = 0; pass < 2; ++pass) {
                cxd* hd = pass == 0 ? d_h() : d_h2();
                multidot(s, N, jmax, dm + 7 * cap, V0, cst(W), d_part(), ni,
                         pass == 0 && sel ? d_npart() : nullptr, pass == 1 ? flag2 : nullptr);
                reduce_parts(s, jmax, dm + 7 * cap, nblk, d_part(), hd, R + 1, 0, ni,
                             pass == 1 ? flag2 : nullptr);
                if (pass == 0 && sel)
                    reorth_flag(s, jmax, dm + 7 * cap, nblk, d_npart(), hd, R + 1, d_flag(), ni);
                multi_axpy(s, N, jmax, dm + 7 * cap, V0, hd, R + 1, W, ni, pass == 1 ? flag2 : nullptr);
            }
            if (sel) HIPCHK(hipMemcpyAsync(hflag, d_flag(), sizeof(int) * ni, hipMemcpyDeviceToHost, s));
            norm2(s, N, cst(W), d_npart(), dn, 1, ni);
            scale_inv(s, N, cst(W), W, dn, 1, ni);
            HIPCHK(hipMemcpyAsync(hh, d_h(), sizeof(cxd) * ni * (R + 1), hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(hh + (size_t)cap * (R + 1), d_h2(), sizeof(cxd) * ni * (R + 1),
                                  hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipMemcpyAsync(hn, dn, sizeof(double) * 3 * cap, hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(ev, s));
        pending = true;
        return true;
    }

    // Wait for the enqueued step, update the host state, enqueue the
    // solution updates of finishing columns.
    void complete() {
        if (!pending) return;
        HIPCHK(hipEventSynchronize(ev));
        pending = false;
        if (!it_cols.empty()) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) precond_ms += ms;
            for (size_t q = 0; q < it_cols.size(); ++q) reorth += h->opts.full_reorth ? 1 : hflag[q];
        }
        if (h->prof_on) h->prof_collect();
        // b norms of fresh columns
        {
            int q = 0;
            for (int c : fresh_cols)
                if (!col[c].have_bnorm) {
                    col[c].bnorm = hn[2 * cap + q++];
                    col[c].have_bnorm = true;
                }
        }
        // residual norms: fresh first, then checks
        int q = 0;
        std::vector<char> skip(cap, 0);
        for (int c : fresh_cols) {
            Column& C = col[c];
            C.beta = hn[cap + q++];
            if (C.r0 < 0.0) C.r0 = C.beta;
            C.est = C.bnorm > 0 ? C.beta / C.bnorm : 0.0;
            if (C.bnorm == 0.0 || C.beta <= C.tol * C.bnorm || !std::isfinite(C.beta)) {
                // already solved (or zero rhs): this step's iteration is discarded
                C.phase = COL_DONE;
                C.converged = std::isfinite(C.beta) && C.beta <= C.tol * C.bnorm;
                C.true_rel = C.est;
                skip[c] = 1;
            } else {
                std::fill(C.g.begin(), C.g.end(), zd(0.0));
                C.g[0] = C.beta;
                C.j = 0;
                C.phase = COL_ACTIVE;
            }
        }
        for (int c : chk_cols) {
            Column& C = col[c];
            const double r = hn[cap + q++];
            C.true_rel = C.bnorm > 0 ? r / C.bnorm : 0.0;
            if (C.true_rel <= C.tol) {
                C.phase = COL_DONE;
                C.converged = true;
            } else if (C.its >= h->max_outer) {
                C.phase = COL_DONE;
                C.converged = false;
            } else {
                C.phase = COL_FRESH;  // restart from the current iterate
                ++C.restarts;
            }
            C.est = C.true_rel;
        }
        // Arnoldi columns
        std::vector<int> fin;
        std::vector<int> finm;
        for (int s2 = 0; s2 < (int)it_cols.size(); ++s2) {
            const int c = it_cols[s2];
            if (skip[c]) continue;
            Column& C = col[c];
            const int j = C.j;
            zd* Hc = &C.H[(size_t)j * (R + 1)];
            for (int i = 0; i <= j; ++i) {
                const cxd a = hh[(size_t)s2 * (R + 1) + i];
                const cxd b = hh[(size_t)cap * (R + 1) + (size_t)s2 * (R + 1) + i];
                Hc[i] = zd(a.x + b.x, a.y + b.y);
            }
            const double hnorm = hn[s2];
            Hc[j + 1] = hnorm;
            for (int i = 0; i < j; ++i) {
                const zd t = C.cs[i] * Hc[i] + C.sn[i] * Hc[i + 1];
                Hc[i + 1] = -std::conj(C.sn[i]) * Hc[i] + std::conj(C.cs[i]) * Hc[i + 1];
                Hc[i] = t;
            }
            const zd a = Hc[j], b = Hc[j + 1];
            const double den = std::sqrt(std::norm(a) + std::norm(b));
            C.cs[j] = den != 0.0 ? std::conj(a) / den : zd(1.0);
            C.sn[j] = den != 0.0 ? std::conj(b) / den : zd(0.0);
            Hc[j] = C.cs[j] * a + C.sn[j] * b;
            Hc[j + 1] = 0.0;
            C.g[j + 1] = -std::conj(C.sn[j]) * C.g[j];
            C.g[j] = C.cs[j] * C.g[j];
            C.its += 1;
            C.j = j + 1;
            C.est = std::abs(C.g[j + 1]) / C.bnorm;
            const bool stop = std::abs(C.g[j + 1]) <= C.tol * C.bnorm || C.its >= h->max_outer ||
                              hnorm == 0.0 || !std::isfinite(hnorm);
            if (stop || C.j == R) {
                // y from the triangular system, x += Z y
                const int mcols = C.j;
                std::vector<zd> y(mcols);
                for (int i = mcols - 1; i >= 0; --i) {
                    zd acc = C.g[i];
                    for (int jj = i + 1; jj < mcols; ++jj) acc -= C.H[i + (size_t)jj * (R + 1)] * y[jj];
                    y[i] = acc / C.H[i + (size_t)i * (R + 1)];
                }
                const int f = (int)fin.size();
                for (int i = 0; i < mcols; ++i) hy[(size_t)f * R + i] = mk(y[i].real(), y[i].imag());
                fin.push_back(c);
                finm.push_back(mcols);
                if (stop) {
                    C.phase = COL_CHECK;
                } else {
                    C.phase = COL_FRESH;  // restart with the updated iterate
                    ++C.restarts;
                }
            }
        }
        if (!fin.empty()) {
            const int nf = (int)fin.size();
            int mmax = 0;
            for (int f = 0; f < nf; ++f) {
                hfin[0 * cap + f] = fin[f] * R;  // Z[c][0]
                hfin[1 * cap + f] = fin[f];      // X[c]
                hfin[2 * cap + f] = finm[f];
                mmax = std::max(mmax, finm[f]);
            }
            // the step maps region is free again after the sync above
            int* dm = d_maps();
            HIPCHK(hipMemcpyAsync(dm, hfin, sizeof(int) * 3 * cap, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(d_y(), hy, sizeof(cxd) * (size_t)nf * R, hipMemcpyHostToDevice, s));
            update_solution<T>(s, N, mmax, dm + 2 * cap, Vec<const cx<T>>{Zb(), N, 0, dm},
                               d_y(), R, Vec<cxd>{Xb(), N, 0, dm + cap}, nf);
        }
    }
};
