// Serving runtime (included at the end of helm_api.cpp only): continuous
// batching of independent solves over per-group column engines.
#pragma once

#include <thread>

namespace {

struct Request {
    long long id = 0;
    int dim = 2, n = 0, levels = 1, nrhs = 0;
    double k = 0, dh = 0, tol = 1e-8;
    const cxd* rhs = nullptr;
    cxd* x = nullptr;
    int status = 0;  // 0 queued, 1 running, 2 done
    int group = -1;
    std::vector<int> cols;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int its = 0;
    bool converged = false;
    double true_rel = 0.0;
};

struct Group {
    int dim = 2, n = 0, levels = 1;
    double k = 0, dh = 0;
    helm_t* h = nullptr;
    void* ws = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    Engine<double>* e64 = nullptr;
    Engine<float>* e32 = nullptr;
    bool enqueued = false;

    bool matches(const Request& r) const {
        return dim == r.dim && n == r.n && levels == r.levels && k == r.k && dh == r.dh;
    }
    int free_slots() const { return e64 ? e64->free_slots() : e32->free_slots(); }
    bool busy() const { return e64 ? e64->busy() : e32->busy(); }
    std::vector<Column>& cols() { return e64 ? e64->col : e32->col; }
    cxd* X() const { return e64 ? e64->Xb() : e32->Xb(); }
    long long N() const { return e64 ? e64->N : e32->N; }
    int admit(long long tag, const cxd* rhs, double tol) {
        return e64 ? e64->admit(tag, rhs, nullptr, tol) : e32->admit(tag, rhs, nullptr, tol);
    }
    bool enqueue() { return e64 ? e64->enqueue() : e32->enqueue(); }
    void complete() {
        if (e64) e64->complete();
        else e32->complete();
    }
    // an iteration is in flight on the device
    bool pending() const { return e64 ? e64->pending : e32->pending; }
    hipEvent_t event() const { return e64 ? e64->ev : e32->ev; }
};

}  // namespace

struct helm_server_s {
    helm_server_opts opts{};
    std::vector<Request> reqs;  // index = id
    std::vector<Group> groups;  // released groups keep h == nullptr
    double in_use = 0.0;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void release(Group& g) {
        if (g.e64) { g.e64->release(); delete g.e64; g.e64 = nullptr; }
        if (g.e32) { g.e32->release(); delete g.e32; g.e32 = nullptr; }
        if (g.h) (void)helm_destroy(g.h);
        if (g.ws) (void)hipFree(g.ws);
        if (g.stream) (void)hipStreamDestroy(g.stream);
        in_use -= (double)g.bytes;
        g = Group{};
    }

    // Workspace bytes of a group for request r, from the sizes alone (the
    // level table and the restart length helm_create would choose; nothing
    // is allocated).
    size_t plan_bytes(const Request& r) const {
        helm_s t;
        helm_opts_default(&t.opts);
        t.dim = r.dim;
        t.n = r.n;
        t.levels = r.levels;
        t.prec = opts.precision;
        t.restart = opts.restart > 0 ? opts.restart : std::min(2000, 3 * (int)std::ceil(r.k) + 30);
        for (int l = 0; l < r.levels; ++l) {
            const int nl = r.n >> l;
            long long Nl = 1;
            for (int d = 0; d < r.dim; ++d) Nl *= (nl + 1);
            t.nl.push_back(nl);
            t.Nl.push_back(Nl);
        }
        t.nv = t.Nl[0];
        return layout(&t, opts.max_cols).total;
    }

    // A group for request r: an existing one with room for its columns, or
    // a new one (another of the same parameters when those are full) if its
    // workspace fits the budget (idle groups are released to make room).
    // -1 if none; a request that cannot fit builds nothing.
    int group_for(const Request& r) {
        for (int q = 0; q < (int)groups.size(); ++q)
            if (groups[q].h && groups[q].matches(r) && groups[q].free_slots() >= r.nrhs) return q;
        const size_t need = plan_bytes(r);
        auto fits_need = [&]() { return in_use + (double)need <= opts.hbm_budget_bytes; };
        if (!fits_need()) {
            for (auto& other : groups)  // release idle groups if that makes room
                if (!fits_need() && other.h && !other.busy() && !other.pending()) release(other);
            if (!fits_need()) return -1;
        }
        helm_mesh mesh{r.dim, r.dim == 2 ? HELM_P1_TRI_RIGHT : HELM_Q1_HEX, r.n, r.levels};
        helm_opts o;
        helm_opts_default(&o);
        o.precision = opts.precision;
        o.restart = opts.restart;
        o.max_outer = opts.max_outer;
        Group g;
        g.dim = r.dim;
        g.n = r.n;
        g.levels = r.levels;
        g.k = r.k;
        g.dh = r.dh;
        HIPCHK(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
        if (helm_create(&mesh, r.k, 0.0, r.dh, nullptr, &o, g.stream, &g.h) != HELM_OK) {
            (void)hipStreamDestroy(g.stream);
            return -1;
        }
        g.bytes = layout(g.h, opts.max_cols).total;
        auto fits = [&]() { return in_use + (double)g.bytes <= opts.hbm_budget_bytes; };
        if (!fits() || hipMalloc(&g.ws, g.bytes) != hipSuccess) {
            (void)helm_destroy(g.h);
            (void)hipStreamDestroy(g.stream);
            return -1;
        }
        in_use += (double)g.bytes;
        if (opts.precision == HELM_FP64) {
            g.e64 = new Engine<double>();
            g.e64->init(g.h, g.ws, opts.max_cols, 1e-8);
            ensure_cycles<double>(g.h, g.e64->Lw, g.ws);
        } else {
            g.e32 = new Engine<float>();
            g.e32->init(g.h, g.ws, opts.max_cols, 1e-8);
            ensure_cycles<float>(g.h, g.e32->Lw, g.ws);
        }
        for (int q = 0; q < (int)groups.size(); ++q)
            if (!groups[q].h) {
                groups[q] = g;
                return q;
            }
        groups.push_back(g);
        return (int)groups.size() - 1;
    }

    void admit_queued() {
        for (auto& r : reqs) {
            if (r.status != 0) continue;
            const int gi = group_for(r);
            if (gi < 0) continue;
            Group& g = groups[gi];
            if (g.free_slots() < r.nrhs) continue;
            const long long N = g.N();
            r.cols.clear();
            for (int c = 0; c < r.nrhs; ++c) r.cols.push_back(g.admit(r.id, r.rhs + c * N, r.tol));
            r.group = gi;
            r.status = 1;
            r.t_admit = now();
        }
    }

    // Requests of group gi whose columns are all done: their solutions are
    // copied out (stream-ordered after the group's last updates) and their
    // slots freed.  Returns the number finished.
    int collect(int gi) {
        Group& g = groups[gi];
        std::vector<Column>& cs = g.cols();
        int done = 0;
        for (auto& r : reqs) {
            if (r.status != 1 || r.group != gi) continue;
            bool all = true;
            for (int c : r.cols) all = all && cs[c].phase == COL_DONE;
            if (!all) continue;
            const long long N = g.N();
            r.its = 0;
            r.converged = true;
            r.true_rel = 0.0;
            for (int q = 0; q < r.nrhs; ++q) {
                const int c = r.cols[q];
                HIPCHK(hipMemcpyAsync(r.x + q * N, g.X() + c * N, sizeof(cxd) * N,
                                      hipMemcpyDeviceToDevice, g.stream));
                r.its = std::max(r.its, cs[c].its);
                r.converged = r.converged && cs[c].converged;
                r.true_rel = std::max(r.true_rel, cs[c].true_rel);
            }
            for (int c : r.cols) cs[c].phase = COL_FREE;
            r.status = 2;
            ++done;
        }
        if (done) {
            // the copies precede the group's next iteration on its stream
            HIPCHK(hipStreamSynchronize(g.stream));
            const double t = now();
            for (auto& r : reqs)
                if (r.status == 2 && r.group == gi && r.t_done == 0.0) r.t_done = t;
        }
        return done;
    }

    // Every group runs on its own stream at its own pace: a group whose
    // iteration has finished on the device is completed at once (Givens
    // rotations, finished requests copied out, queued requests admitted into
    // its free slots) and its next iteration enqueued, while the others keep
    // running.  Returns after at least one group has advanced, or when no
    // group has work.
    int step() {
        int done = 0;
        for (;;) {
            admit_queued();
            bool advanced = false, inflight = false;
            for (int gi = 0; gi < (int)groups.size(); ++gi) {
                if (!groups[gi].h) continue;
                if (groups[gi].pending()) {
                    const hipError_t e = hipEventQuery(groups[gi].event());
                    if (e == hipErrorNotReady) {
                        inflight = true;
                        continue;
                    }
                    HIPCHK(e);
                    groups[gi].complete();
                    done += collect(gi);
                    admit_queued();  // may add groups: index, do not hold references
                    advanced = true;
                }
                if (groups[gi].h && groups[gi].enqueue()) inflight = true;
            }
            if (advanced || !inflight) break;
            std::this_thread::yield();
        }
        return done;
    }
};

extern "C" {

int helm_server_create(const helm_server_opts* opts, helm_server_t** out) {
    if (!out) return HELM_EINVAL;
    *out = nullptr;
    if (!opts || !(opts->hbm_budget_bytes > 0) || opts->max_cols < 1 || opts->max_cols > 256)
        return HELM_EINVAL;
    if (opts->precision != HELM_FP64 && opts->precision != HELM_FP32_MG) return HELM_EINVAL;
    if (opts->restart < 0 || opts->restart > 2000 || opts->max_outer < 0) return HELM_EINVAL;
    helm_server_t* s = new (std::nothrow) helm_server_t;
    if (!s) return HELM_ENOMEM;
    s->opts = *opts;
    *out = s;
    return HELM_OK;
}

int helm_server_submit(helm_server_t* s, int dim, int n, int levels, double k, double delta_hat,
                       const void* rhs, void* x, int nrhs, double tol, long long* id) {
    if (!s || !rhs || !x || !id || nrhs < 1 || nrhs > s->opts.max_cols) return HELM_EINVAL;
    if (!(tol > 0.0 && tol < 1.0) || !(k > 0.0) || !(delta_hat > 0.0)) return HELM_EINVAL;
    if ((dim != 2 && dim != 3) || n < 2 || levels < 1 || levels > 30 ||
        n % (1 << (levels - 1)) != 0)
        return HELM_EINVAL;
    Request r;
    r.id = (long long)s->reqs.size();
    r.dim = dim;
    r.n = n;
    r.levels = levels;
    r.k = k;
    r.dh = delta_hat;
    r.tol = tol;
    r.rhs = static_cast<const cxd*>(rhs);
    r.x = static_cast<cxd*>(x);
    r.nrhs = nrhs;
    r.t_submit = s->now();
    s->reqs.push_back(r);
    *id = r.id;
    return HELM_OK;
}

int helm_server_step(helm_server_t* s, int* n_done) {
    if (!s) return HELM_EINVAL;
    try {
        const int d = s->step();
        if (n_done) *n_done = d;
    } catch (const DevErr&) {
        return HELM_EDEVICE;
    } catch (const std::bad_alloc&) {
        return HELM_ENOMEM;
    }
    return HELM_OK;
}

int helm_server_query(const helm_server_t* s, long long id, helm_request_info* info) {
    if (!s || !info || id < 0 || id >= (long long)s->reqs.size()) return HELM_EINVAL;
    const Request& r = s->reqs[id];
    info->status = r.status;
    info->converged = r.converged ? 1 : 0;
    info->outer_its = r.its;
    info->true_rel_residual = r.true_rel;
    info->t_submit = r.t_submit;
    info->t_admit = r.t_admit;
    info->t_done = r.t_done;
    return HELM_OK;
}

int helm_server_load(const helm_server_t* s, int* queued, int* running, double* bytes_in_use) {
    if (!s) return HELM_EINVAL;
    int q = 0, r = 0;
    for (const auto& x : s->reqs) {
        q += x.status == 0;
        r += x.status == 1;
    }
    if (queued) *queued = q;
    if (running) *running = r;
    if (bytes_in_use) *bytes_in_use = s->in_use;
    return HELM_OK;
}

int helm_server_destroy(helm_server_t* s) {
    if (!s) return HELM_OK;
    for (auto& g : s->groups)
        if (g.h) s->release(g);
    delete s;
    return HELM_OK;
}

}  // extern "C"
