// Serving loop for the Moebius domain-wall solve: requests to solve D5 x = b
// (any resident gauge field, any L5 / M5 / b5 / c5, per-RHS masses, 1..n
// RHS) arrive at any time.  Each is admitted, in arrival order, as soon as its
// device footprint fits next to the requests already running, and runs on
// one of several worker threads, each with its own HIP stream, so the
// kernels of concurrent requests overlap on the device.  Gauge fields stay
// resident for the server's lifetime and are shared by every worker; solver
// buffers are released when a request finishes, returning its footprint.
// A request whose footprint exceeds the whole budget is split into
// sub-batches of the most RHS that fit, solved one after another on its
// worker.
//
// A request's arithmetic does not depend on what else runs (no reduction
// crosses requests, chunking and sub-batching are bitwise neutral), so its
// result equals the same solve run alone.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "ctx.h"

using namespace mdwf;

namespace {

constexpr int kMaxShared = 24;   // RHS of one shared solve at most

double wall() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
    int field = 0;
    int n = 0;                  // RHS
    int kind = 0;               // 0: 5D b / x fields; 1: point sources, 4D wall-field outputs
    mdwf_action act{};
    std::vector<const double*> b;
    std::vector<double*> x;
    std::vector<int> src;       // kind 1: x, y, z, t, spin-colour column per RHS
    std::vector<double*> q;     // kind 1: wall-field outputs
    std::vector<double> mq;
    std::vector<const double*> xref;   // reference solutions (opts.x_ref), or empty
    mdwf_solver_opts opts{};
    size_t footprint = 0;       // of one sub-batch
    int batch = 0;              // RHS per sub-batch
    int shared_rhs = 0;         // RHS of the solve it ran in (its own, or a shared one)
    double t_submit = 0, t_start = 0, t_end = 0;
    bool done = false;
    mdwf_status status = MDWF_OK;
    std::string err;
    std::vector<mdwf_solve_info> info;
};

struct GaugeField {
    mdwf_geometry geom{};
    mdwf_ctx* master = nullptr;   // owns the resident links
};

}  // namespace

struct mdwf_server {
    int device = 0;
    size_t budget = 0;          // device bytes requests may reserve together
    size_t reserved = 0, peak = 0;
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<int> pending;
    std::map<int, Request> reqs;
    std::vector<GaugeField> fields;
    std::vector<std::thread> workers;
    bool stop = false;
    int next_id = 1;
    std::string err;
};

namespace {

mdwf_status sfail(mdwf_server* s, mdwf_status st, const std::string& msg) {
    if (s) s->err = msg;
    return st;
}

// footprint of a request (solver buffers with host I/O; links are resident)
size_t footprint(const GaugeField& f, const mdwf_action& a, int nrhs, mdwf_prec inner, int kind = 0) {
    return solve_footprint(plan_geo(f.geom, a.L5), Prec(inner), nrhs, kind ? IO_POINT : IO_HOST);
}

// One solve of RHS [k0, k0 + k) of the given arrays (5D fields or point sources).
mdwf_status solve_part(mdwf_ctx* c, int kind, int k, const double* const* b, double* const* x, const int* src,
                       double* const* q, const double* mq, const mdwf_solver_opts* o, mdwf_solve_info* info) {
    if (kind == 0) return mdwf_solve(c, k, b, x, mq, o, info);
    const PointIO pt{src, q};
    return mdwf_solve_impl(c, k, nullptr, nullptr, true, mq, o, info, c->stream, &pt);
}

// Requests that can share one solve, so that every hop launch of it reads
// the links once for all their RHS: the same field, the same action apart
// from the masses (each RHS keeps its own), the same solver options, and
// neither split into sub-batches; 5D-field and point requests do not mix.
bool same_opts(const mdwf_solver_opts& a, const mdwf_solver_opts& b) {
    return a.tol == b.tol && a.max_iter == b.max_iter && a.inner == b.inner && a.delta == b.delta &&
           a.check_every == b.check_every && a.schur_form == b.schur_form && a.max_seconds == b.max_seconds;
}
bool can_share(const Request& a, const Request& b) {
    return a.field == b.field && a.act.L5 == b.act.L5 && a.act.M5 == b.act.M5 && a.act.b5 == b.act.b5 &&
           a.act.c5 == b.act.c5 && same_opts(a.opts, b.opts) && a.xref.empty() == b.xref.empty() &&
           a.kind == b.kind && a.batch == a.n && b.batch == b.n;
}

// Status of one request of a shared solve from its RHS's records.
mdwf_status request_status(const Request& r) {
    mdwf_status st = MDWF_OK;
    for (const mdwf_solve_info& i : r.info) {
        if (!std::isfinite(i.true_resid)) return MDWF_ERR_NUMERIC;
        if (i.true_resid > r.opts.tol) st = MDWF_ERR_NOCONV;
    }
    return st;
}

void worker_loop(mdwf_server* s) {
    (void)hipSetDevice(s->device);
    std::map<std::pair<int, int>, mdwf_ctx*> ctxs;   // (field, L5) -> context on this worker's stream
    for (;;) {
        std::vector<Request*> grp;
        size_t fp = 0;
        GaugeField f;
        {
            std::unique_lock<std::mutex> lk(s->m);
            s->cv_work.wait(lk, [&] {
                if (s->pending.empty()) return s->stop;
                const Request& f = s->reqs[s->pending.front()];
                return s->reserved + f.footprint <= s->budget;
            });
            if (s->pending.empty()) break;   // stop requested and nothing left
            Request* r = &s->reqs[s->pending.front()];
            s->pending.pop_front();
            grp.push_back(r);
            fp = r->footprint;
            f = s->fields[r->field];   // copied: add_field may grow the list meanwhile
            // queued requests that can share this solve join it while the
            // combined footprint fits (they would otherwise wait behind it)
            int n = r->n;
            if (r->batch == n) {
                for (auto it = s->pending.begin(); it != s->pending.end() && n < kMaxShared;) {
                    Request& q = s->reqs[*it];
                    const int nq = q.n;
                    const size_t fq = footprint(f, r->act, n + nq, r->opts.inner, r->kind);
                    if (can_share(*r, q) && n + nq <= kMaxShared && s->reserved + fq <= s->budget) {
                        grp.push_back(&q);
                        n += nq;
                        fp = fq;
                        it = s->pending.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            s->reserved += fp;
            s->peak = std::max(s->peak, s->reserved);
            const double t0 = wall();
            for (Request* q : grp) {
                q->t_start = t0;
                q->shared_rhs = n;
            }
        }
        // the request records (map nodes) are not touched by other threads until done
        Request* r = grp[0];
        mdwf_ctx*& c = ctxs[{r->field, r->act.L5}];
        mdwf_status st = MDWF_OK;
        if (!c) {
            st = mdwf_create(&f.geom, s->device, nullptr, &c);
            if (st == MDWF_OK) share_gauge(c, f.master);
        }
        if (st == MDWF_OK) st = mdwf_set_action(c, &r->act);
        std::string msg = st == MDWF_OK ? std::string() : std::string(mdwf_last_error(c));
        if (grp.size() == 1) {
            const int n = r->n;
            // sub-batches in order; one that did not converge still wrote its
            // results, so the rest still run; a hard error stops the request
            for (int k0 = 0; st == MDWF_OK || st == MDWF_ERR_NOCONV || st == MDWF_ERR_NUMERIC; k0 += r->batch) {
                if (k0 >= n) break;
                const int k = std::min(r->batch, n - k0);
                mdwf_solver_opts ok = r->opts;   // the time limit covers the whole request
                if (r->opts.max_seconds > 0.0)
                    ok.max_seconds = std::max(1e-9, r->opts.max_seconds - (wall() - r->t_start));
                ok.x_ref = r->xref.empty() ? nullptr : r->xref.data() + k0;
                const mdwf_status sk =
                    solve_part(c, r->kind, k, r->kind ? nullptr : r->b.data() + k0, r->kind ? nullptr : r->x.data() + k0,
                               r->kind ? r->src.data() + 5 * k0 : nullptr, r->kind ? r->q.data() + k0 : nullptr,
                               r->mq.data() + k0, &ok, r->info.data() + k0);
                if (sk == MDWF_OK) continue;
                const bool hard = sk != MDWF_ERR_NOCONV && sk != MDWF_ERR_NUMERIC;
                if (st == MDWF_OK || hard) {
                    st = sk;
                    msg = mdwf_last_error(c);
                }
            }
            r->status = st;
            r->err = msg;
        } else {
            // one solve for the whole group: RHS of every request side by
            // side, each with its own mass; its results go back per request
            std::vector<const double*> b;
            std::vector<double*> x, qo;
            std::vector<int> src;
            std::vector<double> mq;
            std::vector<const double*> xref;
            int total = 0;
            for (Request* q : grp) {
                b.insert(b.end(), q->b.begin(), q->b.end());
                x.insert(x.end(), q->x.begin(), q->x.end());
                src.insert(src.end(), q->src.begin(), q->src.end());
                qo.insert(qo.end(), q->q.begin(), q->q.end());
                mq.insert(mq.end(), q->mq.begin(), q->mq.end());
                xref.insert(xref.end(), q->xref.begin(), q->xref.end());
                total += q->n;
            }
            std::vector<mdwf_solve_info> info(total);
            if (st == MDWF_OK) {
                mdwf_solver_opts ok = r->opts;
                ok.x_ref = xref.empty() ? nullptr : xref.data();
                st = solve_part(c, r->kind, total, b.data(), x.data(), src.data(), qo.data(), mq.data(), &ok,
                                info.data());
                if (st != MDWF_OK) msg = mdwf_last_error(c);
            }
            const bool hard = st != MDWF_OK && st != MDWF_ERR_NOCONV && st != MDWF_ERR_NUMERIC;
            size_t k0 = 0;
            for (Request* q : grp) {
                std::copy(info.begin() + k0, info.begin() + k0 + q->n, q->info.begin());
                k0 += q->n;
                q->status = hard ? st : request_status(*q);
                q->err = q->status == MDWF_OK ? std::string() : msg;
            }
        }
        if (c) release_solver_buffers(c);
        {
            std::lock_guard<std::mutex> lk(s->m);
            const double t1 = wall();
            for (Request* q : grp) {
                q->t_end = t1;
                q->done = true;
            }
            s->reserved -= fp;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    for (auto& kv : ctxs) mdwf_destroy(kv.second);
}

}  // namespace

extern "C" {

mdwf_status mdwf_server_create(int hip_device, size_t mem_budget, int max_active, mdwf_server** out) {
    if (!out || max_active < 1) return MDWF_ERR_ARG;
    *out = nullptr;
    if (hipSetDevice(hip_device) != hipSuccess) return MDWF_ERR_HIP;
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return MDWF_ERR_HIP;
    mdwf_server* s = new (std::nothrow) mdwf_server;
    if (!s) return MDWF_ERR_OOM;
    s->device = hip_device;
    const size_t cap = freeb / 10 * 9;
    s->budget = (mem_budget == 0 || mem_budget > cap) ? cap : mem_budget;
    for (int w = 0; w < max_active; ++w) s->workers.emplace_back(worker_loop, s);
    *out = s;
    return MDWF_OK;
}

void mdwf_server_destroy(mdwf_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& f : s->fields) mdwf_destroy(f.master);
    delete s;
}

const char* mdwf_server_last_error(const mdwf_server* s) { return s ? s->err.c_str() : ""; }

mdwf_status mdwf_server_add_field(mdwf_server* s, const mdwf_geometry* geom, const double* U, int* field_id) {
    if (!s || !geom || !U || !field_id) return sfail(s, MDWF_ERR_ARG, "null argument");
    mdwf_ctx* c = nullptr;
    mdwf_status st = mdwf_create(geom, s->device, nullptr, &c);
    if (st) return sfail(s, st, mdwf_last_error(nullptr));
    st = mdwf_load_gauge(c, U);
    if (st) {
        const std::string msg = mdwf_last_error(c);
        mdwf_destroy(c);
        return sfail(s, st, msg);
    }
    release_solver_buffers(c);   // drop the upload staging
    {
        std::lock_guard<std::mutex> lk(s->m);
        const size_t gb = gauge_bytes(c);
        s->budget = s->budget > gb ? s->budget - gb : 0;   // the links stay resident
        s->fields.push_back({*geom, c});
        *field_id = int(s->fields.size()) - 1;
        // queued requests were sized for the old budget: shrink their
        // sub-batches to fit the new one, and fail those whose single RHS no
        // longer fits (they could never be admitted)
        for (auto it = s->pending.begin(); it != s->pending.end();) {
            Request& r = s->reqs[*it];
            const GaugeField& fld = s->fields[r.field];
            while (r.batch > 0 && footprint(fld, r.act, r.batch, r.opts.inner, r.kind) > s->budget) --r.batch;
            if (r.batch > 0) {
                r.footprint = footprint(fld, r.act, r.batch, r.opts.inner, r.kind);
                ++it;
                continue;
            }
            r.status = MDWF_ERR_OOM;
            r.err = "after a gauge field was added, one RHS of this request needs " +
                    std::to_string(footprint(fld, r.act, 1, r.opts.inner, r.kind)) + " device bytes, the budget is " +
                    std::to_string(s->budget);
            r.t_start = r.t_end = wall();
            r.done = true;
            it = s->pending.erase(it);
        }
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
    return MDWF_OK;
}

}  // extern "C"

namespace {
// Validate and queue a request whose kind-specific arrays are filled in.
mdwf_status enqueue(mdwf_server* s, int field_id, const mdwf_action* act, Request&& r, const double* mq,
                    const mdwf_solver_opts* opts, int* req_id) {
    {
        std::lock_guard<std::mutex> lk(s->m);
        if (field_id < 0 || field_id >= int(s->fields.size())) return sfail(s, MDWF_ERR_ARG, "unknown field");
        r.field = field_id;
    }
    if (act->L5 < 1 || act->L5 > kMaxL5) return sfail(s, MDWF_ERR_ARG, "need 1 <= L5 <= 32");
    r.act = *act;
    r.mq.assign(r.n, act->mq);
    if (mq) r.mq.assign(mq, mq + r.n);
    mdwf_default_opts(&r.opts);
    if (opts) r.opts = *opts;
    if (r.opts.x_ref) {   // copied like b and x; the fields stay the caller's
        if (r.kind) return sfail(s, MDWF_ERR_ARG, "reference solutions need 5D solutions (not point solves)");
        r.xref.assign(r.opts.x_ref, r.opts.x_ref + r.n);
        for (int k = 0; k < r.n; ++k)
            if (!r.xref[k]) return sfail(s, MDWF_ERR_ARG, "null reference solution pointer");
    }
    r.opts.x_ref = nullptr;
    r.opts.use_graph = 0;       // each solve runs eagerly on its worker's stream
    r.opts.profile_iters = 0;
    r.info.assign(r.n, mdwf_solve_info{});
    std::lock_guard<std::mutex> lk(s->m);
    // the most RHS per sub-batch whose footprint fits the budget
    const GaugeField& fld = s->fields[field_id];
    r.batch = r.n;
    while (r.batch > 0 && footprint(fld, r.act, r.batch, r.opts.inner, r.kind) > s->budget) --r.batch;
    if (r.batch == 0)
        return sfail(s, MDWF_ERR_OOM,
                     "one RHS needs " + std::to_string(footprint(fld, r.act, 1, r.opts.inner, r.kind)) +
                         " device bytes, the budget is " + std::to_string(s->budget));
    r.footprint = footprint(fld, r.act, r.batch, r.opts.inner, r.kind);
    r.t_submit = wall();
    const int id = s->next_id++;
    s->reqs.emplace(id, std::move(r));
    s->pending.push_back(id);
    *req_id = id;
    s->cv_work.notify_all();
    return MDWF_OK;
}
}  // namespace

extern "C" {

mdwf_status mdwf_server_submit(mdwf_server* s, int field_id, const mdwf_action* act, int nrhs,
                               const double* const* b, double* const* x, const double* mq,
                               const mdwf_solver_opts* opts, int* req_id) {
    if (!s || !act || !b || !x || !req_id || nrhs < 1) return sfail(s, MDWF_ERR_ARG, "bad request arguments");
    Request r;
    r.n = nrhs;
    r.b.assign(b, b + nrhs);
    r.x.assign(x, x + nrhs);
    for (int k = 0; k < nrhs; ++k)
        if (!r.b[k] || !r.x[k]) return sfail(s, MDWF_ERR_ARG, "null right-hand side or solution pointer");
    return enqueue(s, field_id, act, std::move(r), mq, opts, req_id);
}

mdwf_status mdwf_server_submit_point(mdwf_server* s, int field_id, const mdwf_action* act, const int* site,
                                     int ncols, const int* cols, const double* mq, const mdwf_solver_opts* opts,
                                     double* const* q, int* req_id) {
    if (!s || !act || !site || !q || !req_id || ncols < 1) return sfail(s, MDWF_ERR_ARG, "bad request arguments");
    Request r;
    r.n = ncols;
    r.kind = 1;
    {
        std::lock_guard<std::mutex> lk(s->m);
        if (field_id < 0 || field_id >= int(s->fields.size())) return sfail(s, MDWF_ERR_ARG, "unknown field");
        const mdwf_geometry& g = s->fields[field_id].geom;
        const int ext[4] = {g.X, g.Y, g.Z, g.T};
        for (int d = 0; d < 4; ++d)
            if (site[d] < 0 || site[d] >= ext[d]) return sfail(s, MDWF_ERR_ARG, "point source site outside the lattice");
    }
    for (int k = 0; k < ncols; ++k) {
        const int col = cols ? cols[k] : k;
        if (col < 0 || col > 11) return sfail(s, MDWF_ERR_ARG, "spin-colour column must be in 0..11");
        if (!q[k]) return sfail(s, MDWF_ERR_ARG, "null wall-field output pointer");
        r.src.insert(r.src.end(), {site[0], site[1], site[2], site[3], col});
    }
    r.q.assign(q, q + ncols);
    return enqueue(s, field_id, act, std::move(r), mq, opts, req_id);
}

mdwf_status mdwf_server_wait(mdwf_server* s, int req_id, mdwf_solve_info* info, double* times) {
    if (!s) return MDWF_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->m);
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return sfail(s, MDWF_ERR_ARG, "unknown request");
    s->cv_done.wait(lk, [&] { return it->second.done; });
    Request& r = it->second;
    if (info) std::copy(r.info.begin(), r.info.end(), info);
    if (times) {
        times[0] = r.t_start - r.t_submit;   // queued
        times[1] = r.t_end - r.t_start;      // on a worker
        times[2] = r.t_end - r.t_submit;     // latency
    }
    const mdwf_status st = r.status;
    if (st != MDWF_OK) s->err = r.err;
    s->reqs.erase(it);
    return st;
}

mdwf_status mdwf_server_stats(mdwf_server* s, size_t* budget, size_t* peak_reserved, int* queued) {
    if (!s) return MDWF_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->m);
    if (budget) *budget = s->budget;
    if (peak_reserved) *peak_reserved = s->peak;
    if (queued) *queued = int(s->pending.size());
    return MDWF_OK;
}

}  // extern "C"
