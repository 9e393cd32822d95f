// Solve D5 x = b for several right-hand sides at once (arXiv:1701.07559,
// Sec. VII: even-odd preconditioned Moebius solve, "double-half" mixed
// precision).
//
//   b'_e = b_e + 1/2 D_eo B K5^-1 b_o
//   CG on the normal equations of S x_e = b'_e in least-squares form:
//     q = S p, alpha = |s|^2/|q|^2, x += alpha p, r -= alpha q,
//     s = S^+ r, beta = |s_new|^2/|s|^2, p = s + beta p
// The solution update is applied every second iteration, in the pass that
// writes the next direction: p alternates between two buffers, an even
// iteration writes p_next = s + beta p beside p (x waits), the odd one adds
// alpha_prev p_prev + alpha p to x and writes its p_next over p_prev.  x is
// read and written once per two iterations.  A reliable update first adds
// a pending alpha_prev p_prev.
//   x_o = K5^-1 (b_o + 1/2 D_oe B x_e)
// The recursion tracks r = b' - S x_e, whose norm equals the full residual
// |b - D5 x| after reconstruction, so it stops on the quantity that matters;
// every stop is confirmed by an FP64 true residual of the full system.
// The symmetric form (schur_form 1) runs the same recursion on
// K5^-1 S x_e = K5^-1 b'_e with the symmetric coefficient table; its
// residual is K5^-1 r, so the tracked target is divided by a bound on |K5|.
// Right preconditioning by B (schur_form 2) runs it on S B^-1 y = b'_e: the
// iterate is y = B x_e (x_hi, x_lo hold y) and the residual is unchanged;
// x_e = B^-1 y is formed for the true residual and the output.
//
// Mixed precision: the inner vectors r, p, s, q and the hop temporary live in
// FP32 or FP16 (per-site norm) and the inner solution x_lo in FP32;
// the FP64 solution x_hi, the prepared source and all reductions stay FP64.
// When the iterated |r| falls below delta times its value at the last update
// (or reaches the target) the solver flushes x_lo into x_hi, recomputes
// r = b' - S x_hi with the FP64 operator and continues from it, keeping the
// search direction p.
//
// Right-hand sides (with their own masses) share every launch of the
// iteration; a per-RHS active flag in device memory lets finished ones drop
// out without re-capturing the iteration graph.  The CG scalars live in
// device memory; the host reads |r|^2 one iteration late so the GPU never
// waits for it.
//
// Memory: per RHS only x_hi and b' (FP64) and r, p, s, q, x_lo (inner) stay
// resident.  The hop temporary is shared by a chunk of RHS, and the FP64
// scratch of reliable updates, source preparation and verification is shared
// and used one RHS at a time; the caller's canonical b and x (device, or host
// through one staging field) are touched only at the start and at the end.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ctx.h"

using namespace mdwf;

namespace {

struct Solver {
    mdwf_ctx* c;
    Geo g;
    hipStream_t st;
    int n;
    Prec pi, px;
    bool mixed;
    size_t H64, Hi, Hx;
    int nbh, nbb;
    int chunk;   // RHS per Schur launch pair (they share the hop temporary)
    // per RHS
    char *xh, *bp;                 // FP64, stride H64
    char *r, *p, *p2, *s, *q, *xl; // inner precision (x_lo: px), strides Hi / Hx; p / p2
                                   // hold the direction of even / odd iterations
    // shared
    char* t;                       // inner hop temporary, `chunk` RHS at stride Hi
    char *be, *bo, *rh, *t64, *ye, *xo;   // FP64 scratch, one RHS each
    double* canon = nullptr;       // canonical staging of one field (host I/O)
    RhsCoef* coef;                 // [n] the action's, then [n] the symmetric form's
    int form = 0;                  // CG operator: 0 S, 1 K5^-1 S, 2 S B^-1
    CGScal* sc;
    int* act;
    int* msk;
    double* part;
    double* sums;
    CGScal* hsc[2];
    double* hsum;
    int* hmask;
    hipEvent_t ev[2];
    // launch timing of sampled iterations: 6 events per iteration around
    // kernels A, B of S and of S^+ (first chunk); prof = the current six
    std::vector<hipEvent_t> pev;
    hipEvent_t* prof = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // even, odd iteration
    hipGraph_t graph[2] = {nullptr, nullptr};
    mdwf_status err = MDWF_OK;
    const double* const* b;
    double* const* x;
    bool host_io;
    size_t canon_bytes;
    const PointIO* pt = nullptr;   // point sources and wall-field outputs

    ~Solver() {
        for (hipEvent_t e : pev) (void)hipEventDestroy(e);
    }

    bool ok(mdwf_status s_) {
        if (s_ != MDWF_OK && err == MDWF_OK) err = s_;
        return err == MDWF_OK;
    }
    bool hipok(hipError_t e, const char* what) { return ok(hip_check(c, e, what)); }

    void upload_mask(int* dst, const std::vector<int>& m) {
        for (int k = 0; k < n; ++k) hmask[k] = m[k];
        hipok(hipMemcpyAsync(dst, hmask, sizeof(int) * n, hipMemcpyHostToDevice, st), "mask upload");
        // the pinned staging is reused: wait until the copy has read it
        hipok(hipStreamSynchronize(st), "mask upload");
    }

    // The CG operator (S or K5^-1 S) or its adjoint on nk consecutive RHS
    // (stride apart) starting at the given pointers; tmp holds nk odd half
    // fields and tmp2 (symmetric adjoint only) nk even ones at the same
    // stride.  k0: index of the first RHS in the coefficient tables.
    void schur(Prec pr, const char* in, char* out, char* tmp, char* tmp2, size_t stride, int nk, int k0,
               const int* mask, bool dag, double* partials, hipEvent_t* evs = nullptr) {
        schur_launch(g, c->gs, pr, form, dag, in, out, tmp, tmp2, stride, nk, coef + k0, coef + n + k0, mask,
                     partials, st, evs);
        hipok(hipGetLastError(), "schur launch");
    }

    // inner-precision operator on all RHS, chunk by chunk; partials [n][nbh].
    // The symmetric adjoint stages K5^-+ in through q, free at both calls.
    void schur_inner(const char* in, char* out, const int* mask, bool dag, double* partials,
                     hipEvent_t* evs = nullptr) {
        for (int k0 = 0; k0 < n; k0 += chunk) {
            const int nk = std::min(chunk, n - k0);
            schur(pi, in + Hi * k0, out + Hi * k0, t, q + Hi * k0, Hi, nk, k0, mask ? mask + k0 : nullptr, dag,
                  partials ? partials + size_t(k0) * nbh : nullptr, k0 == 0 ? evs : nullptr);
        }
    }

    // per-RHS sums of partials (nblk per RHS) -> host vector
    std::vector<double> fetch_sums(int nblk, int nr, const int* mask) {
        launch_scalars(SC_SUM, part, nblk, nr, mask, sc, sums, st);
        hipok(hipMemcpyAsync(hsum, sums, sizeof(double) * nr, hipMemcpyDeviceToHost, st), "sum D2H");
        hipok(hipStreamSynchronize(st), "sum sync");
        return std::vector<double>(hsum, hsum + nr);
    }
    double norm2_one(Prec pr, const void* v) {
        launch_norm2(g, pr, v, 0, 1, nullptr, part, st);
        return fetch_sums(nbb, 1, nullptr)[0];
    }

    // source k, packed into the shared scratch be / bo
    void load_b(int k) {
        if (pt) {   // a point-source column, generated in place
            hipok(hipMemsetAsync(be, 0, H64, st), "memset");
            hipok(hipMemsetAsync(bo, 0, H64, st), "memset");
            launch_point_source(g, pt->src + 5 * k, be, bo, st);
            return;
        }
        const double* src = b[k];
        if (host_io) {
            hipok(hipMemcpyAsync(canon, b[k], canon_bytes, hipMemcpyHostToDevice, st), "b H2D");
            src = canon;
        }
        launch_pack_parity(g, P64, 1, 0, src, be, st);
        launch_pack_parity(g, P64, 1, 1, src, bo, st);
    }

    void* xcur() const { return mixed ? static_cast<void*>(xl) : static_cast<void*>(xh); }
    size_t sxc() const { return mixed ? Hx : H64; }

    // iteration j (odd: the second of a pair) with direction p_j in
    // (odd ? p2 : p)
    void one_iteration(bool odd) {
        char* pc = odd ? p2 : p;
        char* po = odd ? p : p2;
        schur_inner(pc, q, act, false, part, prof);
        launch_scalars(odd ? SC_ALPHA : SC_ALPHA_KEEP, part, nbh, n, act, sc, nullptr, st);
        launch_cg_r(g, pi, r, q, Hi, n, act, sc, part, st);
        launch_scalars(SC_RR, part, nbb, n, act, sc, nullptr, st);
        schur_inner(r, s, act, true, part, prof ? prof + 3 : nullptr);
        launch_scalars(SC_BETA, part, nbh, n, act, sc, nullptr, st);
        if (odd) launch_cg_xp2(g, mixed ? px : P64, pi, xcur(), sxc(), po, pc, s, Hi, n, act, sc, st);
        else launch_cg_p(g, pi, po, pc, s, Hi, n, act, sc, st);
    }
};

double now() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

namespace mdwf {
// The solver's device memory plan, shared by the allocation below and by
// every footprint estimate (the server's admission, mdwf_solve_footprint).
SolvePlan solve_plan(const Geo& g, Prec inner, int io) {
    const bool mixed = inner != P64;
    const size_t H64 = half_field_bytes(P64, g.Vh), Hi = half_field_bytes(inner, g.Vh);
    const size_t Hx = half_field_bytes(P32, g.Vh);
    SolvePlan pl;
    // x_hi and b' in FP64; r, p, p', s, q in the inner precision; the FP32
    // inner solution x_lo when mixed
    pl.per_rhs = 2 * H64 + (mixed ? 5 * Hi + Hx : 5 * H64);
    // FP64 scratch be, bo, r_hi, t64, ye, xo; the canonical staging field
    // (5D for host fields, 4D for wall-field outputs)
    const size_t stage = io == IO_HOST ? size_t(2) * g.Vh * 24 * sizeof(double)
                       : io == IO_POINT ? size_t(2) * g.Vh4 * 24 * sizeof(double) : 0;
    pl.shared = 6 * H64 + stage;
    pl.tmp_per_rhs = mixed ? Hi : H64;   // hop temporary of one RHS of a chunk
    pl.margin = size_t(64) << 20;        // coefficient tables, scalars, partials
    return pl;
}

Geo plan_geo(const mdwf_geometry& geom, int L5) {
    Geo g{};
    g.X = geom.X; g.Y = geom.Y; g.Z = geom.Z; g.T = geom.T;
    g.Xh = geom.X / 2;
    g.Vh4 = int(size_t(geom.X) * geom.Y * geom.Z * geom.T / 2);
    g.L5 = L5;
    g.Vh = g.Vh4 * L5;
    return g;
}

size_t solve_footprint(const Geo& g, Prec inner, int n, int io) {
    const SolvePlan pl = solve_plan(g, inner, io);
    return pl.per_rhs * n + pl.shared + pl.tmp_per_rhs * n + pl.margin;
}
}  // namespace mdwf

mdwf_status mdwf_solve_impl(mdwf_ctx* c, int nrhs, const double* const* b_in, double* const* x_out, bool host_io,
                            const double* mq, const mdwf_solver_opts* o_in, mdwf_solve_info* info, hipStream_t st,
                            const PointIO* pt) {
    const double t_start = now();
    if (pt) {
        if (nrhs < 1 || !pt->src || !pt->q) return fail(c, MDWF_ERR_ARG, "need nrhs >= 1, sources and outputs");
        const int ext[4] = {c->geo.X, c->geo.Y, c->geo.Z, c->geo.T};
        for (int k = 0; k < nrhs; ++k) {
            if (!pt->q[k]) return fail(c, MDWF_ERR_ARG, "null wall-field output pointer");
            for (int d = 0; d < 4; ++d)
                if (pt->src[5 * k + d] < 0 || pt->src[5 * k + d] >= ext[d])
                    return fail(c, MDWF_ERR_ARG, "point source site outside the lattice");
            if (pt->src[5 * k + 4] < 0 || pt->src[5 * k + 4] > 11)
                return fail(c, MDWF_ERR_ARG, "spin-colour column must be in 0..11");
        }
        host_io = true;
    } else {
        if (nrhs < 1 || !b_in || !x_out) return fail(c, MDWF_ERR_ARG, "need nrhs >= 1 and b, x arrays");
        for (int k = 0; k < nrhs; ++k)
            if (!b_in[k] || !x_out[k]) return fail(c, MDWF_ERR_ARG, "null right-hand side or solution pointer");
    }
    mdwf_solver_opts o;
    mdwf_default_opts(&o);
    if (o_in) o = *o_in;
    if (!(o.tol > 0.0) || o.max_iter < 1 || (o.inner != MDWF_F64 && o.inner != MDWF_F32 && o.inner != MDWF_F16) ||
        !(o.delta > 0.0 && o.delta < 1.0) || o.schur_form < 0 || o.schur_form > 2 || !(o.max_seconds >= 0.0))
        return fail(c, MDWF_ERR_ARG,
                    "bad solver options (tol > 0, max_iter >= 1, 0 < delta < 1, schur_form 0-2, max_seconds >= 0)");
    if (o.check_every < 1) o.check_every = 1;
    if (pt && o.x_ref) return fail(c, MDWF_ERR_ARG, "reference solutions need 5D solutions (not point solves)");
    std::vector<double> masses(nrhs, c->act.mq);
    if (mq)
        for (int k = 0; k < nrhs; ++k) {
            if (!(mq[k] >= 0.0 && mq[k] <= 1.0)) return fail(c, MDWF_ERR_ARG, "need 0 <= mq <= 1");
            masses[k] = mq[k];
        }

    Solver S;
    S.c = c;
    S.g = c->geo;
    S.st = st;
    S.n = nrhs;
    S.b = b_in;
    S.x = x_out;
    S.host_io = host_io;
    S.pi = Prec(o.inner);
    S.mixed = S.pi != P64;
    S.px = S.mixed ? P32 : P64;   // inner solution accumulator
    const Geo& g = S.g;
    S.H64 = half_field_bytes(P64, g.Vh);
    S.Hi = half_field_bytes(S.pi, g.Vh);
    S.Hx = half_field_bytes(S.px, g.Vh);
    S.nbh = hop_blocks_per_rhs(g);
    S.nbb = blas_blocks_per_rhs(g);
    S.canon_bytes = pt ? size_t(2) * g.Vh4 * 24 * sizeof(double) : size_t(2) * g.Vh * 24 * sizeof(double);
    S.pt = pt;
    const int n = nrhs;

    // memory plan: the hop temporary is shared by `chunk` RHS; shrink the
    // chunk when the whole batch would not fit next to the resident state
    const SolvePlan plan = solve_plan(g, S.pi, pt ? IO_POINT : host_io ? IO_HOST : IO_DEVICE);
    const size_t per_rhs = plan.per_rhs, shared = plan.shared;
    size_t held = 0;
    for (auto& kv : c->bufs)
        if (kv.first.rfind("sv_", 0) == 0) held += kv.second.n;
    size_t freeb = 0, totalb = 0;
    if (!S.hipok(hipMemGetInfo(&freeb, &totalb), "hipMemGetInfo")) return S.err;
    const size_t avail = freeb + held;
    const size_t need_fixed = per_rhs * n + shared + plan.margin;
    int cap = 0;   // explicit sub-batch size (memory / tests)
    if (const char* e = std::getenv("MDWF_SOLVE_BATCH")) cap = std::max(0, std::atoi(e));
    if (n > 1 && (need_fixed + plan.tmp_per_rhs > avail || (cap > 0 && cap < n))) {
        // the batch does not fit even with a one-RHS hop temporary: solve it
        // in consecutive sub-batches that do (same arithmetic per RHS)
        const size_t base = shared + plan.margin;
        int nb = avail > base + per_rhs + plan.tmp_per_rhs ? int((avail - base - plan.tmp_per_rhs) / per_rhs) : 1;
        if (cap > 0) nb = std::min(nb, cap);
        if (nb < n) {
            mdwf_status worst = MDWF_OK;
            for (int k0 = 0; k0 < n; k0 += nb) {
                const int nk = std::min(nb, n - k0);
                mdwf_solver_opts ok = o;   // the time limit covers the whole call
                if (o.max_seconds > 0.0) ok.max_seconds = std::max(1e-9, o.max_seconds - (now() - t_start));
                if (o.x_ref) ok.x_ref = o.x_ref + k0;
                PointIO pk{};
                if (pt) pk = PointIO{pt->src + 5 * k0, pt->q + k0};
                const mdwf_status r = mdwf_solve_impl(c, nk, pt ? nullptr : b_in + k0, pt ? nullptr : x_out + k0, host_io,
                                                      mq ? mq + k0 : nullptr, &ok, info ? info + k0 : nullptr, st,
                                                      pt ? &pk : nullptr);
                if (r != MDWF_OK && r != MDWF_ERR_NOCONV && r != MDWF_ERR_NUMERIC) return r;
                if (r != MDWF_OK && worst == MDWF_OK) worst = r;
            }
            return worst;
        }
    }
    S.chunk = n;
    if (need_fixed + size_t(n) * plan.tmp_per_rhs > avail) {
        const size_t room = avail > need_fixed ? avail - need_fixed : 0;
        S.chunk = int(std::max<size_t>(1, room / plan.tmp_per_rhs));
        if (S.chunk > n) S.chunk = n;
    }
    if (const char* e = std::getenv("MDWF_SOLVE_CHUNK")) {   // explicit chunk (memory / tests)
        const int v = std::atoi(e);
        if (v >= 1) S.chunk = std::min(v, n);
    }

    mdwf_status s = MDWF_OK;
#define ALLOC(var, name, bytes)                                       \
    S.var = static_cast<decltype(S.var)>(buf(c, name, (bytes), &s)); \
    if (!S.var) return s;
    ALLOC(xh, "sv_xh", S.H64 * n);
    ALLOC(bp, "sv_bp", S.H64 * n);
    if (S.mixed) {
        ALLOC(r, "sv_r", S.Hi * n);
        ALLOC(p, "sv_p", S.Hi * n);
        ALLOC(p2, "sv_p2", S.Hi * n);
        ALLOC(s, "sv_s", S.Hi * n);
        ALLOC(q, "sv_q", S.Hi * n);
        ALLOC(xl, "sv_xl", S.Hx * n);
        ALLOC(t, "sv_t", S.Hi * S.chunk);
    } else {
        ALLOC(r, "sv_r64", S.H64 * n);
        ALLOC(p, "sv_p64", S.H64 * n);
        ALLOC(p2, "sv_p2_64", S.H64 * n);
        ALLOC(s, "sv_s64", S.H64 * n);
        ALLOC(q, "sv_q64", S.H64 * n);
        ALLOC(t, "sv_t64c", S.H64 * S.chunk);
        S.xl = nullptr;
    }
    ALLOC(be, "sv_be", S.H64);
    ALLOC(bo, "sv_bo", S.H64);
    ALLOC(rh, "sv_rh", S.H64);
    ALLOC(t64, "sv_t64", S.H64);
    ALLOC(ye, "sv_ye", S.H64);
    ALLOC(xo, "sv_xo", S.H64);
    if (host_io) {
        ALLOC(canon, "sv_canon", S.canon_bytes);
    }
    if (o.x_ref)
        for (int k = 0; k < n; ++k)
            if (!o.x_ref[k]) return fail(c, MDWF_ERR_ARG, "null reference solution pointer");
    ALLOC(coef, "sv_coef", 2 * sizeof(RhsCoef) * n);
    ALLOC(sc, "sv_scal", sizeof(CGScal) * n);
    ALLOC(act, "sv_act", sizeof(int) * n);
    ALLOC(msk, "sv_msk", sizeof(int) * n);
    ALLOC(part, "sv_part", sizeof(double) * n * (S.nbh > S.nbb ? S.nbh : S.nbb));
    ALLOC(sums, "sv_sums", sizeof(double) * n);
#undef ALLOC
    const size_t pin_bytes = 2 * sizeof(CGScal) * n + sizeof(double) * n + sizeof(int) * n + 2 * sizeof(RhsCoef) * n + 64;
    char* hp = static_cast<char*>(pinned(c, pin_bytes, &s));
    if (!hp) return s;
    S.hsc[0] = reinterpret_cast<CGScal*>(hp);
    S.hsc[1] = S.hsc[0] + n;
    S.hsum = reinterpret_cast<double*>(S.hsc[1] + n);
    S.hmask = reinterpret_cast<int*>(S.hsum + n);
    RhsCoef* hcoef = reinterpret_cast<RhsCoef*>((reinterpret_cast<uintptr_t>(S.hmask + n) + 7) & ~uintptr_t(7));
    const bool sym = o.schur_form == 1;
    S.form = o.schur_form;
    for (int k = 0; k < n; ++k) {
        hcoef[k] = make_coef(c->act, masses[k]);
        hcoef[n + k] = make_coef_sym(c->act, masses[k]);
    }
    if (!S.hipok(hipMemcpyAsync(S.coef, hcoef, 2 * sizeof(RhsCoef) * n, hipMemcpyHostToDevice, st), "coef upload"))
        return S.err;
    // |K5| <= |a| + |b| |C| with |C| = max(1, m_q) = 1: a tracked K5^-1 r
    // below tgt |b| / knorm keeps |r| below tgt |b|
    const double knorm = sym ? std::fabs(hcoef[0].k5[0]) + std::fabs(hcoef[0].k5[1]) : 1.0;
    if (!S.hipok(hipMemsetAsync(S.sc, 0, sizeof(CGScal) * n, st), "memset")) return S.err;
    for (int e = 0; e < 2; ++e)
        if (!S.hipok(hipEventCreateWithFlags(&S.ev[e], hipEventDisableTiming), "event")) return S.err;

    std::vector<int> active(n, 1), done(n, 0), iters(n, 0), updates(n, 0), restarts(n, 0), stopped(n, 0);
    std::vector<double> true_res(n, -1.0), bnorm(n, 0.0), rmax(n, 0.0), err_ref(n, -1.0);

    // ---- source preparation, one RHS at a time: b'_e = b_e + 1/2 D_eo B K5^-1 b_o
    for (int k = 0; k < n && !S.err; ++k) {
        S.load_b(k);
        bnorm[k] = std::sqrt(S.norm2_one(P64, S.be) + S.norm2_one(P64, S.bo));
        launch_fifth(g, P64, FIFTH_K5INV, 0, S.bo, S.t64, S.H64, 1, S.coef + k, nullptr, st);
        HopLaunch L{};
        L.kind = HOP_PREP; L.prec = P64; L.out_parity = 0; L.out = S.bp + S.H64 * k; L.in = S.t64; L.centre = S.be;
        L.stride = S.H64; L.nrhs = 1; L.coef = S.coef + k; L.active = nullptr;
        launch_hop(g, c->gs, L, st);
        if (sym) {   // the symmetric system's source K5^-1 b'_e
            launch_fifth(g, P64, FIFTH_K5INV, 0, S.bp + S.H64 * k, S.t64, S.H64, 1, S.coef + k, nullptr, st);
            S.hipok(hipMemcpyAsync(S.bp + S.H64 * k, S.t64, S.H64, hipMemcpyDeviceToDevice, st), "source copy");
        }
        if (bnorm[k] == 0.0) {   // b = 0: x = 0 exactly
            active[k] = 0;
            done[k] = 1;
            true_res[k] = 0.0;
        }
        if (!std::isfinite(bnorm[k])) {
            active[k] = 0;
            stopped[k] = 2;
        }
    }
    S.hipok(hipMemsetAsync(S.xh, 0, S.H64 * n, st), "memset");
    if (S.mixed) S.hipok(hipMemsetAsync(S.xl, 0, S.Hx * n, st), "memset");
    // the odd-iteration buffer is read (times alpha_prev = 0) before a
    // restart has written it: start it finite
    S.hipok(hipMemsetAsync(S.p2, 0, S.Hi * n, st), "memset");
    int it = 0;   // CG iterations done; odd: an update alpha_prev p is pending
    S.upload_mask(S.act, active);
    if (S.err) return S.err;

    // Reliable update / restart for the RHS in `upd`: r_hi = b' - S x_hi in FP64
    // (one RHS at a time in the shared scratch), then r = r_hi in the inner
    // precision, s = S^+ r, gamma = |s|^2, and p = s where `restart_p`.
    auto refresh = [&](const std::vector<int>& upd, const std::vector<int>& restart_p) {
        S.upload_mask(S.msk, upd);
        if (it & 1) {   // the pending half of a two-iteration update (direction in p)
            launch_cg_xpend(g, S.mixed ? S.px : P64, S.pi, S.xcur(), S.sxc(), S.p, S.Hi, n, S.msk, S.sc, st);
            launch_scalars(SC_CLEAR_PREV, S.part, 0, n, S.msk, S.sc, nullptr, st);
        }
        if (S.mixed) launch_flush(g, S.px, S.xh, S.H64, S.xl, S.Hx, n, S.msk, st);
        std::vector<double> rr(n, 0.0);
        for (int k = 0; k < n; ++k) {
            if (!upd[k]) continue;
            S.schur(P64, S.xh + S.H64 * k, S.rh, S.t64, nullptr, S.H64, 1, k, nullptr, false, nullptr);
            launch_axpby(g, P64, 1.0, S.bp + S.H64 * k, -1.0, S.rh, S.rh, S.H64, 1, nullptr, S.part, st);
            rr[k] = S.fetch_sums(S.nbb, 1, nullptr)[0];
            launch_convert(g, P64, S.pi, S.rh, S.r + S.Hi * k, S.H64, S.Hi, 1, nullptr, st);
        }
        S.schur_inner(S.r, S.s, S.msk, true, S.part);
        launch_scalars(SC_SET_GAMMA, S.part, S.nbh, n, S.msk, S.sc, nullptr, st);
        std::vector<int> rp(n, 0);
        bool any_rp = false;
        for (int k = 0; k < n; ++k) {
            if (!upd[k]) continue;
            rmax[k] = std::sqrt(rr[k]);
            if (restart_p[k]) { rp[k] = 1; any_rp = true; }
        }
        if (any_rp) {   // into the buffer the next iteration reads
            S.upload_mask(S.msk, rp);
            launch_convert(g, S.pi, S.pi, S.s, (it & 1) ? S.p2 : S.p, S.Hi, S.Hi, n, S.msk, st);
        }
        return rr;
    };

    // FP64 true residual |b - D5 x| / |b| of RHS k (x_o reconstructed into
    // the scratch xo); with `write_x` the full solution goes to the caller.
    auto verify = [&](int k, bool write_x) {
        S.load_b(k);
        const char* xk = S.xh + S.H64 * k;
        if (S.form == 2) {   // x_e = B^-1 y
            launch_fifth(g, P64, FIFTH_BINV, 0, xk, S.rh, S.H64, 1, S.coef + k, nullptr, st);
            xk = S.rh;
        }
        HopLaunch L{};
        L.prec = P64; L.stride = S.H64; L.nrhs = 1; L.coef = S.coef + k; L.active = nullptr;
        L.kind = HOP_PREP; L.out_parity = 1; L.out = S.t64; L.in = xk; L.centre = S.bo;
        launch_hop(g, c->gs, L, st);
        launch_fifth(g, P64, FIFTH_K5INV, 0, S.t64, S.xo, S.H64, 1, S.coef + k, nullptr, st);
        L.kind = HOP_D5; L.out_parity = 0; L.out = S.ye; L.in = S.xo; L.centre = xk;
        launch_hop(g, c->gs, L, st);
        L.kind = HOP_D5; L.out_parity = 1; L.out = S.t64; L.in = xk; L.centre = S.xo;
        launch_hop(g, c->gs, L, st);
        launch_axpby(g, P64, 1.0, S.be, -1.0, S.ye, S.ye, S.H64, 1, nullptr, S.part, st);
        const double se = S.fetch_sums(S.nbb, 1, nullptr)[0];
        launch_axpby(g, P64, 1.0, S.bo, -1.0, S.t64, S.t64, S.H64, 1, nullptr, S.part, st);
        const double so = S.fetch_sums(S.nbb, 1, nullptr)[0];
        if (write_x && S.pt) {   // the wall field of the solution, to the host
            launch_wall_field(g, xk, S.xo, S.canon, st);
            S.hipok(hipMemcpyAsync(S.pt->q[k], S.canon, S.canon_bytes, hipMemcpyDeviceToHost, st), "q D2H");
            S.hipok(hipStreamSynchronize(st), "q write");
        } else if (write_x) {
            double* dst = host_io ? S.canon : x_out[k];
            launch_unpack_parity(g, P64, 1, 0, xk, dst, st);
            launch_unpack_parity(g, P64, 1, 1, S.xo, dst, st);
            if (host_io)
                S.hipok(hipMemcpyAsync(x_out[k], S.canon, S.canon_bytes, hipMemcpyDeviceToHost, st), "x D2H");
            S.hipok(hipStreamSynchronize(st), "x write");
            if (o.x_ref) {
                // ||x - x_ref|| / ||x_ref|| over both parities, x_ref packed
                // into the source scratch (free once the residual is known)
                const double* ref = o.x_ref[k];
                if (host_io) {
                    S.hipok(hipMemcpyAsync(S.canon, ref, S.canon_bytes, hipMemcpyHostToDevice, st), "x_ref H2D");
                    ref = S.canon;
                }
                launch_pack_parity(g, P64, 1, 0, ref, S.be, st);
                launch_pack_parity(g, P64, 1, 1, ref, S.bo, st);
                launch_axpby(g, P64, 1.0, xk, -1.0, S.be, S.ye, S.H64, 1, nullptr, S.part, st);
                const double de = S.fetch_sums(S.nbb, 1, nullptr)[0];
                launch_axpby(g, P64, 1.0, S.xo, -1.0, S.bo, S.t64, S.H64, 1, nullptr, S.part, st);
                const double dd = S.fetch_sums(S.nbb, 1, nullptr)[0];
                const double nr = S.norm2_one(P64, S.be) + S.norm2_one(P64, S.bo);
                err_ref[k] = nr > 0.0 ? std::sqrt((de + dd) / nr) : (de + dd > 0.0 ? INFINITY : 0.0);
            }
        }
        return bnorm[k] > 0.0 ? std::sqrt(se + so) / bnorm[k] : 0.0;
    };

    // initial residual and direction (x = 0, so r = b')
    {
        std::vector<int> all(active), rp(active);
        refresh(all, rp);
    }
    if (S.err) return S.err;

    // optional graphs of an even and an odd iteration
    bool use_graph = o.use_graph != 0;
    for (int odd = 0; odd < 2 && use_graph; ++odd) {
        if (!S.hipok(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "capture")) return S.err;
        S.one_iteration(odd == 1);
        hipError_t e = hipStreamEndCapture(st, &S.graph[odd]);
        if (!S.hipok(e, "capture end")) return S.err;
        if (!S.hipok(hipGraphInstantiate(&S.gexec[odd], S.graph[odd], nullptr, nullptr, 0), "graph instantiate"))
            return S.err;
    }

    // launch timing: sampled iterations from the third on, profile_every
    // apart (not with a graph)
    const int nprof = use_graph ? 0 : std::max(0, std::min(o.profile_iters, 64));
    const int pstride = std::max(1, o.profile_every);
    int prof_done = 0;
    for (int e = 0; e < 6 * nprof; ++e) {
        hipEvent_t ev;
        if (!S.hipok(hipEventCreate(&ev), "event")) return S.err;
        S.pev.push_back(ev);
    }

    const double tgt = 0.5 * o.tol / knorm;
    bool pending = false;
    int pend_slot = 0;
    // Each RHS's update schedule must depend on its own residuals only, so a
    // refresh of one RHS never shifts the checks of the others: after a
    // refresh, only the refreshed RHS skip the (pre-refresh) pending copy.
    std::vector<int> skip(n, 0);
    auto any_active = [&]() {
        for (int k = 0; k < n; ++k)
            if (active[k]) return true;
        return false;
    };
    while (any_active() && S.err == MDWF_OK) {
        if (use_graph) {
            S.hipok(hipGraphLaunch(S.gexec[it & 1], st), "graph launch");
        } else {
            S.prof = (it >= 2 && (it - 2) % pstride == 0 && prof_done < nprof) ? &S.pev[6 * prof_done++] : nullptr;
            S.one_iteration((it & 1) != 0);
            S.prof = nullptr;
        }
        ++it;
        for (int k = 0; k < n; ++k)
            if (active[k]) ++iters[k];
        const bool check = (it % o.check_every) == 0;
        int slot = it & 1;
        if (check) {
            S.hipok(hipMemcpyAsync(S.hsc[slot], S.sc, sizeof(CGScal) * n, hipMemcpyDeviceToHost, st), "scal D2H");
            S.hipok(hipEventRecord(S.ev[slot], st), "event");
        }
        // examine the previous check while this iteration runs
        if (!pending) {
            if (check) { pending = true; pend_slot = slot; }
            continue;
        }
        S.hipok(hipEventSynchronize(S.ev[pend_slot]), "event sync");
        const CGScal* h = S.hsc[pend_slot];
        pending = check;
        pend_slot = slot;
        std::vector<int> upd(n, 0), rp(n, 0);
        bool any = false;
        // past max_seconds every active RHS stops as if at max_iter
        const bool late = o.max_seconds > 0.0 && now() - t_start > o.max_seconds;
        auto limit = [&](int k) { return iters[k] >= o.max_iter || late; };
        for (int k = 0; k < n; ++k) {
            if (!active[k] || skip[k]) {
                skip[k] = 0;
                continue;
            }
            if (h[k].bad || !std::isfinite(h[k].rr)) {
                stopped[k] = 2;
                upd[k] = 1;
                any = true;
                continue;
            }
            const double rn = std::sqrt(h[k].rr);
            if (rn <= tgt * bnorm[k] || limit(k)) { upd[k] = 1; any = true; }
            else if (S.mixed && rn < o.delta * rmax[k]) { upd[k] = 1; any = true; }
        }
        if (!any) continue;
        // act on the current state (includes the iteration just enqueued)
        S.hipok(hipStreamSynchronize(st), "sync");
        auto rr = refresh(upd, rp);   // keeps p; restarts handled below
        for (int k = 0; k < n; ++k)
            if (upd[k]) skip[k] = pending ? 1 : 0;
        std::vector<int> again(n, 0), again_rp(n, 0);
        bool any_again = false, any_stop = false;
        for (int k = 0; k < n; ++k) {
            if (!upd[k]) continue;
            if (S.mixed) ++updates[k];
            if (std::sqrt(rr[k]) <= tgt * bnorm[k] || limit(k) || stopped[k] == 2) {
                const double tr = verify(k, false);
                true_res[k] = tr;
                if (tr <= o.tol) { done[k] = 1; active[k] = 0; any_stop = true; }
                else if (limit(k) || stopped[k] == 2) {
                    active[k] = 0;
                    any_stop = true;
                    if (!stopped[k]) stopped[k] = 1;
                } else { ++restarts[k]; again[k] = 1; again_rp[k] = 1; any_again = true; }
            }
        }
        if (any_again) refresh(again, again_rp);   // restart p = s from the true residual
        if (any_stop) S.upload_mask(S.act, active);
    }
    if (S.err) return S.err;

    // mean launch durations of the sampled iterations (all complete by now)
    double hop_us[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = 0; j < prof_done && !S.err; ++j) {
        S.hipok(hipEventSynchronize(S.pev[6 * j + 5]), "event sync");
        for (int q = 0; q < 4; ++q) {
            const int e0 = 6 * j + 3 * (q / 2) + (q % 2);
            float ms = 0.f;
            S.hipok(hipEventElapsedTime(&ms, S.pev[e0], S.pev[e0 + 1]), "event time");
            hop_us[q] += 1e3 * ms / prof_done;
        }
    }

    // reconstruct every RHS, verify and write x
    for (int k = 0; k < n && !S.err; ++k) true_res[k] = verify(k, true);
    for (int odd = 0; odd < 2; ++odd) {
        if (S.gexec[odd]) (void)hipGraphExecDestroy(S.gexec[odd]);
        if (S.graph[odd]) (void)hipGraphDestroy(S.graph[odd]);
    }
    for (int e = 0; e < 2; ++e) (void)hipEventDestroy(S.ev[e]);
    if (S.err) return S.err;

    const double secs = now() - t_start;
    mdwf_status result = MDWF_OK;
    // model counts per RHS
    const double bsI = spinor_site_bytes(S.pi), bsX = spinor_site_bytes(S.px), bs64 = spinor_site_bytes(P64);
    const double blI = link_site_bytes(S.pi, g.L5), bl64 = link_site_bytes(P64, g.L5);
    // A, B, A^+, B^+ (10 inner fields), r -= alpha q (3), the direction update
    // (3 inner fields) and, every second iteration, x read and written with
    // one more inner read: 16.5 inner fields and one x field per iteration.
    // The four hop launches read the links once for all RHS of a chunk, so
    // an RHS is charged its share of them.
    const double rpl = double(std::min(S.chunk, n));
    const double it_bytes = g.Vh * (16.5 * bsI + bsX + 4 * blI / rpl);
    const double it_flops = g.Vh * (2 * (2832.0 + 48.0 * g.L5) + 5 * 48.0);
    // reliable update: FP64 S on one RHS (5 fields, 2 link sets), r_hi =
    // b' - S x (3), conversion (FP64 read, inner write), the batched inner
    // S^+ (5 inner fields, its share of 2 link sets), the flush x_hi += x_lo
    const double up_bytes = g.Vh * (5 * bs64 + 2 * bl64 + 3 * bs64 + bs64 + bsI + 5 * bsI + 2 * blI / rpl +
                                    2 * bs64 + 2 * bsX);
    const double up_flops = g.Vh * (2 * (2832.0 + 48.0 * g.L5) + 3 * 48.0);
    for (int k = 0; k < n; ++k) {
        if (stopped[k] == 2) result = MDWF_ERR_NUMERIC;
        else if (!done[k] && result == MDWF_OK) result = MDWF_ERR_NOCONV;
        if (info) {
            info[k].iters = iters[k];
            info[k].reliable_updates = updates[k];
            info[k].restarts = restarts[k];
            info[k].true_resid = true_res[k];
            info[k].seconds = secs;
            info[k].model_bytes = iters[k] * it_bytes + (updates[k] + restarts[k] + 1) * up_bytes;
            info[k].model_flops = iters[k] * it_flops + (updates[k] + restarts[k] + 1) * up_flops;
            for (int q = 0; q < 4; ++q) info[k].hop_us[q] = hop_us[q];
            info[k].hop_rhs = prof_done ? std::min(S.chunk, n) : 0;
            info[k].hop_samples = prof_done;
            info[k].err_vs_ref = err_ref[k];
            info[k].launch_rhs = std::min(S.chunk, n);
        }
    }
    if (result == MDWF_ERR_NOCONV) fail(c, result, "solver reached max_iter before the target residual");
    if (result == MDWF_ERR_NUMERIC) fail(c, result, "non-finite value or breakdown in the CG recursion");
    return result;
}
