// Context object behind the opaque mdwf_ctx handle.
#pragma once

#include <map>
#include <string>
#include <vector>

#include "../../include/mdwf.h"
#include "mdwf_internal.h"

struct mdwf_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    mdwf_geometry geom{};
    mdwf::Geo geo{};
    bool have_action = false;
    mdwf_action act{};
    bool have_gauge = false;
    mdwf::GaugeSet gs;
    void* gauge_mem = nullptr;
    std::string err;

    // grow-only named device buffers
    struct Buf {
        void* p = nullptr;
        size_t n = 0;
    };
    std::map<std::string, Buf> bufs;

    // per-RHS coefficient table of the context's own action (one entry)
    mdwf::RhsCoef* d_coef1 = nullptr;   // [2]: S, then K5^-1 S
    // pinned host staging for scalars
    void* h_pin = nullptr;
    size_t h_pin_n = 0;
    // autotuned time of one Schur application per precision (0 = not tuned)
    double tuned_us[3] = {0.0, 0.0, 0.0};
};

namespace mdwf {

// Error helpers: record a message on the context and return a status.
mdwf_status fail(mdwf_ctx* c, mdwf_status st, const std::string& msg);
mdwf_status hip_check(mdwf_ctx* c, hipError_t e, const char* what);

// Device buffer of at least n bytes under `name` (contents undefined after growth).
void* buf(mdwf_ctx* c, const std::string& name, size_t n, mdwf_status* st);
void* pinned(mdwf_ctx* c, size_t n, mdwf_status* st);

// Coefficients of the fifth-dimension polynomials for mass mq.
RhsCoef make_coef(const mdwf_action& a, double mq);
RhsCoef make_coef_sym(const mdwf_action& a, double mq);   // kernel B of K5^-1 S
void schur_launch(const Geo& g, const GaugeSet& gs, Prec p, int form, bool dag, const void* in, void* out,
                  void* tmp, void* tmp2, size_t stride, int nrhs, const RhsCoef* cf, const RhsCoef* cfs,
                  const int* active, double* partials, hipStream_t st, hipEvent_t* evs = nullptr);

// Install a launch shape for one precision in the geometry.
void set_tune(Geo& g, Prec p, const mdwf_launch_tune& t);

// Native-layout operator application on `nrhs` right-hand sides stored at
// byte stride `stride` (half fields; a full field is two consecutive halves of
// half_field_bytes each and `stride` then covers both).  For the symmetric
// Schur ops d_coef holds nrhs action tables followed by nrhs make_coef_sym
// tables.
// scratch_mem: device memory for the Schur ops' odd intermediate(s) (two
// fields of nrhs for the symmetric adjoint); nullptr = the context's own
// grow-only buffers.
mdwf_status apply_native(mdwf_ctx* c, mdwf_op op, Prec p, const void* in, void* out, size_t stride, int nrhs,
                         const RhsCoef* d_coef, const int* d_active, hipStream_t st, void* scratch_mem = nullptr);

// Model counts (per application, all right-hand sides counted once).
void op_model(const Geo& g, mdwf_op op, Prec p, double* flops, double* bytes);
double spinor_site_bytes(Prec p);
double link_site_bytes(Prec p, int L5);

}  // namespace mdwf

// Point-source solves: RHS k is spin-colour column src[5k+4] of a unit point
// source at (x, y, z, t) = src[5k..5k+3], generated on the device; its
// solution's wall field q = P- x_0 + P+ x_{L5-1} goes to q[k] (host
// canonical 4D) instead of a 5D x.
struct PointIO {
    const int* src;
    double* const* q;
};

// host_io: b and x are host pointers, streamed through one device staging
// field; pt (b, x unused): point sources and wall-field outputs on the host
mdwf_status mdwf_solve_impl(mdwf_ctx* c, int nrhs, const double* const* b, double* const* x, bool host_io,
                            const double* mq, const mdwf_solver_opts* o, mdwf_solve_info* info, hipStream_t st,
                            const PointIO* pt = nullptr);

namespace mdwf {
// Device memory plan of a solve (bytes): per_rhs resident vectors of one RHS,
// shared FP64 scratch (and host I/O staging), the hop temporary per RHS of a
// launch chunk, and a margin for the small tables.
struct SolvePlan {
    size_t per_rhs, shared, tmp_per_rhs, margin;
};
// Where a solve's right-hand sides and solutions live: device canonical 5D
// fields, host canonical 5D fields (one 5D staging field), or point sources
// with host 4D wall fields (one 4D staging field).
enum SolveIo { IO_DEVICE = 0, IO_HOST = 1, IO_POINT = 2 };
SolvePlan solve_plan(const Geo& g, Prec inner, int io);
// Device bytes a solve of nrhs RHS allocates (solver vectors, shared
// scratch, hop temporary for all RHS at once), as its memory plan counts them.
size_t solve_footprint(const Geo& g, Prec inner, int nrhs, int io);
// Geometry of a lattice at fifth-dimension extent L5 (sizes only: enough for
// memory plans, not for launches).
Geo plan_geo(const mdwf_geometry& geom, int L5);
// Free the solver's device buffers held by the context (grow-only otherwise).
void release_solver_buffers(mdwf_ctx* c);
// Make dst use src's resident links (same geometry; src must outlive dst).
void share_gauge(mdwf_ctx* dst, const mdwf_ctx* src);
// Device bytes of the resident links of a context.
size_t gauge_bytes(const mdwf_ctx* c);
}  // namespace mdwf
