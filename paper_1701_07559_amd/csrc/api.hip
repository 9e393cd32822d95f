// C ABI of libmdwf: context, gauge upload, action, operator application.
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <mutex>
#include <new>
#include <vector>

#include "ctx.h"

using namespace mdwf;

static thread_local std::string g_create_err;

// ------------------------------------------ allocation-free scratch memory
// Device scratch of mdwf_apply_dev_noalloc: the odd-parity intermediate of the
// Schur operators (two of them for the symmetric adjoint), for callers that
// cannot allocate.  Each device holds its own copy for the life of the
// process.  On the host the array's name is only a stand-in for the symbol:
// its device address is looked up once per device (scratch_init, from
// mdwf_create) and only that address is handed to kernels.
static constexpr size_t kStaticScratchBytes = size_t(MDWF_STATIC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
bool g_scratch_done[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
void* g_scratch_ptr[kMaxDevices] = {};

// With `dev` current: the device address of its copy of the scratch array.
void scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[dev]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) (void)hipGetLastError();
    g_scratch_err[dev] = e;
    g_scratch_ptr[dev] = e == hipSuccess ? p : nullptr;
    g_scratch_done[dev] = true;
}

void* scratch_ptr(int dev, hipError_t* err) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices || !g_scratch_done[dev]) {
        *err = hipErrorNotInitialized;
        return nullptr;
    }
    *err = g_scratch_err[dev];
    return g_scratch_ptr[dev];
}
}  // namespace

namespace mdwf {

mdwf_status fail(mdwf_ctx* c, mdwf_status st, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_err = msg;
    return st;
}

mdwf_status hip_check(mdwf_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return MDWF_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(c, e == hipErrorOutOfMemory ? MDWF_ERR_OOM : MDWF_ERR_HIP, m);
}

void* buf(mdwf_ctx* c, const std::string& name, size_t n, mdwf_status* st) {
    auto& b = c->bufs[name];
    if (b.n >= n && b.p) return b.p;
    if (b.p) {
        // launches already enqueued (on any stream) may still read the
        // smaller buffer: let them finish before it goes
        (void)hipDeviceSynchronize();
        (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.n = 0;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, n < 256 ? 256 : n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *st = fail(c, MDWF_ERR_OOM, "device allocation of " + std::to_string(n) + " bytes for '" + name + "' failed");
        return nullptr;
    }
    b.p = p;
    b.n = n;
    return p;
}

void* pinned(mdwf_ctx* c, size_t n, mdwf_status* st) {
    if (c->h_pin_n >= n) return c->h_pin;
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    c->h_pin = nullptr;
    c->h_pin_n = 0;
    if (hipHostMalloc(&c->h_pin, n, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        *st = fail(c, MDWF_ERR_OOM, "pinned host allocation failed");
        return nullptr;
    }
    c->h_pin_n = n;
    return c->h_pin;
}

// K5 = (4 - M5) B + 1 - C = a + b C.  Its inverse on each chirality, using
// C^L5 = -m_q: K5^-1 = [a (1 + m_q z^L5)]^-1 sum_{k<L5} z^k C^k, z = -b/a;
// B K5^-1 is the product of the two polynomials reduced with C^L5 = -m_q.
RhsCoef make_coef(const mdwf_action& a, double mq) {
    RhsCoef c;
    std::memset(&c, 0, sizeof(c));
    const int L5 = a.L5;
    c.mq = mq;
    c.b5 = a.b5;
    c.c5 = a.c5;
    const double ka = 1.0 + a.b5 * (4.0 - a.M5);
    const double kb = a.c5 * (4.0 - a.M5) - 1.0;
    c.k5[0] = ka;
    c.k5[1] = kb;
    const double z = -kb / ka;
    const double norm = 1.0 / (ka * (1.0 + mq * std::pow(z, L5)));
    double zk = 1.0;
    for (int k = 0; k < L5; ++k) {
        c.kinv[k] = zk * norm;
        zk *= z;
    }
    c.m[0] = a.b5 * c.kinv[0] - mq * a.c5 * c.kinv[L5 - 1];
    for (int k = 1; k < L5; ++k) c.m[k] = a.b5 * c.kinv[k] + a.c5 * c.kinv[k - 1];
    // B = b5 + c5 C has the same closed-form inverse with (a, b) -> (b5, c5);
    // K5 B^-1 is again reduced with C^L5 = -m_q
    const double zb = -a.c5 / a.b5;
    double zbl = 1.0;
    for (int k = 0; k < L5; ++k) zbl *= zb;
    const double nb = 1.0 / (a.b5 * (1.0 + mq * zbl));
    double zbk = 1.0;
    for (int k = 0; k < L5; ++k) {
        c.binv[k] = zbk * nb;
        zbk *= zb;
    }
    c.w[0] = ka * c.binv[0] - mq * kb * c.binv[L5 - 1];
    for (int k = 1; k < L5; ++k) c.w[k] = ka * c.binv[k] + kb * c.binv[k - 1];
    return c;
}

// Table of the second kernel of the symmetric Schur form (Sec. VII names
// both even-odd forms) K5^-1 S = 1 - 1/4 K5^-1 D_eo (B K5^-1) D_oe B: its
// dense epilogue is K5^-1 (m = kinv) and its centre term the identity
// (k5 = 1 + 0 C).  K5^-1 does not commute with the hop (C carries the chiral
// projectors, the hop's 1 -+ gamma_mu flips chirality), so it is applied
// after the hop, in kernel B; the adjoint S^+ K5^-+ applies K5^-+ to the
// input first and uses this table's k5 for its centre term, which is then
// the untransformed input.
RhsCoef make_coef_sym(const mdwf_action& a, double mq) {
    RhsCoef c = make_coef(a, mq);
    for (int k = 0; k < kMaxL5; ++k) c.m[k] = c.kinv[k];
    c.k5[0] = 1.0;
    c.k5[1] = 0.0;
    return c;
}

double spinor_site_bytes(Prec p) { return p == P64 ? 192.0 : p == P32 ? 96.0 : 52.0; }
double link_site_bytes(Prec p, int L5) { return (p == P64 ? 8.0 : p == P32 ? 4.0 : 2.0) * 144.0 / L5; }

// Algorithmic model: every field is read or written once per kernel, links
// are 18 reals each (8 per site, shared by the L5 slices); flops count the
// Wilson hop as 1320 per 5D site (8 directions x (12 projection + 132 SU(3))
// + 168 accumulation), 72 for B or K5, 48 L5 for a dense L5 polynomial, 48
// for a combine, 48 per norm.
void op_model(const Geo& g, mdwf_op op, Prec p, double* flops, double* bytes) {
    const double Vh = g.Vh, L5 = g.L5;
    const double bs = spinor_site_bytes(p), bl = link_site_bytes(p, g.L5);
    double f = 0, b = 0;
    switch (op) {
        case MDWF_OP_HOP_EO: case MDWF_OP_HOP_OE: case MDWF_OP_HOP_EO_DAG: case MDWF_OP_HOP_OE_DAG:
            f = 1320; b = 2 * bs + bl; break;
        case MDWF_OP_D5: f = 2 * (1320 + 72 + 72 + 48); b = 2 * (3 * bs + bl); break;
        case MDWF_OP_D5_DAG: f = 2 * (1320 + 72 + 72 + 48); b = 2 * (3 * bs + bl); break;
        case MDWF_OP_SCHUR: case MDWF_OP_SCHUR_DAG: case MDWF_OP_SCHUR_SYM: case MDWF_OP_SCHUR_SYM_DAG:
            f = (1320 + 72 + 48 * L5) + (1320 + 72 + 48); b = (2 * bs + bl) + (3 * bs + bl); break;
        case MDWF_OP_SCHUR_RP: case MDWF_OP_SCHUR_RP_DAG:
            f = (1320 + 48 * L5) + (1320 + 48 * L5 + 48); b = (2 * bs + bl) + (3 * bs + bl); break;
        case MDWF_OP_BINV: case MDWF_OP_BINV_DAG:
            f = 2 * 48 * L5; b = 2 * 2 * bs; break;
        case MDWF_OP_K5: case MDWF_OP_K5_DAG: case MDWF_OP_B: case MDWF_OP_B_DAG:
            f = 2 * 72; b = 2 * 2 * bs; break;
        case MDWF_OP_K5INV: case MDWF_OP_K5INV_DAG:
            f = 2 * 48 * L5; b = 2 * 2 * bs; break;
        default: break;
    }
    *flops = f * Vh;
    *bytes = b * Vh;
}

bool tile_fits(const Geo& g, const int b[4]) {
    const int ext[4] = {g.Xh, g.Y, g.Z, g.T};
    for (int k = 0; k < 4; ++k)
        if (b[k] < 1 || ext[k] % b[k] != 0) return false;
    return true;
}

void set_tune(Geo& g, Prec p, const mdwf_launch_tune& t) {
    Trav& tr = g.trav[p];
    for (int k = 0; k < 4; ++k) tr.b[k] = t.tile[k];
    tr.fTv = FastDiv(uint32_t(t.tile[0] * t.tile[1] * t.tile[2] * t.tile[3]));
    tr.fBx = FastDiv(uint32_t(t.tile[0]));
    tr.fBy = FastDiv(uint32_t(t.tile[1]));
    tr.fBz = FastDiv(uint32_t(t.tile[2]));
    tr.fNt = FastDiv(uint32_t(g.T / t.tile[3]));
    tr.fNx = FastDiv(uint32_t(g.Xh / t.tile[0]));
    tr.fNy = FastDiv(uint32_t(g.Y / t.tile[1]));
    g.xcd_remap[p] = t.xcd_remap ? 1 : 0;
    g.nt_store[p] = t.nt_store ? 1 : 0;
    g.link_mode[p] = (t.link_mode >= 0 && t.link_mode <= 3) ? t.link_mode : 0;
    g.rhs_group[p] = t.rhs_group > 0 ? t.rhs_group : 0;
    g.plane_bt[p] = (t.plane_bt > 0 && g.T % t.plane_bt == 0) ? t.plane_bt : 0;
}

void release_solver_buffers(mdwf_ctx* c) {
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    c->bufs.clear();
}

void share_gauge(mdwf_ctx* dst, const mdwf_ctx* src) {
    dst->gs = src->gs;
    dst->have_gauge = src->have_gauge;
    dst->gauge_mem = nullptr;   // borrowed: src frees it
}

size_t gauge_bytes(const mdwf_ctx* c) {
    size_t tot = 0;
    for (int p = 0; p < 3; ++p) tot += 8 * link_segment_bytes(Prec(p), c->geo.Vh4);
    return tot + 16 * link_rows_bytes(c->geo.Vh4);
}

// The even-odd operator of Schur form `form` or its adjoint on nrhs fields
// `stride` apart: 0 = S, S^+; 1 = K5^-1 S, S^+ K5^-+ (symmetric); 2 = S B^-1,
// B^-+ S^+ (right preconditioning by B).  Kernel A writes tmp, then kernel B
// writes out with block norm partials of out when `partials` is set.  cf: the
// action's tables; cfs: the symmetric form's (make_coef_sym).  The symmetric
// adjoint first writes K5^-+ in to tmp2.  evs: optional events around the two
// hop launches.
void schur_launch(const Geo& g, const GaugeSet& gs, Prec p, int form, bool dag, const void* in, void* out,
                  void* tmp, void* tmp2, size_t stride, int nrhs, const RhsCoef* cf, const RhsCoef* cfs,
                  const int* active, double* partials, hipStream_t st, hipEvent_t* evs) {
    const bool sym = form == 1, rp = form == 2;
    HopLaunch L{};
    L.prec = p;
    L.stride = stride;
    L.nrhs = nrhs;
    L.active = active;
    const void* ain = in;
    if (sym && dag) {
        launch_fifth(g, p, FIFTH_K5INV, 1, in, tmp2, stride, nrhs, cf, active, st);
        ain = tmp2;
    }
    if (evs) (void)hipEventRecord(evs[0], st);
    L.kind = dag ? HOP_SCHUR_A_DAG : (rp ? HOP_SCHUR_A_RP : HOP_SCHUR_A);
    L.coef = cf;
    L.out_parity = 1; L.out = tmp; L.in = ain; L.centre = nullptr; L.partials = nullptr;
    launch_hop(g, gs, L, st);
    if (evs) (void)hipEventRecord(evs[1], st);
    L.kind = rp ? (dag ? HOP_SCHUR_B_DAG_RP : HOP_SCHUR_B_RP)
                : (dag ? HOP_SCHUR_B_DAG : (sym ? HOP_SCHUR_B_SYM : HOP_SCHUR_B));
    L.coef = sym ? cfs : cf;
    L.out_parity = 0; L.out = out; L.in = tmp; L.centre = in; L.partials = partials;
    launch_hop(g, gs, L, st);
    if (evs) (void)hipEventRecord(evs[2], st);
}

mdwf_status apply_native(mdwf_ctx* c, mdwf_op op, Prec p, const void* in, void* out, size_t stride, int nrhs,
                         const RhsCoef* d_coef, const int* d_active, hipStream_t st, void* scratch_mem) {
    const Geo& g = c->geo;
    const size_t hb = half_field_bytes(p, g.Vh);
    const char* ie = static_cast<const char*>(in);
    const char* io = ie + hb;
    char* oe = static_cast<char*>(out);
    char* oo = oe + hb;
    HopLaunch L{};
    L.prec = p;
    L.stride = stride;
    L.nrhs = nrhs;
    L.coef = d_coef;
    L.active = d_active;
    L.partials = nullptr;
    mdwf_status s = MDWF_OK;
    switch (op) {
        case MDWF_OP_D5:
        case MDWF_OP_D5_DAG:
            L.kind = (op == MDWF_OP_D5) ? HOP_D5 : HOP_D5_DAG;
            L.out_parity = 0; L.out = oe; L.in = io; L.centre = ie;
            launch_hop(g, c->gs, L, st);
            L.out_parity = 1; L.out = oo; L.in = ie; L.centre = io;
            launch_hop(g, c->gs, L, st);
            break;
        case MDWF_OP_SCHUR:
        case MDWF_OP_SCHUR_DAG:
        case MDWF_OP_SCHUR_SYM:
        case MDWF_OP_SCHUR_SYM_DAG:
        case MDWF_OP_SCHUR_RP:
        case MDWF_OP_SCHUR_RP_DAG: {
            const bool dag = op == MDWF_OP_SCHUR_DAG || op == MDWF_OP_SCHUR_SYM_DAG || op == MDWF_OP_SCHUR_RP_DAG;
            const bool sym = op == MDWF_OP_SCHUR_SYM || op == MDWF_OP_SCHUR_SYM_DAG;
            const int form = sym ? 1 : (op == MDWF_OP_SCHUR_RP || op == MDWF_OP_SCHUR_RP_DAG) ? 2 : 0;
            void* tmp = scratch_mem ? scratch_mem : buf(c, "apply_tmp", stride * nrhs, &s);
            if (!tmp) return s;
            void* tmp2 = nullptr;
            if (sym && dag) {
                tmp2 = scratch_mem ? static_cast<char*>(scratch_mem) + stride * nrhs
                                   : buf(c, "apply_tmp2", stride * nrhs, &s);
                if (!tmp2) return s;
            }
            schur_launch(g, c->gs, p, form, dag, in, out, tmp, tmp2, stride, nrhs, d_coef,
                         sym ? d_coef + nrhs : nullptr, d_active, nullptr, st);
            break;
        }
        case MDWF_OP_HOP_EO:
        case MDWF_OP_HOP_EO_DAG:
            L.kind = (op == MDWF_OP_HOP_EO) ? HOP_BARE : HOP_BARE_DAG;
            L.out_parity = 0; L.out = out; L.in = in; L.centre = nullptr;
            launch_hop(g, c->gs, L, st);
            break;
        case MDWF_OP_HOP_OE:
        case MDWF_OP_HOP_OE_DAG:
            L.kind = (op == MDWF_OP_HOP_OE) ? HOP_BARE : HOP_BARE_DAG;
            L.out_parity = 1; L.out = out; L.in = in; L.centre = nullptr;
            launch_hop(g, c->gs, L, st);
            break;
        case MDWF_OP_K5: case MDWF_OP_K5_DAG: case MDWF_OP_K5INV: case MDWF_OP_K5INV_DAG:
        case MDWF_OP_B: case MDWF_OP_B_DAG: case MDWF_OP_BINV: case MDWF_OP_BINV_DAG: {
            const FifthKind k = (op == MDWF_OP_K5 || op == MDWF_OP_K5_DAG) ? FIFTH_K5
                              : (op == MDWF_OP_B || op == MDWF_OP_B_DAG) ? FIFTH_B
                              : (op == MDWF_OP_BINV || op == MDWF_OP_BINV_DAG) ? FIFTH_BINV : FIFTH_K5INV;
            const int dag = (op == MDWF_OP_K5_DAG || op == MDWF_OP_K5INV_DAG || op == MDWF_OP_B_DAG ||
                             op == MDWF_OP_BINV_DAG) ? 1 : 0;
            launch_fifth(g, p, k, dag, ie, oe, stride, nrhs, d_coef, d_active, st);
            launch_fifth(g, p, k, dag, io, oo, stride, nrhs, d_coef, d_active, st);
            break;
        }
        default:
            return fail(c, MDWF_ERR_ARG, "unknown operator");
    }
    return hip_check(c, hipGetLastError(), "kernel launch");
}

}  // namespace mdwf

// ------------------------------------------------------------------ helpers
static bool op_schur(mdwf_op op) {
    return op == MDWF_OP_SCHUR || op == MDWF_OP_SCHUR_DAG || op == MDWF_OP_SCHUR_SYM || op == MDWF_OP_SCHUR_SYM_DAG ||
           op == MDWF_OP_SCHUR_RP || op == MDWF_OP_SCHUR_RP_DAG;
}
static bool op_full(mdwf_op op) {
    return !(op_schur(op) || op == MDWF_OP_HOP_EO || op == MDWF_OP_HOP_OE || op == MDWF_OP_HOP_EO_DAG ||
             op == MDWF_OP_HOP_OE_DAG);
}
static int op_in_kind(mdwf_op op) {
    if (op_schur(op)) return MDWF_HALF_EVEN;
    switch (op) {
        case MDWF_OP_HOP_EO: case MDWF_OP_HOP_EO_DAG: return MDWF_HALF_ODD;
        case MDWF_OP_HOP_OE: case MDWF_OP_HOP_OE_DAG: return MDWF_HALF_EVEN;
        default: return MDWF_FULL;
    }
}
static int op_out_kind(mdwf_op op) {
    if (op_schur(op)) return MDWF_HALF_EVEN;
    switch (op) {
        case MDWF_OP_HOP_EO: case MDWF_OP_HOP_EO_DAG: return MDWF_HALF_EVEN;
        case MDWF_OP_HOP_OE: case MDWF_OP_HOP_OE_DAG: return MDWF_HALF_ODD;
        default: return MDWF_FULL;
    }
}

static mdwf_status ready(mdwf_ctx* c) {
    if (!c) return fail(nullptr, MDWF_ERR_ARG, "null context");
    if (!c->have_action) return fail(c, MDWF_ERR_STATE, "mdwf_set_action has not been called");
    if (!c->have_gauge) return fail(c, MDWF_ERR_STATE, "mdwf_load_gauge has not been called");
    return hip_check(c, hipSetDevice(c->device), "hipSetDevice");
}

static bool valid_prec(int p) { return p == MDWF_F64 || p == MDWF_F32 || p == MDWF_F16; }

// ---------------------------------------------------------------- C ABI
extern "C" {

mdwf_status mdwf_create(const mdwf_geometry* geom, int hip_device, void* hip_stream, mdwf_ctx** out) {
    if (!out) return fail(nullptr, MDWF_ERR_ARG, "out is null");
    *out = nullptr;
    if (!geom) return fail(nullptr, MDWF_ERR_ARG, "geometry is null");
    const int L[4] = {geom->X, geom->Y, geom->Z, geom->T};
    for (int k = 0; k < 4; ++k)
        if (L[k] < 2 || (L[k] & 1))
            return fail(nullptr, MDWF_ERR_ARG, "every lattice extent must be even and >= 2");
    const double V = double(geom->X) * geom->Y * geom->Z * geom->T;
    if (V * 32 / 2 >= 2147483647.0) return fail(nullptr, MDWF_ERR_ARG, "lattice too large for 32-bit site indices");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
        (void)hipGetLastError();
        return fail(nullptr, MDWF_ERR_HIP, "no HIP device available");
    }
    if (hip_device < 0 || hip_device >= ndev) return fail(nullptr, MDWF_ERR_ARG, "hip_device out of range");
    mdwf_ctx* c = new (std::nothrow) mdwf_ctx();
    if (!c) return fail(nullptr, MDWF_ERR_OOM, "host allocation failed");
    c->device = hip_device;
    c->geom = *geom;
    if (hipSetDevice(hip_device) != hipSuccess) {
        delete c;
        return fail(nullptr, MDWF_ERR_HIP, "hipSetDevice failed");
    }
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(nullptr, MDWF_ERR_HIP, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    Geo& g = c->geo;
    g.X = geom->X; g.Y = geom->Y; g.Z = geom->Z; g.T = geom->T;
    g.Xh = geom->X / 2;
    g.Vh4 = int(V / 2);
    g.L5 = 0;
    g.Vh = 0;
    g.antiperiodic = geom->antiperiodic_t ? 1 : 0;
    g.fXh = FastDiv(uint32_t(g.Xh));
    g.fY = FastDiv(uint32_t(g.Y));
    g.fZ = FastDiv(uint32_t(g.Z));
    // default launch shape (mdwf_autotune refines it per precision): z-blocks
    // of 4 (or 2) planes with t inside; the MDWF_TILE ("bx,by,bz,bt"),
    // MDWF_XCD_REMAP, MDWF_NT_STORE, MDWF_LINK_MODE and MDWF_RHS_GROUP
    // variables override it
    mdwf_launch_tune t0{{g.Xh, g.Y, (g.Z % 4 == 0) ? 4 : 2, 1}, 1, 0, 0, 0, 0.0, 0};
    if (const char* e = std::getenv("MDWF_TILE")) {
        int b[4];
        if (std::sscanf(e, "%d,%d,%d,%d", &b[0], &b[1], &b[2], &b[3]) == 4 && tile_fits(g, b))
            for (int k = 0; k < 4; ++k) t0.tile[k] = b[k];
    }
    if (const char* e = std::getenv("MDWF_XCD_REMAP")) t0.xcd_remap = std::atoi(e) != 0;
    if (const char* e = std::getenv("MDWF_NT_STORE")) t0.nt_store = std::atoi(e) != 0;
    if (const char* e = std::getenv("MDWF_LINK_MODE")) t0.link_mode = std::atoi(e);
    if (const char* e = std::getenv("MDWF_RHS_GROUP")) t0.rhs_group = std::atoi(e);
    if (const char* e = std::getenv("MDWF_PLANE_BT")) t0.plane_bt = std::atoi(e);
    for (int p = 0; p < 3; ++p) set_tune(g, Prec(p), t0);
    scratch_init(hip_device);   // the device address of this device's static scratch
    if (hipMalloc(&c->d_coef1, 2 * sizeof(RhsCoef)) != hipSuccess) {
        (void)hipGetLastError();
        mdwf_destroy(c);
        return fail(nullptr, MDWF_ERR_OOM, "device allocation failed");
    }
    *out = c;
    return MDWF_OK;
}

void mdwf_destroy(mdwf_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto& kv : c->bufs)
        if (kv.second.p) (void)hipFree(kv.second.p);
    if (c->gauge_mem) (void)hipFree(c->gauge_mem);
    if (c->d_coef1) (void)hipFree(c->d_coef1);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char* mdwf_last_error(const mdwf_ctx* c) { return c ? c->err.c_str() : g_create_err.c_str(); }

void mdwf_default_opts(mdwf_solver_opts* o) {
    if (!o) return;
    o->tol = 1e-10;
    o->max_iter = 100000;
    o->inner = MDWF_F64;
    o->delta = 0.1;
    o->check_every = 1;
    o->use_graph = 0;
    o->profile_iters = 0;
    o->schur_form = 0;
    o->max_seconds = 0.0;
    o->x_ref = nullptr;
    o->profile_every = 0;
}

mdwf_status mdwf_solve_footprint(const mdwf_geometry* geom, int L5, mdwf_prec inner, int nrhs, int host_io,
                                 size_t* bytes) {
    if (!geom || !bytes || nrhs < 1 || L5 < 1 || L5 > kMaxL5 || !valid_prec(inner)) return MDWF_ERR_ARG;
    const int L[4] = {geom->X, geom->Y, geom->Z, geom->T};
    for (int k = 0; k < 4; ++k)
        if (L[k] < 2 || (L[k] & 1)) return MDWF_ERR_ARG;
    if (host_io < 0 || host_io > 2) return MDWF_ERR_ARG;
    *bytes = solve_footprint(plan_geo(*geom, L5), Prec(inner), nrhs, host_io);
    return MDWF_OK;
}

static mdwf_status load_gauge_common(mdwf_ctx* c, const double* U, bool on_device) {
    if (!c) return fail(nullptr, MDWF_ERR_ARG, "null context");
    if (!U) return fail(c, MDWF_ERR_ARG, "gauge pointer is null");
    mdwf_status s = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
    if (s) return s;
    Geo& g = c->geo;
    size_t seg[3], tot = 0;
    for (int p = 0; p < 3; ++p) {
        seg[p] = link_segment_bytes(Prec(p), g.Vh4);
        tot += 8 * seg[p];
    }
    const size_t rows = link_rows_bytes(g.Vh4);
    tot += 16 * rows;
    if (!c->gauge_mem) {
        s = hip_check(c, hipMalloc(&c->gauge_mem, tot), "gauge allocation");
        if (s) return s;
    }
    char* base = static_cast<char*>(c->gauge_mem);
    for (int p = 0; p < 3; ++p) {
        c->gs.seg[p] = base;
        c->gs.seg_bytes[p] = seg[p];
        base += 8 * seg[p];
    }
    c->gs.mrow = base;
    c->gs.mrow_bytes = rows;
    const size_t canon_bytes = size_t(2) * g.Vh4 * 4 * 18 * sizeof(double);
    const double* src = U;
    if (!on_device) {
        void* stage = buf(c, "gauge_stage", canon_bytes, &s);
        if (!stage) return s;
        s = hip_check(c, hipMemcpyAsync(stage, U, canon_bytes, hipMemcpyHostToDevice, c->stream), "gauge H2D");
        if (s) return s;
        src = static_cast<const double*>(stage);
    }
    launch_gauge_layout(g, src, c->gs, c->stream);
    s = hip_check(c, hipGetLastError(), "gauge layout kernel");
    if (s) return s;
    s = hip_check(c, hipStreamSynchronize(c->stream), "gauge upload");
    if (s) return s;
    c->have_gauge = true;
    return MDWF_OK;
}

mdwf_status mdwf_load_gauge(mdwf_ctx* c, const double* U) { return load_gauge_common(c, U, false); }
mdwf_status mdwf_load_gauge_dev(mdwf_ctx* c, const double* U) { return load_gauge_common(c, U, true); }

mdwf_status mdwf_set_action(mdwf_ctx* c, const mdwf_action* a) {
    if (!c) return fail(nullptr, MDWF_ERR_ARG, "null context");
    if (!a) return fail(c, MDWF_ERR_ARG, "action is null");
    if (a->L5 < 1 || a->L5 > kMaxL5) return fail(c, MDWF_ERR_ARG, "L5 must be in [1, 32]");
    // the kernels address a 16-byte element of a field block with a 32-bit
    // byte offset (16 Vh bytes per block)
    if (double(c->geo.Vh4) * a->L5 * 16.0 >= 4294967296.0)
        return fail(c, MDWF_ERR_ARG, "V/2 x L5 too large for 32-bit field offsets (V/2 x L5 < 268435456)");
    if (!(a->c5 >= 0.0) || !(a->b5 > a->c5)) return fail(c, MDWF_ERR_ARG, "need b5 > c5 >= 0");
    if (!(a->mq >= 0.0 && a->mq <= 1.0)) return fail(c, MDWF_ERR_ARG, "need 0 <= mq <= 1");
    if (!(a->M5 > 0.0 && a->M5 < 2.0)) return fail(c, MDWF_ERR_ARG, "need 0 < M5 < 2");
    if (!std::isfinite(a->b5) || !std::isfinite(a->c5) || !std::isfinite(a->M5))
        return fail(c, MDWF_ERR_ARG, "non-finite action parameter");
    mdwf_status s = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
    if (s) return s;
    // launches already enqueued on the context's stream read the coefficient
    // table and the geometry's L5: let them finish before either changes
    s = hip_check(c, hipStreamSynchronize(c->stream), "stream sync");
    if (s) return s;
    c->act = *a;
    c->geo.L5 = a->L5;
    c->geo.Vh = c->geo.Vh4 * a->L5;
    const RhsCoef cf[2] = {make_coef(*a, a->mq), make_coef_sym(*a, a->mq)};
    s = hip_check(c, hipMemcpyAsync(c->d_coef1, cf, sizeof(cf), hipMemcpyHostToDevice, c->stream),
                  "coefficient upload");
    if (s) return s;
    s = hip_check(c, hipStreamSynchronize(c->stream), "coefficient upload");
    if (s) return s;
    c->have_action = true;
    return MDWF_OK;
}

mdwf_status mdwf_field_bytes(const mdwf_ctx* c, mdwf_prec prec, mdwf_field_kind kind, size_t* bytes) {
    if (!c || !bytes) return fail(const_cast<mdwf_ctx*>(c), MDWF_ERR_ARG, "null argument");
    if (!valid_prec(prec)) return fail(const_cast<mdwf_ctx*>(c), MDWF_ERR_ARG, "bad precision");
    if (!c->have_action) return fail(const_cast<mdwf_ctx*>(c), MDWF_ERR_STATE, "mdwf_set_action has not been called");
    const size_t hb = half_field_bytes(Prec(prec), c->geo.Vh);
    *bytes = (kind == MDWF_FULL) ? 2 * hb : hb;
    return MDWF_OK;
}

mdwf_status mdwf_pack_dev(mdwf_ctx* c, mdwf_prec prec, mdwf_field_kind kind, const double* canon, void* native,
                          void* stream) {
    mdwf_status s = ready(c);
    if (s) return s;
    if (!valid_prec(prec) || kind < 0 || kind > 2 || !canon || !native) return fail(c, MDWF_ERR_ARG, "bad argument");
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
    launch_pack(c->geo, Prec(prec), kind, canon, native, st);
    return hip_check(c, hipGetLastError(), "pack kernel");
}

mdwf_status mdwf_unpack_dev(mdwf_ctx* c, mdwf_prec prec, mdwf_field_kind kind, const void* native, double* canon,
                            void* stream) {
    mdwf_status s = ready(c);
    if (s) return s;
    if (!valid_prec(prec) || kind < 0 || kind > 2 || !canon || !native) return fail(c, MDWF_ERR_ARG, "bad argument");
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
    launch_unpack(c->geo, Prec(prec), kind, native, canon, st);
    return hip_check(c, hipGetLastError(), "unpack kernel");
}

mdwf_status mdwf_apply_dev(mdwf_ctx* c, mdwf_op op, mdwf_prec prec, const void* in, void* out, void* stream) {
    mdwf_status s = ready(c);
    if (s) return s;
    if (!valid_prec(prec) || op < 0 || op >= MDWF_OP_COUNT) return fail(c, MDWF_ERR_ARG, "bad operator or precision");
    if (!in || !out) return fail(c, MDWF_ERR_ARG, "null field pointer");
    if (in == out) return fail(c, MDWF_ERR_ARG, "in and out must not overlap");
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
    const size_t hb = half_field_bytes(Prec(prec), c->geo.Vh);
    const size_t stride = op_full(op) ? 2 * hb : hb;
    return apply_native(c, op, Prec(prec), in, out, stride, 1, c->d_coef1, nullptr, st);
}

mdwf_status mdwf_apply_dev_noalloc(mdwf_ctx* c, mdwf_op op, mdwf_prec prec, const void* in, void* out,
                                   void* stream) {
    mdwf_status s = ready(c);
    if (s) return s;
    if (!valid_prec(prec) || op < 0 || op >= MDWF_OP_COUNT) return fail(c, MDWF_ERR_ARG, "bad operator or precision");
    if (!in || !out) return fail(c, MDWF_ERR_ARG, "null field pointer");
    if (in == out) return fail(c, MDWF_ERR_ARG, "in and out must not overlap");
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
    const size_t hb = half_field_bytes(Prec(prec), c->geo.Vh);
    const size_t stride = op_full(op) ? 2 * hb : hb;
    void* mem = nullptr;
    if (op_schur(op)) {
        const size_t need = (op == MDWF_OP_SCHUR_SYM_DAG ? 2 : 1) * stride;
        if (need > kStaticScratchBytes)
            return fail(c, MDWF_ERR_ARG, "the operator's intermediate needs " + std::to_string(need) +
                                             " bytes, more than the " + std::to_string(kStaticScratchBytes) +
                                             "-byte static scratch");
        hipError_t e = hipSuccess;
        mem = scratch_ptr(c->device, &e);
        if (!mem) return hip_check(c, e == hipSuccess ? hipErrorInvalidSymbol : e, "static scratch address");
    }
    return apply_native(c, op, Prec(prec), in, out, stride, 1, c->d_coef1, nullptr, st, mem);
}

mdwf_status mdwf_apply_batch_dev(mdwf_ctx* c, mdwf_op op, mdwf_prec prec, int nrhs, const void* in, void* out,
                                 size_t stride, const double* mq, void* stream) {
    mdwf_status s = ready(c);
    if (s) return s;
    if (!valid_prec(prec) || op < 0 || op >= MDWF_OP_COUNT) return fail(c, MDWF_ERR_ARG, "bad operator or precision");
    if (nrhs < 1) return fail(c, MDWF_ERR_ARG, "need nrhs >= 1");
    if (!in || !out) return fail(c, MDWF_ERR_ARG, "null field pointer");
    const size_t hb = half_field_bytes(Prec(prec), c->geo.Vh);
    const size_t fb = op_full(op) ? 2 * hb : hb;
    if (stride < fb || stride % 256 != 0)
        return fail(c, MDWF_ERR_ARG, "stride must be at least the field's bytes and a multiple of 256");
    const char* ib = static_cast<const char*>(in);
    char* ob = static_cast<char*>(out);
    const size_t span = stride * size_t(nrhs - 1) + fb;
    if (ib < ob + span && ob < ib + span) return fail(c, MDWF_ERR_ARG, "in and out must not overlap");
    std::vector<RhsCoef> hc(2 * size_t(nrhs));
    for (int k = 0; k < nrhs; ++k) {
        const double m = mq ? mq[k] : c->act.mq;
        if (!(m >= 0.0 && m <= 1.0)) return fail(c, MDWF_ERR_ARG, "need 0 <= mq <= 1");
        hc[k] = make_coef(c->act, m);
        hc[nrhs + k] = make_coef_sym(c->act, m);
    }
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
    RhsCoef* dc = static_cast<RhsCoef*>(buf(c, "batch_coef", hc.size() * sizeof(RhsCoef), &s));
    if (!dc) return s;
    if ((s = hip_check(c, hipMemcpyAsync(dc, hc.data(), hc.size() * sizeof(RhsCoef), hipMemcpyHostToDevice, st),
                       "coefficient upload")))
        return s;
    // the table is reused by the next call: keep the host copy alive until
    // the upload has read it
    if ((s = hip_check(c, hipStreamSynchronize(st), "coefficient upload"))) return s;
    return apply_native(c, op, Prec(prec), in, out, stride, nrhs, dc, nullptr, st);
}

mdwf_status mdwf_apply(mdwf_ctx* c, mdwf_op op, mdwf_prec prec, const double* in, double* out) {
    mdwf_status s = ready(c);
    if (s) return s;
    if (!valid_prec(prec) || op < 0 || op >= MDWF_OP_COUNT) return fail(c, MDWF_ERR_ARG, "bad operator or precision");
    if (!in || !out) return fail(c, MDWF_ERR_ARG, "null field pointer");
    const Geo& g = c->geo;
    const int ik = op_in_kind(op), ok = op_out_kind(op);
    const size_t full_canon = size_t(2) * g.Vh * 24 * sizeof(double);
    const size_t in_canon = ik == MDWF_FULL ? full_canon : full_canon / 2;
    const size_t out_canon = ok == MDWF_FULL ? full_canon : full_canon / 2;
    const size_t hb = half_field_bytes(Prec(prec), g.Vh);
    void* cin = buf(c, "apply_canon_in", in_canon, &s);
    if (!cin) return s;
    void* cout = buf(c, "apply_canon_out", out_canon, &s);
    if (!cout) return s;
    void* nin = buf(c, "apply_native_in", 2 * hb, &s);
    if (!nin) return s;
    void* nout = buf(c, "apply_native_out", 2 * hb, &s);
    if (!nout) return s;
    hipStream_t st = c->stream;
    if ((s = hip_check(c, hipMemcpyAsync(cin, in, in_canon, hipMemcpyHostToDevice, st), "H2D"))) return s;
    launch_pack(g, Prec(prec), ik, static_cast<const double*>(cin), nin, st);
    const size_t stride = op_full(op) ? 2 * hb : hb;
    if ((s = apply_native(c, op, Prec(prec), nin, nout, stride, 1, c->d_coef1, nullptr, st))) return s;
    launch_unpack(g, Prec(prec), ok, nout, static_cast<double*>(cout), st);
    if ((s = hip_check(c, hipGetLastError(), "unpack kernel"))) return s;
    if ((s = hip_check(c, hipMemcpyAsync(out, cout, out_canon, hipMemcpyDeviceToHost, st), "D2H"))) return s;
    return hip_check(c, hipStreamSynchronize(st), "apply");
}

mdwf_status mdwf_op_model(const mdwf_ctx* c, mdwf_op op, mdwf_prec prec, double* flops, double* bytes) {
    if (!c || !flops || !bytes) return fail(const_cast<mdwf_ctx*>(c), MDWF_ERR_ARG, "null argument");
    if (!c->have_action) return fail(const_cast<mdwf_ctx*>(c), MDWF_ERR_STATE, "mdwf_set_action has not been called");
    if (!valid_prec(prec) || op < 0 || op >= MDWF_OP_COUNT) return fail(const_cast<mdwf_ctx*>(c), MDWF_ERR_ARG, "bad operator or precision");
    op_model(c->geo, op, Prec(prec), flops, bytes);
    return MDWF_OK;
}

mdwf_status mdwf_get_tune(const mdwf_ctx* c, mdwf_prec prec, mdwf_launch_tune* out) {
    if (!c || !out) return fail(const_cast<mdwf_ctx*>(c), MDWF_ERR_ARG, "null argument");
    if (!valid_prec(prec)) return fail(const_cast<mdwf_ctx*>(c), MDWF_ERR_ARG, "bad precision");
    for (int k = 0; k < 4; ++k) out->tile[k] = c->geo.trav[prec].b[k];
    out->xcd_remap = c->geo.xcd_remap[prec];
    out->nt_store = c->geo.nt_store[prec];
    out->link_mode = c->geo.link_mode[prec];
    out->rhs_group = c->geo.rhs_group[prec];
    out->us = c->tuned_us[prec];
    out->plane_bt = c->geo.plane_bt[prec];
    return MDWF_OK;
}

mdwf_status mdwf_set_tune(mdwf_ctx* c, mdwf_prec prec, const mdwf_launch_tune* t) {
    if (!c || !t) return fail(c, MDWF_ERR_ARG, "null argument");
    if (!valid_prec(prec)) return fail(c, MDWF_ERR_ARG, "bad precision");
    if (!tile_fits(c->geo, t->tile)) return fail(c, MDWF_ERR_ARG, "tile extents must divide the lattice's");
    if (t->plane_bt < 0 || (t->plane_bt > 0 && c->geo.T % t->plane_bt))
        return fail(c, MDWF_ERR_ARG, "plane_bt must divide T");
    set_tune(c->geo, Prec(prec), *t);   // enqueued launches took the old shape by value
    c->tuned_us[prec] = t->us;
    return MDWF_OK;
}

}  // extern "C"

namespace {

// Coordinate-descent tuning of precision p's launch shape on the CG operator
// of Schur form `form` with nrhs RHS per launch (its adjoint too when
// `with_dag`): traversal tile (z-blocks and compact 4D tiles), link mode,
// non-temporal stores and workgroup numbering, then (nrhs > 1) the RHS
// grouping.  Each candidate: 2 warm-up applications, the mean of 5 timed.
// For one RHS without the adjoint (the operator tuning), FP32 and FP16 also
// choose the kernel of the bare hop (lane-per-site or plane-staged).
mdwf_status tune_precision(mdwf_ctx* c, Prec p, int form, int nrhs, bool with_dag, const double* cin,
                           hipEvent_t e0, hipEvent_t e1, mdwf_launch_tune* out) {
    Geo& g = c->geo;
    hipStream_t st = c->stream;
    mdwf_status s = MDWF_OK;
    std::vector<std::array<int, 4>> tiles;
    auto add_tile = [&](int bx, int by, int bz, int bt) {
        const int b4[4] = {bx, by, bz, bt};
        if (!tile_fits(g, b4)) return;
        for (const auto& t : tiles)
            if (t[0] == bx && t[1] == by && t[2] == bz && t[3] == bt) return;
        tiles.push_back({bx, by, bz, bt});
    };
    for (int v : {1, 2, 4, 8, 16}) add_tile(g.Xh, g.Y, v, 1);
    add_tile(g.Xh, g.Y, g.Z, 1);
    for (int bx : {g.Xh, g.Xh / 2})
        for (int by : {4, 6, 8, 12, g.Y})
            for (int bz : {2, 4, 6, 8})
                for (int bt : {1, 2, 4}) {
                    const long vol = long(bx) * by * bz * bt;
                    if (vol >= 384 && vol <= 6912 && (by < g.Y || bt > 1)) add_tile(bx, by, bz, bt);
                }
    const size_t hb = half_field_bytes(p, g.Vh);
    // scratch: nrhs even inputs (packed from the canonical pattern), outputs
    // of the operator and of its adjoint (the input is never overwritten, so
    // repeated applications do not grow it), odd temporaries and, for the
    // symmetric adjoint, one more even set
    char* a = static_cast<char*>(buf(c, "tune_a", hb * nrhs, &s));
    char* b = a ? static_cast<char*>(buf(c, "tune_b", hb * nrhs, &s)) : nullptr;
    char* d = (b && with_dag) ? static_cast<char*>(buf(c, "tune_d", hb * nrhs, &s)) : b;
    char* t = d ? static_cast<char*>(buf(c, "tune_t", hb * nrhs, &s)) : nullptr;
    char* t2 = (t && form == 1 && with_dag) ? static_cast<char*>(buf(c, "tune_t2", hb * nrhs, &s)) : t;
    RhsCoef* cf = t2 ? static_cast<RhsCoef*>(buf(c, "tune_coef", 2 * sizeof(RhsCoef) * nrhs, &s)) : nullptr;
    if (!cf) return s;
    std::vector<RhsCoef> hc(2 * size_t(nrhs));
    for (int k = 0; k < nrhs; ++k) {
        hc[k] = make_coef(c->act, c->act.mq);
        hc[nrhs + k] = make_coef_sym(c->act, c->act.mq);
    }
    if ((s = hip_check(c, hipMemcpyAsync(cf, hc.data(), hc.size() * sizeof(RhsCoef), hipMemcpyHostToDevice, st),
                       "tune coefficients")))
        return s;
    for (int k = 0; k < nrhs; ++k) launch_pack_parity(g, p, 0, 0, cin, a + hb * k, st);
    auto apply = [&]() {
        schur_launch(g, c->gs, p, form, false, a, b, t, t2, hb, nrhs, cf, cf + nrhs, nullptr, nullptr, st);
        if (with_dag)
            schur_launch(g, c->gs, p, form, true, b, d, t, t2, hb, nrhs, cf, cf + nrhs, nullptr, nullptr, st);
    };
    auto timed = [&](mdwf_launch_tune tn) -> mdwf_launch_tune {
        set_tune(g, p, tn);
        const int warm = 2, reps = 5;
        for (int r = 0; r < warm; ++r) apply();
        if ((s = hip_check(c, hipGetLastError(), "autotune launch"))) return tn;
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps; ++r) apply();
        (void)hipEventRecord(e1, st);
        if ((s = hip_check(c, hipEventSynchronize(e1), "autotune"))) return tn;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        tn.us = 1e3 * ms / reps;
        return tn;
    };
    mdwf_launch_tune best{};
    for (int k = 0; k < 4; ++k) best.tile[k] = g.trav[p].b[k];
    best.xcd_remap = 1;
    best.rhs_group = g.rhs_group[p];
    best.plane_bt = g.plane_bt[p];   // bare hops only: kept unless chosen below
    best.us = 1e30;
    for (const auto& tl : tiles) {
        mdwf_launch_tune tn = best;
        for (int k = 0; k < 4; ++k) tn.tile[k] = tl[k];
        tn = timed(tn);
        if (s) return s;
        if (tn.us < best.us) best = tn;
    }
    for (int lm : {1, 2, 3}) {
        if (lm == 1 && 64 / g.L5 > 8) continue;
        if (lm == 2 && (p == P64 || g.L5 < (p == P32 ? 4 : 2))) continue;
        if (lm == 3 && (p != P16 || g.L5 % 4 != 0)) continue;
        mdwf_launch_tune tn = best;
        tn.link_mode = lm;
        tn = timed(tn);
        if (s) return s;
        if (tn.us < best.us) best = tn;
    }
    for (int v = 0; v < 2; ++v) {
        mdwf_launch_tune tn = best;
        if (v == 0) tn.nt_store = 1 - tn.nt_store;
        else tn.xcd_remap = 1 - tn.xcd_remap;
        tn = timed(tn);
        if (s) return s;
        if (tn.us < best.us) best = tn;
    }
    if (nrhs > 1)
        for (int rg : {0, 1, 2, 3, 4, 6}) {
            if (rg >= nrhs || rg == best.rhs_group) continue;
            mdwf_launch_tune tn = best;
            tn.rhs_group = rg;
            tn = timed(tn);
            if (s) return s;
            if (tn.us < best.us) best = tn;
        }
    set_tune(g, p, best);
    // The bare hops (MDWF_OP_HOP_*) can also run plane-staged: keep the
    // plane run that times fastest on one bare hop (0 = the lane kernel).
    // Only the single-RHS operator tuning does this: the solver launches no
    // bare hop.
    if (p != P64 && nrhs == 1 && !with_dag) {
        HopLaunch L{};
        L.kind = HOP_BARE; L.prec = p; L.out_parity = 0; L.out = b; L.in = a; L.centre = nullptr;
        L.stride = hb; L.nrhs = 1; L.coef = cf; L.active = nullptr; L.partials = nullptr;
        float best_ms = 1e30f;
        int best_bt = 0;
        for (int bt : {0, 4, 8, 16}) {
            if (bt && g.T % bt) continue;
            mdwf_launch_tune tn = best;
            tn.plane_bt = bt;
            set_tune(g, p, tn);
            const int warm = 2, reps = 10;
            for (int r = 0; r < warm; ++r) launch_hop(g, c->gs, L, st);
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps; ++r) launch_hop(g, c->gs, L, st);
            (void)hipEventRecord(e1, st);
            if ((s = hip_check(c, hipEventSynchronize(e1), "autotune bare hop"))) return s;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (bt == 0 ? ms < best_ms : ms < 0.98f * best_ms) best_ms = ms, best_bt = bt;   // a clear win only
        }
        best.plane_bt = best_bt;
        set_tune(g, p, best);
    }
    c->tuned_us[p] = best.us;
    if (out) *out = best;
    return MDWF_OK;
}

// shared set-up of both tuning entry points: a canonical scratch field with
// a finite pattern (timing does not depend on the values) and two events
template <typename F>
mdwf_status with_tune_scratch(mdwf_ctx* c, F body) {
    mdwf_status s = MDWF_OK;
    const size_t canon = size_t(c->geo.Vh) * 24 * sizeof(double);
    void* cin = buf(c, "tune_canon", canon, &s);
    if (!cin) return s;
    if ((s = hip_check(c, hipMemsetAsync(cin, 0x3f, canon, c->stream), "memset"))) return s;
    hipEvent_t e0, e1;
    if ((s = hip_check(c, hipEventCreate(&e0), "event"))) return s;
    if ((s = hip_check(c, hipEventCreate(&e1), "event"))) {
        (void)hipEventDestroy(e0);
        return s;
    }
    s = body(static_cast<const double*>(cin), e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

}  // namespace

extern "C" {

mdwf_status mdwf_autotune(mdwf_ctx* c, mdwf_launch_tune* out) {
    mdwf_status s = ready(c);
    if (s) return s;
    return with_tune_scratch(c, [&](const double* cin, hipEvent_t e0, hipEvent_t e1) {
        for (int pi = 0; pi < 3; ++pi) {
            const mdwf_status r = tune_precision(c, Prec(pi), 0, 1, false, cin, e0, e1, out ? out + pi : nullptr);
            if (r) return r;
        }
        return MDWF_OK;
    });
}

mdwf_status mdwf_autotune_solve(mdwf_ctx* c, const mdwf_solver_opts* opts, int nrhs, mdwf_launch_tune* out) {
    mdwf_status s = ready(c);
    if (s) return s;
    mdwf_solver_opts o;
    mdwf_default_opts(&o);
    if (opts) o = *opts;
    if (nrhs < 1 || !valid_prec(o.inner) || o.schur_form < 0 || o.schur_form > 2)
        return fail(c, MDWF_ERR_ARG, "need nrhs >= 1, a valid inner precision and schur_form 0-2");
    for (int pi = 0; pi < 3 && out; ++pi) (void)mdwf_get_tune(c, mdwf_prec(pi), out + pi);
    return with_tune_scratch(c, [&](const double* cin, hipEvent_t e0, hipEvent_t e1) {
        const Prec pi = Prec(o.inner);
        mdwf_status r = tune_precision(c, pi, o.schur_form, nrhs, true, cin, e0, e1, out ? out + pi : nullptr);
        if (!r && pi != P64)   // reliable updates: the FP64 operator, one RHS at a time
            r = tune_precision(c, P64, o.schur_form, 1, false, cin, e0, e1, out ? out + P64 : nullptr);
        return r;
    });
}

mdwf_status mdwf_solve_dev(mdwf_ctx* c, int nrhs, const double* const* b, double* const* x, const double* mq,
                           const mdwf_solver_opts* o, mdwf_solve_info* info, void* stream) {
    mdwf_status s = ready(c);
    if (s) return s;
    hipStream_t st = stream ? static_cast<hipStream_t>(stream) : c->stream;
    return mdwf_solve_impl(c, nrhs, b, x, false, mq, o, info, st);
}

mdwf_status mdwf_solve_point(mdwf_ctx* c, const int* site, int ncols, const int* cols, const double* mq,
                             const mdwf_solver_opts* o, double* const* q, mdwf_solve_info* info) {
    mdwf_status s = ready(c);
    if (s) return s;
    if (!site || !q || ncols < 1) return fail(c, MDWF_ERR_ARG, "need a site, ncols >= 1 and outputs");
    std::vector<int> src;
    for (int k = 0; k < ncols; ++k) src.insert(src.end(), {site[0], site[1], site[2], site[3], cols ? cols[k] : k});
    const PointIO pt{src.data(), q};
    return mdwf_solve_impl(c, ncols, nullptr, nullptr, true, mq, o, info, c->stream, &pt);
}

mdwf_status mdwf_solve(mdwf_ctx* c, int nrhs, const double* const* b, double* const* x, const double* mq,
                       const mdwf_solver_opts* o, mdwf_solve_info* info) {
    mdwf_status s = ready(c);
    if (s) return s;
    return mdwf_solve_impl(c, nrhs, b, x, true, mq, o, info, c->stream);
}

}  // extern "C"
