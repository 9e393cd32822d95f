// The source and sink side of the propagator solves, in FP64 on canonical
// fields: 4D spinors psi[t][z][y][x][spin][col], 5D spinors
// psi[s][t][z][y][x][spin][col], links U[t][z][y][x][mu][3][3].
//
// * Gauge-covariant Gaussian smearing of 4D sources (the paper's propagators
//   start from such sources, Sec. V): N explicit steps of
//       psi <- psi + sigma^2/(4N) Delta psi,
//       (Delta psi)(x) = sum_{i = x,y,z} U_i(x) psi(x+i) + U_i(x-i)^+ psi(x-i) - 2 psi(x),
//   one launch per step, a thread per site and vector.
// * The 5D right-hand side of a 4D source for the Moebius operator
//   D5 = D_W (b5 + c5 C) + 1 - C:  b = (1 - c5 D_W) Pbar eta with
//   (Pbar eta)_{L5-1} = P- eta, (Pbar eta)_0 = P+ eta, whose solution's wall
//   field q = P- x_0 + P+ x_{L5-1} is the 4D quark propagator.  One
//   wavefront per 4D site (up to 16 vectors; one thread per site and vector
//   beyond) applies the Wilson hop to both chiral halves of eta, each
//   neighbour spinor loaded once, and writes the two wall slices of b; a
//   fill kernel zeroes the others.
// * The wall and midpoint fields q and Q = P- x_{L5/2} + P+ x_{L5/2-1} of 5D
//   solutions, and per time slice the pseudoscalar and midpoint correlators
//   C_PP(t) = sum |q|^2, C_mp(t) = sum |Q|^2 over the slice's sites, spins,
//   colours and all vectors, with m_res(t) = C_mp / C_PP (Sec. III, the
//   residual mass with the Shamir midpoint density).  The sums are block
//   partials per time slice added in a fixed order: deterministic.
//
// Chiral basis: g5 = diag(1, 1, -1, -1), P+ = spins 0, 1;
// g_mu = [[0, G_mu], [G_mu^+, 0]], G_x = -i s1, G_y = -i s2, G_z = -i s3, G_t = 1.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ctx.h"

namespace mdwf {
namespace {

constexpr int kSrcBlock = 256;

struct SrcGeo {
    int X, Y, Z, T;
    int antiperiodic;
};

struct Site {
    int x, y, z, t;
};

__device__ __forceinline__ long index_of(const SrcGeo& g, int x, int y, int z, int t) {
    return long(x) + long(g.X) * (y + long(g.Y) * (z + long(g.Z) * t));
}

// neighbour index of s one step along mu in direction d (+1 / -1), periodic
__device__ __forceinline__ long neighbour(const SrcGeo& g, Site s, int mu, int d) {
    if (mu == 0) s.x = (s.x + d + g.X) % g.X;
    else if (mu == 1) s.y = (s.y + d + g.Y) % g.Y;
    else if (mu == 2) s.z = (s.z + d + g.Z) % g.Z;
    else s.t = (s.t + d + g.T) % g.T;
    return index_of(g, s.x, s.y, s.z, s.t);
}

// u = U_mu(site), or its adjoint
__device__ __forceinline__ void ld_link_op(const double2* U, long site, int mu, bool dag, cx<double> u[9]) {
    const double2* p = U + (site * 4 + mu) * 9;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double2 e = dag ? p[b * 3 + a] : p[a * 3 + b];
            u[a * 3 + b] = {e.x, dag ? -e.y : e.y};
        }
}

__device__ __forceinline__ void ld_spinor(const double2* f, long site, cx<double> v[12]) {
    const double2* p = f + site * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) v[k] = {p[k].x, p[k].y};
}

__device__ __forceinline__ void st_spinor(double2* f, long site, const cx<double> v[12]) {
    double2* p = f + site * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) p[k] = make_double2(v[k].re, v[k].im);
}

// w[sp][a] = sum_b u[a][b] v[sp][b] for the nsp spins of v
__device__ __forceinline__ void link_times(const cx<double> u[9], const cx<double>* v, cx<double>* w, int nsp) {
#pragma unroll
    for (int sp = 0; sp < nsp; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int b = 0; b < 3; ++b) s = cmadd(s, u[a * 3 + b], v[sp * 3 + b]);
            w[sp * 3 + a] = s;
        }
}

// G_mu h and G_mu^+ h for a two-spin colour pair h[2][3] (spin-major)
__device__ __forceinline__ void g_apply(int mu, bool dag, const cx<double> h[6], cx<double> o[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<double> h0 = h[a], h1 = h[3 + a];
        cx<double> o0, o1;
        if (mu == 0) {          // G = -i s1 ; G^+ = i s1
            o0 = dag ? timesI(h1) : timesMinusI(h1);
            o1 = dag ? timesI(h0) : timesMinusI(h0);
        } else if (mu == 1) {   // G = -i s2 = [[0, -1], [1, 0]] ; G^+ = [[0, 1], [-1, 0]]
            o0 = dag ? h1 : -1.0 * h1;
            o1 = dag ? -1.0 * h0 : h0;
        } else if (mu == 2) {   // G = -i s3 = diag(-i, i) ; G^+ = diag(i, -i)
            o0 = dag ? timesI(h0) : timesMinusI(h0);
            o1 = dag ? timesMinusI(h1) : timesI(h1);
        } else {                // G = 1
            o0 = h0;
            o1 = h1;
        }
        o[a] = o0;
        o[3 + a] = o1;
    }
}

// ------------------------------------------------------ Gaussian smearing
// One thread per (site, vector, spin), the spin and then the vector fastest:
// the 4 * nvec lanes of a site share every link load, and the 4 spin lanes
// of a vector read the site's 192-byte spinor as one contiguous run.  (One
// thread per (site, vector) carrying all four spins needs fewer link loads
// but twice the registers, and ran 1.7x slower.)
struct SmearIdx {
    FastDiv fG, fX, fY, fZ;   // G = lanes per site
    uint32_t G;
};

// WAVE: one wavefront per site (nvec <= 16; lanes 4 nvec .. 63 idle), so the
// site and its links are wave-uniform and the links come by scalar loads.
// in / out are addressed as base + vector * vs + site * ss (complex units):
// the canonical layout has vs = 12 * sites, ss = 12; the site-major layout
// the steps between the first and the last use has vs = 12, ss = 12 * nvec,
// so a wave's neighbour reads of all vectors are one contiguous run.
struct SmearLayout {
    size_t in_vs, in_ss, out_vs, out_ss;
};

// The one-site-per-wave path is compiled for four waves per SIMD, so the
// compiler keeps all its loads in flight (left free, it aims at eight waves
// and keeps two neighbours' loads in flight; a step was 5 % slower so).
template <bool WAVE>
__global__ void __launch_bounds__(kSrcBlock) __attribute__((amdgpu_waves_per_eu(WAVE ? 4 : 1, WAVE ? 4 : 8)))
k_gauss_step(const SrcGeo g, const SmearIdx ix, const double2* U, const double2* in, double2* out, double kappa,
             uint32_t nsites, uint32_t ntot, const SmearLayout lay) {
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t i, r;
    if constexpr (WAVE) {
        i = uint32_t(__builtin_amdgcn_readfirstlane(int(id >> 6)));
        r = id & 63;
        if (i >= nsites || r >= ix.G) return;
    } else {
        if (id >= ntot) return;
        i = ix.fG.div(id);
        r = id - i * ix.G;
    }
    const uint32_t v = r >> 2, sp = r & 3;
    const uint32_t q1 = ix.fX.div(i), x = i - q1 * g.X;
    const uint32_t q2 = ix.fY.div(q1), y = q1 - q2 * g.Y;
    const uint32_t t = ix.fZ.div(q2), z = q2 - t * g.Z;
    const double2* f = in + size_t(v) * lay.in_vs + sp * 3;
    const uint32_t sy = g.X, sz = uint32_t(g.X) * g.Y;
    // neighbours x+mu, x-mu for mu = x, y, z, in that order
    uint32_t xn[6];
#pragma unroll
    for (int mu = 0; mu < 3; ++mu) {
        const uint32_t c = mu == 0 ? x : mu == 1 ? y : z;
        const uint32_t L = mu == 0 ? g.X : mu == 1 ? g.Y : g.Z;
        const uint32_t st = mu == 0 ? 1u : mu == 1 ? sy : sz;
        xn[2 * mu] = c + 1 == L ? i - (L - 1) * st : i + st;
        xn[2 * mu + 1] = c == 0 ? i + (L - 1) * st : i - st;
    }
    cx<double> acc[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}}, u[9], nb[3], w[3];
    double2 cv[3];
    auto hop = [&](int k, const double2* nv) {   // acc += U_mu(x) psi(x+mu) or U_mu(x-mu)^+ psi(x-mu)
        ld_link_op(U, (k & 1) == 0 ? i : xn[k], k >> 1, (k & 1) != 0, u);
#pragma unroll
        for (int c = 0; c < 3; ++c) nb[c] = {nv[c].x, nv[c].y};
        link_times(u, nb, w, 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = acc[c] + w[c];
    };
    if constexpr (WAVE) {
        // wave-uniform links (scalar loads): the six neighbours and the
        // centre are all requested before the first product
        double2 nv[6][3];
#pragma unroll
        for (int k = 0; k < 6; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) nv[k][c] = f[size_t(xn[k]) * lay.in_ss + c];
#pragma unroll
        for (int c = 0; c < 3; ++c) cv[c] = f[size_t(i) * lay.in_ss + c];
#pragma unroll
        for (int k = 0; k < 6; ++k) hop(k, nv[k]);
    } else {
#pragma unroll 1
        for (int mu = 0; mu < 3; ++mu)
#pragma unroll
            for (int dir = 0; dir < 2; ++dir) hop(2 * mu + dir, f + size_t(xn[2 * mu + dir]) * lay.in_ss);
#pragma unroll
        for (int c = 0; c < 3; ++c) cv[c] = f[size_t(i) * lay.in_ss + c];
    }
    double2* o = out + size_t(v) * lay.out_vs + size_t(i) * lay.out_ss + sp * 3;
    const double cc = 1.0 - 6.0 * kappa;
#pragma unroll
    for (int c = 0; c < 3; ++c) o[c] = make_double2(fma(cc, cv[c].x, kappa * acc[c].re), fma(cc, cv[c].y, kappa * acc[c].im));
}

// ----------------------------------------------------------- wall source
// hp / hm accumulate the hop sum_mu (1 - g_mu) U psi(x+mu) + (1 + g_mu) U^+ psi(x-mu)
// of P+ eta and of P- eta.  (1 - sg g)(u, 0) = (u, -sg G^+ u) and
// (1 - sg g)(0, d) = (-sg G d, d).
// One thread per (site, vector), the vector fastest so that the nvec lanes
// of a site share the link loads; it writes the two wall slices of b (the
// same slice twice when L5 = 1), k_zero_slices the others.
__global__ void __launch_bounds__(kSrcBlock) k_wall_source(const SrcGeo g, const SmearIdx ix, const double2* U,
                                                           const double2* eta, double2* b, double cdiag,
                                                           double chop, int L5, uint32_t nsites, uint32_t ntot) {
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= ntot) return;
    const uint32_t i = ix.fG.div(id), v = id - i * ix.G;
    const double2* f = eta + size_t(v) * nsites * 12;
    Site s;
    const uint32_t q1 = ix.fX.div(i), q2 = ix.fY.div(q1);
    s.x = int(i - q1 * g.X);
    s.y = int(q1 - q2 * g.Y);
    s.t = int(ix.fZ.div(q2));
    s.z = int(q2 - uint32_t(s.t) * g.Z);
    cx<double> hp[12], hm[12], nb[6], w[6], gw[6], u[9];
#pragma unroll
    for (int k = 0; k < 12; ++k) hp[k] = hm[k] = {0.0, 0.0};
#pragma unroll 1
    for (int hop = 0; hop < 8; ++hop) {
        const int mu = hop >> 1, dir = hop & 1;
        const double sg = dir == 0 ? 1.0 : -1.0;
        const long xn = neighbour(g, s, mu, dir == 0 ? +1 : -1);
        // the fermion's antiperiodic time boundary: hops across it carry -1
        const bool wrap = mu == 3 && ((dir == 0 && s.t == g.T - 1) || (dir == 1 && s.t == 0));
        const double bc = (g.antiperiodic && wrap) ? -1.0 : 1.0;
        ld_link_op(U, dir == 0 ? i : xn, mu, dir != 0, u);
#pragma unroll
        for (int half = 0; half < 2; ++half) {   // upper (P+) then lower (P-) spin pair
            const double2* p = f + xn * 12 + half * 6;
#pragma unroll
            for (int k = 0; k < 6; ++k) nb[k] = {bc * p[k].x, bc * p[k].y};
            link_times(u, nb, w, 2);
            if (half == 0) {        // (u, 0) -> (u, -sg G^+ u)
                g_apply(mu, true, w, gw);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    hp[k] = hp[k] + w[k];
                    hp[6 + k] = hp[6 + k] - sg * gw[k];
                }
            } else {                // (0, d) -> (-sg G d, d)
                g_apply(mu, false, w, gw);
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    hm[k] = hm[k] - sg * gw[k];
                    hm[6 + k] = hm[6 + k] + w[k];
                }
            }
        }
    }
    // b_0 = (1 - c5 (4 - M5)) P+ eta + c5/2 hop(P+ eta), b_{L5-1} likewise with P-
    cx<double> e[12], b0[12], bl[12];
    ld_spinor(f, i, e);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
        const cx<double> ep = k < 6 ? e[k] : cx<double>{0.0, 0.0};
        const cx<double> em = k < 6 ? cx<double>{0.0, 0.0} : e[k];
        b0[k] = cdiag * ep + chop * hp[k];
        bl[k] = cdiag * em + chop * hm[k];
    }
    double2* out = b + size_t(v) * L5 * nsites * 12;
    if (L5 == 1) {
#pragma unroll
        for (int k = 0; k < 12; ++k) b0[k] = b0[k] + bl[k];
        st_spinor(out, i, b0);
    } else {
        st_spinor(out, i, b0);
        st_spinor(out + size_t(L5 - 1) * nsites * 12, i, bl);
    }
}

// The value of another lane of the same quad (quad_perm DPP control: xor 1
// swaps the lanes of a spin pair, xor 2 the two pairs), moved by the VALU
// with no LDS round trip.
template <int CTRL> __device__ __forceinline__ double quad_swap(double x) {
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(x));
    const int lo = __builtin_amdgcn_mov_dpp(int(uint32_t(u)), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(int(uint32_t(u >> 32)), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(uint32_t(hi)) << 32) |
                                                       uint32_t(lo)));
}
constexpr int kQuadXor1 = 0xB1;   // lanes (1, 0, 3, 2)
constexpr int kQuadXor2 = 0x4E;   // lanes (2, 3, 0, 1)

// One wavefront per site (nvec <= 16), so the site, its neighbours and its
// links are wave-uniform and the links come by scalar loads.  Lane
// 4 v + 2 h + j (lanes 4 nvec .. 63 idle) carries spin 2 h + j of vector v:
// it multiplies that spin of each neighbour of eta by the link, i.e. its
// share of the hop of P+ eta (h = 0) or of P- eta (h = 1), and keeps two
// outputs of the slice its half feeds (0 for P+, L5 - 1 for P-): spin
// 2 h + j itself and spin 2 (1 - h) + j, the (1 -+ g_mu) image.  That image
// is G_mu^+ (h = 0) or G_mu (h = 1) applied to the spin pair, which for
// mu = x, y takes the other lane of the pair (lane ^ 1, a DPP quad
// permute).  Same sums, same order as the thread-per-vector kernel above.
// Compiled for three waves per SIMD, which lets all 27 loads of a lane be
// in flight at once.
__global__ void __launch_bounds__(kSrcBlock) __attribute__((amdgpu_waves_per_eu(3, 3)))
k_wall_source_wave(const SrcGeo g, const SmearIdx ix, const double2* U, const double2* eta, double2* b, double cdiag,
                   double chop, int L5, uint32_t nsites) {
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t i = uint32_t(__builtin_amdgcn_readfirstlane(int(id >> 6)));
    const uint32_t r = id & 63;
    if (i >= nsites || r >= ix.G) return;   // ix.G = 4 nvec: whole spin quads stay
    const uint32_t v = r >> 2, sp = r & 3, h = sp >> 1, j = sp & 1;
    const double2* f = eta + size_t(v) * nsites * 12 + sp * 3;
    Site st;
    const uint32_t q1 = ix.fX.div(i), q2 = ix.fY.div(q1);
    st.x = int(i - q1 * g.X);
    st.y = int(q1 - q2 * g.Y);
    st.t = int(ix.fZ.div(q2));
    st.z = int(q2 - uint32_t(st.t) * g.Z);
    // the pair image's phase per direction: G^+ for h = 0, G for h = 1
    // (G_x = -i s1, G_y = -i s2, G_z = -i s3, G_t = 1); for x and y it acts
    // on the other spin of the pair
    const double dg = h == 0 ? 1.0 : -1.0, js = j == 0 ? 1.0 : -1.0;
    cx<double> own[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}}, oth[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    // all eight neighbours' spins are requested before the first product
    long xn[8];
    double bc[8];
    double2 nv[8][3];
#pragma unroll
    for (int hop = 0; hop < 8; ++hop) {
        const int mu = hop >> 1, dir = hop & 1;
        xn[hop] = neighbour(g, st, mu, dir == 0 ? +1 : -1);
        const bool wrap = mu == 3 && ((dir == 0 && st.t == g.T - 1) || (dir == 1 && st.t == 0));
        bc[hop] = (g.antiperiodic && wrap) ? -1.0 : 1.0;
        const double2* p = f + xn[hop] * 12;
#pragma unroll
        for (int c = 0; c < 3; ++c) nv[hop][c] = p[c];
    }
    double2 cv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) cv[c] = f[size_t(i) * 12 + c];
    cx<double> u[9], nb[3], w[3];
#pragma unroll
    for (int hop = 0; hop < 8; ++hop) {
        const int mu = hop >> 1, dir = hop & 1;
        const double sg = dir == 0 ? 1.0 : -1.0;
        ld_link_op(U, dir == 0 ? long(i) : xn[hop], mu, dir != 0, u);
#pragma unroll
        for (int c = 0; c < 3; ++c) nb[c] = {bc[hop] * nv[hop][c].x, bc[hop] * nv[hop][c].y};
        link_times(u, nb, w, 1);
        // image = (fr + i fi) * (mu < 2 ? the pair's other w : w)
        double fr, fi;
        if (mu == 0) fr = 0.0, fi = dg;               // G^+ = i s1, G = -i s1
        else if (mu == 1) fr = dg * js, fi = 0.0;     // G^+ = [[0, 1], [-1, 0]], G = -G^+
        else if (mu == 2) fr = 0.0, fi = dg * js;     // G^+ = diag(i, -i), G = -G^+
        else fr = 1.0, fi = 0.0;                      // G = G^+ = 1
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<double> src = w[c];
            if (mu < 2) src = {quad_swap<kQuadXor1>(w[c].re), quad_swap<kQuadXor1>(w[c].im)};
            const cx<double> im = {fr * src.re - fi * src.im, fr * src.im + fi * src.re};
            own[c] = own[c] + w[c];
            oth[c] = oth[c] - sg * im;
        }
    }
    // slice 0: (1 - c5 (4 - M5)) P+ eta + c5/2 hop(P+ eta); slice L5 - 1 likewise with P-
    cx<double> o1[3], o2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o1[c] = cdiag * cx<double>{cv[c].x, cv[c].y} + chop * own[c];
        o2[c] = chop * oth[c];
    }
    double2* out = b + size_t(v) * L5 * nsites * 12 + size_t(i) * 12;
    if (L5 == 1) {   // both halves land on the one slice: lane h = 0 adds lane h = 1's outputs
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const cx<double> a1 = {quad_swap<kQuadXor2>(o2[c].re), quad_swap<kQuadXor2>(o2[c].im)};
            const cx<double> a2 = {quad_swap<kQuadXor2>(o1[c].re), quad_swap<kQuadXor2>(o1[c].im)};
            o1[c] = o1[c] + a1;
            o2[c] = o2[c] + a2;
        }
        if (h) return;
    } else if (h) {
        out += size_t(L5 - 1) * nsites * 12;
    }
    double2* p1 = out + sp * 3;
    double2* p2 = out + (2 * (1 - h) + j) * 3;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        p1[c] = make_double2(o1[c].re, o1[c].im);
        p2[c] = make_double2(o2[c].re, o2[c].im);
    }
}

// zero slices 1 .. L5-2 of nvec 5D fields: n2 = (L5 - 2) * nsites * 12
// double2 per field, starting nsites * 12 into it (a kernel, not a memset,
// so a caller may capture it in a graph)
__global__ void __launch_bounds__(kSrcBlock) k_zero_slices(double2* b, size_t field, size_t first, size_t n2) {
    double2* base = b + size_t(blockIdx.y) * field + first;
    for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < n2; e += size_t(gridDim.x) * blockDim.x)
        base[e] = make_double2(0.0, 0.0);
}

// -------------------------------------------------- wall / midpoint fields
// field = P- x_{slm} + P+ x_{slp}: spins 0, 1 from slice slp, spins 2, 3 from slm
__device__ __forceinline__ void chiral_pick(const double2* x5, long nsites, long i, int slp, int slm,
                                            cx<double> o[12]) {
    const double2* pp = x5 + (long(slp) * nsites + i) * 12;
    const double2* pm = x5 + (long(slm) * nsites + i) * 12;
#pragma unroll
    for (int k = 0; k < 6; ++k) o[k] = {pp[k].x, pp[k].y};
#pragma unroll
    for (int k = 6; k < 12; ++k) o[k] = {pm[k].x, pm[k].y};
}

__global__ void __launch_bounds__(kSrcBlock) k_project(const double2* x5, double2* q, double2* mid, int L5,
                                                       long nsites, long ntot) {
    const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= ntot) return;
    const long v = id / nsites, i = id - v * nsites;
    const double2* x = x5 + v * long(L5) * nsites * 12;
    cx<double> o[12];
    chiral_pick(x, nsites, i, L5 - 1, 0, o);
    st_spinor(q + v * nsites * 12, i, o);
    if (mid) {
        chiral_pick(x, nsites, i, L5 / 2 - 1, L5 / 2, o);
        st_spinor(mid + v * nsites * 12, i, o);
    }
}

// grid (nblk, T): block b of time slice t sums |q|^2 and |Q|^2 over its
// spatial sites and all vectors into partials[(t * nblk + b) * 2 + {0, 1}]
__global__ void __launch_bounds__(kSrcBlock) k_corr_partial(const double2* x5, double* partials, int L5,
                                                            long nsites, long nspat, int nvec) {
    const int t = blockIdx.y, nblk = gridDim.x;
    const long j = long(blockIdx.x) * blockDim.x + threadIdx.x;
    double spp = 0.0, smp = 0.0;
    if (j < nspat) {
        const long i = long(t) * nspat + j;
        for (int v = 0; v < nvec; ++v) {
            const double2* x = x5 + long(v) * L5 * nsites * 12;
            cx<double> o[12];
            chiral_pick(x, nsites, i, L5 - 1, 0, o);
#pragma unroll
            for (int k = 0; k < 12; ++k) spp += o[k].re * o[k].re + o[k].im * o[k].im;
            chiral_pick(x, nsites, i, L5 / 2 - 1, L5 / 2, o);
#pragma unroll
            for (int k = 0; k < 12; ++k) smp += o[k].re * o[k].re + o[k].im * o[k].im;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        spp += __shfl_xor(spp, off, 64);
        smp += __shfl_xor(smp, off, 64);
    }
    __shared__ double ws[2][kSrcBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        ws[0][wave] = spp;
        ws[1][wave] = smp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
#pragma unroll
        for (int w = 0; w < kSrcBlock / 64; ++w) {
            a += ws[0][w];
            c += ws[1][w];
        }
        partials[(long(t) * nblk + blockIdx.x) * 2 + 0] = a;
        partials[(long(t) * nblk + blockIdx.x) * 2 + 1] = c;
    }
}

// the same sums of |q|^2 over nvec 4D fields (any sink): grid (nblk, T),
// one partial per block and time slice, in the order of k_corr_partial
__global__ void __launch_bounds__(kSrcBlock) k_corr4_partial(const double2* q4, double* partials, long nsites,
                                                             long nspat, int nvec) {
    const int t = blockIdx.y, nblk = gridDim.x;
    const long j = long(blockIdx.x) * blockDim.x + threadIdx.x;
    double sum = 0.0;
    if (j < nspat) {
        const long i = long(t) * nspat + j;
        for (int v = 0; v < nvec; ++v) {
            const double2* p = q4 + (long(v) * nsites + i) * 12;
#pragma unroll
            for (int k = 0; k < 12; ++k) sum += p[k].x * p[k].x + p[k].y * p[k].y;
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) sum += __shfl_xor(sum, off, 64);
    __shared__ double ws[kSrcBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) ws[wave] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < kSrcBlock / 64; ++w) a += ws[w];
        partials[long(t) * nblk + blockIdx.x] = a;
    }
}

__global__ void k_corr4_final(const double* partials, double* out, int T, int nblk) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double a = 0.0;
    for (int b = 0; b < nblk; ++b) a += partials[long(t) * nblk + b];
    out[t] = a;
}

// out[t] = C_PP(t), out[T + t] = C_mp(t), out[2T + t] = m_res(t)
__global__ void k_corr_final(const double* partials, double* out, int T, int nblk) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= T) return;
    double a = 0.0, c = 0.0;
    for (int b = 0; b < nblk; ++b) {
        a += partials[(long(t) * nblk + b) * 2 + 0];
        c += partials[(long(t) * nblk + b) * 2 + 1];
    }
    out[t] = a;
    out[T + t] = c;
    out[2 * T + t] = c / a;
}

mdwf_status check_src_geom(const mdwf_geometry* g) {
    if (!g) return fail(nullptr, MDWF_ERR_ARG, "null geometry");
    if (g->X < 1 || g->Y < 1 || g->Z < 1 || g->T < 1) return fail(nullptr, MDWF_ERR_ARG, "extents must be >= 1");
    if (double(g->X) * g->Y * g->Z * g->T > double(1L << 31)) return fail(nullptr, MDWF_ERR_ARG, "lattice too large");
    return MDWF_OK;
}

unsigned blocks_for(long n) { return unsigned((n + kSrcBlock - 1) / kSrcBlock); }

}  // namespace
}  // namespace mdwf

using namespace mdwf;

extern "C" {

mdwf_status mdwf_gauss_smear_dev(const mdwf_geometry* geom, const double* U_dev, int nvec, const double* in_dev,
                                 double* out_dev, double sigma, int niter, void* stream) {
    mdwf_status s = check_src_geom(geom);
    if (s) return s;
    if (!U_dev || !in_dev || !out_dev) return fail(nullptr, MDWF_ERR_ARG, "null pointer");
    if (nvec < 1 || niter < 0 || !(sigma >= 0.0) || !std::isfinite(sigma))
        return fail(nullptr, MDWF_ERR_ARG, "need nvec >= 1, niter >= 0 and a finite sigma >= 0");
    const SrcGeo g{geom->X, geom->Y, geom->Z, geom->T, geom->antiperiodic_t};
    const long nsites = long(g.X) * g.Y * g.Z * g.T, ntot = nsites * nvec;
    const size_t bytes = size_t(ntot) * 12 * sizeof(double2);
    const char* lo_in = reinterpret_cast<const char*>(in_dev);
    const char* lo_out = reinterpret_cast<const char*>(out_dev);
    if (lo_in < lo_out + bytes && lo_out < lo_in + bytes) return fail(nullptr, MDWF_ERR_ARG, "in and out overlap");
    if (double(ntot) * 4.0 >= double(1u << 31))
        return fail(nullptr, MDWF_ERR_ARG, "nvec x sites too large for one smearing launch");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (niter == 0)
        return hip_check(nullptr, hipMemcpyAsync(out_dev, in_dev, bytes, hipMemcpyDeviceToDevice, st), "smear copy");
    double2* tmp = nullptr;
    if (niter > 1 && (s = hip_check(nullptr, hipMalloc(&tmp, bytes), "smearing buffer"))) return s;
    const double kappa = sigma * sigma / (4.0 * niter);
    SmearIdx ix;
    ix.G = uint32_t(4 * nvec);
    ix.fG = FastDiv(ix.G);
    ix.fX = FastDiv(uint32_t(g.X));
    ix.fY = FastDiv(uint32_t(g.Y));
    ix.fZ = FastDiv(uint32_t(g.Z));
    const bool wave = nvec <= 16;   // one wavefront per site
    const uint32_t nthr = wave ? uint32_t(nsites * 64) : uint32_t(ntot * 4);
    if (wave && double(nsites) * 64.0 >= double(1u << 31))
        return fail(nullptr, MDWF_ERR_ARG, "lattice too large for one smearing launch");
    const auto* U = reinterpret_cast<const double2*>(U_dev);
    const double2* src = reinterpret_cast<const double2*>(in_dev);
    double2* out = reinterpret_cast<double2*>(out_dev);
    // the steps between the first and the last keep the fields site-major
    // (all vectors of a site contiguous) when a wavefront holds one site;
    // the last step lands in out, canonical
    const size_t canon_vs = size_t(nsites) * 12, site_ss = size_t(nvec) * 12;
    for (int k = 1; k <= niter && !s; ++k) {
        double2* dst = ((niter - k) % 2 == 0) ? out : tmp;
        SmearLayout lay{canon_vs, 12, canon_vs, 12};
        if (wave) {
            if (k > 1) lay.in_vs = 12, lay.in_ss = site_ss;
            if (k < niter) lay.out_vs = 12, lay.out_ss = site_ss;
            hipLaunchKernelGGL(k_gauss_step<true>, dim3(blocks_for(nthr)), dim3(kSrcBlock), 0, st, g, ix, U, src, dst,
                               kappa, uint32_t(nsites), nthr, lay);
        } else {
            hipLaunchKernelGGL(k_gauss_step<false>, dim3(blocks_for(nthr)), dim3(kSrcBlock), 0, st, g, ix, U, src,
                               dst, kappa, uint32_t(nsites), nthr, lay);
        }
        s = hip_check(nullptr, hipGetLastError(), "smearing kernel");
        src = dst;
    }
    if (tmp) {
        const mdwf_status s2 = hip_check(nullptr, hipStreamSynchronize(st), "smearing");
        (void)hipFree(tmp);
        if (!s) s = s2;
    }
    return s;
}

mdwf_status mdwf_wall_source_dev(const mdwf_geometry* geom, const mdwf_action* act, const double* U_dev, int nvec,
                                 const double* eta_dev, double* b_dev, void* stream) {
    mdwf_status s = check_src_geom(geom);
    if (s) return s;
    if (!act || !U_dev || !eta_dev || !b_dev) return fail(nullptr, MDWF_ERR_ARG, "null pointer");
    if (nvec < 1 || act->L5 < 1 || !std::isfinite(act->M5) || !std::isfinite(act->c5))
        return fail(nullptr, MDWF_ERR_ARG, "need nvec >= 1, L5 >= 1 and finite M5, c5");
    if (nvec > 65535) return fail(nullptr, MDWF_ERR_ARG, "nvec > 65535");
    const SrcGeo g{geom->X, geom->Y, geom->Z, geom->T, geom->antiperiodic_t};
    const long nsites = long(g.X) * g.Y * g.Z * g.T, ntot = nsites * nvec;
    if (ntot >= (1L << 31)) return fail(nullptr, MDWF_ERR_ARG, "nvec x sites too large for one launch");
    // D_W = (4 - M5) - 1/2 hop, so 1 - c5 D_W = (1 - c5 (4 - M5)) + c5/2 hop
    const double cdiag = 1.0 - act->c5 * (4.0 - act->M5), chop = 0.5 * act->c5;
    SmearIdx ix;
    ix.G = uint32_t(nvec);
    ix.fG = FastDiv(ix.G);
    ix.fX = FastDiv(uint32_t(g.X));
    ix.fY = FastDiv(uint32_t(g.Y));
    ix.fZ = FastDiv(uint32_t(g.Z));
    hipStream_t st = static_cast<hipStream_t>(stream);
    double2* b = reinterpret_cast<double2*>(b_dev);
    const auto* U = reinterpret_cast<const double2*>(U_dev);
    const auto* eta = reinterpret_cast<const double2*>(eta_dev);
    if (nvec <= 16 && double(nsites) * 64.0 < double(1u << 31)) {   // one wavefront per site
        SmearIdx iw = ix;
        iw.G = uint32_t(4 * nvec);
        hipLaunchKernelGGL(k_wall_source_wave, dim3(blocks_for(size_t(nsites) * 64)), dim3(kSrcBlock), 0, st, g, iw,
                           U, eta, b, cdiag, chop, act->L5, uint32_t(nsites));
    } else {
        hipLaunchKernelGGL(k_wall_source, dim3(blocks_for(ntot)), dim3(kSrcBlock), 0, st, g, ix, U, eta, b, cdiag,
                           chop, act->L5, uint32_t(nsites), uint32_t(ntot));
    }
    s = hip_check(nullptr, hipGetLastError(), "wall source kernel");
    if (!s && act->L5 > 2) {
        const size_t field = size_t(act->L5) * nsites * 12, n2 = size_t(act->L5 - 2) * nsites * 12;
        const unsigned gx = unsigned(std::min<size_t>((n2 + kSrcBlock - 1) / kSrcBlock, 4096));
        hipLaunchKernelGGL(k_zero_slices, dim3(gx, unsigned(nvec)), dim3(kSrcBlock), 0, st, b, field,
                           size_t(nsites) * 12, n2);
        s = hip_check(nullptr, hipGetLastError(), "wall source kernel");
    }
    return s;
}

mdwf_status mdwf_project_4d_dev(const mdwf_geometry* geom, int L5, int nvec, const double* x_dev, double* q_dev,
                                double* mid_dev, void* stream) {
    mdwf_status s = check_src_geom(geom);
    if (s) return s;
    if (!x_dev || !q_dev) return fail(nullptr, MDWF_ERR_ARG, "null pointer");
    if (nvec < 1 || L5 < 1 || (mid_dev && L5 % 2))
        return fail(nullptr, MDWF_ERR_ARG, "need nvec >= 1, L5 >= 1, and an even L5 for the midpoint");
    const long nsites = long(geom->X) * geom->Y * geom->Z * geom->T, ntot = nsites * nvec;
    hipLaunchKernelGGL(k_project, dim3(blocks_for(ntot)), dim3(kSrcBlock), 0, static_cast<hipStream_t>(stream),
                       reinterpret_cast<const double2*>(x_dev), reinterpret_cast<double2*>(q_dev),
                       reinterpret_cast<double2*>(mid_dev), L5, nsites, ntot);
    return hip_check(nullptr, hipGetLastError(), "projection kernel");
}

mdwf_status mdwf_mres_correlators_dev(const mdwf_geometry* geom, int L5, int nvec, const double* x_dev, void* stream,
                                      double* c_pp, double* c_mp, double* mres) {
    mdwf_status s = check_src_geom(geom);
    if (s) return s;
    if (!x_dev || !c_pp || !c_mp || !mres) return fail(nullptr, MDWF_ERR_ARG, "null pointer");
    if (nvec < 1 || L5 < 2 || L5 % 2) return fail(nullptr, MDWF_ERR_ARG, "need nvec >= 1 and an even L5 >= 2");
    if (geom->T > 65535) return fail(nullptr, MDWF_ERR_ARG, "T > 65535");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int T = geom->T;
    const long nspat = long(geom->X) * geom->Y * geom->Z, nsites = nspat * T;
    const int nblk = int(blocks_for(nspat));
    double* dev = nullptr;
    const size_t npart = size_t(T) * nblk * 2;
    if ((s = hip_check(nullptr, hipMalloc(&dev, sizeof(double) * (npart + 3 * size_t(T))), "correlator buffer")))
        return s;
    hipLaunchKernelGGL(k_corr_partial, dim3(nblk, T), dim3(kSrcBlock), 0, st, reinterpret_cast<const double2*>(x_dev),
                       dev, L5, nsites, nspat, nvec);
    s = hip_check(nullptr, hipGetLastError(), "correlator kernel");
    if (!s) {
        hipLaunchKernelGGL(k_corr_final, dim3((T + 63) / 64), dim3(64), 0, st, dev, dev + npart, T, nblk);
        s = hip_check(nullptr, hipGetLastError(), "correlator kernel");
    }
    std::vector<double> h(3 * size_t(T));
    if (!s)
        s = hip_check(nullptr,
                      hipMemcpyAsync(h.data(), dev + npart, sizeof(double) * 3 * T, hipMemcpyDeviceToHost, st),
                      "correlator D2H");
    if (!s) s = hip_check(nullptr, hipStreamSynchronize(st), "correlators");
    (void)hipFree(dev);
    if (s) return s;
    for (int t = 0; t < T; ++t) {
        c_pp[t] = h[t];
        c_mp[t] = h[T + t];
        mres[t] = h[2 * T + t];
    }
    return MDWF_OK;
}

mdwf_status mdwf_pion_correlator_dev(const mdwf_geometry* geom, int nvec, const double* q_dev, void* stream,
                                     double* c) {
    mdwf_status s = check_src_geom(geom);
    if (s) return s;
    if (!q_dev || !c) return fail(nullptr, MDWF_ERR_ARG, "null pointer");
    if (nvec < 1) return fail(nullptr, MDWF_ERR_ARG, "need nvec >= 1");
    if (geom->T > 65535) return fail(nullptr, MDWF_ERR_ARG, "T > 65535");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int T = geom->T;
    const long nspat = long(geom->X) * geom->Y * geom->Z, nsites = nspat * T;
    const int nblk = int(blocks_for(nspat));
    const size_t npart = size_t(T) * nblk;
    double* dev = nullptr;
    if ((s = hip_check(nullptr, hipMalloc(&dev, sizeof(double) * (npart + size_t(T))), "correlator buffer")))
        return s;
    hipLaunchKernelGGL(k_corr4_partial, dim3(nblk, T), dim3(kSrcBlock), 0, st, reinterpret_cast<const double2*>(q_dev),
                       dev, nsites, nspat, nvec);
    s = hip_check(nullptr, hipGetLastError(), "correlator kernel");
    if (!s) {
        hipLaunchKernelGGL(k_corr4_final, dim3((T + 63) / 64), dim3(64), 0, st, dev, dev + npart, T, nblk);
        s = hip_check(nullptr, hipGetLastError(), "correlator kernel");
    }
    if (!s) s = hip_check(nullptr, hipMemcpyAsync(c, dev + npart, sizeof(double) * T, hipMemcpyDeviceToHost, st),
                          "correlator D2H");
    if (!s) s = hip_check(nullptr, hipStreamSynchronize(st), "correlators");
    (void)hipFree(dev);
    return s;
}

}  // extern "C"
