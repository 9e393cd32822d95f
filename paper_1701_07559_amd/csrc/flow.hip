// Wilson gradient flow of the gauge links (the smearing the paper applies to
// its ensembles before the valence solves, Sec. III, at flow time t_gf = 1),
// in FP64 on canonical links U[t][z][y][x][mu][3][3].
//
// Flow equation (Luscher's Wilson flow, cited in Sec. III):
//   dV/dt = Z(V) V,  Z_mu(x) = -1/2 (O - O^+) + 1/6 tr(O - O^+),
//   O_mu(x) = U_mu(x) * (sum of the six staples of the link),
// integrated with the third-order Runge-Kutta scheme of the same reference
// in its low-storage form: per stage i, E_i = a_i eps Z(W_i) + b_i E_{i-1}
// and W_{i+1} = exp(E_i) W_i with (a, b) = (1/4, 0), (8/9, -17/9), (3/4, -1).
//
// One kernel launch per stage: a thread per link reads the stage's input
// field (the link and its six staples; staple links by their first two
// rows), writes E_i for that link (its eight independent reals) and the
// updated link into a second buffer, so every staple sees the stage's input.
// The exponential of the small traceless antihermitian E is a degree-12
// Taylor polynomial after scaling by a power of two with squaring back.
#include <cmath>
#include <cstdio>
#include <vector>

#include "ctx.h"

namespace mdwf {
namespace {

constexpr int kFlowBlock = 256;
// largest entry of U U^+ - 1 and of det U - 1 the flow accepts
constexpr double kSu3Tol = 1e-10;

struct Su3 {
    cx<double> m[9];
};

__device__ __forceinline__ Su3 ld_link(const double2* U, long link) {
    Su3 r;
    const double2* p = U + link * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = p[k];
        r.m[k] = {v.x, v.y};
    }
    return r;
}

// A staple link from its first two rows: for U in SU(3) (unitary, det U = 1)
// the third row is the complex conjugate of the cross product of the first
// two, so six of the nine entries are loaded and three are computed.  The
// flow keeps every link in SU(3) up to rounding, and the staple gathers, not
// the arithmetic, bound the stage.
__device__ __forceinline__ cx<double> conj_cross(cx<double> a, cx<double> b, cx<double> c, cx<double> d) {
    const cx<double> v = cmadd(cmul(a, b), cx<double>{-c.re, -c.im}, d);   // a b - c d
    return {v.re, -v.im};
}
__device__ __forceinline__ Su3 ld_link12(const double2* U, long link) {
    Su3 r;
    const double2* p = U + link * 9;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double2 v = p[k];
        r.m[k] = {v.x, v.y};
    }
    r.m[6] = conj_cross(r.m[1], r.m[5], r.m[2], r.m[4]);
    r.m[7] = conj_cross(r.m[2], r.m[3], r.m[0], r.m[5]);
    r.m[8] = conj_cross(r.m[0], r.m[4], r.m[1], r.m[3]);
    return r;
}

// The Runge-Kutta accumulator E is traceless antihermitian: eight reals per
// link, stored as four double2 (Im E00, Im E11; E01; E02; E12).
// complete_alg fills in the other entries from those eight.
__device__ __forceinline__ void complete_alg(Su3& r) {
    r.m[0].re = 0.0;
    r.m[4].re = 0.0;
    r.m[8] = {0.0, -(r.m[0].im + r.m[4].im)};
    r.m[3] = {-r.m[1].re, r.m[1].im};
    r.m[6] = {-r.m[2].re, r.m[2].im};
    r.m[7] = {-r.m[5].re, r.m[5].im};
}
__device__ __forceinline__ Su3 ld_alg(const double2* E, long link) {
    const double2* p = E + link * 4;
    const double2 d = p[0], e01 = p[1], e02 = p[2], e12 = p[3];
    Su3 r;
    r.m[0] = {0.0, d.x};
    r.m[4] = {0.0, d.y};
    r.m[1] = {e01.x, e01.y};
    r.m[2] = {e02.x, e02.y};
    r.m[5] = {e12.x, e12.y};
    complete_alg(r);
    return r;
}
__device__ __forceinline__ void st_alg(double2* E, long link, const Su3& a) {
    double2* p = E + link * 4;
    p[0] = make_double2(a.m[0].im, a.m[4].im);
    p[1] = make_double2(a.m[1].re, a.m[1].im);
    p[2] = make_double2(a.m[2].re, a.m[2].im);
    p[3] = make_double2(a.m[5].re, a.m[5].im);
}

__device__ __forceinline__ void st_link(double2* U, long link, const Su3& a) {
    double2* p = U + link * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = make_double2(a.m[k].re, a.m[k].im);
}

// a b, a^+ b, a b^+
__device__ __forceinline__ Su3 mul(const Su3& a, const Su3& b) {
    Su3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s = cmadd(s, a.m[i * 3 + k], b.m[k * 3 + j]);
            r.m[i * 3 + j] = s;
        }
    return r;
}
__device__ __forceinline__ Su3 mul_dn(const Su3& a, const Su3& b) {   // a^+ b
    Su3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) s = cjmadd(s, a.m[k * 3 + i], b.m[k * 3 + j]);
            r.m[i * 3 + j] = s;
        }
    return r;
}
__device__ __forceinline__ Su3 mul_nd(const Su3& a, const Su3& b) {   // a b^+
    Su3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const cx<double> bc = {b.m[j * 3 + k].re, -b.m[j * 3 + k].im};
                s = cmadd(s, a.m[i * 3 + k], bc);
            }
            r.m[i * 3 + j] = s;
        }
    return r;
}

// exp(X) for a traceless antihermitian X: scale by 2^-k until the Frobenius
// norm is at most 1/4, Taylor polynomial of degree 12 by Horner's rule, then
// square k times (truncation below 1e-17 relative)
__device__ Su3 expm_small(Su3 X) {
    double n2 = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) n2 += X.m[k].re * X.m[k].re + X.m[k].im * X.m[k].im;
    int sq = 0;
    double scale = 1.0;
    const double n = sqrt(n2);
    while (n * scale > 0.25 && sq < 40) {
        scale *= 0.5;
        ++sq;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) X.m[k] = scale * X.m[k];
    Su3 R;
#pragma unroll
    for (int k = 0; k < 9; ++k) R.m[k] = {(k % 4 == 0) ? 1.0 : 0.0, 0.0};
    for (int d = 12; d >= 1; --d) {   // R = 1 + X R / d
        Su3 t = mul(X, R);
        const double inv = 1.0 / d;
#pragma unroll
        for (int k = 0; k < 9; ++k) R.m[k] = inv * t.m[k];
        R.m[0].re += 1.0;
        R.m[4].re += 1.0;
        R.m[8].re += 1.0;
    }
    for (int s = 0; s < sq; ++s) R = mul(R, R);
    return R;
}

struct FlowGeo {
    int X, Y, Z, T;
};

__device__ __forceinline__ long nbr(const FlowGeo& g, int x, int y, int z, int t, int mu, int d) {
    if (mu == 0) x = (x + d + g.X) % g.X;
    else if (mu == 1) y = (y + d + g.Y) % g.Y;
    else if (mu == 2) z = (z + d + g.Z) % g.Z;
    else t = (t + d + g.T) % g.T;
    return long(x) + long(g.X) * (y + long(g.Y) * (z + long(g.Z) * t));
}

// one Runge-Kutta stage for every link: E = a Z(Win) + b E, Wout = exp(E) Win
__global__ void __launch_bounds__(kFlowBlock) k_flow_stage(const FlowGeo g, const double2* Win, double2* Wout,
                                                           double2* E, double a, double b, long nlinks) {
    const long l = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (l >= nlinks) return;
    const int mu = int(l & 3);
    const long site = l >> 2;
    const int x = int(site % g.X);
    const int y = int((site / g.X) % g.Y);
    const int z = int((site / (long(g.X) * g.Y)) % g.Z);
    const int t = int(site / (long(g.X) * g.Y * g.Z));
    const long xp = nbr(g, x, y, z, t, mu, 1);
    Su3 S;
#pragma unroll
    for (int k = 0; k < 9; ++k) S.m[k] = {0.0, 0.0};
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        // upper staple U_nu(x+mu) U_mu(x+nu)^+ U_nu(x)^+
        const long xn = nbr(g, x, y, z, t, nu, 1);
        Su3 s1 = mul_nd(ld_link12(Win, xp * 4 + nu), ld_link12(Win, xn * 4 + mu));
        s1 = mul_nd(s1, ld_link12(Win, site * 4 + nu));
        // lower staple U_nu(x+mu-nu)^+ U_mu(x-nu)^+ U_nu(x-nu)
        const long xm = nbr(g, x, y, z, t, nu, -1);
        int cx_[4] = {x, y, z, t};
        cx_[nu] = (cx_[nu] - 1 + (nu == 0 ? g.X : nu == 1 ? g.Y : nu == 2 ? g.Z : g.T)) %
                  (nu == 0 ? g.X : nu == 1 ? g.Y : nu == 2 ? g.Z : g.T);
        const long xpm = nbr(g, cx_[0], cx_[1], cx_[2], cx_[3], mu, 1);
        const Su3 a1 = ld_link12(Win, xpm * 4 + nu);
        const Su3 a2 = ld_link12(Win, xm * 4 + mu);
        // (U_mu(x-nu) U_nu(x+mu-nu))^+ U_nu(x-nu)
        Su3 s2 = mul(a2, a1);
        s2 = mul_dn(s2, ld_link12(Win, xm * 4 + nu));
#pragma unroll
        for (int k = 0; k < 9; ++k) S.m[k] = S.m[k] + s1.m[k] + s2.m[k];
    }
    const Su3 U = ld_link(Win, l);
    const Su3 O = mul(U, S);
    // Z = -1/2 (O - O^+) + 1/6 tr(O - O^+); tr(O - O^+) = 2 i Im tr O
    const double itr = (O.m[0].im + O.m[4].im + O.m[8].im) / 3.0;
    // the eight independent entries of E (upper triangle, first two
    // diagonal ones); the rest follow from antihermiticity and zero trace
    Su3 Ev = (b != 0.0) ? ld_alg(E, l) : Su3{};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            if (i == 2) continue;
            const cx<double> oij = O.m[i * 3 + j], oji = O.m[j * 3 + i];
            cx<double> zij = {-0.5 * (oij.re - oji.re), -0.5 * (oij.im + oji.im)};
            if (i == j) zij.im += itr;
            const cx<double> prev = (b != 0.0) ? Ev.m[i * 3 + j] : cx<double>{0.0, 0.0};
            Ev.m[i * 3 + j] = {a * zij.re + b * prev.re, a * zij.im + b * prev.im};
        }
    st_alg(E, l, Ev);
    complete_alg(Ev);
    st_link(Wout, l, mul(expm_small(Ev), U));
}

// sum over the six planes of Re tr U_mu nu(x), block partials in a fixed order
__global__ void __launch_bounds__(kFlowBlock) k_plaquette(const FlowGeo g, const double2* U, double* partials,
                                                          long nsites) {
    const long site = long(blockIdx.x) * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (site < nsites) {
        const int x = int(site % g.X);
        const int y = int((site / g.X) % g.Y);
        const int z = int((site / (long(g.X) * g.Y)) % g.Z);
        const int t = int(site / (long(g.X) * g.Y * g.Z));
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                const Su3 a = mul(ld_link(U, site * 4 + mu), ld_link(U, nbr(g, x, y, z, t, mu, 1) * 4 + nu));
                const Su3 c = mul_nd(a, ld_link(U, nbr(g, x, y, z, t, nu, 1) * 4 + mu));
                const Su3 p = mul_nd(c, ld_link(U, site * 4 + nu));
                v += p.m[0].re + p.m[4].re + p.m[8].re;
            }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    __shared__ double ws[kFlowBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) ws[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kFlowBlock / 64; ++w) s += ws[w];
        partials[blockIdx.x] = s;
    }
}

// Largest deviation from SU(3) of the links of a block of sites: max over
// each site's four links of the entries of U U^+ - 1 and of det U - 1 (re
// and im parts), so a field the flow stage's two-row staple loads would
// misread is refused.  NaN propagates into the partial.
__device__ __forceinline__ double max_nan(double v, double x) { return (x > v || x != x) ? x : v; }

__global__ void __launch_bounds__(kFlowBlock) k_su3_deviation(const double2* U, double* partials, long nsites) {
    const long site = long(blockIdx.x) * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (site < nsites) {
        for (int mu = 0; mu < 4; ++mu) {
            const Su3 a = ld_link(U, site * 4 + mu);
            const Su3 p = mul_nd(a, a);   // U U^+
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                v = max_nan(v, fabs(p.m[k].re - ((k % 4 == 0) ? 1.0 : 0.0)));
                v = max_nan(v, fabs(p.m[k].im));
            }
            // det U = row 2 . (row 0 x row 1)
            const cx<double> c0 = cmadd(cmul(a.m[1], a.m[5]), cx<double>{-a.m[2].re, -a.m[2].im}, a.m[4]);
            const cx<double> c1 = cmadd(cmul(a.m[2], a.m[3]), cx<double>{-a.m[0].re, -a.m[0].im}, a.m[5]);
            const cx<double> c2 = cmadd(cmul(a.m[0], a.m[4]), cx<double>{-a.m[1].re, -a.m[1].im}, a.m[3]);
            const cx<double> det = cmadd(cmadd(cmul(a.m[6], c0), a.m[7], c1), a.m[8], c2);
            v = max_nan(v, fabs(det.re - 1.0));
            v = max_nan(v, fabs(det.im));
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = max_nan(v, __shfl_xor(v, off, 64));
    __shared__ double ws[kFlowBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) ws[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
#pragma unroll
        for (int w = 0; w < kFlowBlock / 64; ++w) m = max_nan(m, ws[w]);
        partials[blockIdx.x] = m;
    }
}

mdwf_status check_geom(const mdwf_geometry* g) {
    if (!g) return fail(nullptr, MDWF_ERR_ARG, "null geometry");
    if (g->X < 2 || g->Y < 2 || g->Z < 2 || g->T < 2) return fail(nullptr, MDWF_ERR_ARG, "extents must be >= 2");
    return MDWF_OK;
}

// average plaquette of the device field U into *plaq (synchronous on st)
mdwf_status plaquette_dev(const FlowGeo& fg, const double2* U, double* part, double* hpart, long nsites, int nblk,
                          hipStream_t st, double* plaq) {
    hipLaunchKernelGGL(k_plaquette, dim3(nblk), dim3(kFlowBlock), 0, st, fg, U, part, nsites);
    mdwf_status s = hip_check(nullptr, hipGetLastError(), "plaquette kernel");
    if (s) return s;
    if ((s = hip_check(nullptr, hipMemcpyAsync(hpart, part, sizeof(double) * nblk, hipMemcpyDeviceToHost, st),
                       "plaquette D2H")))
        return s;
    if ((s = hip_check(nullptr, hipStreamSynchronize(st), "plaquette"))) return s;
    double tot = 0.0;
    for (int k = 0; k < nblk; ++k) tot += hpart[k];
    *plaq = tot / (3.0 * 6.0 * double(nsites));
    return MDWF_OK;
}

}  // namespace
}  // namespace mdwf

using namespace mdwf;

extern "C" {

mdwf_status mdwf_plaquette_dev(const mdwf_geometry* geom, const double* U_dev, void* stream, double* plaq) {
    mdwf_status s = check_geom(geom);
    if (s) return s;
    if (!U_dev || !plaq) return fail(nullptr, MDWF_ERR_ARG, "null argument");
    const FlowGeo fg{geom->X, geom->Y, geom->Z, geom->T};
    const long nsites = long(fg.X) * fg.Y * fg.Z * fg.T;
    const int nblk = int((nsites + kFlowBlock - 1) / kFlowBlock);
    double* part = nullptr;
    if ((s = hip_check(nullptr, hipMalloc(&part, sizeof(double) * nblk), "plaquette partials"))) return s;
    std::vector<double> hpart(nblk);
    s = plaquette_dev(fg, reinterpret_cast<const double2*>(U_dev), part, hpart.data(), nsites, nblk,
                      static_cast<hipStream_t>(stream), plaq);
    (void)hipFree(part);
    return s;
}

mdwf_status mdwf_wilson_flow_dev(const mdwf_geometry* geom, double* U_dev, double eps, int nsteps, void* stream,
                                 double* plaq) {
    mdwf_status s = check_geom(geom);
    if (s) return s;
    if (!U_dev) return fail(nullptr, MDWF_ERR_ARG, "null gauge field");
    if (!(eps > 0.0) || !std::isfinite(eps) || nsteps < 0)
        return fail(nullptr, MDWF_ERR_ARG, "need eps > 0 and nsteps >= 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const FlowGeo fg{geom->X, geom->Y, geom->Z, geom->T};
    const long nsites = long(fg.X) * fg.Y * fg.Z * fg.T, nlinks = 4 * nsites;
    const size_t bytes = size_t(nlinks) * 9 * sizeof(double2);
    const int nblk_p = int((nsites + kFlowBlock - 1) / kFlowBlock);
    double2 *W2 = nullptr, *E = nullptr;
    double* part = nullptr;
    if ((s = hip_check(nullptr, hipMalloc(&W2, bytes), "flow buffer"))) return s;
    if ((s = hip_check(nullptr, hipMalloc(&E, size_t(nlinks) * 4 * sizeof(double2)), "flow buffer"))) {
        (void)hipFree(W2);
        return s;
    }
    if ((s = hip_check(nullptr, hipMalloc(&part, sizeof(double) * nblk_p), "plaquette partials"))) {
        (void)hipFree(W2);
        (void)hipFree(E);
        return s;
    }
    std::vector<double> hpart(nblk_p);
    double2* W[2] = {reinterpret_cast<double2*>(U_dev), W2};
    {   // the links must be SU(3) (the stage rebuilds staple links' third rows)
        hipLaunchKernelGGL(k_su3_deviation, dim3(nblk_p), dim3(kFlowBlock), 0, st, W[0], part, nsites);
        s = hip_check(nullptr, hipGetLastError(), "SU(3) check kernel");
        if (!s) s = hip_check(nullptr, hipMemcpyAsync(hpart.data(), part, sizeof(double) * nblk_p,
                                                      hipMemcpyDeviceToHost, st), "SU(3) check D2H");
        if (!s) s = hip_check(nullptr, hipStreamSynchronize(st), "SU(3) check");
        double dev = 0.0;
        for (int k = 0; k < nblk_p && !s; ++k) dev = (hpart[k] > dev || hpart[k] != hpart[k]) ? hpart[k] : dev;
        if (!s && !(dev <= kSu3Tol)) {
            char msg[160];
            std::snprintf(msg, sizeof msg, "gauge links are not SU(3): deviation %.3e > %.0e", dev, kSu3Tol);
            s = fail(nullptr, MDWF_ERR_ARG, msg);
        }
    }
    if (!s && plaq) s = plaquette_dev(fg, W[0], part, hpart.data(), nsites, nblk_p, st, plaq);
    const double ca[3] = {0.25, 8.0 / 9.0, 0.75}, cb[3] = {0.0, -17.0 / 9.0, -1.0};
    const unsigned grid = unsigned((nlinks + kFlowBlock - 1) / kFlowBlock);
    int cur = 0;
    for (int n = 0; n < nsteps && !s; ++n)
        for (int i = 0; i < 3 && !s; ++i) {
            hipLaunchKernelGGL(k_flow_stage, dim3(grid), dim3(kFlowBlock), 0, st, fg, W[cur], W[1 - cur], E,
                               ca[i] * eps, cb[i], nlinks);
            s = hip_check(nullptr, hipGetLastError(), "flow kernel");
            cur = 1 - cur;
        }
    // an odd number of stages leaves the result in the scratch buffer
    if (!s && cur == 1) s = hip_check(nullptr, hipMemcpyAsync(U_dev, W2, bytes, hipMemcpyDeviceToDevice, st), "copy");
    if (!s && plaq) s = plaquette_dev(fg, W[0], part, hpart.data(), nsites, nblk_p, st, plaq + 1);
    if (!s) s = hip_check(nullptr, hipStreamSynchronize(st), "flow");
    (void)hipFree(W2);
    (void)hipFree(E);
    (void)hipFree(part);
    return s;
}

mdwf_status mdwf_wilson_flow(const mdwf_geometry* geom, int hip_device, double* U, double eps, int nsteps,
                             double* plaq) {
    mdwf_status s = check_geom(geom);
    if (s) return s;
    if (!U) return fail(nullptr, MDWF_ERR_ARG, "null gauge field");
    if ((s = hip_check(nullptr, hipSetDevice(hip_device), "hipSetDevice"))) return s;
    const size_t bytes = size_t(4) * geom->X * geom->Y * geom->Z * geom->T * 9 * sizeof(double2);
    double* d = nullptr;
    if ((s = hip_check(nullptr, hipMalloc(&d, bytes), "flow field"))) return s;
    s = hip_check(nullptr, hipMemcpy(d, U, bytes, hipMemcpyHostToDevice), "flow H2D");
    if (!s) s = mdwf_wilson_flow_dev(geom, d, eps, nsteps, nullptr, plaq);
    if (!s) s = hip_check(nullptr, hipMemcpy(U, d, bytes, hipMemcpyDeviceToHost), "flow D2H");
    (void)hipFree(d);
    return s;
}

}  // extern "C"
