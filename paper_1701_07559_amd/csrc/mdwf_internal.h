// Internal declarations shared by the HIP translation units of libmdwf.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mdwf {

enum Prec { P64 = 0, P32 = 1, P16 = 2 };
constexpr int kMaxL5 = 32;
constexpr int kBlock = 256;   // threads per workgroup of the site kernels (4 waves)
constexpr int kWaves = kBlock / 64;

template <Prec P> struct Real { using T = float; };
template <> struct Real<P64> { using T = double; };

// ---------------------------------------------------------------- complex
template <typename R> struct cx {
    R re, im;
};
template <typename R> __device__ __forceinline__ cx<R> mk(R a, R b) { return {a, b}; }
template <typename R> __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R> __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R> __device__ __forceinline__ cx<R> timesI(cx<R> a) { return {-a.im, a.re}; }
template <typename R> __device__ __forceinline__ cx<R> timesMinusI(cx<R> a) { return {a.im, -a.re}; }
// a * b
template <typename R> __device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// acc + a * b
template <typename R> __device__ __forceinline__ cx<R> cmadd(cx<R> acc, cx<R> a, cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
    return acc;
}
// acc + conj(a) * b
template <typename R> __device__ __forceinline__ cx<R> cjmadd(cx<R> acc, cx<R> a, cx<R> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(-a.im, b.re, acc.im);
    return acc;
}

// ------------------------------------------------------ integer division
// Division by a runtime-invariant divisor with one multiply-high and a shift
// (Granlund & Montgomery, PLDI 1994, round-up multiplier); exact for
// dividends below 2^31.
struct FastDiv {
    uint32_t d = 1, m = 1, s = 0;
    FastDiv() = default;
    explicit FastDiv(uint32_t div) : d(div) {
        s = 0;
        while ((uint64_t(1) << s) < div) ++s;
        m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << s) - div)) / div + 1);
    }
    __host__ __device__ __forceinline__ uint32_t div(uint32_t n) const {
#if defined(__HIP_DEVICE_COMPILE__)
        uint32_t t = __umulhi(n, m);
#else
        uint32_t t = uint32_t((uint64_t(n) * m) >> 32);
#endif
        return (t + n) >> s;
    }
};

// Traversal order of the hop kernels over the Xh x Y x Z x T parity-
// compressed 4D sites of one parity: tiles of b[0] x b[1] x b[2] x b[3]
// sites (each extent divides the lattice's); inside a tile x runs fastest,
// then y, z, t; tiles follow each other t fastest, then x, y, z.  Tiles of
// full x-y planes and b[3] = 1 are z-blocks with t inside; compact 4D tiles
// keep most neighbours of a site a few tiles apart in traversal order.
struct Trav {
    int b[4];
    FastDiv fTv, fBx, fBy, fBz;   // tile volume and extents
    FastDiv fNt, fNx, fNy;        // tiles along t, x, y
};

// -------------------------------------------------------------- geometry
struct Geo {
    int X, Y, Z, T, Xh;
    int Vh4;   // 4D sites of one parity
    int L5;
    int Vh;    // 5D sites of one parity = Vh4 * L5
    int antiperiodic;
    FastDiv fXh, fY, fZ;
    // launch shape per storage precision (index Prec), set by the autotuner
    Trav trav[3];
    int xcd_remap[3];   // renumber workgroups per XCD (1) or keep hardware order (0)
    int nt_store[3];    // write hop outputs with non-temporal stores
    int link_mode[3];   // 0 per-lane links, 1 LDS stage, 2 lane gather
    int rhs_group[3];   // multi-RHS launches: RHS per group sweeping the tiles together (0 = all)
    int plane_bt[3];    // > 0: bare hops by the plane-staged kernel, this many time planes per workgroup
};

// Coefficients of one right-hand side (its mass); all fifth-dimension
// operators are polynomials in C: sum_k c_k C^k.
struct RhsCoef {
    double mq, b5, c5;
    double k5[2];         // K5 = k5[0] + k5[1] C
    double m[kMaxL5];     // B K5^-1   = sum_k m[k] C^k
    double kinv[kMaxL5];  // K5^-1     = sum_k kinv[k] C^k
    double w[kMaxL5];     // K5 B^-1   = sum_k w[k] C^k
    double binv[kMaxL5];  // B^-1      = sum_k binv[k] C^k
};

// Bytes of a native half field / link segment.
__host__ __device__ inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
inline size_t half_field_bytes(Prec p, size_t Vh) {
    switch (p) {
        case P64: return align256(192 * Vh);
        case P32: return align256(96 * Vh);
        default: return align256(48 * Vh) + align256(4 * Vh);
    }
}
inline size_t link_segment_bytes(Prec p, size_t Vh4) {
    switch (p) {
        case P64: return align256(144 * Vh4);
        case P32: return align256(64 * Vh4) + align256(8 * Vh4);
        default: return align256(32 * Vh4) + align256(4 * Vh4);
    }
}
__host__ __device__ inline size_t norm_offset(size_t Vh) { return align256(48 * Vh); }  // P16 only

// ------------------------------------------------------- native accesses
typedef double nd2 __attribute__((ext_vector_type(2)));
typedef float nf4 __attribute__((ext_vector_type(4)));
typedef unsigned int nu4 __attribute__((ext_vector_type(4)));

// 16-byte store, optionally non-temporal (streamed past the caches)
template <bool NT, typename V> __device__ __forceinline__ void st16(V* p, V v) {
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <Prec P> struct Field;

// 16-byte load, optionally non-temporal (streamed past the caches)
template <bool NT, typename V> __device__ __forceinline__ V ld16(const V* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

template <> struct Field<P64> {
    using R = double;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const void* base, int Vh, int j, cx<R> v[12]) {
        const nd2* p = static_cast<const nd2*>(base);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const nd2 w = ld16<NT>(p + size_t(k) * Vh + j);
            v[k] = {w.x, w.y};
        }
    }
    template <bool NT = false>
    static __device__ __forceinline__ void store(void* base, int Vh, int j, const cx<R> v[12]) {
        nd2* p = static_cast<nd2*>(base);
#pragma unroll
        for (int k = 0; k < 12; ++k) st16<NT>(p + size_t(k) * Vh + j, nd2{v[k].re, v[k].im});
    }
};

template <> struct Field<P32> {
    using R = float;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const void* base, int Vh, int j, cx<R> v[12]) {
        const nf4* p = static_cast<const nf4*>(base);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const nf4 w = ld16<NT>(p + size_t(k) * Vh + j);
            v[2 * k] = {w.x, w.y};
            v[2 * k + 1] = {w.z, w.w};
        }
    }
    template <bool NT = false>
    static __device__ __forceinline__ void store(void* base, int Vh, int j, const cx<R> v[12]) {
        nf4* p = static_cast<nf4*>(base);
#pragma unroll
        for (int k = 0; k < 6; ++k)
            st16<NT>(p + size_t(k) * Vh + j, nf4{v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im});
    }
};

__device__ __forceinline__ float h2f(uint32_t bits16) {
    return __half2float(__ushort_as_half(static_cast<unsigned short>(bits16)));
}
__device__ __forceinline__ uint32_t f2h(float f) {
    return static_cast<uint32_t>(__half_as_ushort(__float2half_rn(f)));
}
__device__ __forceinline__ void unpack_h2(uint32_t w, float s, cx<float>& c) {
    c.re = h2f(w & 0xffffu) * s;
    c.im = h2f(w >> 16) * s;
}
__device__ __forceinline__ uint32_t pack_h2(cx<float> c, float inv) {
    return f2h(c.re * inv) | (f2h(c.im * inv) << 16);
}

template <> struct Field<P16> {
    using R = float;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const void* base, int Vh, int j, cx<R> v[12]) {
        const nu4* p = static_cast<const nu4*>(base);
        const float* nrm = reinterpret_cast<const float*>(static_cast<const char*>(base) + norm_offset(Vh));
        const float s = NT ? __builtin_nontemporal_load(nrm + j) : nrm[j];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const nu4 w = ld16<NT>(p + size_t(k) * Vh + j);
            unpack_h2(w.x, s, v[4 * k]);
            unpack_h2(w.y, s, v[4 * k + 1]);
            unpack_h2(w.z, s, v[4 * k + 2]);
            unpack_h2(w.w, s, v[4 * k + 3]);
        }
    }
    // Stores v / norm in binary16 (round to nearest even) with
    // norm = max |re|, |im| over the site; v is replaced by what was stored.
    // A site whose largest component is below the smallest normal float is
    // stored as zero (its reciprocal would overflow); NaN propagates.
    template <bool NT = false>
    static __device__ __forceinline__ void store(void* base, int Vh, int j, cx<R> v[12]) {
        float n = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) n = fmaxf(n, fmaxf(fabsf(v[k].re), fabsf(v[k].im)));
        float inv = __builtin_amdgcn_rcpf(n);   // scale into [-1, 1] before rounding
        if (n < 1.17549435e-38f) {
            n = 0.f;
            inv = 0.f;
        }
        nu4* p = static_cast<nu4*>(base);
        float* nrm = reinterpret_cast<float*>(static_cast<char*>(base) + norm_offset(Vh));
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            nu4 w;
            w.x = pack_h2(v[4 * k], inv);
            w.y = pack_h2(v[4 * k + 1], inv);
            w.z = pack_h2(v[4 * k + 2], inv);
            w.w = pack_h2(v[4 * k + 3], inv);
            st16<NT>(p + size_t(k) * Vh + j, w);
            unpack_h2(w.x, n, v[4 * k]);
            unpack_h2(w.y, n, v[4 * k + 1]);
            unpack_h2(w.z, n, v[4 * k + 2]);
            unpack_h2(w.w, n, v[4 * k + 3]);
        }
        if (NT) __builtin_nontemporal_store(n, nrm + j);
        else nrm[j] = n;
    }
};

// Links: one segment per (parity, mu) holding the links that live on the
// sites of that parity; 3x3 complex, element a*3+b.
template <Prec P> struct Link;
template <> struct Link<P64> {
    using R = double;
    static __device__ __forceinline__ void load(const char* seg, int Vh4, int i, cx<R> u[9]) {
        const double2* p = reinterpret_cast<const double2*>(seg);
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double2 w = p[size_t(k) * Vh4 + i];
            u[k] = {w.x, w.y};
        }
    }
    static __device__ __forceinline__ void store(char* seg, int Vh4, int i, const cx<double> u[9]) {
        double2* p = reinterpret_cast<double2*>(seg);
#pragma unroll
        for (int k = 0; k < 9; ++k) p[size_t(k) * Vh4 + i] = make_double2(u[k].re, u[k].im);
    }
};
template <> struct Link<P32> {
    using R = float;
    static __device__ __forceinline__ void load(const char* seg, int Vh4, int i, cx<R> u[9]) {
        const float4* p = reinterpret_cast<const float4*>(seg);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float4 w = p[size_t(k) * Vh4 + i];
            u[2 * k] = {w.x, w.y};
            u[2 * k + 1] = {w.z, w.w};
        }
        const float2* q = reinterpret_cast<const float2*>(seg + align256(64 * size_t(Vh4)));
        float2 w = q[i];
        u[8] = {w.x, w.y};
    }
    static __device__ __forceinline__ void store(char* seg, int Vh4, int i, const cx<double> u[9]) {
        float4* p = reinterpret_cast<float4*>(seg);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            p[size_t(k) * Vh4 + i] = make_float4(float(u[2 * k].re), float(u[2 * k].im),
                                                 float(u[2 * k + 1].re), float(u[2 * k + 1].im));
        float2* q = reinterpret_cast<float2*>(seg + align256(64 * size_t(Vh4)));
        q[i] = make_float2(float(u[8].re), float(u[8].im));
    }
};
template <> struct Link<P16> {
    using R = float;
    static __device__ __forceinline__ void load(const char* seg, int Vh4, int i, cx<R> u[9]) {
        const uint4* p = reinterpret_cast<const uint4*>(seg);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            uint4 w = p[size_t(k) * Vh4 + i];
            unpack_h2(w.x, 1.f, u[4 * k]);
            unpack_h2(w.y, 1.f, u[4 * k + 1]);
            unpack_h2(w.z, 1.f, u[4 * k + 2]);
            unpack_h2(w.w, 1.f, u[4 * k + 3]);
        }
        const uint32_t* q = reinterpret_cast<const uint32_t*>(seg + align256(32 * size_t(Vh4)));
        unpack_h2(q[i], 1.f, u[8]);
    }
    static __device__ __forceinline__ void store(char* seg, int Vh4, int i, const cx<double> u[9]) {
        uint4* p = reinterpret_cast<uint4*>(seg);
        cx<float> f[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) f[k] = {float(u[k].re), float(u[k].im)};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            uint4 w;
            w.x = pack_h2(f[4 * k], 1.f);
            w.y = pack_h2(f[4 * k + 1], 1.f);
            w.z = pack_h2(f[4 * k + 2], 1.f);
            w.w = pack_h2(f[4 * k + 3], 1.f);
            p[size_t(k) * Vh4 + i] = w;
        }
        uint32_t* q = reinterpret_cast<uint32_t*>(seg + align256(32 * size_t(Vh4)));
        q[i] = pack_h2(f[8], 1.f);
    }
};

// ------------------------------------------------------------- workgroups
// Workgroups are dealt to the 8 XCDs round-robin.  Renumber them so that each
// XCD works on one contiguous range of logical tiles, keeping neighbouring
// tiles (stencil halo) and the right-hand sides of one tile (shared links) in
// the same L2.
__device__ __forceinline__ int xcd_logical_block(int hw, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = hw & 7, slot = hw >> 3;
    return x * q + (x < r ? x : r) + slot;
}

// Fields of several right-hand sides are stored one after another with a
// fixed byte stride.
__device__ __forceinline__ const void* at_rhs(const void* base, size_t stride, int r) {
    return static_cast<const char*>(base) + stride * size_t(r);
}
__device__ __forceinline__ void* at_rhs(void* base, size_t stride, int r) {
    return static_cast<char*>(base) + stride * size_t(r);
}

// ---------------------------------------------------- host-side launchers
struct GaugeSet {
    char* seg[3] = {nullptr, nullptr, nullptr};   // per precision: 8 segments (parity*4+mu)
    size_t seg_bytes[3] = {0, 0, 0};
    // FP16 links as matrix-core operands (LinkRowsF16): 16 segments
    // (form*8 + parity*4 + mu), form 0 rows of U, form 1 rows of U^+
    char* mrow = nullptr;
    size_t mrow_bytes = 0;
};
// FP16 link rows for the matrix-core hop: per (form, parity, mu) segment
// [4 rows][Vh4] 16-byte entries, a row r < 3 as halves (Re A[r][0..2], 0,
// Im A[r][0..2], 0) with A = U (form 0) or U^+ (form 1); row 3 is zero.
inline size_t link_rows_bytes(size_t Vh4) { return align256(64 * Vh4); }

enum HopKind {
    HOP_BARE = 0,    // out = Dslash in
    HOP_D5,          // out = K5 c - 1/2 Dslash B in
    HOP_D5_DAG,      // out = K5^+ c - 1/2 B^+ Dslash^+ in
    HOP_SCHUR_A,     // out = B K5^-1 Dslash B in
    HOP_SCHUR_B,     // out = K5 c - 1/4 Dslash in
    HOP_SCHUR_A_DAG, // out = (B K5^-1)^+ Dslash^+ in
    HOP_SCHUR_B_DAG, // out = K5^+ c - 1/4 B^+ Dslash^+ in
    HOP_PREP,        // out = c + 1/2 Dslash B in
    HOP_BARE_DAG,    // out = Dslash^+ in
    HOP_SCHUR_B_SYM, // out = c - 1/4 K5^-1 Dslash in (the table's m holds K5^-1)
    // S B^-1 (right preconditioning by B) and its adjoint B^-+ S^+:
    HOP_SCHUR_A_RP,      // out = B K5^-1 Dslash in
    HOP_SCHUR_B_RP,      // out = K5 B^-1 c - 1/4 Dslash in
    HOP_SCHUR_B_DAG_RP   // out = (K5 B^-1)^+ c - 1/4 Dslash^+ in (A^+ is HOP_SCHUR_A_DAG)
};

struct HopLaunch {
    HopKind kind;
    Prec prec;
    int out_parity;
    void* out;
    const void* in;       // neighbour field (parity 1 - out_parity)
    const void* centre;   // field at the output parity (K5 / identity term)
    size_t stride;        // bytes between right-hand sides of in/out/centre
    int nrhs;
    const RhsCoef* coef;  // device, [nrhs]
    const int* active;    // device, [nrhs] or nullptr
    double* partials;     // device, [nrhs][nblocks] when a norm is wanted, else nullptr
    int nblocks_per_rhs;  // filled by the launcher
};

enum FifthKind { FIFTH_K5 = 0, FIFTH_K5INV, FIFTH_B, FIFTH_BINV };

void launch_hop(const Geo& g, const GaugeSet& gs, HopLaunch& L, hipStream_t st);
// The plane-staged bare hop (dslash_plane.hip) when the launch shape selects
// it and it applies to this launch; false (nothing launched) otherwise.
bool launch_hop_plane(const Geo& g, const GaugeSet& gs, HopLaunch& L, hipStream_t st);
size_t plane_lds_limit();
void launch_fifth(const Geo& g, Prec p, FifthKind kind, int dag, const void* in, void* out, size_t stride,
                  int nrhs, const RhsCoef* coef, const int* active, hipStream_t st);
int hop_blocks_per_rhs(const Geo& g);

// BLAS and conversions (blas.hip)
void launch_gauge_layout(const Geo& g, const double* canon, GaugeSet& gs, hipStream_t st);
void launch_pack(const Geo& g, Prec p, int kind, const double* canon, void* native, hipStream_t st);
void launch_unpack(const Geo& g, Prec p, int kind, const void* native, double* canon, hipStream_t st);
// one parity: full = 1 reads/writes the canonical full field, 0 the parity-compressed half
void launch_pack_parity(const Geo& g, Prec p, int full, int par, const double* canon, void* dst, hipStream_t st);
void launch_unpack_parity(const Geo& g, Prec p, int full, int par, const void* src, double* canon, hipStream_t st);
void launch_convert(const Geo& g, Prec pin, Prec pout, const void* in, void* out, size_t sin, size_t sout,
                    int nrhs, const int* active, hipStream_t st);
// z = a*x + b*y per RHS, scalars from host; optional norm partials of z
void launch_axpby(const Geo& g, Prec p, double a, const void* x, double b, const void* y, void* z, size_t stride,
                  int nrhs, const int* active, double* partials, hipStream_t st);
void launch_norm2(const Geo& g, Prec p, const void* x, size_t stride, int nrhs, const int* active,
                  double* partials, hipStream_t st);
// r(pi) -= alpha[r] * q(pi); partials <- |r|^2
struct CGScal;
void launch_cg_r(const Geo& g, Prec pi, void* r, const void* q, size_t si, int nrhs, const int* active,
                 const CGScal* sc, double* partials, hipStream_t st);
// Two-iteration solution update.  Even iteration: pn = s + beta p (x waits).
// Odd iteration: x += alpha_prev pp + alpha p, then pp = s + beta p (pp holds
// the even iteration's direction on entry, the next direction on exit).
void launch_cg_p(const Geo& g, Prec pi, void* pn, const void* p, const void* s, size_t si, int nrhs,
                 const int* active, const CGScal* sc, hipStream_t st);
void launch_cg_xp2(const Geo& g, Prec px, Prec pi, void* x, size_t sx, void* pp, const void* p, const void* s,
                   size_t si, int nrhs, const int* active, const CGScal* sc, hipStream_t st);
// x += alpha_prev p: the pending half of a two-iteration update
void launch_cg_xpend(const Geo& g, Prec px, Prec pi, void* x, size_t sx, const void* p, size_t si, int nrhs,
                     const int* active, const CGScal* sc, hipStream_t st);
// x_hi(P64) += x_lo(px); x_lo = 0
void launch_flush(const Geo& g, Prec px, void* xhi, size_t shi, void* xlo, size_t slo, int nrhs,
                  const int* active, hipStream_t st);
int blas_blocks_per_rhs(const Geo& g);
// Point-source columns and wall fields (blas.hip): src = x, y, z, t and the
// spin-colour column; even / odd are FP64 native halves.
void launch_point_source(const Geo& g, const int src[5], void* even, void* odd, hipStream_t st);
void launch_wall_field(const Geo& g, const void* even, const void* odd, double* q, hipStream_t st);

// Per-RHS scalar state of the CG recursion, in device memory.
struct CGScal {
    double gamma;   // ||s||^2
    double delta;   // ||q||^2
    double alpha, beta;
    double rr;      // ||r||^2 (iterated)
    int bad;        // NaN/Inf or breakdown seen
    int pad;
    double alpha_prev;   // alpha of the last even iteration, its x update pending
};
// SC_ALPHA_KEEP: SC_ALPHA and alpha_prev = alpha (even iterations);
// SC_CLEAR_PREV: alpha_prev = 0 (its update applied)
enum ScalOp { SC_ALPHA = 0, SC_BETA, SC_SET_GAMMA, SC_RR, SC_SUM, SC_ALPHA_KEEP, SC_CLEAR_PREV };
// Reduce partials per RHS in a fixed order and update the scalars.
void launch_scalars(ScalOp op, const double* partials, int nblk, int nrhs, const int* active, CGScal* sc,
                    double* out_sum, hipStream_t st);

}  // namespace mdwf
