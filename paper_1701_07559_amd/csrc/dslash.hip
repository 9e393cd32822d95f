// Wilson hop on every fifth-dimension slice, fused with the fifth-dimension
// operators of the Moebius domain-wall operator (arXiv:1701.07559, Sec. II).
//
// Thread mapping: the L5 slices of one 4D site sit in L5 consecutive lanes of
// one wavefront (64 / L5 sites per wave; the remaining lanes idle).  All lanes
// of a site read the same eight links, so a link is fetched once per site and
// reused across the fifth dimension, and the fifth-dimension couplings (B, C,
// K5 and the dense B K5^-1) become exchanges inside that lane group:
// ds_bpermute for the nearest-slice terms, an LDS tile for the dense L5 x L5
// polynomials.  Spinors are read 16 bytes per lane from the structure-of-
// arrays layout, so a wave's loads of one block are contiguous.
#include "mdwf_internal.h"

namespace mdwf {

// ----------------------------------------------------------- lane exchange
__device__ __forceinline__ float bperm(int addr, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}
__device__ __forceinline__ double bperm(int addr, double v) {
    int lo = __builtin_amdgcn_ds_bpermute(addr, __double2loint(v));
    int hi = __builtin_amdgcn_ds_bpermute(addr, __double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <typename R> __device__ __forceinline__ cx<R> bperm(int addr, cx<R> v) {
    return {bperm(addr, v.re), bperm(addr, v.im)};
}

// Exchange partners of lane s inside its site group: s-1 and s+1 with
// wrap-around; the wrapped term carries -m_q (quark-mass coupling of walls).
template <typename R> struct Nbr5 {
    int am1, ap1;   // bpermute byte addresses of lanes s-1, s+1
    R fm1, fp1;     // 1, or -m_q on the wrap
};

// (C v) with C = P- shift(s+1) + P+ shift(s-1) (dag = 0) or C^+ (dag = 1);
// spins 0,1 are P+ (components 0..5), spins 2,3 are P- (components 6..11).
template <typename R, bool DAGC>
__device__ __forceinline__ void apply_C_lanes(const Nbr5<R>& n, const cx<R> v[12], cx<R> out[12]) {
    const int aU = DAGC ? n.ap1 : n.am1;
    const R fU = DAGC ? n.fp1 : n.fm1;
    const int aD = DAGC ? n.am1 : n.ap1;
    const R fD = DAGC ? n.fm1 : n.fp1;
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = fU * bperm(aU, v[c]);
#pragma unroll
    for (int c = 6; c < 12; ++c) out[c] = fD * bperm(aD, v[c]);
}

// ------------------------------------------------------------ spin algebra
// Chiral basis: g_mu = [[0, G],[G^+, 0]] with G_x = -i s1, G_y = -i s2,
// G_z = -i s3, G_t = 1.  (1 - sg g_mu) psi = (h, -sg G^+ h) with the half
// spinor h = u - sg G d (u, d = upper and lower spin pairs).
template <int MU, typename R>
__device__ __forceinline__ void project(R sg, const cx<R> in[12], cx<R> h[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<R> u0 = in[a], u1 = in[3 + a], d0 = in[6 + a], d1 = in[9 + a];
        if (MU == 0) {        // G d = (-i d1, -i d0)
            h[a] = u0 + sg * timesI(d1);
            h[3 + a] = u1 + sg * timesI(d0);
        } else if (MU == 1) { // G d = (-d1, d0)
            h[a] = u0 + sg * d1;
            h[3 + a] = u1 - sg * d0;
        } else if (MU == 2) { // G d = (-i d0, i d1)
            h[a] = u0 + sg * timesI(d0);
            h[3 + a] = u1 - sg * timesI(d1);
        } else {              // G d = d
            h[a] = u0 - sg * d0;
            h[3 + a] = u1 - sg * d1;
        }
    }
}

template <int MU, typename R>
__device__ __forceinline__ void reconstruct_add(R sg, const cx<R> w[6], cx<R> acc[12]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const cx<R> w0 = w[a], w1 = w[3 + a];
        acc[a] = acc[a] + w0;
        acc[3 + a] = acc[3 + a] + w1;
        if (MU == 0) {        // -sg G^+ w = (-sg i w1, -sg i w0)
            acc[6 + a] = acc[6 + a] - sg * timesI(w1);
            acc[9 + a] = acc[9 + a] - sg * timesI(w0);
        } else if (MU == 1) { // (-sg w1, +sg w0)
            acc[6 + a] = acc[6 + a] - sg * w1;
            acc[9 + a] = acc[9 + a] + sg * w0;
        } else if (MU == 2) { // (-sg i w0, +sg i w1)
            acc[6 + a] = acc[6 + a] - sg * timesI(w0);
            acc[9 + a] = acc[9 + a] + sg * timesI(w1);
        } else {              // (-sg w0, -sg w1)
            acc[6 + a] = acc[6 + a] - sg * w0;
            acc[9 + a] = acc[9 + a] - sg * w1;
        }
    }
}

// w = U h (FWD) or U^+ h, on the two colour vectors of a half spinor.
template <bool FWD, typename R>
__device__ __forceinline__ void su3_mul(const cx<R> U[9], const cx<R> h[6], cx<R> w[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> acc = {R(0), R(0)};
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                if (FWD)
                    acc = cmadd(acc, U[a * 3 + b], h[sp * 3 + b]);
                else
                    acc = cjmadd(acc, U[b * 3 + a], h[sp * 3 + b]);
            }
            w[sp * 3 + a] = acc;
        }
}

// ------------------------------------------------ binary16 packed arithmetic
// FP16 spinors and links hold one complex number per 32-bit word as a pair of
// binary16 values (re, im).  The FP16 hop keeps them packed: projections are
// packed-half adds, and the SU(3) product uses v_dot2_f32_f16, which sums two
// half products into an FP32 accumulator, so the stored values enter the
// product without conversion and every sum is carried in FP32.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ h2 as_h2(uint32_t w) { return __builtin_bit_cast(h2, w); }
__device__ __forceinline__ h2 splat_h2(float f) {
    const _Float16 h = _Float16(f);
    return h2{h, h};
}
// a.x b.x + a.y b.y + c
__device__ __forceinline__ float dot2(h2 a, h2 b, float c) { return __builtin_amdgcn_fdot2(a, b, c, false); }

// From z = u + SGN X d (X = i for TI, else 1) the two packed operands that
// make U z (FWD) or U^+ z a sum of dot2 products with the link element:
//   U z:   re = sum Ur zr - Ui zi = dot(U, (zr, -zi)),  im = dot(U, (zi, zr))
//   U^+ z: re = dot(U, (zr, zi)),                     im = dot(U, (zi, -zr))
// The sign flips and swaps act on u and X d before the packed add, where
// they are operand modifiers.
template <bool TI, int SGN, bool FWD>
__device__ __forceinline__ void comb_h(h2 u, h2 d, h2& z1, h2& z2) {
    const h2 xd = TI ? h2{-d.y, d.x} : d;   // X d
    h2 a1, b1, a2, b2;
    if (FWD) {
        a1 = h2{u.x, -u.y}, b1 = h2{xd.x, -xd.y};   // conjugate
        a2 = h2{u.y, u.x}, b2 = h2{xd.y, xd.x};     // swapped
    } else {
        a1 = u, b1 = xd;
        a2 = h2{u.y, -u.x}, b2 = h2{xd.y, -xd.x};   // swapped conjugate
    }
    z1 = SGN > 0 ? a1 + b1 : a1 - b1;
    z2 = SGN > 0 ? a2 + b2 : a2 - b2;
}

// Packed version of project<MU>, returning the product operands of comb_h.
template <int MU, int SG, bool FWD>
__device__ __forceinline__ void project_h(const h2 in[12], h2 z1[6], h2 z2[6]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const h2 u0 = in[a], u1 = in[3 + a], d0 = in[6 + a], d1 = in[9 + a];
        if (MU == 0) {
            comb_h<true, SG, FWD>(u0, d1, z1[a], z2[a]);
            comb_h<true, SG, FWD>(u1, d0, z1[3 + a], z2[3 + a]);
        } else if (MU == 1) {
            comb_h<false, SG, FWD>(u0, d1, z1[a], z2[a]);
            comb_h<false, -SG, FWD>(u1, d0, z1[3 + a], z2[3 + a]);
        } else if (MU == 2) {
            comb_h<true, SG, FWD>(u0, d0, z1[a], z2[a]);
            comb_h<true, -SG, FWD>(u1, d1, z1[3 + a], z2[3 + a]);
        } else {
            comb_h<false, -SG, FWD>(u0, d0, z1[a], z2[a]);
            comb_h<false, -SG, FWD>(u1, d1, z1[3 + a], z2[3 + a]);
        }
    }
}

// w = U h (FWD) or U^+ h with binary16 inputs and FP32 sums (operands from
// project_h).
template <bool FWD>
__device__ __forceinline__ void su3_mul_h(const h2 U[9], const h2 z1[6], const h2 z2[6], cx<float> w[6]) {
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const h2 u = FWD ? U[a * 3 + b] : U[b * 3 + a];
                re = dot2(u, z1[sp * 3 + b], re);
                im = dot2(u, z2[sp * 3 + b], im);
            }
            w[sp * 3 + a] = {re, im};
        }
}

// ----------------------------------------------------------- hop kernels
struct HopDev {
    void* out;
    const void* in;
    const void* centre;
    const char* links_out;   // segments (mu = 0..3) of the output parity
    const char* links_in;    // segments of the input parity
    size_t lseg;
    size_t stride;
    int nrhs;
    int nblk;
    int out_parity;
    const RhsCoef* coef;
    const int* active;
    double* partials;
};

template <int K> struct HopTraits {
    static constexpr bool dag = (K == HOP_D5_DAG || K == HOP_SCHUR_A_DAG || K == HOP_SCHUR_B_DAG || K == HOP_BARE_DAG ||
                                 K == HOP_SCHUR_B_DAG_RP);
    static constexpr bool preB = (K == HOP_D5 || K == HOP_SCHUR_A || K == HOP_PREP);
    // epilogue on the hop result: 0 none, 1 sum_k m_k C^k (B K5^-1, or K5^-1
    // for the symmetric form's kernel B), 2 its adjoint, 3 B^+
    static constexpr int epi = (K == HOP_SCHUR_A || K == HOP_SCHUR_B_SYM || K == HOP_SCHUR_A_RP) ? 1
                             : (K == HOP_SCHUR_A_DAG) ? 2
                             : (K == HOP_D5_DAG || K == HOP_SCHUR_B_DAG) ? 3 : 0;
    // centre term: 0 none, 1 K5, 2 K5^+, 3 identity, 4 dense K5 B^-1 =
    // sum_k w_k C^k, 5 its adjoint
    static constexpr int cen = (K == HOP_D5 || K == HOP_SCHUR_B) ? 1
                             : (K == HOP_D5_DAG || K == HOP_SCHUR_B_DAG) ? 2
                             : (K == HOP_PREP || K == HOP_SCHUR_B_SYM) ? 3
                             : (K == HOP_SCHUR_B_RP) ? 4 : (K == HOP_SCHUR_B_DAG_RP) ? 5 : 0;
    // kernels B and B^+ also return block partial sums of |out|^2 (CG norms)
    static constexpr bool norm = (K == HOP_SCHUR_B || K == HOP_SCHUR_B_DAG || K == HOP_SCHUR_B_SYM ||
                                  K == HOP_SCHUR_B_RP || K == HOP_SCHUR_B_DAG_RP);
    static constexpr double coef = (K == HOP_D5 || K == HOP_D5_DAG) ? -0.5
                                 : (K == HOP_SCHUR_B || K == HOP_SCHUR_B_DAG || K == HOP_SCHUR_B_SYM ||
                                    K == HOP_SCHUR_B_RP || K == HOP_SCHUR_B_DAG_RP) ? -0.25
                                 : (K == HOP_PREP) ? 0.5 : 1.0;
};

// ------------------------------------------------------ neighbour loads
// Raw registers of one direction: the link and the neighbour spinor exactly
// as stored.  Addresses are a wave-uniform block base plus a 32-bit lane
// offset (the offset of a 16-byte element inside one block stays below 4 GB
// for every lattice this library accepts), so the loads use scalar-base
// addressing and cost one VGPR of address per direction.
template <typename V> __device__ __forceinline__ V ldu(const char* base, uint32_t byte_off) {
    return *reinterpret_cast<const V*>(base + byte_off);
}
typedef float nf2 __attribute__((ext_vector_type(2)));

template <Prec P> struct Raw;

template <> struct Raw<P64> {
    nd2 s[12], u[9];
    __device__ __forceinline__ void load(const char* lseg, uint32_t li, size_t lblk, const char* in, uint32_t jn,
                                         size_t sblk, bool with_link) {
        const uint32_t lo = li * 16u, so = jn * 16u;
        if (with_link)
#pragma unroll
            for (int k = 0; k < 9; ++k) u[k] = ldu<nd2>(lseg + k * lblk, lo);
#pragma unroll
        for (int k = 0; k < 12; ++k) s[k] = ldu<nd2>(in + k * sblk, so);
    }
    __device__ __forceinline__ void link(cx<double> U[9]) const {
#pragma unroll
        for (int k = 0; k < 9; ++k) U[k] = {u[k].x, u[k].y};
    }
    __device__ __forceinline__ void spinor(cx<double> v[12]) const {
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = {s[k].x, s[k].y};
    }
};

template <> struct Raw<P32> {
    nf4 s[6], u[4];
    nf2 u8;
    __device__ __forceinline__ void load(const char* lseg, uint32_t li, size_t lblk, const char* in, uint32_t jn,
                                         size_t sblk, bool with_link) {
        const uint32_t lo = li * 16u, so = jn * 16u;
        if (with_link) {
#pragma unroll
            for (int k = 0; k < 4; ++k) u[k] = ldu<nf4>(lseg + k * lblk, lo);
            u8 = ldu<nf2>(lseg + 4 * lblk, li * 8u);   // 9th element: float2 block after the four float4 blocks
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) s[k] = ldu<nf4>(in + k * sblk, so);
    }
    __device__ __forceinline__ void link(cx<float> U[9]) const {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            U[2 * k] = {u[k].x, u[k].y};
            U[2 * k + 1] = {u[k].z, u[k].w};
        }
        U[8] = {u8.x, u8.y};
    }
    // Gathered link: lane s of the site group loads 16-byte part min(s, 3)
    // and the 8-byte tail itself; the other lanes' parts come by lane
    // exchange from lanes gbase + p (no branch, so loads stay in order).
    __device__ __forceinline__ void load_part(const char* lseg, uint32_t li, size_t lblk, int s) {
        u[0] = ldu<nf4>(lseg + size_t(s < 3 ? s : 3) * lblk, li * 16u);
        u8 = ldu<nf2>(lseg + 4 * lblk, li * 8u);
    }
    __device__ __forceinline__ void link_shfl(int a0, cx<float> U[9]) const {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            U[2 * p] = {bperm(a0 + 4 * p, u[0].x), bperm(a0 + 4 * p, u[0].y)};
            U[2 * p + 1] = {bperm(a0 + 4 * p, u[0].z), bperm(a0 + 4 * p, u[0].w)};
        }
        U[8] = {u8.x, u8.y};
    }
    __device__ __forceinline__ void spinor(cx<float> v[12]) const {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            v[2 * k] = {s[k].x, s[k].y};
            v[2 * k + 1] = {s[k].z, s[k].w};
        }
    }
};

template <> struct Raw<P16> {
    nu4 s[3], u[2];
    uint32_t u8;
    float n;
    __device__ __forceinline__ void load(const char* lseg, uint32_t li, size_t lblk, const char* in, uint32_t jn,
                                         size_t sblk, bool with_link) {
        const uint32_t lo = li * 16u, so = jn * 16u;
        if (with_link) {
#pragma unroll
            for (int k = 0; k < 2; ++k) u[k] = ldu<nu4>(lseg + k * lblk, lo);
            u8 = ldu<uint32_t>(lseg + 2 * lblk, li * 4u);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) s[k] = ldu<nu4>(in + k * sblk, so);
        n = ldu<float>(in + align256(3 * sblk), jn * 4u);   // norm block (see norm_offset)
    }
    __device__ __forceinline__ void link_h(h2 U[9]) const {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            U[4 * k] = as_h2(u[k].x);
            U[4 * k + 1] = as_h2(u[k].y);
            U[4 * k + 2] = as_h2(u[k].z);
            U[4 * k + 3] = as_h2(u[k].w);
        }
        U[8] = as_h2(u8);
    }
    // Gathered link: lane s loads 16-byte part min(s, 1) and the 4-byte tail
    // itself; the two 16-byte parts come by lane exchange from lanes gbase,
    // gbase + 1.
    __device__ __forceinline__ void load_part(const char* lseg, uint32_t li, size_t lblk, int s) {
        u[0] = ldu<nu4>(lseg + size_t(s < 1 ? s : 1) * lblk, li * 16u);
        u8 = ldu<uint32_t>(lseg + 2 * lblk, li * 4u);
    }
    __device__ __forceinline__ void link_shfl_h(int a0, h2 U[9]) const {
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            U[4 * p] = as_h2(uint32_t(__builtin_amdgcn_ds_bpermute(a0 + 4 * p, int(u[0].x))));
            U[4 * p + 1] = as_h2(uint32_t(__builtin_amdgcn_ds_bpermute(a0 + 4 * p, int(u[0].y))));
            U[4 * p + 2] = as_h2(uint32_t(__builtin_amdgcn_ds_bpermute(a0 + 4 * p, int(u[0].z))));
            U[4 * p + 3] = as_h2(uint32_t(__builtin_amdgcn_ds_bpermute(a0 + 4 * p, int(u[0].w))));
        }
        U[8] = as_h2(u8);
    }
    // the stored spinor as binary16 pairs; its value is scale * v
    __device__ __forceinline__ float spinor_h(h2 v[12]) const {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[4 * k] = as_h2(s[k].x);
            v[4 * k + 1] = as_h2(s[k].y);
            v[4 * k + 2] = as_h2(s[k].z);
            v[4 * k + 3] = as_h2(s[k].w);
        }
        return n;
    }
    // B psi = b5 psi_s + c5 (C psi)_s as binary16 pairs times a returned
    // scale.  The three contributing slices carry their own norms; with
    // S = max(b5 n_s, c5 |f| n_s-1, c5 |f| n_s+1, FLT_MIN) every coefficient
    // divided by S lies in [-1, 1], so the packed sum stays in range
    // (|v| <= 2).  The FLT_MIN floor keeps 1/S finite: across the wall f is
    // -m_q, and c5 m_q n can be sub-normal next to a zero slice.
    __device__ __forceinline__ float spinor_B_h(const Nbr5<float>& nb, float b5, float c5, h2 v[12]) const {
        const uint32_t up[6] = {s[0].x, s[0].y, s[0].z, s[0].w, s[1].x, s[1].y};
        const uint32_t dn[6] = {s[1].z, s[1].w, s[2].x, s[2].y, s[2].z, s[2].w};
        const float a0 = b5 * n;
        const float au = c5 * nb.fm1 * bperm(nb.am1, n);   // (C psi) upper from slice s-1
        const float ad = c5 * nb.fp1 * bperm(nb.ap1, n);   // lower from slice s+1
        const float S = fmaxf(fmaxf(a0, 1.17549435e-38f), fmaxf(fabsf(au), fabsf(ad)));
        const float inv = __builtin_amdgcn_rcpf(S);
        const h2 ha = splat_h2(a0 * inv), hu = splat_h2(au * inv), hd = splat_h2(ad * inv);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const h2 o = as_h2(uint32_t(__builtin_amdgcn_ds_bpermute(nb.am1, int(up[k]))));
            v[k] = ha * as_h2(up[k]) + hu * o;
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const h2 o = as_h2(uint32_t(__builtin_amdgcn_ds_bpermute(nb.ap1, int(dn[k]))));
            v[6 + k] = ha * as_h2(dn[k]) + hd * o;
        }
        return S;
    }
};

// Links staged in LDS: 16-byte parts of the 18-real link.  Lane s of a site
// group copies parts s, s + L5, ... of each of its site's eight links; every
// lane then reads its site's links back (a broadcast inside the group), so a
// link crosses the vector-memory path once per site instead of once per lane.
template <Prec P> struct LinkStage;
template <> struct LinkStage<P64> {
    static constexpr int NP = 9;
    static __device__ __forceinline__ void copy_part(const char* seg, size_t lblk, uint32_t idx, int b,
                                                     unsigned char* dst) {
        *reinterpret_cast<nd2*>(dst) = ldu<nd2>(seg + b * lblk, idx * 16u);
    }
    static __device__ __forceinline__ void read(const unsigned char* slot, cx<double> U[9]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const nd2 w = reinterpret_cast<const nd2*>(slot)[k];
            U[k] = {w.x, w.y};
        }
    }
};
template <> struct LinkStage<P32> {
    static constexpr int NP = 5;
    static __device__ __forceinline__ void copy_part(const char* seg, size_t lblk, uint32_t idx, int b,
                                                     unsigned char* dst) {
        if (b < 4) *reinterpret_cast<nf4*>(dst) = ldu<nf4>(seg + b * lblk, idx * 16u);
        else *reinterpret_cast<nf2*>(dst) = ldu<nf2>(seg + 4 * lblk, idx * 8u);
    }
    static __device__ __forceinline__ void read(const unsigned char* slot, cx<float> U[9]) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const nf4 w = reinterpret_cast<const nf4*>(slot)[k];
            U[2 * k] = {w.x, w.y};
            U[2 * k + 1] = {w.z, w.w};
        }
        const nf2 w = *reinterpret_cast<const nf2*>(slot + 64);
        U[8] = {w.x, w.y};
    }
};
template <> struct LinkStage<P16> {
    static constexpr int NP = 3;
    static __device__ __forceinline__ void copy_part(const char* seg, size_t lblk, uint32_t idx, int b,
                                                     unsigned char* dst) {
        if (b < 2) *reinterpret_cast<nu4*>(dst) = ldu<nu4>(seg + b * lblk, idx * 16u);
        else *reinterpret_cast<uint32_t*>(dst) = ldu<uint32_t>(seg + 2 * lblk, idx * 4u);
    }
    static __device__ __forceinline__ void read_h(const unsigned char* slot, h2 U[9]) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const nu4 w = reinterpret_cast<const nu4*>(slot)[k];
            U[4 * k] = as_h2(w.x);
            U[4 * k + 1] = as_h2(w.y);
            U[4 * k + 2] = as_h2(w.z);
            U[4 * k + 3] = as_h2(w.w);
        }
        U[8] = as_h2(*reinterpret_cast<const uint32_t*>(slot + 32));
    }
};

// Accumulate one direction's term from its spinor registers and link.
template <Prec P, bool DAG, bool PREB, int MU, int DIR>
__device__ __forceinline__ void hop_term(cx<typename Real<P>::T> acc[12], const Raw<P>& r,
                                         const cx<typename Real<P>::T> U[9],
                                         const Nbr5<typename Real<P>::T>& nb, typename Real<P>::T b5,
                                         typename Real<P>::T c5) {
    using R = typename Real<P>::T;
    cx<R> psi[12];
    r.spinor(psi);
    if (PREB) {
        cx<R> cpsi[12];
        apply_C_lanes<R, false>(nb, psi, cpsi);
#pragma unroll
        for (int c = 0; c < 12; ++c) psi[c] = b5 * psi[c] + c5 * cpsi[c];
    }
    constexpr R sg = ((DIR > 0) != DAG) ? R(1) : R(-1);
    cx<R> h[6], w[6];
    project<MU>(sg, psi, h);
    su3_mul<(DIR > 0)>(U, h, w);
    reconstruct_add<MU>(sg, w, acc);
}

// FP16 storage: the same term on binary16 pairs (see su3_mul_h); the spinor
// scale (its norm, or the B pre-hop's common scale) is applied once, in FP32,
// when the colour product is added to the accumulator.
template <bool DAG, bool PREB, int MU, int DIR>
__device__ __forceinline__ void hop_term_h(cx<float> acc[12], const Raw<P16>& r, const h2 U[9],
                                           const Nbr5<float>& nb, float b5, float c5) {
    h2 psi[12];
    const float scale = PREB ? r.spinor_B_h(nb, b5, c5, psi) : r.spinor_h(psi);
    constexpr int sg = ((DIR > 0) != DAG) ? 1 : -1;
    h2 z1[6], z2[6];
    project_h<MU, sg, (DIR > 0)>(psi, z1, z2);
    cx<float> w[6];
    su3_mul_h<(DIR > 0)>(U, z1, z2, w);
#pragma unroll
    for (int c = 0; c < 6; ++c) w[c] = scale * w[c];
    reconstruct_add<MU>(float(sg), w, acc);
}

// Direction d of the fixed order x+, x-, y+, y-, z+, z-, t+, t-.  Link mode
// LM: 0 every lane holds the whole link, 1 LDS stage, 2 gathered from the
// part-holding lanes of the site group (a0: byte address of its first lane).
template <Prec P, bool DAG, bool PREB, int D, int LM>
__device__ __forceinline__ void dir_term(cx<typename Real<P>::T> acc[12], const Raw<P>& r,
                                         const unsigned char* slot, int a0, const Nbr5<typename Real<P>::T>& nb,
                                         typename Real<P>::T b5, typename Real<P>::T c5) {
    if constexpr (P == P16) {
        h2 U[9];
        if constexpr (LM == 1) LinkStage<P16>::read_h(slot, U);
        else if constexpr (LM == 2) r.link_shfl_h(a0, U);
        else r.link_h(U);
        hop_term_h<DAG, PREB, D / 2, (D % 2 == 0) ? +1 : -1>(acc, r, U, nb, b5, c5);
    } else {
        cx<typename Real<P>::T> U[9];
        if constexpr (LM == 1) LinkStage<P>::read(slot, U);
        else if constexpr (LM == 2) r.link_shfl(a0, U);
        else r.link(U);
        hop_term<P, DAG, PREB, D / 2, (D % 2 == 0) ? +1 : -1>(acc, r, U, nb, b5, c5);
    }
}

// Link modes (see dir_term): the LDS stage needs at most kStageSites sites per
// wave (L5 >= 8), the lane gather needs L5 >= the number of 16-byte parts.
constexpr int kStageSites = 8;
// 16-byte parts gathered by lane exchange (the short tail is loaded by every lane)
template <Prec P> constexpr int link_parts() { return P == P64 ? 9 : P == P32 ? 4 : 2; }

template <Prec P, int K, int LM>
__global__ void __launch_bounds__(kBlock) k_hop(const Geo g, const HopDev a) {
    using R = typename Real<P>::T;
    using TR = HopTraits<K>;
    const int L5 = g.L5;
    const int spw = 64 / L5;
    const int lb = g.xcd_remap[P] ? xcd_logical_block(blockIdx.x, gridDim.x) : int(blockIdx.x);
    // RHS groups of rg: the blocks of one group sweep the tiles with the
    // group's RHS fastest (they share each tile's links in L2); groups follow
    // each other, so a spinor's neighbour reuse spans rg RHS, not all of them
    int rhs, tile;
    {
        const int rg = (g.rhs_group[P] > 0 && g.rhs_group[P] < a.nrhs) ? g.rhs_group[P] : a.nrhs;
        const int grp = lb / (a.nblk * rg);
        const int base = grp * rg;
        const int gs = min(rg, a.nrhs - base);
        const int off = lb - grp * a.nblk * rg;
        tile = off / gs;
        rhs = base + (off - tile * gs);
    }
    if (a.active && !a.active[rhs]) return;   // uniform over the block
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int sw = lane / L5;
    const int s = lane - sw * L5;
    const int pos = (tile * kWaves + wave) * spw + sw;   // traversal position
    const bool valid = (sw < spw) && (pos < g.Vh4);
    const int gbase = lane - s;
    // traversal position -> tile and place inside it (see Trav) ->
    // coordinates and the parity-compressed index i of the output site
    int xh, y, z, t, i;
    {
        const Trav& tr = g.trav[P];
        const uint32_t p = uint32_t(pos);
        const uint32_t q = tr.fTv.div(p);               // tile number
        const uint32_t r = p - q * uint32_t(tr.b[0] * tr.b[1] * tr.b[2] * tr.b[3]);
        const uint32_t r1 = tr.fBx.div(r), r2 = tr.fBy.div(r1), r3 = tr.fBz.div(r2);   // in-tile
        const uint32_t q1 = tr.fNt.div(q), q2 = tr.fNx.div(q1), q3 = tr.fNy.div(q2);   // tile grid
        const uint32_t nt = tr.fNt.d, nx = tr.fNx.d, ny = tr.fNy.d;
        xh = int(q1 - q2 * nx) * tr.b[0] + int(r - r1 * uint32_t(tr.b[0]));
        y = int(q2 - q3 * ny) * tr.b[1] + int(r1 - r2 * uint32_t(tr.b[1]));
        z = int(q3) * tr.b[2] + int(r2 - r3 * uint32_t(tr.b[2]));
        t = int(q - q1 * nt) * tr.b[3] + int(r3);
        i = xh + g.Xh * (y + g.Y * (z + g.Z * t));
    }

    const RhsCoef& cf = a.coef[rhs];
    const R mq = R(cf.mq), b5 = R(cf.b5), c5 = R(cf.c5);
    Nbr5<R> nb;
    nb.am1 = (gbase + (s == 0 ? L5 - 1 : s - 1)) << 2;
    nb.ap1 = (gbase + (s == L5 - 1 ? 0 : s + 1)) << 2;
    nb.fm1 = (s == 0) ? -mq : R(1);
    nb.fp1 = (s == L5 - 1) ? -mq : R(1);

    const void* in = at_rhs(a.in, a.stride, rhs);
    // -0 is an exact additive identity, so the first direction's sums into
    // res compile to plain moves (+0 would need its own register clears)
    cx<R> res[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) res[c] = {R(-0.0), R(-0.0)};

    // neighbours of the output site (used only by valid lanes)
    const int x = 2 * xh + ((y + z + t + a.out_parity) & 1);
    const int row = i - xh;
    const int sy = g.Xh, sz = g.Xh * g.Y, st = sz * g.Z;
    const int n_xp = row + ((x + 1 == g.X ? 0 : x + 1) >> 1);
    const int n_xm = row + ((x == 0 ? g.X - 1 : x - 1) >> 1);
    const int n_yp = i + (y == g.Y - 1 ? -(g.Y - 1) * sy : sy);
    const int n_ym = i + (y == 0 ? (g.Y - 1) * sy : -sy);
    const int n_zp = i + (z == g.Z - 1 ? -(g.Z - 1) * sz : sz);
    const int n_zm = i + (z == 0 ? (g.Z - 1) * sz : -sz);
    const int n_tp = i + (t == g.T - 1 ? -(g.T - 1) * st : st);
    const int n_tm = i + (t == 0 ? (g.T - 1) * st : -st);

    // links: segment mu of the output parity at i (forward) and of the input
    // parity at the backward neighbour
    const size_t ls = a.lseg;
    const size_t lblk = size_t(g.Vh4) * 16;
    const size_t sblk = size_t(g.Vh) * 16;
    const char* lo = a.links_out;
    const char* lk = a.links_in;
    const char* src = static_cast<const char*>(in);
    constexpr bool D = TR::dag, PB = TR::preB;
    const uint32_t ui = uint32_t(i);
    const char* seg[8] = {lo, lk, lo + ls, lk + ls, lo + 2 * ls, lk + 2 * ls, lo + 3 * ls, lk + 3 * ls};
    const uint32_t lidx[8] = {ui, uint32_t(n_xm), ui, uint32_t(n_ym), ui, uint32_t(n_zm), ui, uint32_t(n_tm)};
    const uint32_t jn[8] = {uint32_t(n_xp * L5 + s), uint32_t(n_xm * L5 + s), uint32_t(n_yp * L5 + s),
                            uint32_t(n_ym * L5 + s), uint32_t(n_zp * L5 + s), uint32_t(n_zm * L5 + s),
                            uint32_t(n_tp * L5 + s), uint32_t(n_tm * L5 + s)};

    // LDS: link stage (when a wave holds at most kStageSites sites) and, for
    // kernels A / A^+, the epilogue tile, which reuses the same bytes
    constexpr int NP = LinkStage<P>::NP;
    constexpr int kDirBytes = kStageSites * NP * 16;
    constexpr int kLinkBytes = LM == 1 ? kWaves * 8 * kDirBytes : 0;
    constexpr int kEpiBytes = (TR::epi == 1 || TR::epi == 2 || TR::cen == 4 || TR::cen == 5)
                                  ? 12 * kBlock * int(sizeof(cx<R>)) : 0;
    constexpr int kSmem = kLinkBytes > kEpiBytes ? kLinkBytes : kEpiBytes;
    __shared__ __align__(16) unsigned char smem[kSmem > 0 ? kSmem : 16];
    unsigned char* lslot = smem + size_t(wave) * 8 * kDirBytes + size_t(sw) * NP * 16;
    const int a0 = gbase << 2;
    if constexpr (LM == 1) {
        if (valid) {
            for (int b = s; b < NP; b += L5)
#pragma unroll
                for (int d = 0; d < 8; ++d)
                    LinkStage<P>::copy_part(seg[d], lblk, lidx[d], b, lslot + d * kDirBytes + b * 16);
        }
        __syncthreads();
    }

    if (valid) {
        if constexpr (P == P64) {
            // FP64: one direction in flight (two would exceed the register file)
            Raw<P> r;
#define MDWF_DIR(d)                                                                 \
    r.load(seg[d], lidx[d], lblk, src, jn[d], sblk, LM == 0);                      \
    dir_term<P, D, PB, d, LM>(res, r, lslot + (d) * kDirBytes, a0, nb, b5, c5);
            MDWF_DIR(0) MDWF_DIR(1) MDWF_DIR(2) MDWF_DIR(3) MDWF_DIR(4) MDWF_DIR(5) MDWF_DIR(6) MDWF_DIR(7)
#undef MDWF_DIR
        } else {
            // two directions in flight: load d + 1 before computing d
            Raw<P> r0, r1;
            r0.load(seg[0], lidx[0], lblk, src, jn[0], sblk, LM == 0);
            if constexpr (LM == 2) r0.load_part(seg[0], lidx[0], lblk, s);
#define MDWF_STEP(d, rc, rn)                                                          \
    rn.load(seg[(d) + 1], lidx[(d) + 1], lblk, src, jn[(d) + 1], sblk, LM == 0);     \
    if constexpr (LM == 2) rn.load_part(seg[(d) + 1], lidx[(d) + 1], lblk, s);        \
    dir_term<P, D, PB, d, LM>(res, rc, lslot + (d) * kDirBytes, a0, nb, b5, c5);
            MDWF_STEP(0, r0, r1) MDWF_STEP(1, r1, r0) MDWF_STEP(2, r0, r1) MDWF_STEP(3, r1, r0)
            MDWF_STEP(4, r0, r1) MDWF_STEP(5, r1, r0) MDWF_STEP(6, r0, r1)
#undef MDWF_STEP
            dir_term<P, D, PB, 7, LM>(res, r1, lslot + 7 * kDirBytes, a0, nb, b5, c5);
        }
    }

    // ---- epilogue on the hop result
    if constexpr (TR::epi == 1 || TR::epi == 2) {
        // dense B K5^-1 = sum_k m_k C^k (or its adjoint) across the L5 lanes;
        // the tile reuses the link stage once every wave is past its hop
        cx<R>* sh = reinterpret_cast<cx<R>*>(smem);
        if constexpr (LM == 1) __syncthreads();
#pragma unroll
        for (int c = 0; c < 12; ++c) sh[c * kBlock + tid] = res[c];
        __syncthreads();
        if (valid) {
            const int tbase = tid - s;
            // k = 0 (C^0 = 1) starts the sums
            cx<R> o[12];
            const R m0 = R(cf.m[0]);
#pragma unroll
            for (int c = 0; c < 12; ++c) o[c] = m0 * sh[c * kBlock + tid];
            for (int k = 1; k < L5; ++k) {
                const R mk = R(cf.m[k]);
                // C^k on P+ reads slice s-k, on P- slice s+k (adjoint: swapped)
                int su = (TR::epi == 1) ? s - k : s + k;
                int sd = (TR::epi == 1) ? s + k : s - k;
                R fu = mk, fd = mk;
                if (su < 0) { su += L5; fu = -mq * mk; }
                if (su >= L5) { su -= L5; fu = -mq * mk; }
                if (sd < 0) { sd += L5; fd = -mq * mk; }
                if (sd >= L5) { sd -= L5; fd = -mq * mk; }
#pragma unroll
                for (int c = 0; c < 6; ++c) o[c] = o[c] + fu * sh[c * kBlock + tbase + su];
#pragma unroll
                for (int c = 6; c < 12; ++c) o[c] = o[c] + fd * sh[c * kBlock + tbase + sd];
            }
#pragma unroll
            for (int c = 0; c < 12; ++c) res[c] = o[c];
        }
    } else if constexpr (TR::epi == 3) {
        if (valid) {   // B^+ = b5 + c5 C^+
            cx<R> cr[12];
            apply_C_lanes<R, true>(nb, res, cr);
#pragma unroll
            for (int c = 0; c < 12; ++c) res[c] = b5 * res[c] + c5 * cr[c];
        }
    }

    // dense centre term sum_k w_k C^k (or its adjoint) on the centre field:
    // the L5 lanes of a site exchange their values through LDS
    cx<R> cd[12];
    if constexpr (TR::cen == 4 || TR::cen == 5) {
        cx<R>* sh = reinterpret_cast<cx<R>*>(smem);
        cx<R> cv[12];
        // lanes past the lattice load site 0 (in bounds; no valid lane reads them)
        Field<P>::load(at_rhs(a.centre, a.stride, rhs), g.Vh, valid ? i * L5 + s : 0, cv);
        if constexpr (LM == 1) __syncthreads();   // every wave is past the link stage
#pragma unroll
        for (int c = 0; c < 12; ++c) sh[c * kBlock + tid] = cv[c];
        __syncthreads();
        if (valid) {
            const int tbase = tid - s;
            const R w0 = R(cf.w[0]);
#pragma unroll
            for (int c = 0; c < 12; ++c) cd[c] = w0 * cv[c];   // k = 0 starts the sums
            for (int k = 1; k < L5; ++k) {
                const R wk = R(cf.w[k]);
                // C^k on P+ reads slice s-k, on P- slice s+k (adjoint: swapped)
                int su = (TR::cen == 4) ? s - k : s + k;
                int sd = (TR::cen == 4) ? s + k : s - k;
                R fu = wk, fd = wk;
                if (su < 0) { su += L5; fu = -mq * wk; }
                if (su >= L5) { su -= L5; fu = -mq * wk; }
                if (sd < 0) { sd += L5; fd = -mq * wk; }
                if (sd >= L5) { sd -= L5; fd = -mq * wk; }
#pragma unroll
                for (int c = 0; c < 6; ++c) cd[c] = cd[c] + fu * sh[c * kBlock + tbase + su];
#pragma unroll
                for (int c = 6; c < 12; ++c) cd[c] = cd[c] + fd * sh[c * kBlock + tbase + sd];
            }
        }
    }

    double n2 = 0.0;
    if (valid) {
        const int j = i * L5 + s;
        const R hc = R(TR::coef);
        if constexpr (TR::cen == 4 || TR::cen == 5) {
#pragma unroll
            for (int c = 0; c < 12; ++c) res[c] = cd[c] + hc * res[c];
        } else if constexpr (TR::cen != 0) {
            cx<R> cv[12];
            Field<P>::load(at_rhs(a.centre, a.stride, rhs), g.Vh, j, cv);
            if constexpr (TR::cen == 1 || TR::cen == 2) {
                cx<R> cc[12];
                apply_C_lanes<R, TR::cen == 2>(nb, cv, cc);
                const R ka = R(cf.k5[0]), kb = R(cf.k5[1]);
#pragma unroll
                for (int c = 0; c < 12; ++c) res[c] = ka * cv[c] + kb * cc[c] + hc * res[c];
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) res[c] = cv[c] + hc * res[c];
            }
        } else if constexpr (TR::coef != 1.0) {
#pragma unroll
            for (int c = 0; c < 12; ++c) res[c] = hc * res[c];
        }
        if (g.nt_store[P]) Field<P>::template store<true>(at_rhs(a.out, a.stride, rhs), g.Vh, j, res);
        else Field<P>::store(at_rhs(a.out, a.stride, rhs), g.Vh, j, res);
        if (TR::norm && a.partials) {
            R acc = R(0);
#pragma unroll
            for (int c = 0; c < 12; ++c) acc += res[c].re * res[c].re + res[c].im * res[c].im;
            n2 = double(acc);
        }
    }
    if (TR::norm && a.partials) {
        // fixed-order reduction: wave (xor butterfly), then the 4 waves
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) n2 += __shfl_xor(n2, off, 64);
        __shared__ double wsum[kWaves];
        if (lane == 0) wsum[wave] = n2;
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += wsum[w];
            a.partials[size_t(rhs) * a.nblk + tile] = t;
        }
    }
}

int hop_blocks_per_rhs(const Geo& g) {
    const int spw = 64 / g.L5;
    const int sites_per_block = kWaves * spw;
    return (g.Vh4 + sites_per_block - 1) / sites_per_block;
}

template <Prec P, int K>
static void launch_hop_t(const Geo& g, const GaugeSet& gs, HopLaunch& L, hipStream_t st) {
    int lm = g.link_mode[P];
    if (lm == 1 && 64 / g.L5 > kStageSites) lm = 0;
    if (lm == 2 && (P == P64 || g.L5 < link_parts<P>())) lm = 0;
    HopDev a;
    a.out = L.out;
    a.in = L.in;
    a.centre = L.centre;
    const size_t seg = gs.seg_bytes[P];
    a.lseg = seg;
    a.links_out = gs.seg[P] + size_t(L.out_parity) * 4 * seg;
    a.links_in = gs.seg[P] + size_t(1 - L.out_parity) * 4 * seg;
    a.stride = L.stride;
    a.nrhs = L.nrhs;
    a.nblk = hop_blocks_per_rhs(g);
    a.out_parity = L.out_parity;
    a.coef = L.coef;
    a.active = L.active;
    a.partials = L.partials;
    L.nblocks_per_rhs = a.nblk;
    dim3 grid(a.nblk * L.nrhs);
    if (lm == 1) {
        hipLaunchKernelGGL((k_hop<P, K, 1>), grid, dim3(kBlock), 0, st, g, a);
    } else if (lm == 2) {
        if constexpr (P != P64) hipLaunchKernelGGL((k_hop<P, K, 2>), grid, dim3(kBlock), 0, st, g, a);
    } else {
        hipLaunchKernelGGL((k_hop<P, K, 0>), grid, dim3(kBlock), 0, st, g, a);
    }
}

template <Prec P>
static void launch_hop_p(const Geo& g, const GaugeSet& gs, HopLaunch& L, hipStream_t st) {
    switch (L.kind) {
        case HOP_BARE: launch_hop_t<P, HOP_BARE>(g, gs, L, st); break;
        case HOP_BARE_DAG: launch_hop_t<P, HOP_BARE_DAG>(g, gs, L, st); break;
        case HOP_D5: launch_hop_t<P, HOP_D5>(g, gs, L, st); break;
        case HOP_D5_DAG: launch_hop_t<P, HOP_D5_DAG>(g, gs, L, st); break;
        case HOP_SCHUR_A: launch_hop_t<P, HOP_SCHUR_A>(g, gs, L, st); break;
        case HOP_SCHUR_B: launch_hop_t<P, HOP_SCHUR_B>(g, gs, L, st); break;
        case HOP_SCHUR_A_DAG: launch_hop_t<P, HOP_SCHUR_A_DAG>(g, gs, L, st); break;
        case HOP_SCHUR_B_DAG: launch_hop_t<P, HOP_SCHUR_B_DAG>(g, gs, L, st); break;
        case HOP_PREP: launch_hop_t<P, HOP_PREP>(g, gs, L, st); break;
        case HOP_SCHUR_B_SYM: launch_hop_t<P, HOP_SCHUR_B_SYM>(g, gs, L, st); break;
        case HOP_SCHUR_A_RP: launch_hop_t<P, HOP_SCHUR_A_RP>(g, gs, L, st); break;
        case HOP_SCHUR_B_RP: launch_hop_t<P, HOP_SCHUR_B_RP>(g, gs, L, st); break;
        case HOP_SCHUR_B_DAG_RP: launch_hop_t<P, HOP_SCHUR_B_DAG_RP>(g, gs, L, st); break;
    }
}

void launch_hop(const Geo& g, const GaugeSet& gs, HopLaunch& L, hipStream_t st) {
    switch (L.prec) {
        case P64: launch_hop_p<P64>(g, gs, L, st); break;
        case P32: launch_hop_p<P32>(g, gs, L, st); break;
        case P16: launch_hop_p<P16>(g, gs, L, st); break;
    }
}

// ------------------------------------------------- site-local 5th dimension
// out = sum_k c_k C^k in (or with C^+), for K5, K5^-1 and B.
template <Prec P>
__global__ void __launch_bounds__(kBlock) k_fifth(const Geo g, int kind, int dag, const void* in, void* out,
                                                   size_t stride, int nrhs, int nblk, const RhsCoef* coef,
                                                   const int* active) {
    using R = typename Real<P>::T;
    const int L5 = g.L5;
    const int spw = 64 / L5;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int rhs = lb % nrhs;
    const int tile = lb / nrhs;
    if (active && !active[rhs]) return;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int sw = lane / L5;
    const int s = lane - sw * L5;
    const int i = (tile * kWaves + wave) * spw + sw;
    const bool valid = (sw < spw) && (i < g.Vh4);
    const int j = i * L5 + s;
    const RhsCoef& cf = coef[rhs];
    const R mq = R(cf.mq);

    __shared__ cx<R> sh[12 * kBlock];
    cx<R> v[12];
    if (valid) Field<P>::load(at_rhs(in, stride, rhs), g.Vh, j, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) sh[c * kBlock + tid] = valid ? v[c] : cx<R>{R(0), R(0)};
    __syncthreads();
    if (!valid) return;

    // K5 = k5[0] + k5[1] C, B = b5 + c5 C, K5^-1 = sum_k kinv[k] C^k,
    // B^-1 = sum_k binv[k] C^k
    double two[2];
    const double* ck;
    if (kind == FIFTH_K5) { two[0] = cf.k5[0]; two[1] = cf.k5[1]; ck = two; }
    else if (kind == FIFTH_B) { two[0] = cf.b5; two[1] = cf.c5; ck = two; }
    else if (kind == FIFTH_BINV) { ck = cf.binv; }
    else { ck = cf.kinv; }
    cx<R> o[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) o[c] = {R(0), R(0)};
    const int tbase = tid - s;
    const int nterms = (kind == FIFTH_K5INV || kind == FIFTH_BINV) ? L5 : 2;
    for (int k = 0; k < nterms; ++k) {
        const R mk = R(ck[k]);
        int su = dag ? s + k : s - k;
        int sd = dag ? s - k : s + k;
        R fu = mk, fd = mk;
        // k may reach L5 only when L5 = 1 (then C^1 = -m_q on the single slice)
        while (su < 0) { su += L5; fu = -mq * fu; }
        while (su >= L5) { su -= L5; fu = -mq * fu; }
        while (sd < 0) { sd += L5; fd = -mq * fd; }
        while (sd >= L5) { sd -= L5; fd = -mq * fd; }
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = o[c] + fu * sh[c * kBlock + tbase + su];
#pragma unroll
        for (int c = 6; c < 12; ++c) o[c] = o[c] + fd * sh[c * kBlock + tbase + sd];
    }
    Field<P>::store(at_rhs(out, stride, rhs), g.Vh, j, o);
}

void launch_fifth(const Geo& g, Prec p, FifthKind kind, int dag, const void* in, void* out, size_t stride,
                  int nrhs, const RhsCoef* coef, const int* active, hipStream_t st) {
    const int nblk = hop_blocks_per_rhs(g);
    dim3 grid(nblk * nrhs);
    switch (p) {
        case P64: hipLaunchKernelGGL(k_fifth<P64>, grid, dim3(kBlock), 0, st, g, int(kind), dag, in, out, stride, nrhs, nblk, coef, active); break;
        case P32: hipLaunchKernelGGL(k_fifth<P32>, grid, dim3(kBlock), 0, st, g, int(kind), dag, in, out, stride, nrhs, nblk, coef, active); break;
        case P16: hipLaunchKernelGGL(k_fifth<P16>, grid, dim3(kBlock), 0, st, g, int(kind), dag, in, out, stride, nrhs, nblk, coef, active); break;
    }
}

}  // namespace mdwf
