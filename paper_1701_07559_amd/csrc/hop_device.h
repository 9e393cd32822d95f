// Device building blocks of the Wilson hop on every fifth-dimension slice
// (arXiv:1701.07559, Sec. II), shared by the hop kernels: lane exchanges for
// the fifth-dimension couplings, the spin projection / reconstruction of the
// chiral basis, the SU(3) products in FP64 / FP32 and on packed binary16
// pairs, the per-precision raw neighbour registers and link staging.
#pragma once

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
    const char* rows_out;    // FP16 link rows of U at the output parity (matrix-core hop)
    const char* rows_in;     // FP16 link rows of U^+ at the input parity
    size_t rseg;             // bytes of one link-row segment
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

// Hop kinds with a dense fifth-dimension polynomial as their centre term
template <int K> constexpr bool dense_centre() { return HopTraits<K>::cen == 4 || HopTraits<K>::cen == 5; }

// out = sum_j T[s][j] v_j across the L5 lanes of each site (lane s of the
// site's group holds slice s), with ct = T[s] the lane's row of coefficient
// pairs (P+ components use .re, P- components .im).  The values go through
// an LDS tile of six components per thread in two passes, the P+ spins and
// then the P- spins; every thread of the workgroup calls this (barriers).
template <typename R>
__device__ __forceinline__ void dense_poly_lanes(const cx<R> v[12], cx<R> out[12], cx<R>* tile, const cx<R>* ct,
                                                 int tid, int s, int L5, bool valid) {
    const cx<R>* col = tile + (tid - s);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        if (half) __syncthreads();   // every lane is done with the P+ pass
#pragma unroll
        for (int c = 0; c < 6; ++c) tile[c * kBlock + tid] = v[6 * half + c];
        __syncthreads();
        if (valid) {
            {
                const cx<R> f = ct[0];
                const R fh = half ? f.im : f.re;
#pragma unroll
                for (int c = 0; c < 6; ++c) out[6 * half + c] = fh * col[c * kBlock];
            }
            // rolled: the six component reads share one address with
            // immediate offsets
#pragma unroll 1
            for (int j = 1; j < L5; ++j) {
                const cx<R> f = ct[j];
                const R fh = half ? f.im : f.re;
#pragma unroll
                for (int c = 0; c < 6; ++c) out[6 * half + c] = out[6 * half + c] + fh * col[c * kBlock + j];
            }
        }
    }
}
// 16-byte parts gathered by lane exchange (the short tail is loaded by every lane)
template <Prec P> constexpr int link_parts() { return P == P64 ? 9 : P == P32 ? 4 : 2; }

}  // namespace mdwf

namespace mdwf {

// ------------------------------------------ FP16 hop on the matrix cores
// v_mfma_f32_4x4x4_16b_f16 multiplies 16 independent 4x4 blocks: block b is
// lanes 4b..4b+3; lane 4b+i holds row i of the block's A (4 halves, index
// k), lane 4b+j holds column j of its B (4 halves) and receives column j of
// the FP32 result D = A B + C (4 floats, index i).  With L5 a multiple of 4,
// the four lanes of a block are four slices of one 4D site, so they share
// its link: A = one row of the link per lane (stored that way, see
// LinkRowsF16), B = each lane's own colour vector, and D accumulates each
// lane's own result.  Real and imaginary parts are separate products:
//   (U h)_re = U_re h_re - U_im h_im,  (U h)_im = U_re h_im + U_im h_re.
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int nu2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4 mma(h4 a, h4 b, f4 c) { return __builtin_amdgcn_mfma_f32_4x4x4f16(a, b, c, 0, 0, 0); }
__device__ __forceinline__ h4 h4_of(uint32_t lo, uint32_t hi) { return __builtin_bit_cast(h4, nu2{lo, hi}); }

// The link row a lane uses as its A operand: Re and Im of row (lane & 3) of
// U (forward hop) or of U^+ (backward hop), and their negatives.
struct RowA {
    h4 re, im, nre, nim;
    __device__ __forceinline__ void set(nu4 w) {
        re = h4_of(w.x, w.y);
        im = h4_of(w.z, w.w);
        nre = h4_of(w.x ^ 0x80008000u, w.y ^ 0x80008000u);
        nim = h4_of(w.z ^ 0x80008000u, w.w ^ 0x80008000u);
    }
};

// acc (re, im) += c w with w = A h and c = +1, -1, +i or -i (C = 0..3).
template <int C>
__device__ __forceinline__ void mma_cw(f4& ar, f4& ai, const RowA& A, h4 hr, h4 hi) {
    if constexpr (C == 0) {        // +w
        ar = mma(A.re, hr, ar); ar = mma(A.nim, hi, ar);
        ai = mma(A.re, hi, ai); ai = mma(A.im, hr, ai);
    } else if constexpr (C == 1) { // -w
        ar = mma(A.nre, hr, ar); ar = mma(A.im, hi, ar);
        ai = mma(A.nre, hi, ai); ai = mma(A.nim, hr, ai);
    } else if constexpr (C == 2) { // +i w = (-w_im, w_re)
        ar = mma(A.nre, hi, ar); ar = mma(A.nim, hr, ar);
        ai = mma(A.re, hr, ai); ai = mma(A.nim, hi, ai);
    } else {                       // -i w = (w_im, -w_re)
        ar = mma(A.re, hi, ar); ar = mma(A.im, hr, ar);
        ai = mma(A.nre, hr, ai); ai = mma(A.im, hi, ai);
    }
}
// code of the factor -s (s = +1 / -1) and -s i, +s i
template <int S> constexpr int neg_code() { return S > 0 ? 1 : 0; }
template <int S> constexpr int negi_code() { return S > 0 ? 3 : 2; }
template <int S> constexpr int posi_code() { return S > 0 ? 2 : 3; }

// One direction's term on the matrix cores: project the stored binary16
// spinor (u +- X d per spin pair, the chiral basis of project<MU>), scale it
// by the neighbour's norm relative to the site's largest (f <= 1), split the
// two colour vectors into real and imaginary halves and accumulate
// U h into the upper spins and the reconstructed lower spins, as
// reconstruct_add<MU> does.  acc: re / im of spins 0..3, colour in the f4.
template <int MU, int SG>
__device__ __forceinline__ void mma_term(f4 acc[8], const RowA& A, const nu4 s[3], float f) {
    h2 v[12];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        v[4 * k] = as_h2(s[k].x);
        v[4 * k + 1] = as_h2(s[k].y);
        v[4 * k + 2] = as_h2(s[k].z);
        v[4 * k + 3] = as_h2(s[k].w);
    }
    const h2 fs = splat_h2(f);
    h2 h[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const h2 u0 = v[a], u1 = v[3 + a], d0 = v[6 + a], d1 = v[9 + a];
        const h2 id0 = h2{-d0.y, d0.x}, id1 = h2{-d1.y, d1.x};   // i d
        if (MU == 0) { h[a] = SG > 0 ? u0 + id1 : u0 - id1; h[3 + a] = SG > 0 ? u1 + id0 : u1 - id0; }
        else if (MU == 1) { h[a] = SG > 0 ? u0 + d1 : u0 - d1; h[3 + a] = SG > 0 ? u1 - d0 : u1 + d0; }
        else if (MU == 2) { h[a] = SG > 0 ? u0 + id0 : u0 - id0; h[3 + a] = SG > 0 ? u1 - id1 : u1 + id1; }
        else { h[a] = SG > 0 ? u0 - d0 : u0 + d0; h[3 + a] = SG > 0 ? u1 - d1 : u1 + d1; }
        h[a] = h[a] * fs;
        h[3 + a] = h[3 + a] * fs;
    }
    const _Float16 z = _Float16(0.f);
    const h4 hr0 = h4{h[0].x, h[1].x, h[2].x, z}, hi0 = h4{h[0].y, h[1].y, h[2].y, z};
    const h4 hr1 = h4{h[3].x, h[4].x, h[5].x, z}, hi1 = h4{h[3].y, h[4].y, h[5].y, z};
    mma_cw<0>(acc[0], acc[1], A, hr0, hi0);   // upper spins: + w
    mma_cw<0>(acc[2], acc[3], A, hr1, hi1);
    if (MU == 0) {        // spin 2 += -sg i w1, spin 3 += -sg i w0
        mma_cw<negi_code<SG>()>(acc[4], acc[5], A, hr1, hi1);
        mma_cw<negi_code<SG>()>(acc[6], acc[7], A, hr0, hi0);
    } else if (MU == 1) { // spin 2 += -sg w1, spin 3 += sg w0
        mma_cw<neg_code<SG>()>(acc[4], acc[5], A, hr1, hi1);
        mma_cw<neg_code<-SG>()>(acc[6], acc[7], A, hr0, hi0);
    } else if (MU == 2) { // spin 2 += -sg i w0, spin 3 += sg i w1
        mma_cw<negi_code<SG>()>(acc[4], acc[5], A, hr0, hi0);
        mma_cw<posi_code<SG>()>(acc[6], acc[7], A, hr1, hi1);
    } else {              // spin 2 += -sg w0, spin 3 += -sg w1
        mma_cw<neg_code<SG>()>(acc[4], acc[5], A, hr0, hi0);
        mma_cw<neg_code<SG>()>(acc[6], acc[7], A, hr1, hi1);
    }
}

}  // namespace mdwf
