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
#include "hop_device.h"

namespace mdwf {

// Waves per SIMD the hop kernels are compiled for: kernels B / B^+ of the
// right-preconditioned FP16 CG operator fit six waves (80 VGPRs, no spills)
// with the table-driven centre term; the others take what their registers
// allow (held to six, kernels A / A^+ would spill).
template <Prec P, int K> constexpr int hop_waves_per_eu() {
    return (P == P16 && (K == HOP_SCHUR_B_RP || K == HOP_SCHUR_B_DAG_RP)) ? 6 : 1;
}

template <Prec P, int K, int LM>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(hop_waves_per_eu<P, K>()))) k_hop(const Geo g, const HopDev a) {
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
    if constexpr (LM == 3) {   // every lane takes part in the matrix products: idle ones read site 0
        if (!valid) xh = y = z = t = i = 0;
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
    // the dense polynomials' tile: all twelve components for the epilogue of
    // kernels A / A^+, six (two passes) for the centre term of B / B^+
    constexpr int kEpiBytes = (TR::epi == 1 || TR::epi == 2) ? 12 * kBlock * int(sizeof(cx<R>))
                            : (TR::cen == 4 || TR::cen == 5) ? 6 * kBlock * int(sizeof(cx<R>)) : 0;
    constexpr int kSmem = kLinkBytes > kEpiBytes ? kLinkBytes : kEpiBytes;
    __shared__ __align__(16) unsigned char smem[kSmem > 0 ? kSmem : 16];
    // Dense centre term sum_k w_k C^k (or its adjoint) of kernels B / B^+:
    // the workgroup's RHS gets a table (dynamic LDS, L5 x L5 entries) of the
    // coefficient each lane applies to each source slice, dtab[s][j] = (P+
    // coefficient, P- coefficient) with the -m_q of the wrap folded in, so
    // the sums run over source slices with no index arithmetic.  C^k moves
    // the P+ spins up (slice s reads s - k) and the P- spins down (s reads
    // s + k); the adjoint swaps the two.  (The same table in the epilogue of
    // kernels A / A^+ cost them occupancy and made them slower.)
    constexpr bool kDense = dense_centre<K>();
    constexpr bool kDenseAdj = TR::cen == 5;
    extern __shared__ __align__(16) unsigned char hop_dyn_lds[];
    cx<R>* const dtab = reinterpret_cast<cx<R>*>(hop_dyn_lds);
    if constexpr (kDense) {
        const double* poly = cf.w;
        for (int e = tid; e < L5 * L5; e += kBlock) {
            const int ss = e / L5, j = e - ss * L5;
            const R dn = (j <= ss) ? R(poly[ss - j]) : -mq * R(poly[ss - j + L5]);   // read j = s - k
            const R up = (j >= ss) ? R(poly[j - ss]) : -mq * R(poly[j - ss + L5]);   // read j = s + k
            dtab[e] = kDenseAdj ? cx<R>{up, dn} : cx<R>{dn, up};
        }
    }
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

    if constexpr (LM == 3) {
        // FP16 on the matrix cores: lane s of the site group holds row s & 3
        // of each link; the neighbour norms are gathered first so that every
        // direction enters one accumulator at a common scale
        const char* rseg[8] = {a.rows_out, a.rows_in, a.rows_out + a.rseg, a.rows_in + a.rseg,
                               a.rows_out + 2 * a.rseg, a.rows_in + 2 * a.rseg, a.rows_out + 3 * a.rseg,
                               a.rows_in + 3 * a.rseg};
        const size_t roff = size_t(s & 3) * lblk;   // this lane's row block
        const char* nsrc = src + align256(3 * sblk);
        float nrm[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) nrm[d] = ldu<float>(nsrc, jn[d] * 4u);
        float S = 1.17549435e-38f;
#pragma unroll
        for (int d = 0; d < 8; ++d) S = fmaxf(S, nrm[d]);
        const float inv = __builtin_amdgcn_rcpf(S);
        f4 acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
        nu4 sp0[3], sp1[3];
        nu4 lr0, lr1;
        auto load = [&](int d, nu4 sp[3], nu4& lr) {
#pragma unroll
            for (int k = 0; k < 3; ++k) sp[k] = ldu<nu4>(src + k * sblk, jn[d] * 16u);
            lr = ldu<nu4>(rseg[d] + roff, lidx[d] * 16u);
        };
        load(0, sp0, lr0);
#define MDWF_MMA(d, spc, lrc, spn, lrn)                                                  \
    if ((d) < 7) load((d) + 1, spn, lrn);                                                \
    {                                                                                    \
        RowA A;                                                                          \
        A.set(lrc);                                                                      \
        mma_term<(d) / 2, (((d) % 2 == 0) != D) ? 1 : -1>(acc, A, spc, nrm[d] * inv);   \
    }
        MDWF_MMA(0, sp0, lr0, sp1, lr1) MDWF_MMA(1, sp1, lr1, sp0, lr0) MDWF_MMA(2, sp0, lr0, sp1, lr1)
        MDWF_MMA(3, sp1, lr1, sp0, lr0) MDWF_MMA(4, sp0, lr0, sp1, lr1) MDWF_MMA(5, sp1, lr1, sp0, lr0)
        MDWF_MMA(6, sp0, lr0, sp1, lr1) MDWF_MMA(7, sp1, lr1, sp0, lr0)
#undef MDWF_MMA
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int c = 0; c < 3; ++c) res[sp * 3 + c] = {S * acc[2 * sp][c], S * acc[2 * sp + 1][c]};
    } else if (valid) {
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
        cx<R> cv[12];
        // lanes past the lattice load site 0 (in bounds; no valid lane reads them)
        Field<P>::load(at_rhs(a.centre, a.stride, rhs), g.Vh, valid ? i * L5 + s : 0, cv);
        if constexpr (LM == 1) __syncthreads();   // every wave is past the link stage
        dense_poly_lanes(cv, cd, reinterpret_cast<cx<R>*>(smem), dtab + s * L5, tid, s, L5, valid);
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
    // matrix cores: FP16, blocks of four slices of one site, no B pre-hop
    if (lm == 3 && (P != P16 || g.L5 % 4 != 0 || HopTraits<K>::preB || !gs.mrow)) lm = 0;
    HopDev a;
    a.out = L.out;
    a.in = L.in;
    a.centre = L.centre;
    const size_t seg = gs.seg_bytes[P];
    a.lseg = seg;
    a.links_out = gs.seg[P] + size_t(L.out_parity) * 4 * seg;
    a.links_in = gs.seg[P] + size_t(1 - L.out_parity) * 4 * seg;
    a.rseg = gs.mrow_bytes;
    a.rows_out = gs.mrow ? gs.mrow + size_t(L.out_parity) * 4 * gs.mrow_bytes : nullptr;
    a.rows_in = gs.mrow ? gs.mrow + size_t(8 + (1 - L.out_parity) * 4) * gs.mrow_bytes : nullptr;
    a.stride = L.stride;
    a.nrhs = L.nrhs;
    a.nblk = hop_blocks_per_rhs(g);
    a.out_parity = L.out_parity;
    a.coef = L.coef;
    a.active = L.active;
    a.partials = L.partials;
    L.nblocks_per_rhs = a.nblk;
    dim3 grid(a.nblk * L.nrhs);
    // the dense polynomial's coefficient table (see k_hop)
    const size_t dyn = dense_centre<K>() ? size_t(g.L5) * g.L5 * sizeof(cx<typename Real<P>::T>) : 0;
    if (lm == 1) {
        hipLaunchKernelGGL((k_hop<P, K, 1>), grid, dim3(kBlock), dyn, st, g, a);
    } else if (lm == 2) {
        if constexpr (P != P64) hipLaunchKernelGGL((k_hop<P, K, 2>), grid, dim3(kBlock), dyn, st, g, a);
    } else if (lm == 3) {
        if constexpr (P == P16 && !HopTraits<K>::preB)
            hipLaunchKernelGGL((k_hop<P, K, 3>), grid, dim3(kBlock), dyn, st, g, a);
    } else {
        hipLaunchKernelGGL((k_hop<P, K, 0>), grid, dim3(kBlock), dyn, st, g, a);
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
    if (launch_hop_plane(g, gs, L, st)) return;
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
