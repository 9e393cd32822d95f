// Plane-staged Wilson hop on every fifth-dimension slice (the Dslash of the
// Moebius operator's D_W, arXiv:1701.07559, Sec. II, and its adjoint).
//
// The lane-per-5D-site hop (dslash.hip) reads each input spinor once per
// neighbour, eight times, through the vector-memory path.  Here a workgroup
// owns a 4 x 4 x 4 block of spatial sites (full coordinates) and a run of bt
// time planes of one right-hand side, and marches along t.  For each input
// plane it copies into LDS, once, every input-parity spinor its hops read
// from that plane -- the 32 sites inside the block and the 48 on its six
// faces, all L5 slices -- together with the 256 links the plane's terms use.
// An input plane t feeds three output planes: its own (the six spatial hops),
// t - 1 (the t+ hop) and t + 1 (the t- hop), so each thread carries the
// accumulators of three planes and finishes one plane per step.
//
// Threads: the L5 slices of one output site in consecutive lanes, as in the
// lane-per-site kernel; 32 output sites per plane.  LDS per workgroup: 80
// spinor slots of L5 sites plus 256 links (see PlaneLds), copied by direct
// global-to-LDS loads that need no registers.
#include "hop_device.h"

namespace mdwf {

constexpr int kPlaneSites = 32;      // output sites of one parity in a 4x4x4 block
constexpr int kPlaneSlots = 80;      // input sites staged per plane (32 inside, 48 on faces)
constexpr int kPlaneLinks = 256;     // 8 link sets x 32 sites
constexpr int kPlaneMaxThreads = 512;

// LDS of one staged plane, filled by direct global-to-LDS loads (each wave
// writes 64 consecutive units): spinor slots [80][blocks][L5] of 16-byte
// units; FP16 norms [80][L5]; links [parts][256] of 16-byte units, then the
// short tail (FP32: re and im arrays of 256 floats, FP16: 256 words); the
// index table [2][80].
template <Prec P> struct PlaneLds;
template <> struct PlaneLds<P32> {
    static constexpr int NB = 6;   // 16-byte blocks per 5D site
    static constexpr int LP = 4;   // 16-byte link parts
    static __host__ __device__ int spinor_bytes(int L5) { return kPlaneSlots * NB * 16 * L5; }
    static __host__ __device__ int link_bytes() { return kPlaneLinks * (LP * 16 + 8); }
};
template <> struct PlaneLds<P16> {
    static constexpr int NB = 3;
    static constexpr int LP = 2;
    static __host__ __device__ int spinor_bytes(int L5) { return kPlaneSlots * (NB * 16 + 4) * L5; }
    static __host__ __device__ int link_bytes() { return kPlaneLinks * (LP * 16 + 4); }
};
template <Prec P> inline size_t plane_lds_bytes(int L5) {
    return size_t(PlaneLds<P>::spinor_bytes(L5)) + PlaneLds<P>::link_bytes() + 2 * kPlaneSlots * sizeof(int);
}

struct PlaneDev {
    int bt;            // time planes per workgroup
    int nbx, nby, nbz, nbt;
    int nthreads;
    FastDiv fUnits;    // 16-byte spinor units per slot: NB * L5
    FastDiv fL5;
};

// Position (lx, ly, lz) inside the block of staged slot `slot` of a plane
// whose input-parity sites satisfy (lx + ly + lz + t) = ip (mod 2), cls =
// (ip + t) mod 2: slots 0..31 inside the block (x fastest, parity-
// compressed), then eight per face in the order x-, x+, y-, y+, z-, z+.
__device__ __forceinline__ void slot_position(int slot, int cls, int& lx, int& ly, int& lz) {
    if (slot < kPlaneSites) {
        ly = (slot >> 1) & 3;
        lz = slot >> 3;
        lx = 2 * (slot & 1) + ((cls + ly + lz) & 1);
        return;
    }
    const int f = (slot - kPlaneSites) & 7, face = (slot - kPlaneSites) >> 3;
    const int v = (face & 1) ? 4 : -1;   // the fixed coordinate
    const int b = f >> 1;
    const int a = 2 * (f & 1) + ((cls + v + b) & 1);
    if (face < 2) { lx = v; ly = a; lz = b; }
    else if (face < 4) { ly = v; lx = a; lz = b; }
    else { lz = v; lx = a; ly = b; }
}

// Slot of a neighbour inside the block (the face slots are computed where
// the hop leaves the block).
__device__ __forceinline__ int inner_slot(int lx, int ly, int lz) { return (lx >> 1) + 2 * (ly + 4 * lz); }

// Direct global-to-LDS copy: lane l of the wave writes `bytes` bytes at
// lds_base + l * bytes (lds_base wave-uniform); inactive lanes write nothing.
template <int BYTES> __device__ __forceinline__ void copy_to_lds(const void* gsrc, void* lds_base) {
    if constexpr (BYTES == 16) __builtin_amdgcn_global_load_lds(gsrc, lds_base, 16, 0, 0);
    else __builtin_amdgcn_global_load_lds(gsrc, lds_base, 4, 0, 0);
}

template <Prec P> struct PlaneIO;

template <> struct PlaneIO<P32> {
    static __device__ __forceinline__ void spinor(const unsigned char* slot, int L5, int s, cx<float> v[12]) {
        const nf4* p = reinterpret_cast<const nf4*>(slot) + s;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const nf4 w = p[k * L5];
            v[2 * k] = {w.x, w.y};
            v[2 * k + 1] = {w.z, w.w};
        }
    }
    static __device__ __forceinline__ void link(const unsigned char* lds, int id, cx<float> U[9]) {
        const nf4* p = reinterpret_cast<const nf4*>(lds) + id;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const nf4 w = p[k * kPlaneLinks];
            U[2 * k] = {w.x, w.y};
            U[2 * k + 1] = {w.z, w.w};
        }
        const float* t = reinterpret_cast<const float*>(lds + 4 * 16 * kPlaneLinks);
        U[8] = {t[id], t[kPlaneLinks + id]};
    }
    // the links of 64 consecutive ids (this lane's link in segment seg at
    // index i; active lanes only)
    static __device__ __forceinline__ void stage_links(const char* seg, size_t lblk, uint32_t i, unsigned char* lds,
                                                       int chunk) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            copy_to_lds<16>(seg + k * lblk + size_t(i) * 16, lds + k * 16 * kPlaneLinks + chunk * 64 * 16);
        unsigned char* t = lds + 4 * 16 * kPlaneLinks;
        const char* tail = seg + 4 * lblk + size_t(i) * 8;
        copy_to_lds<4>(tail, t + chunk * 64 * 4);
        copy_to_lds<4>(tail + 4, t + 4 * kPlaneLinks + chunk * 64 * 4);
    }
};

template <> struct PlaneIO<P16> {
    // the stored binary16 pairs (the site's norm is read separately)
    static __device__ __forceinline__ void spinor_h(const unsigned char* slot, int L5, int s, h2 v[12]) {
        const nu4* p = reinterpret_cast<const nu4*>(slot) + s;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const nu4 w = p[k * L5];
            v[4 * k] = as_h2(w.x);
            v[4 * k + 1] = as_h2(w.y);
            v[4 * k + 2] = as_h2(w.z);
            v[4 * k + 3] = as_h2(w.w);
        }
    }
    static __device__ __forceinline__ void link_h(const unsigned char* lds, int id, h2 U[9]) {
        const nu4* p = reinterpret_cast<const nu4*>(lds) + id;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const nu4 w = p[k * kPlaneLinks];
            U[4 * k] = as_h2(w.x);
            U[4 * k + 1] = as_h2(w.y);
            U[4 * k + 2] = as_h2(w.z);
            U[4 * k + 3] = as_h2(w.w);
        }
        U[8] = as_h2(reinterpret_cast<const uint32_t*>(lds + 2 * 16 * kPlaneLinks)[id]);
    }
    static __device__ __forceinline__ void stage_links(const char* seg, size_t lblk, uint32_t i, unsigned char* lds,
                                                       int chunk) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
            copy_to_lds<16>(seg + k * lblk + size_t(i) * 16, lds + k * 16 * kPlaneLinks + chunk * 64 * 16);
        copy_to_lds<4>(seg + 2 * lblk + size_t(i) * 4, lds + 2 * 16 * kPlaneLinks + chunk * 64 * 4);
    }
};

// One hop term of direction (MU, DIR) from a staged spinor slot and link;
// nrm: the FP16 site norm (unused otherwise).
template <Prec P, bool DAG, int MU, int DIR>
__device__ __forceinline__ void plane_term(cx<typename Real<P>::T> acc[12], const unsigned char* slot, float nrm,
                                           int L5, int s, const unsigned char* lk, int lid) {
    if constexpr (P == P16) {
        h2 psi[12], U[9];
        PlaneIO<P16>::spinor_h(slot, L5, s, psi);
        PlaneIO<P16>::link_h(lk, lid, U);
        constexpr int sg = ((DIR > 0) != DAG) ? 1 : -1;
        h2 z1[6], z2[6];
        project_h<MU, sg, (DIR > 0)>(psi, z1, z2);
        cx<float> w[6];
        su3_mul_h<(DIR > 0)>(U, z1, z2, w);
#pragma unroll
        for (int c = 0; c < 6; ++c) w[c] = nrm * w[c];
        reconstruct_add<MU>(float(sg), w, acc);
    } else {
        using R = typename Real<P>::T;
        cx<R> psi[12], U[9];
        PlaneIO<P>::spinor(slot, L5, s, psi);
        PlaneIO<P>::link(lk, lid, U);
        constexpr R sg = ((DIR > 0) != DAG) ? R(1) : R(-1);
        cx<R> h[6], w[6];
        project<MU>(sg, psi, h);
        su3_mul<(DIR > 0)>(U, h, w);
        reconstruct_add<MU>(sg, w, acc);
    }
}

// Link sets of a staged plane t (output sites k of plane t unless noted):
// 0/1 x forward (at k) / backward (at its x- neighbour), 2/3 y, 4/5 z,
// 6 t forward at the output site of plane t-1 above slot k, 7 t backward at
// the input site of slot k (plane t), used by plane t+1.
template <Prec P, int K>
__global__ void __launch_bounds__(kPlaneMaxThreads) k_hop_plane(const Geo g, const HopDev a, const PlaneDev pd) {
    using R = typename Real<P>::T;
    using IO = PlaneIO<P>;
    constexpr bool DAG = HopTraits<K>::dag;
    extern __shared__ __align__(16) unsigned char plane_lds[];
    const int L5 = g.L5;
    const int units = int(pd.fUnits.d);          // 16-byte spinor units per slot
    const int slot_bytes = units * 16;
    unsigned char* sp = plane_lds;
    const float* snorm = reinterpret_cast<const float*>(sp + size_t(kPlaneSlots) * slot_bytes);   // FP16
    unsigned char* lk = plane_lds + PlaneLds<P>::spinor_bytes(L5);
    int* tab = reinterpret_cast<int*>(lk + PlaneLds<P>::link_bytes());

    // workgroup -> right-hand side (fastest, they share links), block, t-run
    const int lb = g.xcd_remap[P] ? xcd_logical_block(blockIdx.x, gridDim.x) : int(blockIdx.x);
    const int rhs = lb % a.nrhs;
    int rest = lb / a.nrhs;
    const int bx = rest % pd.nbx;
    rest /= pd.nbx;
    const int by = rest % pd.nby;
    rest /= pd.nby;
    const int bz = rest % pd.nbz;
    const int btr = rest / pd.nbz;
    if (a.active && !a.active[rhs]) return;   // uniform over the workgroup
    const int x0 = 4 * bx, y0 = 4 * by, z0 = 4 * bz, t0 = btr * pd.bt;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int nwaves = pd.nthreads >> 6;
    const int spw = 64 / L5;
    const int sw = lane / L5;
    const int s = lane - sw * L5;
    const int k = wave * spw + sw;   // output site of the plane
    const bool valid = sw < spw && k < kPlaneSites;
    const int kk = valid ? k : 0;
    const int ky = (kk >> 1) & 3, kz = kk >> 3;
    const int p = a.out_parity, ip = 1 - p;

    const char* src = static_cast<const char*>(at_rhs(a.in, a.stride, rhs));
    char* dst = static_cast<char*>(at_rhs(a.out, a.stride, rhs));
    const size_t sblk = size_t(g.Vh) * 16;
    const size_t lblk = size_t(g.Vh4) * 16;
    const uint32_t plane_sites = uint32_t(g.Xh * g.Y * g.Z);

    auto gidx = [&](int lx, int ly, int lz, int t) -> uint32_t {
        int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        gx = gx < 0 ? gx + g.X : (gx >= g.X ? gx - g.X : gx);
        gy = gy < 0 ? gy + g.Y : (gy >= g.Y ? gy - g.Y : gy);
        gz = gz < 0 ? gz + g.Z : (gz >= g.Z ? gz - g.Z : gz);
        return uint32_t((gx >> 1) + g.Xh * (gy + g.Y * (gz + g.Z * t)));
    };

    // spatial part of the parity-compressed index of every slot, for both
    // classes of input sites (planes alternate between them)
    for (int e = tid; e < 2 * kPlaneSlots; e += pd.nthreads) {
        int lx, ly, lz;
        slot_position(e % kPlaneSlots, e / kPlaneSlots, lx, ly, lz);
        tab[e] = int(gidx(lx, ly, lz, 0));
    }

    cx<R> acc_prev[12], acc_cur[12], acc_next[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc_prev[c] = acc_cur[c] = acc_next[c] = {R(-0.0), R(-0.0)};

    for (int tp = t0 - 1; tp <= t0 + pd.bt; ++tp) {
        const int t = tp < 0 ? tp + g.T : (tp >= g.T ? tp - g.T : tp);
        const int cin = (ip + t) & 1;        // class of the input sites of plane t
        const bool edge = tp < t0 || tp >= t0 + pd.bt;   // only the t hops use this plane
        const int nslots = edge ? kPlaneSites : kPlaneSlots;
        __syncthreads();   // every thread is done with the previous plane (and the table is written)
        // ---- stage the plane's input spinors: unit u = (slot, block, slice),
        // 64 consecutive units per wave and copy
        const int* ctab = tab + cin * kPlaneSlots;
        const uint32_t tofs = plane_sites * uint32_t(t);
        const int nunits = nslots * units;
        for (int c = wave; c * 64 < nunits; c += nwaves) {
            const int u = c * 64 + lane;
            if (u < nunits) {
                const int slot = int(pd.fUnits.div(uint32_t(u)));
                const int r = u - slot * units;
                const int blk = int(pd.fL5.div(uint32_t(r)));
                const uint32_t j = (uint32_t(ctab[slot]) + tofs) * uint32_t(L5) + uint32_t(r - blk * L5);
                copy_to_lds<16>(src + blk * sblk + size_t(j) * 16, sp + size_t(c) * 64 * 16);
            }
        }
        if constexpr (P == P16) {   // norms [slot][slice]
            const char* nsrc = src + align256(3 * sblk);
            unsigned char* nb = sp + size_t(kPlaneSlots) * slot_bytes;
            const int nn = nslots * L5;
            for (int c = wave; c * 64 < nn; c += nwaves) {
                const int u = c * 64 + lane;
                if (u < nn) {
                    const int slot = int(pd.fL5.div(uint32_t(u)));
                    const uint32_t j = (uint32_t(ctab[slot]) + tofs) * uint32_t(L5) + uint32_t(u - slot * L5);
                    copy_to_lds<4>(nsrc + size_t(j) * 4, nb + size_t(c) * 64 * 4);
                }
            }
        }
        // ---- stage the links of the plane's terms, 64 ids per wave and copy
        for (int c = edge ? 3 : wave; c < 4; c += nwaves) {
            if (edge && wave != 0) break;   // edge planes: one wave copies sets 6 and 7
            const int id = c * 64 + lane;
            const int set = id >> 5, w = id & 31;
            const int wy = (w >> 1) & 3, wz = w >> 3;
            const int mu = set >> 1;
            const bool fwd = (set & 1) == 0;
            int lx, ly = wy, lz = wz, tl = t;
            if (set < 6) {
                lx = 2 * (w & 1) + ((p + t + wy + wz) & 1);   // output site w of plane t
                if (!fwd) {
                    if (mu == 0) lx -= 1;
                    else if (mu == 1) ly -= 1;
                    else lz -= 1;
                }
            } else {
                lx = 2 * (w & 1) + ((cin + wy + wz) & 1);      // input slot w of plane t
                if (fwd) tl = t == 0 ? g.T - 1 : t - 1;        // output site of plane t-1
            }
            const char* seg = (fwd ? a.links_out : a.links_in) + size_t(mu) * a.lseg;
            IO::stage_links(seg, lblk, gidx(lx, ly, lz, tl), lk, c);
        }
        __builtin_amdgcn_s_waitcnt(0);   // this wave's copies have landed
        __syncthreads();
        if (!valid) continue;
        auto norm = [&](int slot) -> float {
            if constexpr (P == P16) return snorm[slot * L5 + s];
            else return 1.f;
        };
        // ---- plane t-1 gets its t+ term and is finished
        if (tp - 1 >= t0) {
            plane_term<P, DAG, 3, +1>(acc_prev, sp + size_t(kk) * slot_bytes, norm(kk), L5, s, lk, 6 * 32 + kk);
            const int lx = 2 * (kk & 1) + ((p + tp - 1 + ky + kz) & 1);
            const uint32_t j = gidx(lx, ky, kz, tp - 1) * uint32_t(L5) + uint32_t(s);
            if (g.nt_store[P]) Field<P>::template store<true>(dst, g.Vh, int(j), acc_prev);
            else Field<P>::store(dst, g.Vh, int(j), acc_prev);
        }
        // ---- plane t: the six spatial terms
        if (!edge) {
            const int lx = 2 * (kk & 1) + ((p + t + ky + kz) & 1);
            const int sxp = lx < 3 ? inner_slot(lx + 1, ky, kz) : 40 + 2 * kz + (ky >> 1);
            const int sxm = lx > 0 ? inner_slot(lx - 1, ky, kz) : 32 + 2 * kz + (ky >> 1);
            const int syp = ky < 3 ? inner_slot(lx, ky + 1, kz) : 56 + 2 * kz + (lx >> 1);
            const int sym = ky > 0 ? inner_slot(lx, ky - 1, kz) : 48 + 2 * kz + (lx >> 1);
            const int szp = kz < 3 ? inner_slot(lx, ky, kz + 1) : 72 + 2 * ky + (lx >> 1);
            const int szm = kz > 0 ? inner_slot(lx, ky, kz - 1) : 64 + 2 * ky + (lx >> 1);
            plane_term<P, DAG, 0, +1>(acc_cur, sp + size_t(sxp) * slot_bytes, norm(sxp), L5, s, lk, 0 * 32 + kk);
            plane_term<P, DAG, 0, -1>(acc_cur, sp + size_t(sxm) * slot_bytes, norm(sxm), L5, s, lk, 1 * 32 + kk);
            plane_term<P, DAG, 1, +1>(acc_cur, sp + size_t(syp) * slot_bytes, norm(syp), L5, s, lk, 2 * 32 + kk);
            plane_term<P, DAG, 1, -1>(acc_cur, sp + size_t(sym) * slot_bytes, norm(sym), L5, s, lk, 3 * 32 + kk);
            plane_term<P, DAG, 2, +1>(acc_cur, sp + size_t(szp) * slot_bytes, norm(szp), L5, s, lk, 4 * 32 + kk);
            plane_term<P, DAG, 2, -1>(acc_cur, sp + size_t(szm) * slot_bytes, norm(szm), L5, s, lk, 5 * 32 + kk);
        }
        // ---- plane t+1 starts with its t- term
        if (tp + 1 < t0 + pd.bt)
            plane_term<P, DAG, 3, -1>(acc_next, sp + size_t(kk) * slot_bytes, norm(kk), L5, s, lk, 7 * 32 + kk);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            acc_prev[c] = acc_cur[c];
            acc_cur[c] = acc_next[c];
            acc_next[c] = {R(-0.0), R(-0.0)};
        }
    }
}

// ------------------------------------------------ register-buffered variant
// FP32 with L5 = 8: the same 4x4x4 blocks and plane march, but the copies of
// the next plane go to registers while the current plane is computed from
// LDS, and are written to LDS between two barriers at the end of the step.
// So their latency hides behind a whole plane of arithmetic instead of
// stalling the workgroup, in the same 80.5 KB of LDS (two workgroups per CU).
// Each thread owns fixed staging elements: the 16-byte spinor units
// c * 256 + tid (c < 15; a unit is (slot, block, slice), slice fastest) and
// the link id tid (four 16-byte parts and the 8-byte tail).  The step loop
// is unrolled by three so that the three planes' accumulators change roles
// without copies.
constexpr int kRbThreads = 256;                                   // 32 sites x 8 slices
constexpr int kRbUnits = kPlaneSlots * 6 * 8 / kRbThreads;        // 15 spinor units per thread
constexpr int kRbSlotBytes = 6 * 8 * 16;                          // one staged site, all slices
constexpr int kRbLinkOff = kPlaneSlots * kRbSlotBytes;            // 61440
constexpr int kRbTailOff = kRbLinkOff + 4 * kPlaneLinks * 16;     // link parts [4][256]
constexpr int kRbTabOff = kRbTailOff + kPlaneLinks * 8;           // link tails [256] float2
constexpr int kRbLdsBytes = kRbTabOff + 2 * kPlaneSlots * 4;      // slot table [2][80]
static_assert(kRbUnits * kRbThreads == kPlaneSlots * 6 * 8, "whole units per thread");

// The staged spinor of a slot (layout [block][slice] of 16-byte units) at
// slice s, and one hop term of it with a staged link id.
// Block k of an odd slot sits at position k ^ 1, so that the 128-byte rows
// read together by neighbouring site groups fall in different LDS bank
// halves.
__device__ __forceinline__ void rb_spinor(const unsigned char* sp, int slot, int s, cx<float> psi[12]) {
    const int b = (slot & 1) * 128;
    const unsigned char* base = sp + slot * kRbSlotBytes + s * 16;
    const nf4* qe = reinterpret_cast<const nf4*>(base + b);   // even k
    const nf4* qo = reinterpret_cast<const nf4*>(base - b);   // odd k
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const nf4 w = (k & 1) ? qo[k * 8] : qe[k * 8];
        psi[2 * k] = {w.x, w.y};
        psi[2 * k + 1] = {w.z, w.w};
    }
}
template <bool DAG, int MU, int DIR>
__device__ __forceinline__ void rb_term(cx<float> acc[12], const cx<float> psi[12], const unsigned char* lk,
                                        int lid) {
    cx<float> U[9];
    const nf4* l = reinterpret_cast<const nf4*>(lk) + lid;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const nf4 w = l[k * kPlaneLinks];
        U[2 * k] = {w.x, w.y};
        U[2 * k + 1] = {w.z, w.w};
    }
    const nf2 tl = reinterpret_cast<const nf2*>(lk + 4 * kPlaneLinks * 16)[lid];
    U[8] = {tl.x, tl.y};
    constexpr float sg = ((DIR > 0) != DAG) ? 1.f : -1.f;
    cx<float> h[6], w[6];
    project<MU>(sg, psi, h);
    su3_mul<(DIR > 0)>(U, h, w);
    reconstruct_add<MU>(sg, w, acc);
}

template <int K>
__global__ void __launch_bounds__(kRbThreads, 2) k_hop_plane_rb(const Geo g, const HopDev a, const PlaneDev pd) {
    constexpr bool DAG = HopTraits<K>::dag;
    extern __shared__ __align__(16) unsigned char plane_lds[];
    unsigned char* const sp = plane_lds;
    unsigned char* const lk = plane_lds + kRbLinkOff;
    int* const tab = reinterpret_cast<int*>(plane_lds + kRbTabOff);

    // workgroup -> right-hand side (fastest), block, t-run
    const int lb = g.xcd_remap[P32] ? xcd_logical_block(blockIdx.x, gridDim.x) : int(blockIdx.x);
    const int rhs = lb % a.nrhs;
    int rest = lb / a.nrhs;
    const int bx = rest % pd.nbx;
    rest /= pd.nbx;
    const int by = rest % pd.nby;
    rest /= pd.nby;
    const int bz = rest % pd.nbz;
    const int btr = rest / pd.nbz;
    if (a.active && !a.active[rhs]) return;   // uniform over the workgroup
    const int x0 = 4 * bx, y0 = 4 * by, z0 = 4 * bz;
    const int t0 = btr * pd.bt, t1 = t0 + pd.bt;

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int s = lane & 7;
    const int kk = (wave << 3) + (lane >> 3);   // output site of the plane
    const int kx = kk & 1, ky = (kk >> 1) & 3, kz = kk >> 3;
    const int p = a.out_parity, ip = 1 - p;
    const char* src = static_cast<const char*>(at_rhs(a.in, a.stride, rhs));
    char* dst = static_cast<char*>(at_rhs(a.out, a.stride, rhs));
    const size_t sblk = size_t(g.Vh) * 16;
    const size_t lblk = size_t(g.Vh4) * 16;
    const uint32_t plane_sites = uint32_t(g.Xh * g.Y * g.Z);
    auto wrapT = [&](int t) { return t < 0 ? t + g.T : (t >= g.T ? t - g.T : t); };
    auto gidx = [&](int lx, int ly, int lz, int t) -> uint32_t {
        int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        gx = gx < 0 ? gx + g.X : (gx >= g.X ? gx - g.X : gx);
        gy = gy < 0 ? gy + g.Y : (gy >= g.Y ? gy - g.Y : gy);
        gz = gz < 0 ? gz + g.Z : (gz >= g.Z ? gz - g.Z : gz);
        return uint32_t((gx >> 1) + g.Xh * (gy + g.Y * (gz + g.Z * t)));
    };

    // spatial part of the parity-compressed index of every slot, both classes
    for (int e = tid; e < 2 * kPlaneSlots; e += kRbThreads) {
        int lx, ly, lz;
        slot_position(e % kPlaneSlots, e / kPlaneSlots, lx, ly, lz);
        tab[e] = int(gidx(lx, ly, lz, 0));
    }

    // this thread's spinor units: unit c*256 + tid is slot uslot[c % 3] +
    // 16 (c / 3), block and slice from ubase[c % 3] and usl[c % 3] (768
    // units = 16 slots, so the parity of the slot depends on c % 3 only)
    int uslot[3], usl[3], uswz[3];
    const char* ubase[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int u = c * kRbThreads + tid;
        uslot[c] = u / 48;
        const int r = u - 48 * uslot[c];
        ubase[c] = src + size_t(r >> 3) * sblk;
        usl[c] = r & 7;
        // LDS position of the unit: block (r >> 3) ^ 1 in odd slots (see rb_spinor)
        uswz[c] = (uslot[c] & 1) ? (((r >> 3) & 1) ? -8 : 8) : 0;
    }
    // this thread's link id: set lset (0/1 x fwd/bwd, 2/3 y, 4/5 z, 6 t fwd at
    // the output site of plane t-1, 7 t bwd at the input site of plane t),
    // site lw of the set
    const int lset = tid >> 5, lw = tid & 31;
    const int lwy = (lw >> 1) & 3, lwz = lw >> 3, lmu = lset >> 1;
    const bool lfwd = (lset & 1) == 0;
    const char* lseg = (lfwd ? a.links_out : a.links_in) + size_t(lmu) * a.lseg;

    nf4 pre[kRbUnits], lpre[4];
    nf2 ltail;
    // kind of a staged plane: 0 the plane before the run (t- hops of its
    // first plane), 1 inside the run, 2 the plane after it (t+ hops of its
    // last plane); the edge planes need the 32 inner slots and one link set
    auto prefetch = [&](int t, int kind) {
        const int cls = (ip + t) & 1;
        const uint32_t tofs = plane_sites * uint32_t(t);
        const int* ctab = tab + cls * kPlaneSlots;
#pragma unroll
        for (int c = 0; c < kRbUnits; ++c) {
            if (kind != 1 && c >= 6) break;   // units below 1536: the 32 inner slots
            const int slot = uslot[c % 3] + 16 * (c / 3);
            const uint32_t j = (uint32_t(ctab[slot]) + tofs) * 8u + uint32_t(usl[c % 3]);
            pre[c] = ldu<nf4>(ubase[c % 3], j * 16u);
        }
        if (kind == 1 || wave == 3) {   // wave 3 holds sets 6 and 7
            int lx, ly = lwy, lz = lwz, tl = t;
            if (lset < 6) {
                lx = 2 * (lw & 1) + ((p + t + lwy + lwz) & 1);   // output site lw of plane t
                if (!lfwd) {
                    if (lmu == 0) lx -= 1;
                    else if (lmu == 1) ly -= 1;
                    else lz -= 1;
                }
            } else {
                lx = 2 * (lw & 1) + ((cls + lwy + lwz) & 1);      // input slot lw of plane t
                if (lfwd) tl = t == 0 ? g.T - 1 : t - 1;
            }
            const uint32_t li = gidx(lx, ly, lz, tl);
            // each link is read once per hop: streamed past the caches when
            // the launch shape asks for non-temporal accesses
            if (g.nt_store[P32]) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    lpre[e] = __builtin_nontemporal_load(reinterpret_cast<const nf4*>(lseg + e * lblk + size_t(li) * 16));
                ltail = __builtin_nontemporal_load(reinterpret_cast<const nf2*>(lseg + 4 * lblk + size_t(li) * 8));
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) lpre[e] = ldu<nf4>(lseg + e * lblk, li * 16u);
                ltail = ldu<nf2>(lseg + 4 * lblk, li * 8u);
            }
        }
    };
    auto commit = [&](int kind) {
#pragma unroll
        for (int c = 0; c < kRbUnits; ++c) {
            if (kind != 1 && c >= 6) break;
            reinterpret_cast<nf4*>(sp)[c * kRbThreads + tid + uswz[c % 3]] = pre[c];
        }
        if (kind == 1 || wave == 3) {
#pragma unroll
            for (int e = 0; e < 4; ++e) reinterpret_cast<nf4*>(lk)[e * kPlaneLinks + tid] = lpre[e];
            reinterpret_cast<nf2*>(lk + 4 * kPlaneLinks * 16)[tid] = ltail;
        }
    };
    auto kind_of = [&](int tp) { return tp < t0 ? 0 : (tp >= t1 ? 2 : 1); };
    auto store = [&](const cx<float> acc[12], int tpl) {
        const int lx = 2 * kx + ((p + tpl + ky + kz) & 1);
        const int j = int(gidx(lx, ky, kz, tpl)) * 8 + s;
        if (g.nt_store[P32]) Field<P32>::store<true>(dst, g.Vh, j, acc);
        else Field<P32>::store(dst, g.Vh, j, acc);
    };

    __syncthreads();   // slot table written
    prefetch(wrapT(t0 - 1), 0);
    commit(0);
    __syncthreads();

    cx<float> A[12], B[12], C[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) A[c] = B[c] = C[c] = {-0.f, -0.f};

    // One step: plane tp is in LDS and the copies of plane tp + 1 are issued
    // first.  The inner slot at the thread's site gives the t+ term of plane
    // tp - 1 (PR, then stored and cleared) and the t- term of plane tp + 1
    // (NX); CU, plane tp, takes the six spatial terms.
#define MDWF_RB_STEP(i, PR, CU, NX)                                                                     \
    {                                                                                                   \
        const int tp = t0 - 1 + (i);                                                                    \
        const int t = wrapT(tp);                                                                        \
        const int kind = kind_of(tp);                                                                   \
        if (tp + 1 <= t1) prefetch(wrapT(tp + 1), kind_of(tp + 1));                                     \
        if (tp - 1 >= t0 || tp + 1 < t1) {                                                              \
            cx<float> psi[12];                                                                          \
            rb_spinor(sp, kk, s, psi);                                                                  \
            if (tp - 1 >= t0) {                                                                         \
                rb_term<DAG, 3, +1>(PR, psi, lk, 6 * 32 + kk);                                          \
                store(PR, wrapT(tp - 1));                                                               \
            }                                                                                           \
            if (tp + 1 < t1) rb_term<DAG, 3, -1>(NX, psi, lk, 7 * 32 + kk);                             \
        }                                                                                               \
        _Pragma("unroll") for (int c = 0; c < 12; ++c) PR[c] = {-0.f, -0.f};                            \
        if (kind == 1) {                                                                                \
            const int lx = 2 * kx + ((p + t + ky + kz) & 1);                                            \
            const int sxp = lx < 3 ? inner_slot(lx + 1, ky, kz) : 40 + 2 * kz + (ky >> 1);              \
            const int sxm = lx > 0 ? inner_slot(lx - 1, ky, kz) : 32 + 2 * kz + (ky >> 1);              \
            const int syp = ky < 3 ? inner_slot(lx, ky + 1, kz) : 56 + 2 * kz + (lx >> 1);              \
            const int sym = ky > 0 ? inner_slot(lx, ky - 1, kz) : 48 + 2 * kz + (lx >> 1);              \
            const int szp = kz < 3 ? inner_slot(lx, ky, kz + 1) : 72 + 2 * ky + (lx >> 1);              \
            const int szm = kz > 0 ? inner_slot(lx, ky, kz - 1) : 64 + 2 * ky + (lx >> 1);              \
            cx<float> psi[12];                                                                          \
            rb_spinor(sp, sxp, s, psi); rb_term<DAG, 0, +1>(CU, psi, lk, 0 * 32 + kk);                  \
            rb_spinor(sp, sxm, s, psi); rb_term<DAG, 0, -1>(CU, psi, lk, 1 * 32 + kk);                  \
            rb_spinor(sp, syp, s, psi); rb_term<DAG, 1, +1>(CU, psi, lk, 2 * 32 + kk);                  \
            rb_spinor(sp, sym, s, psi); rb_term<DAG, 1, -1>(CU, psi, lk, 3 * 32 + kk);                  \
            rb_spinor(sp, szp, s, psi); rb_term<DAG, 2, +1>(CU, psi, lk, 4 * 32 + kk);                  \
            rb_spinor(sp, szm, s, psi); rb_term<DAG, 2, -1>(CU, psi, lk, 5 * 32 + kk);                  \
        }                                                                                               \
        __syncthreads();   /* every wave is done with plane tp */                                       \
        if (tp + 1 <= t1) commit(kind_of(tp + 1));                                                      \
        __syncthreads();                                                                                \
    }
    const int nsteps = pd.bt + 2;
    for (int i = 0; i < nsteps; i += 3) {
        MDWF_RB_STEP(i, A, B, C)
        if (i + 1 >= nsteps) break;
        MDWF_RB_STEP(i + 1, B, C, A)
        if (i + 2 >= nsteps) break;
        MDWF_RB_STEP(i + 2, C, A, B)
    }
#undef MDWF_RB_STEP
}

// Dynamic LDS the plane kernels may take: a CU's whole LDS.
size_t plane_lds_limit() {
    static size_t limit = [] {
        int dev = 0, v = 0;
        size_t lim = 64 * 1024;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            lim = size_t(v);
        (void)hipGetLastError();
        return lim;
    }();
    return limit;
}

template <Prec P, int K>
static void launch_plane_k(const dim3& grid, int nthreads, size_t lds, hipStream_t st, const Geo& g,
                           const HopDev& a, const PlaneDev& pd) {
    static const bool attr = [] {   // allow this instantiation the whole LDS (once per process)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hop_plane<P, K>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(plane_lds_limit()));
        (void)hipGetLastError();
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL((k_hop_plane<P, K>), grid, dim3(nthreads), lds, st, g, a, pd);
}

template <int K>
static void launch_plane_rb(const dim3& grid, hipStream_t st, const Geo& g, const HopDev& a, const PlaneDev& pd) {
    static const bool attr = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hop_plane_rb<K>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kRbLdsBytes);
        (void)hipGetLastError();
        return true;
    }();
    (void)attr;
    hipLaunchKernelGGL((k_hop_plane_rb<K>), grid, dim3(kRbThreads), kRbLdsBytes, st, g, a, pd);
}

// The plane-staged kernel applies when the launch shape asks for it, the
// operator is the bare hop, the spatial extents are multiples of 4, T of bt,
// a workgroup has 128 to 512 threads (L5 from 3 to 16) and the plane fits in
// LDS; it returns false otherwise.
template <Prec P>
static bool launch_plane_p(const Geo& g, const GaugeSet& gs, HopLaunch& L, hipStream_t st) {
    const int bt = g.plane_bt[P];
    if constexpr (P == P64) return false;
    else {
        if (bt <= 0 || (L.kind != HOP_BARE && L.kind != HOP_BARE_DAG)) return false;
        if (g.X % 4 || g.Y % 4 || g.Z % 4 || g.T % bt || g.L5 > 16) return false;
        const int spw = 64 / g.L5;
        const int nthreads = 64 * ((kPlaneSites + spw - 1) / spw);
        const size_t lds = plane_lds_bytes<P>(g.L5);
        if (nthreads < 128 || nthreads > kPlaneMaxThreads || lds > plane_lds_limit()) return false;
        HopDev a{};
        a.out = L.out;
        a.in = L.in;
        a.centre = L.centre;
        const size_t seg = gs.seg_bytes[P];
        a.lseg = seg;
        a.links_out = gs.seg[P] + size_t(L.out_parity) * 4 * seg;
        a.links_in = gs.seg[P] + size_t(1 - L.out_parity) * 4 * seg;
        a.stride = L.stride;
        a.nrhs = L.nrhs;
        a.out_parity = L.out_parity;
        a.coef = L.coef;
        a.active = L.active;
        a.partials = nullptr;
        PlaneDev pd{};
        pd.bt = bt;
        pd.nbx = g.X / 4; pd.nby = g.Y / 4; pd.nbz = g.Z / 4; pd.nbt = g.T / bt;
        pd.nthreads = nthreads;
        pd.fUnits = FastDiv(uint32_t(PlaneLds<P>::NB * g.L5));
        pd.fL5 = FastDiv(uint32_t(g.L5));
        a.nblk = pd.nbx * pd.nby * pd.nbz * pd.nbt;
        L.nblocks_per_rhs = a.nblk;
        const dim3 grid(a.nblk * L.nrhs);
        if (P == P32 && g.L5 == 8 && size_t(kRbLdsBytes) <= plane_lds_limit()) {   // register-buffered variant
            if (L.kind == HOP_BARE) launch_plane_rb<HOP_BARE>(grid, st, g, a, pd);
            else launch_plane_rb<HOP_BARE_DAG>(grid, st, g, a, pd);
            return true;
        }
        if (L.kind == HOP_BARE) launch_plane_k<P, HOP_BARE>(grid, nthreads, lds, st, g, a, pd);
        else launch_plane_k<P, HOP_BARE_DAG>(grid, nthreads, lds, st, g, a, pd);
        return true;
    }
}

bool launch_hop_plane(const Geo& g, const GaugeSet& gs, HopLaunch& L, hipStream_t st) {
    switch (L.prec) {
        case P32: return launch_plane_p<P32>(g, gs, L, st);
        case P16: return launch_plane_p<P16>(g, gs, L, st);
        default: return false;
    }
}

}  // namespace mdwf
