// Streaming kernels of the solver: layout conversions, vector updates of the
// CG recursion and FP64 reductions with a fixed summation order.
//
// One thread per five-dimensional site; a site's 12 complex components are
// read as 16-byte blocks from the structure-of-arrays layout.  Norms are
// accumulated per thread in the compute precision, then summed in FP64 across
// the wavefront (xor butterfly), the workgroup and, in a second small kernel,
// across workgroups in a fixed order, so results do not depend on timing or on
// which other right-hand sides share the launch.
#include "mdwf_internal.h"

namespace mdwf {

constexpr int kBlas = 256;

int blas_blocks_per_rhs(const Geo& g) { return (g.Vh + kBlas - 1) / kBlas; }

// Loads and stores of the streaming kernels.  The CG vector updates touch
// each field once per launch and their fields are far larger than the caches,
// so they read and write non-temporally (NT): a plain float4 triad reaches
// 6.1 TB/s on the MI355X, a non-temporal one 6.5.
template <Prec P, bool NT = false> struct Ld {
    using R = typename Real<P>::T;
    static __device__ __forceinline__ void load(const void* b, int Vh, int j, cx<double> v[12]) {
        cx<R> t[12];
        Field<P>::template load<NT>(b, Vh, j, t);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {double(t[c].re), double(t[c].im)};
    }
    // stores v, replacing it by the stored (rounded) value
    static __device__ __forceinline__ void store(void* b, int Vh, int j, cx<double> v[12]) {
        cx<R> t[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) t[c] = {R(v[c].re), R(v[c].im)};
        Field<P>::template store<NT>(b, Vh, j, t);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = {double(t[c].re), double(t[c].im)};
    }
};

__device__ __forceinline__ double site_norm2(const cx<double> v[12]) {
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) a += v[c].re * v[c].re + v[c].im * v[c].im;
    return a;
}

// Block reduction in a fixed order; thread 0 writes partials[rhs * nb + blk].
__device__ __forceinline__ void block_partial(double v, double* partials, int rhs, int nb, int blk) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    __shared__ double ws[kBlas / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) ws[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlas / 64; ++w) t += ws[w];
        partials[size_t(rhs) * nb + blk] = t;
    }
}

// ------------------------------------------------------------- gauge field
// canonical U[t][z][y][x][mu][3][3] (FP64) -> per (parity, mu) segments in
// FP64, FP32 and FP16, with the antiperiodic sign folded into the t-links on
// the last time slice (it multiplies both the forward hop out of t = T-1 and
// the backward hop into it).
__device__ __forceinline__ void store_link_rows(char* seg, size_t rb, int Vh4, int i, const cx<double> u[9]) {
    // form 0: rows of U; form 1: rows of U^+ (conjugated columns of U)
    nu4* f0 = reinterpret_cast<nu4*>(seg);
    nu4* f1 = reinterpret_cast<nu4*>(seg + 8 * rb);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        nu4 a = {0u, 0u, 0u, 0u}, b = {0u, 0u, 0u, 0u};
        if (r < 3) {
            const cx<double> x0 = u[3 * r], x1 = u[3 * r + 1], x2 = u[3 * r + 2];   // U[r][k]
            const cx<double> y0 = u[r], y1 = u[3 + r], y2 = u[6 + r];               // U[k][r]
            a.x = f2h(float(x0.re)) | (f2h(float(x1.re)) << 16);
            a.y = f2h(float(x2.re));
            a.z = f2h(float(x0.im)) | (f2h(float(x1.im)) << 16);
            a.w = f2h(float(x2.im));
            b.x = f2h(float(y0.re)) | (f2h(float(y1.re)) << 16);
            b.y = f2h(float(y2.re));
            b.z = f2h(float(-y0.im)) | (f2h(float(-y1.im)) << 16);
            b.w = f2h(float(-y2.im));
        }
        f0[size_t(r) * Vh4 + i] = a;
        f1[size_t(r) * Vh4 + i] = b;
    }
}

__global__ void k_gauge_layout(const Geo g, const double* canon, char* s64, size_t b64, char* s32, size_t b32,
                               char* s16, size_t b16, char* rows, size_t rb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * g.Vh4) return;
    const int p = idx / g.Vh4;
    const int i = idx - p * g.Vh4;
    uint32_t r = uint32_t(i);
    uint32_t q = g.fXh.div(r);
    const int xh = int(r - q * uint32_t(g.Xh));
    r = q;
    q = g.fY.div(r);
    const int y = int(r - q * uint32_t(g.Y));
    r = q;
    q = g.fZ.div(r);
    const int z = int(r - q * uint32_t(g.Z));
    const int t = int(q);
    const int x = 2 * xh + ((y + z + t + p) & 1);
    const size_t lex = size_t(x) + size_t(g.X) * (y + size_t(g.Y) * (z + size_t(g.Z) * t));
    for (int mu = 0; mu < 4; ++mu) {
        const double sign = (mu == 3 && t == g.T - 1 && g.antiperiodic) ? -1.0 : 1.0;
        cx<double> u[9];
        const double* src = canon + (lex * 4 + mu) * 18;
#pragma unroll
        for (int k = 0; k < 9; ++k) u[k] = {sign * src[2 * k], sign * src[2 * k + 1]};
        const int sgi = p * 4 + mu;
        Link<P64>::store(s64 + sgi * b64, g.Vh4, i, u);
        Link<P32>::store(s32 + sgi * b32, g.Vh4, i, u);
        Link<P16>::store(s16 + sgi * b16, g.Vh4, i, u);
        if (rows) store_link_rows(rows + sgi * rb, rb, g.Vh4, i, u);
    }
}

void launch_gauge_layout(const Geo& g, const double* canon, GaugeSet& gs, hipStream_t st) {
    const int n = 2 * g.Vh4;
    hipLaunchKernelGGL(k_gauge_layout, dim3((n + 255) / 256), dim3(256), 0, st, g, canon, gs.seg[0], gs.seg_bytes[0],
                       gs.seg[1], gs.seg_bytes[1], gs.seg[2], gs.seg_bytes[2], gs.mrow, gs.mrow_bytes);
}

// ----------------------------------------------------------- pack / unpack
// kind 0: canonical full field, native parity `p`; kind 1/2: canonical
// parity-compressed half field of parity kind-1.
__device__ __forceinline__ size_t canon_offset(const Geo& g, int full, int p, int i, int s) {
    if (!full) return (size_t(s) * g.Vh4 + i) * 24;
    uint32_t r = uint32_t(i);
    uint32_t q = g.fXh.div(r);
    const int xh = int(r - q * uint32_t(g.Xh));
    r = q;
    q = g.fY.div(r);
    const int y = int(r - q * uint32_t(g.Y));
    r = q;
    q = g.fZ.div(r);
    const int z = int(r - q * uint32_t(g.Z));
    const int t = int(q);
    const int x = 2 * xh + ((y + z + t + p) & 1);
    const size_t V = size_t(2) * g.Vh4;
    const size_t lex = size_t(x) + size_t(g.X) * (y + size_t(g.Y) * (z + size_t(g.Z) * t));
    return (size_t(s) * V + lex) * 24;
}

template <Prec P>
__global__ void k_pack(const Geo g, int full, int p, const double* canon, void* native) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    const int i = j / g.L5, s = j - (j / g.L5) * g.L5;
    const double* src = canon + canon_offset(g, full, p, i, s);
    cx<double> v[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = {src[2 * c], src[2 * c + 1]};
    Ld<P>::store(native, g.Vh, j, v);
}

template <Prec P>
__global__ void k_unpack(const Geo g, int full, int p, const void* native, double* canon) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    const int i = j / g.L5, s = j - (j / g.L5) * g.L5;
    double* dst = canon + canon_offset(g, full, p, i, s);
    cx<double> v[12];
    Ld<P>::load(native, g.Vh, j, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        dst[2 * c] = v[c].re;
        dst[2 * c + 1] = v[c].im;
    }
}

void launch_pack_parity(const Geo& g, Prec p, int full, int par, const double* canon, void* dst, hipStream_t st) {
    const dim3 grid((g.Vh + 255) / 256), blk(256);
    switch (p) {
        case P64: hipLaunchKernelGGL(k_pack<P64>, grid, blk, 0, st, g, full, par, canon, dst); break;
        case P32: hipLaunchKernelGGL(k_pack<P32>, grid, blk, 0, st, g, full, par, canon, dst); break;
        case P16: hipLaunchKernelGGL(k_pack<P16>, grid, blk, 0, st, g, full, par, canon, dst); break;
    }
}

void launch_unpack_parity(const Geo& g, Prec p, int full, int par, const void* src, double* canon, hipStream_t st) {
    const dim3 grid((g.Vh + 255) / 256), blk(256);
    switch (p) {
        case P64: hipLaunchKernelGGL(k_unpack<P64>, grid, blk, 0, st, g, full, par, src, canon); break;
        case P32: hipLaunchKernelGGL(k_unpack<P32>, grid, blk, 0, st, g, full, par, src, canon); break;
        case P16: hipLaunchKernelGGL(k_unpack<P16>, grid, blk, 0, st, g, full, par, src, canon); break;
    }
}

// ------------------------------------------------- point sources and wall fields
// The 5D right-hand side of one spin-colour column of a unit point source
// at 4D site (x, y, z, t): P+ eta on slice L5-1 (spins 0, 1) or P- eta on
// slice 0 (spins 2, 3), in the FP64 native halves `even` and `odd` (zeroed
// by the caller); one thread writes the single non-zero entry.
__global__ void k_point_source(const Geo g, int x, int y, int z, int t, int col, void* even, void* odd) {
    const int par = (x + y + z + t) & 1;
    const int i = (x >> 1) + g.Xh * (y + g.Y * (z + g.Z * t));
    const int s = col / 3 < 2 ? g.L5 - 1 : 0;
    double2* dst = static_cast<double2*>(par ? odd : even);
    dst[size_t(col) * g.Vh + size_t(i) * g.L5 + s] = make_double2(1.0, 0.0);
}

void launch_point_source(const Geo& g, const int src[5], void* even, void* odd, hipStream_t st) {
    hipLaunchKernelGGL(k_point_source, dim3(1), dim3(1), 0, st, g, src[0], src[1], src[2], src[3], src[4], even, odd);
}

// The wall field q = P- x_0 + P+ x_{L5-1} of a 5D solution held as FP64
// native halves, written as a canonical 4D field [t][z][y][x][spin][col].
__global__ void k_wall_field(const Geo g, const void* even, const void* odd, double* q) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * g.Vh4) return;
    const int par = idx >= g.Vh4;
    const int i = idx - par * g.Vh4;
    uint32_t r = uint32_t(i);
    uint32_t qd = g.fXh.div(r);
    const int xh = int(r - qd * uint32_t(g.Xh));
    r = qd;
    qd = g.fY.div(r);
    const int y = int(r - qd * uint32_t(g.Y));
    r = qd;
    qd = g.fZ.div(r);
    const int z = int(r - qd * uint32_t(g.Z));
    const int t = int(qd);
    const int x = 2 * xh + ((y + z + t + par) & 1);
    const size_t lex = size_t(x) + size_t(g.X) * (y + size_t(g.Y) * (z + size_t(g.Z) * t));
    const double2* src = static_cast<const double2*>(par ? odd : even);
    const size_t up = size_t(i) * g.L5 + (g.L5 - 1), dn = size_t(i) * g.L5;
    double2* dst = reinterpret_cast<double2*>(q) + lex * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = src[size_t(c) * g.Vh + (c < 6 ? up : dn)];
}

void launch_wall_field(const Geo& g, const void* even, const void* odd, double* q, hipStream_t st) {
    const int n = 2 * g.Vh4;
    hipLaunchKernelGGL(k_wall_field, dim3((n + 255) / 256), dim3(256), 0, st, g, even, odd, q);
}

void launch_pack(const Geo& g, Prec p, int kind, const double* canon, void* native, hipStream_t st) {
    const size_t hb = half_field_bytes(p, g.Vh);
    if (kind == 0) {
        launch_pack_parity(g, p, 1, 0, canon, native, st);
        launch_pack_parity(g, p, 1, 1, canon, static_cast<char*>(native) + hb, st);
    } else {
        launch_pack_parity(g, p, 0, kind - 1, canon, native, st);
    }
}

void launch_unpack(const Geo& g, Prec p, int kind, const void* native, double* canon, hipStream_t st) {
    const size_t hb = half_field_bytes(p, g.Vh);
    if (kind == 0) {
        launch_unpack_parity(g, p, 1, 0, native, canon, st);
        launch_unpack_parity(g, p, 1, 1, static_cast<const char*>(native) + hb, canon, st);
    } else {
        launch_unpack_parity(g, p, 0, kind - 1, native, canon, st);
    }
}

// --------------------------------------------------------------- convert
template <Prec PI, Prec PO>
__global__ void k_convert(const Geo g, const void* in, void* out, size_t sin, size_t sout, const int* active) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    cx<double> v[12];
    Ld<PI, true>::load(at_rhs(in, sin, rhs), g.Vh, j, v);
    Ld<PO, true>::store(at_rhs(out, sout, rhs), g.Vh, j, v);
}

template <Prec PI>
static void convert_to(const Geo& g, Prec po, const void* in, void* out, size_t sin, size_t sout, int nrhs,
                       const int* active, hipStream_t st) {
    const dim3 grid(blas_blocks_per_rhs(g), nrhs), blk(kBlas);
    switch (po) {
        case P64: hipLaunchKernelGGL((k_convert<PI, P64>), grid, blk, 0, st, g, in, out, sin, sout, active); break;
        case P32: hipLaunchKernelGGL((k_convert<PI, P32>), grid, blk, 0, st, g, in, out, sin, sout, active); break;
        case P16: hipLaunchKernelGGL((k_convert<PI, P16>), grid, blk, 0, st, g, in, out, sin, sout, active); break;
    }
}

void launch_convert(const Geo& g, Prec pin, Prec pout, const void* in, void* out, size_t sin, size_t sout, int nrhs,
                    const int* active, hipStream_t st) {
    switch (pin) {
        case P64: convert_to<P64>(g, pout, in, out, sin, sout, nrhs, active, st); break;
        case P32: convert_to<P32>(g, pout, in, out, sin, sout, nrhs, active, st); break;
        case P16: convert_to<P16>(g, pout, in, out, sin, sout, nrhs, active, st); break;
    }
}

// ----------------------------------------------------------------- axpby
template <Prec P>
__global__ void __launch_bounds__(kBlas) k_axpby(const Geo g, double a, const void* x, double b, const void* y,
                                                 void* z, size_t stride, const int* active, double* partials) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double n2 = 0.0;
    if (j < g.Vh) {
        cx<double> vx[12], vy[12];
        Ld<P, true>::load(at_rhs(x, stride, rhs), g.Vh, j, vx);
        if (y) Ld<P, true>::load(at_rhs(y, stride, rhs), g.Vh, j, vy);
#pragma unroll
        for (int c = 0; c < 12; ++c) vx[c] = y ? a * vx[c] + b * vy[c] : a * vx[c];
        Ld<P, true>::store(at_rhs(z, stride, rhs), g.Vh, j, vx);
        n2 = site_norm2(vx);
    }
    if (partials) block_partial(n2, partials, rhs, gridDim.x, blockIdx.x);
}

void launch_axpby(const Geo& g, Prec p, double a, const void* x, double b, const void* y, void* z, size_t stride,
                  int nrhs, const int* active, double* partials, hipStream_t st) {
    const dim3 grid(blas_blocks_per_rhs(g), nrhs), blk(kBlas);
    switch (p) {
        case P64: hipLaunchKernelGGL(k_axpby<P64>, grid, blk, 0, st, g, a, x, b, y, z, stride, active, partials); break;
        case P32: hipLaunchKernelGGL(k_axpby<P32>, grid, blk, 0, st, g, a, x, b, y, z, stride, active, partials); break;
        case P16: hipLaunchKernelGGL(k_axpby<P16>, grid, blk, 0, st, g, a, x, b, y, z, stride, active, partials); break;
    }
}

template <Prec P>
__global__ void __launch_bounds__(kBlas) k_norm2(const Geo g, const void* x, size_t stride, const int* active,
                                                 double* partials) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    double n2 = 0.0;
    if (j < g.Vh) {
        cx<double> v[12];
        Ld<P>::load(at_rhs(x, stride, rhs), g.Vh, j, v);
        n2 = site_norm2(v);
    }
    block_partial(n2, partials, rhs, gridDim.x, blockIdx.x);
}

void launch_norm2(const Geo& g, Prec p, const void* x, size_t stride, int nrhs, const int* active,
                  double* partials, hipStream_t st) {
    const dim3 grid(blas_blocks_per_rhs(g), nrhs), blk(kBlas);
    switch (p) {
        case P64: hipLaunchKernelGGL(k_norm2<P64>, grid, blk, 0, st, g, x, stride, active, partials); break;
        case P32: hipLaunchKernelGGL(k_norm2<P32>, grid, blk, 0, st, g, x, stride, active, partials); break;
        case P16: hipLaunchKernelGGL(k_norm2<P16>, grid, blk, 0, st, g, x, stride, active, partials); break;
    }
}

// ------------------------------------------------------ CG vector updates
// x += alpha p ; r -= alpha q ; partial |r|^2 of the stored r
// r -= alpha q, with the partials of |r|^2
template <Prec PI>
__global__ void __launch_bounds__(kBlas) k_cg_r(const Geo g, void* r, const void* q, size_t si, const int* active,
                                                const CGScal* sc, double* partials) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const double alpha = sc[rhs].alpha;
    double n2 = 0.0;
    if (j < g.Vh) {
        cx<double> vr[12], vq[12];
        Ld<PI, true>::load(at_rhs(r, si, rhs), g.Vh, j, vr);
        Ld<PI, true>::load(at_rhs(q, si, rhs), g.Vh, j, vq);
#pragma unroll
        for (int c = 0; c < 12; ++c) vr[c] = vr[c] - alpha * vq[c];
        Ld<PI, true>::store(at_rhs(r, si, rhs), g.Vh, j, vr);
        n2 = site_norm2(vr);
    }
    block_partial(n2, partials, rhs, gridDim.x, blockIdx.x);
}

void launch_cg_r(const Geo& g, Prec pi, void* r, const void* q, size_t si, int nrhs, const int* active,
                 const CGScal* sc, double* partials, hipStream_t st) {
    const dim3 grid(blas_blocks_per_rhs(g), nrhs), blk(kBlas);
    switch (pi) {
        case P64: hipLaunchKernelGGL(k_cg_r<P64>, grid, blk, 0, st, g, r, q, si, active, sc, partials); break;
        case P32: hipLaunchKernelGGL(k_cg_r<P32>, grid, blk, 0, st, g, r, q, si, active, sc, partials); break;
        case P16: hipLaunchKernelGGL(k_cg_r<P16>, grid, blk, 0, st, g, r, q, si, active, sc, partials); break;
    }
}

// even iteration of the two-iteration update: pn = s + beta p
template <Prec PI>
__global__ void __launch_bounds__(kBlas) k_cg_p(const Geo g, void* pn, const void* p, const void* s, size_t si,
                                                const int* active, const CGScal* sc) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    const double beta = sc[rhs].beta;
    cx<double> vp[12], vs[12];
    Ld<PI, true>::load(at_rhs(p, si, rhs), g.Vh, j, vp);
    Ld<PI, true>::load(at_rhs(s, si, rhs), g.Vh, j, vs);
#pragma unroll
    for (int c = 0; c < 12; ++c) vp[c] = vs[c] + beta * vp[c];
    Ld<PI, true>::store(at_rhs(pn, si, rhs), g.Vh, j, vp);
}

// odd iteration: x += alpha_prev pp + alpha p, then pp = s + beta p
template <Prec PX, Prec PI>
__global__ void __launch_bounds__(kBlas) k_cg_xp2(const Geo g, void* x, size_t sx, void* pp, const void* p,
                                                  const void* s, size_t si, const int* active, const CGScal* sc) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    const double a0 = sc[rhs].alpha_prev, a1 = sc[rhs].alpha, beta = sc[rhs].beta;
    cx<double> vx[12], vq[12], vp[12], vs[12];
    Ld<PX, true>::load(at_rhs(x, sx, rhs), g.Vh, j, vx);
    Ld<PI, true>::load(at_rhs(pp, si, rhs), g.Vh, j, vq);
    Ld<PI, true>::load(at_rhs(p, si, rhs), g.Vh, j, vp);
    Ld<PI, true>::load(at_rhs(s, si, rhs), g.Vh, j, vs);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        vx[c] = vx[c] + a0 * vq[c] + a1 * vp[c];
        vq[c] = vs[c] + beta * vp[c];
    }
    Ld<PX, true>::store(at_rhs(x, sx, rhs), g.Vh, j, vx);
    Ld<PI, true>::store(at_rhs(pp, si, rhs), g.Vh, j, vq);
}

// x += alpha_prev p
template <Prec PX, Prec PI>
__global__ void __launch_bounds__(kBlas) k_cg_xpend(const Geo g, void* x, size_t sx, const void* p, size_t si,
                                                    const int* active, const CGScal* sc) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    const double a0 = sc[rhs].alpha_prev;
    cx<double> vx[12], vp[12];
    Ld<PX, true>::load(at_rhs(x, sx, rhs), g.Vh, j, vx);
    Ld<PI, true>::load(at_rhs(p, si, rhs), g.Vh, j, vp);
#pragma unroll
    for (int c = 0; c < 12; ++c) vx[c] = vx[c] + a0 * vp[c];
    Ld<PX, true>::store(at_rhs(x, sx, rhs), g.Vh, j, vx);
}

void launch_cg_p(const Geo& g, Prec pi, void* pn, const void* p, const void* s, size_t si, int nrhs,
                 const int* active, const CGScal* sc, hipStream_t st) {
    const dim3 grid(blas_blocks_per_rhs(g), nrhs), blk(kBlas);
    switch (pi) {
        case P64: hipLaunchKernelGGL(k_cg_p<P64>, grid, blk, 0, st, g, pn, p, s, si, active, sc); break;
        case P32: hipLaunchKernelGGL(k_cg_p<P32>, grid, blk, 0, st, g, pn, p, s, si, active, sc); break;
        case P16: hipLaunchKernelGGL(k_cg_p<P16>, grid, blk, 0, st, g, pn, p, s, si, active, sc); break;
    }
}

template <Prec PX>
static void cg_xp2_px(const Geo& g, Prec pi, void* x, size_t sx, void* pp, const void* p, const void* s, size_t si,
                      int nrhs, const int* active, const CGScal* sc, hipStream_t st) {
    const dim3 grid(blas_blocks_per_rhs(g), nrhs), blk(kBlas);
    switch (pi) {
        case P64: hipLaunchKernelGGL((k_cg_xp2<PX, P64>), grid, blk, 0, st, g, x, sx, pp, p, s, si, active, sc); break;
        case P32: hipLaunchKernelGGL((k_cg_xp2<PX, P32>), grid, blk, 0, st, g, x, sx, pp, p, s, si, active, sc); break;
        case P16: hipLaunchKernelGGL((k_cg_xp2<PX, P16>), grid, blk, 0, st, g, x, sx, pp, p, s, si, active, sc); break;
    }
}

void launch_cg_xp2(const Geo& g, Prec px, Prec pi, void* x, size_t sx, void* pp, const void* p, const void* s,
                   size_t si, int nrhs, const int* active, const CGScal* sc, hipStream_t st) {
    switch (px) {
        case P64: cg_xp2_px<P64>(g, pi, x, sx, pp, p, s, si, nrhs, active, sc, st); break;
        case P32: cg_xp2_px<P32>(g, pi, x, sx, pp, p, s, si, nrhs, active, sc, st); break;
        case P16: cg_xp2_px<P16>(g, pi, x, sx, pp, p, s, si, nrhs, active, sc, st); break;
    }
}

template <Prec PX>
static void cg_xpend_px(const Geo& g, Prec pi, void* x, size_t sx, const void* p, size_t si, int nrhs,
                        const int* active, const CGScal* sc, hipStream_t st) {
    const dim3 grid(blas_blocks_per_rhs(g), nrhs), blk(kBlas);
    switch (pi) {
        case P64: hipLaunchKernelGGL((k_cg_xpend<PX, P64>), grid, blk, 0, st, g, x, sx, p, si, active, sc); break;
        case P32: hipLaunchKernelGGL((k_cg_xpend<PX, P32>), grid, blk, 0, st, g, x, sx, p, si, active, sc); break;
        case P16: hipLaunchKernelGGL((k_cg_xpend<PX, P16>), grid, blk, 0, st, g, x, sx, p, si, active, sc); break;
    }
}

void launch_cg_xpend(const Geo& g, Prec px, Prec pi, void* x, size_t sx, const void* p, size_t si, int nrhs,
                     const int* active, const CGScal* sc, hipStream_t st) {
    switch (px) {
        case P64: cg_xpend_px<P64>(g, pi, x, sx, p, si, nrhs, active, sc, st); break;
        case P32: cg_xpend_px<P32>(g, pi, x, sx, p, si, nrhs, active, sc, st); break;
        case P16: cg_xpend_px<P16>(g, pi, x, sx, p, si, nrhs, active, sc, st); break;
    }
}

// x_hi += x_lo ; x_lo = 0
template <Prec PX>
__global__ void __launch_bounds__(kBlas) k_flush(const Geo g, void* xhi, size_t shi, void* xlo, size_t slo,
                                                 const int* active) {
    const int rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= g.Vh) return;
    cx<double> vh[12], vl[12];
    Ld<P64, true>::load(at_rhs(xhi, shi, rhs), g.Vh, j, vh);
    Ld<PX, true>::load(at_rhs(xlo, slo, rhs), g.Vh, j, vl);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        vh[c] = vh[c] + vl[c];
        vl[c] = {0.0, 0.0};
    }
    Ld<P64, true>::store(at_rhs(xhi, shi, rhs), g.Vh, j, vh);
    Ld<PX, true>::store(at_rhs(xlo, slo, rhs), g.Vh, j, vl);
}

void launch_flush(const Geo& g, Prec px, void* xhi, size_t shi, void* xlo, size_t slo, int nrhs, const int* active,
                  hipStream_t st) {
    const dim3 grid(blas_blocks_per_rhs(g), nrhs), blk(kBlas);
    switch (px) {
        case P64: hipLaunchKernelGGL(k_flush<P64>, grid, blk, 0, st, g, xhi, shi, xlo, slo, active); break;
        case P32: hipLaunchKernelGGL(k_flush<P32>, grid, blk, 0, st, g, xhi, shi, xlo, slo, active); break;
        case P16: hipLaunchKernelGGL(k_flush<P16>, grid, blk, 0, st, g, xhi, shi, xlo, slo, active); break;
    }
}

// ------------------------------------------------------------ CG scalars
__global__ void __launch_bounds__(256) k_scalars(int op, const double* partials, int nblk, const int* active,
                                                 CGScal* sc, double* out_sum) {
    const int rhs = blockIdx.x;
    if (active && !active[rhs]) return;
    double v = 0.0;
    const double* p = partials + size_t(rhs) * nblk;
    for (int k = threadIdx.x; k < nblk; k += 256) v += p[k];
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double tot = sh[0];
    CGScal& c = sc[rhs];
    const bool ok = isfinite(tot);
    switch (op) {
        case SC_ALPHA:
            c.delta = tot;
            if (ok && tot > 0.0) c.alpha = c.gamma / tot;
            else { c.alpha = 0.0; c.bad = 1; }
            break;
        case SC_BETA:
            if (ok && c.gamma > 0.0) c.beta = tot / c.gamma;
            else { c.beta = 0.0; c.bad = 1; }
            c.gamma = tot;
            break;
        case SC_SET_GAMMA:
            c.gamma = tot;
            if (!ok) c.bad = 1;
            break;
        case SC_RR:
            c.rr = tot;
            if (!ok) c.bad = 1;
            break;
        case SC_ALPHA_KEEP:
            c.delta = tot;
            if (ok && tot > 0.0) c.alpha = c.gamma / tot;
            else { c.alpha = 0.0; c.bad = 1; }
            c.alpha_prev = c.alpha;
            break;
        case SC_CLEAR_PREV:
            c.alpha_prev = 0.0;
            break;
        default: break;
    }
    if (out_sum) out_sum[rhs] = tot;
}

void launch_scalars(ScalOp op, const double* partials, int nblk, int nrhs, const int* active, CGScal* sc,
                    double* out_sum, hipStream_t st) {
    hipLaunchKernelGGL(k_scalars, dim3(nrhs), dim3(256), 0, st, int(op), partials, nblk, active, sc, out_sum);
}

}  // namespace mdwf
