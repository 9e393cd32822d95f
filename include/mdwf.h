/*
 * mdwf.h -- C ABI of libmdwf, an MI355X (gfx950) solver for the Moebius
 * domain-wall fermion operator of arXiv:1701.07559.
 *
 * What is computed (paper Sec. II and Sec. VII):
 *   The 5D Moebius domain-wall operator on SU(3) links with domain-wall height
 *   M5, fifth-dimension extent L5, Moebius parameters b5, c5 and quark mass m_q.
 *   Its 4D kernel is the paper's Moebius kernel
 *     D^M = (b5 + c5) D_W(M5) / (2 + (b5 - c5) D_W(M5))            (Sec. II)
 *   realised in 5D as
 *     D5 = D_W B + 1 - C,  B = b5 + c5 C,
 *     (C psi)_s = P- psi_{s+1} + P+ psi_{s-1}, with -m_q on the wrap,
 *     D_W = (4 - M5) - 1/2 Dslash,
 *     Dslash psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^+ psi(x-mu).
 *   D5 splits into the 4D-site-local K5 = (4 - M5) B + 1 - C and the hop
 *   -1/2 Dslash B.  The solver works on the asymmetric even-odd Schur
 *   complement the paper names (Sec. VII):
 *     S = K5 - 1/4 D_eo B K5^-1 D_oe B   on the even 4D sites,
 *   and solves D5 x = b by CG on the normal equations (least-squares form) of
 *   S, of the symmetric form K5^-1 S (Sec. VII) or of S B^-1 (right
 *   preconditioning by B), optionally with an FP32 or FP16 inner solve and
 *   FP64 reliable updates (the paper's "double-half" mixed-precision solver,
 *   Sec. VII).
 *
 * Conventions:
 *   Euclidean chiral gamma basis, g5 = diag(1, 1, -1, -1); P+ = spins 0,1.
 *   4D parity = (x + y + z + t) mod 2; every lattice extent must be even.
 *   Time may be antiperiodic for the fermions (hops across the t boundary
 *   carry -1); x, y, z are periodic.
 *
 * Host canonical layouts (all FP64, complex as re,im pairs):
 *   gauge     U[t][z][y][x][mu][a][b]        mu = 0..3 -> x, y, z, t; row a, col b
 *   full 5D   psi[s][t][z][y][x][spin][col]  x fastest
 *   half 5D   psi[s][t][z][y][x/2][spin][col]  the sites of one parity, in the
 *             same order with x compressed (used by the SCHUR and HOP ops)
 *
 * Device native layout (what *_dev entry points take), per half field of
 * Vh = L5 * V/2 five-dimensional sites, 5D site index j = i * L5 + s with i
 * the parity-compressed 4D index:
 *   F64: 12 blocks of double2 [12][Vh]  (one complex component per block)
 *   F32:  6 blocks of float4  [6][Vh]   (two complex components per block)
 *   F16:  3 blocks of 8 x half [3][Vh], then one float norm per site [Vh];
 *         a stored value is half(v / norm) with norm = max |re|,|im| of the site
 * Component order inside a site is spin-major: c = spin * 3 + colour.
 * A half field occupies mdwf_field_bytes(..., MDWF_HALF_*) bytes; a full field
 * is the even half followed by the odd half.
 *
 * Errors: every call returns a status; nothing aborts or throws across the
 * ABI.  mdwf_last_error() describes the last failure on a context.
 * Threading: one context per host thread.  A context's device temporaries
 * (the Schur operators' odd intermediate, the batched coefficient table, the
 * solver's vectors) serve all of its calls, so work that one context enqueues
 * on different streams must be ordered by the caller; a temporary that has to
 * grow waits for the device first.  Ownership: the caller owns every
 * pointer it passes; the library copies what it needs and frees only memory it
 * allocated itself.
 */
#ifndef MDWF_H
#define MDWF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdwf_ctx mdwf_ctx;

typedef enum {
    MDWF_OK = 0,
    MDWF_ERR_ARG = 1,      /* invalid argument (extent, parameter, null pointer) */
    MDWF_ERR_STATE = 2,    /* call out of order (no gauge field / action yet)   */
    MDWF_ERR_OOM = 3,      /* device allocation failed                          */
    MDWF_ERR_HIP = 4,      /* HIP runtime error                                 */
    MDWF_ERR_NOCONV = 5,   /* solver stopped at max_iter or max_seconds; best x written */
    MDWF_ERR_NUMERIC = 6   /* NaN/Inf or breakdown in a reduction               */
} mdwf_status;

typedef enum { MDWF_F64 = 0, MDWF_F32 = 1, MDWF_F16 = 2 } mdwf_prec;

typedef enum {
    MDWF_FULL = 0,     /* both parities, even half then odd half */
    MDWF_HALF_EVEN = 1,
    MDWF_HALF_ODD = 2
} mdwf_field_kind;

/* Operators.  Field kinds in -> out are given for each. */
typedef enum {
    MDWF_OP_D5 = 0,          /* full -> full : D5                                 */
    MDWF_OP_D5_DAG = 1,      /* full -> full : D5^+ = B^+ D_W^+ + 1 - C^+         */
    MDWF_OP_SCHUR = 2,       /* even -> even : S                                  */
    MDWF_OP_SCHUR_DAG = 3,   /* even -> even : S^+                                */
    MDWF_OP_HOP_EO = 4,      /* odd -> even  : Dslash (bare hop, no factor)       */
    MDWF_OP_HOP_OE = 5,      /* even -> odd  : Dslash                             */
    MDWF_OP_K5 = 6,          /* full -> full : K5                                 */
    MDWF_OP_K5INV = 7,       /* full -> full : K5^-1                              */
    MDWF_OP_HOP_EO_DAG = 8,  /* odd -> even  : Dslash^+ = g5 Dslash g5            */
    MDWF_OP_HOP_OE_DAG = 9,  /* even -> odd  : Dslash^+                           */
    MDWF_OP_K5_DAG = 10,     /* full -> full : K5^+                               */
    MDWF_OP_K5INV_DAG = 11,  /* full -> full : (K5^+)^-1                          */
    MDWF_OP_B = 12,          /* full -> full : B = b5 + c5 C                      */
    MDWF_OP_B_DAG = 13,      /* full -> full : B^+                                */
    MDWF_OP_SCHUR_SYM = 14,  /* even -> even : K5^-1 S (symmetric form, Sec. VII) */
    MDWF_OP_SCHUR_SYM_DAG = 15, /* even -> even : S^+ K5^-+                      */
    MDWF_OP_SCHUR_RP = 16,   /* even -> even : S B^-1 (right preconditioning by B) */
    MDWF_OP_SCHUR_RP_DAG = 17, /* even -> even : B^-+ S^+                        */
    MDWF_OP_BINV = 18,       /* full -> full : B^-1                               */
    MDWF_OP_BINV_DAG = 19,   /* full -> full : (B^+)^-1                           */
    MDWF_OP_COUNT = 20
} mdwf_op;

typedef struct {
    int X, Y, Z, T;        /* all even, >= 2 */
    int antiperiodic_t;    /* 1: fermion fields antiperiodic in t */
} mdwf_geometry;

/* Action parameters (paper Sec. II / III.A): requires b5 > c5 >= 0,
 * 0 <= mq <= 1, 1 <= L5 <= 32, 0 < M5 < 2, and L5 x V/2 < 268435456 (the
 * kernels address a field block with 32-bit byte offsets). */
typedef struct {
    double M5, b5, c5, mq;
    int L5;
} mdwf_action;

typedef struct {
    double tol;          /* target ||b - D5 x|| / ||b||, e.g. 1e-10            */
    int max_iter;        /* cap on inner CG iterations per right-hand side     */
    mdwf_prec inner;     /* precision of the inner CG (F64 = plain FP64 CG)    */
    double delta;        /* reliable update when ||r|| < delta * ||r_last||    */
    int check_every;     /* host convergence check period in iterations (>=1)  */
    int use_graph;       /* 1: replay CG iterations from a captured hipGraph   */
    int profile_iters;   /* time the inner operator launches of this many CG
                            iterations (from the third on, profile_every
                            apart) with HIP events on the solve stream;
                            0 = off, at most 64, ignored with use_graph      */
    int schur_form;      /* CG operator: 0 the asymmetric S x_e = b'_e;
                            1 the symmetric K5^-1 S x_e = K5^-1 b'_e (Sec.
                            VII); 2 S B^-1 y = b'_e, x_e = B^-1 y (right
                            preconditioning by B: no B before the first hop,
                            none after the adjoint's second).  The stop is
                            the same true residual ||b - D5 x|| / ||b||     */
    double max_seconds;  /* > 0: a time limit for the call; once it has run
                            this long every unconverged RHS stops as at
                            max_iter (ERR_NOCONV, best x written); 0 = none */
    const double *const *x_ref; /* optional reference solutions, one per RHS
                            (NULL = none): canonical full FP64 fields in the
                            memory space of x (host for mdwf_solve, device for
                            mdwf_solve_dev), e.g. the plain FP64 CG solutions
                            of the same systems.  Each is read once, after its
                            RHS has been solved, to fill info.err_vs_ref */
    int profile_every;   /* > 1: the profiled iterations are the third, then
                            every profile_every-th (so the samples can span
                            the whole solve); 0 or 1: consecutive            */
} mdwf_solver_opts;
/* There is no switch for deterministic solves: every solve is.  The CG dot
 * products are summed per RHS in a fixed order (wavefront butterfly, then the
 * workgroup, then the workgroup partials in index order), no reduction
 * crosses right-hand sides, and no atomics are used, so a solve repeated with
 * the same inputs, launch shape and device gives the same bits, and an RHS
 * gives the same bits alone, in any batch, chunk or sub-batch and in a served
 * request. */

typedef struct {
    int iters;            /* inner CG iterations                                  */
    int reliable_updates; /* FP64 residual recomputations                         */
    int restarts;         /* true-residual checks that failed and restarted       */
    double true_resid;    /* ||b - D5 x|| / ||b|| in FP64 on the returned x        */
    double seconds;       /* wall time of the solve call                          */
    double model_flops;   /* flops of the model counted for this right-hand side  */
    double model_bytes;   /* algorithmic HBM bytes of the model for this RHS       */
    double hop_us[4];     /* profile_iters > 0: mean duration (us) of one launch of
                             kernel A, B, A^+, B^+ of the CG operator (inner
                             precision, first chunk of right-hand sides, all its
                             RHS together); else 0 */
    int hop_rhs;          /* right-hand sides in those launches                   */
    int hop_samples;      /* iterations sampled                                   */
    double err_vs_ref;    /* ||x - x_ref|| / ||x_ref|| in FP64 over the full 5D
                             field when opts.x_ref is given, else -1 (a mixed-
                             precision solution against the FP64 one: the
                             per-solve error of the mixed solver, Sec. VII)    */
    int launch_rhs;       /* right-hand sides that shared this RHS's operator
                             launches (served requests: of every request in
                             the shared solve)                                 */
} mdwf_solve_info;

/* Create a context for one lattice geometry on HIP device `hip_device`.
 * hip_stream: a hipStream_t to run on, or NULL for a stream the library owns.
 * Fails with ERR_ARG on odd or non-positive extents, ERR_HIP on a bad device. */
mdwf_status mdwf_create(const mdwf_geometry *geom, int hip_device, void *hip_stream, mdwf_ctx **out);

/* Release all device memory the context owns.  NULL is ignored. */
void mdwf_destroy(mdwf_ctx *ctx);

/* Description of the last error on ctx (or of the last failed create when ctx
 * is NULL).  Valid until the next call on the same context. */
const char *mdwf_last_error(const mdwf_ctx *ctx);

/* Copy the SU(3) gauge links U_mu(x) the Wilson hop of D_W uses (Sec. I:
 * the 4D links are copied onto every fifth-dimension slice) from host memory
 * (canonical layout, FP64) to the device, in FP64, FP32 and FP16 native link
 * layouts (the three precisions of the mixed solver, Sec. VII), with the
 * antiperiodic time sign folded into the links on the last time slice.
 * The FP16 copy holds the entries as binary16 with no scale, which suits
 * SU(3) links (every entry at most 1 in magnitude); FP64 and FP32 take any
 * links.  Synchronous.  ERR_ARG on a null pointer. */
mdwf_status mdwf_load_gauge(mdwf_ctx *ctx, const double *U);

/* Same as mdwf_load_gauge from a device pointer in the canonical layout. */
mdwf_status mdwf_load_gauge_dev(mdwf_ctx *ctx, const double *U_dev);

/* Set M5, b5, c5, L5, m_q (paper Sec. II, the Moebius kernel, and Sec. III.A,
 * the tuned parameters).  Validates as documented above.  Waits for the work
 * already enqueued on the context's stream, which reads the coefficient
 * table this call replaces; launches that mdwf_apply_dev enqueued on another
 * stream must have completed before this call (the caller synchronizes that
 * stream). */
mdwf_status mdwf_set_action(mdwf_ctx *ctx, const mdwf_action *act);

/* Bytes of one field of the given kind and precision in the native layout. */
mdwf_status mdwf_field_bytes(const mdwf_ctx *ctx, mdwf_prec prec, mdwf_field_kind kind, size_t *bytes);

/* Convert between the canonical FP64 layout and the native layout, both on the
 * device.  For MDWF_HALF_* the canonical array is the parity-compressed one. */
mdwf_status mdwf_pack_dev(mdwf_ctx *ctx, mdwf_prec prec, mdwf_field_kind kind,
                          const double *canon_dev, void *native_dev, void *stream);
mdwf_status mdwf_unpack_dev(mdwf_ctx *ctx, mdwf_prec prec, mdwf_field_kind kind,
                            const void *native_dev, double *canon_dev, void *stream);

/* Apply an operator of the list above -- D5 (the Moebius operator, Sec. II),
 * the even-odd Schur complements (Sec. VII) or their parts -- to a host
 * canonical FP64 field; the arithmetic runs on the device in precision
 * `prec` (input rounded to it, output widened back).  Synchronous.  ERR_ARG
 * on a bad operator, precision or null pointer; ERR_STATE before
 * mdwf_set_action / mdwf_load_gauge. */
mdwf_status mdwf_apply(mdwf_ctx *ctx, mdwf_op op, mdwf_prec prec, const double *in, double *out);

/* Apply an operator to device native fields in precision `prec` on `stream`
 * (NULL = the context's stream).  in and out must not overlap.  Asynchronous:
 * returns after enqueueing. */
mdwf_status mdwf_apply_dev(mdwf_ctx *ctx, mdwf_op op, mdwf_prec prec, const void *in, void *out,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same as
 * mdwf_apply_dev (asynchronous on `stream`, NULL = the context's stream),
 * but it calls no allocating routine.  The Schur operators' odd-parity
 * intermediate (two of them for MDWF_OP_SCHUR_SYM_DAG) lives in a static
 * device array of MDWF_STATIC_SCRATCH_BYTES that the library holds on each
 * device it runs on until the process ends; an operator whose intermediate
 * does not fit fails with ERR_ARG.  The intermediate is written in full
 * before it is read, so nothing in the array needs clearing.  Every call on
 * one device shares that device's array and it keeps the last call's
 * contents: calls whose work overlaps on one device (different streams or
 * host threads, or a caller's graph replayed beside them) race, and the
 * caller must order them.  The caller still owns and passes in and out. */
#define MDWF_STATIC_SCRATCH_BYTES (256u << 20)
mdwf_status mdwf_apply_dev_noalloc(mdwf_ctx *ctx, mdwf_op op, mdwf_prec prec, const void *in, void *out,
                                   void *stream);

/* Apply an operator to nrhs device native fields at once, right-hand side k
 * at in + k * stride and out + k * stride (bytes; stride >= the field's
 * bytes, a multiple of 256), each with its own quark mass mq[k] (host array;
 * NULL = the action's m_q for all).  Every launch takes all RHS together and
 * reads each link once for them, as the solver's multi-RHS iterations do
 * (Sec. III.A: propagators at several masses and sources), in the launch
 * shape installed for `prec` (mdwf_autotune_solve).  Symmetric-form ops are
 * not batched here (ERR_ARG).  Asynchronous on `stream` (NULL = the context's
 * stream); in and out must not overlap.  Allocates (grow-only, kept by the
 * context) a coefficient table and, for the Schur ops, the odd temporary of
 * nrhs fields. */
mdwf_status mdwf_apply_batch_dev(mdwf_ctx *ctx, mdwf_op op, mdwf_prec prec, int nrhs, const void *in, void *out,
                                 size_t stride, const double *mq, void *stream);

/* Solve D5 x_k = b_k for k < nrhs (host canonical full FP64 fields): the
 * MDWF propagator solves of the paper (Sec. III.A) by CG on the normal
 * equations of the even-odd system (Sec. VII), in FP64 or with the FP32 /
 * FP16 inner solve and FP64 reliable updates of the mixed solver (Sec. VII).
 * mq: per-RHS quark mass (NULL = the action's m_q); all other action
 * parameters are shared.  info: array of nrhs records (may be NULL).
 * All RHS share every operator launch; when their vectors do not fit in
 * free device memory together, consecutive sub-batches are solved in turn.
 * Returns ERR_NOCONV if any RHS hit max_iter or the time limit (its best x is
 * still written). */
mdwf_status mdwf_solve(mdwf_ctx *ctx, int nrhs, const double *const *b, double *const *x,
                       const double *mq, const mdwf_solver_opts *opts, mdwf_solve_info *info);

/* Same as mdwf_solve with canonical FP64 fields already in device memory.
 * Synchronous with respect to `stream` (NULL = the context's stream). */
mdwf_status mdwf_solve_dev(mdwf_ctx *ctx, int nrhs, const double *const *b_dev, double *const *x_dev,
                           const double *mq, const mdwf_solver_opts *opts, mdwf_solve_info *info,
                           void *stream);

/* The propagator solves of a point source (Sec. III.A: MDWF propagators from
 * point and smeared sources): column k < ncols is the 5D right-hand side of
 * spin-colour column cols[k] (NULL: k; c = spin * 3 + colour) of a unit
 * point source eta at site = (x, y, z, t): P+ eta on slice L5-1 for spins
 * 0, 1 and P- eta on slice 0 for spins 2, 3.  The sources are generated on
 * the device and no 5D field crosses to the host: q[k] (host, canonical 4D
 * [t][z][y][x][spin][col] complex) receives the wall field
 * q = P- x_0 + P+ x_{L5-1} of the solution, from which the 4D propagator
 * and the pseudoscalar correlator follow (mdwf_pion_correlator_dev).
 * Otherwise as mdwf_solve (opts.x_ref must be NULL).  ERR_ARG on a site
 * outside the lattice or a column outside 0..11. */
mdwf_status mdwf_solve_point(mdwf_ctx *ctx, const int *site, int ncols, const int *cols, const double *mq,
                             const mdwf_solver_opts *opts, double *const *q, mdwf_solve_info *info);

/* Fill opts with defaults: tol 1e-10, max_iter 100000, inner F64, delta 0.1,
 * check_every 1, use_graph 0, profile_iters 0, schur_form 0, max_seconds 0,
 * x_ref NULL. */
void mdwf_default_opts(mdwf_solver_opts *opts);

/* Device bytes a solve of nrhs RHS on this lattice at fifth-dimension extent
 * L5 allocates (its memory plan: per RHS x_hi and b' in FP64, r, p, p', s, q
 * in the inner precision and an FP32 x_lo when mixed; shared FP64 scratch,
 * the hop temporary, a canonical staging field and a margin for small
 * tables).  host_io: 0 device fields (mdwf_solve_dev, no staging), 1 host
 * fields (mdwf_solve, a 5D staging field), 2 point sources with host wall
 * fields (mdwf_solve_point, a 4D staging field).  Host arithmetic only, no
 * device needed.  ERR_ARG on a bad geometry, L5, precision, host_io or
 * nrhs < 1. */
mdwf_status mdwf_solve_footprint(const mdwf_geometry *geom, int L5, mdwf_prec inner, int nrhs, int host_io,
                                 size_t *bytes);

/* Launch shape of the hop kernels for one storage precision. */
typedef struct {
    int tile[4];     /* traversal tile in parity-compressed sites (X/2, Y, Z, T
                        extents, each dividing the lattice's): inside a tile x
                        runs fastest, then y, z, t; tiles follow t fastest,
                        then x, y, z.  {X/2, Y, zb, 1} are z-blocks, t inside */
    int xcd_remap;   /* 1: workgroups renumbered so each XCD walks one contiguous range */
    int nt_store;    /* 1: hop outputs written with non-temporal stores               */
    int link_mode;   /* links: 0 loaded by every lane, 1 staged in LDS (L5 >= 8),
                        2 one 16-byte part per lane, gathered by lane exchange
                        (FP32 / FP16, L5 >= 4 / 2), 3 FP16 SU(3) products on
                        the matrix cores (4x4x4 blocks of four slices of one
                        site: L5 a multiple of 4; kernels without a B
                        pre-hop); otherwise 0 is used                      */
    int rhs_group;   /* multi-RHS launches: groups of this many RHS sweep the tiles
                        together, RHS fastest (they share each tile's links);
                        groups follow each other; 0 = all RHS in one group    */
    double us;       /* measured time of one Schur application with this shape (us)   */
    int plane_bt;    /* > 0 (dividing T): the bare hops (MDWF_OP_HOP_*) of FP32 and FP16
                        run plane-staged: a workgroup copies each time plane of
                        a 4x4x4 spatial block and its faces into LDS once and
                        marches plane_bt planes along t (spatial extents
                        multiples of 4, L5 <= 16, else the lane-per-site
                        kernel runs); 0 = off.  mdwf_autotune sets it for
                        FP32 / FP16 when it times faster on one bare hop. */
} mdwf_launch_tune;

/* Autotuner: for each precision (index mdwf_prec), time one Schur operator
 * application (the two fused hop kernels) on scratch fields, choosing in turn
 * the traversal tile (z-blocks and compact 4D tiles), the link mode, then
 * non-temporal stores and workgroup numbering, and keep the fastest in the
 * context; for FP32 and FP16 it then times one bare hop with the lane-per-site
 * kernel and with plane_bt 4, 8, 16 (those dividing T) and keeps a plane run
 * that is at least 2 % faster.  out[3] (may be NULL) receives the chosen
 * shapes.  Needs the action and gauge field; allocates scratch device memory
 * (three half fields of each precision). */
mdwf_status mdwf_autotune(mdwf_ctx *ctx, mdwf_launch_tune *out);

/* Autotuner for the launches of one solve shape: the inner precision
 * opts->inner is tuned on the CG operator of opts->schur_form and its
 * adjoint with nrhs RHS per launch (as one CG iteration launches them;
 * candidates also include the RHS grouping), and, for a mixed inner
 * precision, FP64 on that operator with one RHS (the reliable updates).
 * Other precisions keep their shapes.  out[3] (may be NULL) receives every
 * precision's shape.  opts NULL = defaults.  Scratch: four (symmetric
 * form: five) inner-precision half fields per RHS.  ERR_ARG on nrhs < 1 or
 * bad options. */
mdwf_status mdwf_autotune_solve(mdwf_ctx *ctx, const mdwf_solver_opts *opts, int nrhs, mdwf_launch_tune *out);

/* Current launch shape of precision `prec` (defaults before autotuning). */
mdwf_status mdwf_get_tune(const mdwf_ctx *ctx, mdwf_prec prec, mdwf_launch_tune *out);

/* Install a launch shape for precision `prec` (e.g. one mdwf_autotune chose
 * earlier).  Launches already enqueued keep the shape they were given.
 * ERR_ARG if a tile extent does not divide the lattice's or plane_bt does not
 * divide T. */
mdwf_status mdwf_set_tune(mdwf_ctx *ctx, mdwf_prec prec, const mdwf_launch_tune *t);

/* Model flop and byte counts for one application of an operator (per call). */
mdwf_status mdwf_op_model(const mdwf_ctx *ctx, mdwf_op op, mdwf_prec prec, double *flops, double *bytes);

/* ------------------------------------------------------- gradient flow
 * Wilson gradient flow of a gauge field, the smearing the paper applies to
 * its ensembles before the valence solves (Sec. III; flow time t_gf = 1):
 *   dV/dt = Z(V) V,  Z_mu(x) = -1/2 (O - O^+) + 1/6 tr(O - O^+),
 *   O_mu(x) = U_mu(x) * (sum of the six staples of the link),
 * integrated in FP64 with Luscher's third-order Runge-Kutta scheme, nsteps
 * steps of size eps (flow time nsteps * eps).  U is a canonical gauge field
 * (layout of mdwf_load_gauge), flowed in place; all directions periodic (the
 * fermion boundary condition plays no part).  plaq (may be NULL) receives
 * the average plaquette before and after.  The links must be SU(3) to
 * rounding (unitary, det 1): the staple links enter through their first two
 * rows, the third being the conjugated cross product of those.  A field
 * with an entry of U U^+ - 1 or of det U - 1 beyond 1e-10 (or a NaN) is
 * refused with ERR_ARG before anything is written.  Extents >= 2; ERR_ARG
 * on eps <= 0 or nsteps < 0.  Synchronous; allocates one link field and
 * eight reals per link of scratch. */
mdwf_status mdwf_wilson_flow(const mdwf_geometry *geom, int hip_device, double *U, double eps, int nsteps,
                             double *plaq);
/* Same on a device field, on `stream` (NULL = the null stream). */
mdwf_status mdwf_wilson_flow_dev(const mdwf_geometry *geom, double *U_dev, double eps, int nsteps, void *stream,
                                 double *plaq);
/* Average plaquette (1/3) Re tr U(p) over sites and the six planes of a
 * device gauge field (fixed-order reduction).  Synchronous on `stream`. */
mdwf_status mdwf_plaquette_dev(const mdwf_geometry *geom, const double *U_dev, void *stream, double *plaq);

/* ------------------------------------------------ sources and sinks
 * The steps around the solves of a propagator (paper Sec. V: MDWF
 * propagators from gauge-covariant Gaussian-smeared sources; Sec. III: the
 * residual mass m_res from the midpoint and wall pseudoscalar correlators,
 * with the Shamir midpoint density).  All fields are canonical FP64 device
 * arrays, nvec of them back to back:
 *   4D spinor  psi[t][z][y][x][spin][col]   (12 complex per site)
 *   5D spinor  psi[s][t][z][y][x][spin][col]
 * U_dev is a canonical gauge field (layout of mdwf_load_gauge).  Extents
 * only need to be >= 1 here (no even-odd split).  Each call is asynchronous
 * on `stream` (NULL = the null stream) unless stated; errors: ERR_ARG on a
 * null pointer, a bad count or parameter, ERR_HIP / ERR_OOM from the runtime.
 *
 * mdwf_gauss_smear_dev: out = (1 + sigma^2/(4 niter) Delta)^niter in, with
 *   the covariant spatial Laplacian
 *   (Delta psi)(x) = sum_{i=x,y,z} U_i(x) psi(x+i) + U_i(x-i)^+ psi(x-i) - 2 psi(x),
 *   periodic in space, each time slice on its own.  in and out must not
 *   overlap; niter = 0 copies.  For niter >= 2 it allocates one scratch
 *   field set and returns after the stream has finished it. */
mdwf_status mdwf_gauss_smear_dev(const mdwf_geometry *geom, const double *U_dev, int nvec, const double *in_dev,
                                 double *out_dev, double sigma, int niter, void *stream);

/* mdwf_wall_source_dev: the 5D right-hand side whose solution of D5 x = b
 *   carries the 4D quark propagator of the 4D source eta:
 *     b = (1 - c5 D_W) Pbar eta,  (Pbar eta)_{L5-1} = P- eta, (Pbar eta)_0 = P+ eta,
 *   all other slices zero (c5 = 0 gives the Shamir source).  The wall field
 *   q = P- x_0 + P+ x_{L5-1} of the solution is then (D_eff^-1 - 1)/(1 - m_q) eta
 *   with D_eff the 4D effective operator of D5.  Uses M5, c5 and L5 of act
 *   (L5 >= 1) and the fermion time boundary of geom; b holds nvec 5D fields. */
mdwf_status mdwf_wall_source_dev(const mdwf_geometry *geom, const mdwf_action *act, const double *U_dev, int nvec,
                                 const double *eta_dev, double *b_dev, void *stream);

/* mdwf_project_4d_dev: from nvec 5D fields x, the wall fields
 *   q = P- x_0 + P+ x_{L5-1} into q_dev and, if mid_dev is not NULL (L5 even),
 *   the midpoint fields Q = P- x_{L5/2} + P+ x_{L5/2-1} into mid_dev (4D). */
mdwf_status mdwf_project_4d_dev(const mdwf_geometry *geom, int L5, int nvec, const double *x_dev, double *q_dev,
                                double *mid_dev, void *stream);

/* mdwf_mres_correlators_dev: for each time slice t (host arrays of T):
 *   c_pp[t] = sum over the slice's sites, spins, colours and the nvec
 *             solutions of |q|^2 (the pseudoscalar correlator of a source's
 *             spin-colour columns),
 *   c_mp[t] = the same of |Q|^2 (the midpoint correlator),
 *   mres[t] = c_mp[t] / c_pp[t]   (NaN or inf where c_pp[t] = 0).
 *   L5 even >= 2, T <= 65535.  Fixed-order reductions (deterministic).  Synchronous;
 *   allocates a small partial-sum buffer. */
mdwf_status mdwf_mres_correlators_dev(const mdwf_geometry *geom, int L5, int nvec, const double *x_dev, void *stream,
                                      double *c_pp, double *c_mp, double *mres);

/* mdwf_pion_correlator_dev: c[t] (host, T values) = sum over the slice's
 *   sites, spins, colours and the nvec 4D fields q of |q|^2: the
 *   pseudoscalar correlator of a source's columns with any sink, e.g. the
 *   wall fields of mdwf_project_4d_dev as they are (then c equals c_pp
 *   above, bit for bit) or after mdwf_gauss_smear_dev (a smeared sink).
 *   T <= 65535.  Fixed-order reductions.  Synchronous; allocates a small
 *   partial-sum buffer. */
mdwf_status mdwf_pion_correlator_dev(const mdwf_geometry *geom, int nvec, const double *q_dev, void *stream,
                                     double *c);

/* ------------------------------------------------------------ serving
 * A request server for many solves of D5 x = b (the paper computes
 * propagators for several ensembles, masses and sources, Sec. III): gauge
 * fields are uploaded once and stay resident; requests (field, action incl.
 * L5, per-RHS masses, 1..n RHS, solver options) may be submitted at any time
 * from any thread.  Each is admitted in arrival order as soon as its device
 * footprint (the solver's memory plan) fits in the budget next to the
 * requests already running, and runs on one of max_active worker threads
 * with its own HIP stream, so the work of concurrent requests overlaps on the
 * device.  A request's result is bitwise the same as the same mdwf_solve run
 * alone.  b and x are host canonical fields owned by the caller; they must
 * stay valid until mdwf_server_wait returns for the request. */
typedef struct mdwf_server mdwf_server;

/* mem_budget: device bytes the requests may occupy together (0 = 90 % of the
 * free memory now); resident links are taken out of it.  ERR_ARG if
 * max_active < 1, ERR_HIP on a bad device. */
mdwf_status mdwf_server_create(int hip_device, size_t mem_budget, int max_active, mdwf_server **out);

/* Finish every submitted request, stop the workers and free everything. */
void mdwf_server_destroy(mdwf_server *srv);

/* Description of the last failure reported by the server. */
const char *mdwf_server_last_error(const mdwf_server *srv);

/* Upload a gauge field (host canonical, as mdwf_load_gauge); *field_id
 * names it in requests.  Its resident links come out of the budget: queued
 * requests are re-split into sub-batches that fit the smaller budget, and a
 * queued request of which not even one RHS fits any more ends at once with
 * ERR_OOM (its mdwf_server_wait returns that status). */
mdwf_status mdwf_server_add_field(mdwf_server *srv, const mdwf_geometry *geom, const double *U, int *field_id);

/* Queue a solve of nrhs RHS on field_id with action act (mq: per-RHS masses
 * or NULL for act->mq; opts NULL = defaults; use_graph and profile_iters are
 * ignored; max_seconds > 0 is the request's time limit from the moment it
 * starts running, across its sub-batches).  Returns at once with *req_id.
 * A request whose footprint exceeds the budget is split into sub-batches of
 * the most RHS that fit, solved one after another (bitwise the same
 * results).  When a worker takes the request at the head of the queue, the
 * queued requests that can share its solve (same field, L5, M5, b5, c5 and
 * solver options, none split) join it while the combined footprint fits, up
 * to 24 RHS: their RHS then share every operator launch and its link loads,
 * each with its own mass, and each request's results are still bitwise
 * those of the same request solved alone (info.launch_rhs tells how many RHS
 * shared the launches).  ERR_ARG on bad arguments, ERR_OOM if not even one
 * RHS fits the budget. */
mdwf_status mdwf_server_submit(mdwf_server *srv, int field_id, const mdwf_action *act, int nrhs,
                               const double *const *b, double *const *x, const double *mq,
                               const mdwf_solver_opts *opts, int *req_id);

/* Queue the point-source propagator solves of mdwf_solve_point on field_id:
 * ncols columns (cols: spin-colour indices, NULL = 0..ncols-1) of a unit
 * point source at site[4], generated on the device; q[k] receives the
 * wall field of column k (host canonical 4D, valid until mdwf_server_wait
 * returns).  No 5D field crosses the host, so a request costs its solver
 * state on the device and 4D fields on the host.  Admitted, split and
 * shared like mdwf_server_submit (point requests share solves with point
 * requests).  ERR_ARG on bad arguments, ERR_OOM if not even one RHS fits. */
mdwf_status mdwf_server_submit_point(mdwf_server *srv, int field_id, const mdwf_action *act, const int *site,
                                     int ncols, const int *cols, const double *mq, const mdwf_solver_opts *opts,
                                     double *const *q, int *req_id);

/* Block until request req_id has finished; fill info[nrhs] (may be NULL) and
 * times[3] (may be NULL): seconds queued, seconds running, total latency.
 * Returns the solve's status; the request is forgotten afterwards. */
mdwf_status mdwf_server_wait(mdwf_server *srv, int req_id, mdwf_solve_info *info, double *times);

/* Budget, the largest footprint reserved at once so far, and requests queued. */
mdwf_status mdwf_server_stats(mdwf_server *srv, size_t *budget, size_t *peak_reserved, int *queued);

#ifdef __cplusplus
}
#endif

#endif /* MDWF_H */
