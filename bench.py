#!/usr/bin/env python3
"""Benchmark of the Moebius domain-wall solve on one MI355X.

Workload (the paper's a12m310-volume ensemble shape, Table I; action values
M5 = 1.3, b5 = 1.5, c5 = 0.5): 24^3 x 64 lattice, L5 = 8, m_q = 0.0102,
smooth random SU(3) links exp(i 0.25 H) (average plaquette ~0.65, standing in
for the gradient-flowed HISQ ensembles that are not available), and a point
source at a seeded site whose 12 spin-colour columns form the right-hand
sides.

One step = one pass of the whole hot path: source preparation, the
mixed-precision CG on the normal equations of the even-odd Schur operator for
all 12 columns in one multi-RHS launch (fused hop kernels, reductions,
precision conversions, FP64 reliable updates), odd-site reconstruction and the
FP64 true-residual check of every column to 1e-10.  By default the CG runs on
S B^-1 (right preconditioning by B = b5 + c5 C, --schur-form rp); the plain
FP64 CG it is compared with runs on S (--fp64-form asym).

value = algorithmic HBM bytes of the step (model of every kernel it ran) /
step time, in GB/s.  Inputs are resident in HBM before the timed region.
Beside it: the solve time of plain FP64 CG on the same columns, the dslash
kernels' achieved bandwidth against the 8 TB/s HBM peak (timed with HIP events
on the launch stream), and the FP64 CPU oracle timed on a bounded sample.

--workload batched: the a12m220 volume, 32^3 x 64 at L5 = 10, 36 RHS (the
12 columns at m_q = 0.0074, 0.02, 0.04) as three multi-mass launches of 12.
--workload flow: the Wilson gradient flow of the 24^3 x 64 field to t = 1.
--workload mres: the source and sink side around the headline solve
(Gaussian-smeared point source, Moebius wall sources, m_res correlators).
--summarize: write the rocprofv3 summary of the dominant kernels (no GPU).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# the timed solve's operator launches are timed in every PROFILE_EVERY-th CG
# iteration from the third (at most 64 samples), so they span the solve
PROFILE_EVERY = 8
DIMS = (24, 24, 24, 64)
L5 = 8
ACTION = dict(M5=1.3, b5=1.5, c5=0.5, mq=0.0102)
EPS, GAUGE_SEED, SITE_SEED, SRC_SEED = 0.25, 103, 403, 303
MASSES = [0.0102]
GROUPS = 1   # launches per step; the RHS are split evenly over them

# Workloads: "mixed" is the headline one (the a12m310 volume, Table I);
# "batched" is the a12m220 volume (Table I) at L5 = 10 with the 12 columns of
# one point source at three masses, 36 RHS.  Its canonical FP64 solutions
# (4 GB each) cannot all stay in HBM beside the solver state, so the step is
# three multi-mass launches of 12 RHS (4 columns x 3 masses each), every
# input and output resident in HBM.
WORKLOADS = {
    "mixed": dict(DIMS=(24, 24, 24, 64), L5=8, MASSES=[0.0102], GAUGE_SEED=103, SITE_SEED=403, GROUPS=1),
    "batched": dict(DIMS=(32, 32, 32, 64), L5=10, MASSES=[0.0074, 0.02, 0.04], GAUGE_SEED=104, SITE_SEED=404,
                    GROUPS=3),
    # the a15m310 volume and mass (Table I, Table III): plain FP64 CG on one
    # Gaussian source, with the dslash bandwidth of each precision
    "fp64": dict(DIMS=(16, 16, 16, 48), L5=12, MASSES=[0.0158], GAUGE_SEED=102, SITE_SEED=None, SRC_SEED=302,
                 GROUPS=1),
    "serving": None,   # its own driver, serve_main
    "flow": None,      # its own driver, flow_main
    "mres": None,      # its own driver, mres_main
}

# Serving: four resident gauge fields shaped like the paper's ensembles
# (Table I): (lattice, L5, gauge seed, point-source site seed).  Requests draw
# a field, 1..n RHS (spin-colour columns of that field's point source) and a
# mass per RHS.  A 48^3 x 64 x 10 FP64 field is 13.6 GB of host memory, for the
# source and for the solution of every RHS, so requests on it carry 1..2 RHS.
SERVE_FIELDS = [((16, 16, 16, 48), 12, 201, 401), ((24, 24, 24, 64), 8, 202, 402),
                ((32, 32, 32, 64), 10, 203, 403), ((48, 48, 48, 64), 10, 204, 404)]
SERVE_MASSES = (0.0048, 0.0102, 0.02)
SERVE_WEIGHTS = (0.35, 0.3, 0.2, 0.15)
SERVE_MAX_RHS = (12, 12, 12, 12)
ARRIVAL_SEED = 501
FORMS = {"asym": 0, "sym": 1, "rp": 2}
FORM_NAMES = {"asym": "asymmetric", "sym": "symmetric", "rp": "right-B-preconditioned"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_apply(M, torch, ctx, op, prec, reps, warm=5):
    """Average duration of one mdwf_apply_dev(op) on torch's current stream."""
    kin, kout = M.OP_KINDS[op]
    nb_in = M.mdwf_field_bytes(ctx, prec, kin)
    nb_out = M.mdwf_field_bytes(ctx, prec, kout)
    dev = torch.device("cuda:0")
    a = torch.empty(nb_in, dtype=torch.uint8, device=dev)
    b = torch.empty(nb_out, dtype=torch.uint8, device=dev)
    # a valid field: pack a Gaussian canonical half/full field
    X, Y, Z, T = DIMS
    nsites = X * Y * Z * T * L5 // (1 if kin == M.MDWF_FULL else 2)
    g = torch.Generator(device=dev)
    g.manual_seed(SRC_SEED)
    canon = torch.randn(nsites * 24, dtype=torch.float64, device=dev, generator=g)
    st = torch.cuda.current_stream().cuda_stream
    M.mdwf_pack_dev(ctx, prec, kin, canon.data_ptr(), a.data_ptr(), st)
    del canon
    for _ in range(warm):
        M.mdwf_apply_dev(ctx, op, prec, a.data_ptr(), b.data_ptr(), st)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        M.mdwf_apply_dev(ctx, op, prec, a.data_ptr(), b.data_ptr(), st)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops, bytes_ = M.mdwf_op_model(ctx, op, prec)
    return dict(ms=ms, GBps=bytes_ / (ms * 1e-3) / 1e9, GFLOPs=flops / (ms * 1e-3) / 1e9,
                model_bytes=bytes_, model_flops=flops)


def host_cpu_info():
    """The host's CPU model and the threads the oracle may use: the CPU share
    given to this process (OMP_NUM_THREADS when set, else its affinity)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        aff = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        aff = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = int(omp) if omp.isdigit() and int(omp) > 0 else aff
    return dict(model=model, nproc=os.cpu_count(), affinity=aff, threads=max(1, min(threads, aff)))


def _timed(f, *a):
    t0 = time.perf_counter()
    r = f(*a)
    return r, time.perf_counter() - t0


def cpu_baseline(U, dims, L5_, act_kw, fp64_iters=None, ncols=1, check=None):
    """The FP64 oracle (plain C, as it stands) on the host cores, in the same
    run: its Schur operator on the workload's lattice on one thread and on all
    the threads the host gives this process (the OpenMP timing build of the
    same source), one D5 and one CG iteration on all threads, and the
    CPU-sized configuration (4^3 x 8, L5 = 8, m_q = 0.05) solved to 1e-10 on
    both.  value = algorithmic GB/s of the all-threads Schur application (the
    GPU kernels' byte model).  With fp64_iters, the oracle's FP64 CG time to
    solution on the workload is extrapolated from its iteration time and the
    GPU FP64 CG's iteration counts (labelled as such).  check = (b, x) of a
    GPU solution: the oracle's D5 gives its true residual."""
    import oracle
    from paper_1701_07559_amd import inputs as I
    info = host_cpu_info()
    nt = info["threads"]
    act = oracle.Action(dims, L5_, **act_kw)
    rng = np.random.default_rng(SRC_SEED)
    psi = rng.standard_normal(act.shape5) + 1j * rng.standard_normal(act.shape5)
    X, Y, Z, T = dims
    Vh = X * Y * Z * T * L5_ // 2
    schur_bytes = Vh * ((120 + 288 / L5_) * 8)   # the same algorithmic model as the GPU kernels
    out = dict(kind="oracle", unit="GB/s", cpu_model=info["model"], nproc=info["nproc"],
               affinity=info["affinity"])
    try:
        oracle.use_threads(1)
        _, t1 = _timed(oracle.schur, act, U, psi)
        nt = oracle.use_threads(nt) if nt > 1 else 1
        _, tn = _timed(oracle.schur, act, U, psi)
        _, tn2 = _timed(oracle.schur, act, U, psi)
        tn = min(tn, tn2)
        _, td5 = _timed(oracle.D5, act, U, psi)
        # one CG iteration of the oracle's solve (S, S^+, vector updates)
        x = np.zeros_like(psi)
        r = psi.copy()
        sv = oracle.schur(act, U, r, dag=True)
        pv = sv.copy()
        q = np.zeros_like(psi)
        gam = float(np.vdot(sv, sv).real)
        _, tit = _timed(oracle.cgls_step, act, U, x, r, pv, sv, q, gam)
        del x, r, sv, pv, q
        oracle_resid = None
        if check is not None:
            oracle_resid, tchk = _timed(oracle.true_residual, act, U, check[0], check[1])
        # the CPU-sized configuration, whole solve
        a1 = oracle.Action((4, 4, 4, 8), 8, M5=1.3, b5=1.5, c5=0.5, mq=0.05)
        U1 = I.random_links((4, 4, 4, 8), 0.3, 101)
        b1 = I.gaussian_source((4, 4, 4, 8), 8, 301)
        (_, i1n), ts1n = _timed(oracle.solve, a1, U1, b1)
        oracle.use_threads(1)
        (_, i11), ts11 = _timed(oracle.solve, a1, U1, b1)
    finally:
        oracle.use_threads(1)
    out.update(value=round(schur_bytes / tn / 1e9, 4), cores=nt,
               sample="FP64 oracle on %dx%dx%dx%d L5=%d: Schur application %.2f s on %d threads (best of 2), "
                      "%.2f s on 1 thread; D5 %.2f s and one CG iteration %.2f s on %d threads; 4^3x8 L5=8 "
                      "solve to 1e-10 (%d iterations) %.3f s on %d threads, %.3f s on 1" %
                      (X, Y, Z, T, L5_, tn, nt, t1, td5, tit, nt, i1n["iters"], ts1n, nt, ts11),
               single_thread=dict(value=round(schur_bytes / t1 / 1e9, 4), unit="GB/s", cores=1,
                                  schur_s=round(t1, 3)),
               schur_s=round(tn, 3), d5_s=round(td5, 3), cg_iteration_s=round(tit, 3),
               config1_solve=dict(dims=[4, 4, 4, 8], L5=8, iters=i1n["iters"], true_resid=i1n["true_resid"],
                                  seconds_all_threads=round(ts1n, 4), seconds_1_thread=round(ts11, 4)))
    if fp64_iters:
        secs = tit * float(np.sum(fp64_iters)) * (ncols / len(fp64_iters))
        out["time_to_solution_extrapolated"] = dict(
            seconds=round(secs, 1), threads=nt,
            note="extrapolated: oracle CG iteration time x the GPU FP64 CG iteration counts, %d columns" % ncols)
    if oracle_resid is not None:
        out["oracle_true_resid_of_gpu_solution"] = oracle_resid
        out["oracle_check_s"] = round(tchk, 2)
    return out


def hop_launch_bytes(inner, Vh, nr):
    """Algorithmic HBM bytes of one batched launch of kernels A, B, A^+, B^+
    for nr right-hand sides: each spinor field read or written once per RHS
    (FP16: 2-byte reals plus a 4-byte norm per 5D site), the links of the
    launch once (144 reals per 4D site: 8 links of 18 reals)."""
    w, nrm = {"f16": (2, 4), "f32": (4, 0), "f64": (8, 0)}[inner]
    links = Vh * 144 * w / L5
    a = Vh * nr * (48 * w + 2 * nrm) + links        # in psi, out t
    b_ = Vh * nr * (72 * w + 3 * nrm) + links       # in t, centre psi, out
    return [a, b_, a, b_]


# What the counters show limits the hop kernels below the HBM roofline
# (rocprofv3 summaries under profiles/).
LIMITER = {
    "f16": "co-limited: texture addresser 94-97% busy on 56-61 load instructions per wave "
           "(profiles/hop_ta_busy_24c64_L8_12rhs.md) and VALU 89% busy in kernels A / A_dag, 73-76% in B / B_dag "
           "(profiles/hop_valu_busy_24c64_L8.md), moving 5.9-6.7 TB/s beyond L2, 2.2x the algorithmic bytes "
           "(profiles/schur_rp_f16_24c64_L8_12rhs_counters.md)",
    "f32": "re-reads of the input field beyond L2 (2.26x) at a rate near the streaming limit "
           "(profiles/hop_f32_plane_24c64_L8_counters.md)",
    "f64": "re-reads of the input field beyond L2 (1.75-2.5x) at 5.3-6.6 TB/s "
           "(profiles/hop_f64_24c64_L8_counters.md)",
}

# Vector-ALU roofline of the FP16-storage hop kernels, which the counters show
# issue-bound.  Per 5D site and RHS the model flops of kernel A / B of the
# CG operator are 1320 + 48 L5 (+ 48 for B's combination).  The fewest gfx950
# VALU instructions that execute them, without packed FP32: the eight SU(3)
# products (8 x 132 flops) as v_dot2_f32_f16 at 4 flops per lane, the eight
# projections (8 x 12) as packed-half adds at 2, the sum over directions
# (168) as FP32 adds at 1, the dense fifth-dimension polynomial (48 L5) and
# B's combination (48) as FP32 FMAs at 2.  One VALU instruction per lane and
# cycle on 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz then gives the peak flop
# rate of this instruction mix.
VALU_LANE_RATE = 256 * 4 * 16 * 2.4e9


def alu_peak_tflops(l5):
    flops = (1320 + 48 * l5) + (1320 + 48 * l5 + 48)
    instr = 2 * (1056 / 4 + 96 / 2 + 168) + 2 * (48 * l5 / 2) + 48 / 2
    return flops / instr * VALU_LANE_RATE / 1e12


def hop_launch_flops(Vh, nr, form):
    """Model flops of one batched launch of kernel A and of kernel B."""
    a = 1320 + 48 * L5 + (72 if form != "rp" else 0)
    b = 1320 + 48 * L5 + 48 if form == "rp" else 1320 + 72 + 48
    return [Vh * nr * a, Vh * nr * b]


def roofline(info, inner, Vh, form):
    """Dominant kernels of the step: the batched CG operator (S, K5^-1 S or
    S B^-1) = kernel A then kernel B, as launched inside the timed solve
    (durations from HIP events the library records on its launch stream)."""
    us, nr = info.get("hop_us"), info.get("hop_rhs", 0)
    if not us or nr <= 0 or us[0] <= 0:
        return None
    by = hop_launch_bytes(inner, Vh, nr)
    ach = (by[0] + by[1]) / ((us[0] + us[1]) * 1e-6) / 1e9
    names = ("A", "B", "A_dag", "B_dag")
    kernel = ("%s Schur operator: k_hop<%s, %d> (kernel A) + k_hop<%s, %d> (kernel B), %d RHS per "
              "launch, mean of %d CG iterations sampled every %d across the solve" %
              (FORM_NAMES[form], inner.upper(), FORM_KINDS[form][0], inner.upper(), FORM_KINDS[form][1],
               nr, info["hop_samples"], PROFILE_EVERY))
    launches = {n: dict(us=round(u, 1), algorithmic_bytes=int(b), GBps=round(b / (u * 1e-6) / 1e9, 1))
                for n, u, b in zip(names, us, by)}
    hbm = dict(achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s", frac=round(ach / HBM_PEAK_GBS, 4))
    if inner == "f16" and form == "rp":
        # issue-bound (VALU busy 73-90 %): priced against the vector ALUs,
        # the HBM fraction kept beside it
        fl = hop_launch_flops(Vh, nr, form)
        tf = (fl[0] + fl[1]) / ((us[0] + us[1]) * 1e-6) / 1e12
        pk = alu_peak_tflops(L5)
        return dict(bound="alu", kernel=kernel, achieved=round(tf, 2), peak=round(pk, 1), unit="TFLOP/s",
                    frac=round(tf / pk, 4),
                    peak_derivation="model flops of kernels A+B over the fewest VALU instructions that execute "
                                    "them (SU(3) products as v_dot2_f32_f16, FP32 sums, packed-half projections), "
                                    "one VALU instruction per lane and cycle, 256 CUs x 64 lanes x 2.4 GHz",
                    frac_of_fp32_vector_peak=round(tf / 157.3, 4),
                    traffic=None, hbm=hbm, limiter=LIMITER.get(inner), launches=launches)
    return dict(bound="hbm", kernel=kernel, traffic=None, limiter=LIMITER.get(inner), launches=launches, **hbm)


_PKG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1701_07559_amd")
# what decides the hop kernels' machine code: their source, the shared
# device header and the compiler flags
KERNEL_SRC = os.path.join(_PKG, "csrc", "dslash.hip")
KERNEL_DEPS = [KERNEL_SRC, os.path.join(_PKG, "csrc", "hop_device.h"), os.path.join(_PKG, "csrc", "mdwf_internal.h")]
TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                            "schur_rp_f16_24c64_L8_12rhs_counters.md")
# hop kinds (HopKind) of kernels A, B, A^+, B^+ of each CG operator
FORM_KINDS = {"asym": (3, 4, 5, 6), "sym": (3, 9, 5, 6), "rp": (10, 11, 5, 12)}


def kernel_sha():
    """Digest of the hop kernels' source, the shared device header and the
    compiler flags: a stored counter record applies only while it matches."""
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_DEPS:
        with open(path, "rb") as f:
            h.update(f.read())
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_1701_07559_amd import build as B
    h.update(" ".join(B.HIPCC_FLAGS).encode())
    return h.hexdigest()


def stored_traffic(form):
    """Per-launch HBM traffic of the batched FP16 CG-operator launches
    (kernels A + B) recorded by a counter run, if the hop source is unchanged
    since and the run used the same Schur form."""
    try:
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if line.startswith("traffic-record: "):
                    rec = json.loads(line[len("traffic-record: "):])
                    if rec.get("dslash_sha256") == kernel_sha() and rec.get("form") == form:
                        return rec
    except OSError:
        pass
    return None


def _kernel_label(name):
    import re
    n = re.sub(r"\(mdwf::Geo.*", "", name).replace("void ", "")
    return n.replace("(mdwf::Prec)0", "F64").replace("(mdwf::Prec)1", "F32").replace("(mdwf::Prec)2", "F16")


def summarize(args):
    """Markdown summary of rocprofv3 databases: kernel-trace statistics, the
    12-RHS kernel A / B launches of the solve (selected by grid size), and
    FETCH_SIZE / WRITE_SIZE per launch calibrated on the 1 GiB copy."""
    import collections
    import sqlite3
    X, Y, Z, T = DIMS
    Vh4 = X * Y * Z * T // 2
    Vh = Vh4 * L5
    nblk = (Vh4 + 4 * (64 // L5) - 1) // (4 * (64 // L5))
    grid12 = nblk * 12 * 256
    lines = []
    cmds = [c for c in args.summary_cmds.split("||") if c.strip()]
    form = args.schur_form
    kinds = FORM_KINDS[form]
    names = dict(zip(kinds, ("A", "B", "A_dag", "B_dag")))
    lines.append("# rocprofv3 summary: batched FP16 %s Schur operator in bench.py (24^3x64, L5=8, 12 RHS)" %
                 FORM_NAMES[form])
    lines.append("")
    lines.append("Commands (from the repository root on one MI355X, with `export TMPDIR=/tmp`):")
    lines.append("")
    for c in cmds:
        lines.append("    " + c.strip())
    lines.append("")
    db = sqlite3.connect(args.summarize[0])
    rows = db.execute("select name, duration, grid_x from kernels").fetchall()
    agg = collections.defaultdict(list)
    for name, dur, gx in rows:
        agg[_kernel_label(name)].append(dur / 1e3)
    tot = sum(sum(v) for v in agg.values())
    lines.append("Kernel trace (all dispatches of the run):")
    lines.append("")
    lines.append("| kernel | calls | total us | average us | % |")
    lines.append("|---|---|---|---|---|")
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:16]:
        lines.append("| `%s` | %d | %.1f | %.2f | %.1f |" % (k[:90], len(v), sum(v), sum(v) / len(v), 100 * sum(v) / tot))
    lines.append("")
    sel = collections.defaultdict(list)
    for name, dur, gx in rows:
        lab = _kernel_label(name)
        if gx == grid12 and lab.startswith("mdwf::k_hop<F16"):
            kind = int(lab.split(",")[1])
            sel[kind].append(dur / 1e3)
    lines.append("12-RHS launches of the solve (grid %d threads):" % grid12)
    lines.append("")
    lines.append("| kernel | launches | average us |")
    lines.append("|---|---|---|")
    for kind in kinds:
        v = sel.get(kind, [])
        if v:
            lines.append("| %s (`k_hop<F16, %d, *>`) | %d | %.1f |" % (names[kind], kind, len(v), sum(v) / len(v)))
    lines.append("")
    if args.summary_bench:
        with open(args.summary_bench) as f:
            bl = [json.loads(x) for x in f if x.startswith("{")]
        la = (bl[-1].get("roofline") or {}).get("launches") if bl else None
        if la:
            tr = {k: sum(sel.get(kind, [0])) / max(1, len(sel.get(kind, [])))
                  for k, kind in (("A", kinds[0]), ("B", kinds[1]))}
            lines.append("Agreement: bench.py in the traced run timed the same launches with HIP events on the "
                         "solve stream (`mdwf_solve_info.hop_us`): A %.1f us, B %.1f us, against %.1f and %.1f us "
                         "in the trace (sum %+.1f %%)." % (la["A"]["us"], la["B"]["us"], tr["A"], tr["B"],
                         100 * ((la["A"]["us"] + la["B"]["us"]) / (tr["A"] + tr["B"]) - 1)))
            lines.append("")
    rec = None
    if args.summarize[1] != "-" and args.summarize[2] != "-":
        def counters(path, cname):
            d = sqlite3.connect(path)
            out = collections.defaultdict(list)
            for kn, gsz, val in d.execute("select kernel_name, grid_size, value from counters_collection "
                                         "where counter_name = ?", (cname,)):
                lab = _kernel_label(kn)
                if gsz == grid12 and lab.startswith("mdwf::k_hop<F16"):
                    out[int(lab.split(",")[1])].append(val)
                elif "copybuffer" in lab.lower():
                    out["copy"].append(val)   # the largest is the 1 GiB calibration copy
            return out
        fe = counters(args.summarize[1], "FETCH_SIZE")
        wr = counters(args.summarize[2], "WRITE_SIZE")
        gib = float(1 << 30)
        f_r = gib / (max(fe["copy"]) * 1024.0)
        f_w = gib / (max(wr["copy"]) * 1024.0)
        lines.append("Counters (KiB per dispatch; calibration: the 1 GiB device copy reads %.3f GiB by "
                     "FETCH_SIZE and writes %.3f GiB by WRITE_SIZE, so FETCH_SIZE is scaled by %.3f and "
                     "WRITE_SIZE by %.3f):" % (1 / f_r, 1 / f_w, f_r, f_w))
        lines.append("")
        lines.append("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) |")
        lines.append("|---|---|---|---|")
        per = {}
        for kind in kinds:
            if fe.get(kind) and wr.get(kind):
                fk = sum(fe[kind]) / len(fe[kind])
                wk = sum(wr[kind]) / len(wr[kind])
                per[kind] = fk * 1024 * f_r + wk * 1024 * f_w
                lines.append("| %s | %.0f | %.0f | %.4g |" % (names[kind], fk, wk, per[kind]))
        lines.append("")
        if kinds[0] in per and kinds[1] in per:
            rec = dict(traffic_bytes_per_launch=per[kinds[0]] + per[kinds[1]], kernels="A+B, 12 RHS, FP16",
                       form=form, fetch_scale=round(f_r, 4), write_scale=round(f_w, 4), dslash_sha256=kernel_sha())
            lines.append("HBM traffic of one batched operator application (kernels A + B): %.4g bytes." %
                         rec["traffic_bytes_per_launch"])
            lines.append("")
            lines.append("traffic-record: " + json.dumps(rec))
    text = "\n".join(lines) + "\n"
    if args.summary_out:
        with open(args.summary_out, "w") as f:
            f.write(text)
    print(text)


def pmc_summary(args):
    """Markdown summary of a rocprofv3 counter database with SQ_ACTIVE_INST_VALU,
    SQ_ACTIVE_INST_LDS and GRBM_GUI_ACTIVE: per kernel and grid, the share of
    the dispatch time the vector ALUs (and LDS) were busy, rocprofv3's
    VALUBusy = 100 sum(SQ_ACTIVE_INST_VALU) / CU_NUM / max(GRBM_GUI_ACTIVE).
    The database holds each counter summed over its dimensions, so the
    per-XCD maximum of GRBM_GUI_ACTIVE is taken as that sum / 8 XCDs (the
    XCDs run the dispatch side by side)."""
    import collections
    import sqlite3
    cu_num, n_xcd = 256, 8
    db = sqlite3.connect(args.pmc_summary)
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    meta = {}
    for did, kn, gs, cn, v in db.execute("select dispatch_id, kernel_name, grid_size, counter_name, value "
                                         "from counters_collection"):
        per[did][cn].append(v)
        meta[did] = (_kernel_label(kn), gs)
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for did, cs in per.items():
        if "GRBM_GUI_ACTIVE" not in cs or "SQ_ACTIVE_INST_VALU" not in cs:
            continue
        g = sum(cs["GRBM_GUI_ACTIVE"]) / n_xcd
        if g <= 0:
            continue
        key = meta[did]
        agg[key]["valu"].append(100.0 * sum(cs["SQ_ACTIVE_INST_VALU"]) / cu_num / g)
        if "SQ_ACTIVE_INST_LDS" in cs:
            agg[key]["lds"].append(100.0 * sum(cs["SQ_ACTIVE_INST_LDS"]) / cu_num / g)
        if "SQ_INSTS_VALU" in cs and sum(cs.get("SQ_WAVES", [0])) > 0:
            agg[key]["ipw"].append(sum(cs["SQ_INSTS_VALU"]) / sum(cs["SQ_WAVES"]))
    lines = ["# rocprofv3 counters: vector ALU and LDS busy share of the hop and CG kernels", "",
             "Commands (from the repository root on one MI355X, with `export TMPDIR=/tmp`):", ""]
    lines += ["    " + c.strip() for c in args.summary_cmds.split("||") if c.strip()]
    lines += ["", "VALU busy = 100 sum(SQ_ACTIVE_INST_VALU) / 256 CUs / GRBM_GUI_ACTIVE per XCD, per dispatch "
              "(rocprofv3's VALUBusy; the database sums GRBM_GUI_ACTIVE over the 8 XCDs, divided back "
              "here), LDS busy likewise from SQ_ACTIVE_INST_LDS; means over the dispatches of each "
              "kernel and grid.", "",
              "VALU instructions per wave = SQ_INSTS_VALU / SQ_WAVES (a wave covers 64 lanes: 64 / L5 "
              "sites of the hop kernels, 64 sites of the vector kernels).", "",
              "| kernel | grid (threads) | dispatches | VALU busy % | LDS busy % | VALU instr. per wave |",
              "|---|---|---|---|---|---|"]
    rows = sorted(agg.items(), key=lambda kv: -len(kv[1]["valu"]))
    for (name, gs), d in rows:
        if not (name.startswith("mdwf::k_hop") or name.startswith("mdwf::k_cg")):
            continue
        lds = "%.1f" % (sum(d["lds"]) / len(d["lds"])) if d["lds"] else "-"
        ipw = "%.0f" % (sum(d["ipw"]) / len(d["ipw"])) if d["ipw"] else "-"
        lines.append("| `%s` | %d | %d | %.1f | %s | %s |" % (name, gs, len(d["valu"]),
                                                               sum(d["valu"]) / len(d["valu"]), lds, ipw))
    text = "\n".join(lines) + "\n"
    if args.summary_out:
        with open(args.summary_out, "w") as f:
            f.write(text)
    print(text)


# Gradient flow model per link and Runge-Kutta stage: 26 products of 3x3
# complex matrices (12 for the six staples, one for the link times their sum,
# 12 for the degree-12 Taylor exponential, one for the update; 216 flops each)
# and, in FP64, the input link and the output link read / written once (144 B
# each) and the exponent accumulator, eight reals (64 B), read and written
# (written only by the first stage).
FLOW_FLOPS_PER_LINK = 26 * 216
FLOW_BYTES_PER_LINK = ((144 + 144 + 64) + 2 * (144 + 144 + 64 + 64)) / 3.0


def flow_main(args):
    """Flow workload: the 24^3 x 64 exp(i 0.25 H) field flowed to t_gf = 1
    (the paper's flow time) in steps of 0.01, on the device."""
    import torch
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_1701_07559_amd import inputs as I
    from paper_1701_07559_amd import mdwf as M
    dims, eps, nsteps = (24, 24, 24, 64), 0.01, 100
    log("generating links", dims)
    U = I.random_links(dims, EPS, GAUGE_SEED)
    dev = torch.device("cuda:0")
    work = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(work)
    U0 = torch.from_numpy(U.view(np.float64).copy()).to(dev)
    Ud = torch.empty_like(U0)
    stream = work.cuda_stream
    nlinks = 4 * int(np.prod(dims))
    for w in range(args.warmup):
        Ud.copy_(U0)
        M.mdwf_wilson_flow_dev(dims, Ud.data_ptr(), eps, 2, stream, plaquette=False)
    times, kern = [], []
    plaq = None
    for k in range(args.steps):
        Ud.copy_(U0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(work)
        M.mdwf_wilson_flow_dev(dims, Ud.data_ptr(), eps, nsteps, stream, plaquette=False)   # stage kernels only
        e1.record(work)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        kern.append(e0.elapsed_time(e1) * 1e3 / (3 * nsteps))
        log("flow to t=%.2f: %.3f s, %.1f us per stage" % (eps * nsteps, times[-1], kern[-1]))
    p0 = M.mdwf_plaquette_dev(dims, U0.data_ptr(), stream)
    p1 = M.mdwf_plaquette_dev(dims, Ud.data_ptr(), stream)
    ms = 1e3 * float(np.mean(times))
    stage_us = float(np.mean(kern))
    bytes_step = FLOW_BYTES_PER_LINK * nlinks * 3 * nsteps
    flops_stage = FLOW_FLOPS_PER_LINK * nlinks
    value = bytes_step / (ms * 1e-3) / 1e9
    achieved = flops_stage / (stage_us * 1e-6) / 1e12
    cpu = None
    if not args.no_cpu:
        from oracle import flow as F
        small = (8, 8, 8, 16)
        Us = I.random_links(small, EPS, GAUGE_SEED)
        t0 = time.perf_counter()
        n = 0
        while True:
            Us = F.flow_step(Us, eps)
            n += 1
            if time.perf_counter() - t0 > 12.0 or n >= 4:
                break
        dt = (time.perf_counter() - t0) / n
        nl = 4 * int(np.prod(small))
        cpu = dict(value=round(FLOW_BYTES_PER_LINK * nl * 3 / dt / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                   sample="%d FP64 Runge-Kutta flow steps of the numpy oracle on 8^3x16 (%.2f s each), the same "
                          "per-link byte model" % (n, dt))
    out = {
        "metric": "Moebius DWF dslash GB/s (% HBM peak); time to r=1e-10 solve, mixed vs FP64",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Wilson gradient flow of the 24x24x24x64 exp(i0.25H) gauge field to t_gf = 1 "
                               "(%d Runge-Kutta steps of %g), FP64" % (nsteps, eps),
                   "name": "flow", "lattice": list(dims), "eps": eps, "nsteps": nsteps},
        "flow": {"plaquette_before": p0, "plaquette_after": p1, "seconds": round(ms / 1e3, 4),
                 "stage_us": round(stage_us, 1)},
        "roofline": {"bound": "alu", "kernel": "k_flow_stage (one Runge-Kutta stage, FP64)",
                     "achieved": round(achieved, 2), "peak": 78.6, "unit": "TFLOP/s",
                     "frac": round(achieved / 78.6, 4), "traffic": None,
                     "model": "26 complex 3x3 products per link and stage (216 flops each)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def serve_requests(n, rng):
    """n requests of the serving mix: (field index, RHS count, mass per RHS)."""
    out = []
    for _ in range(n):
        f = int(rng.choice(len(SERVE_FIELDS), p=SERVE_WEIGHTS))
        k = int(rng.integers(1, SERVE_MAX_RHS[f] + 1))
        out.append((f, k, [float(SERVE_MASSES[j]) for j in rng.integers(0, len(SERVE_MASSES), size=k)]))
    return out


def _digest(a):
    try:
        import xxhash
        return xxhash.xxh3_64_hexdigest(memoryview(a).cast("B"))
    except ImportError:
        import hashlib
        return hashlib.blake2b(memoryview(a).cast("B"), digest_size=16).hexdigest()


def run_phase(M, srv, fids, sites, qshapes, reqs, arrivals, opts, host_cap, serial=False, digest=True):
    """Submit reqs at the given arrival offsets (s) while a waiter thread
    collects them in submission order.  A request of k RHS solves the
    spin-colour columns 0..k-1 of its field's point source at sites[f]; the
    server generates the sources on the device and returns the 4D wall
    fields (shape qshapes[f]), which are hashed (digest) and freed once the
    request is collected.  Outstanding output memory on the host is bounded
    by host_cap bytes (a submission past it waits, and the wait is
    recorded).  serial: submit each request only after the previous one
    finished (no overlap).  Returns (records, wall seconds from the first
    submission to the last completion the server recorded)."""
    import threading
    cv = threading.Condition()
    queue, recs = [], [None] * len(reqs)
    state = dict(out=0, closed=False, done=0)

    def waiter():
        i = 0
        while True:
            with cv:
                cv.wait_for(lambda: i < len(queue) or state["closed"])
                if i >= len(queue):
                    return
                rid, idx, xs, nbytes, held, t_sub = queue[i]
            i += 1
            st, info, times = srv.wait(rid)
            log("request %d: status %d, %d RHS, latency %.2f s" % (idx, st, len(info), times[2]))
            recs[idx] = dict(status=st, info=info, times=times, held=held, t_end=t_sub + times[2],
                             digest=[_digest(x) for x in xs] if digest else None)
            xs.clear()
            with cv:
                state["out"] -= nbytes
                state["done"] += 1
                cv.notify_all()

    th = threading.Thread(target=waiter, daemon=True)
    th.start()
    t0 = time.perf_counter()
    for idx, ((f, k, masses), ta) in enumerate(zip(reqs, arrivals)):
        delay = ta - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        l5 = SERVE_FIELDS[f][1]
        nbytes = k * int(np.prod(qshapes[f])) * 16
        with cv:
            if serial:
                cv.wait_for(lambda: state["done"] == idx)
            t_ready = time.perf_counter()
            cv.wait_for(lambda: state["out"] == 0 or state["out"] + nbytes <= host_cap)
            state["out"] += nbytes
        held = time.perf_counter() - t_ready
        xs = [np.empty(qshapes[f], complex) for _ in range(k)]
        t_sub = time.perf_counter() - t0
        rid = srv.submit_point(fids[f], ACTION["M5"], ACTION["b5"], ACTION["c5"], masses[0], l5, sites[f],
                               list(range(k)), xs, masses=masses, opts=opts)
        with cv:
            queue.append((rid, idx, xs, nbytes, held, t_sub))
            cv.notify_all()
        del xs
    with cv:
        state["closed"] = True
        cv.notify_all()
    th.join()
    return recs, max(r["t_end"] for r in recs)


def serve_work(req):
    """Work of a request in RHS x 5D sites (the Poisson rate is set in it)."""
    f, k, _ = req
    dims, l5 = SERVE_FIELDS[f][0], SERVE_FIELDS[f][1]
    return k * float(np.prod(dims)) * l5


def phase_summary(reqs, recs, wall):
    lat = np.array([r["times"][2] for r in recs])
    nrhs = sum(k for _, k, _ in reqs)
    by = {}
    for (f, k, _), r in zip(reqs, recs):
        by.setdefault("%dx%dx%dx%d L5=%d" % (tuple(SERVE_FIELDS[f][0]) + (SERVE_FIELDS[f][1],)), []).append(
            r["times"][2])
    return dict(by_lattice={n: dict(requests=len(v), p50_latency_s=round(float(np.percentile(v, 50)), 3))
                            for n, v in sorted(by.items())},
                requests=len(reqs), rhs=nrhs, wall_s=round(wall, 3),
                solves_per_s=round(len(reqs) / wall, 4), rhs_solves_per_s=round(nrhs / wall, 3),
                p50_latency_s=round(float(np.percentile(lat, 50)), 3),
                p99_latency_s=round(float(np.percentile(lat, 99)), 3),
                mean_queued_s=round(float(np.mean([r["times"][0] for r in recs])), 3),
                host_cap_wait_s=round(float(sum(r["held"] for r in recs)), 3),
                # RHS per operator launch, averaged over RHS (more than the
                # request's own when it shared a solve with queued requests)
                mean_launch_rhs=round(float(np.mean([i.get("launch_rhs", 0) for r in recs for i in r["info"]])), 2),
                shared_requests=sum(1 for (_, k, _), r in zip(reqs, recs)
                                    if any(i.get("launch_rhs", 0) > k for i in r["info"])),
                model_GBps=round(sum(i["model_bytes"] for r in recs for i in r["info"]) / wall / 1e9, 1),
                max_true_resid=max(i["true_resid"] for r in recs for i in r["info"]),
                all_ok=all(r["status"] == 0 and all(i["true_resid"] <= 1e-10 for i in r["info"]) for r in recs))


def serve_main(args):
    """Serving workload: a burst of requests (throughput), the same requests
    one at a time (no overlap; also the alone-vs-mix bitwise check), then a
    Poisson stream at a fraction of the measured throughput (latency)."""
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_1701_07559_amd import inputs as I
    # links first, in forked workers, before this process touches the GPU
    workers = max(1, min(16, os.cpu_count() or 1))
    links = []
    for dims, l5, gseed, _ in SERVE_FIELDS:
        t = time.perf_counter()
        links.append(I.random_links(dims, EPS, gseed, workers=workers))
        log("links %s seed %d: %.1f s (%d workers)" % (dims, gseed, time.perf_counter() - t, workers))
    from paper_1701_07559_amd import mdwf as M

    rng = np.random.default_rng(ARRIVAL_SEED)
    burst = serve_requests(args.requests, rng)
    stream = serve_requests(args.poisson_requests, rng)
    gaps = rng.exponential(1.0, size=len(stream))   # unit-rate gaps, scaled once the rate is known
    srv = M.Server(hip_device=0, mem_budget=0, max_active=args.max_active)
    out = None
    try:
        fids = []
        for i, ((dims, l5, _, _), U) in enumerate(zip(SERVE_FIELDS, links)):
            fids.append(srv.add_field(dims, U))
            if i > 0:
                links[i] = None
        sites = [I.random_point_site(dims, sseed) for dims, _, _, sseed in SERVE_FIELDS]
        qshapes = [tuple(reversed(dims)) + (4, 3) for dims, _, _, _ in SERVE_FIELDS]
        st0 = srv.stats()
        log("server: budget %.1f GB after %d resident fields" % (st0["budget"] / 1e9, len(fids)))
        inner = M.MDWF_F16 if args.inner == "f16" else M.MDWF_F32
        opts = dict(tol=1e-10, inner=inner, max_iter=args.max_iter, delta=0.1, schur_form=FORMS[args.schur_form])
        cap = int(args.host_cap_gb * 1e9)
        for f, k, ms in burst:
            log("burst request: %s L5=%d nrhs=%d masses=%s" % (SERVE_FIELDS[f][0], SERVE_FIELDS[f][1], k, ms))

        serial = None
        if not args.no_serial:
            rs, ws = run_phase(M, srv, fids, sites, qshapes, burst, [0.0] * len(burst), opts, cap, serial=True)
            serial = phase_summary(burst, rs, ws)
            log("one at a time: %s" % serial)
        ra, wa = run_phase(M, srv, fids, sites, qshapes, burst, [0.0] * len(burst), opts, cap)
        conc = phase_summary(burst, ra, wa)
        log("burst: %s" % conc)
        same = None
        if serial is not None:
            same = all(a["digest"] == b["digest"] for a, b in zip(ra, rs))
            conc["bitwise_equal_to_one_at_a_time"] = same
            conc["speedup_vs_one_at_a_time"] = round(serial["wall_s"] / wa, 3)
        # offered load: args.load x the burst's throughput in RHS x 5D sites
        rate = args.load * sum(serve_work(q) for q in burst) / wa / np.mean([serve_work(q) for q in stream])
        arrivals = list(np.cumsum(gaps / rate))
        for f, k, ms in stream:
            log("poisson request: %s L5=%d nrhs=%d" % (SERVE_FIELDS[f][0], SERVE_FIELDS[f][1], k))
        rp, wp = run_phase(M, srv, fids, sites, qshapes, stream, arrivals, opts, cap, digest=False)
        pois = phase_summary(stream, rp, wp)
        pois["arrival_rate_per_s"] = round(rate, 4)
        log("poisson: %s" % pois)
        stats = srv.stats()
    finally:
        srv.close()

    cpu = None
    if not args.no_cpu:
        cpu = serve_cpu_baseline(links[0], burst, ra)
    value = conc["model_GBps"]
    out = {
        "metric": "Moebius DWF dslash GB/s (% HBM peak); time to r=1e-10 solve, mixed vs FP64",
        "value": value,
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": round(wa * 1e3, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.inner,
        "data": "synthetic",
        "config": {
            "workload": "serving: %d resident exp(i0.25H) fields %s, M5=1.3 b5=1.5 c5=0.5, m_q per RHS from %s, "
                        "point-source requests (columns 0..k-1 of the field's point source generated on the device, 4D wall fields "
                        "returned), %s inner, %s Schur form, every solve to true residual 1e-10; a burst of %d "
                        "requests (throughput) then %d Poisson arrivals offering %.2f x that throughput in RHS x 5D sites (latency)" %
                        (len(SERVE_FIELDS), ["%dx%dx%dx%d L5=%d" % (tuple(d) + (l5,)) for d, l5, _, _ in SERVE_FIELDS],
                         list(SERVE_MASSES), args.inner, FORM_NAMES[args.schur_form], len(burst), len(stream),
                         args.load),
            "name": "serving", "max_active": args.max_active, "host_cap_gb": args.host_cap_gb,
            "request_seed": ARRIVAL_SEED,
        },
        "serving": dict(burst=conc, one_at_a_time=serial, poisson=pois,
                        budget_bytes=stats["budget"], peak_reserved_bytes=stats["peak_reserved"]),
        "roofline": None,
        "roofline_note": "per-launch timing is off in the server: launches of concurrent requests share the "
                         "device, so one stream's events do not time one kernel",
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def serve_cpu_baseline(U16, burst, recs, budget_s=25.0):
    """The FP64 oracle's Schur operator timed on the 16^3 x 48 x 12 field and
    projected to the burst: two applications (S and S^+) per CG iteration of
    every RHS, at the iteration counts the burst ran, time scaled by the
    5D volume of each request's lattice."""
    import oracle
    dims, l5 = SERVE_FIELDS[0][0], SERVE_FIELDS[0][1]
    act = oracle.Action(dims, l5, M5=ACTION["M5"], b5=ACTION["b5"], c5=ACTION["c5"], mq=SERVE_MASSES[1])
    rng = np.random.default_rng(SRC_SEED)
    psi = rng.standard_normal(act.shape5) + 1j * rng.standard_normal(act.shape5)
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.schur(act, U16, psi)
        n += 1
        if time.perf_counter() - t0 > budget_s * 0.5 or n >= 3:
            break
    dt = (time.perf_counter() - t0) / n
    vol0 = np.prod(dims) * l5
    secs = 0.0
    for (f, k, _), r in zip(burst, recs):
        d, lf = SERVE_FIELDS[f][0], SERVE_FIELDS[f][1]
        secs += sum(i["iters"] for i in r["info"]) * 2 * dt * (np.prod(d) * lf / vol0)
    return dict(value=float("%.4g" % (len(burst) / secs)), unit="solves/s", cores=1, kind="oracle",
                sample="%d FP64 Schur applications on 16^3x48 L5=12 (single thread, %.2f s each), projected "
                       "over the burst's %d requests at their CG iteration counts (2 applications per "
                       "iteration, time proportional to 5D volume)" % (n, dt, len(burst)))


# Source/sink model per 4D site: a Gaussian smearing step reads and writes
# every vector once (192 B each way) and the three spatial links once
# (432 B); the wall source reads a vector and the four links and writes L5
# slices of its 5D field; the correlators read the four slices they use.
SMEAR_SIGMA, SMEAR_ITERS = 4.0, 30


def smear_bytes(V, nvec):
    return V * (nvec * 384.0 + 432.0)


def wall_bytes(V, nvec, L5_):
    return V * (nvec * (192.0 + 192.0 * L5_) + 576.0)


def corr_bytes(V, nvec):
    return V * nvec * 4 * 96.0


def mres_main(args):
    """Source/sink workload: the 12 spin-colour columns of a point source on
    the 24^3 x 64 field, Gaussian-smeared, turned into 5D Moebius sources,
    solved (the headline mixed solve) and contracted into the pseudoscalar
    and midpoint correlators and m_res(t)."""
    import torch
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_1701_07559_amd import inputs as I
    from paper_1701_07559_amd import mdwf as M
    dims, L5_ = DIMS, L5
    X, Y, Z, T = dims
    V = X * Y * Z * T
    act_t = (ACTION["M5"], ACTION["b5"], ACTION["c5"], ACTION["mq"], L5_)
    dev = torch.device("cuda:0")
    work = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(work)
    stream = work.cuda_stream
    log("generating links", dims)
    U = I.random_links(dims, EPS, GAUGE_SEED, workers=8)
    Ud = torch.from_numpy(U.view(np.float64).copy()).to(dev)
    del U
    xs, ys, zs, ts = I.random_point_site(dims, SITE_SEED)
    eta = torch.zeros((12, V * 24), dtype=torch.float64, device=dev)
    for j in range(12):
        eta[j, 2 * ((((ts * Z + zs) * Y + ys) * X + xs) * 12 + j)] = 1.0
    sm = torch.empty_like(eta)
    n5 = L5_ * V * 24
    b = torch.empty((12, n5), dtype=torch.float64, device=dev)
    x = torch.zeros((12, n5), dtype=torch.float64, device=dev)
    ctx = M.mdwf_create(dims, antiperiodic_t=True, hip_device=0, hip_stream=stream)
    M.mdwf_set_action(ctx, *act_t)
    M.mdwf_load_gauge_dev(ctx, Ud.data_ptr())
    opts = dict(tol=1e-10, inner=M.MDWF_F16, max_iter=args.max_iter, delta=0.1,
                schur_form=FORMS[args.schur_form])
    if not args.no_tune:
        M.mdwf_autotune_solve(ctx, 12, opts)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step():
        e = [ev() for _ in range(4)]
        e[0].record(work)
        M.mdwf_gauss_smear_dev(dims, Ud.data_ptr(), 12, eta.data_ptr(), sm.data_ptr(), SMEAR_SIGMA, SMEAR_ITERS,
                               stream)
        e[1].record(work)
        M.mdwf_wall_source_dev(dims, act_t, Ud.data_ptr(), 12, sm.data_ptr(), b.data_ptr(), True, stream)
        e[2].record(work)
        st, infos = M.mdwf_solve_dev(ctx, [b[k].data_ptr() for k in range(12)], [x[k].data_ptr() for k in range(12)],
                                     opts=opts, stream=stream)
        e[3].record(work)
        c0 = time.perf_counter()
        corr = M.mdwf_mres_correlators_dev(dims, L5_, 12, x.data_ptr(), stream)
        corr_s = time.perf_counter() - c0
        torch.cuda.synchronize()
        return st, infos, corr, dict(smear_ms=e[0].elapsed_time(e[1]), wall_ms=e[1].elapsed_time(e[2]),
                                     solve_ms=e[2].elapsed_time(e[3]), corr_ms=1e3 * corr_s)

    for w in range(args.warmup):
        st, infos, _, kt = step()
        log("warmup %d: status %d, %s" % (w, st, kt))
    times, kts = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, infos, corr, kt = step()
        times.append(time.perf_counter() - t0)
        kts.append(kt)
        log("step %d: %.3f s status %d max true resid %.2e  %s" % (k, times[-1], st,
                                                                  max(i["true_resid"] for i in infos), kt))
    cpp, cmp_, mres = corr
    # integrated axial Ward identity: sum_t [C_mp + m C_PP] = Re sum_cols <source, q(source)>
    q = torch.empty_like(sm)
    M.mdwf_project_4d_dev(dims, L5_, 12, x.data_ptr(), q.data_ptr(), None, stream)
    torch.cuda.synchronize()
    ward_rhs = float(torch.sum(sm * q).item())      # Re <a, b> = sum of re*re + im*im
    ward_lhs = float(np.sum(cmp_ + act_t[3] * cpp))
    ms = 1e3 * float(np.mean(times))
    kmean = {k: float(np.mean([d[k] for d in kts])) for k in kts[0]}
    sb, wb, cb = smear_bytes(V, 12), wall_bytes(V, 12, L5_), corr_bytes(V, 12)
    solve_bytes = sum(i["model_bytes"] for i in infos)
    step_bytes = SMEAR_ITERS * sb + wb + solve_bytes + cb
    value = step_bytes / (ms * 1e-3) / 1e9
    smear_us = 1e3 * kmean["smear_ms"] / SMEAR_ITERS
    achieved = sb / (smear_us * 1e-6) / 1e9
    far = [t for t in range(T) if min((t - ts) % T, (ts - t) % T) >= 6]
    cpu = None
    if not args.no_cpu:
        from oracle import sources as SRC
        import oracle
        small = (8, 8, 8, 16)
        Us = I.random_links(small, EPS, GAUGE_SEED)
        acts = oracle.Action(small, L5_, *act_t[:4])
        Vs = int(np.prod(small))
        t0 = time.perf_counter()
        cols = []
        for j in range(12):
            e_ = SRC.gauss_smear(Us, SRC.point_source(small, (0, 0, 0, 0), j // 3, j % 3), SMEAR_SIGMA, SMEAR_ITERS)
            cols.append(SRC.wall_source(acts, Us, e_))      # stands in for the solution: same size, same reads
        with np.errstate(all="ignore"):                    # slices the stand-in leaves empty give 0/0
            SRC.correlators(cols)
        dt = time.perf_counter() - t0
        cpu = dict(value=round((SMEAR_ITERS * smear_bytes(Vs, 12) + wall_bytes(Vs, 12, L5_) + corr_bytes(Vs, 12))
                               / dt / 1e9, 4), unit="GB/s", cores=1, kind="oracle",
                   sample="the numpy oracle's source and sink side (12 columns smeared by %d steps, wall sources, "
                          "correlators) on 8^3x16, L5=%d, %.2f s; the solve's CPU baseline is the mixed workload's"
                          % (SMEAR_ITERS, L5_, dt))
    out = {
        "metric": "Moebius DWF dslash GB/s (% HBM peak); time to r=1e-10 solve, mixed vs FP64",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f16",
        "data": "synthetic",
        "config": {"workload": "m_res chain on %dx%dx%dx%d L5=%d M5=%g b5=%g c5=%g m_q=%g, exp(i0.25H) links: 12 "
                               "point-source columns Gaussian-smeared (sigma=%g, %d steps), Moebius wall sources, "
                               "mixed FP16 solve to 1e-10 (%s form), midpoint and wall correlators"
                               % (X, Y, Z, T, L5_, act_t[0], act_t[1], act_t[2], act_t[3], SMEAR_SIGMA, SMEAR_ITERS,
                                  FORM_NAMES[args.schur_form]),
                   "name": "mres", "lattice": list(dims), "L5": L5_, "source_site": [xs, ys, zs, ts]},
        "kernels": {"smear_us_per_step": round(smear_us, 1), "smear_GBps": round(achieved, 1),
                    "wall_source_us": round(1e3 * kmean["wall_ms"], 1),
                    "wall_source_GBps": round(wb / (kmean["wall_ms"] * 1e-3) / 1e9, 1),
                    "correlators_us_incl_copy": round(1e3 * kmean["corr_ms"], 1),
                    "solve_s": round(kmean["solve_ms"] / 1e3, 3),
                    "solve_iters": max(i["iters"] for i in infos)},
        "mres": {"mres_t": [float("%.6g" % v) for v in mres], "mres_far_mean": float(np.mean(mres[far])),
                 "far_slices": "|t - t_src| >= 6", "ward_lhs": ward_lhs, "ward_rhs": ward_rhs,
                 "ward_rel": abs(ward_lhs - ward_rhs) / abs(ward_rhs),
                 "max_true_resid": max(i["true_resid"] for i in infos)},
        "roofline": {"bound": "hbm", "kernel": "k_gauss_step (one smearing step, 12 vectors, FP64)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "model": "per site: 12 x (192 B read + 192 B written) + 3 spatial links (432 B)"},
        "cpu_baseline": cpu,
    }
    M.mdwf_destroy(ctx)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="mixed")
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--inner", choices=["f16", "f32"], default="f16")
    ap.add_argument("--nrhs", type=int, default=12)
    ap.add_argument("--fp64-cols", type=int, default=-1,
                    help="columns solved with plain FP64 CG for the comparison (-1: all 12 for the mixed "
                         "workload, one per mass for the batched one; 0: none)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-micro", action="store_true")
    ap.add_argument("--graph", type=int, default=0,
                    help="1: replay CG iterations from a hipGraph (no per-launch timing then)")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner")
    ap.add_argument("--delta", type=float, default=0.1,
                    help="reliable update of the mixed solve when ||r|| falls below delta x its value "
                         "at the last update")
    ap.add_argument("--micro-only", action="store_true", help="time the operator kernels and stop")
    ap.add_argument("--micro-reps", type=int, default=50)
    ap.add_argument("--micro-precs", default="f64,f32,f16")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one plain device copy of 1 GiB (counter calibration)")
    ap.add_argument("--max-iter", type=int, default=50000,
                    help="cap on CG iterations (a short cap only for counter runs)")
    ap.add_argument("--summarize", nargs=3, metavar=("TRACE_DB", "FETCH_DB", "WRITE_DB"),
                    help="write the rocprofv3 summary of the dominant kernels (no GPU use); "
                         "FETCH_DB / WRITE_DB may be '-'")
    ap.add_argument("--pmc-summary", default=None, metavar="DB",
                    help="write the VALU / LDS busy summary of a rocprofv3 counter database (no GPU use)")
    ap.add_argument("--summary-out", default=None)
    ap.add_argument("--summary-cmds", default="", help="commands that produced the databases ('||'-separated)")
    ap.add_argument("--summary-bench", default=None, help="the JSON line bench.py printed in the traced run")
    ap.add_argument("--requests", type=int, default=12, help="serving: requests in the burst")
    ap.add_argument("--poisson-requests", type=int, default=16, help="serving: requests in the Poisson stream")
    ap.add_argument("--load", type=float, default=0.7, help="serving: Poisson rate / burst throughput")
    ap.add_argument("--max-active", type=int, default=4, help="serving: worker streams")
    ap.add_argument("--host-cap-gb", type=float, default=160.0, help="serving: outstanding solution memory on the host")
    ap.add_argument("--no-serial", action="store_true", help="serving: skip the one-at-a-time pass")
    ap.add_argument("--schur-form", choices=["asym", "sym", "rp"], default="rp",
                    help="CG operator of the mixed solve: S, the symmetric K5^-1 S, or S B^-1")
    ap.add_argument("--fp64-form", choices=["asym", "sym", "rp"], default="asym",
                    help="CG operator of the plain FP64 comparison solve")
    ap.add_argument("--shamir", action="store_true", help="b5 = 1, c5 = 0 instead of the Moebius b5, c5")
    args = ap.parse_args()
    if args.summarize:
        summarize(args)
        return
    if args.pmc_summary:
        pmc_summary(args)
        return

    if args.gpus != 1:
        print("bench.py runs on one GPU only (this build has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "serving":
        serve_main(args)
        return
    if args.workload == "flow":
        flow_main(args)
        return
    if args.workload == "mres":
        mres_main(args)
        return
    global DIMS, L5, MASSES, GAUGE_SEED, SITE_SEED, GROUPS, SRC_SEED, EPS
    wl = WORKLOADS[args.workload]
    DIMS, L5, MASSES, GROUPS = wl["DIMS"], wl["L5"], wl["MASSES"], wl["GROUPS"]
    GAUGE_SEED, SITE_SEED = wl["GAUGE_SEED"], wl["SITE_SEED"]
    SRC_SEED = wl.get("SRC_SEED", SRC_SEED)
    ACTION["mq"] = MASSES[0]
    if args.shamir:
        ACTION["b5"], ACTION["c5"] = 1.0, 0.0
    fp64_workload = args.workload == "fp64"

    import torch
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from paper_1701_07559_amd import inputs as I
    from paper_1701_07559_amd import mdwf as M

    dev = torch.device("cuda:0")
    # One explicit stream for torch and the library: torch's default stream
    # is the null handle, which the C ABI reads as "the context's stream".
    work = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(work)
    X, Y, Z, T = DIMS
    V = X * Y * Z * T
    Vh = V * L5 // 2
    log("generating links", DIMS)
    U = I.random_links(DIMS, EPS, GAUGE_SEED, workers=min(8, host_cpu_info()["threads"]))
    plaq = I.plaquette(U)
    log("plaquette %.4f" % plaq)

    ctx = M.mdwf_create(DIMS, antiperiodic_t=True, hip_device=0, hip_stream=work.cuda_stream)
    M.mdwf_set_action(ctx, ACTION["M5"], ACTION["b5"], ACTION["c5"], ACTION["mq"], L5)
    M.mdwf_load_gauge(ctx, U)
    stream = work.cuda_stream
    assert stream and torch.cuda.current_stream().cuda_stream == stream
    tune = None
    if not args.no_tune:
        tune = M.mdwf_autotune(ctx)
        for pn, t in zip(("f64", "f32", "f16"), tune):
            log("autotune %s: tile %s xcd_remap %d nt_store %d link_mode %d plane_bt %d  schur %.1f us" %
                (pn, t["tile"], t["xcd_remap"], t["nt_store"], t["link_mode"], t["plane_bt"], t["us"]))

    if args.copy_calib:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    micro = {}
    if not args.no_micro:
        precs = [p for p in (("f64", 0), ("f32", 1), ("f16", 2)) if p[0] in args.micro_precs.split(",")]
        for pname, prec in precs:
            for oname, op in (("hop", M.MDWF_OP_HOP_EO), ("schur", M.MDWF_OP_SCHUR),
                              ("schur_dag", M.MDWF_OP_SCHUR_DAG)):
                r = time_apply(M, torch, ctx, op, prec, reps=args.micro_reps)
                micro["%s_%s" % (oname, pname)] = r
                log("%s %s: %.3f ms  %.0f GB/s  %.0f GFLOP/s" % (oname, pname, r["ms"], r["GBps"], r["GFLOPs"]))
    if args.micro_only:
        print(json.dumps({k: dict(ms=v["ms"], GBps=v["GBps"]) for k, v in micro.items()}), flush=True)
        M.mdwf_destroy(ctx)
        return

    ncan = L5 * V * 24
    if fp64_workload:
        # one Gaussian 5D source (the a15m310 row: a single RHS), solved by
        # plain FP64 CG on the asymmetric Schur system
        nrhs, ncol = 1, 1
        src = I.gaussian_source(DIMS, L5, SRC_SEED)
        b = torch.from_numpy(src.view(np.float64).ravel()).to(dev).view(1, ncan)
        del src
        rhs_col, rhs_mass = [0], [MASSES[0]]
        inner_name = "f64"
        inner = M.MDWF_F64
        form = args.fp64_form
    else:
        # the 12 spin-colour columns of a point source, FP64 canonical, built
        # on the device; RHS k is column k // len(MASSES) at mass k % len(MASSES)
        nrhs = args.nrhs if args.workload == "mixed" else 12 * len(MASSES)
        ncol = min(12, nrhs) if args.workload == "mixed" else 12
        site = I.random_point_site(DIMS, SITE_SEED)
        b = torch.zeros((ncol, ncan), dtype=torch.float64, device=dev)
        xs, ys, zs, ts = site
        for k in range(ncol):
            spin, colour = k // 3, k % 3
            s = L5 - 1 if spin < 2 else 0
            idx = ((((s * T + ts) * Z + zs) * Y + ys) * X + xs) * 12 + spin * 3 + colour
            b[k, 2 * idx] = 1.0
        rhs_col = [(k // len(MASSES)) % ncol for k in range(nrhs)]
        rhs_mass = [MASSES[k % len(MASSES)] for k in range(nrhs)]
        inner_name = args.inner
        inner = M.MDWF_F16 if args.inner == "f16" else M.MDWF_F32
        form = args.schur_form
    per = nrhs // GROUPS
    x = torch.zeros((per, ncan), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    # profile_iters / profile_every: the library times its batched hop
    # launches with HIP events on the solve stream (the roofline figure) in
    # every 8th CG iteration from the third, so the samples span the whole
    # timed solve (up to 64 of them)
    opts = dict(tol=1e-10, inner=inner, max_iter=args.max_iter, delta=args.delta, use_graph=args.graph,
                profile_iters=0 if args.graph else 64, profile_every=PROFILE_EVERY, schur_form=FORMS[form])
    bptr = [b[rhs_col[k]].data_ptr() for k in range(nrhs)]
    xptr = [x[k].data_ptr() for k in range(per)]
    # launch shapes for the solve itself: the inner precision on its CG
    # operator with `per` RHS per launch, FP64 on it with one RHS
    solve_tune = None
    if not args.no_tune:
        solve_tune = M.mdwf_autotune_solve(ctx, per, opts)
        for pn, t in zip(("f64", "f32", "f16"), solve_tune):
            log("solve autotune %s: tile %s xcd_remap %d nt_store %d link_mode %d rhs_group %d  %.1f us" %
                (pn, t["tile"], t["xcd_remap"], t["nt_store"], t["link_mode"], t["rhs_group"], t["us"]))

    def step():
        """The whole step: every launch group solved to 1e-10 (status, infos)."""
        st_all, info_all = M.MDWF_OK, []
        for g in range(GROUPS):
            ks = range(g * per, (g + 1) * per)
            st, inf = M.mdwf_solve_dev(ctx, [bptr[k] for k in ks], xptr, mq=[rhs_mass[k] for k in ks],
                                       opts=opts, stream=stream)
            if st != M.MDWF_OK and st_all == M.MDWF_OK:
                st_all = st
            info_all += inf
        return st_all, info_all

    for w in range(args.warmup):
        st, info = step()
        log("warmup %d: status %d iters %s" % (w, st, [i["iters"] for i in info]))
    torch.cuda.synchronize()
    times, infos = [], None
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts0 = time.perf_counter()
        st, infos = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts0)
        log("step %d: %.3f s status %d max true resid %.2e" % (k, times[-1], st,
                                                                max(i["true_resid"] for i in infos)))
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = 1e3 * total / args.steps
    step_bytes = sum(i["model_bytes"] for i in infos)
    step_flops = sum(i["model_flops"] for i in infos)
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    all_ok = st == M.MDWF_OK and all(i["true_resid"] <= 1e-10 for i in infos)

    # the other side of "mixed vs FP64": for the mixed workloads, plain FP64
    # CG on the same columns, one at a time, every solution kept; for the
    # FP64 workload, the mixed (FP16-inner) solve of the same source
    fp64 = None
    errs = None
    other = None
    if fp64_workload:
        xm = torch.zeros((1, ncan), dtype=torch.float64, device=dev)
        om = dict(tol=1e-10, inner=M.MDWF_F16, max_iter=args.max_iter, schur_form=FORMS["rp"],
                  x_ref=[x[0].data_ptr()])
        M.mdwf_autotune_solve(ctx, 1, om)
        t_a = time.perf_counter()
        stm, im = M.mdwf_solve_dev(ctx, [bptr[0]], [xm[0].data_ptr()], mq=[rhs_mass[0]], opts=om, stream=stream)
        torch.cuda.synchronize()
        tm = time.perf_counter() - t_a
        log("mixed f16 solve: %.3f s iters %d resid %.2e err vs fp64 %.2e" %
            (tm, im[0]["iters"], im[0]["true_resid"], im[0]["err_vs_ref"]))
        other = dict(inner="f16", form=FORM_NAMES["rp"], seconds=round(tm, 4), iters=im[0]["iters"],
                     reliable_updates=im[0]["reliable_updates"], true_resid=im[0]["true_resid"],
                     err_vs_fp64=im[0]["err_vs_ref"], speedup_vs_fp64=round((ms_per_step / 1e3) / tm, 3),
                     note="includes its own first-call allocations; tuned for 1 RHS")
        del xm
    elif args.fp64_cols != 0:
        ncols64 = nrhs if args.fp64_cols < 0 and args.workload == "mixed" else \
            (len(MASSES) if args.fp64_cols < 0 else min(args.fp64_cols, nrhs))
        # columns measured: all of them (mixed), or one per mass (batched)
        cols = list(range(ncols64)) if args.workload == "mixed" else \
            [k * (nrhs // ncols64) + (k % len(MASSES)) for k in range(ncols64)]
        o64 = dict(tol=1e-10, inner=M.MDWF_F64, max_iter=50000, use_graph=args.graph,
                   schur_form=FORMS[args.fp64_form])
        x64 = torch.zeros((len(cols), ncan), dtype=torch.float64, device=dev)
        t64, it64, r64 = [], [], []
        for j, k in enumerate(cols):
            t_a = time.perf_counter()
            st64, i64 = M.mdwf_solve_dev(ctx, [bptr[k]], [x64[j].data_ptr()], mq=[rhs_mass[k]], opts=o64,
                                         stream=stream)
            torch.cuda.synchronize()
            t64.append(time.perf_counter() - t_a)
            it64.append(i64[0]["iters"])
            r64.append(i64[0]["true_resid"])
            log("fp64 column %d: %.3f s iters %d resid %.2e" % (k, t64[-1], it64[-1], r64[-1]))
        measured_all = len(cols) == nrhs
        fp64 = dict(form=FORM_NAMES[args.fp64_form], columns_solved=len(cols), seconds=[round(t, 4) for t in t64],
                    iters=it64, max_true_resid=max(r64),
                    cg_iteration_ms=round(1e3 * sum(t64) / max(1, sum(it64)), 4),
                    seconds_all_columns=round(sum(t64) if measured_all else float(np.mean(t64)) * nrhs, 4),
                    note="measured: sum over the %d columns" % nrhs if measured_all else
                    "sum over %d columns = mean of %d measured columns x %d" % (nrhs, len(cols), nrhs))
        # per-solve error of the mixed solution against the FP64 one: the
        # mixed solve of the measured columns once more, outside the timed
        # region, with the FP64 solutions as references
        for g0 in range(0, len(cols), per):
            gc = cols[g0:g0 + per]
            xe = torch.zeros((len(gc), ncan), dtype=torch.float64, device=dev)
            oe = dict(opts, profile_iters=0, x_ref=[x64[g0 + j].data_ptr() for j in range(len(gc))])
            ste, ie = M.mdwf_solve_dev(ctx, [bptr[k] for k in gc], [v.data_ptr() for v in xe],
                                       mq=[rhs_mass[k] for k in gc], opts=oe, stream=stream)
            torch.cuda.synchronize()
            errs = (errs or []) + [i["err_vs_ref"] for i in ie]
            del xe
        log("err vs fp64 per column: %s" % ", ".join("%.2e" % e for e in errs))
        del x64

    roof = roofline(infos[0], inner_name, Vh, form)
    rec = stored_traffic(args.schur_form) if (roof and args.inner == "f16" and args.workload == "mixed"
                                              and nrhs == 12 and not args.shamir) else None
    if rec:
        roof["traffic"] = round(rec["traffic_bytes_per_launch"], 0)
        roof["traffic_note"] = "HBM bytes per operator application (kernels A + B) from rocprofv3 FETCH_SIZE / WRITE_SIZE, " \
                               "scaled by the 1 GiB copy calibration; %s" % os.path.relpath(TRAFFIC_FILE)

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle")
        bk = b[rhs_col[0]].cpu().numpy().view(np.complex128).reshape(L5, T, Z, Y, X, 4, 3)
        xk = x[0].cpu().numpy().view(np.complex128).reshape(L5, T, Z, Y, X, 4, 3)
        it_ref = fp64["iters"] if fp64 else [infos[0]["iters"]] if fp64_workload else None
        cpu = cpu_baseline(U, DIMS, L5, dict(ACTION, mq=rhs_mass[0]), fp64_iters=it_ref, ncols=nrhs,
                           check=(bk, xk))
        del bk, xk
        log("cpu oracle %.3f GB/s on %d threads (%.3f on 1); oracle true residual of column 0: %.2e" %
            (cpu["value"], cpu["cores"], cpu["single_thread"]["value"], cpu["oracle_true_resid_of_gpu_solution"]))

    t_step = ms_per_step / 1e3
    out = {
        "metric": "Moebius DWF dslash GB/s (% HBM peak); time to r=1e-10 solve, mixed vs FP64",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": inner_name,
        "data": "synthetic",
        "value_definition": "algorithmic HBM bytes of every kernel of the step (per 5D site: each spinor field "
                            "read or written once per kernel, the links once per multi-RHS launch) / step time; "
                            "the dslash kernels alone are in roofline.achieved",
        "config": {
            "workload": ("%dx%dx%dx%d L5=%d M5=%g b5=%g c5=%g m_q=%s, exp(i0.25H) links (plaquette %.3f), "
                         "1 Gaussian RHS, plain FP64 CG on the %s Schur form to true residual 1e-10" %
                         (X, Y, Z, T, L5, ACTION["M5"], ACTION["b5"], ACTION["c5"], MASSES[0], plaq,
                          FORM_NAMES[form])) if fp64_workload else
                        ("%dx%dx%dx%d L5=%d M5=%g b5=%g c5=%g m_q=%s, exp(i0.25H) links (plaquette %.3f), "
                         "%d point-source RHS (%d columns x %d masses) in %d multi-RHS %s-inner launch(es) of %d, "
                         "%s Schur form, each to true residual 1e-10" %
                         (X, Y, Z, T, L5, ACTION["M5"], ACTION["b5"], ACTION["c5"],
                          "/".join(str(m) for m in MASSES), plaq, nrhs, ncol, len(MASSES),
                          GROUPS, args.inner, per, FORM_NAMES[form])),
            "name": args.workload,
            "lattice": list(DIMS), "L5": L5, "nrhs": nrhs, "masses": MASSES, "inner": inner_name,
            "schur_form": form, "b5": ACTION["b5"], "c5": ACTION["c5"], "delta": args.delta,
            "launch_tune": ({pn: t for pn, t in zip(("f64", "f32", "f16"), tune)} if tune else None),
            "solve_tune": ({pn: t for pn, t in zip(("f64", "f32", "f16"), solve_tune)} if solve_tune else None),
        },
        "solve": {
            "seconds": round(t_step, 4),
            "iters": [i["iters"] for i in infos],
            "reliable_updates": [i["reliable_updates"] for i in infos],
            "max_true_resid": max(i["true_resid"] for i in infos),
            "all_within_1e-10": bool(all_ok),
            "model_GFLOPs": round(step_flops / (ms_per_step * 1e-3) / 1e9, 1),
            "model_bytes": step_bytes,
            "err_vs_fp64": [float("%.3g" % e) for e in errs] if errs else None,
            # wall time of one iteration of the batched solve (all its RHS),
            # source preparation, reliable updates and verification included
            "cg_iteration_ms": round(ms_per_step / max(i["iters"] for i in infos), 4),
        },
        "fp64_cg": fp64,
        "mixed_solve": other,
        "speedup_mixed_multirhs_vs_fp64": (round(fp64["seconds_all_columns"] / t_step, 3) if fp64 else None),
        "dslash_GBps": ((roof["hbm"] if "hbm" in roof else roof)["achieved"]) if roof else None,
        "dslash": {k: dict(ms=round(v["ms"], 4), GBps=round(v["GBps"], 1), frac=round(v["GBps"] / HBM_PEAK_GBS, 4),
                           GFLOPs=round(v["GFLOPs"], 1)) for k, v in micro.items()},
        "roofline": roof,
        "cpu_baseline": cpu,
        "paper": "QUDA double-half MDWF solver, 1250 GFLOP/s on 2x K40 (Surface), 1785 on 4x K80 dies "
                 "(RZHasGPU), volume not stated (context only)",
    }
    if fp64_workload:
        out["note"] = ("FP64 working set of one hop launch (in + out + links) is about %.0f MB, so part of it can "
                       "sit in the 256 MB Infinity Cache" % ((2 * Vh * 192 + V * 4 * 144) / 1e6))
    print(json.dumps(out), flush=True)
    M.mdwf_destroy(ctx)


if __name__ == "__main__":
    main()
