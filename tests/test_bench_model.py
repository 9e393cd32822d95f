"""The benchmark's byte, flop and peak models and its guards, on the host:
the per-site bytes of one Schur-operator application against the scope
table's figures, the vector-ALU peak of the FP16 kernels against its
instruction count, the counter record applying only to the kernel source it
was taken on, the flow stage's byte model, the one-GPU guard, and the
counter summary that writes that record from rocprofv3 databases."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture
def l5_8(monkeypatch):
    monkeypatch.setattr(bench, "L5", 8)


@pytest.mark.parametrize("inner,per_site", [("f16", 332), ("f32", 624), ("f64", 1248)])
def test_schur_bytes_per_site_match_the_scope_table(l5_8, inner, per_site):
    # one RHS: kernels A + B of S move (120 + 288 / L5) reals per 5D site
    # (plus three FP16 norms), i.e. 332 / 624 / 1248 bytes at L5 = 8
    vh = 1000
    a, b, a_dag, b_dag = bench.hop_launch_bytes(inner, vh, 1)
    assert a + b == pytest.approx(per_site * vh)
    assert (a_dag, b_dag) == (a, b)


def test_batched_launch_charges_the_links_once(l5_8):
    # twelve RHS in one launch: twelve times the spinor bytes, one set of links
    vh = 3538944
    one = bench.hop_launch_bytes("f16", vh, 1)
    twelve = bench.hop_launch_bytes("f16", vh, 12)
    links = vh * 144 * 2 / 8
    for k in range(4):
        assert twelve[k] - links == pytest.approx(12 * (one[k] - links))
    assert twelve[0] == 4544004096 and twelve[1] == 6752305152   # 1284 and 1908 bytes per 5D site


def test_alu_peak_is_the_instruction_count_derivation():
    # 3456 model flops per 5D site and RHS for kernels A + B at L5 = 8 over
    # 1368 lane-instructions: 288 x 2 dot2 (4 flops), 96 x 2 packed-half adds
    # (2), 168 x 2 FP32 adds, 384 + 24 FP32 FMAs (2), at 256 x 4 x 16 lanes
    # and 2.4 GHz
    flops = 1704 + 1752
    instr = 2 * 264 + 2 * 48 + 2 * 168 + 2 * 192 + 24
    assert instr == 1368
    assert bench.alu_peak_tflops(8) == pytest.approx(flops / instr * 256 * 4 * 16 * 2.4e9 / 1e12)
    assert 99.2 < bench.alu_peak_tflops(8) < 99.4


def test_counter_record_applies_only_to_its_kernel_source(monkeypatch):
    with open(bench.TRAFFIC_FILE) as f:
        line = next(l for l in f if l.startswith("traffic-record: "))
    rec = json.loads(line[len("traffic-record: "):])
    monkeypatch.setattr(bench, "kernel_sha", lambda: rec["dslash_sha256"])
    got = bench.stored_traffic("rp")
    assert got is not None and got["traffic_bytes_per_launch"] == rec["traffic_bytes_per_launch"]
    assert bench.stored_traffic("asym") is None            # another Schur form
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 64)
    assert bench.stored_traffic("rp") is None              # the hop source changed since


def test_flow_byte_model():
    # old and new link (144 B each) per stage, the eight-real accumulator
    # (64 B) written by every stage and read by the second and third
    assert bench.FLOW_BYTES_PER_LINK == pytest.approx((352 + 2 * 416) / 3)
    assert bench.FLOW_FLOPS_PER_LINK == 26 * 216


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_counter_summary_computes_the_traffic_record(tmp_path, monkeypatch):
    """bench.py --summarize on small stand-in rocprofv3 databases: the
    12-RHS launches are picked by grid size, FETCH_SIZE and WRITE_SIZE are
    scaled by what the 1 GiB copy reads and writes, and the record is A + B."""
    import argparse
    import sqlite3
    monkeypatch.setattr(bench, "DIMS", (24, 24, 24, 64))
    monkeypatch.setattr(bench, "L5", 8)
    grid12 = 13824 * 12 * 256

    def name(kind):
        return "void mdwf::k_hop<(mdwf::Prec)2, %d, 0>(mdwf::Geo, mdwf::HopDev)" % kind

    trace = str(tmp_path / "trace.db")
    d = sqlite3.connect(trace)
    d.execute("create table kernels (name text, duration integer, grid_x integer)")
    d.executemany("insert into kernels values (?, ?, ?)",
                  [(name(10), 1800000, grid12), (name(10), 1820000, grid12), (name(11), 2100000, grid12),
                   (name(11), 2000000, 3538944), (name(5), 1700000, grid12), (name(12), 2000000, grid12),
                   ("void mdwf::k_cg_r<(mdwf::Prec)2>(mdwf::Geo)", 1000000, 3538944)])
    d.commit()
    vals = {"FETCH_SIZE": {10: 4400000.0, 11: 5800000.0, "copy": 524288.0},
            "WRITE_SIZE": {10: 2150000.0, 11: 2160000.0, "copy": 1048576.0}}
    paths = {}
    for cname, per in vals.items():
        p = str(tmp_path / (cname + ".db"))
        d = sqlite3.connect(p)
        d.execute("create table counters_collection (kernel_name text, grid_size integer, counter_name text, "
                  "value real)")
        rows = [(name(k), grid12, cname, v) for k, v in per.items() if k != "copy"]
        rows += [(name(11), 3538944, cname, 1.0),                     # a one-RHS launch: not selected
                 ("__amd_rocclr_copyBuffer", 134217728, cname, per["copy"]),
                 ("__amd_rocclr_copyBuffer", 64, cname, 0.5)]
        d.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
        d.commit()
        paths[cname] = p
    out = tmp_path / "summary.md"
    args = argparse.Namespace(summarize=[trace, paths["FETCH_SIZE"], paths["WRITE_SIZE"]], summary_cmds="cmd",
                              schur_form="rp", summary_bench=None, summary_out=str(out))
    bench.summarize(args)
    text = out.read_text()
    rec = json.loads(next(l for l in text.splitlines() if l.startswith("traffic-record: "))[len("traffic-record: "):])
    expect = (4400000.0 * 2 + 2150000.0) * 1024 + (5800000.0 * 2 + 2160000.0) * 1024
    assert rec["traffic_bytes_per_launch"] == pytest.approx(expect)
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0 and rec["form"] == "rp"
    assert "| A (`k_hop<F16, 10, *>`) | 2 | 1810.0 |" in text
    assert "| B (`k_hop<F16, 11, *>`) | 1 | 2100.0 |" in text


def test_roofline_of_the_batched_operator(l5_8):
    """The roofline object from the solve's launch timing: the FP16 S B^-1
    pair is priced against the derived vector-ALU peak with the HBM rate
    beside it; other inner precisions against HBM."""
    vh = 3538944
    info = dict(hop_us=[1800.0, 2100.0, 1790.0, 2080.0], hop_rhs=12, hop_samples=46)
    r = bench.roofline(info, "f16", vh, "rp")
    secs = (1800.0 + 2100.0) * 1e-6
    flops = 12 * vh * ((1320 + 48 * 8) + (1320 + 48 * 8 + 48))
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(flops / secs / 1e12, abs=0.01)
    assert r["frac"] == pytest.approx(flops / secs / 1e12 / bench.alu_peak_tflops(8), abs=1e-4)
    assert r["hbm"]["achieved"] == pytest.approx((4544004096 + 6752305152) / secs / 1e9, abs=0.1)
    assert r["launches"]["B"]["algorithmic_bytes"] == 6752305152
    r32 = bench.roofline(info, "f32", vh, "rp")
    assert r32["bound"] == "hbm" and r32["unit"] == "GB/s" and r32["peak"] == 8000.0
    assert bench.roofline(dict(hop_us=[0, 0, 0, 0], hop_rhs=0), "f16", vh, "rp") is None
