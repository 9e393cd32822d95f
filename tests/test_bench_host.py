"""Host logic of the serving benchmark driver, against a stand-in server that
runs no GPU code: every request is collected once, solutions are freed after
collection, the host-memory cap on outstanding solutions holds, and the
one-at-a-time pass never overlaps two requests."""
import threading
import time

import numpy as np

import bench


class FakeServer:
    def __init__(self, solve_s=0.02):
        self.solve_s = solve_s
        self.lock = threading.Lock()
        self.next = 1
        self.jobs = {}
        self.active = 0
        self.max_active = 0
        self.out = 0       # bytes of solutions submitted and not yet collected
        self.max_out = 0

    def submit_point(self, field, M5, b5, c5, mq, L5, site, cols, xs, masses=None, opts=None):
        assert len(cols) == len(xs) == len(masses) and cols == list(range(len(xs))) and len(site) == 4
        with self.lock:
            rid = self.next
            self.next += 1
            ev = threading.Event()
            self.jobs[rid] = (ev, len(xs), time.perf_counter(), sum(x.nbytes for x in xs))
            self.out += self.jobs[rid][3]
            self.max_out = max(self.max_out, self.out)

        def run():
            with self.lock:
                self.active += 1
                self.max_active = max(self.max_active, self.active)
            time.sleep(self.solve_s)
            for k, x in enumerate(xs):
                x[...] = rid * 100 + k
            with self.lock:
                self.active -= 1
            ev.set()

        threading.Thread(target=run, daemon=True).start()
        return rid

    def wait(self, rid):
        ev, n, t0, nbytes = self.jobs.pop(rid)
        ev.wait()
        with self.lock:
            self.out -= nbytes
        lat = time.perf_counter() - t0
        info = [dict(model_bytes=1e6, true_resid=1e-11, iters=10, launch_rhs=n) for _ in range(n)]
        return 0, info, (0.0, lat, lat)


SITES = [(0, 0, 0, 0)] * 4
# field f: outputs of 8 * (f + 1) complex numbers
QSHAPES = [(8 * (f + 1),) for f in range(4)]


def test_serving_driver_collects_every_request_within_the_host_cap():
    rng = np.random.default_rng(1)
    reqs = bench.serve_requests(10, rng)
    assert all(1 <= k <= bench.SERVE_MAX_RHS[f] and len(m) == k for f, k, m in reqs)
    biggest = max(k * 16 * QSHAPES[f][0] for f, k, _ in reqs)
    cap = biggest  # at most one of the largest requests' solutions outstanding
    srv = FakeServer()
    recs, wall = bench.run_phase(None, srv, [0, 1, 2, 3], SITES, QSHAPES, reqs, [0.0] * len(reqs), {}, cap)
    assert wall > 0 and all(r is not None for r in recs)
    assert all(len(r["digest"]) == k for r, (_, k, _) in zip(recs, reqs))
    s = bench.phase_summary(reqs, recs, wall)
    assert s["requests"] == 10 and s["all_ok"] and s["rhs"] == sum(k for _, k, _ in reqs)
    assert s["shared_requests"] == 0 and s["mean_launch_rhs"] >= 1
    assert not srv.jobs and srv.max_out <= cap


def test_serving_driver_one_at_a_time_never_overlaps():
    rng = np.random.default_rng(2)
    reqs = bench.serve_requests(6, rng)
    srv = FakeServer()
    recs, _ = bench.run_phase(None, srv, [0, 1, 2, 3], SITES, QSHAPES, reqs, [0.0] * 6, {}, 1 << 40,
                              serial=True)
    assert srv.max_active == 1 and len(recs) == 6
    srv2 = FakeServer(solve_s=0.05)
    bench.run_phase(None, srv2, [0, 1, 2, 3], SITES, QSHAPES, reqs, [0.0] * 6, {}, 1 << 40)
    assert srv2.max_active > 1


def test_serving_digest_sees_every_byte():
    a = np.zeros(1000, complex)
    b = a.copy()
    b[999] = 1e-300
    assert bench._digest(a) != bench._digest(b)
    assert bench._digest(a) == bench._digest(a.copy())
