"""Solve-server policy on the CPU (fake backend with a virtual clock):
admission by footprint never exceeds the budget, requests that arrive while
others run join the resident set (continuous batching), a failing request
fails alone, and latency accounting is consistent."""
import math
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2501_00923_amd import inputs as I
from paper_2501_00923_amd import serving as S


def _req(rid, arrival, ni=64, nj=32, nv=16, adj=False, name="w"):
    g = SimpleNamespace(ni=ni, nj=nj)
    wl = SimpleNamespace(grid=g, vgrid=SimpleNamespace(n1=nv, n2=nv), name=name)
    return SimpleNamespace(rid=rid, arrival=arrival, workload=wl, want_adjoint=adj)


def _stream(n=60, rate=200.0, seed=3):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        ni, nj = I.SERVE_MESHES[rng.integers(3)]
        nv = I.SERVE_VGRIDS[rng.integers(3)]
        out.append(_req(i, t, ni, nj, nv, bool(rng.random() < 0.5)))
    return out


def test_all_complete_within_budget_and_batches_mix():
    reqs = _stream()
    fb = S.FakeBackend(cost_per_pair=2e-12)
    budget = 6 * 256 * 128 * 64 * 64 * 16
    out = S.serve(reqs, fb, S.ServeConfig(memory_budget=budget, sweeps_per_check=10, tol=1e-6),
                  clock=fb.clock, sleep=fb.sleep)
    assert out["completed"] == len(reqs) and out["failed"] == 0
    assert fb.max_live_bytes <= budget and out["peak_bytes"] <= budget
    assert max(fb.batches) > 1                     # requests ran together
    assert len(fb.live) == 0                       # everything released
    for r in out["results"]:
        assert r.admitted >= r.arrival - 1e-12 and r.finished >= r.admitted
        assert r.status == "ok" and r.J == float(r.rid)
        assert (r.adjoint_iters > 0) == reqs[r.rid].want_adjoint
    lat = sorted(r.latency for r in out["results"])
    assert out["p50_ms"] == pytest.approx(1e3 * np.percentile(lat, 50))
    assert out["p99_ms"] >= out["p50_ms"]


def test_one_at_a_time_runs_singletons_and_is_slower_in_p99():
    reqs = _stream(40, rate=400.0)
    cfg = S.ServeConfig(memory_budget=10 ** 12, sweeps_per_check=10, tol=1e-6)
    fb1 = S.FakeBackend(cost_per_pair=2e-12)
    one = S.serve_one_at_a_time(reqs, fb1, cfg, clock=fb1.clock, sleep=fb1.sleep)
    assert set(fb1.batches) == {1}
    fb2 = S.FakeBackend(cost_per_pair=2e-12)
    many = S.serve(reqs, fb2, cfg, clock=fb2.clock, sleep=fb2.sleep)
    assert one["completed"] == many["completed"] == len(reqs)
    assert max(fb2.batches) > 1


def test_oversized_and_failing_requests_fail_alone():
    reqs = [_req(0, 0.0), _req(1, 0.0, ni=256, nj=128, nv=64, adj=True), _req(2, 0.001, name="nan_case"),
            _req(3, 0.002), _req(4, 0.003)]
    fb = S.FakeBackend(fail_create={3})
    budget = 64 * 32 * 16 * 16 * 16 * 4 * 3
    out = S.serve(reqs, fb, S.ServeConfig(memory_budget=budget, sweeps_per_check=5, tol=1e-6),
                  clock=fb.clock, sleep=fb.sleep)
    st = {r.rid: r.status for r in out["results"]}
    assert st == {0: "ok", 1: "failed", 2: "failed", 3: "failed", 4: "ok"}
    errs = {r.rid: r.error for r in out["results"]}
    assert "budget" in errs[1] and "non-finite" in errs[2] and "injected" in errs[3]
    assert len(fb.live) == 0


def test_on_finish_reports_every_request_once():
    reqs = _stream(n=20)
    fb = S.FakeBackend(fail_create={3})
    seen = []
    out = S.serve(reqs, fb, S.ServeConfig(memory_budget=1 << 40, sweeps_per_check=10, tol=1e-6),
                  clock=fb.clock, sleep=fb.sleep, on_finish=lambda res, n: seen.append((res.rid, n)))
    assert sorted(r for r, _ in seen) == sorted(r.rid for r in reqs)
    assert [n for _, n in seen] == list(range(1, len(reqs) + 1))
    assert out["failed"] == 1


def test_iteration_cap_marks_notconv_but_returns_result():
    reqs = [_req(0, 0.0, adj=True)]
    fb = S.FakeBackend()
    out = S.serve(reqs, fb, S.ServeConfig(memory_budget=10 ** 12, sweeps_per_check=5, tol=1e-300,
                                          adjoint_tol=1e-300, max_iter=20), clock=fb.clock, sleep=fb.sleep)
    r = out["results"][0]
    assert r.status == "notconv" and r.primal_iters == 20 and r.adjoint_iters == 20 and not math.isnan(r.J)


def test_poisson_stream_is_seeded():
    a = I.poisson_stream(5, 10.0, seed=7, mesh_choices=[(64, 32)], vgrid_choices=[16])
    b = I.poisson_stream(5, 10.0, seed=7, mesh_choices=[(64, 32)], vgrid_choices=[16])
    assert [r.arrival for r in a] == [r.arrival for r in b]
    assert [r.workload.flow.Kn for r in a] == [r.workload.flow.Kn for r in b]
    assert all(np.array_equal(x.workload.grid.nodes, y.workload.grid.nodes) for x, y in zip(a, b))
    assert all(1e-3 <= r.workload.flow.Kn <= 10 and 0.3 <= r.workload.flow.Ma <= 2.0 for r in a)


def test_converged_and_capped_solves_are_reported_apart():
    """Solves stopped at the sweep cap are counted apart from converged ones
    (solves/s and latency of each, and the cap rate per decade of Kn)."""
    reqs = _stream(40, rate=400.0, seed=5)
    for r in reqs:
        r.workload.flow = SimpleNamespace(Kn=10.0 ** (-3 + 4 * (r.rid % 8) / 8))
    fb = S.FakeBackend(cost_per_pair=2e-12)
    cfg = S.ServeConfig(memory_budget=10 ** 12, sweeps_per_check=10, tol=1e-6, adjoint_tol=1e-6, max_iter=60)
    out = S.serve(reqs, fb, cfg, clock=fb.clock, sleep=fb.sleep)
    conv = [r for r in out["results"] if r.status == "ok"]
    capped = [r for r in out["results"] if r.status == "notconv"]
    assert conv and capped
    assert out["converged"]["count"] == len(conv) and out["capped"]["count"] == len(capped)
    assert out["completed"] == len(conv) + len(capped)
    assert out["converged"]["p50_ms"] == pytest.approx(1e3 * np.percentile([r.latency for r in conv], 50))
    assert out["converged"]["solves_per_s"] == pytest.approx(len(conv) / out["wall_s"])
    by_kn = out["capped_by_kn"]
    assert sum(v["requests"] for v in by_kn.values()) == len(reqs)
    assert sum(v["capped"] for v in by_kn.values()) == len(capped)
