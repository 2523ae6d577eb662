"""Serving: continuous batching of CP-ALS requests (mtk_server_* through the C
ABI).  Each request's result must be bitwise the same in the mix as alone
(a lone als_sweep on the same inputs), admission must respect the HBM budget,
and a failing request must not disturb the others."""

import numpy as np
import pytest

from paper_2411_04785_amd import synth

pytestmark = pytest.mark.gpu


def _reqs(n, seed=7, lo=32, hi=72, ranks=(8, 16)):
    g = np.random.default_rng(seed)
    out = []
    for q in range(n):
        dims = tuple(int(x) for x in g.integers(lo, hi + 1, 3))
        R = int(g.choice(ranks))
        w = synth.Workload(f"r{q}", dims, R, R, 1e-4, 1000 + q)
        out.append((q, synth.tensor(w, threads=2), synth.init_factors(w)))
    return out


def _alone(X, init, prec, sweeps):
    import torch
    from paper_2411_04785_amd.mttkrp import Context
    from gpu_util import dev, host
    with Context(0) as ctx:
        fd = [dev(f) for f in init]
        lam = dev(np.ones(init[0].shape[1]))
        ctx.als_sweep(dev(X), fd, lam, sweeps, prec)
        return [host(f) for f in fd], host(lam)


def _drain(srv, n, timeout=120.0):
    import time
    got = {}
    t0 = time.time()
    while len(got) < n and time.time() - t0 < timeout:
        for r in srv.poll(timeout_s=1.0):
            got[r["id"]] = r
    assert len(got) == n, f"only {len(got)} of {n} finished"
    return got


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mix_equals_alone(prec):
    from paper_2411_04785_amd.mttkrp import Server
    reqs = _reqs(8)
    srv = Server(0, budget_bytes=2 * 10**9, max_slots=4)
    for q, X, init in reqs:
        srv.submit(q, X, init, prec, sweeps=4)
    got = _drain(srv, len(reqs))
    srv.close()
    for q, X, init in reqs:
        r = got[q]
        assert r["status"] == 0
        f, lam = _alone(X, init, prec, 4)
        for a, b in zip(r["factors"], f):
            assert np.array_equal(a, b), q
        assert np.array_equal(r["lambda"], lam), q
        assert 0.0 < r["fit"] <= 1.0


def test_budget_admission_and_overlap_counts():
    from paper_2411_04785_amd.mttkrp import Server, MtkError, MTK_EBUDGET
    reqs = _reqs(5, seed=9, lo=40, hi=60, ranks=(8,))
    # Budget for one request at a time: bytes of the largest + a little.
    from paper_2411_04785_amd import mttkrp as b
    big = max(X.nbytes for _, X, _ in reqs)
    budget = 3 * big + (8 << 20)
    srv = Server(0, budget_bytes=budget, max_slots=8)
    for q, X, init in reqs:
        srv.submit(q, X, init, "fp32", sweeps=3)
    got = _drain(srv, len(reqs))
    st = srv.stats()
    assert st["peak_bytes"] <= budget and st["resident"] == 0 and st["bytes_in_use"] == 0
    assert all(r["status"] == 0 for r in got.values())
    huge = np.zeros((400, 400, 400), np.float32)
    with pytest.raises(MtkError) as ei:
        srv.submit(99, huge, [np.ones((400, 8), np.float32)] * 3, "fp32", sweeps=1)
    assert ei.value.status == MTK_EBUDGET
    srv.close()


def test_failing_request_leaves_others_unchanged():
    from paper_2411_04785_amd.mttkrp import Server, MTK_ENOTSPD
    reqs = _reqs(4, seed=13)
    bad_q, bad_X, bad_init = 100, reqs[0][1], [f.copy() for f in reqs[0][2]]
    bad_init[1][:, 0] = 0.0          # zero column of B: mode-1 normal equations singular
    bad_init[2][:, 0] = 0.0
    srv = Server(0, budget_bytes=2 * 10**9, max_slots=3)
    srv.submit(reqs[0][0], reqs[0][1], reqs[0][2], "fp32", sweeps=3)
    srv.submit(bad_q, bad_X, bad_init, "fp32", sweeps=3)
    for q, X, init in reqs[1:]:
        srv.submit(q, X, init, "fp32", sweeps=3)
    got = _drain(srv, len(reqs) + 1)
    srv.close()
    assert got[bad_q]["status"] == MTK_ENOTSPD
    for q, X, init in reqs:
        assert got[q]["status"] == 0
        f, lam = _alone(X, init, "fp32", 3)
        assert all(np.array_equal(a, b) for a, b in zip(got[q]["factors"], f))


def test_mix_equals_alone_large_rank_dimension_tree():
    # R > 32 (no inversion riding in the Y launch) and K >= 8R (the sweep uses
    # the dimension tree), next to requests that do not use it.
    from paper_2411_04785_amd.mttkrp import Context, Server
    reqs = []
    for q, (dims, R) in enumerate((((40, 36, 320), 40), ((33, 30, 400), 48), ((50, 45, 60), 40), ((30, 28, 64), 8))):
        w = synth.Workload(f"t{q}", dims, min(R, 8), R, 1e-4, 2000 + q)
        reqs.append((q, synth.tensor(w, threads=2), synth.init_factors(w)))
    assert Context.sweep_uses_dimtree((40, 36, 320), 40, "fp32")
    assert not Context.sweep_uses_dimtree((50, 45, 60), 40, "fp32")
    srv = Server(0, budget_bytes=2 * 10**9, max_slots=4)
    for q, X, init in reqs:
        srv.submit(q, X, init, "fp32", sweeps=3)
    got = _drain(srv, len(reqs))
    srv.close()
    for q, X, init in reqs:
        assert got[q]["status"] == 0
        f, lam = _alone(X, init, "fp32", 3)
        for a, b in zip(got[q]["factors"], f):
            assert np.array_equal(a, b), q
        assert np.array_equal(got[q]["lambda"], lam), q
