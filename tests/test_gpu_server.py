"""Serving: continuous batching of CP-ALS requests (mtk_server_* through the C
ABI), every resident request advancing one mode update per scheduler step
through grouped launches.  Each request's result must be bitwise the same
in the mix as served alone, close to the FP64 oracle's CP-ALS, admission
must keep the server's device memory within the HBM budget, and a failing
request must not disturb the others."""

import sys

import numpy as np
import pytest

import oracle
from paper_2411_04785_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _reqs(n, seed=7, lo=32, hi=72, ranks=(8, 16)):
    g = np.random.default_rng(seed)
    out = []
    for q in range(n):
        dims = tuple(int(x) for x in g.integers(lo, hi + 1, 3))
        R = int(g.choice(ranks))
        w = synth.Workload(f"r{q}", dims, R, R, 1e-4, 1000 + q)
        out.append((q, synth.tensor(w, threads=2), synth.init_factors(w)))
    return out


def _drain(srv, n, timeout=120.0):
    import time
    got = {}
    t0 = time.time()
    while len(got) < n and time.time() - t0 < timeout:
        for r in srv.poll(timeout_s=1.0):
            got[r["id"]] = r
    assert len(got) == n, f"only {len(got)} of {n} finished"
    return got


def _served(reqs, prec, sweeps, slots=4, budget=2 * 10**9):
    from paper_2411_04785_amd.mttkrp import Server
    srv = Server(0, budget_bytes=budget, max_slots=slots)
    for q, X, init in reqs:
        srv.submit(q, X, init, prec, sweeps=sweeps)
    got = _drain(srv, len(reqs))
    st = srv.stats()
    srv.close()
    return got, st


def _same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a["factors"], b["factors"])) and \
        np.array_equal(a["lambda"], b["lambda"])


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mix_equals_alone(prec):
    # Uneven shapes and ranks (R 8..64, strided and contiguous reductions,
    # K % 4 != 0 for some) in one mix of 4 slots; each result equals the
    # same request served alone, bit for bit.
    reqs = _reqs(8, ranks=(8, 16, 32, 64))
    got, st = _served(reqs, prec, 4)
    _say(prec, "steps", st["steps"], "max batch", st["max_batch"])
    assert st["max_batch"] >= 2               # requests really shared steps
    for q, X, init in reqs:
        r = got[q]
        assert r["status"] == 0
        alone, _ = _served([(q, X, init)], prec, 4, slots=1)
        assert _same(r, alone[q]), q
        assert r["fit"] == alone[q]["fit"]
        assert 0.0 < r["fit"] <= 1.0


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_served_results_match_oracle(prec):
    # A seeded sample of requests against the oracle's CP-ALS from the same
    # start: the served fit (direct residual) and the reconstructed model.
    reqs = _reqs(5, seed=21, lo=32, hi=96, ranks=(8, 16, 32))
    got, _ = _served(reqs, prec, 6)
    for q, X, init in reqs:
        r = got[q]
        of, ol, ofits = oracle.cp_als(X, init, 6)
        model = oracle.reconstruct_slices(r["factors"], r["lambda"], 0, X.shape[0])
        ref = oracle.reconstruct_slices(of, ol, 0, X.shape[0])
        me = float(np.linalg.norm(model - ref) / np.linalg.norm(ref))
        _say(prec, q, X.shape, init[0].shape[1], f"fit {r['fit']:.9f} oracle {ofits[-1]:.9f} model {me:.2e}")
        assert r["status"] == 0
        assert abs(r["fit"] - ofits[-1]) <= 1e-4
        assert me <= 1e-3


def test_budget_admission_and_footprint():
    from paper_2411_04785_amd.mttkrp import Server, MtkError, MTK_EBUDGET
    reqs = _reqs(6, seed=9, lo=40, hi=60, ranks=(8,))
    # A budget for about three requests at a time: the arena (device bytes
    # actually allocated) must stay within it, so at most three are resident.
    big = max(X.nbytes for _, X, _ in reqs)
    budget = 3 * big + (8 << 20)
    srv = Server(0, budget_bytes=budget, max_slots=8)
    for q, X, init in reqs:
        srv.submit(q, X, init, "fp32", sweeps=3)
    got = _drain(srv, len(reqs))
    st = srv.stats()
    _say("budget", budget, st)
    assert st["device_bytes"] <= budget and st["peak_bytes_in_use"] <= budget
    assert st["resident"] == 0 and st["bytes_in_use"] == 0
    assert all(r["status"] == 0 for r in got.values())
    huge = np.zeros((400, 400, 400), np.float32)
    with pytest.raises(MtkError) as ei:
        srv.submit(99, huge, [np.ones((400, 8), np.float32)] * 3, "fp32", sweeps=1)
    assert ei.value.status == MTK_EBUDGET
    srv.close()


def test_large_request_admitted_after_small_ones_fill_the_arena():
    # The arena grows in chunks of budget / 8.  Small requests take a chunk;
    # the large one needs a chunk of its own size, which does not fit next
    # to theirs within the budget (budget = 16/15 of its bytes), so it waits
    # until they are gone, then the arena gives its free chunks back and
    # takes one of the request's size.
    from paper_2411_04785_amd.mttkrp import Server
    small = _reqs(3, seed=31, lo=32, hi=40, ranks=(8,))
    w = synth.Workload("big", (96, 90, 100), 8, 8, 1e-4, 77)
    big = (50, synth.tensor(w, threads=2), synth.init_factors(w))
    nbig = Server.request_bytes(big[1].shape, 8, "fp32")
    budget = nbig * 16 // 15 + 256
    assert all(Server.request_bytes(X.shape, 8, "fp32") <= budget // 8 for _, X, _ in small)
    srv = Server(0, budget_bytes=budget, max_slots=4)
    for q, X, init in small + [big]:
        srv.submit(q, X, init, "fp32", sweeps=2)
    got = _drain(srv, 4)
    st = srv.stats()
    srv.close()
    assert all(r["status"] == 0 for r in got.values())
    assert st["device_bytes"] <= budget


def test_failing_request_leaves_others_unchanged():
    from paper_2411_04785_amd.mttkrp import MTK_ENOTSPD
    reqs = _reqs(4, seed=13)
    bad_q, bad_X, bad_init = 100, reqs[0][1], [f.copy() for f in reqs[0][2]]
    bad_init[1][:, 0] = 0.0          # zero column of B and C: mode-1 normal equations singular
    bad_init[2][:, 0] = 0.0
    mix = [reqs[0], (bad_q, bad_X, bad_init)] + reqs[1:]
    got, _ = _served(mix, "fp32", 3, slots=3)
    assert got[bad_q]["status"] == MTK_ENOTSPD
    for q, X, init in reqs:
        assert got[q]["status"] == 0
        alone, _ = _served([(q, X, init)], "fp32", 3, slots=1)
        assert _same(got[q], alone[q]), q


def test_large_ranks_and_zero_sweeps():
    # R up to 128 (eight column tiles, the largest inversion), next to a
    # request with no sweep (its fit is the initial model's).
    reqs = []
    for q, (dims, R) in enumerate((((40, 36, 64), 128), ((33, 30, 40), 96), ((50, 45, 60), 40))):
        w = synth.Workload(f"t{q}", dims, min(R, 8), R, 1e-4, 2000 + q)
        reqs.append((q, synth.tensor(w, threads=2), synth.init_factors(w)))
    got, _ = _served(reqs, "fp32", 2)
    for q, X, init in reqs:
        assert got[q]["status"] == 0
        alone, _ = _served([(q, X, init)], "fp32", 2, slots=1)
        assert _same(got[q], alone[q]), q
    q, X, init = reqs[2]
    z, _ = _served([(7, X, init)], "fp32", 0, slots=1)
    assert z[7]["status"] == 0
    assert abs(z[7]["fit"] - oracle.fit(X, init, np.ones(init[0].shape[1]))) <= 1e-10


def test_bf16x6_is_not_served():
    # The grouped serving kernels are built for FP32 and bf16x3 requests.
    from paper_2411_04785_amd.mttkrp import Server, MtkError, MTK_EINVAL
    q, X, init = _reqs(1, seed=3)[0]
    srv = Server(0, budget_bytes=10**9, max_slots=2)
    with pytest.raises(MtkError) as ei:
        srv.submit(q, X, init, "bf16x6", sweeps=1)
    assert ei.value.status == MTK_EINVAL
    srv.close()
