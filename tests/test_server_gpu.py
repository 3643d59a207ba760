"""GPU tests of the continuous-batching least-squares server.

Each result must be the same alone and in the mix: both are the FP64
least-squares solution of the stored A to the 1e-10 normal-equations
criterion, so they agree to well within 1e-9 relative (they may differ in the
last bits: atomics make the sketch's summation order vary).  The oracle
recomputes the criterion for every caller-supplied request.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads
from oracle.ls import ne_criterion

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2606_20195_amd import ACC_F16_RN, ACC_F32, Server, Sketch, SketchError  # noqa: E402
from paper_2606_20195_amd import footprint  # noqa: E402

DEV = "cuda:0"
GiB = 1 << 30

SHAPES = [(20000, 16, 64, np.float16), (150000, 64, 256, np.float16), (5000, 33, 132, np.float32),
          (80000, 128, 512, np.float16), (30000, 8, 32, np.float32), (120000, 40, 160, np.float16),
          (9000, 100, 400, np.float16), (60000, 24, 96, np.float32)]


def _problem(k, m, n, dtype):
    A = workloads.coherent(m, n, 500 + k, dtype) if k % 3 == 0 else workloads.gaussian(m, n, 500 + k, dtype)
    b = A.astype(np.float64) @ workloads.rng(600 + k).standard_normal(n) + 1e-6 * workloads.rng(700 + k).standard_normal(m)
    return A, b


def _req(k, m, n, d, dtype, Ad, bd):
    rounding = ACC_F16_RN if dtype == np.float16 else ACC_F32
    return Server.request(m, n, d, s=4, seed=k + 1, rounding=rounding, A=Ad, b=bd)


def test_results_alone_equal_results_in_the_mix():
    data = [(_problem(k, m, n, dt), (m, n, d, dt)) for k, (m, n, d, dt) in enumerate(SHAPES)]
    dev = [(torch.from_numpy(A).to(DEV), torch.from_numpy(b).to(DEV)) for (A, b), _ in data]
    alone = []
    for k, ((A, b), (m, n, d, dt)) in enumerate(data):
        sk = Sketch(m, d, 4, k + 1, ACC_F16_RN if dt == np.float16 else ACC_F32)
        x, info = sk.solve(*dev[k])
        assert info["converged"] == 1
        alone.append(x.cpu().numpy())
    srv = Server(4 * GiB, slots=3)
    tickets = []
    for k, ((A, b), (m, n, d, dt)) in enumerate(data):
        r, keep = _req(k, m, n, d, dt, *dev[k])
        tickets.append((srv.submit(r, keep), keep[2]))
    results = [(srv.wait(t), x) for t, x in tickets]
    stats = srv.stats()
    srv.close()
    for k, ((res, x), ((A, b), _)) in enumerate(zip(results, data)):
        assert res["status"] == 0 and res["converged"] == 1, res
        xm = x.cpu().numpy()
        assert ne_criterion(A, b, xm) <= 1.5e-10
        assert np.linalg.norm(xm - alone[k]) <= 1e-9 * np.linalg.norm(alone[k])
    # the requests overlapped on the device: some admission precedes an earlier request's completion
    spans = sorted((r["t_admit"], r["t_done"]) for r, _ in results)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))
    assert stats["completed"] == len(SHAPES) and stats["bytes_high_water"] <= stats["budget"]


def test_admission_by_footprint():
    # a budget that holds the two largest requests but not three
    data = [_problem(k, 150000, 64, np.float16) for k in range(5)]
    dev = [(torch.from_numpy(A).to(DEV), torch.from_numpy(b).to(DEV)) for A, b in data]
    reqs = [_req(k, 150000, 64, 256, np.float16, *dev[k]) for k in range(5)]
    fp = footprint(reqs[0][0])
    srv = Server(int(2.5 * fp), slots=4)
    tickets = [srv.submit(r, keep) for r, keep in reqs]
    res = [srv.wait(t) for t in tickets]
    stats = srv.stats()
    srv.close()
    assert stats["bytes_high_water"] <= 2 * ((fp + 255) // 256 * 256)
    for t in np.unique([r["t_admit"] for r in res]):
        running = sum(1 for r in res if r["t_admit"] <= t < r["t_done"])
        assert running <= 2
    admits = [r["t_admit"] for r in res]
    assert admits == sorted(admits)                       # first come, first admitted
    for (A, b), r, (_, keep) in zip(data, res, reqs):
        assert r["converged"] == 1
        assert ne_criterion(A, b, keep[2].cpu().numpy()) <= 1.5e-10


def test_oversized_request_is_refused_and_bad_requests_fail_cleanly():
    A, b = _problem(0, 100000, 64, np.float16)
    Ad, bd = torch.from_numpy(A).to(DEV), torch.from_numpy(b).to(DEV)
    r, keep = _req(0, 100000, 64, 256, np.float16, Ad, bd)
    srv = Server(footprint(r) // 2, slots=2)
    with pytest.raises(SketchError) as ei:
        srv.submit(r, keep)
    assert ei.value.code == -6
    srv.close()
    # a rank-deficient request completes with an error status and frees its memory
    A0 = A.copy()
    A0[:, 3] = 0
    Ad0 = torch.from_numpy(A0).to(DEV)
    srv = Server(4 * GiB, slots=2)
    r, keep = _req(1, 100000, 64, 256, np.float16, Ad0, bd)
    t = srv.submit(r, keep)
    res = srv.wait(t)
    assert res["status"] == -1
    good, keepg = _req(2, 100000, 64, 256, np.float16, Ad, bd)
    assert srv.wait(srv.submit(good, keepg))["status"] == 0
    assert srv.stats()["bytes_in_use"] == 0
    srv.close()


def test_generated_requests_converge_and_repeat():
    srv = Server(8 * GiB, slots=4)
    out = {}
    for rep in range(2):
        for k, (m, n) in enumerate([(1 << 16, 16), (300000, 128), (1 << 20, 64), (50000, 256)]):
            for gen in (1, 2):
                r, keep = Server.request(m, n, 4 * n, s=4, seed=k, rounding=ACC_F16_RN, gen=gen, gen_seed=10 * k + gen)
                out.setdefault((k, gen), []).append((srv.submit(r, keep), keep[2]))
    for key, runs in out.items():
        xs = []
        for t, x in runs:
            res = srv.wait(t)
            assert res["status"] == 0 and res["converged"] == 1 and res["crit"] <= 1e-10, (key, res)
            assert res["ms_ingest"] > 0
            xs.append(x.cpu().numpy())
        assert np.linalg.norm(xs[0] - xs[1]) <= 1e-9 * np.linalg.norm(xs[0])
    srv.close()
