"""GPU parity of batched sketches: one persistent launch over many problems,
graph replay, and the schedule autotuner, all through the C ABI.

Bit-exact comparisons use inputs whose results are unique: FP32 mode on
integer-valued A (exact sums, one final rounding), and FP16 modes with one
unit per problem (one rounding site and one FP16 atomic per entry).  The
rest is held to the same relative Frobenius bounds as single applies (1e-5
FP32, 4e-3 FP16).
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads
from oracle import model
from oracle.sketch import apply_f64

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2606_20195_amd import (ACC_F16_DITHER, ACC_F16_RN, ACC_F16_SR, ACC_F32, Batch, Sketch,  # noqa: E402
                                  clear_tuning, load_tuning, tune_batch)

DEV = "cuda:0"


def _specs(shapes, rounding, dtype, integer=False, lim=6, seed0=100):
    specs, hosts = [], []
    for k, (m, n, d, s) in enumerate(shapes):
        if integer:
            A = workloads.integers(m, n, seed=seed0 + k, lim=lim).astype(dtype)
        elif k % 5 == 0:
            A = workloads.coherent(m, n, seed0 + k, dtype)
        else:
            A = workloads.gaussian(m, n, seed0 + k, dtype)
        out_dt = torch.float32 if rounding == ACC_F32 else torch.float16
        SA = torch.full((d, n + (n & 1)), float("nan"), dtype=out_dt, device=DEV)[:, :n]
        specs.append(dict(A=torch.from_numpy(A).to(DEV), SA=SA, d=d, s=s, seed=7 * k + 1, rounding=rounding,
                          epoch=k))
        hosts.append(A)
    return specs, hosts


MIXED = [(5000, 8, 32, 4), (70000, 64, 256, 4), (4096, 16, 64, 4), (33333, 33, 132, 4), (12000, 128, 512, 4),
         (9000, 100, 400, 4), (65, 40, 160, 4), (150000, 32, 128, 4)]


def _rel(got, ref):
    return np.linalg.norm(got - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("rounding", [ACC_F16_RN, ACC_F16_SR, ACC_F16_DITHER])
def test_batched_fp16_matches_oracle(rounding):
    specs, hosts = _specs(MIXED, rounding, np.float16)
    b = Batch(specs)
    b.apply()
    torch.cuda.synchronize()
    for sp, A in zip(specs, hosts):
        ref = apply_f64(A, sp["d"], sp["s"], sp["seed"])
        assert _rel(sp["SA"].double().cpu().numpy(), ref) <= 4e-3


def test_batched_fp32_integer_is_bit_exact_mixed_s():
    shapes = [(5000, 8, 32, 4), (20000, 64, 256, 8), (4096, 16, 48, 3), (30000, 33, 132, 1), (7000, 40, 160, 2)]
    specs, hosts = _specs(shapes, ACC_F32, np.float32, integer=True)
    b = Batch(specs)                 # s = 3 forces one block per workgroup for the batch
    b.apply()
    torch.cuda.synchronize()
    for sp, A in zip(specs, hosts):
        ref = model.apply_f32_exact_int(A, sp["d"], sp["s"], sp["seed"])
        assert np.array_equal(sp["SA"].cpu().numpy(), ref)


@pytest.mark.parametrize("rounding", [ACC_F16_RN, ACC_F16_SR, ACC_F16_DITHER])
def test_batched_fp16_one_unit_is_bit_exact(rounding):
    shapes = [(3000, 24, 96, 4), (4096, 64, 256, 4), (1000, 7, 28, 4), (2500, 130, 520, 4)]
    specs, hosts = _specs(shapes, rounding, np.float16, integer=True)
    b = Batch(specs, chunk_rows=4096)
    b.apply()
    torch.cuda.synchronize()
    for sp, A in zip(specs, hosts):
        got = sp["SA"].cpu().numpy().view(np.uint16)
        ref = model.apply_f16_model(A, sp["d"], sp["s"], sp["seed"], rounding, sp["epoch"],
                                    chunk_rows=A.shape[0]).view(np.uint16)
        assert np.array_equal(got, ref)


def test_batched_equals_single_apply():
    specs, hosts = _specs(MIXED[:5], ACC_F32, np.float16, integer=True, lim=4)
    b = Batch(specs, chunk_rows=2048)
    b.apply()
    torch.cuda.synchronize()
    for sp in specs:
        sk = Sketch(sp["A"].shape[0], sp["d"], sp["s"], sp["seed"], ACC_F32)
        single = sk.apply(sp["A"])
        torch.cuda.synchronize()
        assert torch.equal(single, sp["SA"])


def test_graph_replay_equals_eager():
    specs, hosts = _specs(MIXED, ACC_F32, np.float32, integer=True)
    b = Batch(specs)
    b.apply()
    torch.cuda.synchronize()
    eager = [sp["SA"].clone() for sp in specs]
    for rep in range(4):
        for sp in specs:                       # eager work between replays
            sp["SA"].fill_(float(rep) + 0.5)
        torch.cuda.synchronize()
        b.graph()
        torch.cuda.synchronize()
        for sp, e in zip(specs, eager):
            assert torch.equal(sp["SA"], e), rep


def test_every_schedule_gives_the_same_fp32_bits():
    specs, hosts = _specs(MIXED[:6], ACC_F32, np.float32, integer=True)
    refs = [model.apply_f32_exact_int(A, sp["d"], sp["s"], sp["seed"]) for sp, A in zip(specs, hosts)]
    for chunk, waves in [(2048, 4), (4096, 8), (8192, 8), (16384, 4)]:
        b = Batch(specs, chunk_rows=chunk, waves=waves)
        b.apply()
        torch.cuda.synchronize()
        assert b.schedule()["chunk_rows"] == chunk
        for sp, ref in zip(specs, refs):
            assert np.array_equal(sp["SA"].cpu().numpy(), ref), (chunk, waves)
        b.close()


def test_tuners_write_and_reload_their_choice(tmp_path):
    clear_tuning()
    specs, hosts = _specs(MIXED[:4], ACC_F16_RN, np.float16)
    path = str(tmp_path / "tune.json")
    best = tune_batch(specs, cache_path=path)
    assert best["chunk_rows"] in (2048, 4096, 8192, 16384) and best["waves"] in (4, 8, 16)
    b = Batch(specs)                           # planned from the table
    assert b.schedule()["chunk_rows"] == best["chunk_rows"]
    b.apply()
    torch.cuda.synchronize()
    for sp, A in zip(specs, hosts):
        assert _rel(sp["SA"].double().cpu().numpy(), apply_f64(A, sp["d"], sp["s"], sp["seed"])) <= 4e-3
    # single-apply tuner: the planner then uses the tuned schedule
    A = workloads.integers(50000, 64, seed=3, lim=5).astype(np.float32)
    sk = Sketch(50000, 256, 4, 5, ACC_F32)
    Ad = torch.from_numpy(A).to(DEV)
    tuned = sk.tune(Ad, cache_path=path)
    plan = sk.plan(0, 50000, 64)
    assert (plan["block_group"], plan["waves"]) == (tuned["block_group"], tuned["waves"])
    SA = sk.apply(Ad)
    torch.cuda.synchronize()
    assert np.array_equal(SA.cpu().numpy(), model.apply_f32_exact_int(A, 256, 4, 5))
    clear_tuning()
    assert load_tuning(path) >= 2
    clear_tuning()


@pytest.mark.parametrize("rounding", [ACC_F16_RN, ACC_F16_DITHER])
def test_batched_real_valued_one_unit_matches_the_model(rounding):
    """Gaussian and coherent (outlier) problems, one unit each: every
    problem's FP16 result equals the oracle's fixed-point model with the
    batch's schedule (8-column tiles for n <= 16, 32 otherwise)."""
    shapes = [(3000, 8, 32, 4), (4000, 16, 64, 4), (2500, 40, 160, 4), (3500, 12, 48, 4), (1500, 64, 256, 4)]
    specs, hosts = _specs(shapes, rounding, np.float16, seed0=300)
    b = Batch(specs, chunk_rows=4096)
    b.apply()
    torch.cuda.synchronize()
    sch = b.schedule()
    for sp, A in zip(specs, hosts):
        nt = 8 if A.shape[1] <= 16 else 32
        got = sp["SA"].cpu().numpy().view(np.uint16)
        ref = model.apply_f16_model(A, sp["d"], sp["s"], sp["seed"], rounding, sp["epoch"], chunk_rows=4096,
                                    waves=sch["waves"], block_group=sch["block_group"], col_tile=nt)
        bad = np.flatnonzero(got != ref.view(np.uint16))
        assert bad.size == 0, (A.shape, bad[:8])
