"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws matrices and vectors only; it holds none of the sketching
method's arithmetic.  Every generator is numpy PCG64 in FP64 followed by a
round-to-nearest cast to the storage dtype, row-major.

Workload families (shapes and value distributions follow the paper's test
problems, Section 5):
  gaussian     iid N(0,1): the incoherent case (Section 5.2).
  coherent     tau * N(0,1) with the first n rows replaced by c * I_n: an
               identity-like, high-leverage block over a weak dense tail
               (the coherent construction of Section 5.3, here with the
               identity rows on top and scaled by c; tau = 1e-3, c = 100).
  spikes       zeros except n unit entries A[k * (m // n), k]: every column
               direction sits on one row (the adversarial identity input of
               Section 5.2), spread evenly over the rows.
  integers     uniform integers in [-lim, lim]: inputs whose partial sums are
               exact in FP32, for bit-exact checks.
  table1       the coherent adversarial least-squares problem of Section 5.3
               (Table 1): A = [I_n; tau G / sqrt(m - n)], b = [x* + eta;
               (tau G / sqrt(m - n)) x*] with eta = noise * N(0,1), the rows
               of A and b permuted together.
"""
from __future__ import annotations

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(m, n, seed, dtype=np.float32):
    return rng(seed).standard_normal((m, n)).astype(dtype)


def coherent(m, n, seed, dtype=np.float32, tau=1e-3, top=100.0):
    A = tau * rng(seed).standard_normal((m, n))
    k = min(m, n)
    A[:k, :] = 0.0
    A[np.arange(k), np.arange(k)] = top
    return A.astype(dtype)


def spikes(m, n, dtype=np.float32):
    A = np.zeros((m, n), dtype=dtype)
    step = max(m // n, 1)
    for k in range(min(n, m)):
        A[(k * step) % m, k] = 1
    return A


def integers(m, n, seed, lim=8, dtype=np.float32):
    return rng(seed).integers(-lim, lim + 1, size=(m, n)).astype(dtype)


def table1(m, n, seed, dtype=np.float32, tau=1e-3, noise=0.5):
    """(A, b, x*): the Section 5.3 construction at m x n; A stored in
    `dtype`, b in FP64 from the FP64 tail (before the cast)."""
    g = rng(seed)
    tail = g.standard_normal((m - n, n)) * (tau / np.sqrt(m - n))
    xs = g.standard_normal(n)
    eta = noise * g.standard_normal(n)
    perm = g.permutation(m)
    A = np.empty((m, n))
    b = np.empty(m)
    A[perm[:n]] = np.eye(n)
    A[perm[n:]] = tail
    b[perm[:n]] = xs + eta
    b[perm[n:]] = tail @ xs
    return A.astype(dtype), b, xs


def family(name, m, n, seed, dtype=np.float32):
    if name == "gaussian":
        return gaussian(m, n, seed, dtype)
    if name == "coherent":
        return coherent(m, n, seed, dtype)
    if name == "spikes":
        return spikes(m, n, dtype)
    if name == "integers":
        return integers(m, n, seed, dtype=dtype)
    if name == "table1":
        return table1(m, n, seed, dtype)[0]
    raise ValueError(name)


# ---- the named configurations -------------------------------------------

SMALL = dict(m=16384, n=32, d=256, s=4, seed=0)          # correctness case
APPLY = dict(m=4194304, n=64, d=1024)                    # single sketch_apply
LSQ = dict(m=2097152, n=256, d=1024, s=4)                # least squares


def small_case():
    """16384 x 32 FP32 Gaussian (PCG64 seed 0), d = 256, s = 4."""
    return gaussian(SMALL["m"], SMALL["n"], SMALL["seed"])


def apply_case(kind, dtype=np.float16, m=APPLY["m"], n=APPLY["n"]):
    """4194304 x 64 input of one family: gaussian (seed 0), coherent (seed 1:
    1e-3 N(0,1) with rows 0..63 = 100 I), spikes."""
    if kind == "gaussian":
        return gaussian(m, n, 0, dtype)
    if kind == "coherent":
        return coherent(m, n, 1, dtype)
    if kind == "spikes":
        return spikes(m, n, dtype)
    raise ValueError(kind)


def ls_case(m=LSQ["m"], n=LSQ["n"], dtype=np.float16, noise=1e-6):
    """Coherent least-squares problem: A = 1e-3 N(0,1) (seed 2) with rows
    0..n-1 = 100 I, stored in `dtype`; x* ~ N(0,1) (seed 3); b = A x* in FP64
    (from the stored A) + noise * N(0,1) (seed 4)."""
    A = coherent(m, n, 2, dtype)
    xs = rng(3).standard_normal(n)
    b = A.astype(np.float64) @ xs + noise * rng(4).standard_normal(m)
    return A, b, xs


def batch_specs(count=512, seed=5, mlog=(12, 20), ns=(8, 16, 32, 64, 128)):
    """Shapes of the batched workload: m = floor(2**(12 + 8U)), n uniform in
    {8,...,128}, d = 4n, s = 4, family coherent iff p % 10 == 0."""
    g = rng(seed)
    lo, hi = mlog
    U = g.random(count)
    ms = np.floor(2.0 ** (lo + (hi - lo) * U)).astype(np.int64)
    nn = g.choice(np.array(ns), size=count)
    return [dict(p=p, m=int(ms[p]), n=int(nn[p]), d=4 * int(nn[p]), s=4,
                 kind="coherent" if p % 10 == 0 else "gaussian", seed=1000 + p)
            for p in range(count)]


def arrivals(count, rate=200.0, seed=6, mlog=(14, 22), ns=(16, 32, 64, 128, 256)):
    """Poisson request stream: exponential gaps at `rate` per second, m
    log-uniform on [2**14, 2**22], n uniform in {16,...,256}, d = 4n."""
    g = rng(seed)
    gaps = g.exponential(1.0 / rate, size=count)
    lo, hi = mlog
    ms = np.floor(2.0 ** (lo + (hi - lo) * g.random(count))).astype(np.int64)
    nn = g.choice(np.array(ns), size=count)
    t = np.cumsum(gaps)
    return [dict(t=float(t[k]), m=int(ms[k]), n=int(nn[k]), d=4 * int(nn[k]), s=4,
                 seed=10_000 + k, kind="coherent" if k % 10 == 0 else "gaussian")
            for k in range(count)]
