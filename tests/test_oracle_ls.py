"""Pins of the oracle's least-squares references (CPU only)."""
import numpy as np
import scipy.sparse.linalg as spla

import workloads
from oracle import native
from oracle.ls import householder_lstsq, lsqr, ne_criterion, sketch_solve_model
from oracle.sketch import apply_f64


def test_householder_matches_lapack():
    for A in (workloads.gaussian(300, 20, 1, np.float64), workloads.coherent(500, 12, 2, np.float64)):
        b = np.random.default_rng(3).standard_normal(A.shape[0])
        ref = np.linalg.lstsq(A, b, rcond=None)[0]
        assert np.allclose(householder_lstsq(A, b), ref, rtol=1e-10, atol=1e-12)
        assert np.allclose(native.lstsq(A, b), ref, rtol=1e-10, atol=1e-12)


def test_consistent_system_recovers_solution():
    A = workloads.coherent(2000, 16, 4, np.float16)
    xs = np.random.default_rng(5).standard_normal(16)
    b = A.astype(np.float64) @ xs
    assert np.allclose(householder_lstsq(A, b), xs, rtol=0, atol=1e-10)
    assert np.allclose(native.lstsq(A, b), xs, rtol=0, atol=1e-10)


def test_lsqr_iterates_match_scipy():
    A = workloads.gaussian(200, 15, 6, np.float64)
    b = np.random.default_rng(7).standard_normal(200)
    mine = lsqr(lambda v: A @ v, lambda u: A.T @ u, b, 15, 12)
    for k in (1, 3, 7, 12):
        ref = spla.lsqr(A, b, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        assert np.allclose(mine[k - 1], ref, rtol=1e-9, atol=1e-12)


def test_refinement_driver_reaches_the_lstsq_solution():
    m, n, d, s = 8192, 16, 64, 4
    A, b, _ = workloads.ls_case(m, n, dtype=np.float16)
    SA = apply_f64(A, d, s, 0)
    Sb = apply_f64(b[:, None], d, s, 0)[:, 0]
    x, steps = sketch_solve_model(A, b, SA, Sb, tol=1e-10)
    ref = np.linalg.lstsq(A.astype(np.float64), b, rcond=None)[0]
    assert ne_criterion(A, b, x) <= 1e-10
    assert np.linalg.norm(x - ref) <= 1e-8 * np.linalg.norm(ref)
    assert steps >= 1
