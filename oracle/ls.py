"""Least-squares references in FP64.

The paper's downstream solver is sketch-and-solve: form SA and Sb, take a
reduced QR of SA and solve min ||SAx - Sb|| with a triangular solve (Section
5.1); the reported quality is ||Ax - b|| / ||b|| (Section 5.1) and kappa(SA)
(Section 5.1, Table 1).  It names sketch-and-precondition only as related and
future work (Section 3.1; Section 6).  The library's solver takes R from the
QR of SA as a right preconditioner for LSQR (Paige and Saunders, ACM TOMS
8(1), 1982, Section 4 "LSQR") inside FP64 iterative refinement.  That solver
converges to the exact least-squares solution, which has a plain definition;
so the parity reference here is that definition, computed by Householder QR
(Golub and Van Loan, Section 5.3) in FP64.

Functions
  householder_lstsq   argmin ||Ax - b||_2, FP64 Householder QR.
                      Pinned by: numpy.linalg.lstsq (LAPACK); exact solution
                      of consistent systems.
  lsqr                Plain LSQR iterates (Paige-Saunders 1982, Section 4,
                      steps 1-6).  Pinned by: scipy.sparse.linalg.lsqr
                      iterates on the same operator.
  ne_criterion        ||A^T r|| / (||A||_F ||r||) (Paige-Saunders stopping
                      rule S2), the library's reading of "1e-10 residual".
  sketch_solve_model  The sketch-and-precondition + refinement driver in
                      FP64, used to check the algorithm's design on the CPU.
                      Its output is held to householder_lstsq.
"""
from __future__ import annotations

import numpy as np


def householder_qr(A):
    """Reduced QR by Householder reflections; returns (reflectors, R)."""
    A = np.array(A, dtype=np.float64, copy=True)
    m, n = A.shape
    vs = []
    R = A
    for k in range(n):
        x = R[k:, k].copy()
        nrm = np.linalg.norm(x)
        alpha = -nrm if x[0] > 0 else nrm
        v = x.copy()
        v[0] -= alpha
        vv = float(v @ v)
        if vv > 0:
            R[k:, k:] -= np.outer(v, (2.0 / vv) * (v @ R[k:, k:]))
        vs.append((v, vv))
    return vs, np.triu(R[:n, :n])


def householder_lstsq(A, b):
    """argmin ||Ax - b||_2 in FP64 (A upcast exactly)."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    vs, R = householder_qr(A)
    y = b.copy()
    for k, (v, vv) in enumerate(vs):
        if vv > 0:
            y[k:] -= (2.0 / vv) * (v @ y[k:]) * v
    return back_substitute(R, y[:n])


def back_substitute(R, y):
    n = R.shape[0]
    x = np.zeros(n)
    for k in range(n - 1, -1, -1):
        x[k] = (y[k] - R[k, k + 1:] @ x[k + 1:]) / R[k, k]
    return x


def ne_criterion(A, b, x, fro=None):
    """||A^T r|| / (||A||_F ||r||) with r = b - Ax, all FP64."""
    A = np.asarray(A, dtype=np.float64)
    r = np.asarray(b, dtype=np.float64) - A @ x
    rn = np.linalg.norm(r)
    if rn == 0:
        return 0.0
    fro = np.linalg.norm(A) if fro is None else fro
    return float(np.linalg.norm(A.T @ r) / (fro * rn))


def lsqr(matvec, rmatvec, b, n, iters):
    """LSQR (Paige-Saunders 1982, Section 4): k iterations from x0 = 0.

    matvec(v) = A v, rmatvec(u) = A^T u.  Returns the list of iterates
    x_1..x_iters (no damping, no reorthogonalisation).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n)
    beta = np.linalg.norm(b)
    u = b / beta if beta > 0 else b.copy()
    v = rmatvec(u)
    alpha = np.linalg.norm(v)
    v = v / alpha if alpha > 0 else v
    w = v.copy()
    phibar, rhobar = beta, alpha
    out = []
    for _ in range(iters):
        u = matvec(v) - alpha * u
        beta = np.linalg.norm(u)
        if beta > 0:
            u = u / beta
        v = rmatvec(u) - beta * v
        alpha = np.linalg.norm(v)
        if alpha > 0:
            v = v / alpha
        rho = np.hypot(rhobar, beta)
        c, s = rhobar / rho, beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        x = x + (phi / rho) * w
        w = v - (theta / rho) * w
        out.append(x.copy())
    return out


def sketch_solve_model(A, b, SA, Sb, tol=1e-10, inner_iters=30, max_refine=10):
    """FP64 model of the sketch-and-precondition refinement driver.

    R from QR(SA); x0 = R^{-1} Q^T Sb (sketch-and-solve, Section 5.1); then
    repeat: r = b - A x; stop when ne_criterion <= tol (or ||r|| <= tol ||b||);
    LSQR on min ||A R^{-1} y - r/||r|| ||; x += R^{-1} y ||r||.
    Returns (x, number of refinement steps).
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = A.shape[1]
    Q, R = np.linalg.qr(np.asarray(SA, dtype=np.float64))
    x = np.linalg.solve(R, Q.T @ np.asarray(Sb, dtype=np.float64))
    fro = np.linalg.norm(A)
    bn = np.linalg.norm(b)
    Rinv = lambda y: np.linalg.solve(R, y)            # noqa: E731
    RinvT = lambda z: np.linalg.solve(R.T, z)         # noqa: E731
    for k in range(max_refine + 1):
        r = b - A @ x
        rn = np.linalg.norm(r)
        if rn <= tol * bn or ne_criterion(A, b, x, fro) <= tol:
            return x, k
        if k == max_refine:
            break
        its = lsqr(lambda y: A @ Rinv(y), lambda z: RinvT(A.T @ z), r / rn, n, inner_iters)
        x = x + Rinv(its[-1]) * rn
    return x, max_refine
