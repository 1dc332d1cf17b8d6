"""The local linear problem of MPS-LCC and its solution, FP64.

The first-order equation of the RS hierarchy (Theory section, eq. for Phi^(n)) restricted
to the two-site space reads  Q (H_eff - E0) Q x = Q b, with Q = 1 - v v^T the complement of
the zeroth-order state's image v in that space (or Q = 1 when no v is given).  Its solution
is the stationary point of the local Hylleraas functional (Implementation section),
written here in the standard form J(x) = x^T A x - 2 b^T x; at the solution J = -b^T x.
The Implementation section names conjugate gradients as the local solver; `cg` is that
method in its textbook form (no preconditioner, x0 = 0 unless given).
"""
from __future__ import annotations

import numpy as np


def project(v, z):
    if v is None:
        return z
    return z - v * float(v @ z)


def make_operator(apply_heff, e0: float, v=None):
    """A z = Q (H_eff - e0) Q z on flat FP64 vectors."""
    def A(z):
        zq = project(v, z)
        return project(v, apply_heff(zq) - e0 * zq)
    return A


def hylleraas(A, x, b) -> float:
    return float(x @ A(x) - 2.0 * (b @ x))


def dense_solution(heff: np.ndarray, b: np.ndarray, e0: float, v=None):
    """x* in range(Q) with Q(H-e0)Q x* = Q b, by one dense LU solve (small problems).

    With Q = 1 - v v^T the system (Q(H-e0)Q + v v^T) x = Q b is non-singular whenever
    Q(H-e0)Q is positive definite on range(Q), and its solution has v^T x = 0.
    """
    n = heff.shape[0]
    A = heff - e0 * np.eye(n)
    if v is None:
        return np.linalg.solve(0.5 * (A + A.T), b)
    Av = A @ v
    vAv = float(v @ Av)
    QAQ = A - np.outer(v, Av) - np.outer(Av, v) + vAv * np.outer(v, v)
    QAQ = 0.5 * (QAQ + QAQ.T)
    return np.linalg.solve(QAQ + np.outer(v, v), project(v, b))


def cg(A, b: np.ndarray, x0=None, tol: float = 1e-13, max_iter: int = 5000, v=None):
    """Plain conjugate gradients on A x = Q b.  Returns (x, iterations, rel. residual, J history)."""
    bq = project(v, b)
    x = np.zeros_like(bq) if x0 is None else project(v, np.array(x0, dtype=np.float64))
    r = bq - A(x)
    p = r.copy()
    rr = float(r @ r)
    bn = float(np.sqrt(bq @ bq))
    hist = []
    if bn == 0.0:
        return x, 0, 0.0, hist
    it = 0
    while it < max_iter and np.sqrt(rr) > tol * bn:
        Ap = A(p)
        pAp = float(p @ Ap)
        if pAp <= 0.0:
            raise ArithmeticError("operator is not positive definite on the Krylov space")
        alpha = rr / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(float(-(x @ r) - (bq @ x)))  # J(x) = x^T A x - 2 b^T x = -x^T r - b^T x
    return x, it, float(np.sqrt(rr) / bn), hist


def lanczos_lowest(apply_heff, n: int, steps: int = 100, seed: int = 0):
    """Lowest Ritz value of H_eff and its residual norm (full re-orthogonalisation)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = rng.standard_normal(n)
    q /= np.linalg.norm(q)
    Qs = [q]
    alphas, betas = [], []
    for k in range(min(steps, n)):
        w = apply_heff(Qs[-1])
        a = float(Qs[-1] @ w)
        alphas.append(a)
        w = w - a * Qs[-1] - (betas[-1] * Qs[-2] if betas else 0.0)
        for qq in Qs:
            w -= qq * float(qq @ w)
        bnext = float(np.linalg.norm(w))
        if bnext < 1e-12 or k == min(steps, n) - 1:
            break
        betas.append(bnext)
        Qs.append(w / bnext)
    T = np.diag(alphas) + np.diag(betas[: len(alphas) - 1], 1) + np.diag(betas[: len(alphas) - 1], -1)
    th, S = np.linalg.eigh(T)
    u = np.array(Qs[: len(alphas)]).T @ S[:, 0]
    res = float(np.linalg.norm(apply_heff(u) - th[0] * u))
    return float(th[0]), res, u
