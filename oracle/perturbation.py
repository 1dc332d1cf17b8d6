"""First-order perturbation theory in Fock space, FP64 (test infrastructure: the oracle of the
first-order MPS-LCC sweep; nothing here is used by the library).

Theory section, the perturbation series with zeroth-order Hamiltonian H0 and perturbation U:
Phi1 solves the first-order equation (H0 - E0) Phi1 = -Q (U - E1) Phi0 with Q = 1 - |Phi0><Phi0|
and <Phi0|Phi1> = 0, and the Wigner 2n+1 expressions give, for n = 1,
    E2 = <Phi0| U |Phi1>,   E3 = <Phi1| U |Phi1> - E1 <Phi1|Phi1>.
Projector approximation (same section): with H0~ = P H0 P + Q H0 Q and U~ = H - H0~ the
first-order equation keeps its operator and its right-hand side becomes -Q H Phi0 (the printed
sign is garbled; the minus follows from -Q U~ Phi0 = -Q H Phi0 since Q Phi0 = 0), and
E2 = <Phi0| H |Phi1>.  Both are the operator O of `first_order`: O = U or O = H.

The equation is solved directly: Q (H0 - E0) Q restricted to the orthogonal complement of Phi0
(an orthonormal basis of it from a complete QR factorisation) is a plain dense system.
`rayleigh_schrodinger` is the textbook spectral form of E2 and E3 (sums over the eigenstates of
H0) for a non-degenerate ground state, a second route to the same numbers.
"""
from __future__ import annotations

import numpy as np


def complement_basis(phi0: np.ndarray) -> np.ndarray:
    """Orthonormal columns spanning the orthogonal complement of the unit vector phi0."""
    q, _ = np.linalg.qr(np.column_stack([phi0, np.eye(phi0.size)[:, : phi0.size - 1]]), mode="complete")
    # the first column of q is +-phi0; the others span its complement
    return q[:, 1:]


def first_order(h0: np.ndarray, op: np.ndarray, u: np.ndarray, phi0: np.ndarray) -> dict:
    """Phi1 of (H0 - E0) Phi1 = -Q O Phi0 (Phi1 orthogonal to Phi0), E0 = <Phi0|H0|Phi0>, and the
    energies E2 = <Phi0|O|Phi1>, E3 = <Phi1|U|Phi1> - E1 <Phi1|Phi1> with E1 = <Phi0|U|Phi0>.
    Dense matrices of the sector; phi0 is normalised here."""
    phi0 = phi0 / np.linalg.norm(phi0)
    e0 = float(phi0 @ h0 @ phi0)
    e1 = float(phi0 @ u @ phi0)
    c = float(phi0 @ op @ phi0)
    B = complement_basis(phi0)
    A = B.T @ (h0 - e0 * np.eye(h0.shape[0])) @ B
    rhs = -(B.T @ (op @ phi0))  # B^T Q = B^T
    y = np.linalg.solve(A, rhs)
    phi1 = B @ y
    e2 = float(phi0 @ op @ phi1)
    e3 = float(phi1 @ u @ phi1) - e1 * float(phi1 @ phi1)
    return {"e0": e0, "e1": e1, "c": c, "phi1": phi1, "e2": e2, "e3": e3,
            "lambda_min": float(np.linalg.eigvalsh(A)[0])}


def hylleraas(h0: np.ndarray, op: np.ndarray, phi0: np.ndarray, phi: np.ndarray) -> float:
    """J[Phi] = <Phi|H0 - E0|Phi> + 2 <Phi|Q O|Phi0> for Phi orthogonal to Phi0 (stationary, and
    equal to E2, at Phi1; a minimum when Q (H0 - E0) Q is positive on the complement)."""
    phi0 = phi0 / np.linalg.norm(phi0)
    e0 = float(phi0 @ h0 @ phi0)
    qo = op @ phi0 - phi0 * float(phi0 @ op @ phi0)
    return float(phi @ h0 @ phi) - e0 * float(phi @ phi) + 2.0 * float(phi @ qo)


def rayleigh_schrodinger(h0: np.ndarray, u: np.ndarray) -> dict:
    """E0..E3 of the lowest eigenstate of H0 by the spectral sums of textbook RS perturbation
    theory:  E2 = -sum_k |U_k0|^2 / (E_k - E_0),
             E3 = sum_{k,m} U_0k (U_km - E1 delta_km) U_m0 / ((E_k - E_0)(E_m - E_0)),  k, m != 0."""
    w, V = np.linalg.eigh(h0)
    if w[1] - w[0] < 1e-8:
        raise ValueError("degenerate ground state of H0")
    Ut = V.T @ u @ V
    e1 = float(Ut[0, 0])
    d = w[1:] - w[0]
    u0 = Ut[1:, 0]
    e2 = -float(np.sum(u0 * u0 / d))
    t = u0 / d
    e3 = float(t @ (Ut[1:, 1:] - e1 * np.eye(d.size)) @ t)
    return {"e0": float(w[0]), "e1": e1, "e2": e2, "e3": e3, "phi0": V[:, 0]}
