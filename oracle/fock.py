"""O1: brute-force Fock-space oracle.

The Hamiltonian is the one- plus two-body operator of the Theory section (partitioned
Hamiltonian equation) with the conventional 1/2 on the two-body part:

    H = sum h_ij a+_{i s} a_{j s} + 1/2 sum (ij|kl) a+_{i s} a+_{k t} a_{l t} a_{j s}
        + sum u_i n_{i up} n_{i dn} + e_const

Spin orbital p = 2 i + s (s = 0 up, 1 down).  A Fock state is a bit mask over spin
orbitals and means prod_{p ascending, occupied} a+_p |vac>, so a+_p / a_p carry the sign
(-1)^(number of occupied q < p).  This is the ordering under which the site-by-site
tensor product of local states |0>,|up>,|dn>,|updn> (|updn> = a+_up a+_dn |0>) is the
Fock state itself, which is how the MPS equation's physical indices are read here.

H_eff of the two-site block is P^T H P where the columns of P are the Fock-space vectors
|a>_L |s1> |s2> |b>_R of the canonical MPS (Implementation section: the derivative of
<Psi|H|Phi> with respect to the local tensor is the graph with that tensor removed; for an
isometric P that is exactly P^T H P).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

# local state -> (n_up, n_dn)
_LOCAL_OCC = ((0, 0), (1, 0), (0, 1), (1, 1))


def sector_basis(n_orb: int, n_elec: int, two_sz: int) -> np.ndarray:
    """Sorted bit masks of all Fock states with N electrons and 2Sz = n_up - n_dn."""
    n_up = (n_elec + two_sz) // 2
    n_dn = (n_elec - two_sz) // 2
    if n_up + n_dn != n_elec or n_up < 0 or n_dn < 0:
        return np.zeros(0, dtype=np.int64)
    out = []
    for ups in itertools.combinations(range(n_orb), n_up):
        mu = sum(1 << (2 * i) for i in ups)
        for dns in itertools.combinations(range(n_orb), n_dn):
            out.append(mu | sum(1 << (2 * i + 1) for i in dns))
    return np.array(sorted(out), dtype=np.int64)


def _below_parity(states: np.ndarray, p: int) -> np.ndarray:
    mask = np.int64((1 << p) - 1)
    return np.bitwise_count(states & mask).astype(np.int64) & 1


def apply_op(states: np.ndarray, amps: np.ndarray, p: int, dagger: bool):
    """Apply a+_p (dagger) or a_p to a batch of basis states with amplitudes."""
    bit = np.int64(1 << p)
    occ = (states & bit) != 0
    ok = ~occ if dagger else occ
    st = states[ok]
    sign = 1.0 - 2.0 * _below_parity(st, p)
    st = st ^ bit
    return st, amps[ok] * sign, ok


def in_part(spec: dict, ops) -> bool:
    """Theory section, partitioned Hamiltonian: with orbital classes (0 core, 1 active, 2
    virtual) H0 keeps the operator strings that transfer no electron between the classes (in
    every class as many creators as annihilators) and U = H - H0 the others.  spec['part']: 0
    the whole H, 1 H0, 2 U."""
    part = spec.get("part", 0)
    if not part:
        return True
    bal = [0, 0, 0]
    for p, dag in ops:
        bal[int(spec["orb_class"][p // 2])] += 1 if dag else -1
    keeps = bal == [0, 0, 0]
    return keeps if part == 1 else not keeps


def constant(spec: dict) -> float:
    """The constant term: part of H and H0, not of U."""
    return 0.0 if spec.get("part", 0) == 2 else float(spec.get("e_const", 0.0))


def operator_strings(spec: dict):
    """Yield (coefficient, [(spin_orbital, dagger), ...]) in written operator order (only the
    strings of the selected part of the Hamiltonian, see in_part)."""
    for coef, ops in _all_operator_strings(spec):
        if in_part(spec, ops):
            yield coef, ops


def _all_operator_strings(spec: dict):
    n = spec["n_orb"]
    h = spec["h"]
    for i in range(n):
        for j in range(n):
            if h[i, j] != 0.0:
                for s in (0, 1):
                    yield h[i, j], [(2 * i + s, True), (2 * j + s, False)]
    if spec.get("u") is not None:
        for i in range(n):
            if spec["u"][i] != 0.0:
                yield spec["u"][i], [(2 * i, True), (2 * i, False), (2 * i + 1, True), (2 * i + 1, False)]
    eri = spec.get("eri")
    if eri is not None:
        for i, j, k, l in itertools.product(range(n), repeat=4):
            v = eri[i, j, k, l]
            if v == 0.0:
                continue
            for s, t in itertools.product((0, 1), repeat=2):
                yield 0.5 * v, [(2 * i + s, True), (2 * k + t, True), (2 * l + t, False), (2 * j + s, False)]


def hamiltonian_matrix(spec: dict, basis: np.ndarray | None = None) -> sp.csr_matrix:
    """H in the (N, 2Sz) sector basis, term by term from the operator definition."""
    if basis is None:
        basis = sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    dim = basis.size
    rows, cols, vals = [], [], []
    col_index = np.arange(dim)
    ones = np.ones(dim)
    for coef, ops in operator_strings(spec):
        st, amp, idx = basis, ones, col_index
        for p, dag in reversed(ops):  # rightmost operator acts first
            st, amp, ok = apply_op(st, amp, p, dag)
            idx = idx[ok]
            if st.size == 0:
                break
        if st.size == 0:
            continue
        pos = np.searchsorted(basis, st)
        valid = (pos < dim)
        valid[valid] &= basis[pos[valid]] == st[valid]
        rows.append(pos[valid])
        cols.append(idx[valid])
        vals.append(coef * amp[valid])
    if constant(spec) != 0.0:
        rows.append(col_index)
        cols.append(col_index)
        vals.append(np.full(dim, constant(spec)))
    if not rows:
        return sp.csr_matrix((dim, dim))
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    return sp.coo_matrix((v, (r, c)), shape=(dim, dim)).tocsr()


def _dense_site(mps: dict, j: int) -> np.ndarray:
    """Site tensor j as a dense (M_left, 4, M_right) array in sector-offset order."""
    bl, br = mps["bonds"][j], mps["bonds"][j + 1]
    offl = np.concatenate([[0], np.cumsum([d for _, _, d in bl])])
    offr = np.concatenate([[0], np.cumsum([d for _, _, d in br])])
    a = np.zeros((offl[-1], 4, offr[-1]))
    for il, s, ir, blk in mps["sites"][j]:
        a[offl[il]:offl[il + 1], s, offr[ir]:offr[ir + 1]] = blk
    return a


def left_basis(mps: dict, l: int) -> np.ndarray:
    """(4^l, M_l): column a is the Fock-space amplitude of |a>_L over configs of sites 0..l-1.

    Row index = sum_j s_j 4^(l-1-j) (site 0 most significant).
    """
    vec = np.ones((1, 1))
    for j in range(l):
        a = _dense_site(mps, j)
        vec = np.einsum("ca,asb->csb", vec, a).reshape(-1, a.shape[2])
    return vec


def right_basis(mps: dict, r: int) -> np.ndarray:
    """(M_r, 4^(K-r)): row b is |b>_R over configs of sites r..K-1 (site r most significant)."""
    K = mps["n_sites"]
    vec = np.ones((1, 1))
    for j in range(K - 1, r - 1, -1):
        a = _dense_site(mps, j)
        vec = np.einsum("asb,bc->asc", a, vec).reshape(a.shape[0], -1)
    return vec


def _config_masks(first_site: int, n_sites: int) -> np.ndarray:
    """Bit masks of all 4^n_sites local configurations of sites first_site.. (lexicographic)."""
    masks = np.zeros(1, dtype=np.int64)
    for j in range(first_site, first_site + n_sites):
        loc = np.array([(nu << (2 * j)) | (nd << (2 * j + 1)) for nu, nd in _LOCAL_OCC], dtype=np.int64)
        masks = (masks[:, None] | loc[None, :]).reshape(-1)
    return masks


def two_site_isometry(mps: dict, basis: np.ndarray, blocks: list) -> np.ndarray:
    """P: (sector dim, two-site dim) with columns ordered by `blocks`, row-major inside a block."""
    K = mps["n_sites"]
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 2]
    offl = np.concatenate([[0], np.cumsum([d for _, _, d in bl])])
    offr = np.concatenate([[0], np.cumsum([d for _, _, d in br])])
    LB = left_basis(mps, l)
    RB = right_basis(mps, l + 2)
    lmask = _config_masks(0, l)
    rmask = _config_masks(l + 2, K - l - 2)
    ncols = sum(bl[a][2] * br[b][2] for a, _, _, b in blocks)
    P = np.zeros((basis.size, ncols))
    col = 0
    for ia, s1, s2, ib in blocks:
        m1 = (_LOCAL_OCC[s1][0] << (2 * l)) | (_LOCAL_OCC[s1][1] << (2 * l + 1))
        m2 = (_LOCAL_OCC[s2][0] << (2 * l + 2)) | (_LOCAL_OCC[s2][1] << (2 * l + 3))
        full = (lmask[:, None] | rmask[None, :]) | (m1 | m2)
        pos = np.searchsorted(basis, full.reshape(-1))
        pos = np.minimum(pos, basis.size - 1)
        hit = basis[pos] == full.reshape(-1)
        for a in range(bl[ia][2]):
            la = LB[:, offl[ia] + a]
            for b in range(br[ib][2]):
                rb = RB[offr[ib] + b, :]
                amp = np.outer(la, rb).reshape(-1)
                nz = hit & (amp != 0.0)
                P[pos[nz], col] += amp[nz]
                # amplitude on configurations outside the sector must vanish
                col += 1
    return P


def effective_hamiltonian(spec: dict, mps: dict, blocks: list) -> np.ndarray:
    """Dense H_eff = P^T H P of the two-site block at mps['center'] (complete construction)."""
    basis = sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    H = hamiltonian_matrix(spec, basis)
    P = two_site_isometry(mps, basis, blocks)
    HP = H @ P
    return P.T @ HP


def one_site_isometry(mps: dict, basis: np.ndarray, blocks: list) -> np.ndarray:
    """P1: (sector dim, one-site dim) for the site tensor at mps['center'] (Implementation
    section, local-derivative figure: the derivative with respect to the one tensor A^{n_l});
    column (a, s, b) is |a>_L |s> |b>_R, with |a>_L from the sites left of the center and |b>_R
    from the sites right of it.  Columns ordered by `blocks` ((ia, s, ib) or (ia, s, 0, ib)),
    row-major inside a block."""
    K = mps["n_sites"]
    l = mps["center"]
    bl, br = mps["bonds"][l], mps["bonds"][l + 1]
    offl = np.concatenate([[0], np.cumsum([d for _, _, d in bl])])
    offr = np.concatenate([[0], np.cumsum([d for _, _, d in br])])
    LB = left_basis(mps, l)
    RB = right_basis(mps, l + 1)
    lmask = _config_masks(0, l)
    rmask = _config_masks(l + 1, K - l - 1)
    keys = [(k[0], k[1], k[-1]) for k in blocks]
    ncols = sum(bl[a][2] * br[b][2] for a, _, b in keys)
    P = np.zeros((basis.size, ncols))
    col = 0
    for ia, s, ib in keys:
        m = (_LOCAL_OCC[s][0] << (2 * l)) | (_LOCAL_OCC[s][1] << (2 * l + 1))
        full = (lmask[:, None] | rmask[None, :]) | m
        pos = np.searchsorted(basis, full.reshape(-1))
        pos = np.minimum(pos, basis.size - 1)
        hit = basis[pos] == full.reshape(-1)
        for a in range(bl[ia][2]):
            la = LB[:, offl[ia] + a]
            for b in range(br[ib][2]):
                amp = np.outer(la, RB[offr[ib] + b, :]).reshape(-1)
                nz = hit & (amp != 0.0)
                P[pos[nz], col] += amp[nz]
                col += 1
    return P


def effective_hamiltonian_one_site(spec: dict, mps: dict, blocks: list) -> np.ndarray:
    """Dense one-site H_eff = P1^T H P1 of the site tensor at mps['center']."""
    basis = sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    H = hamiltonian_matrix(spec, basis)
    P = one_site_isometry(mps, basis, blocks)
    return P.T @ (H @ P)


def ground_energy(spec: dict, k: int = 1) -> np.ndarray:
    """Lowest k eigenvalues of H in its sector (exact diagonalisation)."""
    H = hamiltonian_matrix(spec)
    if H.shape[0] <= 6000:
        return np.linalg.eigvalsh(H.toarray())[:k]
    import scipy.sparse.linalg as sla
    vals = sla.eigsh(H, k=k, which="SA", tol=1e-12)[0]
    return np.sort(vals)


def config_index(basis: np.ndarray, n_sites: int) -> np.ndarray:
    """Position of each sector state in the site-product ordering of left_basis (site 0 most
    significant, local index n_up + 2 n_dn)."""
    idx = np.zeros(basis.size, dtype=np.int64)
    for j in range(n_sites):
        idx = idx * 4 + ((basis >> (2 * j)) & 1) + 2 * ((basis >> (2 * j + 1)) & 1)
    return idx


def mps_state(mps: dict, basis: np.ndarray) -> np.ndarray:
    """The state of an MPS (MPS equation: all site tensors contracted) as a vector over `basis`."""
    K = mps["n_sites"]
    full = left_basis(mps, K)[:, 0]
    return full[config_index(basis, K)]


def first_order_vectors(spec: dict, bra: dict, ket: dict, blocks: list, one_site: bool = False):
    """Local vectors of the first-order equation at the bra's two-site block (Theory section,
    first-order equation; Implementation section, its local form): with P the bra's two-site
    isometry and Phi0 the ket state,
        u = P^T H Phi0,   v = P^T Phi0,   e1 = <Phi0|H|Phi0> / <Phi0|Phi0>,
    so that P^T Q H Phi0 = u - e1 v for Q = 1 - |Phi0><Phi0| / <Phi0|Phi0>.  Columns of P in
    `blocks` order, row-major inside a block; one_site: P is the one-site isometry of the bra's
    center tensor."""
    basis = sector_basis(spec["n_orb"], spec["n_elec"], spec["two_sz"])
    H = hamiltonian_matrix(spec, basis)
    phi0 = mps_state(ket, basis)
    P = one_site_isometry(bra, basis, blocks) if one_site else two_site_isometry(bra, basis, blocks)
    hphi = H @ phi0
    return P.T @ hphi, P.T @ phi0, float(phi0 @ hphi) / float(phi0 @ phi0)
