"""Seeded synthetic Hamiltonians (inputs only; no part of the method's arithmetic).

Every generator returns a plain dict describing

    H = sum_{ij,sigma} h[i,j] a+_{i sigma} a_{j sigma}
        + 1/2 sum_{ijkl,sigma tau} eri[i,j,k,l] a+_{i sigma} a+_{k tau} a_{l tau} a_{j sigma}
        + sum_i u[i] n_{i up} n_{i down} + e_const

with `eri` in chemists' order (ij|kl).  This is the one- plus two-body
Hamiltonian of the Theory section (the partitioned Hamiltonian equation),
read with the conventional factor 1/2 and spatial orbitals, which the printed
formula leaves implicit.  Orbital (site) index = position in the MPS chain.

Keys: n_orb, h (n,n) float64, eri (n,n,n,n) float64 or None, u (n,) float64 or
None, e_const float, n_elec int, two_sz int, name str.
"""
from __future__ import annotations

import numpy as np


def _spec(name, h, n_elec, two_sz, u=None, eri=None, e_const=0.0):
    n = h.shape[0]
    return {
        "name": name,
        "n_orb": int(n),
        "h": np.ascontiguousarray(h, dtype=np.float64),
        "eri": None if eri is None else np.ascontiguousarray(eri, dtype=np.float64),
        "u": None if u is None else np.ascontiguousarray(u, dtype=np.float64),
        "e_const": float(e_const),
        "n_elec": int(n_elec),
        "two_sz": int(two_sz),
    }


def hubbard_chain(n_sites: int, t: float = 1.0, U: float = 4.0, n_elec: int | None = None,
                  two_sz: int = 0, pbc: bool = False) -> dict:
    """1-D Hubbard chain, H = -t sum_<ij> (c+ c + h.c.) + U sum n_up n_dn."""
    h = np.zeros((n_sites, n_sites))
    for i in range(n_sites - 1):
        h[i, i + 1] = h[i + 1, i] = -t
    if pbc and n_sites > 2:
        h[0, n_sites - 1] = h[n_sites - 1, 0] = -t
    if n_elec is None:
        n_elec = n_sites
    return _spec(f"hubbard1d_L{n_sites}_U{U:g}", h, n_elec, two_sz, u=np.full(n_sites, float(U)))


def snake_order_2d(lx: int, ly: int) -> list[tuple[int, int]]:
    """Column snake: column x = 0..lx-1; y ascends in even columns, descends in odd ones."""
    order = []
    for x in range(lx):
        ys = range(ly) if x % 2 == 0 else range(ly - 1, -1, -1)
        for y in ys:
            order.append((x, y))
    return order


def hubbard_2d(lx: int, ly: int, t: float = 1.0, U: float = 4.0, n_elec: int | None = None,
               two_sz: int = 0, pbc: bool = True) -> dict:
    """Square-lattice 1-band Hubbard model on an lx x ly torus, column-snake orbital order."""
    order = snake_order_2d(lx, ly)
    index = {xy: i for i, xy in enumerate(order)}
    n = lx * ly
    h = np.zeros((n, n))
    for (x, y), i in index.items():
        for dx, dy in ((1, 0), (0, 1)):
            nx, ny = x + dx, y + dy
            if pbc:
                nx %= lx
                ny %= ly
            if not (0 <= nx < lx and 0 <= ny < ly):
                continue
            j = index[(nx, ny)]
            if i == j:
                continue
            # a torus of extent 2 would count the same pair twice; keep one bond
            h[i, j] = h[j, i] = -t
    if n_elec is None:
        n_elec = n
    return _spec(f"hubbard2d_{lx}x{ly}_U{U:g}", h, n_elec, two_sz, u=np.full(n, float(U)))


def three_band(cells_x: int = 4, cells_y: int = 2, tpd: float = 1.3, tpp: float = 0.65,
               delta: float = 3.6, Ud: float = 8.4, Up: float = 0.0,
               n_holes: int | None = None, two_sz: int = 1) -> dict:
    """Cu-O (d, px, py) three-band Hubbard model in hole language.

    Cell (i, j) holds d at (i, j), px at (i + 1/2, j), py at (i, j + 1/2).  Periodic along x,
    open along y.  Phase convention: a d-p bond has sign +1 when the p orbital sits at +x/2 or
    +y/2 of the Cu and -1 otherwise; a p-p bond px(i,j)-py(i',j') has sign
    -(sign of the x offset) * (sign of the y offset), i.e. the standard alternating pattern.
    H = sum eps n + sum t s (c+ c + h.c.) + Ud n_up n_dn (d) + Up n_up n_dn (p),
    eps_d = 0, eps_p = delta.  Orbitals are ordered cell by cell along a column snake,
    inside a cell as (d, px, py).
    """
    cells = snake_order_2d(cells_x, cells_y)
    idx = {}
    for c, (x, y) in enumerate(cells):
        idx[("d", x, y)] = 3 * c
        idx[("px", x, y)] = 3 * c + 1
        idx[("py", x, y)] = 3 * c + 2
    n = 3 * len(cells)
    h = np.zeros((n, n))
    u = np.zeros(n)

    def add(a, b, val):
        if a == b:
            return
        h[a, b] += val
        h[b, a] += val

    for (x, y) in cells:
        d = idx[("d", x, y)]
        h[idx[("px", x, y)], idx[("px", x, y)]] = delta
        h[idx[("py", x, y)], idx[("py", x, y)]] = delta
        u[d] = Ud
        u[idx[("px", x, y)]] = Up
        u[idx[("py", x, y)]] = Up
        # d - p bonds: px at +x/2 (own cell), px at -x/2 (cell x-1), py at +y/2, py at -y/2
        add(d, idx[("px", x, y)], tpd)
        add(d, idx[("px", (x - 1) % cells_x, y)], -tpd)
        add(d, idx[("py", x, y)], tpd)
        if y - 1 >= 0:
            add(d, idx[("py", x, y - 1)], -tpd)
        # p - p bonds around this Cu: (px at +-x/2) with (py at +-y/2)
        for sx, px in ((+1, idx[("px", x, y)]), (-1, idx[("px", (x - 1) % cells_x, y)])):
            for sy, yy in ((+1, y), (-1, y - 1)):
                if yy < 0:
                    continue
                py = idx[("py", x, yy)]
                add(px, py, -sx * sy * tpp)
    if n_holes is None:
        n_holes = len(cells) + max(1, len(cells) // 8)
    return _spec(f"threeband_{cells_x}x{cells_y}", h, n_holes, two_sz, u=u)


def random_ab_initio(n_orb: int, n_elec: int, two_sz: int = 0, seed: int = 1003,
                     decay: float = 4.0) -> dict:
    """Random real integrals with 8-fold symmetry and N(0,1)*exp(-distance/decay) magnitude.

    h[i,j] = h[j,i] ~ N(0,1) exp(-|i-j|/decay); the diagonal is then sorted ascending in
    place.  (ij|kl) ~ N(0,1) exp(-(|i-j| + |k-l|)/decay), drawn once per canonical quadruple
    (i>=j, k>=l, ij>=kl) in lexicographic order and copied to its 8 images.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = n_orb
    h = np.zeros((n, n))
    for i in range(n):
        for j in range(i + 1):
            v = rng.standard_normal() * np.exp(-abs(i - j) / decay)
            h[i, j] = h[j, i] = v
    diag = np.sort(np.diag(h).copy())
    h[np.arange(n), np.arange(n)] = diag
    eri = np.zeros((n, n, n, n))
    pairs = [(i, j) for i in range(n) for j in range(i + 1)]
    for a, (i, j) in enumerate(pairs):
        for (k, l) in pairs[: a + 1]:
            v = rng.standard_normal() * np.exp(-(abs(i - j) + abs(k - l)) / decay)
            for (p, q, r, s) in ((i, j, k, l), (j, i, k, l), (i, j, l, k), (j, i, l, k),
                                 (k, l, i, j), (l, k, i, j), (k, l, j, i), (l, k, j, i)):
                eri[p, q, r, s] = v
    return _spec(f"abinitio_K{n}_seed{seed}", h, n_elec, two_sz, eri=eri)


def number_operator(n_orb: int, n_elec: int, two_sz: int = 0) -> dict:
    """N-hat as a Hamiltonian (h = identity); a state with n electrons has eigenvalue n."""
    return _spec(f"number_K{n_orb}", np.eye(n_orb), n_elec, two_sz)


def rotate_orbitals(spec: dict, c: np.ndarray) -> dict:
    """Express `spec` in the orbital basis phi'_p = sum_i c[i,p] phi_i (c orthogonal).

    The on-site term u_i n_{i up} n_{i dn} is first written as (ii|ii) = u_i, so the
    result always carries a full `eri`.  The spectrum is unchanged.
    """
    n = spec["n_orb"]
    eri = np.zeros((n, n, n, n)) if spec["eri"] is None else spec["eri"].copy()
    if spec["u"] is not None:
        for i in range(n):
            eri[i, i, i, i] += spec["u"][i]
    h2 = c.T @ spec["h"] @ c
    eri2 = np.einsum("ijkl,ip,jq,kr,ls->pqrs", eri, c, c, c, c, optimize=True)
    out = _spec(spec["name"] + "_rot", h2, spec["n_elec"], spec["two_sz"], eri=eri2,
                e_const=spec["e_const"])
    return out


def random_orthogonal(n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    return q * np.sign(np.diag(r))


def with_partition(spec: dict, orb_class, part: int) -> dict:
    """The same Hamiltonian with orbital classes (0 core, 1 active, 2 virtual per orbital) and a
    selected part: 0 the whole H, 1 H0, 2 U (see the partitioned-Hamiltonian equation)."""
    out = dict(spec)
    out["orb_class"] = np.ascontiguousarray(orb_class, dtype=np.int32)
    out["part"] = int(part)
    out["name"] = spec["name"] + ("", "_H0", "_U")[int(part)]
    return out


def reorder(spec: dict, order) -> dict:
    """The Hamiltonian with orbital order[p] placed at chain position p."""
    o = np.asarray(order)
    out = dict(spec)
    out["h"] = np.ascontiguousarray(spec["h"][np.ix_(o, o)])
    if spec.get("eri") is not None:
        out["eri"] = np.ascontiguousarray(spec["eri"][np.ix_(o, o, o, o)])
    if spec.get("u") is not None:
        out["u"] = np.ascontiguousarray(spec["u"][o])
    if spec.get("orb_class") is not None:
        out["orb_class"] = np.ascontiguousarray(spec["orb_class"][o])
    out["name"] = spec["name"] + "_reordered"
    return out
