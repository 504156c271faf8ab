"""Seeded synthetic inputs shared by the tests, the bench and the oracle checks.

This module holds the workloads only: site tensors drawn from a seed, the
spin-1/2 bond operator, and the lists of plaquette terms that define the two
models of the paper (square-lattice Heisenberg model, Sec. III A; Shastry-
Sutherland model, Eq. SSM).  It contains none of the contraction method's
arithmetic, so both the GPU path and the CPU oracle can be fed from it without
sharing any of the method's code.

Conventions
-----------
* A site tensor is A[sigma, l, u, r, d] (C order), the rank-5 PEPS tensor of
  Eq. PEPS with physical index first and the four virtual legs clockwise from
  the left.  All workloads are real (float64).
* Unit cell: Lx columns by Ly rows of PEPS sites; ``pattern[y][x]`` is the
  index of the distinct tensor sitting at column x, row y (rows grow downward).
* A plaquette term (px, py, a, b, coef) names the 2x2 plaquette whose upper-left
  site is (px, py) and two of its sites, numbered 0 = top-left, 1 = top-right,
  2 = bottom-left, 3 = bottom-right.  The energy per site is
  (1 / (Lx*Ly)) * sum(coef * <h_ab>).
"""
from __future__ import annotations

import numpy as np

TL, TR, BL, BR = 0, 1, 2, 3


def site_tensors(n_tensors: int, d: int, D: int, seed: int, dist: str) -> np.ndarray:
    """Draw ``n_tensors`` site tensors A_t[sigma,l,u,r,d] and normalise each.

    Tensors are drawn one after the other from ``numpy.random.default_rng(seed)``
    in C order, ``dist`` is ``"uniform"`` (entries in [-1, 1]) or ``"normal"``
    (entries N(0, 1)); each tensor is then scaled to unit Frobenius norm.
    Returns an array of shape (n_tensors, d, D, D, D, D).
    """
    rng = np.random.default_rng(seed)
    shape = (d, D, D, D, D)
    out = np.empty((n_tensors,) + shape, dtype=np.float64)
    for t in range(n_tensors):
        if dist == "uniform":
            a = rng.uniform(-1.0, 1.0, size=shape)
        elif dist == "normal":
            a = rng.standard_normal(size=shape)
        else:
            raise ValueError(f"unknown distribution {dist!r}")
        out[t] = a / np.linalg.norm(a)
    return out


def spin_half_ops():
    """Real spin-1/2 operators (Sx, i*Sy, Sz) in the basis (up, down)."""
    sx = np.array([[0.0, 0.5], [0.5, 0.0]])
    isy = np.array([[0.0, 0.5], [-0.5, 0.0]])  # i * Sy, real
    sz = np.array([[0.5, 0.0], [0.0, -0.5]])
    return sx, isy, sz


def heisenberg_bond() -> np.ndarray:
    """S_a . S_b as a 4x4 matrix H[(s_a s_b), (s_a' s_b')] with s_a the major index."""
    sx, isy, sz = spin_half_ops()
    # Sy (x) Sy = -(i Sy) (x) (i Sy)
    return np.kron(sx, sx) - np.kron(isy, isy) + np.kron(sz, sz)


def heisenberg_bond_rotated() -> np.ndarray:
    """S_a . S_b with site b rotated by pi about the y axis (Sx -> -Sx, Sy -> Sy,
    Sz -> -Sz): -SxSx + SySy - SzSz, real.  With every nearest-neighbour bond of
    the square lattice joining the two sublattices, this one bond term on all
    bonds describes the Heisenberg model after the local rotation -i sigma_y of
    one sublattice (Discussion), so a Neel-ordered checkerboard state becomes
    translation invariant and fits a 1x1 cell."""
    sx, isy, sz = spin_half_ops()
    return -np.kron(sx, sx) - np.kron(isy, isy) - np.kron(sz, sz)


def rotate_physical(A: np.ndarray) -> np.ndarray:
    """Site tensors with -i sigma_y = [[0, -1], [1, 0]] (real) applied to the physical index."""
    U = np.array([[0.0, -1.0], [1.0, 0.0]])
    return np.einsum("st,ntlurd->nslurd", U, A)


def heisenberg_terms(Lx: int, Ly: int, J: float = 1.0):
    """Nearest-neighbour terms of H = J sum S_i.S_j on an Lx x Ly cell.

    Every plaquette carries its four edges with weight J/2: each bond of the
    square lattice lies on two plaquettes, so the per-site energy counts every
    bond exactly once.
    """
    terms = []
    for py in range(Ly):
        for px in range(Lx):
            for a, b in ((TL, TR), (BL, BR), (TL, BL), (TR, BR)):
                terms.append((px, py, a, b, 0.5 * J))
    return terms


def shastry_sutherland_terms(J_nn: float, J_dimer: float):
    """Terms of Eq. SSM on the 2x2 cell.

    ``J_nn`` couples the square-lattice nearest neighbours, ``J_dimer`` the
    orthogonal diagonal dimers.  Dimers sit on the diagonals of plaquettes
    (0,0) (top-left to bottom-right) and (1,1) (top-right to bottom-left), so
    every site belongs to exactly one dimer; plaquettes (1,0) and (0,1) are the
    two inequivalent empty squares.
    """
    terms = heisenberg_terms(2, 2, J_nn)
    terms.append((0, 0, TL, BR, J_dimer))
    terms.append((1, 1, TR, BL, J_dimer))
    return terms


# --- the five workloads --------------------------------------------------
# name -> dict(model, d, D, chi, Lx, Ly, pattern, dist, sweeps, precision)
CONFIGS = {
    "heis_d2_chi8": dict(model="heisenberg", J=1.0, d=2, D=2, chi=8, Lx=1, Ly=1,
                         pattern=[[0]], n_tensors=1, dist="uniform", sweeps=100, tol=1e-10),
    "heis_d4_chi32": dict(model="heisenberg", J=1.0, d=2, D=4, chi=32, Lx=1, Ly=1,
                          pattern=[[0]], n_tensors=1, dist="normal", sweeps=40, tol=0.0),
    "ssm_d6_chi72": dict(model="ssm", J_nn=0.8, J_dimer=1.0, d=2, D=6, chi=72, Lx=2, Ly=2,
                         pattern=[[0, 1], [2, 3]], n_tensors=4, dist="uniform", sweeps=30, tol=0.0),
    "heis_d9_chi100": dict(model="heisenberg", J=1.0, d=2, D=9, chi=100, Lx=2, Ly=1,
                           pattern=[[0, 1]], n_tensors=2, dist="normal", sweeps=20, tol=0.0),
    "ssm_d5_chi50": dict(model="ssm", J_nn=0.7, J_dimer=1.0, d=2, D=5, chi=50, Lx=2, Ly=2,
                         pattern=[[0, 1], [2, 3]], n_tensors=4, dist="uniform", sweeps=30, tol=0.0),
}


def config_terms(cfg: dict):
    if cfg["model"] == "heisenberg":
        return heisenberg_terms(cfg["Lx"], cfg["Ly"], cfg.get("J", 1.0))
    if cfg["model"] == "ssm":
        return shastry_sutherland_terms(cfg["J_nn"], cfg["J_dimer"])
    raise ValueError(cfg["model"])


def config_tensors(cfg: dict, seed: int = 0) -> np.ndarray:
    return site_tensors(cfg["n_tensors"], cfg["d"], cfg["D"], seed, cfg["dist"])


def product_state_tensors(vectors, D: int = 1) -> np.ndarray:
    """D=1 (or index-0-padded) tensors of product states: A_t[s,0,0,0,0] = v_t[s]."""
    vectors = np.asarray(vectors, dtype=np.float64)
    n, d = vectors.shape
    out = np.zeros((n, d, D, D, D, D))
    out[:, :, 0, 0, 0, 0] = vectors
    return out


def singlet_amplitude() -> np.ndarray:
    """eps[s1, s2] of the singlet |up,down> - |down,up> (unnormalised)."""
    return np.array([[0.0, 1.0], [-1.0, 0.0]])


def columnar_dimer_tensors() -> np.ndarray:
    """2x1 cell, D=2: a singlet on every horizontal bond (0,y)-(1,y).

    Site 0 copies its spin onto its right leg; site 1 closes the singlet on its
    left leg.  All other legs carry index 0.
    """
    eps = singlet_amplitude()
    A = np.zeros((2, 2, 2, 2, 2, 2))
    for s in range(2):
        A[0, s, 0, 0, s, 0] = 1.0
        for l in range(2):
            A[1, s, l, 0, 0, 0] = eps[l, s]
    return A


def orthogonal_dimer_tensors() -> np.ndarray:
    """2x2 cell, D=2, pattern [[0,1],[2,3]]: singlets on the Shastry-Sutherland dimers.

    In absolute coordinates the dimers are (2m, 2n)-(2m+1, 2n+1) (diagonal of
    plaquette (0,0)) and (2m+2, 2n+1)-(2m+1, 2n+2) (anti-diagonal of plaquette
    (1,1)).  Each singlet is routed over two bonds of the square lattice:
    dimer 1 as (0,0).r -> (1,0).l, (1,0).d -> (1,1).u; dimer 2 as
    (0,1).l -> (1,1).r (across the cell edge), (1,1).d -> (1,0).u (across the
    cell edge).  Sites (0,0) and (0,1) copy their spin onto a virtual leg;
    sites (1,0) and (1,1) close one singlet on their up leg and pass the other
    dimer through.  All unused legs carry index 0.
    """
    eps = singlet_amplitude()
    A = np.zeros((4, 2, 2, 2, 2, 2))
    for s in range(2):
        A[0, s, 0, 0, s, 0] = 1.0                       # (0,0): spin out right
        A[2, s, s, 0, 0, 0] = 1.0                       # (0,1): spin out left
        for u in range(2):
            for p in range(2):
                A[1, s, p, u, 0, p] = eps[u, s]         # (1,0): close dimer 2, pass dimer 1 l -> d
                A[3, s, 0, u, p, p] = eps[u, s]         # (1,1): close dimer 1, pass dimer 2 r -> d
    return A


def vertical_chain_tensors(seed: int, d: int = 2, Dv: int = 2, D: int = 2) -> np.ndarray:
    """1x1 cell: random vertical MPS with bond Dv, horizontal legs fixed to index 0.

    The PEPS is then a product of independent infinite vertical chains.
    """
    rng = np.random.default_rng(seed)
    A = np.zeros((1, d, D, D, D, D))
    A[0, :, 0, :Dv, 0, :Dv] = rng.uniform(-1.0, 1.0, size=(d, Dv, Dv))
    A /= np.linalg.norm(A)
    return A


def gauge_transform(A: np.ndarray, pattern, seed: int) -> np.ndarray:
    """Apply a random invertible gauge G, G^-1 to every virtual bond of the unit cell.

    The wave function is unchanged (G G^-1 = 1 on every bond) while the site
    tensors lose any special structure.  Each tensor must occur once in the
    pattern so that every bond of the cell gets its own gauge.
    """
    A = np.array(A, dtype=np.float64)
    Ly, Lx = len(pattern), len(pattern[0])
    ids = [pattern[y][x] for y in range(Ly) for x in range(Lx)]
    assert len(set(ids)) == len(ids), "gauge_transform needs distinct tensors"
    D = A.shape[2]
    rng = np.random.default_rng(seed)
    gh = {(x, y): np.eye(D) + 0.5 * rng.uniform(-1, 1, (D, D)) for y in range(Ly) for x in range(Lx)}
    gv = {(x, y): np.eye(D) + 0.5 * rng.uniform(-1, 1, (D, D)) for y in range(Ly) for x in range(Lx)}
    out = A.copy()
    for y in range(Ly):
        for x in range(Lx):
            t = pattern[y][x]
            a = A[t]
            a = np.einsum("slurd,rR->sluRd", a, gh[(x, y)])
            a = np.einsum("slurd,dE->slurE", a, gv[(x, y)])
            a = np.einsum("Ll,slurd->sLurd", np.linalg.inv(gh[((x - 1) % Lx, y)]), a)
            a = np.einsum("Uu,slurd->slUrd", np.linalg.inv(gv[(x, (y - 1) % Ly)]), a)
            out[t] = a
    return out


def nested_leg_dims(D: int, d: int):
    """Leg dimensions (l, u, r, d) of the four nested site kinds K, Y, X, B (Eq. XY and its footnote)."""
    return {"K": (D, D, D * d, D), "Y": (D * d, D, D, D * d), "X": (D, D, D, D), "B": (D, D * d, D, D)}


def random_env_flat(chi: int, D: int, d: int, Lx: int, Ly: int, seed: int) -> np.ndarray:
    """A seeded uniform [0, 1) starting environment in the library's flat layout.

    Layout: nested positions (I, J) of the 2Ly x 2Lx cell in row-major order,
    each with C1, C2, C3, C4 (chi x chi) then T1, T2, T3, T4 (chi x leg x chi),
    where the leg of T1/T2/T3/T4 is the up/right/down/left leg of the nested
    site at (I, J) (K at even/even, Y at even/odd, X at odd/even, B at odd/odd).
    """
    legs = nested_leg_dims(D, d)
    kind = {(0, 0): "K", (0, 1): "Y", (1, 0): "X", (1, 1): "B"}
    n = 0
    for I in range(2 * Ly):
        for J in range(2 * Lx):
            l, u, r, dn = legs[kind[(I % 2, J % 2)]]
            n += 4 * chi * chi + chi * chi * (u + r + dn + l)
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=n)


def random_double_env_flat(chi: int, D: int, Lx: int, Ly: int, seed: int) -> np.ndarray:
    """A seeded uniform [0, 1) starting environment of the double-layer network (Eq. Tred).

    Layout as ``random_env_flat`` but over the Ly x Lx PEPS positions (y, x)
    in row-major order, every edge tensor being chi x D^2 x chi (the fused
    ket/bra leg of the reduced tensor).
    """
    n = Lx * Ly * (4 * chi * chi + 4 * chi * D * D * chi)
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=n)


def near_product_tensors(n_tensors: int, d: int, D: int, seed: int, eps: float = 0.2) -> np.ndarray:
    """Random site tensors close to a product state (short correlation length).

    A_t = v_t (x) e_0 e_0 e_0 e_0 + eps * G / |G| with G a N(0, 1) tensor, then
    unit Frobenius norm, with v_t a random unit vector of the physical space.  CTMRG on such states
    converges in a few sweeps and is well conditioned, which makes them the
    workload for tight multi-sweep comparisons.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n_tensors, d, D, D, D, D))
    for t in range(n_tensors):
        v = rng.standard_normal(d)
        g = rng.standard_normal((d, D, D, D, D))
        a = eps * g / np.linalg.norm(g)
        a[:, 0, 0, 0, 0] += v / np.linalg.norm(v)
        out[t] = a / np.linalg.norm(a)
    return out
