"""Double-layer CTMRG (Eq. Tred): the method the nested one is compared with.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The conventional route contracts ket and bra of every site into one reduced
tensor a = sum_s A[s] A*[s] of Eq. Tred, whose four legs are the pairs of ket
and bra virtual legs (bond dimension D^2), and runs CTMRG on the resulting
square lattice of Lx x Ly reduced tensors.  The projectors of a cut then act
on (chi D^2)-dimensional spaces instead of the (chi D)-dimensional ones of the
nested network (Sec. II C).  At finite chi the two methods truncate different
networks and give different environments; both become exact as chi grows,
so their energies must converge to each other (Appendix, Fig. SM-Compare;
Sec. IV).

The environment iteration itself (start environment, projectors from QR and
truncated SVD, Eqs. PQ and QRSVD, the left move and the four-move sweep) is
the generic multi-site CTMRG of ``ctmrg``: it only sees a grid of
(l, u, r, d) tensors, here the reduced tensors instead of the nested sites.
What is written separately here is the lattice (reduced tensors with
fused ket/bra legs) and the 2x2 reduced density matrix of a plaquette of
open reduced tensors.

Fused legs are (ket index major, bra index minor).
"""
from __future__ import annotations

import torch

from types import SimpleNamespace

from .ctmrg import corner_spectra, env_from_flat, init_env, spectra_delta, sweep
from .network import LT, as_t, contract_all, site_frames
from .rdm import ORDER, energy_from_rdms


def reduced_tensor(A):
    """a[(l l'), (u u'), (r r'), (d d')] = sum_s A[s, l, u, r, d] conj(A)[s, l', u', r', d'] (Eq. Tred)."""
    A = as_t(A)
    D = A.shape[1]
    a = torch.einsum("slurd,sLURD->lLuUrRdD", A, A.conj())
    return a.reshape(D * D, D * D, D * D, D * D)


def open_reduced_tensor(A):
    """Reduced tensor with its physical indices open: ao[(l l'), (u u'), (r r'), (d d'), k, b] = A[k,...] conj(A)[b,...]."""
    A = as_t(A)
    d, D = A.shape[0], A.shape[1]
    a = torch.einsum("klurd,bLURD->lLuUrRdDkb", A, A.conj())
    return a.reshape(D * D, D * D, D * D, D * D, d, d)


def double_cell(A, pattern):
    """Ly x Lx grid of reduced tensors: entry [y][x] belongs to PEPS site (x, y)."""
    A = as_t(A)
    Ly, Lx = len(pattern), len(pattern[0])
    return [[reduced_tensor(A[pattern[y][x]]) for x in range(Lx)] for y in range(Ly)]


class DoubleLayerCTM:
    """CTMRG state of the double-layer network of one set of site tensors."""

    def __init__(self, A, pattern, chi, cutoff=1e-10, env0=None):
        """``env0``: optional starting environment in the flat layout of ``ctmrg.env_to_flat``
        over the reduced tensors; by default the sites-derived start of ``ctmrg.init_env``."""
        self.A = as_t(A)
        self.pattern, self.chi, self.cutoff = pattern, chi, cutoff
        self.sites = double_cell(self.A, pattern)
        self.frames = site_frames(self.sites)
        self.env = init_env(self.sites) if env0 is None else env_from_flat(env0, self.sites, chi)
        self.spectra = corner_spectra(self.env, chi)

    def run(self, max_sweeps, tol=0.0):
        """Sweep until delta < tol or ``max_sweeps``; returns (sweeps done, last delta)."""
        delta = float("inf")
        n = 0
        for n in range(1, max_sweeps + 1):
            self.env = sweep(self.frames, self.env, self.chi, self.cutoff)
            sp = corner_spectra(self.env, self.chi)
            delta = spectra_delta(sp, self.spectra)
            self.spectra = sp
            if delta < tol:
                break
        return n, delta


def plaquette_rdm(ctm: DoubleLayerCTM, x, y):
    """rho[(k_TL k_TR k_BL k_BR), (b_TL b_TR b_BL b_BR)] of the plaquette with top-left site (x, y), not normalised.

    The four sites of the plaquette are open reduced tensors; the boundary is
    C1, T1 T1 (top), C2, T2 T2 (right), C3, T3 T3 (bottom), C4, T4 T4 (left)
    of the positions on the plaquette's border.  Each quadrant (one corner,
    two edges, one open site) is formed first, then the upper and the lower
    pairs, then the two halves.
    """
    Ly, Lx = len(ctm.pattern), len(ctm.pattern[0])
    x1, y1 = (x + 1) % Lx, (y + 1) % Ly
    env = ctm.env
    site = lambda xx, yy: open_reduced_tensor(ctm.A[ctm.pattern[yy][xx]])
    # environment legs in the counter-clockwise order of each tensor
    C1 = LT(env[y][x]["C1"], ("L0", "t0"))
    T1a = LT(env[y][x]["T1"], ("t0", "v0", "t1"))
    T1b = LT(env[y][x1]["T1"], ("t1", "v1", "t2"))
    C2 = LT(env[y][x1]["C2"], ("t2", "R0"))
    T2a = LT(env[y][x1]["T2"], ("R0", "e0", "R1"))
    T2b = LT(env[y1][x1]["T2"], ("R1", "e1", "R2"))
    C3 = LT(env[y1][x1]["C3"], ("R2", "b2"))
    T3b = LT(env[y1][x1]["T3"], ("b2", "w1", "b1"))
    T3a = LT(env[y1][x]["T3"], ("b1", "w0", "b0"))
    C4 = LT(env[y1][x]["C4"], ("b0", "L2"))
    T4b = LT(env[y1][x]["T4"], ("L2", "f1", "L1"))
    T4a = LT(env[y][x]["T4"], ("L1", "f0", "L0"))
    tl = LT(site(x, y), ("f0", "v0", "m0", "n0", "kTL", "bTL"))
    tr = LT(site(x1, y), ("m0", "v1", "e0", "n1", "kTR", "bTR"))
    bl = LT(site(x, y1), ("f1", "n0", "m1", "w0", "kBL", "bBL"))
    br = LT(site(x1, y1), ("m1", "n1", "e1", "w1", "kBR", "bBR"))
    ul = contract_all([C1, T1a, T4a, tl])
    ur = contract_all([T1b, C2, T2a, tr])
    dl = contract_all([T4b, C4, T3a, bl])
    dr = contract_all([T2b, C3, T3b, br])
    rho = contract_all([contract_all([ul, ur]), contract_all([dl, dr])])
    t = rho.order([f"k{n}" for n in ORDER] + [f"b{n}" for n in ORDER])
    d = t.shape[0]
    return t.reshape(d ** 4, d ** 4)


def energy(ctm: DoubleLayerCTM, H, terms):
    """Energy per site (Eq. ExpH) from the double-layer environment, with the plaquette terms of ``synth``."""
    Ly, Lx = len(ctm.pattern), len(ctm.pattern[0])
    needed = sorted({(t[0], t[1]) for t in terms})
    rdms = {p: plaquette_rdm(ctm, p[0], p[1]) for p in needed}
    return energy_from_rdms(rdms, H, terms, Lx * Ly)


def energy_after_sweeps(A, pattern, chi, env0, n_sweeps, H, terms, cutoff=1e-10, eta=1e-12):
    """E(A) after ``n_sweeps`` double-layer sweeps from the constant environment
    ``env0``, differentiable in A (Eq. AD on the network of Eq. Tred): the
    reduced tensors are formed by einsum from A, the sweep is the generic one
    with the projector block of ``adjoint.projector_fn`` (hand-written
    derivative, Lorentzian width eta), the energy that of ``energy`` above.
    Returns (E, env_final)."""
    from .adjoint import projector_fn
    A = as_t(A) if not torch.is_tensor(A) else A
    frames = site_frames(double_cell(A, pattern))
    proj = projector_fn(eta)
    env = env0
    for _ in range(n_sweeps):
        env = sweep(frames, env, chi, cutoff, proj=proj)
    E = energy(SimpleNamespace(A=A, pattern=pattern, env=env), H, terms)
    return E, env


def energy_and_grad(A, pattern, chi, env0, n_sweeps, H, terms, cutoff=1e-10, eta=1e-12):
    """(E, dE/dA, final environment) for ``energy_after_sweeps``."""
    A = torch.as_tensor(A, dtype=torch.float64).clone().requires_grad_(True)
    env0 = [[{k: v.detach().clone() for k, v in e.items()} for e in row] for row in env0]
    E, env = energy_after_sweeps(A, pattern, chi, env0, n_sweeps, H, terms, cutoff, eta)
    (g,) = torch.autograd.grad(E, A)
    return E.item(), g, [[{k: v.detach() for k, v in e.items()} for e in row] for row in env]
