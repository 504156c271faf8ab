"""Order parameters from plaquette density matrices (Eqs. Mag1 and Mag2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Input: a plaquette rho[(k_TL k_TR k_BL k_BR), (b_TL b_TR b_BL b_BR)] as built
for the energy (Eq. ExpH), a d^4 x d^4 matrix, not normalised.  Spin-1/2 sites
(d = 2) with basis (up, down): S^a = sigma^a / 2.  Expectation values follow
the energy's convention <O> = Tr(O rho') / Tr rho' = sum O[b, k] rho'[k, b],
rho' the reduced matrix of the sites O acts on (the other sites traced).

* Moment of site s (Eq. Mag1): m_s = (<S^x>, <S^y>, <S^z>) from the one-site
  matrix.  The magnetisation M is the mean of |m_i| over the inequivalent
  sites i of the cell.
* Bond correlation <S_a . S_b> from the two-site matrix.  The plaquette
  order parameter of Eq. Mag2 is a quarter of the absolute difference of the
  sums of <S_i . S_j> over the four nearest-neighbour bonds of two plaquettes
  (the empty plaquettes A and B of the Shastry-Sutherland lattice).

Reading: the site tensors are real, so rho is real; Tr(S^y rho_s) is then
purely imaginary, (i/2)(rho_s[0,1] - rho_s[1,0]), and vanishes when rho is
Hermitian.  The raw nested rho need not be exactly Hermitian, so its
imaginary part measures that defect, not a moment: <S^y> is the real part of
the trace, which is zero.

Outputs per plaquette (18 values): the moments of TL, TR, BL, BR (x, y, z
each), then <S_a . S_b> for the site pairs of BONDS.
"""
from __future__ import annotations

import torch

from .rdm import pair_rdm

SX = 0.5 * torch.tensor([[0, 1], [1, 0]], dtype=torch.complex128)
SY = 0.5 * torch.tensor([[0, -1j], [1j, 0]], dtype=torch.complex128)
SZ = 0.5 * torch.tensor([[1, 0], [0, -1]], dtype=torch.complex128)

# sites 0 = TL, 1 = TR, 2 = BL, 3 = BR: the four edges of the plaquette, then its two diagonals
BONDS = ((0, 1), (2, 3), (0, 2), (1, 3), (0, 3), (1, 2))
N_OBS = 4 * 3 + len(BONDS)


def site_rdm(rho, s):
    """One-site matrix rho_s[k_s, b_s]: the three other sites of the plaquette traced."""
    d = round(rho.shape[0] ** 0.25)
    t = rho.reshape([d] * 8)
    k = list("abcd")
    b = list("efgh")
    for i in range(4):
        if i != s:
            b[i] = k[i]
    return torch.einsum("".join(k) + "".join(b) + "->" + k[s] + b[s], t)


def site_moment(rho, s):
    """(<S^x>, <S^y>, <S^z>) of site s (Eq. Mag1), real parts of Tr(S^a rho_s) / Tr rho_s."""
    r = site_rdm(rho, s).to(torch.complex128)
    tr = torch.trace(r).real
    return torch.stack([torch.trace(S @ r).real / tr for S in (SX, SY, SZ)])


def bond_correlation(rho, a, b):
    """<S_a . S_b> = Tr((S_a . S_b) rho_ab) / Tr rho_ab over the two-site matrix."""
    r = pair_rdm(rho, a, b).to(torch.complex128)
    ss = sum(torch.kron(S, S) for S in (SX, SY, SZ))
    return (torch.trace(ss @ r) / torch.trace(r)).real


def plaquette_observables(rho):
    """The 18 values of one plaquette: 4 site moments (x, y, z), then the BONDS correlations."""
    m = [site_moment(rho, s) for s in range(4)]
    c = [bond_correlation(rho, a, b).reshape(1) for a, b in BONDS]
    return torch.cat(m + c)


def magnetization(moments):
    """M = (1/N) sum_i |m_i| over the N rows (x, y, z) of ``moments`` (Eq. Mag1)."""
    return torch.linalg.vector_norm(moments, dim=1).mean()


def plaquette_order(obs_a, obs_b):
    """M_p = |sum of the four edge correlations of plaquette A minus those of B| / 4 (Eq. Mag2),
    from two rows of plaquette_observables output."""
    edges = slice(12, 16)
    return (obs_a[edges].sum() - obs_b[edges].sum()).abs() / 4
