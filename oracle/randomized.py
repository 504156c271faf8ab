"""Projectors from a partial SVD found by a randomized range finder.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Only the chi leading singular triplets of M = R_n R_s^T enter the projectors
of Eq. PQ (Sec. II C), while an exact SVD computes all r = chi D of them.
The cheaper projectors that the paper's outlook proposes (Sec. IV: partial
or randomized SVD) are built here with the randomized range finder and the
subsequent SVD of Halko, Martinsson and Tropp (SIAM Rev. 53, 217 (2011)):
their Algorithm 4.4 (randomized subspace iteration: a test matrix Omega,
Y = M Omega, and q passes that multiply by M^T and by M again, each product
orthonormalised), and Algorithm 5.1 (B = Q^T M, the SVD of the small B, and
U = Q U_B).

Test matrix: Omega[i, j] = 2 u - 1 with u = (splitmix64(seed, i * k + j) >> 11)
* 2^-53, k = chi + oversample columns, the same SplitMix64 counter rule as the
surrogate's initialisation; both implementations generate it from this
definition.

The result is exact (to rounding) whenever M has rank at most k; otherwise
the kept triplets approach the exact ones as (s_{k+1} / s_chi)^(2q+1).
"""
from __future__ import annotations

import numpy as np
import torch

from .ctmrg import check_cut, projector_signs, truncated_inverse_sqrt
from .mlp import uniform_counter


def test_matrix(r: int, k: int, seed: int) -> torch.Tensor:
    """Omega (r x k), entries 2u - 1 from SplitMix64 with counter i * k + j."""
    u = uniform_counter(seed, 0, r * k)
    return torch.from_numpy(2.0 * u - 1.0).reshape(r, k)


def leading_triplets(M, k, power, seed):
    """Approximate leading singular triplets (U, s, V) of M (r x r) from a k-column
    range finder with ``power`` subspace iterations (Algorithms 4.4 and 5.1)."""
    r = M.shape[0]
    Q = torch.linalg.qr(M @ test_matrix(r, k, seed), mode="reduced")[0]
    for _ in range(power):
        Z = torch.linalg.qr(M.T @ Q, mode="reduced")[0]
        Q = torch.linalg.qr(M @ Z, mode="reduced")[0]
    B = Q.T @ M
    Ub, s, Vh = torch.linalg.svd(B, full_matrices=False)
    return Q @ Ub, s, Vh.T


def randomized_bond_projectors(N, S, chi, cutoff, oversample=8, power=2, seed=0):
    """P, Q of Eq. PQ with the truncated SVD of M replaced by its randomized partial SVD.

    The QR factors and the pseudo-inverse weights are those of ``ctmrg.bond_projectors``;
    the k = min(chi + oversample, r) approximate triplets stand in for the exact ones,
    of which chi' = min(chi, k) are kept; column signs as in ``projector_signs``.
    """
    Rn = torch.linalg.qr(N, mode="reduced")[1]
    Rs = torch.linalg.qr(S, mode="reduced")[1]
    M = Rn @ Rs.T
    r = M.shape[0]
    k = min(chi + oversample, r)
    U, s, V = leading_triplets(M, k, power, seed)
    check_cut(s, N, S)
    kk, w = truncated_inverse_sqrt(s, chi, cutoff)
    P = (Rs.T @ V[:, :kk]) * w
    Q = (Rn.T @ U[:, :kk]) * w
    sg = projector_signs(P)
    return P * sg, Q * sg, s


def projector_fn(oversample=8, power=2, seed=0):
    """A ``proj`` argument for ``ctmrg.left_move`` / ``CTM.run`` with randomized projectors."""
    def proj(N, S, chi, cutoff):
        return randomized_bond_projectors(N, S, chi, cutoff, oversample, power, seed)
    return proj
