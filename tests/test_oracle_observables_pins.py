"""Pins of the oracle's order parameters (Eqs. Mag1, Mag2) on states whose
moments and bond correlations have closed forms."""
import math

import numpy as np
import torch

from oracle.observables import BONDS, magnetization, plaquette_observables, plaquette_order


def rho_of(psi, scale=1.0):
    """Unnormalised plaquette matrix rho[k; b] = scale * psi[k] psi[b] of a real 16-vector psi."""
    p = torch.as_tensor(psi, dtype=torch.float64)
    return scale * torch.outer(p, p)


SINGLET = np.array([0.0, 1.0, -1.0, 0.0]) / math.sqrt(2.0)   # (|ud> - |du>)/sqrt 2, basis (u, d)


def test_product_state_moments_and_bonds():
    # cos t|u> + sin t|d> per site: <S^x> = sin(2t)/2, <S^z> = cos(2t)/2, |m| = 1/2;
    # a product state has <S_a . S_b> = m_a . m_b
    th = [0.3, -1.1, 2.0, 0.7]
    psi = np.ones(1)
    for t in th:
        psi = np.kron(psi, [math.cos(t), math.sin(t)])
    obs = plaquette_observables(rho_of(psi, 3.7))
    m = np.array([[math.sin(2 * t) / 2, 0.0, math.cos(2 * t) / 2] for t in th])
    assert np.allclose(obs[:12].numpy(), m.ravel(), atol=1e-15)
    for i, (a, b) in enumerate(BONDS):
        assert abs(obs[12 + i].item() - m[a] @ m[b]) < 1e-15
    assert abs(magnetization(obs[:12].reshape(4, 3)).item() - 0.5) < 1e-15


def test_two_singlets():
    # singlets on TL-TR and BL-BR: <S.S> = -3/4 on those bonds, 0 across (the two pairs are independent
    # and each has zero moment); every moment vanishes
    psi = np.kron(SINGLET, SINGLET)
    obs = plaquette_observables(rho_of(psi, 0.2))
    assert np.allclose(obs[:12].numpy(), 0.0, atol=1e-15)
    want = {(0, 1): -0.75, (2, 3): -0.75}
    for i, ab in enumerate(BONDS):
        assert abs(obs[12 + i].item() - want.get(ab, 0.0)) < 1e-15, ab
    assert magnetization(obs[:12].reshape(4, 3)).item() == 0.0


def test_triplet_and_vertical_singlets_plaquette_order():
    # |uu> on TL-TR (S.S = +1/4) times |dd> on BL-BR; vertical singlets TL-BL, TR-BR (-3/4 each).
    # Sites in plaquette order TL, TR, BL, BR: the vertical-singlet state is built on (TL, BL) x (TR, BR)
    # and its axes reordered.
    up, dn = np.array([1.0, 0.0]), np.array([0.0, 1.0])
    ferro = np.kron(np.kron(up, up), np.kron(dn, dn))
    t = np.kron(SINGLET, SINGLET).reshape(2, 2, 2, 2)          # axes TL, BL, TR, BR
    vert = t.transpose(0, 2, 1, 3).ravel()                      # axes TL, TR, BL, BR
    oa = plaquette_observables(rho_of(ferro))
    ob = plaquette_observables(rho_of(vert))
    # ferro: edges TL-TR +1/4, BL-BR +1/4, TL-BL -1/4, TR-BR -1/4 (sum 0); vertical: 0 + 0 - 3/4 - 3/4
    assert np.allclose(oa[12:16].numpy(), [0.25, 0.25, -0.25, -0.25], atol=1e-15)
    assert np.allclose(ob[12:16].numpy(), [0.0, 0.0, -0.75, -0.75], atol=1e-15)
    assert abs(plaquette_order(oa, ob).item() - 1.5 / 4) < 1e-15
    # moments: ferro sites +-1/2 along z
    assert np.allclose(oa[:12].numpy(), [0, 0, 0.5, 0, 0, 0.5, 0, 0, -0.5, 0, 0, -0.5], atol=1e-15)


def test_mixture_and_non_hermitian_rho():
    # an equal mixture halves the singlet correlations; a non-symmetric real rho leaves <S^y> = 0 and
    # gives <S^x> from the symmetric part
    psi = np.kron(SINGLET, SINGLET)
    t = psi.reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).ravel()
    rho = 0.5 * (rho_of(psi) + rho_of(t))
    obs = plaquette_observables(rho)
    assert np.allclose(obs[12:16].numpy(), [-0.375, -0.375, -0.375, -0.375], atol=1e-15)
    g = torch.Generator().manual_seed(3)
    r = torch.rand(16, 16, generator=g, dtype=torch.float64) + 4 * torch.eye(16, dtype=torch.float64)
    o1 = plaquette_observables(r)
    o2 = plaquette_observables(0.5 * (r + r.T))
    assert torch.allclose(o1, o2, atol=1e-15)
    assert o1[1::3][:4].abs().max().item() == 0.0
