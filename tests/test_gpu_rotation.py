"""Sublattice rotation (Discussion): the Heisenberg model with one sublattice
rotated by -i sigma_y has the bond term -SxSx + SySy - SzSz on every bond, so a
Neel-ordered state fits a 1x1 cell instead of the 2x2 checkerboard.

The library takes the rotated bond term like any other H_bond; compared with
the oracle are the closed forms of product states and the converged energies
of the 1x1 rotated cell and of the equivalent checkerboard cell.
"""
import numpy as np
import pytest
import torch

import synth
from oracle.ctmrg import CTM as OCTM
from oracle.rdm import energy as oenergy

pytestmark = pytest.mark.gpu

H = synth.heisenberg_bond()
HR = synth.heisenberg_bond_rotated()


@pytest.fixture(scope="module")
def ctm_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_14414_amd as m
    return m


def test_rotated_product_states(ctm_mod):
    """Uniform up and x-polarised product states under the rotated term: the
    Neel energies -1/2 per site of the unrotated model."""
    t = synth.heisenberg_terms(1, 1)
    for v in ([1.0, 0.0], [1.0, 1.0]):
        g = ctm_mod.CTM(synth.product_state_tensors([v]), [[0]], 2)
        g.sweep(3)
        assert abs(g.energy(HR, t) + 0.5) < 1e-13


@pytest.mark.parametrize("chi", [4, 8])
def test_rotated_cell_and_checkerboard_against_oracle(ctm_mod, chi):
    """Converged (delta < 1e-11) energies of the 1x1 rotated cell and of the
    checkerboard 2x2 cell, each against the oracle's (1e-10); their
    difference shrinks with chi as in the oracle (the same network, truncated
    at different nested positions)."""
    A = synth.near_product_tensors(1, 2, 2, 2, 1.0)
    B = np.concatenate([A, synth.rotate_physical(A)])
    t1, t2 = synth.heisenberg_terms(1, 1), synth.heisenberg_terms(2, 2)
    g1 = ctm_mod.CTM(A, [[0]], chi)
    assert g1.sweep(600, tol=1e-11)[2]
    E1 = g1.energy(HR, t1)
    g2 = ctm_mod.CTM(B, [[0, 1], [1, 0]], chi)
    assert g2.sweep(600, tol=1e-11)[2]
    E2 = g2.energy(H, t2)
    o1 = OCTM(A, [[0]], chi)
    o1.run(600, tol=1e-11)
    o2 = OCTM(B, [[0, 1], [1, 0]], chi)
    o2.run(600, tol=1e-11)
    Eo1 = oenergy(o1, torch.as_tensor(HR), t1).item()
    Eo2 = oenergy(o2, torch.as_tensor(H), t2).item()
    print(f"chi {chi}: rotated 1x1 {E1:.12f} (oracle {Eo1:.12f}), checkerboard {E2:.12f} (oracle {Eo2:.12f})")
    assert abs(E1 - Eo1) < 1e-10 and abs(E2 - Eo2) < 1e-10
    assert abs(abs(E1 - E2) - abs(Eo1 - Eo2)) < 1e-10
