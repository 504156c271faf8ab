"""Pins of the oracle's convergence test, its double-layer counterpart and the chi limit.

* delta (Sec. II C: the corner spectra converge) against hand-computed values,
  its invariances, and 0 at an exact fixed point;
* the double-layer CTMRG of Eq. Tred against closed forms (product states,
  singlet products, decoupled chains), independently of the nested network;
* nested and double-layer energies converging to each other as chi grows on
  generic correlated states (Appendix, Fig. SM-Compare; Sec. IV);
* the empty-cut case (a bond density matrix that vanishes to working
  precision) raising on the sites-derived start of exact singlet products;
* the stored run of the D=2, chi=8 Heisenberg workload to delta < 1e-10.
"""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import double_layer as dl
from oracle.ctmrg import CTM, DegenerateCut, corner_spectra, spectra_delta
from oracle.exact import brute_rdm
from oracle.rdm import energy, pair_rdm
from test_oracle_pins import _chain_exact

H = synth.heisenberg_bond()
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _diag_env(values_by_slot, chi):
    """A 1x1 grid whose corners are diagonal matrices with the given (possibly short) diagonals."""
    e = {}
    for k in ("C1", "C2", "C3", "C4"):
        v = torch.tensor(values_by_slot[k], dtype=torch.float64)
        e[k] = torch.diag(v)
    return [[e]]


def test_spectra_delta_hand_computed():
    chi = 3
    a = _diag_env({"C1": [3, 1], "C2": [3, 1], "C3": [3, 1], "C4": [3, 1]}, chi)
    b = _diag_env({"C1": [3, 1], "C2": [2, 1, 1], "C3": [3, 1], "C4": [1, 3]}, chi)
    sa, sb = corner_spectra(a, chi), corner_spectra(b, chi)
    # normalised, descending, zero-padded to chi
    assert torch.allclose(sa[0], torch.tensor([0.75, 0.25, 0.0], dtype=torch.float64), rtol=0, atol=1e-15)
    assert torch.allclose(sb[1], torch.tensor([0.5, 0.25, 0.25], dtype=torch.float64), rtol=0, atol=1e-15)
    # |0.75-0.5| + |0.25-0.25| + |0-0.25| on C2; C4 has the same spectrum in another order
    assert abs(spectra_delta(sb, sa) - 0.5) < 1e-15
    assert spectra_delta(sa, sa) == 0.0


def test_spectra_delta_gauge_and_scale_invariant():
    g = torch.Generator().manual_seed(0)
    chi = 5
    e = {k: torch.randn(chi, chi, generator=g, dtype=torch.float64) for k in ("C1", "C2", "C3", "C4")}
    f = {}
    for k, c in e.items():
        u = torch.linalg.qr(torch.randn(chi, chi, generator=g, dtype=torch.float64))[0]
        v = torch.linalg.qr(torch.randn(chi, chi, generator=g, dtype=torch.float64))[0]
        f[k] = 7.3 * (u @ c @ v.T)
    assert spectra_delta(corner_spectra([[f]], chi), corner_spectra([[e]], chi)) < 1e-14
    # a change of one singular value of one corner is seen
    f2 = dict(e)
    u, s, vh = torch.linalg.svd(e["C3"])
    s = s.clone()
    s[-1] *= 2.0
    f2["C3"] = u @ torch.diag(s) @ vh
    sp0, sp1 = corner_spectra([[e]], chi), corner_spectra([[f2]], chi)
    ref = (sp1[2] - sp0[2]).abs().sum().item()
    assert ref > 1e-3 and abs(spectra_delta(sp1, sp0) - ref) < 1e-15


def test_delta_vanishes_at_exact_fixed_point():
    # Neel product state on a 2-site cell: the environment is exact (rank 1) after one sweep
    A = synth.product_state_tensors(np.array([[1.0, 0.0], [0.0, 1.0]]))
    c = CTM(A, [[0, 1], [1, 0]], chi=4)
    c.run(1)
    _, delta = c.run(1)
    assert delta < 1e-14
    assert abs(energy(c, H, synth.heisenberg_terms(2, 2)).item() + 0.5) < 1e-14


# --- the double-layer network on its own --------------------------------------------

def test_double_layer_product_states():
    t1 = synth.heisenberg_terms(1, 1)
    c = dl.DoubleLayerCTM(synth.product_state_tensors(np.array([[1.0, 0.0]])), [[0]], 4)
    c.run(3)
    assert abs(dl.energy(c, H, t1).item() - 0.5) < 1e-14
    c = dl.DoubleLayerCTM(synth.product_state_tensors(np.array([[1.0, 0.0], [0.0, 1.0]])), [[0, 1], [1, 0]], 4)
    c.run(3)
    assert abs(dl.energy(c, H, synth.heisenberg_terms(2, 2)).item() + 0.5) < 1e-14
    # random product state, bond by bond: <S_a . S_b> = n_a . n_b / 4
    rng = np.random.default_rng(4)
    v = rng.standard_normal((2, 2))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    c = dl.DoubleLayerCTM(synth.product_state_tensors(v), [[0, 1]], 4)
    c.run(3)
    rho = dl.plaquette_rdm(c, 0, 0)
    n = [np.array([2 * a[0] * a[1], 0.0, a[0] ** 2 - a[1] ** 2]) for a in v]
    r2 = pair_rdm(rho, 0, 1)
    got = (torch.einsum("ji,ij->", torch.as_tensor(H), r2) / torch.trace(rho)).item()
    assert abs(got - n[0] @ n[1] / 4) < 1e-14


def test_double_layer_columnar_dimer_plaquette():
    A0 = synth.columnar_dimer_tensors()
    A = synth.gauge_transform(A0, [[0, 1]], 1)
    c = dl.DoubleLayerCTM(A, [[0, 1]], 8)
    c.run(8)
    assert abs(dl.energy(c, H, synth.heisenberg_terms(2, 1)).item() + 0.375) < 1e-13
    pat4 = [[[0, 1][x % 2] for x in range(4)] for _ in range(4)]
    for p in [(0, 0), (1, 0)]:
        rho = dl.plaquette_rdm(c, *p)
        ex = brute_rdm(A0, pat4, [p, (p[0] + 1, p[1]), (p[0], p[1] + 1), (p[0] + 1, p[1] + 1)]).reshape(16, 16)
        assert torch.allclose(rho / torch.trace(rho), ex / torch.trace(ex), atol=1e-13, rtol=0)


@pytest.mark.parametrize("seed", [3, 11])
def test_double_layer_decoupled_chains(seed):
    # corners of decoupled chains are rank one, so delta is 0 from the start and
    # says nothing about the edges: a fixed number of sweeps is run instead
    A = synth.vertical_chain_tensors(seed)
    eh, ev = _chain_exact(A)
    c = dl.DoubleLayerCTM(A, [[0]], 4, env0=synth.random_double_env_flat(4, 2, 1, 1, 1))
    c.run(600)
    rho = dl.plaquette_rdm(c, 0, 0)
    Ht = torch.as_tensor(H)
    got_h = (torch.einsum("ji,ij->", Ht, pair_rdm(rho, 0, 1)) / torch.trace(rho)).item()
    got_v = (torch.einsum("ji,ij->", Ht, pair_rdm(rho, 0, 2)) / torch.trace(rho)).item()
    assert abs(got_h - eh) < 1e-12 and abs(got_v - ev) < 1e-12


# --- chi limit: nested and double-layer agree (P6) -----------------------------------

@pytest.mark.parametrize("D,eps,seed,chis,last", [(2, 1.0, 2, (4, 8, 16), 5e-9), (3, 1.5, 5, (6, 12), 2e-7)])
def test_nested_and_double_layer_converge_with_chi(D, eps, seed, chis, last):
    """Correlated seeded states (product + relative noise eps): |E_nested(chi) - E_double(chi)|
    falls by more than 10x per chi step (measured: D=2 1.1e-5, 3.9e-8, 7.2e-10; D=3 1.9e-6, 4.7e-8)."""
    A = synth.near_product_tensors(1, 2, D, seed, eps=eps)
    t = synth.heisenberg_terms(1, 1)
    diffs = []
    for chi in chis:
        n = CTM(A, [[0]], chi)
        _, dn = n.run(400, tol=1e-11)
        d = dl.DoubleLayerCTM(A, [[0]], chi)
        _, dd = d.run(400, tol=1e-11)
        assert dn < 1e-11 and dd < 1e-11
        diffs.append(abs(energy(n, H, t).item() - dl.energy(d, H, t).item()))
    for a, b in zip(diffs, diffs[1:]):
        assert b < a / 10, diffs
    assert diffs[-1] < last, diffs


# --- the empty cut --------------------------------------------------------------------

@pytest.mark.parametrize("which", ["columnar", "orthogonal"])
def test_exact_singlet_products_from_sites_start_have_an_empty_cut(which):
    if which == "columnar":
        A, pattern = synth.gauge_transform(synth.columnar_dimer_tensors(), [[0, 1]], 1), [[0, 1]]
    else:
        A, pattern = synth.gauge_transform(synth.orthogonal_dimer_tensors(), [[0, 1], [2, 3]], 2), [[0, 1], [2, 3]]
    c = CTM(A, pattern, chi=8)
    with pytest.raises(DegenerateCut):
        c.run(10)


# --- the D=2, chi=8 Heisenberg workload run to convergence -----------------------------

def test_heisenberg_d2_chi8_stored_convergence_run():
    """The stored oracle run of this workload (tests/golden/heis_d2_chi8_convergence.json,
    written by tests/golden/make_golden.py) needs more than the 100-sweep budget to reach
    delta < 1e-10; the budget's last energy is within 1e-5 of the converged one, and the
    double-layer run converges in a few sweeps to an energy a finite-chi amount away."""
    with open(os.path.join(GOLDEN, "heis_d2_chi8_convergence.json")) as f:
        g = json.load(f)
    cfg = synth.CONFIGS["heis_d2_chi8"]
    A = synth.config_tensors(cfg, 0)
    t = synth.config_terms(cfg)
    c = CTM(A, cfg["pattern"], cfg["chi"])
    n, delta = c.run(cfg["sweeps"], tol=cfg["tol"])
    assert n == cfg["sweeps"] and delta > cfg["tol"]
    assert g["nested_sweeps_to_tol"] > cfg["sweeps"]
    assert abs(energy(c, H, t).item() - g["nested_E_converged"]) < 1e-5
    d = dl.DoubleLayerCTM(A, cfg["pattern"], cfg["chi"])
    n, delta = d.run(cfg["sweeps"], tol=cfg["tol"])
    assert delta < cfg["tol"] and n < 50
    assert abs(dl.energy(d, H, t).item() - g["double_E_converged"]) < 1e-10
    assert 1e-5 < abs(g["double_E_converged"] - g["nested_E_converged"]) < 1e-3


# --- the fixed-point gradient -----------------------------------------------------------

def test_converged_environment_is_a_fixed_point_entry_by_entry():
    """With the gauge reading (projector column signs, tensor signs) a converged
    environment is reproduced by one more sweep to rounding, not only up to signs."""
    from oracle.ctmrg import sweep
    for nt, pattern in [(1, [[0]]), (2, [[0, 1]])]:
        A = synth.near_product_tensors(nt, 2, 2, 6, eps=0.3)
        c = CTM(A, pattern, 8)
        _, delta = c.run(400, tol=1e-14)
        assert delta < 1e-14
        out = sweep(c.frames, c.env, c.chi, c.cutoff)
        gap = max((out[I][J][k] - c.env[I][J][k]).abs().max().item()
                  for I in range(len(out)) for J in range(len(out[0])) for k in out[I][J])
        assert gap < 1e-12


def test_fixed_point_gradient_matches_differences_of_the_reconverged_energy():
    """dE/dA of the converged energy (implicit differentiation at the fixed point,
    Eq. AD / Sec. IV) against fourth-order central differences (h = 1e-4) of the
    energy re-converged to delta < 1e-14 for each displaced A, on 4 seeded entries,
    pseudo-inverse cutoff 1e-6 (measured 7.6e-10); the gradient of one sweep from
    the converged environment misses by 1.3e-2 on the same entries."""
    from oracle.adjoint import detach_env, energy_and_grad, fixed_point_grad
    A = synth.near_product_tensors(1, 2, 2, 2, eps=1.0)
    t = synth.heisenberg_terms(1, 1)
    chi, cut = 8, 1e-6

    def reconverged(Ax):
        c = CTM(Ax, [[0]], chi, cutoff=cut)
        _, delta = c.run(3000, tol=1e-14)
        assert delta < 1e-14
        return energy(c, H, t).item(), c

    E0, c0 = reconverged(A)
    E, g, iters, gap = fixed_point_grad(A, [[0]], chi, c0.env, H, t, cutoff=cut)
    assert abs(E - E0) < 1e-13 and gap < 1e-12 and iters < 100
    idx = np.random.default_rng(0).choice(A.size, 4, replace=False)
    h = 1e-4
    fd = []
    for i in idx:
        vals = []
        for k in (-2, -1, 1, 2):
            Ap = A.copy().reshape(-1)
            Ap[i] += k * h
            vals.append(reconverged(Ap.reshape(A.shape))[0])
        fd.append((vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h))
    fd = np.array(fd)
    assert np.abs(g.reshape(-1)[idx].numpy() - fd).max() < 1e-8
    _, g1, _ = energy_and_grad(A, [[0]], chi, detach_env(c0.env), 1, H, t, cutoff=cut)
    assert np.abs(g1.reshape(-1)[idx].numpy() - fd).max() > 1e-3


def test_double_layer_gradient_against_central_differences():
    """dE/dA of the double-layer energy after 2 sweeps from a converged
    environment (autograd with the hand-written projector derivative) against
    fourth-order central differences of the same function (h = 1e-4, 4 seeded
    entries, cutoff 1e-6), and the scale identity <A, dE/dA> = 0."""
    A = synth.near_product_tensors(1, 2, 2, 5, 0.3)
    t = synth.heisenberg_terms(1, 1)
    Ht = torch.as_tensor(H)
    d = dl.DoubleLayerCTM(A, [[0]], 8, cutoff=1e-6)
    d.run(60, tol=1e-12)
    E, g, _ = dl.energy_and_grad(A, [[0]], 8, d.env, 2, Ht, t, cutoff=1e-6)
    flat = torch.as_tensor(A).reshape(-1)
    h = 1e-4
    for idx in np.random.default_rng(3).choice(flat.numel(), 4, replace=False):
        vals = []
        for k in (-2, -1, 1, 2):
            Ap = flat.clone()
            Ap[idx] += k * h
            vals.append(dl.energy_after_sweeps(Ap.reshape(A.shape), [[0]], 8, d.env, 2, Ht, t, cutoff=1e-6)[0].item())
        fd = (vals[0] - 8 * vals[1] + 8 * vals[2] - vals[3]) / (12 * h)
        assert abs(fd - g.reshape(-1)[idx].item()) < 1e-9, (idx, fd, g.reshape(-1)[idx].item())
    assert abs((torch.as_tensor(A) * g).sum().item()) < 1e-12
