"""Edge cases of the library against the oracle and the boundary's error rules.

* ragged sizes: chi and chi D not multiples of the 16-wide matrix-core tiles
  (chi = 13 with D = 3, chi = 9 with D = 2) on 2x2 and 1x2 cells;
* the smallest environment the nested network allows, chi = D d;
* no energy terms (E = 0, gradient 0), zero sweeps, a chain of 0
  differentiated sweeps (the energy's own derivative at a fixed environment);
* invalid terms and a too small corner-spectra buffer are refused with
  CTM_EINVAL and leave the context usable;
* a caller allocator behind a context (ctm_set_allocator) gives the default
  allocator's results and gets every block back.
"""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle.adjoint import energy_and_grad
from oracle.ctmrg import CTM as OCTM, env_to_flat
from oracle.rdm import energy as oenergy

pytestmark = pytest.mark.gpu

H = synth.heisenberg_bond()


@pytest.fixture(scope="module")
def ctm_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_14414_amd as m
    return m


RAGGED = [
    # name, tensors, chi, pattern, sweeps
    ("2x2_D3_chi13", synth.near_product_tensors(4, 2, 3, 11, 0.3), 13, [[0, 1], [2, 3]], 6),
    ("1x2_D2_chi9", synth.near_product_tensors(2, 2, 2, 12, 0.3), 9, [[0], [1]], 8),
    ("1x1_D3_chi6_minimum", synth.near_product_tensors(1, 2, 3, 13, 0.3), 6, [[0]], 8),
]


@pytest.mark.parametrize("name,A,chi,pattern,sweeps", RAGGED, ids=[c[0] for c in RAGGED])
def test_ragged_and_minimal_sizes_against_oracle(ctm_mod, name, A, chi, pattern, sweeps):
    """Weakly entangled states: delta of every sweep to 1e-8 + 1e-6 delta and the
    energy after the sweeps to 1e-10."""
    Ly, Lx = len(pattern), len(pattern[0])
    terms = synth.heisenberg_terms(Lx, Ly)
    g = ctm_mod.CTM(A, pattern, chi)
    o = OCTM(A, pattern, chi)
    err = 0.0
    for _ in range(sweeps):
        _, dg, _ = g.sweep(1, tol=1e-300)
        _, do = o.run(1)
        err = max(err, abs(dg - do) - 1e-6 * do)
    E, Eo = g.energy(H, terms), oenergy(o, H, terms).item()
    print(f"{name}: max delta excess {err:.1e}, E {E:.14f} oracle {Eo:.14f}")
    assert err < 1e-8
    assert abs(E - Eo) < 1e-10


def test_no_terms_zero_sweeps_and_zero_chain(ctm_mod):
    """No terms: E = 0 and dE/dA = 0.  sweep(0) changes nothing.  A chain of 0
    differentiated sweeps is the derivative of the energy at the fixed
    environment, against the oracle's autograd of the same (1e-10)."""
    A = synth.near_product_tensors(1, 2, 2, 5, 0.3)
    chi = 8
    g = ctm_mod.CTM(A, [[0]], chi)
    g.set_option("svd_cutoff", 1e-6)
    env0 = g.get_env().clone()
    n, delta, ok = g.sweep(0)
    assert n == 0 and torch.equal(g.get_env(), env0)
    assert g.energy(H, []) == 0.0
    E, grad = g.energy_grad(1, H, [])
    assert E == 0.0 and grad.abs().max().item() == 0.0
    g.set_env(env0)
    terms = synth.heisenberg_terms(1, 1)
    o = OCTM(A, [[0]], chi, cutoff=1e-6)
    o.run(4)
    g.set_env(env_to_flat(o.env, o.sites, chi))
    E0, g0 = g.energy_grad(0, H, terms)
    Eo, go, _ = energy_and_grad(A, [[0]], chi, o.env, 0, torch.as_tensor(H), terms, cutoff=1e-6)
    print(f"n = 0: E {E0:.14f} oracle {Eo:.14f}, max|dg| {(g0.cpu() - go).abs().max().item():.2e}")
    assert abs(E0 - Eo) < 1e-12
    assert (g0.cpu() - go).abs().max().item() < 1e-10 * max(1.0, go.abs().max().item())


def test_invalid_terms_and_small_buffers_are_refused(ctm_mod):
    A = synth.near_product_tensors(1, 2, 2, 5, 0.3)
    g = ctm_mod.CTM(A, [[0]], 8)
    for bad in ([(1, 0, 0, 1, 0.5)], [(0, 0, 2, 2, 0.5)], [(0, 0, 0, 4, 0.5)]):
        with pytest.raises(ctm_mod.CTMError) as err:
            g.energy(H, bad)
        assert err.value.code == -1
    # a corner-spectra buffer too small for all spectra
    lib = ctm_mod.LIB
    n = ctypes.c_int64()
    assert lib.ctm_corner_spectra(g._h, None, 0, ctypes.byref(n)) == 0
    small = (ctypes.c_double * 3)()
    rc = lib.ctm_corner_spectra(g._h, small, 3, ctypes.byref(n))
    assert rc == -1
    # the context still works
    g.sweep(2)
    assert np.isfinite(g.energy(H, synth.heisenberg_terms(1, 1)))


def test_caller_allocator_backs_the_context(ctm_mod):
    """ctm_set_allocator: with PyTorch's caching allocator behind a context
    (through counting wrappers), sweeps, the energy and E&grad give the
    default allocator's results bit for bit, the new blocks come from the
    caller's allocator, and every one of them is handed back, with the stream
    it was made for, by ctm_free at the latest."""
    A = synth.near_product_tensors(4, 2, 3, 11, 0.3)
    pattern, chi = [[0, 1], [2, 3]], 12
    terms = synth.shastry_sutherland_terms(0.7, 1.0)

    def run(g):
        g.set_option("svd_cutoff", 1e-6)
        g.sweep(4)
        E = g.energy(H, terms)
        Eg, grad = g.energy_grad(2, H, terms)
        return g.get_env().cpu().clone(), E, Eg, grad.cpu().clone()

    g0 = ctm_mod.CTM(A, pattern, chi)
    ref = run(g0)
    g0.close()
    talloc, tfree = ctm_mod.torch_allocator()
    live = {}
    counts = {"alloc": 0, "free": 0}

    def alloc(n, stream):
        p = talloc(n, stream)
        if p:
            live[p] = stream
            counts["alloc"] += 1
        return p

    def free(p, stream):
        assert live.pop(p) == stream
        counts["free"] += 1
        tfree(p, stream)

    g1 = ctm_mod.CTM(A, pattern, chi)
    g1.set_allocator(alloc, free)
    out = run(g1)
    assert counts["alloc"] > 0
    g1.close()
    print(f"caller allocator: {counts['alloc']} blocks made, {counts['free']} handed back")
    assert not live and counts["free"] == counts["alloc"]
    for a, b in zip(ref, out):
        if isinstance(a, torch.Tensor):
            assert torch.equal(a, b)
        else:
            assert a == b
    # exactly one of the two callbacks: refused by the binding and by the library
    g2 = ctm_mod.CTM(A, pattern, chi)
    with pytest.raises(ValueError):
        g2.set_allocator(alloc, None)
    from paper_2512_14414_amd.binding import ALLOC_FN, FREE_FN
    only_free = FREE_FN(lambda p, st, u: None)
    assert ctm_mod.LIB.ctm_set_allocator(g2._h, ALLOC_FN(), only_free, None) == -1
    g2.sweep(1)
