"""Gradient of the energy (Eq. AD) from the library against the oracle.

E(A) is the energy after n sweeps from a given environment held constant
(Sec. IV); the environment is the oracle's converged one, where the iteration
is contracting and E is a smooth function of A.

Pseudo-inverse cutoff.  Every gradient here is taken with the cutoff 1e-6
on both sides.  With the default 1e-10, kept singular values between 1e-10
and 1e-6 of s_1 enter the derivative with weights up to s^(-3/2) (and their
pairs with terms 1/(s_i^2 - s_j^2)): the oracle's own gradient then moves by
up to 1e-6 relative under LAPACK's other SVD driver or a 1e-14 change of its
environment, which no bar of 1e-8 can accommodate.  With 1e-6 the spread is
at the rounding level.

Bar.  1e-8 of max(1, max|dE/dA|) in FP64 mode (three times the spread under
LAPACK's other SVD driver where that is measured and larger); FP32 mode 1e-6.
"""
import numpy as np
import pytest
import scipy.linalg
import torch

import synth
from oracle.adjoint import energy_and_grad
from oracle.ctmrg import CTM as OCTM, env_to_flat

pytestmark = pytest.mark.gpu

H = synth.heisenberg_bond()
CUT = 1e-6


@pytest.fixture(scope="module")
def ctm_mod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2512_14414_amd as m
    return m


GRAD_CASES = [
    # name, n_tensors, D, chi, pattern, kind, seed, converge sweeps, differentiated sweeps, calibrated bar
    ("rand_1x1_D2_chi8", 1, 2, 8, [[0]], "uniform", 1, 80, 2, False),
    ("np_2x2_D2_chi8", 4, 2, 8, [[0, 1], [2, 3]], "near_product", 5, 60, 1, True),
    ("np_2x1_D3_chi12", 2, 3, 12, [[0, 1]], "near_product", 5, 60, 1, True),
    ("np_2x2_D3_chi12", 4, 3, 12, [[0, 1], [2, 3]], "near_product", 5, 60, 1, True),
]


def _tensors(nt, D, kind, seed):
    if kind == "near_product":
        return synth.near_product_tensors(nt, 2, D, seed, 0.3)
    return synth.site_tensors(nt, 2, D, seed, kind)


def _converged(A, pattern, chi, sweeps):
    o = OCTM(A, pattern, chi, cutoff=CUT)
    o.run(sweeps)
    return o


def _ctx(m, A, pattern, chi, precision="fp64"):
    g = m.CTM(A, pattern, chi, precision=precision)
    g.set_option("svd_cutoff", CUT)
    return g


def _gesvd(M, full_matrices=False):
    U, s, Vh = scipy.linalg.svd(M.detach().numpy(), full_matrices=False, lapack_driver="gesvd")
    return torch.from_numpy(U), torch.from_numpy(s), torch.from_numpy(Vh)


@pytest.mark.parametrize("name,nt,D,chi,pattern,dist,seed,conv,n,calibrated", GRAD_CASES)
def test_energy_grad_matches_oracle(ctm_mod, monkeypatch, name, nt, D, chi, pattern, dist, seed, conv, n, calibrated):
    A = _tensors(nt, D, dist, seed)
    Ly, Lx = len(pattern), len(pattern[0])
    terms = synth.heisenberg_terms(Lx, Ly)
    o = _converged(A, pattern, chi, conv)
    Eo, go, _ = energy_and_grad(A, pattern, chi, o.env, n, H, terms, cutoff=CUT)
    scale = go.abs().max().item()
    bar = 1e-8 * max(1.0, scale)
    if calibrated:
        with monkeypatch.context() as mp:
            mp.setattr(torch.linalg, "svd", _gesvd)
            _, go2, _ = energy_and_grad(A, pattern, chi, o.env, n, H, terms, cutoff=CUT)
        bar = max(bar, 3 * (go2 - go).abs().max().item())
    g = _ctx(ctm_mod, A, pattern, chi)
    g.set_env(env_to_flat(o.env, o.sites, chi))
    E, grad = g.energy_grad(n, H, terms)
    err = (grad.cpu() - go).abs().max().item()
    print(f"{name}: E {E:.14f} |dE| {abs(E - Eo):.2e}; |dg|max {err:.2e} bar {bar:.2e} (|g|max {scale:.2e})")
    assert abs(E - Eo) < 1e-10 * max(1.0, abs(Eo))
    assert err <= bar


def test_energy_grad_fp32_mode(ctm_mod):
    name, nt, D, chi, pattern, dist, seed, conv, n, _ = GRAD_CASES[0]
    A = _tensors(nt, D, dist, seed)
    terms = synth.heisenberg_terms(1, 1)
    o = _converged(A, pattern, chi, conv)
    Eo, go, _ = energy_and_grad(A, pattern, chi, o.env, n, H, terms, cutoff=CUT)
    g = _ctx(ctm_mod, A, pattern, chi, precision="fp32")
    g.set_env(env_to_flat(o.env, o.sites, chi))
    E, grad = g.energy_grad(n, H, terms)
    err = (grad.cpu() - go).abs().max().item()
    print(f"fp32: |dE| {abs(E - Eo):.2e} |dg|max {err:.2e}")
    assert abs(E - Eo) < 1e-6
    assert err <= 1e-6 * max(1.0, go.abs().max().item())


def test_energy_grad_central_differences(ctm_mod):
    """Central differences (h = 1e-6) of the library's own energy on 6 seeded entries."""
    name, nt, D, chi, pattern, dist, seed, conv, n, _ = GRAD_CASES[1]
    A = _tensors(nt, D, dist, seed)
    terms = synth.heisenberg_terms(2, 2)
    o = _converged(A, pattern, chi, conv)
    env0 = env_to_flat(o.env, o.sites, chi)
    g = _ctx(ctm_mod, A, pattern, chi)
    g.set_env(env0)
    E, grad = g.energy_grad(n, H, terms)
    grad = grad.cpu()
    rng = np.random.default_rng(3)
    flat = torch.as_tensor(A).reshape(-1)
    h = 1e-6
    for idx in rng.choice(flat.numel(), 6, replace=False):
        vals = []
        for sgn in (1, -1):
            Ap = flat.clone()
            Ap[idx] += sgn * h
            g.set_tensors(Ap.reshape(A.shape))
            g.set_env(env0)
            g.sweep(n)
            vals.append(g.energy(H, terms))
        fd = (vals[0] - vals[1]) / (2 * h)
        gi = grad.reshape(-1)[idx].item()
        print(f"entry {idx}: fd {fd:.10f} grad {gi:.10f}")
        assert abs(fd - gi) < 1e-6 * max(1.0, abs(gi))


def test_autograd_function(ctm_mod):
    name, nt, D, chi, pattern, dist, seed, conv, n, _ = GRAD_CASES[0]
    A = _tensors(nt, D, dist, seed)
    terms = synth.heisenberg_terms(1, 1)
    o = _converged(A, pattern, chi, conv)
    env0 = env_to_flat(o.env, o.sites, chi)
    g = ctm_mod.CTM(A, pattern, chi)
    g.set_env(env0)
    E_ref, grad_ref = g.energy_grad(n, H, terms)
    g.set_env(env0)
    At = torch.as_tensor(A, dtype=torch.float64).cuda().requires_grad_(True)
    E = ctm_mod.CTMEnergy.apply(At, g, n, H, terms)
    (2.0 * E).backward()
    assert abs(E.item() - E_ref) < 1e-14
    assert torch.allclose(At.grad, 2.0 * grad_ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 3])
def test_cfg2_heisenberg_d4_chi32(ctm_mod, monkeypatch, n):
    """The D=4, chi=32 Heisenberg configuration (one tensor, N(0,1) seed 0):
    40 oracle sweeps, then E and dE/dA after n differentiated sweeps (n = 3
    recomputes two checkpointed sweeps) in FP64 and FP32 mode against the
    oracle, and central differences (h = 1e-6) of the library's own FP64
    energy after n sweeps on 20 seeded entries."""
    cfg = synth.CONFIGS["heis_d4_chi32"]
    A = synth.config_tensors(cfg, 0)
    terms = synth.config_terms(cfg)
    o = _converged(A, cfg["pattern"], cfg["chi"], 40)
    Eo, go, _ = energy_and_grad(A, cfg["pattern"], cfg["chi"], o.env, n, H, terms, cutoff=CUT)
    with monkeypatch.context() as mp:
        mp.setattr(torch.linalg, "svd", _gesvd)
        _, go2, _ = energy_and_grad(A, cfg["pattern"], cfg["chi"], o.env, n, H, terms, cutoff=CUT)
    scale = go.abs().max().item()
    spread = (go2 - go).abs().max().item()
    env0 = env_to_flat(o.env, o.sites, cfg["chi"])
    for precision, floor in (("fp64", 1e-8), ("fp32", 1e-6)):
        g = _ctx(ctm_mod, A, cfg["pattern"], cfg["chi"], precision=precision)
        g.set_env(env0)
        E, grad = g.energy_grad(n, H, terms)
        err = (grad.cpu() - go).abs().max().item()
        bar = max(floor * max(1.0, scale), 3 * spread)
        print(f"cfg2 n={n} {precision}: |dE| {abs(E - Eo):.2e}; |dg|max {err:.2e} bar {bar:.2e} (|g|max {scale:.2e}, "
              f"driver spread {spread:.2e})")
        assert abs(E - Eo) < (1e-10 if precision == "fp64" else 1e-6) * max(1.0, abs(Eo))
        assert err <= bar
    g = _ctx(ctm_mod, A, cfg["pattern"], cfg["chi"])
    g.set_env(env0)
    _, grad = g.energy_grad(n, H, terms)
    grad = grad.cpu().reshape(-1)
    flat = torch.as_tensor(A).reshape(-1)
    rng = np.random.default_rng(11)
    h = 1e-6
    worst = 0.0
    for idx in rng.choice(flat.numel(), 20, replace=False):
        vals = []
        for sgn in (1, -1):
            Ap = flat.clone()
            Ap[idx] += sgn * h
            g.set_tensors(Ap.reshape(A.shape))
            g.set_env(env0)
            g.sweep(n)
            vals.append(g.energy(H, terms))
        fd = (vals[0] - vals[1]) / (2 * h)
        worst = max(worst, abs(fd - grad[idx].item()))
    print(f"cfg2 n={n} central differences: max |fd - grad| {worst:.2e} (|g|max {scale:.2e})")
    assert worst < 1e-6 * max(1.0, scale)


def test_rowmajor_bf16_products_in_the_gradient(ctm_mod):
    """E and dE/dA of the D=6, chi=72 2x2 cell in BF16 mode with the dedicated
    kernel for large row-major (and transposed, and split-index) products on
    and off: the forward joins and their adjoints take it, with the same bf16
    products and accumulation order as the general kernel, so the results agree
    to 1e-6 of max |dE/dA| (observed: identical)."""
    cfg = synth.CONFIGS["ssm_d6_chi72"]
    A = synth.near_product_tensors(cfg["n_tensors"], 2, cfg["D"], 5, 0.3)
    terms = synth.config_terms(cfg)
    g = ctm_mod.CTM(A, cfg["pattern"], cfg["chi"], precision="bf16")
    g.sweep(2)
    env0 = g.get_env()
    out = []
    try:
        for flag in (1, 0):
            g.set_option("rowmajor_bf16", flag)
            g.set_env(env0)
            E, grad = g.energy_grad(1, H, terms)
            out.append((E, grad.cpu()))
    finally:
        g.set_option("rowmajor_bf16", 1)
    (E1, g1), (E0, g0) = out
    scale = g0.abs().max().item()
    print(f"rowmajor in E&grad: |dE| {abs(E1 - E0):.2e}, max |d grad| {(g1 - g0).abs().max().item():.2e} of {scale:.2e}")
    assert abs(E1 - E0) < 1e-8
    assert (g1 - g0).abs().max().item() <= 1e-6 * scale


@pytest.mark.parametrize("precision,key", [("fp64", "rowmajor_f64"), ("fp32", "rowmajor_f32")])
def test_rowmajor_mfma_products_in_the_gradient(ctm_mod, precision, key):
    """E and dE/dA of the D=6, chi=72 2x2 cell in FP64 and FP32 mode with the
    dedicated kernel for large products (A contiguous along k, B along n) on
    and off: the forward joins and their adjoints take it, and it runs the
    same MFMA chain over k in the same order as the general kernel for every
    output, so energy and gradient are identical."""
    cfg = synth.CONFIGS["ssm_d6_chi72"]
    A = synth.near_product_tensors(cfg["n_tensors"], 2, cfg["D"], 5, 0.3)
    terms = synth.config_terms(cfg)
    g = ctm_mod.CTM(A, cfg["pattern"], cfg["chi"], precision=precision)
    g.sweep(2)
    env0 = g.get_env()
    out = []
    try:
        for flag in (1, 0):
            g.set_option(key, flag)
            g.set_env(env0)
            E, grad = g.energy_grad(1, H, terms)
            out.append((E, grad.cpu()))
    finally:
        g.set_option(key, 1)
    (E1, g1), (E0, g0) = out
    scale = g0.abs().max().item()
    print(f"{key} in E&grad: |dE| {abs(E1 - E0):.2e}, max |d grad| {(g1 - g0).abs().max().item():.2e} of {scale:.2e}")
    assert E1 == E0
    assert torch.equal(g1, g0)


@pytest.mark.parametrize("name,n", [("ssm_d3_chi12", 3), ("ssm_d6_chi72", 2)])
def test_projector_cache_gives_identical_gradients(ctm_mod, name, n):
    """Option proj_cache: the reverse pass of ctm_energy_grad takes the
    projector blocks of the forward sweeps it recomputes instead of
    factorising again.  Energy and gradient equal, bit for bit, those of the
    run that recomputes them (n - 1 recomputed sweeps), and the environment the
    call leaves behind is the same."""
    if name == "ssm_d3_chi12":
        A = synth.near_product_tensors(4, 2, 3, 5, 0.3)
        pattern, chi = [[0, 1], [2, 3]], 12
        env0 = synth.random_env_flat(chi, 3, 2, 2, 2, 3)
    else:
        cfg = synth.CONFIGS[name]
        A = synth.near_product_tensors(cfg["n_tensors"], 2, cfg["D"], 5, 0.3)
        pattern, chi = cfg["pattern"], cfg["chi"]
        env0 = synth.random_env_flat(chi, cfg["D"], 2, 2, 2, 7)
    terms = synth.shastry_sutherland_terms(0.8, 1.0)
    out = []
    for cache in (0, 1):
        g = ctm_mod.CTM(A, pattern, chi)
        g.set_option("svd_cutoff", CUT)
        g.set_option("proj_cache", cache)
        g.set_env(torch.tensor(env0))
        E, grad = g.energy_grad(n, H, terms)
        out.append((E, grad.cpu(), g.get_env().cpu()))
        g.close()
    assert out[0][0] == out[1][0]
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][2], out[1][2])


def test_gradient_chain_takes_the_exact_svd(ctm_mod):
    """With the randomized projector SVD selected for plain sweeps, a
    differentiated chain of 2 sweeps (its forward sweep recomputed in the
    reverse pass) still takes the exact SVD in every sweep: E and dE/dA equal
    those of a context on the exact SVD bit for bit, with and without the
    projector cache, and the option is back in force afterwards."""
    A = synth.near_product_tensors(4, 2, 3, 5, 0.3)
    pattern, chi = [[0, 1], [2, 3]], 12
    env0 = torch.tensor(synth.random_env_flat(chi, 3, 2, 2, 2, 3))
    terms = synth.shastry_sutherland_terms(0.8, 1.0)
    out = []
    for method, cache in ((0, 1), (1, 1), (1, 0)):
        g = ctm_mod.CTM(A, pattern, chi)
        g.set_option("svd_cutoff", CUT)
        g.set_option("svd_method", method)
        g.set_option("proj_cache", cache)
        g.set_env(env0)
        E, grad = g.energy_grad(2, H, terms)
        g.set_env(env0)
        g.sweep(1)
        out.append((E, grad.cpu(), g.get_env().cpu()))
        g.close()
    for E, grad, _ in out[1:]:
        assert E == out[0][0] and torch.equal(grad, out[0][1])
    # the plain sweep afterwards follows the selected method again
    assert not torch.equal(out[1][2], out[0][2])
