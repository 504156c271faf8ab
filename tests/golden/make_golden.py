"""Write the stored expected values under tests/golden/ from the CPU oracle only.

Every value here is computed by ``oracle/`` from the seeded inputs of
``synth``; nothing comes from the GPU library.  Usage:

    python tests/golden/make_golden.py heis_d2_chi8_convergence

Each fixture records the command that wrote it.
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import torch  # noqa: E402

import synth  # noqa: E402
from oracle import double_layer as dl  # noqa: E402
from oracle.ctmrg import CTM  # noqa: E402
from oracle.rdm import energy  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def heis_d2_chi8_convergence():
    """Nested and double-layer runs of the D=2, chi=8 Heisenberg workload (seed 0) to delta < 1e-10."""
    cfg = synth.CONFIGS["heis_d2_chi8"]
    A = synth.config_tensors(cfg, 0)
    H = synth.heisenberg_bond()
    t = synth.config_terms(cfg)
    c = CTM(A, cfg["pattern"], cfg["chi"])
    trace = []
    n, delta, E100 = 0, float("inf"), None
    while delta >= cfg["tol"] and n < 5000:
        _, delta = c.run(1)
        n += 1
        if n == cfg["sweeps"]:
            E100 = energy(c, H, t).item()
        if n % 100 == 0:
            trace.append([n, energy(c, H, t).item(), delta])
    En = energy(c, H, t).item()
    d = dl.DoubleLayerCTM(A, cfg["pattern"], cfg["chi"])
    nd, dd = d.run(500, tol=cfg["tol"])
    return {
        "command": "python tests/golden/make_golden.py heis_d2_chi8_convergence",
        "workload": "Heisenberg square lattice, 1x1 cell, d=2 D=2 chi=8, A uniform[-1,1] seed 0 normalised",
        "nested_sweeps_to_tol": n, "nested_delta": delta, "nested_E_converged": En, "nested_E_at_100": E100,
        "nested_trace_every_100": trace,
        "double_sweeps_to_tol": nd, "double_delta": dd, "double_E_converged": dl.energy(d, H, t).item(),
    }


def _d6_state():
    cfg = synth.CONFIGS["ssm_d6_chi72"]
    # weakly entangled (product + 0.3 noise): the iteration settles from the
    # sites-derived start, so both sides reach the same environment
    A = synth.near_product_tensors(cfg["n_tensors"], 2, cfg["D"], 5, 0.3)
    return cfg, A


# Gradient fixtures.  Start environment: a seeded random one (no exactly
# degenerate singular values, unlike the sites-derived start, whose pairs of
# equal values are split by rounding and then weighted ~1e8 by the Lorentzian
# derivative), then 4 sweeps.  Pseudo-inverse cutoff 1e-6: with the default
# 1e-10, kept singular values between 1e-10 and 1e-6 of s_1 enter the
# derivative with weights up to s^(-3/2) and make the gradient move by 1e-6
# (relative) under rounding-level changes.
GRAD_CUTOFF = 1e-6
GRAD_START_SEED = 7


def _normalized_by_division(t):
    """The normalisation with its other rounding: t / |t| then the sign (the oracle multiplies by sign / |t|)."""
    flat = t.detach().reshape(-1)
    sg = -1.0 if flat[flat.abs().argmax()] < 0 else 1.0
    return (t / torch.linalg.norm(t)) * sg


def ssm_d6_chi72_grad():
    """E and dE/dA after n = 1, 2 sweeps from the environment of 4 sweeps from a seeded
    random start, Shastry-Sutherland J_nn = 0.8, d=2 D=6 chi=72, 2x2 cell, pseudo-inverse
    cutoff GRAD_CUTOFF in every sweep; the spread of the n = 1 result when every
    normalisation of the 4 + 1 sweeps rounds the other way."""
    import numpy as np
    import oracle.ctmrg as octm
    from oracle.adjoint import detach_env, energy_and_grad
    cfg, A = _d6_state()
    H = synth.heisenberg_bond()
    t = synth.config_terms(cfg)
    start = synth.random_env_flat(cfg["chi"], cfg["D"], 2, cfg["Lx"], cfg["Ly"], GRAD_START_SEED)
    c = CTM(A, cfg["pattern"], cfg["chi"], cutoff=GRAD_CUTOFF, env0=start)
    c.run(4)
    env0 = detach_env(c.env)
    out = {"command": "python tests/golden/make_golden.py ssm_d6_chi72_grad",
           "workload": "Shastry-Sutherland J_dimer=1 J_nn=0.8, 2x2 cell, d=2 D=6 chi=72, "
                       "synth.near_product_tensors(4, 2, 6, seed 5, eps 0.3); env0 = 4 sweeps from "
                       "synth.random_env_flat(72, 6, 2, 2, 2, seed 7)",
           "svd_cutoff": GRAD_CUTOFF, "start_seed": GRAD_START_SEED, "env0_sweeps": 4,
           "E_env0": energy(c, H, t).item(), "n": {}}
    sample = None
    for n in (1, 2):
        E, g, _ = energy_and_grad(A, cfg["pattern"], cfg["chi"], env0, n, H, t, cutoff=GRAD_CUTOFF)
        g = g.reshape(-1)
        if os.environ.get("GOLDEN_FULL_DIR"):
            torch.save(g.clone(), os.path.join(os.environ["GOLDEN_FULL_DIR"], f"ssm_d6_chi72_grad_n{n}.pt"))
        if sample is None:
            top = torch.argsort(g.abs(), descending=True)[:64].tolist()
            rng = np.random.default_rng(0)
            rest = rng.choice(g.numel(), size=448, replace=False).tolist()
            sample = sorted(set(top) | set(rest))
            out["sample"] = sample
        gt = g.reshape(cfg["n_tensors"], -1)
        out["n"][str(n)] = {"E": E, "grad_max": g.abs().max().item(),
                            "grad_norm_per_tensor": gt.norm(dim=1).tolist(),
                            "grad_sample": g[sample].tolist()}
    # the oracle's own spread: the same computation with the other rounding of every normalisation
    saved = octm.normalized
    octm.normalized = _normalized_by_division
    try:
        c1 = CTM(A, cfg["pattern"], cfg["chi"], cutoff=GRAD_CUTOFF, env0=start)
        c1.run(4)
        E1, g1, _ = energy_and_grad(A, cfg["pattern"], cfg["chi"], detach_env(c1.env), 1, H, t, cutoff=GRAD_CUTOFF)
    finally:
        octm.normalized = saved
    g1 = g1.reshape(-1)
    ref = out["n"]["1"]
    ref["spread_E"] = abs(E1 - ref["E"])
    ref["spread_grad_sample"] = max(abs(a - b) for a, b in zip(g1[sample].tolist(), ref["grad_sample"]))
    ref["spread_grad_norms"] = max(abs(a - b) for a, b in zip(g1.reshape(cfg["n_tensors"], -1).norm(dim=1).tolist(),
                                                              ref["grad_norm_per_tensor"]))
    return out


def ssm_d6_chi72_rdms():
    """Plaquette density matrices of all four plaquettes of the D=6, chi=72
    Shastry-Sutherland workload's own seeded tensors (uniform[-1,1], seed 0) at the
    sites-derived start environment, and the energy per site from them."""
    from oracle.rdm import plaquette_rdm
    cfg = synth.CONFIGS["ssm_d6_chi72"]
    A = synth.config_tensors(cfg, 0)
    H = synth.heisenberg_bond()
    t = synth.config_terms(cfg)
    c = CTM(A, cfg["pattern"], cfg["chi"])
    plaqs = [(0, 0), (1, 0), (0, 1), (1, 1)]
    return {"command": "python tests/golden/make_golden.py ssm_d6_chi72_rdms",
            "workload": "Shastry-Sutherland J_dimer=1 J_nn=0.8, 2x2 cell, d=2 D=6 chi=72, uniform[-1,1] seed 0; "
                        "sites-derived start environment",
            "plaquettes": plaqs,
            "rho": [plaquette_rdm(c.sites, c.env, *p).reshape(-1).tolist() for p in plaqs],
            "E": energy(c, H, t).item()}


FIXTURES = {"heis_d2_chi8_convergence": heis_d2_chi8_convergence, "ssm_d6_chi72_grad": ssm_d6_chi72_grad,
            "ssm_d6_chi72_rdms": ssm_d6_chi72_rdms}

if __name__ == "__main__":
    names = sys.argv[1:] or list(FIXTURES)
    for name in names:
        t0 = time.time()
        out = FIXTURES[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)
