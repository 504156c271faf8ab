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


def ssm_d6_chi72_grad():
    """E and dE/dA after n = 1, 2 sweeps from the environment of 4 sweeps from the
    sites-derived start, Shastry-Sutherland J_nn = 0.8, d=2 D=6 chi=72, 2x2 cell."""
    import numpy as np
    import torch
    from oracle.adjoint import detach_env, energy_and_grad
    cfg, A = _d6_state()
    H = synth.heisenberg_bond()
    t = synth.config_terms(cfg)
    c = CTM(A, cfg["pattern"], cfg["chi"])
    c.run(4)
    env0 = detach_env(c.env)
    out = {"command": "python tests/golden/make_golden.py ssm_d6_chi72_grad",
           "workload": "Shastry-Sutherland J_dimer=1 J_nn=0.8, 2x2 cell, d=2 D=6 chi=72, "
                       "synth.near_product_tensors(4, 2, 6, seed 5, eps 0.3); env0 = 4 sweeps from the sites start",
           "env0_sweeps": 4, "E_env0": energy(c, H, t).item(), "n": {}}
    sample = None
    for n in (1, 2):
        E, g, _ = energy_and_grad(A, cfg["pattern"], cfg["chi"], env0, n, H, t)
        g = g.reshape(-1)
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
    # the oracle's own spread: env0 perturbed by 1e-14 relative
    rng = np.random.default_rng(3)
    env1 = [[{k: v * (1 + 1e-14 * torch.from_numpy(rng.standard_normal(tuple(v.shape)))) for k, v in e.items()}
             for e in row] for row in env0]
    E1, g1, _ = energy_and_grad(A, cfg["pattern"], cfg["chi"], env1, 1, H, t)
    g1 = g1.reshape(-1)
    out["n"]["1"]["spread_E"] = abs(E1 - out["n"]["1"]["E"])
    out["n"]["1"]["spread_grad_sample"] = max(abs(a - b) for a, b in zip(g1[out["sample"]].tolist(),
                                                                        out["n"]["1"]["grad_sample"]))
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
