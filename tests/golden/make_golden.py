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


FIXTURES = {"heis_d2_chi8_convergence": heis_d2_chi8_convergence}

if __name__ == "__main__":
    names = sys.argv[1:] or list(FIXTURES)
    for name in names:
        t0 = time.time()
        out = FIXTURES[name]()
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f, indent=1)
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)
