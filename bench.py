#!/usr/bin/env python
"""Benchmark of the nested CTMRG hot path on one MI355X.

Workload: the Shastry-Sutherland model (J_dimer = 1 on the orthogonal dimers,
J_nn = 0.8 on the square-lattice bonds) on a 2x2 cell of four distinct site
tensors, d = 2, D = 6, chi = 72, each tensor uniform in [-1, 1] (seed 0) and
normalised; bulk contractions in the requested precision (default bf16 with
FP32 accumulation), projector QR/SVD in FP64.

A step is one CTMRG sweep (left, right, up and down moves: 64 projector
computations and the environment updates); ``value`` is sweeps per second.
The same line reports the energy evaluation time, the FP64-mode sweep rate,
the roofline of the MFMA contraction kernel measured live with HIP events on
the library's stream, and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision bf16|fp32|fp64]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CTMRG sweeps/s + E&grad evals/s at D=6,chi=72 (mixed vs FP64), |dE| vs oracle"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}   # MI355X dense matrix-core peaks


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16", choices=("bf16", "fp32", "fp64"))
    ap.add_argument("--config", default="ssm_d6_chi72")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    import paper_2512_14414_amd as ctm

    cfg = synth.CONFIGS[args.config]
    A = synth.config_tensors(cfg, 0)
    H = synth.heisenberg_bond()
    terms = synth.config_terms(cfg)
    chi = cfg["chi"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    # ---- production precision: warm-up, timed sweeps
    g = ctm.CTM(A, cfg["pattern"], chi, precision=args.precision)
    log(f"[bench] {args.config} precision={args.precision}: warmup {args.warmup}")
    g.sweep(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} sweeps")
    t0 = time.perf_counter()
    g.sweep(args.steps)
    torch.cuda.synchronize()
    t_sweeps = time.perf_counter() - t0
    sweeps_per_s = args.steps / t_sweeps

    # ---- live roofline of the contraction kernel over one more sweep
    g.profile_begin()
    t0 = time.perf_counter()
    g.sweep(1)
    torch.cuda.synchronize()
    t_prof = time.perf_counter() - t0
    prof = g.profile_end()
    log(f"[bench] profiled sweep {t_prof * 1e3:.1f} ms: {prof}")

    # ---- energy (2x2 reduced density matrices of all four plaquettes)
    E, t_energy = None, None
    if not args.no_energy:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E = g.energy(H, terms)
        torch.cuda.synchronize()
        t_energy = time.perf_counter() - t0
        log(f"[bench] energy {E:.10f} in {t_energy * 1e3:.1f} ms")

    # ---- FP64 mode for comparison
    fp64_sweeps_per_s = None
    if args.precision != "fp64" and args.fp64_steps > 0:
        g64 = ctm.CTM(A, cfg["pattern"], chi, precision="fp64")
        g64.sweep(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g64.sweep(args.fp64_steps)
        torch.cuda.synchronize()
        fp64_sweeps_per_s = args.fp64_steps / (time.perf_counter() - t0)
        log(f"[bench] fp64 sweeps/s {fp64_sweeps_per_s:.3f}")
        g64.close()

    # ---- roofline of the dominant kernel family (bulk contractions in the production path)
    path = args.precision
    ms, flops, launches = prof[path]
    if launches == 0:
        path = "fp64"
        ms, flops, launches = prof[path]
    achieved = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    roofline = {
        "kernel": f"contract_kernel ({path} MFMA path)",
        "bound": "mfma",
        "achieved": round(achieved, 3),
        "peak": PEAK_TFLOPS[path],
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_TFLOPS[path], 5),
        "traffic": None,
        "launches_per_sweep": launches,
        "avg_launch_us": round(ms * 1e3 / max(launches, 1), 2),
        "algorithmic_flops_per_sweep": flops,
        "kernel_ms_per_sweep": round(ms, 3),
        "fp64_path_ms_per_sweep": round(prof["fp64"][0], 3),
        "sweep_ms": round(t_prof * 1e3, 2),
    }

    # ---- CPU oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.ctmrg import CTM as OracleCTM
        n_cpu = 3
        o = OracleCTM(A, cfg["pattern"], chi)
        t0 = time.perf_counter()
        o.run(n_cpu)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": round(n_cpu / t_cpu, 5), "unit": "sweeps/s", "cores": torch.get_num_threads(),
               "kind": "oracle", "sample": f"{n_cpu} sweeps of the same workload (float64, sites-derived start)"}
        log(f"[bench] oracle {n_cpu} sweeps in {t_cpu:.1f} s")

    out = {
        "metric": METRIC,
        "value": round(sweeps_per_s, 4),
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_sweeps / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{args.config}: Shastry-Sutherland J_dimer=1 J_nn=0.8, 2x2 cell of 4 tensors, "
                               f"d=2 D=6 chi=72, uniform[-1,1] seed 0; step = 1 CTMRG sweep",
                   "precision": args.precision, "projectors": "fp64 QR+SVD"},
        "fp64_sweeps_per_s": None if fp64_sweeps_per_s is None else round(fp64_sweeps_per_s, 4),
        "energy_s": None if t_energy is None else round(t_energy, 4),
        "energy": E,
        "egrad_per_s": None,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
