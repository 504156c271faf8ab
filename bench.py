#!/usr/bin/env python
"""Benchmark of the nested CTMRG hot path on one MI355X.

Workload: the Shastry-Sutherland model (J_dimer = 1 on the orthogonal dimers,
J_nn = 0.8 on the square-lattice bonds) on a 2x2 cell of four distinct site
tensors, d = 2, D = 6, chi = 72, each tensor uniform in [-1, 1] (seed 0) and
normalised; bulk contractions in the requested precision (default bf16 with
FP32 accumulation), projector QR/SVD in FP64.

A step is one CTMRG sweep (left, right, up and down moves: 64 projector
computations and the environment updates); ``value`` is sweeps per second.
The same line reports:
* energy+gradient evaluations per second (energy after n differentiated
  sweeps from the current environment, n = 2 by default so that the
  checkpointed recompute of the earlier sweep is timed, and its gradient by
  the hand-written reverse pass) in every precision mode, ``egrad_per_s``
  being the mixed mode (FP64 sweep, FP32 energy), whose gradient meets the
  1e-6 bar against the oracle;
* each mode's error of E and dE/dA against the stored FP64 oracle values of
  tests/golden/ssm_d6_chi72_grad.json (a weakly entangled state of the same
  shape, 4 sweeps, pseudo-inverse cutoff 1e-6) and against FP64 mode;
* the roofline of the kernel family that dominates a sweep (timed live with
  HIP events on the library's stream), its fraction counted with the
  method's 21 r^3 flops per r x r SVD, and the matrix-core fraction of the
  absorption contractions;
* the D = 9, chi = 100 Heisenberg 2x1 workload: sweeps/s and E&grad/s with
  n = 2 checkpointed sweeps, FP64 against mixed;
* the CPU oracle timed on a bounded sample with all host threads and with one.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision bf16|fp32|fp64|mixed]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CTMRG sweeps/s + E&grad evals/s at D=6,chi=72 (mixed vs FP64), |dE| vs oracle"
# MI355X peaks: dense matrix cores per path, FP64 vector ALU for the Jacobi and QR families
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "jacobi": 78.6, "qr_panel": 78.6}
BOUND = {"fp64": "mfma", "fp32": "mfma", "bf16": "mfma", "jacobi": "alu", "qr_panel": "alu"}
# HBM traffic per launch of the Jacobi kernel (one launch runs the whole
# iteration of one batched SVD) from two rocprofv3 --pmc passes over this
# workload's sweeps (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, averaged
# over the 16 dispatches of the event-timed sweep, the last 16 of the 128 after the
# default 2 warm-up and 5 timed sweeps), each scaled by what the counter reads
# for a copy of known size
# (bench.py --copy-probe 256: FETCH_SIZE reads half of the bytes copied, so x2;
# WRITE_SIZE reads them exactly, x1).  Valid for the kernel source it was taken
# on (hash of the kernel's text), else reported as null.
TRAFFIC = {"jacobi": {"workload": "ssm_d6_chi72", "precision": "bf16",
                      "fetch_kib": 2776636.3, "fetch_scale": 2.0, "write_kib": 4943883.5, "write_scale": 1.0,
                      "source_sha256": "28f137f25291d48796d5e8bd2394262b3ab9b71e71f09e193c65ce0894d1e2e5",
                      "source": ("paper_2512_14414_amd/csrc/kernels.hip", "constexpr int BJ_BW = 8;",
                                 "hipError_t launch_bjac_round(")}}
KERNEL = {"fp64": "contract_kernel<MODE_F64> (FP64 MFMA)", "fp32": "contract_kernel<MODE_F32> (FP32 MFMA)",
          "bf16": "contract_kernel<MODE_BF16> (BF16 MFMA, FP32 accumulation)",
          "jacobi": "bjac_svd_kernel (block one-sided Jacobi, all sweeps of one batched SVD per launch, FP64)",
          "qr_panel": "panel_kernel (Householder QR panel, FP64)"}


def workload_name(name, cfg):
    if cfg["model"] == "ssm":
        model = f"Shastry-Sutherland J_dimer={cfg['J_dimer']:g} J_nn={cfg['J_nn']:g}"
    else:
        model = f"Heisenberg J={cfg.get('J', 1.0):g}"
    dist = "uniform[-1,1]" if cfg["dist"] == "uniform" else "N(0,1)"
    return (f"{name}: {model}, {cfg['Lx']}x{cfg['Ly']} cell of {cfg['n_tensors']} tensors, d={cfg['d']} "
            f"D={cfg['D']} chi={cfg['chi']}, {dist} seed 0, normalised; step = 1 CTMRG sweep")


def traffic_per_launch(fam, config, precision):
    """HBM bytes per launch of family ``fam`` from the counter runs, or None
    when none were taken for this workload and precision or the kernel's
    source changed since."""
    import hashlib
    t = TRAFFIC.get(fam)
    if t is None or t["workload"] != config or t["precision"] != precision:
        return None
    path, first, last = t["source"]
    try:
        text = open(os.path.join(ROOT, path)).read()
        a, b = text.index(first), text.index(last)
    except (OSError, ValueError):
        return None
    if hashlib.sha256(text[a:b].encode()).hexdigest() != t["source_sha256"]:
        return None
    return round(1024.0 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16", choices=("bf16", "fp32", "fp64", "mixed"))
    ap.add_argument("--config", default="ssm_d6_chi72")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--egrad-sweeps", type=int, default=2)
    ap.add_argument("--d9-egrad-sweeps", type=int, default=2,
                    help="differentiated sweeps of the D=9, chi=100 E&grad (checkpointed: all but the last recomputed)")
    ap.add_argument("--no-d9", action="store_true", help="skip the D=9, chi=100 sub-record")
    ap.add_argument("--no-randomized", action="store_true", help="skip the sweeps with randomized projectors")
    ap.add_argument("--no-double-layer", action="store_true",
                    help="skip the nested against double-layer sweeps at D=5, chi=50")
    ap.add_argument("--plain-jacobi-launch", action="store_true",
                    help="launch the one-launch Jacobi kernel plainly instead of cooperatively (same results); "
                         "rocprofv3's counter collection does not survive cooperative launches")
    ap.add_argument("--no-egrad", action="store_true")
    ap.add_argument("--egrad-warmup", type=int, default=1, help="untimed E&grad evaluations before the timed one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--lbfgs", action="store_true",
                    help="instead of the sweep benchmark: time to |E - E_plain| < 1e-5 of L-BFGS on the D=5, chi=50 "
                         "Shastry-Sutherland workload, plain FP64 against the mixed mode with and without the surrogate")
    ap.add_argument("--lbfgs-iters", type=int, default=120)
    ap.add_argument("--lbfgs-sweeps", type=int, default=10, help="differentiated sweeps per L-BFGS evaluation")
    ap.add_argument("--lbfgs-objective", choices=("chain", "fixed_point"), default="chain",
                    help="chain: E and dE/dA after --lbfgs-sweeps differentiated sweeps from one fixed environment; "
                         "fixed_point: sweeps from the previous evaluation's environment until the plaquette density "
                         "matrices settle (conv_rdm, 1e-10, at most --lbfgs-max-sweeps), then the fixed-point "
                         "gradient of the converged energy")
    ap.add_argument("--lbfgs-max-sweeps", type=int, default=50)
    ap.add_argument("--lbfgs-D", type=int, default=None, help="bond dimension of the L-BFGS workload (default 5)")
    ap.add_argument("--lbfgs-chi", type=int, default=None, help="environment dimension of the L-BFGS workload (default 50)")
    ap.add_argument("--lbfgs-sur-start", type=int, default=51, help="first L-BFGS iteration the surrogate screens")
    ap.add_argument("--lbfgs-runs", default="all",
                    help="comma-separated subset of plain_fp64,mixed,mixed_surrogate (runs of about ten minutes "
                         "each can then go into separate invocations)")
    ap.add_argument("--lbfgs-e-plain", type=float, default=None,
                    help="E_plain of an earlier plain FP64 run, when that run is not part of this invocation")
    ap.add_argument("--lbfgs-plain-seconds", type=float, default=None,
                    help="the earlier plain FP64 run's seconds to target, for the speedup")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a device buffer of MIB mebibytes once (calibration of the HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: --gpus must be 1 (the library has no multi-GPU path)"}))
        sys.exit(2)

    import torch
    if args.copy_probe > 0:
        # source and destination are written first, then a buffer as large as
        # both is written so that neither stays in the last-level cache
        n = args.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        flush = torch.zeros(2 * n, dtype=torch.float32, device="cuda:0")
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "check": float(y[-1].item()) + float(flush[0].item())}), flush=True)
        return
    import synth
    import paper_2512_14414_amd as ctm
    if args.lbfgs:
        return lbfgs_time_to_target(args, torch, synth, ctm)

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
    if args.plain_jacobi_launch:
        g.set_option("jacobi_cooperative", 0)
    log(f"[bench] {args.config} precision={args.precision}: warmup {args.warmup}")
    g.sweep(args.warmup)
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} sweeps")
    t0 = time.perf_counter()
    g.sweep(args.steps)
    torch.cuda.synchronize()
    t_sweeps = time.perf_counter() - t0
    sweeps_per_s = args.steps / t_sweeps
    log(f"[bench] {sweeps_per_s:.3f} sweeps/s")

    # ---- the same sweeps with the randomized partial-SVD projectors (k = chi + 8, 2 passes)
    sweeps_per_s_rand = None
    if not args.no_randomized:
        gr = ctm.CTM(A, cfg["pattern"], chi, precision=args.precision)
        gr.set_option("svd_method", 1)
        gr.sweep(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gr.sweep(args.steps)
        torch.cuda.synchronize()
        sweeps_per_s_rand = args.steps / (time.perf_counter() - t0)
        gr.close()
        log(f"[bench] randomized projectors: {sweeps_per_s_rand:.3f} sweeps/s")

    # ---- live kernel timing over one more sweep
    g.profile_begin()
    t0 = time.perf_counter()
    g.sweep(1)
    torch.cuda.synchronize()
    t_prof = time.perf_counter() - t0
    prof = g.profile_end()
    log(f"[bench] profiled sweep {t_prof * 1e3:.1f} ms: {prof}")

    # ---- energy (2x2 reduced density matrices of all four plaquettes)
    E, t_energy, prof_energy = None, None, None
    if not args.no_energy:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E = g.energy(H, terms)
        torch.cuda.synchronize()
        t_energy = time.perf_counter() - t0
        log(f"[bench] energy {E:.10f} in {t_energy * 1e3:.1f} ms")
        # the same evaluation with the families timed: the density-matrix joins
        # are the largest contractions of the path
        g.profile_begin()
        g.energy(H, terms)
        prof_energy = g.profile_end()
        log(f"[bench] energy families: {prof_energy}")

    # ---- energy + gradient throughput in every mode, from one shared environment
    MODES = ("mixed", "fp64", "fp32", "bf16")
    egrad = {}
    env_shared = g.get_env()
    g.close()
    if not args.no_egrad:
        for label in MODES:
            ctx = ctm.CTM(A, cfg["pattern"], chi, precision=label)
            # one untimed evaluation first: the timed one runs with the context's
            # work buffers already allocated, as in an optimiser's later steps
            for _ in range(args.egrad_warmup):
                ctx.set_env(env_shared)
                ctx.energy_grad(args.egrad_sweeps, H, terms)
            ctx.set_env(env_shared)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.energy_grad(args.egrad_sweeps, H, terms)
            torch.cuda.synchronize()
            egrad[label] = time.perf_counter() - t0
            ctx.close()
            log(f"[bench] E&grad {label} ({args.egrad_sweeps} sweeps): {egrad[label]:.3f} s")
    fp64_sweeps_per_s = None
    if args.precision != "fp64" and args.fp64_steps > 0:
        g64 = ctm.CTM(A, cfg["pattern"], chi, precision="fp64")
        g64.set_env(env_shared)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g64.sweep(args.fp64_steps)
        torch.cuda.synchronize()
        fp64_sweeps_per_s = args.fp64_steps / (time.perf_counter() - t0)
        g64.close()
        log(f"[bench] fp64 sweeps/s {fp64_sweeps_per_s:.3f}")

    # ---- error of every mode against the stored FP64 oracle values (and FP64 mode)
    # on a weakly entangled state of this shape: the random tensors above do not
    # settle, and a gradient is only defined up to rounding where the iteration
    # is contracting (see tests/golden/make_golden.py for the cutoff)
    accuracy = None
    gold_path = os.path.join(ROOT, "tests", "golden", "ssm_d6_chi72_grad.json")
    if not args.no_egrad and args.config == "ssm_d6_chi72" and os.path.exists(gold_path):
        gold = json.load(open(gold_path))
        An = synth.near_product_tensors(len(A), 2, cfg["D"], 5, 0.3)
        accuracy = {"state": "weakly entangled (product + 0.3 noise, seed 5), same shape, pseudo-inverse cutoff "
                             f"{gold['svd_cutoff']:g}, {gold['env0_sweeps']} sweeps from a seeded random start, "
                             f"then E&grad with {args.egrad_sweeps} sweeps",
                    "oracle": "tests/golden/ssm_d6_chi72_grad.json (oracle, CPU FP64): E and 512 gradient entries",
                    "bar_fp64": 1e-8, "bar_mixed": 1e-6}
        ref = gold["n"].get(str(args.egrad_sweeps))
        res = {}
        for label in MODES:
            h = ctm.CTM(An, cfg["pattern"], chi, precision=label)
            h.set_option("svd_cutoff", gold["svd_cutoff"])
            h.set_env(torch.tensor(synth.random_env_flat(chi, cfg["D"], 2, cfg["Lx"], cfg["Ly"], gold["start_seed"])))
            h.sweep(gold["env0_sweeps"])
            E_m, g_m = h.energy_grad(args.egrad_sweeps, H, terms)
            h.close()
            res[label] = (E_m, g_m.cpu().reshape(-1))
        E64, g64v = res["fp64"]
        scale = max(1.0, g64v.abs().max().item())
        for label in MODES:
            E_m, g_m = res[label]
            row = {"dE_vs_fp64": abs(E_m - E64), "dgrad_vs_fp64_rel": (g_m - g64v).abs().max().item() / scale}
            if ref is not None:
                samp = torch.tensor(ref["grad_sample"], dtype=torch.float64)
                row["dE_vs_oracle"] = abs(E_m - ref["E"])
                row["dgrad_vs_oracle_rel"] = (g_m[gold["sample"]] - samp).abs().max().item() / max(1.0, ref["grad_max"])
            res[label] = row
        accuracy.update(res)
        log(f"[bench] accuracy: {accuracy}")

    # ---- the D = 9, chi = 100 Heisenberg 2x1 workload: sweeps and checkpointed E&grad, FP64 against mixed
    d9 = None
    if not args.no_d9 and args.config == "ssm_d6_chi72":
        c9 = synth.CONFIGS["heis_d9_chi100"]
        A9 = synth.config_tensors(c9, 0)
        t9 = synth.config_terms(c9)
        n9 = args.d9_egrad_sweeps
        d9 = {"workload": workload_name("heis_d9_chi100", c9).replace("; step = 1 CTMRG sweep", ""),
              "egrad_sweeps": n9}
        env9 = None
        g9 = {}
        for label in ("bf16", "fp64", "mixed"):
            h = ctm.CTM(A9, c9["pattern"], c9["chi"], precision=label)
            if env9 is None:
                h.sweep(1)
                env9 = h.get_env()
            h.set_env(env9)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.sweep(2)
            torch.cuda.synchronize()
            d9[f"sweeps_per_s_{label}"] = round(2 / (time.perf_counter() - t0), 4)
            if label != "bf16" and not args.no_egrad:
                if n9 <= 4:   # a warm-up evaluation, unless one evaluation is long by itself
                    h.set_env(env9)
                    h.energy_grad(n9, H, t9)
                h.set_env(env9)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                h.energy_grad(n9, H, t9)
                torch.cuda.synchronize()
                d9[f"egrad_per_s_{label}"] = round(1.0 / (time.perf_counter() - t0), 4)
            h.close()
        if not args.no_egrad:
            # the accuracy of the chain on a weakly entangled D = 9 state (product + 0.3 noise, seed 5, cutoff
            # 1e-6): from the workload's own N(0,1) tensors the first sweeps are chaotic and the derivative of
            # E after n sweeps explodes through the SVD derivative's s^(-3/2) weights (1e10 at n = 2, 1e113
            # at n = 20), so only the timing above is taken there
            An = synth.near_product_tensors(len(A9), 2, c9["D"], 5, 0.3)
            for label in ("fp64", "mixed"):
                h = ctm.CTM(An, c9["pattern"], c9["chi"], precision=label)
                h.set_option("svd_cutoff", 1e-6)
                h.sweep(1)
                g9[label] = h.energy_grad(n9, H, t9)
                h.close()
            (E64, gr64), (Emx, grmx) = g9["fp64"], g9["mixed"]
            gr64, grmx = gr64.cpu().reshape(len(An), -1), grmx.cpu().reshape(len(An), -1)
            d9["accuracy_state"] = "product + 0.3 noise (seed 5), cutoff 1e-6, 1 sweep from the sites-derived start"
            d9["dE_mixed_vs_fp64"] = abs(Emx - E64)
            d9["dgrad_mixed_vs_fp64_rel"] = (grmx - gr64).abs().max().item() / max(1.0, gr64.abs().max().item())
            d9["scale_identity_fp64"] = (torch.as_tensor(An).reshape(len(An), -1) * gr64).sum(1).abs().max().item()
        log(f"[bench] D=9: {d9}")

    # ---- nested against double-layer CTMRG (Eq. Tred; Appendix) at the D = 5, chi = 50 Shastry-Sutherland
    # shape: FP64 sweeps from the sites-derived start of the seeded tensors, each network with its own
    # environment; the double-layer cuts are (chi D^2) = 1250 wide, so both solvers are timed there
    dl = None
    if not args.no_double_layer and args.config == "ssm_d6_chi72":
        c5 = synth.CONFIGS["ssm_d5_chi50"]
        A5 = synth.config_tensors(c5, 0)
        t5 = synth.config_terms(c5)
        dl = {"workload": "ssm_d5_chi50: Shastry-Sutherland J_nn=0.7, 2x2 cell, d=2 D=5 chi=50, seeded "
                          "uniform[-1,1] tensors, FP64, sites-derived start; 2 untimed + 3 timed sweeps"}
        E5 = {}
        for layout, method in (("nested", 0), ("double", 0), ("double", 1)):
            key = f"{layout}_{'randomized' if method else 'exact'}_svd"
            h = ctm.CTM(A5, c5["pattern"], c5["chi"], precision="fp64", layout=layout)
            h.set_option("svd_method", method)
            h.sweep(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h.sweep(3)
            torch.cuda.synchronize()
            dl[f"sweeps_per_s_{key}"] = round(3 / (time.perf_counter() - t0), 4)
            if layout == "double":
                E5[method] = h.energy(H, t5)
            h.close()
        # the two double-layer runs follow the same iteration (the randomized SVD keeps the chi + 8 leading
        # triplets to its own accuracy); the nested one from this start is still in its chaotic phase
        dl["dE_double_randomized_vs_exact_after_5_sweeps"] = abs(E5[1] - E5[0])
        log(f"[bench] nested vs double layer: {dl}")

    # ---- roofline of the kernel family with the largest share of the profiled sweep
    fam = max(prof, key=lambda k: prof[k][0])
    ms, impl_flops, launches = prof[fam]
    # the method's count: 21 r^3 per r x r SVD (r = chi D), 16 Lx Ly SVDs per sweep;
    # the other families count 2 M N K per contraction (QR panels: their own count)
    r = chi * cfg["D"]
    svd_flops = 16 * cfg["Lx"] * cfg["Ly"] * 21.0 * r ** 3
    alg_flops = svd_flops if fam == "jacobi" else impl_flops
    achieved = alg_flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    fam_tf = {k: round(v[1] / (v[0] * 1e-3) / 1e12, 4) if v[0] > 0 else 0.0 for k, v in prof.items()}
    roofline = {
        "kernel": KERNEL[fam],
        "bound": BOUND[fam],
        "achieved": round(achieved, 4),
        "peak": PEAK_TFLOPS[fam],
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_TFLOPS[fam], 6),
        "traffic": traffic_per_launch(fam, args.config, args.precision),
        "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE x2 + WRITE_SIZE x1)",
        "launches_per_sweep": launches,
        # event-timed on the library's stream (includes the dispatch gap before each launch)
        "avg_launch_us": round(ms * 1e3 / max(launches, 1), 2),
        "algorithmic_flops_per_sweep": alg_flops,
        "algorithmic_flops_rule": ("21 r^3 per r x r SVD, r = chi*D = %d, %d SVDs per sweep" %
                                   (r, 16 * cfg["Lx"] * cfg["Ly"])) if fam == "jacobi" else "2 M N K per product",
        "implementation_flops_per_sweep": impl_flops,
        "kernel_ms_per_sweep": round(ms, 3),
        "sweep_ms": round(t_prof * 1e3, 2),
        "families_ms_per_sweep": {k: round(v[0], 2) for k, v in prof.items()},
        "families_tflops": fam_tf,
        # the absorption contractions of the sweep (enlarged corners, half systems,
        # environment update) on the matrix cores of the production precision
        "absorption_mfma_frac": {k: round(fam_tf[k] / PEAK_TFLOPS[k], 6) for k in ("fp64", "fp32", "bf16")
                                 if prof[k][2] > 0},
    }

    # ---- CPU oracle on a bounded sample of the same workload, all threads and one
    cpu = None
    if not args.no_cpu_baseline:
        from oracle.ctmrg import CTM as OracleCTM
        n_cpu = 3
        o = OracleCTM(A, cfg["pattern"], chi)
        t0 = time.perf_counter()
        o.run(n_cpu)
        t_cpu = time.perf_counter() - t0
        threads = torch.get_num_threads()
        torch.set_num_threads(1)
        o1 = OracleCTM(A, cfg["pattern"], chi)
        t0 = time.perf_counter()
        o1.run(n_cpu)
        t_cpu1 = time.perf_counter() - t0
        torch.set_num_threads(threads)
        cpu = {"value": round(n_cpu / t_cpu, 5), "unit": "sweeps/s", "cores": threads,
               "kind": "oracle", "sample": f"{n_cpu} sweeps of the same workload (float64, sites-derived start)",
               "value_1_thread": round(n_cpu / t_cpu1, 5)}
        log(f"[bench] oracle {n_cpu} sweeps in {t_cpu:.1f} s ({threads} threads), {t_cpu1:.1f} s (1 thread)")

    em = egrad.get("mixed")
    e64 = egrad.get("fp64")
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
        "config": {"workload": workload_name(args.config, cfg),
                   "precision": args.precision, "projectors": "fp64 QR+SVD"},
        "fp64_sweeps_per_s": None if fp64_sweeps_per_s is None else round(fp64_sweeps_per_s, 4),
        # the same workload and precision with the randomized partial-SVD projectors (svd_method = 1:
        # k = chi + 8, 2 subspace passes); tests/test_gpu_randomized.py: energies equal to the exact-SVD
        # ones to 1e-16 and corner spectra to 4e-10 on a weakly entangled state of this shape
        "sweeps_per_s_randomized_svd": None if sweeps_per_s_rand is None else round(sweeps_per_s_rand, 4),
        "energy_s": None if t_energy is None else round(t_energy, 4),
        "energy_families": None if prof_energy is None else {
            k: {"ms": round(v[0], 3), "tflops": round(v[1] / (v[0] * 1e-3) / 1e12, 3) if v[0] > 0 else 0.0,
                "frac_of_peak": round(v[1] / (v[0] * 1e-3) / 1e12 / PEAK_TFLOPS[k], 5) if v[0] > 0 else 0.0}
            for k, v in prof_energy.items() if v[2] > 0},
        # the mixed mode (FP64 sweep, FP32 energy) is the one whose gradient meets 1e-6
        "egrad_per_s": None if em is None else round(1.0 / em, 4),
        "egrad_mode": "mixed",
        "egrad_per_s_by_mode": {k: round(1.0 / v, 4) for k, v in egrad.items()},
        "egrad_sweeps": args.egrad_sweeps,
        "egrad_warmup": args.egrad_warmup,
        "egrad_speedup_mixed_vs_fp64": None if (em is None or e64 is None) else round(e64 / em, 3),
        "accuracy": accuracy,
        "d9_chi100": d9,
        "nested_vs_double_layer_d5_chi50": dl,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def lbfgs_time_to_target(args, torch, synth, ctm):
    """L-BFGS on the D=5, chi=50 Shastry-Sutherland workload (J_nn = 0.7, 2x2 cell) from a seeded
    weakly entangled start (product + 0.3 noise, seed 0); pseudo-inverse cutoff 1e-6.

    The objective is E_n(A): the energy after n = --lbfgs-sweeps sweeps from one fixed seeded
    random environment (seed 7), with its exact gradient by the checkpointed adjoint of those
    sweeps (Eq. AD).  It is a function of A alone, so the strong-Wolfe search sees values and
    slopes that agree; a warm start from the previous evaluation's environment makes the value
    depend on the history of trial points, and the nested iteration at chi = 50 moves its
    environment by ~1e-3 per sweep for hundreds of sweeps, so neither a converged environment
    nor a fixed-point gradient is within reach per evaluation.  An evaluation that fails (a
    non-finite environment at a wild trial point) returns +inf, which the search treats as a
    failed Armijo test.

    E_plain is the energy a plain FP64 run reaches in --lbfgs-iters iterations; every run's
    wall time to its first iterate with E < E_plain + 1e-5 is reported.  Runs: plain FP64 (FP64
    contractions, plain line search), mixed (FP64 sweep, FP32 energy and its adjoint) with the
    plain line search, and mixed with the surrogate (5000 -> 256 -> 256 -> 1, trained on the
    exact evaluations of the iterations before --lbfgs-sur-start, default 51, then screening 8
    trial steps per line search, every accepted step confirmed by an exact evaluation)."""
    name = "ssm_d5_chi50"
    cfg = dict(synth.CONFIGS[name])
    if args.lbfgs_D is not None or args.lbfgs_chi is not None:
        # the same model and cell at another bond dimension (a smaller one lets the run reach the
        # surrogate's start within minutes); the surrogate's input width follows d * D^4 per tensor
        cfg["D"] = args.lbfgs_D or cfg["D"]
        cfg["chi"] = args.lbfgs_chi or cfg["chi"]
        name = f"ssm_d{cfg['D']}_chi{cfg['chi']}"
    A0 = torch.tensor(synth.near_product_tensors(cfg["n_tensors"], 2, cfg["D"], 0, 0.3))
    env0 = torch.tensor(synth.random_env_flat(cfg["chi"], cfg["D"], 2, cfg["Lx"], cfg["Ly"], 7))
    H = synth.heisenberg_bond()
    terms = synth.config_terms(cfg)
    n = A0.numel()
    nsw = args.lbfgs_sweeps

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    def run(label, precision, sur_start):
        c = ctm.CTM(A0, cfg["pattern"], cfg["chi"], precision=precision)
        c.set_option("svd_cutoff", 1e-6)
        env_dev = env0.to(c.A.device)
        times, fs = [], []
        failed = [0]
        t_start = [None]
        last = [time.perf_counter()]

        if args.lbfgs_objective == "fixed_point":
            c.set_option("conv_rdm", 1)

        def fn(x):
            c.set_tensors(x.reshape(A0.shape))
            try:
                if args.lbfgs_objective == "fixed_point":
                    # warm start from the previous evaluation's environment; converged when the plaquette
                    # density matrices settle, then the derivative of the converged energy
                    c.sweep(args.lbfgs_max_sweeps, tol=1e-10)
                    E, g, _, _, _ = c.energy_grad_fp(H, terms, tol=1e-8, max_iter=200)
                else:
                    c.set_env(env_dev)
                    E, g = c.energy_grad(nsw, H, terms)
            except ctm.CTMError as e:
                failed[0] += 1
                log(f"[lbfgs] {label}: evaluation {len(fs) + 1} failed ({e}); returned +inf")
                E, g = float("inf"), torch.zeros_like(x)
            now = time.perf_counter()
            times.append(now - t_start[0])
            fs.append(E)
            if now - last[0] > 30:
                last[0] = now
                log(f"[lbfgs] {label}: {len(fs)} evaluations, {times[-1]:.0f} s, E {E:.10f}")
            return E, g.reshape(-1)

        obj = ctm.python_objective(fn, n)
        sur = ctm.Surrogate(n, 256, seed=0) if sur_start > 0 else None
        params = ctm.lbfgs_params(max_iter=args.lbfgs_iters, gtol=1e-7, sur_start=sur_start, n_trials=8,
                                  refit_every=10, refit_steps=200, n_blocks=cfg["n_tensors"])
        torch.cuda.synchronize()
        t_start[0] = time.perf_counter()
        x, recs, conv = ctm.lbfgs(A0.reshape(-1), obj, sur=sur, params=params)
        total = time.perf_counter() - t_start[0]
        c.close()
        if sur is not None:
            sur.close()
        # iteration records (iter, evals, screened, f, gmax, step): an iterate's time is that of its last evaluation
        its = [(r[3], times[r[1] - 1], r[1], r[2]) for r in recs]
        res = {"iterations": len(recs), "evaluations": len(fs), "failed_evaluations": failed[0],
               "seconds": round(total, 2), "seconds_per_evaluation": round(total / max(1, len(fs)), 3),
               "final_E": recs[-1][3], "screened_steps": sum(r[2] for r in recs), "converged": conv}
        log(f"[lbfgs] {label}: {json.dumps(res)}")
        res["its"] = its
        return res

    kinds = {"plain_fp64": ("plain fp64", "fp64", 0), "mixed": ("mixed", "mixed", 0),
             "mixed_surrogate": ("mixed+surrogate", "mixed", args.lbfgs_sur_start)}
    which = list(kinds) if args.lbfgs_runs == "all" else args.lbfgs_runs.split(",")
    if "plain_fp64" not in which and args.lbfgs_e_plain is None:
        sys.exit("--lbfgs-e-plain is needed when the plain FP64 run is not part of this invocation")
    out_runs = {k: run(*kinds[k]) for k in which}
    E_plain = out_runs["plain_fp64"]["final_E"] if "plain_fp64" in out_runs else args.lbfgs_e_plain
    target = E_plain + 1e-5
    for r in out_runs.values():
        hit = next((t for (f, t, e, scr) in r["its"] if f < target), None)
        r["seconds_to_target"] = None if hit is None else round(hit, 2)
        r["evaluations_to_target"] = next((e for (f, t, e, scr) in r["its"] if f < target), None)
        del r["its"]
    tp = out_runs["plain_fp64"]["seconds_to_target"] if "plain_fp64" in out_runs else args.lbfgs_plain_seconds
    ts = out_runs["mixed_surrogate"]["seconds_to_target"] if "mixed_surrogate" in out_runs else None
    out = {"metric": "wall time to |E - E_plain| < 1e-5 per site, L-BFGS (mixed + surrogate vs plain FP64)",
           "value": ts, "unit": "s", "higher_is_better": False, "n_gpus": 1,
           "config": {"workload": f"{name}: Shastry-Sutherland J_dimer=1 J_nn=0.7, 2x2 cell of 4 tensors, d=2 "
                                  f"D={cfg['D']} chi={cfg['chi']}, start: product + 0.3 noise (seed 0), normalised; "
                                  f"pseudo-inverse cutoff "
                                  f"1e-6; L-BFGS {args.lbfgs_iters} iterations, m = 10, strong Wolfe, surrogate from "
                                  f"iteration {args.lbfgs_sur_start}; an evaluation: "
                                  + (f"E and dE/dA after {nsw} differentiated sweeps from a fixed seeded random "
                                     "environment" if args.lbfgs_objective == "chain" else
                                     "warm-started sweeps until the plaquette density matrices change by < 1e-10 "
                                     f"(at most {args.lbfgs_max_sweeps}), energy and fixed-point gradient")},
           "E_plain": E_plain, "runs": out_runs,
           "speedup_vs_plain_fp64": None if (tp is None or ts is None) else round(tp / ts, 3),
           "data": "synthetic"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
