"""Benchmark: particle-steps/s of the Riemann-WCSPH dam break on one MI355X.

A step is one advection step of the whole hot path: time-step reductions,
density re-initialisation, the acoustic sub-steps (pressure and density
relaxation, position Verlet) and the configuration update (cell binning and
neighbour lists); the timed region ends with the FP64 diagnostics reduction.
Inputs are seeded synthetic dam breaks (no dataset), resident in device
memory before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload large|medium|small|ensemble|sloshing|surrogate]

Default workload: the 3D dam break (2.0 M fluid and 0.596 M wall particles,
dp = 0.01, 2 000 advection steps). Its timed window starts mid-run (after
1 000 untimed advection steps and the warm-up), so the window holds the
flow after release rather than the resting column; the whole 2 000-step run
from t = 0 is timed as well and reported in config.whole_run.

Prints one JSON line. value = fluid particles x acoustic sub-steps / wall
time, in millions per second (summed over the cases for the ensemble of 64
uneven dam breaks, which all advance in the same launches). The sloshing
workload is a 2D tank of the same particle count under prescribed sway and
roll (moving walls re-posed and re-sorted at every configuration update).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (M) WCSPH dam-break; surrogate speedup at ≤1% front error"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_TFLOPS = 157.3       # MI355X FP32 vector peak
FP64_VALU_TFLOPS = 78.6
BF16_MFMA_TFLOPS = 2500.0      # MI355X dense bf16 matrix peak


def algorithmic_bytes(dim, precision, n_fluid):
    """Compulsory bytes per launch of the two sub-step kernels, state only:
    each fluid particle's own fields read and written once (r = 4 bytes per
    FP32 field, 8 per FP64 field; positions always FP64).
    Pressure relaxation: reads rho, drho/dt, v and the frozen offsets, writes
    rho^{n+1/2} and v^{n+1}: (3 + 3d) r.
    Density relaxation: reads v^{n+1}, v^n, rho, the offsets and x, writes
    rho, drho/dt and x: (3d + 3) r + 16 d.
    (2D FP32: 36 and 68 bytes per particle; 3D FP32: 48 and 96.) The stored
    neighbour configuration is not compulsory state: it is reported apart
    (configuration_bytes)."""
    r = 4 if precision == 1 else 8
    k1 = n_fluid * (3 + 3 * dim) * r
    k2 = n_fluid * ((3 * dim + 3) * r + 16 * dim)
    return k1, k2


def configuration_bytes(inner_pairs, contact_pairs, n_fluid, bytes_per_pair=4.0, bytes_per_particle=8.0):
    """Bytes of the stored neighbour configuration one pair kernel reads per
    launch (entries per directed pair plus per-particle counts or masks)."""
    return int(bytes_per_pair * (inner_pairs + contact_pairs) + bytes_per_particle * n_fluid)


FLOPS_PER_PAIR = 55  # geometry ~25 (incl. rsqrt) + Riemann and accumulation ~30, per directed pair


def roofline(nbytes, flops, ms, precision):
    """Roofline of one launch: time bound max(bytes / HBM peak, flops / VALU
    peak); frac = that bound over the measured launch time, reported against
    the bound that is larger."""
    valu = FP32_VALU_TFLOPS if precision == 1 else FP64_VALU_TFLOPS
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_alu = flops / (valu * 1e12)
    t = ms * 1e-3
    if t_hbm >= t_alu:
        out = {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        out = {"bound": "alu", "achieved": flops / t / 1e12, "peak": valu, "unit": "TFLOP/s"}
    out["frac"] = max(t_hbm, t_alu) / t
    out["hbm_frac"] = t_hbm / t
    out["alu_frac"] = t_alu / t
    return out


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2010_12375_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when there is
    no summary or the kernels have changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}_hot_kernels.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if "```json" not in text:
        return None
    blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    if blob.get("kernel") != kernel or blob.get("source_hash") != kernel_source_hash():
        return None
    return int(blob["traffic_bytes_per_launch"])


def cpu_baseline(case, budget_s=15.0):
    """The FP64 oracle as it stands, on the host cores, on the first
    advection steps of the same workload (time-boxed)."""
    import oracle as O
    o = O.Oracle(case)
    m = getattr(case, "wall_motion", None)
    if m is not None:
        o.set_wall_motion(amp=m.amp, omega=m.omega, roll=m.roll, pivot=m.pivot)
    o.build_config()
    t0 = time.perf_counter()
    nsub = 0
    steps = 0
    while time.perf_counter() - t0 < budget_s:
        nsub += o.advance(1e9)
        steps += 1
    wall = time.perf_counter() - t0
    return {"value": case.n_fluid * nsub / wall / 1e6, "unit": "M particle-steps/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"first {steps} advection steps ({nsub} acoustic sub-steps) of {case.name} from t=0, "
                      f"{wall:.1f} s, FP64 oracle, OpenMP"}


def cpu_baseline_ensemble(cases, budget_s=15.0):
    """The FP64 oracle on the ensemble's cases from t=0: every case's
    configuration is built, then the cases take advection steps in turn,
    one step each per round, until the time budget is spent."""
    import oracle as O
    t0 = time.perf_counter()
    orcs = []
    for c in cases:
        o = O.Oracle(c)
        o.build_config()
        orcs.append(o)
    work = 0
    nsub = 0
    rounds = 0
    done = 0
    while time.perf_counter() - t0 < budget_s:
        for c, o in zip(cases, orcs):
            n = o.advance(1e9)
            work += c.n_fluid * n
            nsub += n
            done += 1
            if time.perf_counter() - t0 >= budget_s:
                break
        rounds += 1
    wall = time.perf_counter() - t0
    for o in orcs:
        o.close()
    return {"value": work / wall / 1e6, "unit": "M particle-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{done} advection steps ({nsub} acoustic sub-steps) over the {len(cases)} ensemble cases "
                      f"from t=0, round robin ({rounds} rounds), configuration builds included, {wall:.1f} s, "
                      f"FP64 oracle, OpenMP"}


def surrogate_bench(args):
    """Surrogate line: train on plain-scheme trajectories, then time the plain
    scheme and the surrogate (with its fallback) on held-out cases over the
    same number of windows, for a sweep of forced plain windows; report the
    fastest setting whose surge front stays within 1 % of the plain run."""
    import torch
    from paper_2010_12375_amd import sphx
    from paper_2010_12375_amd import surrogate as S
    from paper_2010_12375_amd import workloads as wl
    stream = torch.cuda.Stream()
    sync = torch.cuda.synchronize
    log = lambda m: print(m, file=sys.stderr, flush=True)
    tr = S.make_cases(range(args.train_cases))
    te = S.make_cases(range(S.TEST_SEED0, S.TEST_SEED0 + args.test_cases))
    t0 = time.perf_counter()
    samples = []
    for b in range(0, len(tr), 64):
        samples += S.generate(tr[b:b + 64], t_end=1.5, every=16, stream=stream)
    gen_s = time.perf_counter() - t0
    log(f"surrogate: {sum(len(x) for x in samples)} samples from {len(tr)} trajectories in {gen_s:.1f} s")
    t0 = time.perf_counter()
    params, losses = S.train(tr, samples, args.train_iters, batch=16, lr=1e-3, lr_final=1e-4, init_scale=0.3,
                             stream=stream, log=log)
    train_s = time.perf_counter() - t0
    sweep = []
    for pe in (0, 8, 4, 2, 1):
        r = S.evaluate(params, te, windows=args.windows, max_drho=0.01, plain_every=pe, stream=stream, sync=sync)
        r["plain_every"] = pe
        log("surrogate: " + json.dumps(r))
        sweep.append(r)
    ok = [r for r in sweep if r["front_err"] <= 0.01]
    best = max(ok, key=lambda r: r["speedup"]) if ok else None
    # kernel profile of the surrogate on the held-out batch
    sim = sphx.Simulation.from_cases(te, wl.FP32, stream=stream)
    sim.gnn_set_params(params)
    sim.build_neighbors()
    gp = sim.gnn_profile(20)
    sim.close()
    E, N = gp["edges"], gp["nodes"]
    # the fused layer: reads the edge features (8 FP32), the edge's two
    # endpoints, P and Q once per node, writes A; the matrix cores do the edge
    # encoder (K = 32, 8 of it features) and the edge product (K = 64)
    fused_bytes = E * (8 * 4 + 8) + N * (4 + 3 * 64 * 4)
    fused_flops = E * (2 * 32 * 64 + 2 * 64 * 64)
    ms = gp["fused_layer"]
    t_hbm = fused_bytes / (HBM_PEAK_GBS * 1e9)
    t_mfma = fused_flops / (BF16_MFMA_TFLOPS * 1e12)
    n_fluid = sum(c.n_fluid for c in te)
    ref = best or sweep[0]
    rate_plain = n_fluid * (ref["nsub_plain"] / len(te)) / ref["wall_plain"] / 1e6
    out = {
        "metric": METRIC,
        "value": round(rate_plain * (best["speedup"] if best else 0.0), 3),
        "unit": "M particle-steps/s",
        "n_gpus": 1,
        "steps": 2 * args.windows,
        "warmup": 0,
        "ms_per_step": round(ref["wall_surrogate"] / (2 * args.windows) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": f"surrogate_dambreak2d_dp0.0125 ({len(te)} held-out cases, {n_fluid} fluid particles)",
            "value_is": "plain-equivalent particle-steps/s of the surrogate run at the fastest setting within 1 % "
                        "front error (0 if none)",
            "train": {"trajectories": len(tr), "samples": int(sum(len(x) for x in samples)),
                      "iters": args.train_iters, "batch": 16, "loss_first": losses[0],
                      "loss_last100": float(np.mean(losses[-100:])), "generate_s": round(gen_s, 1),
                      "train_s": round(train_s, 1)},
            "gnn_kernel_ms": {k: round(v, 5) for k, v in gp.items() if k not in ("nodes", "edges")},
            "forward_speedup_fused": round(gp["forward_unfused"] / gp["forward"], 3),
            "graph": {"nodes": N, "edges": E},
        },
        "surrogate": {
            "speedup": round(best["speedup"], 4) if best else None,
            "front_err": best["front_err"] if best else None,
            "setting": {"max_drho": 0.01, "plain_every": best["plain_every"]} if best else None,
            "plain_rate": round(rate_plain, 3),
            "sweep": [{k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()} for r in sweep],
        },
        "roofline": {
            "kernel": "fused_message_layer",
            "bound": "hbm" if t_hbm >= t_mfma else "mfma",
            "achieved": round(fused_bytes / (ms * 1e-3) / 1e9, 2) if t_hbm >= t_mfma
            else round(fused_flops / (ms * 1e-3) / 1e12, 3),
            "peak": HBM_PEAK_GBS if t_hbm >= t_mfma else BF16_MFMA_TFLOPS,
            "unit": "GB/s" if t_hbm >= t_mfma else "TFLOP/s",
            "frac": round(max(t_hbm, t_mfma) / (ms * 1e-3), 4),
            "traffic": None,
            "alg_bytes_per_launch": int(fused_bytes),
            "alg_flops_per_launch": int(fused_flops),
            "ms_per_launch": round(ms, 5),
            "hbm_frac": round(t_hbm / (ms * 1e-3), 4),
            "mfma_frac": round(t_mfma / (ms * 1e-3), 4),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_ensemble(te, args.cpu_budget)
    print(json.dumps(out), flush=True)


LARGE_START_STEP = 1000  # mid-run of the 2 000-step 3D dam break


def kernel_breakdown(prof, nsub_per_step):
    """Per-step time of each hot kernel from its HIP-event launch time: the
    two relaxations run once per acoustic sub-step, the neighbour build (with
    the fused density re-initialisation) once per advection step."""
    per_step = {"pressure_relaxation": prof["pressure"] * nsub_per_step,
                "density_relaxation": prof["density"] * nsub_per_step,
                "neighbor_build": prof["neighbors"]}
    total = sum(per_step.values())
    return {k: {"ms_per_launch": round({"pressure_relaxation": prof["pressure"],
                                        "density_relaxation": prof["density"],
                                        "neighbor_build": prof["neighbors"]}[k], 5),
                "launches_per_step": round(nsub_per_step, 3) if k != "neighbor_build" else 1,
                "ms_per_step": round(v, 5), "share": round(v / total, 4)}
            for k, v in per_step.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large", "ensemble", "sloshing", "surrogate"])
    ap.add_argument("--start-step", type=int, default=-1,
                    help="advection steps taken (untimed) before the warm-up; -1: 1000 for the 3D dam break "
                         "(mid-run of its 2 000 steps), 0 otherwise")
    ap.add_argument("--whole-run", type=int, default=-1,
                    help="also time the first N advection steps from t=0 as one figure (-1: 2000 for the 3D dam "
                         "break, 0 otherwise); the headline window lies inside this run")
    ap.add_argument("--train-cases", type=int, default=256, help="surrogate: training trajectories")
    ap.add_argument("--test-cases", type=int, default=32, help="surrogate: held-out trajectories")
    ap.add_argument("--train-iters", type=int, default=2000, help="surrogate: Adam steps (16 snapshots each)")
    ap.add_argument("--windows", type=int, default=250, help="surrogate: evaluation windows (2 advection steps)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the pair-kernel lanes per particle first (always for the ensemble)")
    ap.add_argument("--lanes", type=int, default=0, help="pair-kernel lanes per particle (0: the library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads for cpu_baseline (0: all)")
    ap.add_argument("--profile-reps", type=int, default=50)
    ap.add_argument("--no-torch", action="store_true", help="let the library create its own stream")
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="MiB: only run a plain device-to-device copy of this size five times (the "
                         "reference kernel for scaling the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch
        n = int(args.copy_calibration * 2 ** 20) // 4
        a = torch.ones(n, device="cuda", dtype=torch.float32)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path (slabs along x "
              "with halo exchanges over RCCL) is designed, not built.", file=sys.stderr)
        sys.exit(2)

    from paper_2010_12375_amd import sphx
    from paper_2010_12375_amd import workloads as wl

    if args.workload == "surrogate":
        return surrogate_bench(args)

    log = lambda m: print(m, file=sys.stderr, flush=True)
    cases = None
    if args.workload == "small":
        case = wl.config_small(0)
        case.precision = wl.FP32
    elif args.workload == "medium":
        case = wl.config_medium(0)
    elif args.workload == "large":
        case = wl.config_large(0)
    elif args.workload == "sloshing":
        case = wl.sloshing_2d(0.00625, roll=0.05, precision=wl.FP32, name="sloshing2d_51k")
    else:
        cases = wl.ensemble_cases(64, seed=0)
        case = cases[0]
    precision = case.precision
    large = args.workload == "large"
    start_step = args.start_step if args.start_step >= 0 else (LARGE_START_STEP if large else 0)
    whole = args.whole_run if args.whole_run >= 0 else (case.n_adv_steps if large else 0)

    stream = None
    torch = None
    try:
        if args.no_torch:
            raise ImportError
        import torch  # noqa: F401
        if torch.cuda.is_available():
            stream = torch.cuda.Stream()
        else:
            torch = None
    except Exception:
        torch = None

    def sync():
        if torch is not None:
            torch.cuda.synchronize()

    if cases is None:
        sim = sphx.Simulation(sphx.params_from_case(case, precision), stream=stream)
        sim.set_fluid(case.fluid_pos)
        if case.n_wall:
            sim.set_walls(case.wall_pos, case.wall_normal)
            sim.set_case_motion(case)
        n_fluid, n_wall, name = case.n_fluid, case.n_wall, case.name
    else:
        sim = sphx.Simulation.from_cases(cases, precision, stream=stream)
        n_fluid = sum(c.n_fluid for c in cases)
        n_wall = sum(c.n_wall for c in cases)
        name = f"ensemble64_dambreak2d ({n_fluid} fluid particles in 64 cases)"
    sim.build_neighbors()
    lanes = None
    if args.lanes:
        sim.set_lanes(args.lanes)
        lanes = args.lanes
    if args.autotune or (cases is not None and not args.lanes):
        lanes = sim.autotune(10)
    nf = [c.n_fluid for c in cases] if cases is not None else [case.n_fluid]

    def work_between(a, b):
        return sum(n * (y["n_substeps"] - x["n_substeps"]) for n, x, y in zip(nf, a, b))

    # set-up: the run up to the start of the window (untimed for the headline,
    # but part of the whole-run figure)
    sync()
    d_start = sim.diagnostics_all()
    t_run = time.perf_counter()
    if start_step:
        log(f"bench: {name}: advancing {start_step} advection steps to the start of the timed window")
        sim.advance(start_step)
    sim.advance(args.warmup)
    sync()
    d0 = sim.diagnostics_all()
    t0 = time.perf_counter()
    sim.advance(args.steps)
    d1 = sim.diagnostics_all()
    sync()
    t1 = time.perf_counter()
    wall = t1 - t0
    whole_run = None
    if whole and d1[0]["n_steps"] < whole:
        sim.advance(whole - d1[0]["n_steps"])
        dw = sim.diagnostics_all()
        sync()
        t_end = time.perf_counter()
        # the host-side reads of the diagnostics between the windows are inside this figure
        wr_wall = t_end - t_run
        whole_run = {"advection_steps": dw[0]["n_steps"] - d_start[0]["n_steps"],
                     "acoustic_substeps": int(dw[0]["n_substeps"] - d_start[0]["n_substeps"]),
                     "t_end": dw[0]["t"], "wall_s": round(wr_wall, 4),
                     "value": round(work_between(d_start, dw) / wr_wall / 1e6, 3)}
        log(f"bench: whole run {whole_run}")

    steps_done = d1[0]["n_steps"] - d0[0]["n_steps"]
    steps_all = sum(b["n_steps"] - a["n_steps"] for a, b in zip(d0, d1))
    nsub = sum(b["n_substeps"] - a["n_substeps"] for a, b in zip(d0, d1))
    work = work_between(d0, d1)
    cnt = sim.counts()
    pairs = cnt["inner_pairs"] + cnt["contact_pairs"]
    value = work / wall / 1e6
    # directed pair evaluations: two relaxations per sub-step, each case its own sub-steps
    pair_evals = 0.0
    for k, (a, b) in enumerate(zip(d0, d1)):
        ck = sim.counts(case=k) if cases is not None else cnt
        pair_evals += 2.0 * (ck["inner_pairs"] + ck["contact_pairs"]) * (b["n_substeps"] - a["n_substeps"])
    pair_evals /= wall

    prof = sim.profile(args.profile_reps)
    nsub_per_step = nsub / max(steps_all, 1)
    breakdown = kernel_breakdown(prof, nsub_per_step)
    k1_bytes, k2_bytes = algorithmic_bytes(case.dim, precision, n_fluid)
    flops = FLOPS_PER_PAIR * pairs
    sub = {"pressure_relaxation": (prof["pressure"], k1_bytes), "density_relaxation": (prof["density"], k2_bytes)}
    kname = max(sub, key=lambda k: sub[k][0])
    ms, nbytes = sub[kname]
    rl = roofline(nbytes, flops, ms, precision)
    cfg_bytes = configuration_bytes(cnt["inner_pairs"], cnt["contact_pairs"], n_fluid)
    step_dom = max(breakdown, key=lambda k: breakdown[k]["ms_per_step"])
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "M particle-steps/s",
        "n_gpus": 1,
        "steps": steps_done,
        "warmup": args.warmup,
        "ms_per_step": round(wall / max(steps_done, 1) * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precision == 1 else "f64",
        "data": "synthetic",
        "config": {
            "workload": name,
            "dim": case.dim,
            "n_fluid": n_fluid,
            "n_wall": n_wall,
            "dp": case.dp if cases is None else sorted({c.dp for c in cases}),
            "precision": "FP32 fields and pair arithmetic; FP64 positions, clock, diagnostics"
            if precision == 1 else "FP64",
            "window": f"advection steps {start_step + args.warmup} to {start_step + args.warmup + steps_done} "
                      f"(after {start_step} untimed set-up and {args.warmup} warm-up steps)",
            "acoustic_substeps": int(nsub),
            "substeps_per_step": round(nsub_per_step, 3),
            "pair_evals_per_s": round(pair_evals, 1),
            "t_start": d0[0]["t"],
            "t_end": d1[0]["t"],
            "kernel_ms": {k: round(v, 5) for k, v in prof.items()},
            "kernels_per_step": breakdown,
            "step_dominant_kernel": step_dom,
            "pair_lanes": lanes,
            "whole_run": whole_run,
        },
        "roofline": {
            "kernel": kname,
            "bound": rl["bound"],
            "achieved": round(rl["achieved"], 3),
            "peak": rl["peak"],
            "unit": rl["unit"],
            "frac": round(rl["frac"], 4),
            "traffic": measured_traffic(case.name if cases is None else "ensemble64", kname),
            "alg_bytes_per_launch": int(nbytes),
            "alg_flops_per_launch": int(flops),
            "ms_per_launch": round(ms, 5),
            "hbm_frac": round(rl["hbm_frac"], 4),
            "alu_frac": round(rl["alu_frac"], 4),
            "config_bytes_per_launch": cfg_bytes,
            "hbm_frac_with_config": round((nbytes + cfg_bytes) / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
            "step_dominant_kernel": step_dom,
        },
    }
    if not args.no_cpu_baseline:
        if args.cpu_threads > 0:
            import oracle as O
            O.set_num_threads(args.cpu_threads)
        out["cpu_baseline"] = (cpu_baseline(case, args.cpu_budget) if cases is None
                               else cpu_baseline_ensemble(cases, args.cpu_budget))
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
