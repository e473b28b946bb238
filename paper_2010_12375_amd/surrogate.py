"""Training data, training and evaluation of the message-passing surrogate,
driven through the library's C ABI (every step runs in the HIP kernels; this
module only moves arrays and keeps time).

Workload: 2D dam breaks at dp = 0.0125 (12 800 fluid particles at the
standard column), column aspect a = H/L uniform in [0.25, 1] at fixed area
L H = 2, seeded jitter; training trajectories are seeds 0 .. n-1, held-out
test trajectories seeds 10 000 and up. A sample is the state after a
configuration update and, as the target, the mean acceleration and density
rate of the plain scheme over the next two advection steps (about ten
acoustic sub-steps), scaled as the network's output.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import gnn_inputs as gi
from . import sphx
from . import workloads as wl

DP = 0.0125
TEST_SEED0 = 10_000


def make_cases(seeds, precision=wl.FP32):
    out = []
    for s in seeds:
        rng = np.random.Generator(np.random.PCG64(50_000 + int(s)))
        a = float(rng.uniform(0.25, 1.0))
        out.append(wl.dam_break_2d(DP, seed=int(s), L=math.sqrt(2.0 / a), H=math.sqrt(2.0 * a),
                                   precision=precision, name=f"sur{s}_a{a:.3f}"))
    return out


def targets(case, v1, v2, r1, r2, dt):
    """Mean rates over dt in the network's output scaling."""
    g = float(np.linalg.norm(case.gravity))
    a = (v2 - v1) / dt / g
    dr = 1e3 * (r2 - r1) / dt * case.h / (case.rho0 * case.u_ref)
    return np.column_stack([a, dr]).astype(np.float32)


def generate(cases, t_end, every, stream=None):
    """Plain-scheme trajectories of all cases in one batch from t = 0; every
    `every` advection steps one sample per case. Returns, per case, a list of
    (pos, vel, rho, target) float32 arrays."""
    sim = sphx.Simulation.from_cases(cases, wl.FP32, stream=stream)
    samples = [[] for _ in cases]
    F = sphx
    while True:
        d1 = sim.diagnostics_all()
        if min(x["t"] for x in d1) >= t_end:
            break
        s1 = [(sim.get_field(F.SPHX_FIELD_POS, k), sim.get_field(F.SPHX_FIELD_VEL, k),
               sim.get_field(F.SPHX_FIELD_RHO, k)) for k in range(len(cases))]
        sim.advance(2)
        d2 = sim.diagnostics_all()
        for k, c in enumerate(cases):
            v2 = sim.get_field(F.SPHX_FIELD_VEL, k)
            r2 = sim.get_field(F.SPHX_FIELD_RHO, k)
            x1, v1, r1 = s1[k]
            T = targets(c, v1, v2, r1, r2, d2[k]["t"] - d1[k]["t"])
            samples[k].append((x1.astype(np.float32), v1.astype(np.float32), r1.astype(np.float32), T))
        if every > 2:
            sim.advance(every - 2)
    sim.close()
    return samples


def train(cases, samples, iters, batch=16, lr=1e-3, seed=0, init_scale=0.3, params=None, stream=None,
          log=None, lr_final=None):
    """Adam on minibatches of `batch` samples drawn uniformly over all
    (trajectory, snapshot) pairs; one batch context whose cases take each
    sample's parameters (same cell grid). Returns (params, losses)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pool = [(k, s) for k in range(len(cases)) for s in range(len(samples[k]))]
    first = [pool[i] for i in rng.integers(0, len(pool), batch)]
    sim = sphx.Simulation([sphx.params_from_case(cases[k], wl.FP32) for k, _ in first], stream=stream)
    wall = cases[0]
    for b in range(batch):
        sim.set_walls(wall.wall_pos, wall.wall_normal, case=b)
    sim.gnn_set_params(gi.init_params(seed, init_scale) if params is None else params)
    losses = []
    t0 = time.perf_counter()
    for it in range(iters):
        picks = [pool[i] for i in rng.integers(0, len(pool), batch)]
        for b, (k, s) in enumerate(picks):
            sim.set_params(sphx.params_from_case(cases[k], wl.FP32), case=b)
            x, v, r, _ = samples[k][s]
            sim.set_fluid(x, v, r, case=b)
        sim.build_neighbors()
        for b, (k, s) in enumerate(picks):
            sim.gnn_set_target(samples[k][s][3], case=b)
        step_lr = lr if lr_final is None else lr * (lr_final / lr) ** (it / max(iters - 1, 1))
        losses.append(sim.gnn_train_step(step_lr))
        if log and (it % max(iters // 10, 1) == 0 or it == iters - 1):
            log(f"train iter {it} loss {losses[-1]:.4e} lr {step_lr:.2e} ({time.perf_counter() - t0:.1f} s)")
    p = sim.gnn_get_params()
    sim.close()
    return p, losses


def _fronts(sim):
    return np.array([d["front"] for d in sim.diagnostics_all()]), np.array([d["t"] for d in sim.diagnostics_all()])


def evaluate(params, cases, windows, max_drho=0.01, plain_every=0, chunks=5, stream=None, sync=None):
    """Plain scheme against the surrogate (with its fallback) on the same
    cases from t = 0, each over `windows` windows of two advection steps.
    Returns wall times, simulated times, the largest relative surge-front
    difference (the plain front interpolated at the surrogate's times, at
    the end of every chunk of windows) and fallback counts."""
    sync = sync or (lambda: None)
    # plain reference with observations after every window (not timed)
    ref = sphx.Simulation.from_cases(cases, wl.FP32, stream=stream)
    ref.build_neighbors()
    hist_t, hist_f = [], []
    f, t = _fronts(ref)
    hist_t.append(t)
    hist_f.append(f)
    for _ in range(windows):
        ref.advance(2)
        f, t = _fronts(ref)
        hist_t.append(t)
        hist_f.append(f)
    ref.close()
    hist_t, hist_f = np.array(hist_t), np.array(hist_f)
    # plain, timed
    pl = sphx.Simulation.from_cases(cases, wl.FP32, stream=stream)
    pl.build_neighbors()
    sync()
    t0 = time.perf_counter()
    pl.advance(2 * windows)
    sync()
    wall_plain = time.perf_counter() - t0
    t_plain = np.array([d["t"] for d in pl.diagnostics_all()])
    nsub_plain = np.array([d["n_substeps"] for d in pl.diagnostics_all()])
    pl.close()
    # surrogate, timed in chunks (front checks between chunks)
    su = sphx.Simulation.from_cases(cases, wl.FP32, stream=stream)
    su.gnn_set_params(params)
    su.build_neighbors()
    per = [windows // chunks + (1 if i < windows % chunks else 0) for i in range(chunks)]
    wall_sur = 0.0
    worst = 0.0
    nfb = nsu = 0
    failed = None
    for w in per:
        if w == 0:
            continue
        sync()
        t0 = time.perf_counter()
        try:
            a, b = su.surrogate_advance(w, max_drho, plain_every)
        except sphx.SphxError as e:   # a case the surrogate drove into an invalid state
            failed = str(e)
            worst = float("inf")
            break
        sync()
        wall_sur += time.perf_counter() - t0
        nfb += a
        nsu += b
        fs, ts = _fronts(su)
        for k in range(len(cases)):
            fr = np.interp(ts[k], hist_t[:, k], hist_f[:, k])
            worst = max(worst, abs(fs[k] - fr) / fr)
    t_sur = np.array([d["t"] for d in su.diagnostics_all()])
    su.close()
    return dict(wall_plain=wall_plain, wall_surrogate=wall_sur, t_plain=float(t_plain.mean()),
                t_surrogate=float(t_sur.mean()), front_err=float(worst), n_fallback=int(nfb), n_surrogate=int(nsu),
                nsub_plain=int(nsub_plain.sum()), failed=failed,
                speedup=float((t_sur.mean() / wall_sur) / (t_plain.mean() / wall_plain)))
