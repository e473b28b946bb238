"""Message-passing surrogate on the GPU against its FP64 reference
(oracle/gnn_oracle.py), through the C ABI. Both sides take the same seeded
parameters, the same particles and the same targets; the reference rounds
every matrix-product operand to bfloat16 where the kernels do.

Tolerances. Besides FP32 accumulation (~1e-6 relative), the two sides
compute features and activations in different precisions before rounding
them to bf16; where a value lies within that difference of a rounding
boundary the two roundings differ by one bf16 ulp (2^-8 relative) in that
element. Such flips are rare (~1e-5 of the elements); one flip moves the
output of the particle it occurs in by about 2^-8 of that particle's own
output (which reaches several times the root-mean-square output) and, less,
the outputs of its three-hop neighbourhood (three message-passing layers).
So per particle the error must stay within 8 x 2^-8 (3 %) of the rms output,
at 90 % of the particles within 2^-8, and at the median within 1e-4 (any
systematic mistake breaks the last two); gradients within 5e-3 of each
tensor's norm (the same flips, summed over the 800 particles of the case;
measured at most 2.0e-3).

Inference runs the fused layer kernel (edge encoder, edge product,
messages and their sums in one kernel); training runs the layer through
device memory (it keeps the pre-activations for the backward pass). Both
are held to the same reference bars.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from oracle import gnn_oracle as G
from paper_2010_12375_amd import gnn_inputs as gi
from paper_2010_12375_amd import sphx
from paper_2010_12375_amd import workloads as wl
from parity import developed_state

pytestmark = pytest.mark.gpu

FP64, FP32 = sphx.SPHX_FP64, sphx.SPHX_FP32


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def prm_of(case):
    return dict(h=case.h, rho0=case.rho0, u_ref=case.u_ref, g=1.0, c0=case.c0, gvec=case.gravity)


def oracle_forward(case, state, params):
    o = O.Oracle(case)
    o.set_fluid(case.fluid_pos, *state)
    o.build_config()
    g = G.graph_from_oracle(o)
    o.close()
    vel, rho, _ = state
    F, E = G.features(g, case.fluid_pos, vel, rho, case.wall_pos, prm_of(case))
    Y, cache = G.forward(params.astype(np.float64), g, F, E, emu=True)
    return g, Y, cache


def gpu_sim(cases, states, precision, params):
    s = sphx.Simulation.from_cases(cases, precision) if len(cases) > 1 else sphx.Simulation.from_case(cases[0], precision)
    for k, (c, st) in enumerate(zip(cases, states)):
        s.set_fluid(c.fluid_pos, *st, case=k)
    s.gnn_set_params(params)
    s.build_neighbors()
    return s


def assert_outputs_match(Yg, Yo, what):
    rms = float(np.sqrt((Yo ** 2).mean()))
    e = np.abs(Yg - Yo).max(axis=1) / rms
    mx, p99, p90, med = e.max(), np.quantile(e, 0.99), np.quantile(e, 0.9), np.median(e)
    say(f"{what}: err / rms max {mx:.3e}, p99 {p99:.3e}, p90 {p90:.3e}, median {med:.3e}")
    assert mx <= 8 * 2.0 ** -8 and p90 <= 2.0 ** -8 and med <= 1e-4


@pytest.mark.parametrize("precision", [FP32, FP64])
def test_forward_matches_reference(precision):
    case = wl.config_small(0)
    st = developed_state(case, seed=0)
    params = gi.init_params(11)
    _, Yo, _ = oracle_forward(case, st, params)
    s = gpu_sim([case], [st], precision, params)
    s.gnn_forward()
    assert_outputs_match(s.gnn_output(), Yo, "forward")
    s.close()


def test_forward_full_size_and_batch_invariance():
    """The surrogate's own workload size (dp = 0.0125, 12 800 particles):
    reference parity, and a batch of three cases gives each case exactly what
    it gives alone."""
    cases = [wl.dam_break_2d(0.0125, seed=k, L=math.sqrt(2 / a), H=math.sqrt(2 * a), precision=FP32)
             for k, a in enumerate((0.4, 0.7, 1.0))]
    states = [developed_state(c, seed=k) for k, c in enumerate(cases)]
    params = gi.init_params(12)
    b = gpu_sim(cases, states, FP32, params)
    b.gnn_forward()
    outs = [b.gnn_output(case=k) for k in range(3)]
    b.close()
    for k, (c, st) in enumerate(zip(cases, states)):
        s = gpu_sim([c], [st], FP32, params)
        s.gnn_forward()
        assert np.array_equal(s.gnn_output(), outs[k])
        s.close()
    _, Yo, _ = oracle_forward(cases[2], states[2], params)
    assert_outputs_match(outs[2], Yo, "forward 12.8k")


def test_training_step_matches_reference():
    case = wl.config_small(1)
    st = developed_state(case, seed=1)
    params = gi.init_params(13)
    rng = np.random.Generator(np.random.PCG64(99))
    T = rng.normal(0, 1, (case.n_fluid, 3))
    g, Yo, cache = oracle_forward(case, st, params)
    loss_o, dY = G.loss_grad(Yo, T)
    grad_o = G.backward(params.astype(np.float64), g, cache, dY, emu=True)
    lr = 1e-3
    p_o, _, _ = G.adam(params.astype(np.float64), grad_o, np.zeros_like(grad_o), np.zeros_like(grad_o), 1, lr)
    s = gpu_sim([case], [st], FP32, params)
    s.gnn_set_target(T)
    loss_g = s.gnn_train_step(lr)
    grad_g = s.gnn_get_grad().astype(np.float64)
    p_g = s.gnn_get_params().astype(np.float64)
    say("loss", loss_g, loss_o)
    assert loss_g == pytest.approx(loss_o, rel=1e-3)
    pg, names = G.unpack(grad_g)
    po, _ = G.unpack(grad_o)
    for n in names:
        nrm = np.linalg.norm(po[n])
        err = np.linalg.norm(pg[n] - po[n])
        say(f"grad {n}: rel err {err / max(nrm, 1e-30):.2e}")
        if nrm > 0:
            assert err <= 5e-3 * nrm, n
        else:
            assert err == 0.0, n
    # Adam's first step moves every parameter by lr against its gradient's sign
    big = np.abs(grad_o) > 1e-3 * np.abs(grad_o).max()
    assert np.allclose(p_g[big], p_o[big], rtol=0, atol=1e-6)
    assert np.all(np.abs(p_g - params) <= lr * 1.001 + 1e-7)
    s.close()


def test_surrogate_with_every_window_rejected_is_the_plain_scheme():
    cases = [wl.dam_break_2d(0.025, seed=k, precision=FP32) for k in range(2)]
    params = gi.init_params(14)
    a = sphx.Simulation.from_cases(cases, FP32)
    a.gnn_set_params(params)
    nfb, nsu = a.surrogate_advance(5, max_drho=-1.0)
    assert nfb == 10 and nsu == 0
    b = sphx.Simulation.from_cases(cases, FP32)
    b.advance(10)
    for k in range(2):
        for f in (sphx.SPHX_FIELD_POS, sphx.SPHX_FIELD_VEL, sphx.SPHX_FIELD_RHO):
            assert np.array_equal(a.get_field(f, case=k), b.get_field(f, case=k))
        assert a.diagnostics(case=k)["t"] == b.diagnostics(case=k)["t"]
    a.close()
    b.close()


def test_accepted_window_applies_the_reference_update():
    case = wl.config_small(2)
    st = developed_state(case, seed=2, speed=0.2)
    params = gi.init_params(15, scale=0.05)   # small outputs: the window is accepted
    _, Yo, _ = oracle_forward(case, st, params)
    s = gpu_sim([case], [st], FP64, params)
    vel, rho, _ = st
    vmax = float(np.sqrt((vel ** 2).sum(1)).max())
    dt = 2.0 * 0.25 * case.h / max(vmax, case.u_ref)
    nfb, nsu = s.surrogate_advance(1, max_drho=1.0)
    assert nsu == 1 and nfb == 0
    x2, v2, r2 = G.apply(Yo, case.fluid_pos, vel, rho, dt, prm_of(case))
    d = s.diagnostics()
    assert d["t"] == pytest.approx(dt, rel=1e-12) and d["n_steps"] == 2
    tol = 8 * 2.0 ** -8 * float(np.sqrt((Yo ** 2).mean()))   # output tolerance, as above
    assert np.abs(s.get_field(sphx.SPHX_FIELD_VEL) - v2).max() <= tol * dt + 1e-12
    assert np.abs(s.get_field(sphx.SPHX_FIELD_POS) - x2).max() <= tol * dt * dt + 1e-12
    assert np.abs(s.get_field(sphx.SPHX_FIELD_RHO) - r2).max() <= tol * case.u_ref / case.h * dt + 1e-12
    s.close()
