"""Pins of the surrogate's FP64 reference (oracle/gnn_oracle.py), on the CPU:
the bf16 rounding against torch's own conversion, the hand-written backward
against central finite differences, symmetries the network has by
construction, closed forms of degenerate parameter sets, Adam's first step,
and the state update's exactness for constant rates."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import gnn_oracle as G
from paper_2010_12375_amd import gnn_inputs as gi
from paper_2010_12375_amd import workloads as wl
from parity import developed_state


def small_graph(seed=0):
    case = wl.config_small(seed)
    vel, rho, drho = developed_state(case, seed=seed)
    o = O.Oracle(case)
    o.set_fluid(case.fluid_pos, vel, rho, drho)
    o.build_config()
    g = G.graph_from_oracle(o)
    o.close()
    prm = dict(h=case.h, rho0=case.rho0, u_ref=case.u_ref, g=1.0, c0=case.c0, gvec=case.gravity)
    F, E = G.features(g, case.fluid_pos, vel, rho, case.wall_pos, prm)
    return case, g, F, E, prm


def test_bf16_matches_torch_conversion():
    rng = np.random.Generator(np.random.PCG64(1))
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 5000), rng.normal(0, 1e3, 5000)])
    # exact ties: float32 values halfway between two bf16 neighbours
    base = rng.integers(0x3F800000, 0x40000000, 2000, dtype=np.uint64).astype(np.uint32) & 0xFFFF0000
    ties = (base | 0x8000).view(np.float32).astype(np.float64)
    x = np.concatenate([x, ties, -ties, [0.0, -0.0, 1.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(G.bf16(x), ref)


def test_parameter_layouts_agree():
    flat = gi.init_params(3)
    assert flat.size == gi.n_params()
    p, names = G.unpack(flat)
    q = gi.unpack(flat)
    assert names == [n for n, _ in gi.layout()]
    for n in names:
        assert np.array_equal(p[n], q[n].astype(np.float64))
    assert np.all(p["Wn"][8:] == 0) and np.all(p["We"][8:] == 0)


def test_features_of_the_sph_graph():
    case, g, F, E, prm = small_graph()
    assert g.src.size > 10 * g.n
    assert np.all(E[:, 2] < 2.0) and np.all(E[:, 2] > 0.0)       # inside the support 2h
    assert np.all((E[:, 5] > 0) & (E[:, 5] <= 1.0))
    assert np.array_equal(E[:, 6] == 1.0, g.wall)
    assert np.allclose(np.hypot(E[:, 0], E[:, 1]), E[:, 2], rtol=1e-12)
    assert np.all(F[:, 8:] == 0) and np.all(E[:, 8:] == 0)
    # inner edges come in reverse pairs with opposite geometry
    inner = ~g.wall
    key = {(int(a), int(b)): k for k, (a, b) in enumerate(zip(g.src[inner], g.dst[inner]))}
    Ei = E[inner]
    for (a, b), k in list(key.items())[:2000]:
        kr = key[(b, a)]
        assert np.allclose(Ei[k, 0:2], -Ei[kr, 0:2], atol=1e-12) and Ei[k, 2] == pytest.approx(Ei[kr, 2], rel=1e-12)
        assert Ei[k, 7] == pytest.approx(-Ei[kr, 7], rel=1e-12, abs=1e-12)


def test_pressure_feature_is_hydrostatic_height_difference():
    """In a hydrostatic column (p = rho0 g (H - y)) the pressure feature of
    every fluid-fluid edge is (y_i - y_j)/h, and of a wall edge the wall's
    one-sided state: rho_i g.(x_w - x_i)/(rho0 g h)."""
    case = wl.hydrostatic_column_2d(dp=0.05)
    H = case.column[1]
    rho = case.rho0 + case.rho0 * 1.0 * (H - case.fluid_pos[:, 1]) / case.c0 ** 2
    o = O.Oracle(case)
    o.set_fluid(case.fluid_pos, None, rho, None)
    o.build_config()
    g = G.graph_from_oracle(o)
    o.close()
    prm = dict(h=case.h, rho0=case.rho0, u_ref=case.u_ref, g=1.0, c0=case.c0, gvec=case.gravity)
    F, E = G.features(g, case.fluid_pos, np.zeros_like(case.fluid_pos), rho, case.wall_pos, prm)
    inner = ~g.wall
    dy = case.fluid_pos[g.src[inner], 1] - case.fluid_pos[g.dst[inner], 1]
    assert np.allclose(E[inner, 7], dy / case.h, rtol=1e-9, atol=1e-9)
    wy = case.wall_pos[g.dst[~inner], 1] - case.fluid_pos[g.src[~inner], 1]
    assert np.allclose(E[~inner, 7], -rho[g.src[~inner]] * wy / (case.rho0 * case.h), rtol=1e-12)


def test_backward_matches_finite_differences():
    case, g, F, E, prm = small_graph(1)
    flat = gi.init_params(5, scale=1.5).astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(7))
    dY = rng.normal(0, 1, (g.n, 3))
    grad = G.backward(flat, g, G.forward(flat, g, F, E, emu=False)[1], dY, emu=False)
    f = lambda w: float((G.forward(w, g, F, E, emu=False)[0] * dY).sum())
    p, names = G.unpack(flat)
    offs = np.cumsum([0] + [p[n].size for n in names])
    checked = 0
    for k, name in enumerate(names):
        lo, hi = offs[k], offs[k + 1]
        cand = np.arange(lo, hi)
        if name in ("Wn", "We"):
            cand = cand[(cand - lo) // 64 < 8]   # the padding rows have no effect
        for idx in rng.choice(cand, size=min(3, cand.size), replace=False):
            eps = 1e-8 * max(1.0, abs(flat[idx]))  # small enough to cross no relu kink
            wp, wm = flat.copy(), flat.copy()
            wp[idx] += eps
            wm[idx] -= eps
            fd = (f(wp) - f(wm)) / (2 * eps)
            assert fd == pytest.approx(grad[idx], rel=1e-5, abs=1e-7 * (abs(grad).max())), (name, idx)
            checked += 1
    assert checked >= 3 * len(names) - 2


def test_permutation_equivariance():
    case, g, F, E, prm = small_graph(2)
    flat = gi.init_params(6).astype(np.float64)
    Y, _ = G.forward(flat, g, F, E, emu=False)
    rng = np.random.Generator(np.random.PCG64(3))
    perm = rng.permutation(g.n)          # new index k holds old particle perm[k]
    inv = np.argsort(perm)
    g2 = G.Graph.__new__(G.Graph)
    g2.n = g.n
    order = np.argsort(inv[g.src], kind="stable")
    g2.src = inv[g.src][order]
    g2.dst = np.where(g.wall, g.dst, inv[np.where(g.wall, 0, g.dst)])[order]
    g2.wall = g.wall[order]
    g2.n_inner, g2.n_wall = g.n_inner[perm], g.n_wall[perm]
    Y2, _ = G.forward(flat, g2, F[perm], E[order], emu=False)
    assert np.allclose(Y2, Y[perm], rtol=1e-12, atol=1e-12)


def test_translation_invariance():
    case, g, F, E, prm = small_graph(3)
    vel, rho, _ = developed_state(case, seed=3)
    F2, E2 = G.features(g, case.fluid_pos + 0.37, vel, rho, case.wall_pos + 0.37, prm)
    assert np.allclose(F2, F) and np.allclose(E2, E, atol=1e-9)


def test_bias_only_network_closed_form():
    case, g, F, E, prm = small_graph(4)
    flat = gi.init_params(8).astype(np.float64)
    p, names = G.unpack(flat)
    for n in names:
        if n.startswith("W"):
            p[n][...] = 0.0
    z = G.pack(p, names)
    Y, _ = G.forward(z, g, F, E, emu=True)
    # H = relu(bn) + sum_l relu(bu_l) for every node; D1 = relu(bo1) (Wo1 = 0)
    expect = np.maximum(p["bo1"], 0.0) @ p["Wo2"] + p["bo2"]
    assert np.allclose(Y, expect[None, :], rtol=0, atol=0)


def test_adam_first_step_is_a_signed_step():
    rng = np.random.Generator(np.random.PCG64(9))
    w = rng.normal(0, 1, 100)
    gr = rng.normal(0, 1, 100)
    w2, m, v = G.adam(w, gr, np.zeros(100), np.zeros(100), 1, 1e-3)
    assert np.allclose(w2, w - 1e-3 * gr / (np.abs(gr) + 1e-8), rtol=1e-13, atol=1e-16)
    assert np.allclose(m, 0.1 * gr) and np.allclose(v, 0.001 * gr * gr)


def test_apply_is_exact_for_constant_rates():
    rng = np.random.Generator(np.random.PCG64(4))
    n = 50
    x, v, rho = rng.normal(0, 1, (n, 2)), rng.normal(0, 1, (n, 2)), 1 + rng.normal(0, 1e-3, n)
    Y = rng.normal(0, 1, (n, 3))
    prm = dict(h=0.1, rho0=1.0, u_ref=2.0, g=1.0)
    dt = 0.0123
    x2, v2, r2 = G.apply(Y, x, v, rho, dt, prm)
    a = Y[:, :2]
    assert np.allclose(x2, x + v * dt + 0.5 * a * dt * dt, rtol=1e-14, atol=1e-15)
    assert np.allclose(v2, v + a * dt, rtol=1e-14, atol=1e-15)
    assert np.allclose(r2, rho + Y[:, 2] * 0.02 * dt, rtol=1e-14, atol=1e-15)


def test_two_node_forward_by_hand():
    """A two-particle graph (0 <-> 1, and a wall edge of particle 0) with a
    parameter set sparse enough to evaluate the network by hand (FP64, no
    bf16 rounding). Hidden unit 0 carries v_x/u_ref; the first layer's
    message unit 2 is relu(P_i + Q_j + R_e) with P_i = h_i, Q_j = 2 h_j (qw =
    0.5 for the wall) and R_e = relu((x_j - x_i)/h); the node update moves
    relu(A_2) into unit 5, which the decoder passes to the first output.
    So Y_0 = relu(0.3 + 2 0.1 + 0.5) + relu(0.3 + 0.5 + relu(-0.4)) = 1.8 and
    Y_1 = relu(0.1 + 2 0.3 + relu(-0.5)) = 0.7; with the roles of the source
    and the destination swapped (P_j + Q_i) Y_0 would be 1.2 + 0.8 = 2.0, with
    the messages summed at the destination instead of the source Y_1 would be
    1.0, and with R left out Y_0 would be 1.3."""
    g = G.Graph(2, np.array([0, 1, 2]), np.array([1, 0]), np.array([0, 1, 1]), np.array([0]))
    h, u = 0.1, 2.0
    prm = dict(h=h, rho0=1.0, u_ref=u, g=1.0, c0=20.0, gvec=(0.0, -1.0, 0.0))
    x = np.array([[1.0, 1.0], [1.0 + 0.5 * h, 1.0]])
    v = np.array([[0.3 * u, 0.0], [0.1 * u, 0.0]])
    rho = np.array([1.0, 1.0])
    xw = np.array([[1.0 - 0.4 * h, 1.0]])
    F, E = G.features(g, x, v, rho, xw, prm)
    flat = np.zeros(gi.n_params())
    p, names = G.unpack(flat)
    p = {k: np.zeros_like(a) for k, a in p.items()}
    p["Wn"][0, 0] = 1.0            # H[:, 0] = relu(v_x / u_ref)
    p["We"][0, 1] = 1.0            # E0[:, 1] = relu((x_j - x_i) / h)
    p["Wa0"][0, 2] = 1.0           # P[:, 2] = H[:, 0]
    p["Wb0"][0, 2] = 2.0           # Q[:, 2] = 2 H[:, 0]
    p["Wc0"][1, 2] = 1.0           # R[:, 2] = E0[:, 1]
    p["qw0"][2] = 0.5              # a wall edge's Q
    p["Wu0"][64 + 2, 5] = 1.0      # H[:, 5] += relu(A[:, 2])
    p["Wo1"][5, 0] = 1.0
    p["Wo2"][0, 0] = 1.0
    flat = G.pack(p, names)
    Y, _ = G.forward(flat, g, F, E, emu=False)
    assert Y[0, 0] == pytest.approx(1.8, abs=1e-12)
    assert Y[1, 0] == pytest.approx(0.7, abs=1e-12)
    assert np.all(Y[:, 1:] == 0.0)
