"""Moving walls and obstacles (Section 2.3 with a wall velocity u_w, Eq.
eqrienoslip; the sloshing, piston and obstacle cases) on the GPU against the
FP64 oracle, through the C ABI, with the bars of the static path: neighbour
lists bit-exact after the walls have moved, rates within 1e-9 (FP64) and
1e-4 (FP32), FP64 runs tracking the oracle to rounding, FP32 runs within 1 %,
batching and static flags changing nothing."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2010_12375_amd import sphx
from paper_2010_12375_amd import workloads as wl
from parity import developed_state, make_pair, rate_errors

pytestmark = pytest.mark.gpu

FP64, FP32 = sphx.SPHX_FP64, sphx.SPHX_FP32


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_to(sim_g, orc, stops):
    rows = []
    for T in stops:
        sim_g.advance(100000, T)
        while orc.t < T:
            orc.advance(T)
        rows.append((sim_g.diagnostics(), orc.diagnostics()))
    return rows


def same_lists(g, o):
    for kind in (sphx.SPHX_INNER, sphx.SPHX_CONTACT):
        og, ig = g.get_neighbors(kind)
        oo, io = o.neighbors(kind)
        assert np.array_equal(og, oo) and np.array_equal(ig, io)


def slosh(dp=0.05, roll=0.1, precision=FP64):
    return wl.sloshing_2d(dp, roll=roll, precision=precision)


def test_lists_bit_exact_after_the_walls_moved():
    case = slosh()
    g, o = make_pair(case, FP64)
    g.build_neighbors()
    o.build_config()
    same_lists(g, o)
    for T in (0.2, 0.45):
        run_to(g, o, [T])
        say("t", g.t, o.t)
        same_lists(g, o)


@pytest.mark.parametrize("which", ["sway_roll", "piston", "obstacle", "viscous_roll"])
def test_fp64_rates_parity_with_moving_walls(which):
    """Rates of one sub-step after the walls have moved (both sides advanced
    in FP64 to the same time), with the wall velocity non-zero."""
    eta = 0.0
    if which == "sway_roll":
        case = slosh()
    elif which == "piston":
        case = wl.piston_2d(0.02)
    elif which == "obstacle":
        case = wl.dam_break_obstacle_2d(0.05, seed=2)
    else:
        case = slosh()
        case.eta = eta = 0.01
    st = developed_state(case, seed=4, speed=0.2)
    g, o = make_pair(case, FP64, st)
    T = 0.25
    run_to(g, o, [T])
    dt_ad, dt_ac = o.time_steps()
    ag, dg = g.compute_rates(dt_ac)
    ao, do = o.compute_rates(dt_ac)
    ea, ed = rate_errors(ag, ao, dg, do, gmag=1.0)
    say(which, "t", g.t, "max err a", ea.max(), "drho", ed.max())
    assert ea.max() <= 1e-9 and ed.max() <= 1e-9


def test_fp32_rates_parity_at_an_obstacle():
    """FP32 rates with the column against a fixed obstacle (its faces and
    corners in the contact lists), on the seeded developed state."""
    case = wl.dam_break_obstacle_2d(0.025, seed=1, obstacle=(2.0, 2.2, 0.4), precision=FP32)
    g, o = make_pair(case, FP32, developed_state(case, seed=6))
    g.build_neighbors()
    o.build_config()
    n_obstacle = len(wl.obstacle_walls_2d(2.0, 2.2, 0.4, 0.025)[0])
    assert np.count_nonzero(o.neighbors(1)[1] >= case.n_wall - n_obstacle) > 100
    dt_ad, dt_ac = o.time_steps()
    ag, dg = g.compute_rates(dt_ac)
    ao, do = o.compute_rates(dt_ac)
    ea, ed = rate_errors(ag, ao, dg, do, gmag=1.0)
    say("obstacle max err a", ea.max(), "drho", ed.max())
    assert ea.max() <= 1e-4 and ed.max() <= 1e-4


@pytest.mark.parametrize("which", ["sway_roll_2d", "sway_3d"])
def test_fp32_rates_parity_with_moving_walls(which):
    """FP32 rates on the state an FP32 run reached (the oracle takes that
    state, clock and wall pose), within 1e-4."""
    if which == "sway_roll_2d":
        case = slosh(0.025, precision=FP32)
    else:
        case = wl.sloshing_3d(0.05, W=0.4, precision=FP32)
    g = sphx.Simulation.from_case(case, FP32)
    g.advance(100000, 0.3)
    t = g.t
    pos = g.get_field(sphx.SPHX_FIELD_POS)
    vel = g.get_field(sphx.SPHX_FIELD_VEL)
    rho = g.get_field(sphx.SPHX_FIELD_RHO)
    drho = g.get_field(sphx.SPHX_FIELD_DRHO)
    o = O.Oracle(params=O.params_from_case(case))
    o.set_fluid(pos, vel=vel, rho=rho, drho=drho)
    o.set_walls(case.wall_pos, case.wall_normal)
    m = case.wall_motion
    if m is not None:
        o.set_wall_motion(amp=m.amp, omega=m.omega, roll=m.roll, pivot=m.pivot)
    o.t = t
    o.build_config()
    dt_ad, dt_ac = o.time_steps()
    ag, dg = g.compute_rates(dt_ac)
    ao, do = o.compute_rates(dt_ac)
    ea, ed = rate_errors(ag, ao, dg, do, gmag=1.0)
    say(which, "t", t, "max err a", ea.max(), "drho", ed.max())
    assert ea.max() <= 1e-4 and ed.max() <= 1e-4


@pytest.mark.parametrize("which", ["sloshing", "piston", "obstacle", "sloshing_3d"])
def test_fp64_runs_track_the_oracle(which):
    if which == "sloshing":
        case, stops = slosh(roll=0.05), [0.3, 0.6, 1.0]
    elif which == "piston":
        case, stops = wl.piston_2d(0.02), [0.02, 0.04]
    elif which == "obstacle":
        case, stops = wl.dam_break_obstacle_2d(0.05, seed=1), [0.3, 0.6]
    else:
        case, stops = wl.sloshing_3d(0.1, W=0.8, precision=FP64), [0.2, 0.4]
    g, o = make_pair(case, FP64)
    for dg, do in run_to(g, o, stops):
        assert dg["t"] == pytest.approx(do["t"], abs=1e-12)
        assert dg["e_kin"] == pytest.approx(do["e_kin"], rel=1e-9, abs=1e-14)
        assert dg["front"] == pytest.approx(do["front"], rel=1e-9)
    d = np.abs(g.get_field(sphx.SPHX_FIELD_POS) - o.field(O.FIELD_POS))
    if case.periodic[2] or case.periodic[1]:
        per = np.array(case.hi[:case.dim]) - np.array(case.lo[:case.dim])
        d = np.minimum(d, per - d)
    say(which, "max position difference", d.max())
    assert d.max() < 1e-8


def test_fp32_sloshing_within_one_percent():
    case = slosh(0.025, roll=0.05, precision=FP32)
    g, o = make_pair(case, FP32)
    o.build_config()
    d0 = o.diagnostics()
    E0 = d0["e_kin"] + d0["e_pot"] + d0["e_int"]
    for dg, do in run_to(g, o, [0.5, 1.0, 1.5, 2.0]):
        Eg = dg["e_kin"] + dg["e_pot"] + dg["e_int"]
        Eo = do["e_kin"] + do["e_pot"] + do["e_int"]
        say("t", do["t"], "E", Eg / E0, Eo / E0, "front", dg["front"], do["front"])
        assert abs(Eg - Eo) <= 0.01 * abs(E0)
        assert abs(dg["front"] - do["front"]) <= 0.01 * abs(do["front"])


def _fields(sim, case=0):
    return [sim.get_field(f, case) for f in (sphx.SPHX_FIELD_POS, sphx.SPHX_FIELD_VEL, sphx.SPHX_FIELD_RHO)]


def test_batch_with_moving_and_static_cases_is_bit_identical_to_single_runs():
    cases = [slosh(0.05, roll=0.08), wl.dam_break_2d(0.05, seed=4), wl.piston_2d(0.025)]
    batch = sphx.Simulation.from_cases(cases, FP64, nsub_queue=2)
    batch.advance(25)
    for k, c in enumerate(cases):
        one = sphx.Simulation.from_case(c, FP64, nsub_queue=2)
        one.advance(25)
        for a, b in zip(_fields(batch, k), _fields(one)):
            assert np.array_equal(a, b), c.name
        one.close()


def test_walls_flagged_static_match_static_walls():
    case = slosh(0.05, roll=0.1)
    ref = sphx.Simulation.from_case(case, FP64)
    case.wall_moving = np.zeros(case.n_wall, dtype=np.int32)
    flagged = sphx.Simulation.from_case(case, FP64)
    case.wall_motion = None
    static = sphx.Simulation.from_case(case, FP64)
    flagged.advance(30)
    static.advance(30)
    ref.advance(30)
    for a, b in zip(_fields(flagged), _fields(static)):
        assert np.array_equal(a, b)
    assert not np.array_equal(_fields(ref)[0], _fields(static)[0])


def test_motion_outside_the_box_or_along_a_periodic_axis_is_refused():
    case = slosh(0.05)
    g = sphx.Simulation.from_case(case, FP64)
    m = case.wall_motion
    with pytest.raises(sphx.SphxError) as e:
        g.set_wall_motion((5.0, 0.0), m.omega, 0.0, m.pivot)
    assert e.value.code == sphx.SPHX_EINVAL
    with pytest.raises(sphx.SphxError):
        g.set_wall_motion(m.amp, m.omega, 3.0, m.pivot)
    with pytest.raises(sphx.SphxError):
        g.set_wall_motion(m.amp, float("nan"), 0.0, m.pivot)
    p = wl.piston_2d(0.02)
    gp = sphx.Simulation.from_case(p, FP64)
    with pytest.raises(sphx.SphxError):
        gp.set_wall_motion((0.0, 0.01), 1.0, 0.0, (0.0, 0.0))  # y is periodic
    # the refused calls left the accepted motion in place
    g.advance(3)


def test_surrogate_refuses_moving_walls():
    from paper_2010_12375_amd import gnn_inputs as gi
    g = sphx.Simulation.from_case(slosh(0.05), FP32)
    g.build_neighbors()
    with pytest.raises(sphx.SphxError):
        g.gnn_set_params(gi.init_params(0, 0.3))
        g.gnn_forward()


def lid(dp=0.05, precision=FP64, jitter=0.2):
    return wl.lid_cavity_2d(dp, Re=50.0, U=0.5, seed=3, jitter=jitter, precision=precision)


def sliding_slosh(precision=FP64):
    """Sway and roll plus a given velocity on the floor (a belt): both wall
    velocities add."""
    case = slosh(0.05, roll=0.08, precision=precision)
    case.eta = 0.01
    v = np.zeros((case.n_wall, 2))
    v[case.wall_pos[:, 1] < 0.0, 0] = 0.3
    case.wall_velocity = v
    return case


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-9), (FP32, 1e-4)])
@pytest.mark.parametrize("which", ["couette", "lid_cavity", "belt_in_sloshing_tank"])
def test_rates_parity_with_given_wall_velocities(which, precision, tol):
    """Rates with walls carrying given velocities (a sliding lid or belt, no
    slip): the velocity in the wall Riemann states and in the shear."""
    if which == "couette":
        case = wl.couette_2d(precision=precision)
    elif which == "lid_cavity":
        case = lid(0.025, precision)
    else:
        case = sliding_slosh(precision)
    st = developed_state(case, seed=7, speed=0.1)
    g, o = make_pair(case, precision, st)
    g.build_neighbors()
    o.build_config()
    dt_ad, dt_ac = o.time_steps()
    ag, dg = g.compute_rates(dt_ac)
    ao, do = o.compute_rates(dt_ac)
    ea, ed = rate_errors(ag, ao, dg, do, gmag=1.0)
    say(which, precision, "max err a", ea.max(), "drho", ed.max())
    assert ea.max() <= tol and ed.max() <= tol
    # the velocities matter: without them the rates differ
    g.set_wall_velocity(None)
    g.build_neighbors()
    a0, _ = g.compute_rates(dt_ac)
    assert np.abs(a0 - ag).max() > 100 * tol * (np.abs(ao).max() + 1.0)


@pytest.mark.parametrize("which", ["couette", "lid_cavity", "belt_in_sloshing_tank"])
def test_fp64_runs_with_given_wall_velocities_track_the_oracle(which):
    if which == "couette":
        case, stops = wl.couette_2d(), [0.1, 0.3]
    elif which == "lid_cavity":
        case, stops = lid(), [0.1, 0.25]
    else:
        case, stops = sliding_slosh(), [0.2, 0.4]
    g, o = make_pair(case, FP64)
    for dg, do in run_to(g, o, stops):
        assert dg["t"] == pytest.approx(do["t"], abs=1e-12)
        assert dg["e_kin"] == pytest.approx(do["e_kin"], rel=1e-9, abs=1e-14)
    d = np.abs(g.get_field(sphx.SPHX_FIELD_POS) - o.field(O.FIELD_POS))
    if case.periodic[0]:
        per = case.hi[0] - case.lo[0]
        d[:, 0] = np.minimum(d[:, 0], per - d[:, 0])
    say(which, "max position difference", d.max())
    assert d.max() < 1e-8


def test_fp32_lid_cavity_within_one_percent():
    case = lid(0.025, FP32, jitter=0.0)
    g, o = make_pair(case, FP32)
    o.build_config()
    for dg, do in run_to(g, o, [0.2, 0.4]):
        say("t", do["t"], "E_kin", dg["e_kin"], do["e_kin"])
        assert abs(dg["e_kin"] - do["e_kin"]) <= 0.01 * abs(do["e_kin"])


def test_given_wall_velocities_in_a_batch_and_all_zero():
    """A batch of a lid cavity, a dam break and a belt-driven sloshing tank
    is bit-identical to the single runs; all-zero given velocities are the
    static walls bit for bit; set_walls clears them."""
    cases = [lid(), wl.dam_break_2d(0.05, seed=4), sliding_slosh()]
    batch = sphx.Simulation.from_cases(cases, FP64, nsub_queue=2)
    batch.advance(20)
    for k, c in enumerate(cases):
        one = sphx.Simulation.from_case(c, FP64, nsub_queue=2)
        one.advance(20)
        for a, b in zip(_fields(batch, k), _fields(one)):
            assert np.array_equal(a, b), c.name
        one.close()
    case = lid()
    zero = sphx.Simulation.from_case(case, FP64)
    zero.set_wall_velocity(np.zeros_like(case.wall_velocity))
    case.wall_velocity = None
    static = sphx.Simulation.from_case(case, FP64)
    reset = sphx.Simulation.from_case(lid(), FP64)
    reset.set_walls(case.wall_pos, case.wall_normal)
    for s in (zero, static, reset):
        s.advance(15)
    for a, b, c in zip(_fields(zero), _fields(static), _fields(reset)):
        assert np.array_equal(a, b) and np.array_equal(a, c)
    with pytest.raises(sphx.SphxError) as e:
        v = np.zeros((case.n_wall, 2))
        v[3, 1] = float("inf")
        static.set_wall_velocity(v)
    assert e.value.code == sphx.SPHX_EINVAL


def test_surrogate_refuses_given_wall_velocities():
    from paper_2010_12375_amd import gnn_inputs as gi
    g = sphx.Simulation.from_case(lid(), FP32)
    g.build_neighbors()
    with pytest.raises(sphx.SphxError):
        g.gnn_set_params(gi.init_params(0, 0.3))
        g.gnn_forward()


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-9), (FP32, 1e-4)])
@pytest.mark.parametrize("lanes", [2, 8])
def test_wall_velocity_terms_at_other_lane_counts(lanes, precision, tol):
    """The moving-wall, given-velocity and shear terms at 2 lanes per
    particle (128-thread blocks) and at 8: a viscous sloshing tank with a
    belt, run on the GPU to t = 0.2; the oracle takes that state, clock and
    wall pose, and the rates agree."""
    case = sliding_slosh(precision)
    g = sphx.Simulation.from_case(case, precision)
    g.set_lanes(lanes)
    g.advance(100000, 0.2)
    fields = [g.get_field(f) for f in (sphx.SPHX_FIELD_POS, sphx.SPHX_FIELD_VEL, sphx.SPHX_FIELD_RHO,
                                       sphx.SPHX_FIELD_DRHO)]
    o = O.Oracle(params=O.params_from_case(case))
    o.set_fluid(fields[0], vel=fields[1], rho=fields[2], drho=fields[3])
    o.set_walls(case.wall_pos, case.wall_normal)
    m = case.wall_motion
    o.set_wall_motion(amp=m.amp, omega=m.omega, roll=m.roll, pivot=m.pivot)
    o.set_wall_velocity(case.wall_velocity)
    o.t = g.t
    o.build_config()
    dt_ad, dt_ac = o.time_steps()
    ag, dg = g.compute_rates(dt_ac)
    ao, do = o.compute_rates(dt_ac)
    ea, ed = rate_errors(ag, ao, dg, do, gmag=1.0)
    say("lanes", lanes, precision, "t", g.t, "max err a", ea.max(), "drho", ed.max())
    assert ea.max() <= tol and ed.max() <= tol
