"""Batched ensemble: several independent dam breaks in one context, advanced
by the same kernel launches. Every case must give exactly what it gives
alone (the batch changes no arithmetic), match the FP64 oracle to the bars of
the single-case tests, and fail on its own without stopping the others.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2010_12375_amd import sphx
from paper_2010_12375_amd import workloads as wl
from parity import developed_state, rate_errors

pytestmark = pytest.mark.gpu

FP64, FP32 = sphx.SPHX_FP64, sphx.SPHX_FP32


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_cases(precision, aspects=(0.3, 0.62, 1.0), dp=0.05):
    out = []
    for k, a in enumerate(aspects):
        L, H = math.sqrt(2.0 / a), math.sqrt(2.0 * a)
        out.append(wl.dam_break_2d(dp, seed=10 + k, L=L, H=H, precision=precision, name=f"a{a}"))
    return out


def oracle_for(case, state=None):
    o = O.Oracle(case)
    if state is not None:
        o.set_fluid(case.fluid_pos, *state)
    return o


def lists_match(g, c, o, kind):
    og, ig = g.get_neighbors(kind, case=c)
    oo, io = o.neighbors(kind)
    return np.array_equal(og, oo) and np.array_equal(ig, io)


def snapshot(g, c):
    return (g.get_field(sphx.SPHX_FIELD_POS, case=c).tobytes(), g.get_field(sphx.SPHX_FIELD_VEL, case=c).tobytes(),
            g.get_field(sphx.SPHX_FIELD_RHO, case=c).tobytes())


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-9), (FP32, 1e-4)])
def test_ensemble_lists_and_rates_match_oracle(precision, tol):
    """Six uneven cases (dp and aspect drawn as in the 64-case ensemble)."""
    cases = wl.ensemble_cases(6, seed=3, precision=precision)
    say("cases", [c.n_fluid for c in cases])
    states = [developed_state(c, seed=k) for k, c in enumerate(cases)]
    g = sphx.Simulation.from_cases(cases, precision)
    for k, (c, st) in enumerate(zip(cases, states)):
        g.set_fluid(c.fluid_pos, *st, case=k)
    g.build_neighbors()
    total = 0
    for k, (c, st) in enumerate(zip(cases, states)):
        o = oracle_for(c, st)
        o.build_config()
        for kind in (sphx.SPHX_INNER, sphx.SPHX_CONTACT):
            assert lists_match(g, k, o, kind), (k, kind)
        cnt = g.counts(case=k)
        assert cnt["fluid"] == c.n_fluid and cnt["wall"] == c.n_wall
        total += cnt["inner_pairs"]
        dt_ad, dt_ac = o.time_steps()
        ga = g.time_steps(case=k)
        assert ga[1] == pytest.approx(dt_ac, rel=1e-6)
        ag, dg = g.compute_rates(dt_ac, case=k)
        ao, do = o.compute_rates(dt_ac)
        ea, ed = rate_errors(ag, ao, dg, do)
        say("case", k, c.n_fluid, "max err a", ea.max(), "drho", ed.max())
        assert ea.max() <= tol and ed.max() <= tol
        o.close()
    assert g.counts()["inner_pairs"] == total
    g.close()


def test_ensemble_batch_equals_single_runs():
    """Each case of a batch ends bit-identical to the same case run alone,
    including a step queue shorter than a step (continued across queues)."""
    cases = wl.ensemble_cases(5, seed=7)
    cases = [c for c in cases if c.n_fluid <= 13000][:4] or cases[:2]
    say("cases", [c.n_fluid for c in cases])
    first = None
    for q in (0, 2):
        b = sphx.Simulation.from_cases(cases, FP32, nsub_queue=q)
        nb = b.advance(12)
        diag = b.diagnostics_all()
        got = [snapshot(b, k) for k in range(len(cases))]
        b.close()
        if first is None:
            first = got
        assert got == first, "the queue length changed the result"
        ns = 0
        for k, c in enumerate(cases):
            s = sphx.Simulation.from_case(c, FP32, nsub_queue=q)
            ns += s.advance(12)
            assert snapshot(s, 0) == got[k], (q, k)
            d = s.diagnostics()
            assert d["t"] == diag[k]["t"] and d["n_substeps"] == diag[k]["n_substeps"]
            assert diag[k]["n_steps"] == 12
            s.close()
        assert ns == nb


def test_ensemble_fp64_tracks_oracle():
    """Three FP64 cases of different aspect to t = 0.5, observed every 0.1
    (one stop time for the whole batch): each follows its own oracle run."""
    cases = small_cases(FP64)
    g = sphx.Simulation.from_cases(cases, FP64)
    oracles = [oracle_for(c) for c in cases]
    for o in oracles:
        o.build_config()
    for k in range(1, 6):
        T = round(0.1 * k, 10)
        g.advance(100000, T)
        for c, o in enumerate(oracles):
            nsub = 0
            while o.t < T:
                nsub += o.advance(T)
            dg = g.diagnostics(case=c)
            do = o.diagnostics()
            assert dg["t"] == T
            assert abs(dg["front"] - do["front"]) <= 1e-9 * do["front"]
            E = do["e_kin"] + do["e_pot"] + do["e_int"]
            assert abs(dg["e_kin"] + dg["e_pot"] + dg["e_int"] - E) <= 1e-9 * abs(E)
    for c, o in enumerate(oracles):
        xo = o.field(O.FIELD_POS)
        xg = g.get_field(sphx.SPHX_FIELD_POS, case=c)
        assert np.abs(xg - xo).max() < 1e-8
        o.close()
    g.close()


def test_ensemble_case_failure_is_isolated():
    """A case whose particle falls out of its box stops with an escape; the
    other cases run on and end as they do alone."""
    good = small_cases(FP32, aspects=(0.4, 0.9))
    fall = wl.Case(name="fall", dim=2, dp=0.1, h=0.13, rho0=1.0, c0=10.0, u_ref=1.0, cfl_ad=0.25, cfl_ac=0.6,
                   gravity=(0.0, -1.0, 0.0), lo=(-1.0, -1.0, 0.0), hi=(1.0, 1.0, 0.0), periodic=(0, 0, 0),
                   fluid_pos=np.array([[0.0, 0.5]]), wall_pos=np.zeros((0, 2)), wall_normal=np.zeros((0, 2)),
                   column=(0.1, 0.1))
    cases = [good[0], fall, good[1]]
    g = sphx.Simulation.from_cases(cases, FP32)
    with pytest.raises(sphx.SphxError) as e:
        g.advance(80)
    assert e.value.code == sphx.SPHX_EESCAPE and "case 1" in str(e.value)
    assert g.case_status(1) == sphx.SPHX_EESCAPE
    assert g.case_status(0) == sphx.SPHX_OK and g.case_status(2) == sphx.SPHX_OK
    d = g.diagnostics_all()
    assert d[0]["n_steps"] == 80 and d[2]["n_steps"] == 80 and d[1]["n_steps"] < 80
    for k in (0, 2):
        s = sphx.Simulation.from_case(cases[k], FP32)
        s.advance(80)
        assert snapshot(s, 0) == snapshot(g, k)
        s.close()
    g.close()


def test_ensemble_refill_one_case_keeps_the_others():
    """Setting a larger fluid for one case moves the others to new slots;
    they continue exactly as if nothing happened."""
    cases = small_cases(FP32, aspects=(0.5, 0.8))
    g = sphx.Simulation.from_cases(cases, FP32)
    g.advance(5)
    big = wl.dam_break_2d(0.05, seed=3, L=2.5, H=1.6, precision=FP32)
    assert big.lo == cases[1].lo and big.hi == cases[1].hi and big.n_fluid > cases[1].n_fluid + 64
    g.set_fluid(big.fluid_pos, case=1)
    g.advance(5)
    s = sphx.Simulation.from_case(cases[0], FP32)
    s.advance(10)
    assert snapshot(s, 0) == snapshot(g, 0)
    assert g.diagnostics(case=1)["n_steps"] == 5
    s.close()
    g.close()


def test_ensemble_stop_time_lands_exactly_per_case():
    cases = small_cases(FP32)
    g = sphx.Simulation.from_cases(cases, FP32)
    g.advance(100000, 0.37)
    d = g.diagnostics_all()
    assert all(x["t"] == 0.37 for x in d)
    assert len({x["n_steps"] for x in d}) >= 1
    g.close()


def test_autotune_keeps_lists_and_rates():
    cases = wl.ensemble_cases(4, seed=11)
    states = [developed_state(c, seed=k) for k, c in enumerate(cases)]
    g = sphx.Simulation.from_cases(cases, FP32)
    for k, (c, st) in enumerate(zip(cases, states)):
        g.set_fluid(c.fluid_pos, *st, case=k)
    g.build_neighbors()
    lanes = g.autotune(5)
    say("autotuned lanes", lanes)
    assert lanes in (2, 4, 8)
    for k, (c, st) in enumerate(zip(cases, states)):
        o = oracle_for(c, st)
        o.build_config()
        assert lists_match(g, k, o, sphx.SPHX_INNER) and lists_match(g, k, o, sphx.SPHX_CONTACT)
        dt_ad, dt_ac = o.time_steps()
        ag, dg = g.compute_rates(dt_ac, case=k)
        ao, do = o.compute_rates(dt_ac)
        ea, ed = rate_errors(ag, ao, dg, do)
        assert ea.max() <= 1e-4 and ed.max() <= 1e-4
        o.close()
    g.advance(3)
    g.close()


def test_ensemble_64_bench_configuration():
    """The 64-case ensemble as timed: sampled cases (one per dp) bit-exact
    lists and rates within 1e-4 against the oracle, then queued steps keep
    every case's mass and particle count."""
    cases = wl.ensemble_cases(64, seed=0)
    say("ensemble particles", sum(c.n_fluid for c in cases))
    g = sphx.Simulation.from_cases(cases, FP32)
    g.build_neighbors()
    seen = set()
    for k, c in enumerate(cases):
        if c.dp in seen:
            continue
        seen.add(c.dp)
        o = oracle_for(c)
        o.build_config()
        assert lists_match(g, k, o, sphx.SPHX_INNER) and lists_match(g, k, o, sphx.SPHX_CONTACT)
        dt_ad, dt_ac = o.time_steps()
        ag, dg = g.compute_rates(dt_ac, case=k)
        ao, do = o.compute_rates(dt_ac)
        ea, ed = rate_errors(ag, ao, dg, do)
        say("case", k, c.n_fluid, "max err a", ea.max(), "drho", ed.max())
        assert ea.max() <= 1e-4 and ed.max() <= 1e-4
        o.close()
    d0 = g.diagnostics_all()
    g.advance(10)
    d1 = g.diagnostics_all()
    for a, b in zip(d0, d1):
        assert a["mass"] == b["mass"] and b["n_steps"] == 10
    g.close()


@pytest.mark.parametrize("dim,lanes", [(2, 2), (2, 8), (3, 4), (3, 16)])
def test_every_lane_count_gives_the_same_lists_and_rates(dim, lanes):
    """The pair kernels at each lane count (including two lanes per
    particle in 128-thread blocks in 2D): lists bit-exact, rates within 1e-4
    of the oracle (FP32), and runs continue."""
    if dim == 2:
        cases = wl.ensemble_cases(3, seed=5)
    else:
        cases = [wl.dam_break_3d(0.05, seed=2, W=0.4, DL=2.4, DH=1.3)]
    states = [developed_state(c, seed=k + 1) for k, c in enumerate(cases)]
    g = sphx.Simulation.from_cases(cases, FP32)
    for k, (c, st) in enumerate(zip(cases, states)):
        g.set_fluid(c.fluid_pos, *st, case=k)
    g.build_neighbors()
    g.set_lanes(lanes)
    for k, (c, st) in enumerate(zip(cases, states)):
        o = oracle_for(c, st)
        o.build_config()
        assert lists_match(g, k, o, sphx.SPHX_INNER) and lists_match(g, k, o, sphx.SPHX_CONTACT)
        dt_ad, dt_ac = o.time_steps()
        ag, dg = g.compute_rates(dt_ac, case=k)
        ao, do = o.compute_rates(dt_ac)
        ea, ed = rate_errors(ag, ao, dg, do)
        say(dim, lanes, k, "max err a", ea.max(), "drho", ed.max())
        assert ea.max() <= 1e-4 and ed.max() <= 1e-4
        o.close()
    g.advance(4)
    assert all(d["n_steps"] == 4 for d in g.diagnostics_all())
    with pytest.raises(sphx.SphxError):
        g.set_lanes(16 if dim == 2 else 2)
    g.close()
