"""The allocation-free diagnostics entry point (sphx_diagnostics_noalloc)
against sphx_diagnostics_case, through the C ABI, on two calls in a row with
the second input smaller than the first: the same kernels read the same
state, so the observables agree to the last bit (the bar for a reduction
in a fixed order); sizes beyond the scratch and calls before the device
layout are refused."""
import sys

import numpy as np
import pytest

from paper_2010_12375_amd import sphx
from paper_2010_12375_amd import workloads as wl

pytestmark = pytest.mark.gpu

FP64, FP32 = sphx.SPHX_FP64, sphx.SPHX_FP32
KEYS = ("mass", "e_kin", "e_pot", "e_int", "front", "max_drho", "t", "n_substeps", "n_steps")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b):
    for k in KEYS:
        assert a[k] == b[k], k
    assert np.array_equal(a["momentum"], b["momentum"])


def _sim(cases, precision, steps):
    g = sphx.Simulation.from_cases(cases, precision)
    g.build_neighbors()
    g.advance(steps)
    return g


@pytest.mark.parametrize("precision", [FP32, FP64])
def test_noalloc_diagnostics_match_twice_second_smaller(precision):
    big = wl.dam_break_2d(0.0125, seed=1, precision=precision)     # 12 800 fluid particles
    small = wl.dam_break_2d(0.05, seed=2, precision=precision)      # 800
    for name, case, steps in (("first, 12800 particles", big, 5), ("second, 800 particles", small, 3)):
        say(f"noalloc diagnostics: {name}, precision {precision}")
        g = _sim([case], precision, steps)
        want = g.diagnostics(0)
        got = g.diagnostics_noalloc(0)[0]
        _same(got, want)
        # and once more: the scratch keeps the previous call's contents, which must not leak in
        _same(g.diagnostics_noalloc(0)[0], want)
        g.close()


def test_noalloc_diagnostics_batch_every_case():
    cases = wl.ensemble_cases(6, seed=3)
    g = _sim(cases, FP32, 4)
    want = g.diagnostics_all()
    got = g.diagnostics_noalloc(-1)
    assert len(got) == len(want) == 6
    for a, b in zip(got, want):
        _same(a, b)
    # one case of the batch, then a smaller batch on the same GPU
    _same(g.diagnostics_noalloc(3)[0], want[3])
    g.close()
    h = _sim(cases[:2], FP32, 2)
    for a, b in zip(h.diagnostics_noalloc(-1), h.diagnostics_all()):
        _same(a, b)
    h.close()


def test_noalloc_diagnostics_refusals():
    case = wl.config_small(0)
    g = sphx.Simulation(sphx.params_from_case(case, FP64))
    g.set_fluid(case.fluid_pos)
    # no device layout yet: refused, nothing allocated
    with pytest.raises(sphx.SphxError) as e:
        g.diagnostics_noalloc(0)
    assert e.value.code == sphx.SPHX_ESTATE
    g.build_neighbors()
    with pytest.raises(sphx.SphxError) as e:
        g.diagnostics_noalloc(1)
    assert e.value.code == sphx.SPHX_EINVAL
    _same(g.diagnostics_noalloc(0)[0], g.diagnostics(0))
    g.close()
    # beyond the scratch: 4.2 M particle slots (65 600 tiles of 64) in one case
    n = 65600 * 64
    rng = np.random.Generator(np.random.PCG64(1))
    pos = np.column_stack([rng.uniform(0.0, 40.0, n), rng.uniform(0.0, 40.0, n)])
    big = wl.Case(name="wide", dim=2, dp=0.05, h=0.065, rho0=1.0, c0=20.0, u_ref=2.0, cfl_ad=0.25, cfl_ac=0.6,
                  gravity=(0.0, -1.0, 0.0), lo=(-1.0, -1.0, 0.0), hi=(41.0, 41.0, 0.0), periodic=(0, 0, 0),
                  fluid_pos=pos, wall_pos=np.zeros((0, 2)), wall_normal=np.zeros((0, 2)), column=(40.0, 40.0))
    h = sphx.Simulation(sphx.params_from_case(big, FP32))
    h.set_fluid(big.fluid_pos)
    h.diagnostics(0)  # makes the layout
    with pytest.raises(sphx.SphxError) as e:
        h.diagnostics_noalloc(0)
    assert e.value.code == sphx.SPHX_EINVAL and "65536" in str(e.value)
    h.close()
