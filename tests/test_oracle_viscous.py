"""Pins of the oracle's viscous, transport-velocity and no-free-surface terms
(Eqs. eqviscous, transport, eqrhosumnosurface; the h^2/nu advection
criterion, Eq. dt-advection), on the CPU, against what the mathematics
fixes: the Laplacian of a quadratic velocity field, symmetries, closed forms
and restoring directions."""
import numpy as np
import pytest

import oracle as O
from oracle_cases import lattice, params


def _block(ratio, n=25, dp=0.1, eta=0.0, p0=0.0, mode=0, periodic=False):
    pts = lattice((n, n), dp, origin=(-n * dp / 2,) * 2)
    if periodic:
        half = n * dp / 2
        p = params(2, dp=dp, h_ratio=ratio, lo=(-half, -half, -1), hi=(half, half, 1), periodic=(1, 1, 0))
    else:
        p = params(2, dp=dp, h_ratio=ratio, lo=(-2, -2, -2), hi=(2, 2, 2))
    p.eta, p.p_background, p.reinit_mode = eta, p0, mode
    centre = int(np.argmin((pts ** 2).sum(1)))
    return p, pts, centre


@pytest.mark.parametrize("ratio,tol", [(1.3, 0.05), (2.0, 0.01)])
def test_viscous_term_is_the_laplacian_of_a_quadratic_field(ratio, tol):
    """u = kappa y^2 (at rest otherwise, uniform density): nu lap u = 2 nu
    kappa along x at the centre, reached as h/dp grows. Pins the sign, the
    factor 2 and the 1/r W' weight of Eq. (eqviscous). kappa is small so the
    Riemann dissipation (second order in the velocity differences) stays
    negligible."""
    eta, kappa = 0.05, 1e-4
    p, pts, c = _block(ratio, eta=eta)
    vel = np.zeros_like(pts)
    vel[:, 0] = kappa * pts[:, 1] ** 2
    o = O.Oracle(params=p)
    o.set_fluid(pts, vel=vel)
    o.build_config()
    a, _ = o.compute_rates(0.0)
    expect = 2.0 * (eta / 1.0) * kappa
    assert abs(a[c, 0] / expect - 1.0) < tol
    assert abs(a[c, 1]) < 1e-6 * expect


def test_viscous_term_vanishes_for_uniform_motion_and_linear_shear():
    p, pts, c = _block(1.3, eta=0.05)
    for vel in (np.tile([0.3, -0.2], (len(pts), 1)), np.stack([0.4 * pts[:, 1], np.zeros(len(pts))], 1)):
        o = O.Oracle(params=p)
        o.set_fluid(pts, vel=vel)
        o.build_config()
        a, _ = o.compute_rates(0.0)
        assert np.abs(a[c]).max() < 1e-12


def test_viscous_and_pressure_forces_conserve_momentum():
    rng = np.random.Generator(np.random.PCG64(5))
    n, dp = 400, 0.1
    box = np.sqrt(n) * dp
    pts = rng.uniform(0, box, (n, 2))
    p = params(2, dp=dp, lo=(0, 0, -1), hi=(box, box, 1), periodic=(1, 1, 0))
    p.eta = 0.02
    o = O.Oracle(params=p)
    o.set_fluid(pts, vel=rng.normal(0, 0.5, (n, 2)), rho=1.0 + rng.normal(0, 1e-3, n))
    o.build_config()
    a, _ = o.compute_rates(1e-4)
    assert np.abs(a.sum(0)).max() < 1e-10 * np.abs(a).max()


def test_static_wall_slows_a_sliding_layer():
    """Fluid sliding along a static wall at uniform speed: the no-slip wall
    term decelerates the layers within 2h of the wall and nothing beyond."""
    dp = 0.1
    pts = lattice((20, 10), dp, origin=(-1.0, 0.0))
    wall = lattice((20, 4), dp, origin=(-1.0, -0.4))
    nrm = np.tile([0.0, 1.0], (len(wall), 1))
    p = params(2, dp=dp, lo=(-1.0, -0.5, -1), hi=(1.0, 1.5, 1), periodic=(1, 0, 0))
    p.eta = 0.05
    o = O.Oracle(params=p)
    o.set_fluid(pts, vel=np.tile([1.0, 0.0], (len(pts), 1)))
    o.set_walls(wall, nrm)
    o.build_config()
    a, _ = o.compute_rates(0.0)
    # the first wall layer sits at y = -dp/2: particles within 2h of it
    near = pts[:, 1] + dp / 2 < 2 * 1.3 * dp
    far = ~near
    assert np.all(a[near, 0] < 0)
    assert np.abs(a[far, 0]).max() < 1e-12


def test_viscous_time_step_criterion():
    p, pts, c = _block(1.3, eta=2.0)
    o = O.Oracle(params=p)
    o.set_fluid(pts)
    dt_ad, dt_ac = o.time_steps()
    h = p.h
    assert dt_ad == pytest.approx(0.25 * h * h / (2.0 / 1.0), rel=1e-14)
    assert dt_ac == pytest.approx(0.6 * h / 10.0, rel=1e-14)
    p2, _, _ = _block(1.3, eta=1e-6)
    o2 = O.Oracle(params=p2)
    o2.set_fluid(pts)
    assert o2.time_steps()[0] == pytest.approx(0.25 * h / 1.0, rel=1e-14)


def _moved_by_transport(pts, p0, disp_index=None, disp=None):
    p, _, _ = _block(1.3, p0=p0, periodic=True)
    x = pts.copy()
    if disp_index is not None:
        x[disp_index] += disp
    o = O.Oracle(params=p)
    o.set_fluid(x)
    o.build_config()
    o.advance(0.002)
    return o.field(O.FIELD_POS), x


def test_transport_correction_is_zero_on_a_lattice_and_restoring():
    pts = lattice((25, 25), 0.1, origin=(-1.25, -1.25))
    x1, x0 = _moved_by_transport(pts, 10.0)
    assert np.abs(x1 - x0).max() < 1e-13
    k = 300
    d = np.array([0.013, -0.007])
    xt, xs = _moved_by_transport(pts, 10.0, k, d)
    xn, _ = _moved_by_transport(pts, 0.0, k, d)
    shift = xt[k] - xn[k]
    assert np.dot(shift, d) < 0                     # back towards the lattice site
    assert np.linalg.norm(shift) < np.linalg.norm(d)
    others = np.delete(np.arange(len(pts)), k)
    assert np.abs((xt - xn)[others]).max() < np.linalg.norm(shift)


def test_no_surface_reinit_ignores_the_previous_density():
    pts = lattice((25, 25), 0.1, origin=(-1.25, -1.25))
    for mode, expect_high in ((0, True), (1, False)):
        p, _, c = _block(1.3, mode=mode)
        o = O.Oracle(params=p)
        o.set_fluid(pts, rho=np.full(len(pts), 1.5))
        o.build_config()
        o.density_reinit()
        r = o.field(O.FIELD_RHO)
        if expect_high:
            assert r[c] == 1.5
        else:
            assert r[c] == pytest.approx(1.0, abs=1e-12)
