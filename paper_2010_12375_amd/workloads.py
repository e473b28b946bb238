"""Seeded synthetic inputs for the dam-break workloads.

This module only builds inputs: particle lattices, seeded position jitter,
wall dummy particles with their normals, the domain box and the case
parameters. It holds none of the method's arithmetic (no kernel, no Riemann
solver, no time stepping) and is shared by the HIP path's callers and by the
tests that drive the oracle.

Geometry follows the paper's dam-break cases (Section 10.1, 2D and 3D dam
break): a water column at rest in the lower-left corner of a tank, released
at t = 0 under gravity, with the tank walls made of wall dummy particles.
The particle generators mirror the lattice generator of the paper's particle
generator table (Section 9): particles sit at ((k + 1/2) dp, ...).

Readings (the paper does not state these):
* wall: 4 layers of lattice points outside the tank interior, so that the
  wall lattice continues the fluid lattice; normals are the normalised sum of
  the outward box-face normals the point lies beyond, i.e. unit vectors
  pointing into the fluid, diagonal in the corners;
* jitter: i.i.d. uniform in [-0.01 dp, 0.01 dp] per coordinate of every fluid
  particle, numpy PCG64(seed);
* 3D: x is the length, y the height (gravity along -y) and z the width; the
  width is periodic and walls cover the floor, the ceiling and both end
  walls;
* sound speed c0 = 20 sqrt(g H) with H the water column height and reference
  speed U_ref = c0 / 10 (Section 2.1: c = 10 U_max keeps density variation
  near 1 %).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

FP64 = 0
FP32 = 1


@dataclasses.dataclass
class WallMotion:
    """Prescribed rigid wall motion: displacement amp sin(omega t) and
    rotation roll sin(omega t) (radians, in the x-y plane) about the centre
    pivot + displacement."""

    amp: tuple = (0.0, 0.0, 0.0)
    omega: float = 0.0
    roll: float = 0.0
    pivot: tuple = (0.0, 0.0, 0.0)


@dataclasses.dataclass
class Case:
    """One simulation input: parameters plus fluid and wall particles."""

    name: str
    dim: int
    dp: float
    h: float
    rho0: float
    c0: float
    u_ref: float
    cfl_ad: float
    cfl_ac: float
    gravity: tuple
    lo: tuple
    hi: tuple
    periodic: tuple
    fluid_pos: np.ndarray          # (n_f, dim) float64
    wall_pos: np.ndarray           # (n_w, dim) float64
    wall_normal: np.ndarray        # (n_w, dim) float64, unit, into the fluid
    precision: int = FP64
    t_end: Optional[float] = None
    n_adv_steps: Optional[int] = None
    column: tuple = ()             # (L, H[, W]) of the water column
    tank: tuple = ()               # (DL, DH[, DW]) of the tank interior
    seed: int = 0
    eta: float = 0.0               # dynamic viscosity (0: inviscid)
    p_background: float = 0.0      # transport-velocity background pressure (0: off)
    reinit_mode: int = 0           # 0: free-surface density re-init, 1: no free surface
    wall_motion: Optional[WallMotion] = None   # None: static walls
    wall_moving: Optional[np.ndarray] = None   # per wall particle 0/1 (None: all follow the motion)
    wall_velocity: Optional[np.ndarray] = None  # (n_w, dim) given wall velocities (None: none)

    @property
    def n_fluid(self) -> int:
        return int(self.fluid_pos.shape[0])

    @property
    def n_wall(self) -> int:
        return int(self.wall_pos.shape[0])


def _lattice(counts, dp):
    axes = [(np.arange(n, dtype=np.float64) + 0.5) * dp for n in counts]
    grids = np.meshgrid(*axes, indexing="ij")
    # particle order: x fastest is irrelevant to the method; keep ij order
    return np.stack([g.reshape(-1) for g in grids], axis=1)


def _jitter(pos, dp, seed, amp=0.01):
    rng = np.random.Generator(np.random.PCG64(seed))
    return pos + rng.uniform(-amp * dp, amp * dp, size=pos.shape)


def tank_walls_2d(DL, DH, dp, layers=4):
    """Wall dummy particles around the box [0, DL] x [0, DH] in 2D."""
    k = np.arange(-layers, int(math.floor(DL / dp + layers - 0.5)) + 1)
    l = np.arange(-layers, int(math.floor(DH / dp + layers - 0.5)) + 1)
    x = (k + 0.5) * dp
    y = (l + 0.5) * dp
    X, Y = np.meshgrid(x, y, indexing="ij")
    X = X.reshape(-1)
    Y = Y.reshape(-1)
    inside = (X >= 0) & (X <= DL) & (Y >= 0) & (Y <= DH)
    keep = (~inside) & (X >= -layers * dp) & (X <= DL + layers * dp) & \
        (Y >= -layers * dp) & (Y <= DH + layers * dp)
    X = X[keep]
    Y = Y[keep]
    nx = np.where(X < 0, 1.0, np.where(X > DL, -1.0, 0.0))
    ny = np.where(Y < 0, 1.0, np.where(Y > DH, -1.0, 0.0))
    nn = np.sqrt(nx * nx + ny * ny)
    pos = np.stack([X, Y], axis=1)
    nrm = np.stack([nx / nn, ny / nn], axis=1)
    return pos, nrm


def _params(dim, dp, H, g=1.0, h_ratio=1.3):
    c0 = 20.0 * math.sqrt(g * H)
    return dict(dim=dim, dp=dp, h=h_ratio * dp, rho0=1.0, c0=c0, u_ref=c0 / 10.0,
                cfl_ad=0.25, cfl_ac=0.6)


def dam_break_2d(dp, seed=0, L=2.0, H=1.0, DL=5.366, DH=5.366, precision=FP64,
                 t_end=None, jitter=0.01, name=None, layers=4):
    """2D dam break: column L x H at the lower-left of a DL x DH tank."""
    nx = int(round(L / dp))
    ny = int(round(H / dp))
    pos = _lattice((nx, ny), dp)
    if jitter:
        pos = _jitter(pos, dp, seed, jitter)
    wpos, wn = tank_walls_2d(DL, DH, dp, layers)
    prm = _params(2, dp, H)
    pad = layers * dp + 2.0 * prm["h"]
    return Case(name=name or f"dambreak2d_dp{dp:g}", gravity=(0.0, -1.0, 0.0),
                lo=(-pad, -pad, 0.0), hi=(DL + pad, DH + pad, 0.0), periodic=(0, 0, 0),
                fluid_pos=pos, wall_pos=wpos, wall_normal=wn, precision=precision,
                t_end=t_end, column=(nx * dp, ny * dp), tank=(DL, DH), seed=seed, **prm)


def dam_break_3d(dp, seed=0, L=2.0, H=1.0, W=1.0, DL=5.366, DH=2.0, precision=FP32,
                 n_adv_steps=None, jitter=0.01, name=None, layers=4):
    """3D dam break, periodic in the width z: column L x H x W in a DL x DH tank."""
    nx = int(round(L / dp))
    ny = int(round(H / dp))
    nz = int(round(W / dp))
    pos = _lattice((nx, ny, nz), dp)
    if jitter:
        pos = _jitter(pos, dp, seed, jitter)
    w2, n2 = tank_walls_2d(DL, DH, dp, layers)
    zs = (np.arange(nz, dtype=np.float64) + 0.5) * dp
    wpos = np.concatenate([np.column_stack([w2, np.full(len(w2), z)]) for z in zs])
    wn = np.concatenate([np.column_stack([n2, np.zeros(len(n2))]) for _ in zs])
    prm = _params(3, dp, H)
    pad = layers * dp + 2.0 * prm["h"]
    return Case(name=name or f"dambreak3d_dp{dp:g}", gravity=(0.0, -1.0, 0.0),
                lo=(-pad, -pad, 0.0), hi=(DL + pad, DH + pad, nz * dp), periodic=(0, 0, 1),
                fluid_pos=pos, wall_pos=wpos, wall_normal=wn, precision=precision,
                n_adv_steps=n_adv_steps, column=(nx * dp, ny * dp, nz * dp),
                tank=(DL, DH, nz * dp), seed=seed, **prm)


# --- the configurations the build is measured on --------------------------

def config_small(seed=0):
    """2D, dp = 0.05 (800 fluid particles), FP64, run to t = 1."""
    return dam_break_2d(0.05, seed=seed, precision=FP64, t_end=1.0, name="dambreak2d_800")


def config_medium(seed=0, precision=FP32):
    """2D, dp = 0.00625 (51 200 fluid particles), FP32 fields, run to t = 20."""
    return dam_break_2d(0.00625, seed=seed, precision=precision, t_end=20.0,
                        name="dambreak2d_51k")


def config_large(seed=0, precision=FP32):
    """3D, dp = 0.01 (2.0 M fluid, 0.596 M wall particles), 2 000 advection steps."""
    return dam_break_3d(0.01, seed=seed, precision=precision, n_adv_steps=2000,
                        name="dambreak3d_2M")


ENSEMBLE_DPS = (0.05, 0.025, 0.0125, 0.00625)


def ensemble_cases(n_cases=64, seed=0, precision=FP32) -> List[Case]:
    """Batched ensemble of uneven 2D dam breaks: dp drawn uniformly from
    ENSEMBLE_DPS, column aspect a = H/L uniform in [0.25, 1] with the column
    area fixed at L H = 2 (so L = sqrt(2/a), H = sqrt(2a)); per-case sound
    speed from its own column height."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for c in range(n_cases):
        dp = float(ENSEMBLE_DPS[int(rng.integers(0, len(ENSEMBLE_DPS)))])
        a = float(rng.uniform(0.25, 1.0))
        L = math.sqrt(2.0 / a)
        H = math.sqrt(2.0 * a)
        case = dam_break_2d(dp, seed=seed * 1000 + c, L=L, H=H, precision=precision,
                            name=f"ens{c:02d}_dp{dp:g}_a{a:.3f}")
        out.append(case)
    return out


def taylor_green_2d(dp=0.02, Re=100.0, U=1.0, seed=0, jitter=0.0, tvf=True, precision=FP64):
    """Decaying Taylor-Green vortex in the periodic unit square (flow
    without free surface): u = -U cos(2 pi x) sin(2 pi y), v = U sin(2 pi x)
    cos(2 pi y), p = rho0 U^2 (cos(4 pi x) + cos(4 pi y)) / 4, viscosity
    eta = rho0 U L / Re with L = 1, no gravity, c0 = 10 U; the velocity
    decays as exp(-8 pi^2 nu t). With `tvf` the transport-velocity
    correction uses the background pressure 0.1 rho0 c0^2 (the paper gives no
    value; rho0 c0^2 makes the correction applied over each acoustic sub-step
    overshoot, 0.1 rho0 c0^2 stays stable)."""
    n = int(round(1.0 / dp))
    pos = _lattice((n, n), dp)
    if jitter:
        pos = _jitter(pos, dp, seed, jitter)
    c0 = 10.0 * U
    rho0 = 1.0
    return Case(name=f"taylorgreen2d_dp{dp:g}_Re{Re:g}", dim=2, dp=dp, h=1.3 * dp, rho0=rho0, c0=c0, u_ref=U,
                cfl_ad=0.25, cfl_ac=0.6, gravity=(0.0, 0.0, 0.0), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 0.0),
                periodic=(1, 1, 0), fluid_pos=pos, wall_pos=np.zeros((0, 2)), wall_normal=np.zeros((0, 2)),
                precision=precision, column=(1.0, 1.0), seed=seed, eta=rho0 * U / Re,
                p_background=0.1 * rho0 * c0 * c0 if tvf else 0.0, reinit_mode=1)


def taylor_green_state(case, U=1.0):
    """Initial velocity and density (from the pressure through the EoS)."""
    x, y = case.fluid_pos[:, 0], case.fluid_pos[:, 1]
    vel = np.stack([-U * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * y),
                    U * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)], axis=1)
    p = case.rho0 * U * U * (np.cos(4 * np.pi * x) + np.cos(4 * np.pi * y)) / 4.0
    return vel, case.rho0 + p / case.c0 ** 2


def hydrostatic_column_2d(dp=0.05, L=1.0, H=1.0, seed=0, jitter=0.0):
    """Water column filling a closed 2D box of width L (walls on both sides),
    for the resting-column check; densities are set by the caller."""
    nx = int(round(L / dp))
    ny = int(round(H / dp))
    pos = _lattice((nx, ny), dp)
    if jitter:
        pos = _jitter(pos, dp, seed, jitter)
    DH = 2.0 * H
    wpos, wn = tank_walls_2d(L, DH, dp)
    prm = _params(2, dp, H)
    pad = 4 * dp + 2.0 * prm["h"]
    return Case(name=f"column2d_dp{dp:g}", gravity=(0.0, -1.0, 0.0),
                lo=(-pad, -pad, 0.0), hi=(L + pad, DH + pad, 0.0), periodic=(0, 0, 0),
                fluid_pos=pos, wall_pos=wpos, wall_normal=wn, precision=FP64,
                column=(nx * dp, ny * dp), tank=(L, DH), seed=seed, **prm)


# --- moving walls and obstacles ------------------------------------------

def motion_reach(wall_pos, motion, moving=None):
    """Per axis, the largest distance a wall particle can move from its
    given position under `motion` (translation amplitude plus the chord of
    the largest rotation)."""
    d = wall_pos.shape[1]
    reach = np.array([abs(float(motion.amp[k])) for k in range(d)])
    if motion.roll:
        sel = wall_pos if moving is None else wall_pos[np.asarray(moving) != 0]
        if len(sel):
            arm = np.sqrt(((sel[:, :2] - np.asarray(motion.pivot[:2])) ** 2).sum(1)).max()
            reach[:2] += abs(float(motion.roll)) * arm
    return reach


def sloshing_first_mode(L, H, g=1.0):
    """Angular frequency of the first sloshing mode of a rectangular tank of
    length L filled to depth H (linear water-wave dispersion relation)."""
    k = math.pi / L
    return math.sqrt(g * k * math.tanh(k * H))


def sloshing_2d(dp, seed=0, L=2.0, H=1.0, DH=2.0, amp=0.05, roll=0.0, omega=None, precision=FP64,
                jitter=0.01, name=None, layers=4):
    """2D sloshing tank: a closed L x DH tank filled to depth H, excited by a
    horizontal sway amp * L * sin(omega t) and a roll about the centre of the
    still water line, omega the first sloshing mode by default. The whole
    tank wall is one rigid moving body; the domain box holds the tank over
    its whole motion."""
    nx = int(round(L / dp))
    ny = int(round(H / dp))
    pos = _lattice((nx, ny), dp)
    if jitter:
        pos = _jitter(pos, dp, seed, jitter)
    wpos, wn = tank_walls_2d(L, DH, dp, layers)
    prm = _params(2, dp, H)
    om = sloshing_first_mode(L, H) if omega is None else float(omega)
    mo = WallMotion(amp=(amp * L, 0.0, 0.0), omega=om, roll=float(roll), pivot=(0.5 * L, H, 0.0))
    reach = motion_reach(wpos, mo)
    pad = layers * dp + 2.0 * prm["h"]
    lo = (-pad - reach[0], -pad - reach[1], 0.0)
    hi = (L + pad + reach[0], DH + pad + reach[1], 0.0)
    return Case(name=name or f"sloshing2d_dp{dp:g}", gravity=(0.0, -1.0, 0.0), lo=lo, hi=hi,
                periodic=(0, 0, 0), fluid_pos=pos, wall_pos=wpos, wall_normal=wn, precision=precision,
                column=(nx * dp, ny * dp), tank=(L, DH), seed=seed, wall_motion=mo, **prm)


def sloshing_3d(dp, seed=0, L=2.0, H=1.0, DH=2.0, W=0.5, amp=0.05, roll=0.0, omega=None, precision=FP32,
                jitter=0.01, name=None, layers=4):
    """3D sloshing tank, periodic in the width z: the 2D tank extruded."""
    nx, ny, nz = int(round(L / dp)), int(round(H / dp)), int(round(W / dp))
    pos = _lattice((nx, ny, nz), dp)
    if jitter:
        pos = _jitter(pos, dp, seed, jitter)
    w2, n2 = tank_walls_2d(L, DH, dp, layers)
    zs = (np.arange(nz, dtype=np.float64) + 0.5) * dp
    wpos = np.concatenate([np.column_stack([w2, np.full(len(w2), z)]) for z in zs])
    wn = np.concatenate([np.column_stack([n2, np.zeros(len(n2))]) for _ in zs])
    prm = _params(3, dp, H)
    om = sloshing_first_mode(L, H) if omega is None else float(omega)
    mo = WallMotion(amp=(amp * L, 0.0, 0.0), omega=om, roll=float(roll), pivot=(0.5 * L, H, 0.0))
    reach = motion_reach(wpos, mo)
    pad = layers * dp + 2.0 * prm["h"]
    lo = (-pad - reach[0], -pad - reach[1], 0.0)
    hi = (L + pad + reach[0], DH + pad + reach[1], nz * dp)
    return Case(name=name or f"sloshing3d_dp{dp:g}", gravity=(0.0, -1.0, 0.0), lo=lo, hi=hi,
                periodic=(0, 0, 1), fluid_pos=pos, wall_pos=wpos, wall_normal=wn, precision=precision,
                column=(nx * dp, ny * dp, nz * dp), tank=(L, DH, nz * dp), seed=seed, wall_motion=mo, **prm)


def obstacle_walls_2d(x0, x1, top, dp, layers=4):
    """Wall particles of a rectangular obstacle [x0, x1] x [0, top] standing
    on the tank floor: lattice points inside it within `layers` spacings of
    its exposed faces (left, right, top); normals point out of the nearest
    exposed face(s), the normalised sum where two are equally near."""
    k = np.arange(int(round(x0 / dp)), int(round(x1 / dp)))
    l = np.arange(0, int(round(top / dp)))
    X, Y = np.meshgrid((k + 0.5) * dp, (l + 0.5) * dp, indexing="ij")
    X, Y = X.reshape(-1), Y.reshape(-1)
    dl, dr, dt = X - x0, x1 - X, top - Y
    dmin = np.minimum(np.minimum(dl, dr), dt)
    keep = dmin < layers * dp
    X, Y, dl, dr, dt, dmin = X[keep], Y[keep], dl[keep], dr[keep], dt[keep], dmin[keep]
    tol = 1e-9 * dp
    nx = np.where(np.abs(dl - dmin) < tol, -1.0, 0.0) + np.where(np.abs(dr - dmin) < tol, 1.0, 0.0)
    ny = np.where(np.abs(dt - dmin) < tol, 1.0, 0.0)
    nn = np.sqrt(nx * nx + ny * ny)
    return np.stack([X, Y], axis=1), np.stack([nx / nn, ny / nn], axis=1)


def dam_break_obstacle_2d(dp, seed=0, obstacle=(3.0, 3.2, 0.4), precision=FP64, t_end=None, name=None):
    """2D dam break hitting a fixed rectangular obstacle on the tank floor
    (the paper's dam break with an obstacle, Section 10.1): the standard
    column and tank plus the obstacle's wall particles."""
    case = dam_break_2d(dp, seed=seed, precision=precision, t_end=t_end,
                        name=name or f"dambreak_obstacle2d_dp{dp:g}")
    opos, on = obstacle_walls_2d(obstacle[0], obstacle[1], obstacle[2], dp)
    case.wall_pos = np.concatenate([case.wall_pos, opos])
    case.wall_normal = np.concatenate([case.wall_normal, on])
    return case


def piston_2d(dp, V=0.2, L=2.0, W=0.4, omega=0.5, precision=FP64, layers=4, name=None):
    """Fluid at rest in a channel periodic across its width W (no gravity),
    pushed from x = 0 by a piston (a wall slab of `layers` spacings) moving
    in +x with velocity V cos(omega t) (displacement V/omega sin(omega t)),
    its far end x = L a free surface."""
    nx, ny = int(round(L / dp)), int(round(W / dp))
    pos = _lattice((nx, ny), dp)
    wpos = _lattice((layers, ny), dp) - np.array([layers * dp, 0.0])
    wn = np.tile([1.0, 0.0], (len(wpos), 1))
    prm = _params(2, dp, 1.0)
    mo = WallMotion(amp=(V / omega, 0.0, 0.0), omega=omega)
    pad = layers * dp + 2.0 * prm["h"]
    # the box holds the piston over its whole stroke [-V/omega, V/omega]
    return Case(name=name or f"piston2d_dp{dp:g}", gravity=(0.0, 0.0, 0.0),
                lo=(-pad - V / omega, 0.0, 0.0), hi=(L + V / omega + pad + 1.0, W, 0.0), periodic=(0, 1, 0),
                fluid_pos=pos, wall_pos=wpos, wall_normal=wn, precision=precision, column=(L, W),
                wall_motion=mo, **prm)


def couette_2d(dp=0.02, H=0.2, L=0.2, U=0.1, nu=0.05, precision=FP64):
    """Plane Couette flow: fluid between a fixed bottom wall and a top wall
    sliding along itself with velocity U (a given wall velocity, the walls do
    not move), periodic along x, no gravity, viscosity nu; the steady profile
    is linear."""
    nx, ny = int(round(L / dp)), int(round(H / dp))
    pos = _lattice((nx, ny), dp)
    wb = _lattice((nx, 4), dp) - np.array([0.0, 4 * dp])
    wt = _lattice((nx, 4), dp) + np.array([0.0, H])
    wpos = np.concatenate([wb, wt])
    wn = np.concatenate([np.tile([0.0, 1.0], (len(wb), 1)), np.tile([0.0, -1.0], (len(wt), 1))])
    wv = np.concatenate([np.zeros((len(wb), 2)), np.tile([U, 0.0], (len(wt), 1))])
    c0 = 10.0 * U
    return Case(name=f"couette2d_dp{dp:g}", dim=2, dp=dp, h=1.3 * dp, rho0=1.0, c0=c0, u_ref=U, cfl_ad=0.25,
                cfl_ac=0.6, gravity=(0.0, 0.0, 0.0), lo=(0.0, -0.2 * H - 4 * dp, 0.0), hi=(L, 1.2 * H + 4 * dp, 0.0),
                periodic=(1, 0, 0), fluid_pos=pos, wall_pos=wpos, wall_normal=wn, precision=precision, column=(L, H),
                eta=nu, reinit_mode=1, wall_velocity=wv)


def lid_cavity_2d(dp=0.02, Re=100.0, U=1.0, L=1.0, seed=0, jitter=0.0, precision=FP64, layers=4):
    """Lid-driven cavity: fluid filling a closed L x L box whose top wall
    slides along itself with velocity U (a given wall velocity), no gravity,
    viscosity rho0 U L / Re, c0 = 10 U, density re-initialisation without
    free surface (a flow without free surface)."""
    n = int(round(L / dp))
    pos = _lattice((n, n), dp)
    if jitter:
        pos = _jitter(pos, dp, seed, jitter)
    wpos, wn = tank_walls_2d(L, L, dp, layers)
    wv = np.where((wpos[:, 1] > L)[:, None], np.array([U, 0.0]), 0.0)
    c0 = 10.0 * U
    pad = layers * dp + 2.6 * dp
    return Case(name=f"lidcavity2d_dp{dp:g}_Re{Re:g}", dim=2, dp=dp, h=1.3 * dp, rho0=1.0, c0=c0, u_ref=U,
                cfl_ad=0.25, cfl_ac=0.6, gravity=(0.0, 0.0, 0.0), lo=(-pad, -pad, 0.0), hi=(L + pad, L + pad, 0.0),
                periodic=(0, 0, 0), fluid_pos=pos, wall_pos=wpos, wall_normal=wn, precision=precision, column=(L, L),
                tank=(L, L), seed=seed, eta=U * L / Re, reinit_mode=1, wall_velocity=wv)
