"""Small hand-made inputs for oracle pins and parity cases (no method arithmetic)."""
import numpy as np

import oracle as O


def params(dim, dp=0.1, h_ratio=1.3, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0),
           periodic=(0, 0, 0), g=(0.0, 0.0, 0.0), c0=10.0, rho0=1.0, u_ref=None,
           cfl_ad=0.25, cfl_ac=0.6, sigma0=0.0):
    p = O.orc_params()
    p.dim = dim
    for k in range(3):
        p.periodic[k] = int(periodic[k])
        p.g[k] = float(g[k])
        p.lo[k] = float(lo[k])
        p.hi[k] = float(hi[k])
    p.dp = dp
    p.h = h_ratio * dp
    p.rho0 = rho0
    p.c0 = c0
    p.u_ref = c0 / 10.0 if u_ref is None else u_ref
    p.cfl_ad = cfl_ad
    p.cfl_ac = cfl_ac
    p.sigma0 = sigma0
    return p


def lattice(counts, dp, origin=None):
    axes = [(np.arange(n, dtype=np.float64) + 0.5) * dp for n in counts]
    g = np.meshgrid(*axes, indexing="ij")
    pts = np.stack([a.reshape(-1) for a in g], axis=1)
    if origin is not None:
        pts = pts + np.asarray(origin, dtype=np.float64)
    return pts


def jitter(pts, amp, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return pts + rng.uniform(-amp, amp, size=pts.shape)


def brute_force_pairs(xa, xb, rc2, same_body, periodic=(0, 0, 0), lo=None, hi=None):
    """All (i, j) with the predicate r^2 < rc2 evaluated with the same IEEE
    operations the method states: dx = x_i - x_j (one minimum-image wrap on
    periodic axes), r^2 = dx0*dx0 + dx1*dx1 (+ dx2*dx2) left to right."""
    d = xa.shape[1]
    dx = [xa[:, None, k] - xb[None, :, k] for k in range(d)]
    for k in range(d):
        if periodic[k]:
            P = hi[k] - lo[k]
            half = 0.5 * P
            t = dx[k]
            t = np.where(t > half, t - P, np.where(t < -half, t + P, t))
            dx[k] = t
    r2 = dx[0] * dx[0] + dx[1] * dx[1]
    if d == 3:
        r2 = r2 + dx[2] * dx[2]
    m = r2 < rc2
    if same_body:
        np.fill_diagonal(m, False)
    return m


def csr_to_sets(off, idx):
    return [set(idx[off[i]:off[i + 1]].tolist()) for i in range(len(off) - 1)]
