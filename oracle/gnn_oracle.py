"""FP64 reference of the message-passing surrogate (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module. It shares no code with the HIP path: it receives the SPH
neighbour graph (the inner and contact relations of the configuration,
Section 9 of the SPHinXsys paper) from the FP64 oracle, plain numpy state
arrays and the flat parameter array, and computes the network in numpy.

The surrogate is not part of the paper. It predicts, for every fluid
particle, the mean acceleration and density rate over the next two
advection steps (about 10 acoustic sub-steps); the plain scheme stays the
fallback whenever the predicted density deviates by more than 1 % (the
density variation the artificial sound speed is chosen for, Section 2.1).

Network (hidden width 64, 3 message-passing layers):
  node features f_i: v/u_ref (2), (rho - rho0)/(0.01 rho0), inner and contact
    neighbour counts / 32 and / 16, zero-padded to 32;
  edge features g_e of e = (i -> j), j a fluid or a wall particle:
    (x_j - x_i)/h (2), r/h, (v_j - v_i)/u_ref (2; v_j = 0 for a wall),
    W(r)/W(0), 1 for a wall edge, the pressure difference
    (p_j - p_i)/(rho0 |g| h) with p = c0^2 (rho - rho0) (for a wall the
    one-sided wall state of Section 2.3, p_w - p_i = rho_i g.(x_w - x_i)),
    zero-padded to 32; a difference taken before any rounding, since the
    pressure gradient lives in density differences far below bf16
    resolution of the density itself;
  H = relu(F Wn + bn),  E0 = relu(G We + be)
  layer l:  P = H Wa + bm,  Q = H Wb,  R = E0 Wc
            m_e = relu(P_i + Q_j + R_e)   (wall edge: qw in place of Q_j)
            A_i = sum of m_e over the edges of i
            H <- H + relu([H | A] Wu + bu)
  decoder:  Y = relu(H Wo1 + bo1) Wo2 + bo2,  Y = (a_x/g, a_y/g, 1000 Drho h/(rho0 u_ref))
  (the density rate in units of 0.1 % of rho0 per h/u_ref, so that all three
  outputs are of order one)
With `emu`, every operand of every matrix product is rounded to bfloat16
(round to nearest even) first, as the MFMA kernels take them, except the last
product (D1 Wo2), which stays unrounded; sums are FP64 here.

Parity: gradients are pinned against central finite differences in FP64
(emu off); bf16 rounding against torch's own bfloat16 conversion.
"""
import numpy as np

HIDDEN = 64
LAYERS = 3
FEAT_PAD = 32


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The value is first rounded to float32, as the kernels store it."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(flat):
    """The parameter layout (storage order), as views of a float64 copy."""
    H = HIDDEN
    shapes = [("Wn", (FEAT_PAD, H)), ("bn", (H,)), ("We", (FEAT_PAD, H)), ("be", (H,))]
    for l in range(LAYERS):
        shapes += [(f"Wa{l}", (H, H)), (f"Wb{l}", (H, H)), (f"Wc{l}", (H, H)), (f"bm{l}", (H,)),
                   (f"qw{l}", (H,)), (f"Wu{l}", (2 * H, H)), (f"bu{l}", (H,))]
    shapes += [("Wo1", (H, H)), ("bo1", (H,)), ("Wo2", (H, 3)), ("bo2", (3,))]
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shape in shapes:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    if o != flat.size:
        raise ValueError("parameter array of the wrong size")
    return out, [s for s, _ in shapes]


def pack(d, names):
    return np.concatenate([np.asarray(d[n], dtype=np.float64).reshape(-1) for n in names])


class Graph:
    """The SPH neighbour graph of one configuration: for every fluid particle
    its inner edges then its contact (wall) edges, each in the given list
    order. dst is the fluid index j or the wall index w."""

    def __init__(self, n, inner_off, inner_idx, wall_off, wall_idx):
        self.n = n
        rows, dst, wall = [], [], []
        for i in range(n):
            a, b = inner_off[i], inner_off[i + 1]
            c, d = wall_off[i], wall_off[i + 1]
            rows.append(np.full(b - a + d - c, i, dtype=np.int64))
            dst.append(np.concatenate([inner_idx[a:b], wall_idx[c:d]]).astype(np.int64))
            wall.append(np.concatenate([np.zeros(b - a, bool), np.ones(d - c, bool)]))
        self.src = np.concatenate(rows) if rows else np.zeros(0, np.int64)
        self.dst = np.concatenate(dst) if dst else np.zeros(0, np.int64)
        self.wall = np.concatenate(wall) if wall else np.zeros(0, bool)
        self.n_inner = np.diff(np.asarray(inner_off))
        self.n_wall = np.diff(np.asarray(wall_off))


def graph_from_oracle(orc):
    io, ii = orc.neighbors(0)
    wo, wi = orc.neighbors(1)
    return Graph(len(io) - 1, io, ii, wo, wi)


def wendland_ratio(q):
    """W(r)/W(0) of the Wendland C2 kernel at q = r/h (support 2h)."""
    s = np.clip(1.0 - 0.5 * q, 0.0, None)
    return s ** 4 * (1.0 + 2.0 * q)


def features(graph, x, v, rho, xw, prm):
    """Node and edge features (float64, zero-padded to 32 columns).
    x, v: fluid positions and velocities at the configuration time; xw: wall
    positions; prm: dict with h, rho0, u_ref, c0, gvec (gravity vector)."""
    n, h, u = graph.n, prm["h"], prm["u_ref"]
    F = np.zeros((n, FEAT_PAD))
    F[:, 0:2] = v[:, :2] / u
    F[:, 2] = (rho - prm["rho0"]) / (0.01 * prm["rho0"])
    F[:, 3] = graph.n_inner / 32.0
    F[:, 4] = graph.n_wall / 16.0
    E = graph.src.size
    G = np.zeros((E, FEAT_PAD))
    xi = x[graph.src, :2]
    inner = ~graph.wall
    xj = np.where(inner[:, None], x[np.where(inner, graph.dst, 0), :2], xw[np.where(inner, 0, graph.dst), :2])
    vj = np.where(inner[:, None], v[np.where(inner, graph.dst, 0), :2], 0.0)
    d = xj - xi
    r = np.sqrt((d ** 2).sum(1))
    G[:, 0:2] = d / h
    G[:, 2] = r / h
    G[:, 3:5] = (vj - v[graph.src, :2]) / u
    G[:, 5] = wendland_ratio(r / h)
    G[:, 6] = graph.wall.astype(float)
    gvec = np.asarray(prm["gvec"], dtype=float)[:2]
    gmag = float(np.linalg.norm(gvec))
    rj = np.where(inner, rho[np.where(inner, graph.dst, 0)], 0.0)
    ri = rho[graph.src]
    dp_inner = prm["c0"] ** 2 * (rj - ri)
    dp_wall = ri * (d @ gvec)
    G[:, 7] = np.where(inner, dp_inner, dp_wall) / (prm["rho0"] * gmag * h)
    return F, G


def _mm(a, b, emu):
    return (bf16(a) @ bf16(b)) if emu else a @ b


def forward(flat, graph, F, G, emu=True):
    """Returns Y (n x 3) and the cache for backward."""
    p, _ = unpack(flat)
    relu = lambda z: np.maximum(z, 0.0)
    H = relu(_mm(F, p["Wn"], emu) + p["bn"])
    E0 = relu(_mm(G, p["We"], emu) + p["be"])
    cache = {"F": F, "G": G, "H0": H, "E0": E0, "layers": []}
    inner = ~graph.wall
    for l in range(LAYERS):
        P = _mm(H, p[f"Wa{l}"], emu) + p[f"bm{l}"]
        Q = _mm(H, p[f"Wb{l}"], emu)
        R = _mm(E0, p[f"Wc{l}"], emu)
        pre = P[graph.src] + R
        pre[inner] += Q[graph.dst[inner]]
        pre[~inner] += p[f"qw{l}"]
        M = relu(pre)
        A = np.zeros_like(H)
        np.add.at(A, graph.src, M)
        X = np.concatenate([H, A], axis=1)
        Z = _mm(X, p[f"Wu{l}"], emu) + p[f"bu{l}"]
        cache["layers"].append({"H": H, "pre": pre, "X": X, "Z": Z})
        H = H + relu(Z)
    Z1 = _mm(H, p["Wo1"], emu) + p["bo1"]
    D1 = relu(Z1)
    Y = D1 @ p["Wo2"] + p["bo2"]
    cache.update(H=H, Z1=Z1, D1=D1)
    return Y, cache


def backward(flat, graph, cache, dY, emu=True):
    """Gradient of sum(dY * Y) with respect to the flat parameters."""
    p, names = unpack(flat)
    g = {k: np.zeros_like(v) for k, v in p.items()}
    inner = ~graph.wall
    mmT = lambda a, b: _mm(a.T, b, emu)          # a^T b
    mmW = lambda d, W: _mm(d, W.T, emu)          # d W^T
    D1, H = cache["D1"], cache["H"]
    g["Wo2"] = D1.T @ dY
    g["bo2"] = dY.sum(0)
    dZ1 = (dY @ p["Wo2"].T) * (cache["Z1"] > 0)
    g["Wo1"] = mmT(H, dZ1)
    g["bo1"] = dZ1.sum(0)
    dH = mmW(dZ1, p["Wo1"])
    dE0 = np.zeros_like(cache["E0"])
    E0 = cache["E0"]
    for l in reversed(range(LAYERS)):
        c = cache["layers"][l]
        dZ = dH * (c["Z"] > 0)
        g[f"Wu{l}"] = mmT(c["X"], dZ)
        g[f"bu{l}"] = dZ.sum(0)
        dX = mmW(dZ, p[f"Wu{l}"])
        dHin = dH + dX[:, :HIDDEN]
        dA = dX[:, HIDDEN:]
        dM = dA[graph.src] * (c["pre"] > 0)
        dP = np.zeros_like(dA)
        np.add.at(dP, graph.src, dM)
        dQ = np.zeros_like(dA)
        np.add.at(dQ, graph.dst[inner], dM[inner])
        g[f"qw{l}"] = dM[~inner].sum(0)
        g[f"bm{l}"] = dP.sum(0)
        g[f"Wa{l}"] = mmT(c["H"], dP)
        g[f"Wb{l}"] = mmT(c["H"], dQ)
        g[f"Wc{l}"] = mmT(E0, dM)
        dHin = dHin + mmW(dP, p[f"Wa{l}"]) + mmW(dQ, p[f"Wb{l}"])
        dE0 = dE0 + mmW(dM, p[f"Wc{l}"])
        dH = dHin
    dZe = dE0 * (E0 > 0)
    g["We"] = mmT(cache["G"], dZe)
    g["be"] = dZe.sum(0)
    dZn = dH * (cache["H0"] > 0)
    g["Wn"] = mmT(cache["F"], dZn)
    g["bn"] = dZn.sum(0)
    return pack(g, names)


def loss_grad(Y, T):
    """Mean squared error over all entries and its gradient."""
    diff = Y - T
    return float((diff ** 2).mean()), 2.0 * diff / diff.size


def adam(flat, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1). Returns new (flat, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def apply(Y, x, v, rho, dt, prm):
    """The surrogate's state update over dt from its predicted mean rates:
    v' = v + a dt, x' = x + (v + v')/2 dt, rho' = rho + Drho dt."""
    a = Y[:, 0:2] * prm["g"]
    drho = Y[:, 2] * 1e-3 * prm["rho0"] * prm["u_ref"] / prm["h"]
    v2 = v.copy()
    v2[:, :2] = v[:, :2] + a * dt
    x2 = x.copy()
    x2[:, :2] = x[:, :2] + 0.5 * (v[:, :2] + v2[:, :2]) * dt
    return x2, v2, rho + drho * dt
