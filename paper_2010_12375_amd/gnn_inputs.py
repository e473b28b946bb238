"""Seeded inputs of the message-passing surrogate: the parameter layout and
its random initial values. Shared by the HIP path (through the C ABI) and the
oracle; it holds none of the network's arithmetic.

Layout (float32, one flat array, in this order; every matrix row-major with
the input dimension first, K x 64):
  Wn [32, 64], bn [64]            node encoder (8 features, zero-padded to 32)
  We [32, 64], be [64]            edge encoder (8 features, zero-padded to 32)
  per layer l = 0, 1, 2:
    Wa [64, 64], Wb [64, 64], Wc [64, 64], bm [64], qw [64], Wu [128, 64], bu [64]
  Wo1 [64, 64], bo1 [64], Wo2 [64, 3], bo2 [3]
"""
import numpy as np

HIDDEN = 64
LAYERS = 3
FEAT = 8        # node and edge input features used
FEAT_PAD = 32   # padded input width of the encoders
OUT = 3


def layout():
    """[(name, shape)] in storage order."""
    H = HIDDEN
    out = [("Wn", (FEAT_PAD, H)), ("bn", (H,)), ("We", (FEAT_PAD, H)), ("be", (H,))]
    for l in range(LAYERS):
        out += [(f"Wa{l}", (H, H)), (f"Wb{l}", (H, H)), (f"Wc{l}", (H, H)), (f"bm{l}", (H,)),
                (f"qw{l}", (H,)), (f"Wu{l}", (2 * H, H)), (f"bu{l}", (H,))]
    out += [("Wo1", (H, H)), ("bo1", (H,)), ("Wo2", (H, OUT)), ("bo2", (OUT,))]
    return out


def n_params():
    return int(sum(np.prod(s) for _, s in layout()))


def unpack(flat):
    """Views of the flat array by name."""
    flat = np.asarray(flat)
    out = {}
    o = 0
    for name, shape in layout():
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    assert o == flat.size
    return out


def init_params(seed=0, scale=1.0):
    """Glorot-uniform matrices (zero rows for the padding of the encoder
    inputs), small uniform biases, numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for name, shape in layout():
        if len(shape) == 2:
            fan_in = FEAT if name in ("Wn", "We") else shape[0]
            lim = scale * np.sqrt(6.0 / (fan_in + shape[1]))
            w = rng.uniform(-lim, lim, size=shape)
            if name in ("Wn", "We"):
                w[FEAT:, :] = 0.0
            parts.append(w.reshape(-1))
        else:
            parts.append(rng.uniform(-0.05, 0.05, size=shape).reshape(-1))
    return np.concatenate(parts).astype(np.float32)
