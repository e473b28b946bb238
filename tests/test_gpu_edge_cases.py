"""Edge cases of the hot path on the GPU against the FP64 oracle, through
the C ABI: particle counts around the 64-slot tile (1, 63, 64, 65, 129),
a tight cluster in one cell, the neighbour-list capacity reached exactly and
exceeded by one, positions on the domain boundary, and empty inputs."""
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


def case_from(pos, dp=0.1, lo=(-1.0, -1.0, 0.0), hi=(1.0, 1.0, 0.0), walls=None, periodic=(0, 0, 0)):
    dim = pos.shape[1]
    if walls is None:
        wpos, wn = np.zeros((0, dim)), np.zeros((0, dim))
    else:
        wpos, wn = walls
    return wl.Case(name="edge", dim=dim, dp=dp, h=1.3 * dp, rho0=1.0, c0=10.0, u_ref=1.0, cfl_ad=0.25, cfl_ac=0.6,
                   gravity=(0.0, -1.0, 0.0), lo=lo, hi=hi, periodic=periodic, fluid_pos=pos, wall_pos=wpos,
                   wall_normal=wn, column=(1.0, 1.0))


def lists_equal(g, o):
    for kind in (sphx.SPHX_INNER, sphx.SPHX_CONTACT):
        og, ig = g.get_neighbors(kind)
        oo, io = o.neighbors(kind)
        if not (np.array_equal(og, oo) and np.array_equal(ig, io)):
            return False
    return True


@pytest.mark.parametrize("n", [1, 63, 64, 65, 129])
@pytest.mark.parametrize("precision,tol", [(FP64, 1e-9), (FP32, 1e-4)])
def test_ragged_particle_counts(n, precision, tol):
    """Counts below, at and above the 64-slot tile (the last tile of a case
    partly filled, its unused slots in the padding cell)."""
    rng = np.random.Generator(np.random.PCG64(100 + n))
    lat = wl._lattice((12, 11), 0.1) + np.array([-0.6, -0.4])  # first n sites of a jittered block
    pos = lat[:n] + rng.uniform(-0.001, 0.001, size=(n, 2))
    wpos = np.column_stack([np.linspace(-0.8, 0.8, 17), np.full(17, -0.45)])
    wn = np.tile([0.0, 1.0], (17, 1))
    case = case_from(pos, walls=(wpos, wn))
    st = developed_state(case, seed=n, speed=0.2)
    g, o = make_pair(case, precision, st)
    g.build_neighbors()
    o.build_config()
    assert lists_equal(g, o)
    dt = o.time_steps()[1]
    ag, dg = g.compute_rates(dt)
    ao, do = o.compute_rates(dt)
    ea, ed = rate_errors(ag, ao, dg, do, gmag=1.0)
    assert ea.max() <= tol and ed.max() <= tol
    # a few whole steps: the clock and the sub-step count agree
    ng = g.advance(3)
    no = sum(o.advance(1e9) for _ in range(3))
    if precision == FP64:
        assert ng == no and g.t == pytest.approx(o.t, abs=1e-12)
    else:  # dt from an FP32 |v|max
        assert g.t == pytest.approx(o.t, rel=1e-5)


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_tight_cluster_in_one_cell(precision):
    """40 particles within a disc of radius 0.6h (one cell, every pair a
    neighbour), next to a lattice block."""
    rng = np.random.Generator(np.random.PCG64(7))
    dp = 0.1
    r = 0.6 * 1.3 * dp * np.sqrt(rng.uniform(0, 1, 40))
    a = rng.uniform(0, 2 * np.pi, 40)
    cluster = np.column_stack([0.05 + r * np.cos(a), 0.05 + r * np.sin(a)])
    block = wl._lattice((6, 6), dp) + np.array([0.3, -0.3])
    pos = np.concatenate([cluster, block])
    case = case_from(pos)
    g, o = make_pair(case, precision)
    g.build_neighbors()
    o.build_config()
    assert lists_equal(g, o)
    off, _ = o.neighbors(0)
    assert (np.diff(off)[:40] >= 39).all()
    dt = o.time_steps()[1]
    ag, dg = g.compute_rates(dt)
    ao, do = o.compute_rates(dt)
    ea, ed = rate_errors(ag, ao, dg, do, gmag=1.0)
    assert ea.max() <= (1e-9 if precision == FP64 else 1e-4) and ed.max() <= (1e-9 if precision == FP64 else 1e-4)


def _ring(m):
    """A particle at the centre of a ring of m particles at radius 1.5h: the
    centre has exactly m neighbours, every ring particle fewer."""
    dp = 0.1
    h = 1.3 * dp
    a = 2 * np.pi * (np.arange(m) + 0.25) / m
    ring = np.column_stack([1.5 * h * np.cos(a), 1.5 * h * np.sin(a)])
    return case_from(np.concatenate([[[0.0, 0.0]], ring]), dp=dp)


def test_list_capacity_reached_exactly_then_exceeded():
    """The 2D inner-list capacity is 48 entries: 48 neighbours build exact
    lists, 49 report an overflow."""
    case = _ring(48)
    g, o = make_pair(case, FP64)
    g.build_neighbors()
    o.build_config()
    off, _ = o.neighbors(0)
    assert off[1] - off[0] == 48 and np.diff(off).max() == 48
    assert lists_equal(g, o)
    case = _ring(49)
    g2 = sphx.Simulation.from_case(case, FP64)
    with pytest.raises(sphx.SphxError) as e:
        g2.build_neighbors()
    assert e.value.code == sphx.SPHX_EOVERFLOW


def test_positions_on_the_domain_boundary():
    """A particle exactly on the lower box face is inside (the box is
    half-open); one exactly on the upper face has escaped."""
    pos = np.array([[-1.0, 0.0], [0.0, -1.0], [0.1, 0.1]])
    g, o = make_pair(case_from(pos), FP64)
    g.build_neighbors()
    o.build_config()
    assert lists_equal(g, o)
    pos2 = np.array([[1.0, 0.0], [0.1, 0.1]])
    g2 = sphx.Simulation.from_case(case_from(pos2), FP64)
    with pytest.raises(sphx.SphxError) as e:
        g2.build_neighbors()
    assert e.value.code == sphx.SPHX_EESCAPE


def test_empty_fluid_and_empty_walls():
    case = case_from(np.zeros((0, 2)))
    g = sphx.Simulation(sphx.params_from_case(case, FP64))
    g.set_fluid(np.zeros((0, 2)))
    with pytest.raises(sphx.SphxError) as e:
        g.build_neighbors()
    assert e.value.code == sphx.SPHX_ESTATE
    with pytest.raises(sphx.SphxError) as e:
        g.advance(1)
    assert e.value.code == sphx.SPHX_ESTATE
    # no walls at all: the contact lists are empty
    g.set_fluid(np.array([[0.0, 0.0], [0.05, 0.0]]))
    g.set_walls(np.zeros((0, 2)), np.zeros((0, 2)))
    g.build_neighbors()
    off, idx = g.get_neighbors(sphx.SPHX_CONTACT)
    assert off.tolist() == [0, 0, 0] and idx.size == 0
    off, idx = g.get_neighbors(sphx.SPHX_INNER)
    assert off.tolist() == [0, 1, 2] and idx.tolist() == [1, 0]


# ---------------------------------------------------------------------------
# checkpoints and device-memory input/output

def _state(g, case=0):
    return [g.get_field(f, case).tobytes() for f in (sphx.SPHX_FIELD_POS, sphx.SPHX_FIELD_VEL, sphx.SPHX_FIELD_RHO,
                                                      sphx.SPHX_FIELD_DRHO)]


@pytest.mark.parametrize("which", ["dambreak2d_fp32", "sloshing2d_fp64", "batch_fp32", "dambreak3d_fp32",
                                   "lidcavity2d_fp64"])
def test_checkpoint_restart_is_bit_identical(which, tmp_path):
    """Run, save, run on; a fresh context that loads the file and runs on
    ends bit-identical (all cases, clocks and sub-step counts)."""
    if which == "dambreak2d_fp32":
        cases = [wl.config_small(2)]
        prec = FP32
    elif which == "sloshing2d_fp64":
        cases = [wl.sloshing_2d(0.05, roll=0.05)]
        prec = FP64
    elif which == "lidcavity2d_fp64":
        cases = [wl.lid_cavity_2d(0.05, Re=50.0, U=0.5)]
        prec = FP64
    elif which == "batch_fp32":
        cases = [wl.dam_break_2d(0.05, seed=1, L=1.5, H=1.2), wl.dam_break_2d(0.025, seed=2),
                 wl.sloshing_2d(0.05, roll=0.1)]
        prec = FP32
    else:
        cases = [wl.dam_break_3d(0.05, seed=3, W=0.4, DL=2.4, DH=1.3)]
        prec = FP32
    a = sphx.Simulation.from_cases(cases, prec, nsub_queue=3)
    a.advance(7)
    path = tmp_path / "run.ckpt"
    a.save(path)
    a.advance(9)
    b = sphx.Simulation([sphx.params_from_case(c, prec, 3) for c in cases])
    b.load(path)
    b.advance(9)
    for k in range(len(cases)):
        assert _state(a, k) == _state(b, k), (which, k)
        da, db = a.diagnostics(k), b.diagnostics(k)
        assert da["t"] == db["t"] and da["n_substeps"] == db["n_substeps"] and da["n_steps"] == db["n_steps"]


def test_checkpoint_refused_for_other_parameters(tmp_path):
    case = wl.config_small(0)
    a = sphx.Simulation.from_case(case, FP32)
    a.advance(2)
    path = tmp_path / "run.ckpt"
    a.save(path)
    p = sphx.params_from_case(case, FP32)
    p.c0 = p.c0 * 1.01
    b = sphx.Simulation(p)
    with pytest.raises(sphx.SphxError) as e:
        b.load(path)
    assert e.value.code == sphx.SPHX_EINVAL
    c = sphx.Simulation(sphx.params_from_case(case, FP64))
    with pytest.raises(sphx.SphxError):
        c.load(path)
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(path.read_bytes()[:100])
    d = sphx.Simulation(sphx.params_from_case(case, FP32))
    with pytest.raises(sphx.SphxError):
        d.load(bad)


@pytest.mark.parametrize("flaw", ["duplicate_id", "id_out_of_range", "nan_position", "nan_clock", "error_bits"])
def test_checkpoint_with_corrupt_contents_refused(flaw, tmp_path):
    """A full-length checkpoint whose contents are corrupt (ids that are not
    a permutation, non-finite positions or clock, unknown error bits) is
    refused with SPHX_EINVAL, and the context stays usable."""
    import ctypes as C
    case = wl.config_small(0)
    a = sphx.Simulation.from_case(case, FP32)
    a.advance(2)
    path = tmp_path / "run.ckpt"
    a.save(path)
    raw = bytearray(path.read_bytes())
    n = ((case.n_fluid + 63) // 64) * 64          # slots of the one case (whole tiles)
    ids = len(raw) - 4 * n                         # the ids close the file
    pos0 = ids - 16 * n - 8 * n * case.dim         # FP32 records (16 B) before the ids, positions before them
    ctrl = 8 + 16 + C.sizeof(sphx.sphx_params) + 16  # magic, header, parameters, layout
    if flaw == "duplicate_id":
        raw[ids + 4:ids + 8] = raw[ids:ids + 4]
    elif flaw == "id_out_of_range":
        raw[ids:ids + 4] = np.int32(case.n_fluid).tobytes()
    elif flaw == "nan_position":
        raw[pos0 + 8 * 5:pos0 + 8 * 6] = np.float64(np.nan).tobytes()
    elif flaw == "nan_clock":
        raw[ctrl:ctrl + 8] = np.float64(np.nan).tobytes()
    else:
        err = ctrl + 5 * 8 + 8 + 2 * 32 + 2 * 4 + 3 * 8  # Ctrl.err after the doubles, sub-steps, flags, counters
        raw[err:err + 4] = np.uint32(1 << 7).tobytes()
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(bytes(raw))
    b = sphx.Simulation(sphx.params_from_case(case, FP32))
    b.set_fluid(case.fluid_pos)
    b.set_walls(case.wall_pos, case.wall_normal)
    with pytest.raises(sphx.SphxError) as e:
        b.load(bad)
    assert e.value.code == sphx.SPHX_EINVAL
    assert "corrupt checkpoint" in str(e.value)
    # the intact file still loads into the same context
    b.load(path)
    b.advance(1)
    assert b.diagnostics()["n_steps"] == 3


class _DeviceBuffer:
    """Device memory from the HIP runtime (standing in for a framework
    tensor): a data_ptr() and host copies in and out."""

    def __init__(self, hip, arr):
        import ctypes as C
        self._hip, self.shape = hip, arr.shape
        self.nbytes = arr.nbytes
        self.ptr = C.c_void_p()
        assert hip.hipMalloc(C.byref(self.ptr), C.c_size_t(max(self.nbytes, 8))) == 0
        assert hip.hipMemcpy(self.ptr, arr.ctypes.data_as(C.c_void_p), C.c_size_t(self.nbytes), 1) == 0

    def data_ptr(self):
        return self.ptr.value

    def to_host(self):
        import ctypes as C
        out = np.zeros(self.shape)
        assert self._hip.hipMemcpy(out.ctypes.data_as(C.c_void_p), self.ptr, C.c_size_t(self.nbytes), 2) == 0
        return out

    def free(self):
        self._hip.hipFree(self.ptr)


def test_device_memory_input_and_output():
    """Fluid from device buffers and fields into device buffers give the same
    state and fields as the host calls."""
    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipFree.argtypes = [C.c_void_p]
    case = wl.config_small(3)
    vel, rho, drho = developed_state(case, seed=3)
    h = sphx.Simulation(sphx.params_from_case(case, FP64))
    h.set_fluid(case.fluid_pos, vel, rho, drho)
    h.set_walls(case.wall_pos, case.wall_normal)
    d = sphx.Simulation(sphx.params_from_case(case, FP64))
    bufs = [_DeviceBuffer(hip, np.ascontiguousarray(a, dtype=np.float64)) for a in (case.fluid_pos, vel, rho, drho)]
    d.set_fluid_device(case.n_fluid, *bufs)
    d.set_walls(case.wall_pos, case.wall_normal)
    for g in (h, d):
        g.advance(4)
    assert _state(h) == _state(d)
    out = _DeviceBuffer(hip, np.zeros((case.n_fluid, 2)))
    d.get_field_device(sphx.SPHX_FIELD_VEL, out)
    assert np.array_equal(out.to_host(), d.get_field(sphx.SPHX_FIELD_VEL))
    # refill in place from device memory, now on the device layout
    d.set_fluid_device(case.n_fluid, *bufs)
    h.set_fluid(case.fluid_pos, vel, rho, drho)
    for g in (h, d):
        g.advance(2)
    assert _state(h) == _state(d)
    for b in bufs + [out]:
        b.free()
