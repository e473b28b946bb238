"""Thin ctypes binding of libsphx_hip.so (the C ABI in include/sphx.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. There is no CPU fallback: if the library is missing or fails to
load, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libsphx_hip.so")

SPHX_OK = 0
SPHX_EINVAL, SPHX_ENOMEM, SPHX_EHIP, SPHX_EESCAPE = -1, -2, -3, -4
SPHX_ENAN, SPHX_ECAP, SPHX_EOVERFLOW, SPHX_ESTATE = -5, -6, -7, -8
SPHX_FP64, SPHX_FP32 = 0, 1
SPHX_INNER, SPHX_CONTACT = 0, 1
SPHX_FIELD_POS, SPHX_FIELD_VEL, SPHX_FIELD_RHO, SPHX_FIELD_P, SPHX_FIELD_DRHO = 0, 1, 2, 3, 4

ERROR_NAMES = {SPHX_EINVAL: "EINVAL", SPHX_ENOMEM: "ENOMEM", SPHX_EHIP: "EHIP", SPHX_EESCAPE: "EESCAPE",
               SPHX_ENAN: "ENAN", SPHX_ECAP: "ECAP", SPHX_EOVERFLOW: "EOVERFLOW", SPHX_ESTATE: "ESTATE"}

EXPORTED = ("sphx_create", "sphx_create_batch", "sphx_num_cases", "sphx_set_params_case", "sphx_destroy", "sphx_last_error",
            "sphx_set_fluid", "sphx_set_fluid_case", "sphx_set_walls", "sphx_set_walls_case",
            "sphx_set_wall_motion", "sphx_set_wall_motion_case", "sphx_set_wall_velocity", "sphx_set_wall_velocity_case",
            "sphx_set_fluid_device", "sphx_get_field_device",
            "sphx_save", "sphx_load",
            "sphx_build_neighbors", "sphx_get_neighbors", "sphx_get_neighbors_case", "sphx_density_reinit",
            "sphx_time_steps", "sphx_time_steps_case", "sphx_compute_rates", "sphx_compute_rates_case",
            "sphx_advance", "sphx_case_status", "sphx_get_field", "sphx_get_field_case", "sphx_diagnostics",
            "sphx_diagnostics_case", "sphx_diagnostics_noalloc", "sphx_profile", "sphx_counts", "sphx_counts_case", "sphx_autotune", "sphx_set_lanes",
            "sphx_gnn_num_params", "sphx_gnn_set_params", "sphx_gnn_get_params", "sphx_gnn_get_grad",
            "sphx_gnn_forward", "sphx_gnn_get_output_case", "sphx_gnn_set_target_case", "sphx_gnn_train_step",
            "sphx_gnn_profile", "sphx_surrogate_advance")


class SphxError(RuntimeError):
    def __init__(self, code, what, msg=""):
        super().__init__(f"{what} failed: {ERROR_NAMES.get(code, code)} {msg}".strip())
        self.code = code


class sphx_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("periodic", C.c_int32 * 3),
                ("nsub_queue", C.c_int32), ("dp", C.c_double), ("h", C.c_double), ("rho0", C.c_double),
                ("c0", C.c_double), ("u_ref", C.c_double), ("cfl_ad", C.c_double), ("cfl_ac", C.c_double),
                ("gravity", C.c_double * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("sigma0", C.c_double), ("eta", C.c_double), ("p_background", C.c_double),
                ("reinit_mode", C.c_int32), ("pad_", C.c_int32)]


class sphx_wall_motion(C.Structure):
    _fields_ = [("amp", C.c_double * 3), ("omega", C.c_double), ("roll", C.c_double),
                ("pivot", C.c_double * 3)]


class sphx_diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("momentum", C.c_double * 3), ("e_kin", C.c_double),
                ("e_pot", C.c_double), ("e_int", C.c_double), ("front", C.c_double),
                ("max_drho", C.c_double), ("t", C.c_double), ("n_substeps", C.c_int64),
                ("n_steps", C.c_int64)]


_lib = None


def load(path=None):
    """Load the HIP library (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"HIP library not built: {p} (build it with: python -m paper_2010_12375_amd.build)")
    L = C.CDLL(p)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    pd, pi64 = C.POINTER(C.c_double), C.POINTER(C.c_int64)
    sig = {
        "sphx_create": [C.POINTER(sphx_params), vp, C.POINTER(vp)],
        "sphx_create_batch": [C.POINTER(sphx_params), i32, vp, C.POINTER(vp)],
        "sphx_num_cases": [vp],
        "sphx_set_params_case": [vp, i32, C.POINTER(sphx_params)],
        "sphx_set_fluid": [vp, i64, vp, vp, vp, vp],
        "sphx_set_fluid_case": [vp, i32, i64, vp, vp, vp, vp],
        "sphx_set_walls": [vp, i64, vp, vp],
        "sphx_set_walls_case": [vp, i32, i64, vp, vp],
        "sphx_set_wall_motion": [vp, C.POINTER(sphx_wall_motion), vp],
        "sphx_set_wall_motion_case": [vp, i32, C.POINTER(sphx_wall_motion), vp],
        "sphx_set_wall_velocity": [vp, vp],
        "sphx_set_wall_velocity_case": [vp, i32, vp],
        "sphx_set_fluid_device": [vp, i32, i64, vp, vp, vp, vp],
        "sphx_get_field_device": [vp, i32, C.c_int, vp],
        "sphx_save": [vp, C.c_char_p],
        "sphx_load": [vp, C.c_char_p],
        "sphx_build_neighbors": [vp],
        "sphx_get_neighbors": [vp, C.c_int, vp, vp, i64, pi64],
        "sphx_get_neighbors_case": [vp, i32, C.c_int, vp, vp, i64, pi64],
        "sphx_density_reinit": [vp],
        "sphx_time_steps": [vp, pd, pd],
        "sphx_time_steps_case": [vp, i32, pd, pd],
        "sphx_compute_rates": [vp, d, vp, vp],
        "sphx_compute_rates_case": [vp, i32, d, vp, vp],
        "sphx_advance": [vp, i32, d, pi64, pd],
        "sphx_case_status": [vp, i32],
        "sphx_get_field": [vp, C.c_int, vp],
        "sphx_get_field_case": [vp, i32, C.c_int, vp],
        "sphx_diagnostics": [vp, C.POINTER(sphx_diag)],
        "sphx_diagnostics_case": [vp, i32, C.POINTER(sphx_diag)],
        "sphx_diagnostics_noalloc": [vp, i32, C.POINTER(sphx_diag)],
        "sphx_profile": [vp, i32, pd],
        "sphx_counts": [vp, pi64],
        "sphx_counts_case": [vp, i32, pi64],
        "sphx_autotune": [vp, i32, C.POINTER(i32), pd],
        "sphx_set_lanes": [vp, i32],
        "sphx_gnn_set_params": [vp, vp, i64],
        "sphx_gnn_get_params": [vp, vp, i64],
        "sphx_gnn_get_grad": [vp, vp, i64],
        "sphx_gnn_forward": [vp],
        "sphx_gnn_get_output_case": [vp, i32, vp],
        "sphx_gnn_set_target_case": [vp, i32, vp],
        "sphx_gnn_train_step": [vp, d, pd],
        "sphx_surrogate_advance": [vp, i32, d, i32, pi64, pi64],
        "sphx_gnn_profile": [vp, i32, pd, pi64],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.restype = C.c_int
        f.argtypes = args
    L.sphx_gnn_num_params.restype = i64
    L.sphx_gnn_num_params.argtypes = []
    L.sphx_destroy.restype = None
    L.sphx_destroy.argtypes = [vp]
    L.sphx_last_error.restype = C.c_char_p
    L.sphx_last_error.argtypes = [vp]
    if path is None:
        _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def params_from_case(case, precision=None, nsub_queue=0, sigma0=0.0):
    p = sphx_params()
    p.dim = case.dim
    p.precision = case.precision if precision is None else precision
    for k in range(3):
        p.periodic[k] = int(case.periodic[k])
        p.gravity[k] = float(case.gravity[k])
        p.lo[k] = float(case.lo[k])
        p.hi[k] = float(case.hi[k])
    p.nsub_queue = nsub_queue
    p.dp, p.h, p.rho0, p.c0 = case.dp, case.h, case.rho0, case.c0
    p.u_ref, p.cfl_ad, p.cfl_ac = case.u_ref, case.cfl_ad, case.cfl_ac
    p.sigma0 = sigma0
    p.eta = float(getattr(case, "eta", 0.0))
    p.p_background = float(getattr(case, "p_background", 0.0))
    p.reinit_mode = int(getattr(case, "reinit_mode", 0))
    return p


class Simulation:
    """One library context: a batch of cases (one by default), each a fluid
    body and a wall body (static or moving). Per-case methods take `case`
    (default 0)."""

    def __init__(self, params, stream=None, lib=None):
        self._L = lib or load()
        plist = list(params) if isinstance(params, (list, tuple)) else [params]
        self.params = plist[0]
        self.dim = plist[0].dim
        self.n_cases = len(plist)
        h = C.c_void_p()
        s = None
        if stream is not None:
            s = getattr(stream, "cuda_stream", stream) or None
        if len(plist) == 1:
            rc = self._L.sphx_create(C.byref(plist[0]), s, C.byref(h))
            what = "sphx_create"
        else:
            arr = (sphx_params * len(plist))(*plist)
            rc = self._L.sphx_create_batch(arr, len(plist), s, C.byref(h))
            what = "sphx_create_batch"
        if rc != SPHX_OK:
            raise SphxError(rc, what)
        self._h = h
        self.nf = [0] * self.n_cases

    @classmethod
    def from_case(cls, case, precision=None, nsub_queue=0, stream=None, with_walls=True):
        sim = cls(params_from_case(case, precision, nsub_queue), stream=stream)
        sim.set_fluid(case.fluid_pos)
        if with_walls and case.n_wall:
            sim.set_walls(case.wall_pos, case.wall_normal)
            sim.set_case_motion(case)
        return sim

    @classmethod
    def from_cases(cls, cases, precision=None, nsub_queue=0, stream=None, with_walls=True):
        """A batch of several cases in one context (same dim and precision)."""
        sim = cls([params_from_case(c, precision, nsub_queue) for c in cases], stream=stream)
        for k, c in enumerate(cases):
            sim.set_fluid(c.fluid_pos, case=k)
            if with_walls and c.n_wall:
                sim.set_walls(c.wall_pos, c.wall_normal, case=k)
                sim.set_case_motion(c, case=k)
        return sim

    def close(self):
        if getattr(self, "_h", None):
            self._L.sphx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != SPHX_OK:
            msg = self._L.sphx_last_error(self._h)
            raise SphxError(rc, what, msg.decode() if msg else "")

    def set_fluid(self, pos, vel=None, rho=None, drho=None, case=0):
        pos, vel, rho, drho = _f64(pos), _f64(vel), _f64(rho), _f64(drho)
        self._check(self._L.sphx_set_fluid_case(self._h, case, pos.shape[0], _ptr(pos), _ptr(vel), _ptr(rho),
                                                _ptr(drho)), "sphx_set_fluid_case")
        self.nf[case] = pos.shape[0]

    def set_params(self, params, case=0):
        """Replace case `case`'s parameters (same cell grid)."""
        self._check(self._L.sphx_set_params_case(self._h, case, C.byref(params)), "sphx_set_params_case")

    def set_walls(self, pos, normal, case=0):
        pos, normal = _f64(pos), _f64(normal)
        self._check(self._L.sphx_set_walls_case(self._h, case, pos.shape[0], _ptr(pos), _ptr(normal)),
                    "sphx_set_walls_case")

    def save(self, path):
        """Checkpoint the whole batch to `path`."""
        self._check(self._L.sphx_save(self._h, str(path).encode()), "sphx_save")

    def load(self, path):
        """Restore a checkpoint written by a context with the same parameters."""
        self._check(self._L.sphx_load(self._h, str(path).encode()), "sphx_load")
        self.nf = [int(self.counts(case=k)["fluid"]) for k in range(self.n_cases)]

    @staticmethod
    def _dptr(t):
        """Device address of a tensor-like object (data_ptr()) or an int."""
        if t is None:
            return None
        return C.c_void_p(t.data_ptr() if hasattr(t, "data_ptr") else int(t))

    def set_fluid_device(self, n, pos, vel=None, rho=None, drho=None, case=0):
        """Fluid from device buffers (FP64, original order), e.g. tensors."""
        self._check(self._L.sphx_set_fluid_device(self._h, case, int(n), self._dptr(pos), self._dptr(vel),
                                                  self._dptr(rho), self._dptr(drho)), "sphx_set_fluid_device")
        self.nf[case] = int(n)

    def get_field_device(self, which, out, case=0):
        """Write a field (FP64, original order) into a device buffer."""
        self._check(self._L.sphx_get_field_device(self._h, case, which, self._dptr(out)), "sphx_get_field_device")

    def set_wall_motion(self, amp=(0.0, 0.0, 0.0), omega=0.0, roll=0.0, pivot=(0.0, 0.0, 0.0), moving=None,
                        case=0, static=False):
        """Prescribed rigid motion of case `case`'s walls (static=True: static
        again); `moving`: one flag per wall particle (None: all move)."""
        if static:
            self._check(self._L.sphx_set_wall_motion_case(self._h, case, None, None), "sphx_set_wall_motion_case")
            return
        m = sphx_wall_motion()
        for k in range(3):
            m.amp[k] = float(amp[k]) if k < len(amp) else 0.0
            m.pivot[k] = float(pivot[k]) if k < len(pivot) else 0.0
        m.omega, m.roll = float(omega), float(roll)
        flags = None if moving is None else np.ascontiguousarray(moving, dtype=np.int32)
        self._check(self._L.sphx_set_wall_motion_case(self._h, case, C.byref(m), _ptr(flags)),
                    "sphx_set_wall_motion_case")

    def set_wall_velocity(self, vel, case=0):
        """Given velocities of case `case`'s wall particles (n_wall x dim; None
        clears them); the walls do not move with them."""
        v = _f64(vel)
        self._check(self._L.sphx_set_wall_velocity_case(self._h, case, _ptr(v)), "sphx_set_wall_velocity_case")

    def set_case_motion(self, c, case=0):
        """Apply a workload case's wall motion and given wall velocities, if
        it has them."""
        m = getattr(c, "wall_motion", None)
        if m is not None:
            self.set_wall_motion(m.amp, m.omega, m.roll, m.pivot, getattr(c, "wall_moving", None), case=case)
        v = getattr(c, "wall_velocity", None)
        if v is not None:
            self.set_wall_velocity(v, case=case)

    def build_neighbors(self):
        self._check(self._L.sphx_build_neighbors(self._h), "sphx_build_neighbors")

    def get_neighbors(self, kind=SPHX_INNER, case=0):
        n = C.c_int64()
        off = np.zeros(self.nf[case] + 1, dtype=np.int64)
        self._check(self._L.sphx_get_neighbors_case(self._h, case, kind, _ptr(off), None, 0, C.byref(n)),
                    "sphx_get_neighbors_case")
        idx = np.zeros(max(n.value, 1), dtype=np.int64)
        self._check(self._L.sphx_get_neighbors_case(self._h, case, kind, None, _ptr(idx), n.value, C.byref(n)),
                    "sphx_get_neighbors_case")
        return off, idx[:n.value]

    def density_reinit(self):
        self._check(self._L.sphx_density_reinit(self._h), "sphx_density_reinit")

    def time_steps(self, case=0):
        a, b = C.c_double(), C.c_double()
        self._check(self._L.sphx_time_steps_case(self._h, case, C.byref(a), C.byref(b)), "sphx_time_steps_case")
        return a.value, b.value

    def compute_rates(self, dt, case=0):
        dvdt = np.zeros((self.nf[case], self.dim), dtype=np.float64)
        drho = np.zeros(self.nf[case], dtype=np.float64)
        self._check(self._L.sphx_compute_rates_case(self._h, case, float(dt), _ptr(dvdt), _ptr(drho)),
                    "sphx_compute_rates_case")
        return dvdt, drho

    def advance(self, n_steps=1, t_stop=float("inf")):
        """Advance every case; returns the acoustic sub-steps done (summed
        over the cases)."""
        n = C.c_int64()
        t = C.c_double()
        self._check(self._L.sphx_advance(self._h, int(n_steps), float(t_stop), C.byref(n), C.byref(t)),
                    "sphx_advance")
        return n.value

    def case_status(self, case):
        return self._L.sphx_case_status(self._h, case)

    def get_field(self, which, case=0):
        nf = self.nf[case]
        shape = (nf, self.dim) if which in (SPHX_FIELD_POS, SPHX_FIELD_VEL) else (nf,)
        out = np.zeros(shape, dtype=np.float64)
        self._check(self._L.sphx_get_field_case(self._h, case, which, _ptr(out)), "sphx_get_field_case")
        return out

    @staticmethod
    def _diag_dict(d):
        return dict(mass=d.mass, momentum=np.array(d.momentum[:]), e_kin=d.e_kin, e_pot=d.e_pot,
                    e_int=d.e_int, front=d.front, max_drho=d.max_drho, t=d.t, n_substeps=d.n_substeps,
                    n_steps=d.n_steps)

    def diagnostics(self, case=0):
        d = sphx_diag()
        self._check(self._L.sphx_diagnostics_case(self._h, case, C.byref(d)), "sphx_diagnostics_case")
        return self._diag_dict(d)

    def diagnostics_noalloc(self, case=-1):
        """sphx_diagnostics_noalloc: the observables with no allocation in the
        call (case < 0: every case)."""
        n = self.n_cases if case < 0 else 1
        arr = (sphx_diag * n)()
        self._check(self._L.sphx_diagnostics_noalloc(self._h, case, arr), "sphx_diagnostics_noalloc")
        return [self._diag_dict(d) for d in arr]

    def diagnostics_all(self):
        arr = (sphx_diag * self.n_cases)()
        self._check(self._L.sphx_diagnostics_case(self._h, -1, arr), "sphx_diagnostics_case")
        return [self._diag_dict(d) for d in arr]

    @property
    def t(self):
        return self.diagnostics()["t"]

    def profile(self, reps=20):
        ms = (C.c_double * 4)()
        self._check(self._L.sphx_profile(self._h, int(reps), ms), "sphx_profile")
        return dict(pressure=ms[0], density=ms[1], neighbors=ms[2], reinit=ms[3])

    def counts(self, case=None):
        out = (C.c_int64 * 4)()
        if case is None:
            self._check(self._L.sphx_counts(self._h, out), "sphx_counts")
        else:
            self._check(self._L.sphx_counts_case(self._h, case, out), "sphx_counts_case")
        return dict(fluid=out[0], wall=out[1], inner_pairs=out[2], contact_pairs=out[3])

    # -- message-passing surrogate (2D) --
    def gnn_num_params(self):
        return int(self._L.sphx_gnn_num_params())

    def gnn_set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self._L.sphx_gnn_set_params(self._h, _ptr(p), p.size), "sphx_gnn_set_params")

    def gnn_get_params(self):
        p = np.zeros(self.gnn_num_params(), dtype=np.float32)
        self._check(self._L.sphx_gnn_get_params(self._h, _ptr(p), p.size), "sphx_gnn_get_params")
        return p

    def gnn_get_grad(self):
        p = np.zeros(self.gnn_num_params(), dtype=np.float32)
        self._check(self._L.sphx_gnn_get_grad(self._h, _ptr(p), p.size), "sphx_gnn_get_grad")
        return p

    def gnn_forward(self):
        self._check(self._L.sphx_gnn_forward(self._h), "sphx_gnn_forward")

    def gnn_output(self, case=0):
        out = np.zeros((self.nf[case], 3), dtype=np.float64)
        self._check(self._L.sphx_gnn_get_output_case(self._h, case, _ptr(out)), "sphx_gnn_get_output_case")
        return out

    def gnn_set_target(self, target, case=0):
        t = np.ascontiguousarray(target, dtype=np.float64)
        self._check(self._L.sphx_gnn_set_target_case(self._h, case, _ptr(t)), "sphx_gnn_set_target_case")

    def gnn_train_step(self, lr):
        loss = C.c_double()
        self._check(self._L.sphx_gnn_train_step(self._h, float(lr), C.byref(loss)), "sphx_gnn_train_step")
        return loss.value

    def gnn_profile(self, reps=20):
        ms = (C.c_double * 7)()
        sz = (C.c_int64 * 2)()
        self._check(self._L.sphx_gnn_profile(self._h, int(reps), ms, sz), "sphx_gnn_profile")
        return dict(fused_layer=ms[0], edge_features=ms[1], node_gemm=ms[2], forward=ms[3],
                    forward_unfused=ms[4], edge_gemm_unfused=ms[5], messages_unfused=ms[6], nodes=sz[0], edges=sz[1])

    def surrogate_advance(self, windows, max_drho=0.01, plain_every=0):
        a, b = C.c_int64(), C.c_int64()
        self._check(self._L.sphx_surrogate_advance(self._h, int(windows), float(max_drho), int(plain_every),
                                                   C.byref(a), C.byref(b)), "sphx_surrogate_advance")
        return a.value, b.value

    def set_lanes(self, lanes):
        """Lanes per particle of the pair kernels (2, 4, 8 in 2D; 4, 8, 16 in 3D)."""
        self._check(self._L.sphx_set_lanes(self._h, int(lanes)), "sphx_set_lanes")

    def autotune(self, reps=10, with_times=False):
        lanes = C.c_int32()
        times = (C.c_double * 3)()
        self._check(self._L.sphx_autotune(self._h, int(reps), C.byref(lanes), times), "sphx_autotune")
        if with_times:
            return lanes.value, dict(zip((2, 4, 8) if self.dim == 2 else (4, 8, 16), times[:]))
        return lanes.value
