"""ctypes binding of the FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package. It is independent of the HIP library: it loads its own shared
object built from ``sphx_oracle.c`` and imports nothing from the product
package except through the caller, which hands it plain numpy inputs.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SPHX_ORACLE_LIB") or os.path.join(HERE, "liboracle_sphx.so")

OK, EINVAL, ENOMEM, EESCAPE, ENAN, ECAP = 0, -1, -2, -4, -5, -6
FIELD_POS, FIELD_VEL, FIELD_RHO, FIELD_P, FIELD_DRHO = 0, 1, 2, 3, 4


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


class orc_params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("periodic", C.c_int32 * 3), ("dp", C.c_double),
                ("h", C.c_double), ("rho0", C.c_double), ("c0", C.c_double),
                ("u_ref", C.c_double), ("cfl_ad", C.c_double), ("cfl_ac", C.c_double),
                ("g", C.c_double * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("sigma0", C.c_double), ("eta", C.c_double), ("p_background", C.c_double),
                ("reinit_mode", C.c_int32), ("pad_", C.c_int32)]


class orc_wall_motion(C.Structure):
    _fields_ = [("amp", C.c_double * 3), ("omega", C.c_double), ("roll", C.c_double),
                ("pivot", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        pd = C.POINTER(C.c_double)
        L.orc_kernel_W.restype = d
        L.orc_kernel_W.argtypes = [C.c_int, d, d]
        L.orc_kernel_dW.restype = d
        L.orc_kernel_dW.argtypes = [C.c_int, d, d]
        L.orc_lattice_sigma0.restype = d
        L.orc_lattice_sigma0.argtypes = [C.c_int, d, d]
        L.orc_riemann.restype = None
        L.orc_riemann.argtypes = [d, d, d, d, d, d, d, pd, pd]
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.POINTER(orc_params)]
        L.orc_destroy.argtypes = [vp]
        L.orc_destroy.restype = None
        L.orc_sigma0.restype = d
        L.orc_sigma0.argtypes = [vp]
        L.orc_time.restype = d
        L.orc_time.argtypes = [vp]
        L.orc_set_time.restype = None
        L.orc_set_time.argtypes = [vp, d]
        L.orc_set_fluid.restype = C.c_int
        L.orc_set_fluid.argtypes = [vp, i64, vp, vp, vp, vp]
        L.orc_set_walls.restype = C.c_int
        L.orc_set_walls.argtypes = [vp, i64, vp, vp]
        L.orc_set_wall_motion.restype = C.c_int
        L.orc_set_wall_motion.argtypes = [vp, C.POINTER(orc_wall_motion), vp]
        L.orc_set_wall_velocity.restype = C.c_int
        L.orc_set_wall_velocity.argtypes = [vp, vp]
        L.orc_wall_kinematics.restype = C.c_int
        L.orc_wall_kinematics.argtypes = [vp, d, vp, vp, vp]
        L.orc_build_config.restype = C.c_int
        L.orc_build_config.argtypes = [vp]
        L.orc_get_neighbors.restype = i64
        L.orc_get_neighbors.argtypes = [vp, C.c_int, vp, vp, i64]
        L.orc_density_reinit.restype = None
        L.orc_density_reinit.argtypes = [vp]
        L.orc_kernel_sums.restype = None
        L.orc_kernel_sums.argtypes = [vp, vp]
        L.orc_time_steps.restype = None
        L.orc_time_steps.argtypes = [vp, pd, pd]
        L.orc_compute_rates.restype = C.c_int
        L.orc_compute_rates.argtypes = [vp, d, vp, vp]
        L.orc_advance.restype = C.c_int
        L.orc_advance.argtypes = [vp, d, C.POINTER(i32), pd]
        L.orc_get_field.restype = C.c_int
        L.orc_get_field.argtypes = [vp, C.c_int, vp]
        L.orc_diagnostics.restype = None
        L.orc_diagnostics.argtypes = [vp, vp]
        L.orc_num_threads.restype = C.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def kernel_W(dim, h, r):
    return lib().orc_kernel_W(dim, h, r)


def kernel_dW(dim, h, r):
    return lib().orc_kernel_dW(dim, h, r)


def lattice_sigma0(dim, dp, h):
    return lib().orc_lattice_sigma0(dim, dp, h)


def riemann(rhoL, UL, PL, rhoR, UR, PR, c):
    us, ps = C.c_double(), C.c_double()
    lib().orc_riemann(rhoL, UL, PL, rhoR, UR, PR, c, C.byref(us), C.byref(ps))
    return us.value, ps.value


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


def params_from_case(case, sigma0=0.0):
    p = orc_params()
    p.dim = case.dim
    for k in range(3):
        p.periodic[k] = int(case.periodic[k])
        p.g[k] = float(case.gravity[k])
        p.lo[k] = float(case.lo[k])
        p.hi[k] = float(case.hi[k])
    p.dp, p.h, p.rho0, p.c0 = case.dp, case.h, case.rho0, case.c0
    p.u_ref, p.cfl_ad, p.cfl_ac = case.u_ref, case.cfl_ad, case.cfl_ac
    p.sigma0 = sigma0
    p.eta = float(getattr(case, "eta", 0.0))
    p.p_background = float(getattr(case, "p_background", 0.0))
    p.reinit_mode = int(getattr(case, "reinit_mode", 0))
    return p


class Oracle:
    """One FP64 oracle simulation (fluid body + wall body, static or moving)."""

    def __init__(self, case=None, params=None, sigma0=0.0, with_walls=True):
        self._L = lib()
        if params is None:
            params = params_from_case(case, sigma0)
        self.params = params
        self.dim = params.dim
        self._h = self._L.orc_create(C.byref(params))
        if not self._h:
            raise OracleError(EINVAL, "create")
        self.nf = 0
        if case is not None:
            self.set_fluid(case.fluid_pos)
            if with_walls and case.n_wall:
                self.set_walls(case.wall_pos, case.wall_normal)

    def close(self):
        if self._h:
            self._L.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc < 0:
            raise OracleError(rc, what)
        return rc

    @property
    def sigma0(self):
        return self._L.orc_sigma0(self._h)

    @property
    def t(self):
        return self._L.orc_time(self._h)

    @t.setter
    def t(self, value):
        self._L.orc_set_time(self._h, float(value))

    def set_fluid(self, pos, vel=None, rho=None, drho=None):
        pos = _f64(pos)
        n = pos.shape[0]
        vel = _f64(vel)
        rho = _f64(rho)
        drho = _f64(drho)
        self._keep = (pos, vel, rho, drho)
        self._check(self._L.orc_set_fluid(self._h, n, _ptr(pos), _ptr(vel), _ptr(rho), _ptr(drho)),
                    "set_fluid")
        self.nf = n

    def set_walls(self, pos, normal):
        pos = _f64(pos)
        normal = _f64(normal)
        self._check(self._L.orc_set_walls(self._h, pos.shape[0], _ptr(pos), _ptr(normal)),
                    "set_walls")

    def set_wall_motion(self, amp=(0.0, 0.0, 0.0), omega=0.0, roll=0.0, pivot=(0.0, 0.0, 0.0),
                        moving=None, static=False):
        """Prescribed rigid wall motion (static=True: walls static again);
        `moving`: one flag per wall particle (None: all move)."""
        if static:
            self._check(self._L.orc_set_wall_motion(self._h, None, None), "set_wall_motion")
            return
        m = orc_wall_motion()
        for k in range(3):
            m.amp[k] = float(amp[k]) if k < len(amp) else 0.0
            m.pivot[k] = float(pivot[k]) if k < len(pivot) else 0.0
        m.omega, m.roll = float(omega), float(roll)
        flags = None if moving is None else np.ascontiguousarray(moving, dtype=np.int32)
        self._flags = flags
        self._check(self._L.orc_set_wall_motion(self._h, C.byref(m), _ptr(flags)), "set_wall_motion")

    def set_wall_velocity(self, vel):
        """Given velocity of every wall particle (None: none)."""
        v = None if vel is None else _f64(vel)
        self._wv = v
        self._check(self._L.orc_set_wall_velocity(self._h, _ptr(v)), "set_wall_velocity")

    def wall_kinematics(self, t, n_wall):
        """(positions, normals, velocities) of the wall particles at time t."""
        pos = np.zeros((n_wall, self.dim))
        nrm = np.zeros((n_wall, self.dim))
        vel = np.zeros((n_wall, self.dim))
        self._check(self._L.orc_wall_kinematics(self._h, float(t), _ptr(pos), _ptr(nrm), _ptr(vel)),
                    "wall_kinematics")
        return pos, nrm, vel

    def build_config(self):
        self._check(self._L.orc_build_config(self._h), "build_config")

    def neighbors(self, kind=0):
        """(off, idx) CSR of original ids; kind 0 inner, 1 contact."""
        total = self._check(self._L.orc_get_neighbors(self._h, kind, None, None, 0), "neighbors")
        off = np.zeros(self.nf + 1, dtype=np.int64)
        idx = np.zeros(max(total, 1), dtype=np.int64)
        self._check(self._L.orc_get_neighbors(self._h, kind, _ptr(off), _ptr(idx), total),
                    "neighbors")
        return off, idx[:total]

    def density_reinit(self):
        self._L.orc_density_reinit(self._h)

    def kernel_sums(self):
        out = np.zeros(self.nf, dtype=np.float64)
        self._L.orc_kernel_sums(self._h, _ptr(out))
        return out

    def time_steps(self):
        a, b = C.c_double(), C.c_double()
        self._L.orc_time_steps(self._h, C.byref(a), C.byref(b))
        return a.value, b.value

    def compute_rates(self, dt):
        dvdt = np.zeros((self.nf, self.dim), dtype=np.float64)
        drho = np.zeros(self.nf, dtype=np.float64)
        self._check(self._L.orc_compute_rates(self._h, dt, _ptr(dvdt), _ptr(drho)), "compute_rates")
        return dvdt, drho

    def advance(self, t_stop):
        """One advection step clipped to t_stop; returns the sub-step count."""
        n = C.c_int32()
        t = C.c_double()
        self._check(self._L.orc_advance(self._h, float(t_stop), C.byref(n), C.byref(t)), "advance")
        return n.value

    def field(self, which):
        shape = (self.nf, self.dim) if which in (FIELD_POS, FIELD_VEL) else (self.nf,)
        out = np.zeros(shape, dtype=np.float64)
        self._check(self._L.orc_get_field(self._h, which, _ptr(out)), "get_field")
        return out

    def diagnostics(self):
        out = np.zeros(10, dtype=np.float64)
        self._L.orc_diagnostics(self._h, _ptr(out))
        return dict(mass=out[0], momentum=out[1:4].copy(), e_kin=out[4], e_pot=out[5],
                    e_int=out[6], front=out[7], max_drho=out[8], t=out[9])
