"""ctypes front end of the FP64 CPU oracle (``oracle/sphx_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to check and time the GPU library.  Nothing in the
product package imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SPHX_ORACLE_LIB", os.path.join(HERE, "libsphx_oracle.so"))

MAX_PISTON = 16
X, U, RHO, A, DRHO, AP, AV, AS, SDRHO, SAP, SAV, SAS, P, GRADC, TENSOR = range(15)
_VEC = {X, U, A, AP, AV, AS, GRADC}


class _Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("visc_form", C.c_int32), ("cont_form", C.c_int32),
        ("renorm_every", C.c_int32),
        ("h", C.c_double), ("gamma", C.c_double), ("delta_coef", C.c_double),
        ("alpha_s", C.c_double),
        ("gravity", C.c_double * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("periodic", C.c_int32 * 3),
        ("c_cfl", C.c_double), ("c_force", C.c_double),
        ("c_visc", C.c_double), ("c_st", C.c_double), ("dt_fixed", C.c_double),
        ("n_piston", C.c_int32), ("piston_t_end", C.c_double),
        ("piston_a", C.c_double * MAX_PISTON), ("piston_w", C.c_double * MAX_PISTON),
        ("piston_phi", C.c_double * MAX_PISTON),
    ]


class _Phase(C.Structure):
    _fields_ = [("rho0", C.c_double), ("nu", C.c_double), ("c0", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run oracle/build.py)")
        L = C.CDLL(LIB_PATH)
        d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        L.so_kernel_w.restype = d
        L.so_kernel_w.argtypes = [i32, d, d]
        L.so_kernel_f.restype = d
        L.so_kernel_f.argtypes = [i32, d, d]
        L.so_eos.restype = d
        L.so_eos.argtypes = [d, d, d, d]
        L.so_piston.restype = None
        L.so_piston.argtypes = [C.POINTER(_Params), d, C.POINTER(d), C.POINTER(d)]
        L.so_set_moving.restype = None
        L.so_set_moving.argtypes = [vp, vp, vp]
        L.so_create.restype = vp
        L.so_create.argtypes = [C.POINTER(_Params), C.POINTER(_Phase), i32, i64] + [vp] * 6
        L.so_destroy.argtypes = [vp]
        L.so_set_threads.argtypes = [i32]
        L.so_get_threads.restype = i32
        L.so_set_neighbor_method.argtypes = [vp, i32]
        L.so_neighbors.restype = i64
        L.so_neighbors.argtypes = [vp, vp, vp, i64]
        L.so_renormalize.argtypes = [vp]
        L.so_rates.restype = i64
        L.so_rates.argtypes = [vp]
        L.so_dt.restype = d
        L.so_dt.argtypes = [vp]
        L.so_step.restype = i64
        L.so_step.argtypes = [vp, i32]
        L.so_time.restype = d
        L.so_time.argtypes = [vp]
        L.so_stepcount.restype = i64
        L.so_stepcount.argtypes = [vp]
        L.so_get.restype = i32
        L.so_get.argtypes = [vp, i32, vp]
        L.so_set.restype = i32
        L.so_set.argtypes = [vp, i32, vp]
        L.so_pair_terms.restype = i32
        L.so_pair_terms.argtypes = [vp, i64, i64, vp]
        _lib = L
    return _lib


def make_params(p: dict) -> _Params:
    s = _Params()
    s.dim = int(p["dim"])
    s.visc_form = int(p.get("visc_form", 0))
    s.cont_form = int(p.get("cont_form", 0))
    s.renorm_every = int(p.get("renorm_every", 1))
    for k in ("h", "gamma", "delta_coef", "alpha_s", "c_cfl", "c_force",
              "c_visc", "c_st", "dt_fixed"):
        setattr(s, k, float(p[k]))
    for k in ("gravity", "lo", "hi"):
        arr = getattr(s, k)
        for d in range(3):
            arr[d] = float(p[k][d])
    for d in range(3):
        s.periodic[d] = int(p["periodic"][d])
    npis = len(p.get("piston_a", []))
    if npis > MAX_PISTON:
        raise ValueError("too many piston components")
    s.n_piston = npis
    s.piston_t_end = float(p.get("piston_t_end", 0.0))
    for k in range(npis):
        s.piston_a[k] = p["piston_a"][k]
        s.piston_w[k] = p["piston_w"][k]
        s.piston_phi[k] = p["piston_phi"][k]
    return s


def kernel_w(dim, h, r):
    return lib().so_kernel_w(dim, h, r)


def kernel_f(dim, h, r):
    return lib().so_kernel_f(dim, h, r)


def eos(rho, rho0, c0, gamma=7.0):
    return lib().so_eos(rho, rho0, c0, gamma)


def piston(params: dict, t: float):
    d, v = C.c_double(), C.c_double()
    lib().so_piston(C.byref(make_params(params)), t, C.byref(d), C.byref(v))
    return d.value, v.value


def set_threads(n: int):
    lib().so_set_threads(int(n))


def get_threads() -> int:
    return int(lib().so_get_threads())


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """One instance of the FP64 oracle, holding its own copy of the state."""

    def __init__(self, scene, inst: int = 0):
        if scene.ninst != 1:
            scene = scene.instance(inst)
        self.scene = scene
        self.n = scene.n
        self.dim = scene.dim
        self._p = make_params(scene.params[0])
        phs = scene.phases[0]
        arr = (_Phase * len(phs))()
        for k, (r0, nu, c0) in enumerate(phs):
            arr[k].rho0, arr[k].nu, arr[k].c0 = r0, nu, c0
        self._keep = [np.ascontiguousarray(a) for a in (
            scene.x.astype(np.float64), scene.u.astype(np.float64),
            scene.rho.astype(np.float64), scene.m.astype(np.float64),
            scene.phase.astype(np.uint8), scene.kind.astype(np.uint8))]
        self.ctx = lib().so_create(C.byref(self._p), arr, len(phs), self.n,
                                   *[_ptr(a) for a in self._keep])
        if not self.ctx:
            raise ValueError("so_create rejected the scene")

    def __del__(self):
        if getattr(self, "ctx", None):
            lib().so_destroy(self.ctx)
            self.ctx = None

    def set_neighbor_method(self, method: int):
        lib().so_set_neighbor_method(self.ctx, int(method))

    def neighbors(self):
        off = np.zeros(self.n + 1, np.int64)
        total = lib().so_neighbors(self.ctx, _ptr(off), None, 0)
        idx = np.zeros(max(total, 1), np.int32)
        lib().so_neighbors(self.ctx, _ptr(off), _ptr(idx), total)
        return off, idx[:total]

    def renormalize(self):
        lib().so_renormalize(self.ctx)

    def rates(self) -> int:
        return int(lib().so_rates(self.ctx))

    def dt(self) -> float:
        return float(lib().so_dt(self.ctx))

    def step(self, nsteps: int = 1) -> int:
        return int(lib().so_step(self.ctx, int(nsteps)))

    def set_moving(self, disp, vel):
        """MOVING particles at x0 + disp + vel (t - t_now) from now on."""
        dv = np.ascontiguousarray(disp, np.float64).reshape(3)
        vv = np.ascontiguousarray(vel, np.float64).reshape(3)
        lib().so_set_moving(self.ctx, _ptr(dv), _ptr(vv))

    @property
    def t(self) -> float:
        return float(lib().so_time(self.ctx))

    @property
    def nstep(self) -> int:
        return int(lib().so_stepcount(self.ctx))

    def get(self, field: int) -> np.ndarray:
        if field == TENSOR:
            out = np.zeros((self.n, 3, 3))
        elif field in _VEC:
            out = np.zeros((self.n, 3))
        else:
            out = np.zeros(self.n)
        if lib().so_get(self.ctx, field, _ptr(out)) != 0:
            raise ValueError(field)
        return out

    def set(self, field: int, values):
        a = np.ascontiguousarray(values, dtype=np.float64)
        if lib().so_set(self.ctx, field, _ptr(a)) != 0:
            raise ValueError(field)

    def pair_terms(self, i: int, j: int):
        out = np.zeros(10)
        if lib().so_pair_terms(self.ctx, int(i), int(j), _ptr(out)) != 0:
            return None
        return out
