"""Python binding of the sphx C ABI (``include/sphx.h``).

Argument marshalling only: every step of the particle loop runs in the gfx950
kernels of ``libsphx.so``.  PyTorch provides the device workspace and the HIP
stream.  There is no fallback: without the built library, or without an
MI355X, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsphx.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "sphx.h")

FP64, FP32_CELLREL = 0, 1
MAX_PISTON = 16
F_X, F_U, F_RHO, F_A, F_DRHO, F_AP, F_AV, F_AS, F_P, F_GRADC = 0, 1, 2, 3, 4, 5, 6, 7, 12, 13
_VEC = {F_X, F_U, F_A, F_AP, F_AV, F_AS, F_GRADC}
OPT_DEBUG_TERMS, OPT_BLOCK, OPT_XCD_REMAP, OPT_GRAPH, OPT_LANES, OPT_PROFILE = 1, 2, 3, 4, 5, 6
OPT_FORCE_LANES = 7
OPT_ONE_LAUNCH_BUILD = 8
OPT_FORCE_STALL = 9
OPT_COLOUR_IN_PREDICT = 10
PHASES = ("build", "renorm", "colour", "force", "integrate")
STATUS = {0: "SPHX_OK", 1: "SPHX_E_ARG", 2: "SPHX_E_NODEV", 3: "SPHX_E_HIP", 4: "SPHX_E_WORKSPACE",
          5: "SPHX_E_STATE", 6: "SPHX_E_NONFINITE", 7: "SPHX_E_DOMAIN", 8: "SPHX_E_DT", 9: "SPHX_E_STALL"}


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("visc_form", C.c_int32), ("cont_form", C.c_int32),
        ("renorm_every", C.c_int32),
        ("h", C.c_double), ("gamma", C.c_double), ("delta_coef", C.c_double),
        ("alpha_s", C.c_double),
        ("gravity", C.c_double * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("periodic", C.c_int32 * 3),
        ("skin_coef", C.c_double), ("c_cfl", C.c_double), ("c_force", C.c_double),
        ("c_visc", C.c_double), ("c_st", C.c_double), ("dt_fixed", C.c_double),
        ("n_piston", C.c_int32), ("piston_t_end", C.c_double),
        ("piston_a", C.c_double * MAX_PISTON), ("piston_w", C.c_double * MAX_PISTON),
        ("piston_phi", C.c_double * MAX_PISTON),
    ]


class Phase(C.Structure):
    _fields_ = [("rho0", C.c_double), ("nu", C.c_double), ("c0", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("t", C.c_double), ("dt", C.c_double),
                ("interactions", C.c_int64), ("ncells", C.c_int64), ("builds", C.c_int64),
                ("phase_ms", C.c_double * 5), ("phase_launches", C.c_int64 * 5),
                ("colour_particles", C.c_int64), ("two_level_builds", C.c_int64)]


class SphxError(RuntimeError):
    def __init__(self, code, where, msg=""):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} {msg}".strip())


_lib = None


def lib():
    """Load ``libsphx.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH}; run __graft_entry__.build()")
        # torch first: its HIP runtime carries the same soname as the system one that
        # libsphx.so names, so the library then binds to the runtime torch uses.  Loaded
        # the other way round, the process would hold two HIP runtimes, and the second
        # to start finds no device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
        sig = {
            "sphx_workspace_size": (sz, [i32, vp, i32, vp]),
            "sphx_create": (i32, [i32, vp, vp, i32, i32, vp, vp, C.POINTER(vp)]),
            "sphx_destroy": (None, [vp]),
            "sphx_last_error": (C.c_char_p, [vp]),
            "sphx_bind_workspace": (i32, [vp, vp, sz]),
            "sphx_bind_static_workspace": (i32, [vp]),
            "sphx_init_particles": (i32, [vp] + [vp] * 6),
            "sphx_build_neighbors": (i32, [vp]),
            "sphx_renormalize_density": (i32, [vp]),
            "sphx_compute_forces": (i32, [vp]),
            "sphx_integrate_step": (i32, [vp, d]),
            "sphx_step": (i32, [vp, i32]),
            "sphx_set_option": (i32, [vp, i32, i64]),
            "sphx_get_option": (i32, [vp, i32, C.POINTER(i64)]),
            "sphx_set_moving": (i32, [vp, i32, vp, vp]),
            "sphx_sync": (i32, [vp]),
            "sphx_get_stats": (i32, [vp, C.POINTER(Stats)]),
            "sphx_reset_interactions": (i32, [vp]),
            "sphx_get_field": (i32, [vp, i32, vp]),
            "sphx_get_neighbors": (i32, [vp, vp, vp, i64, C.POINTER(i64)]),
            "sphx_get_state": (i32, [vp, vp, sz, C.POINTER(sz)]),
            "sphx_set_state": (i32, [vp, vp, sz]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions():
    """Names of every function the public header declares."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sphx_[a-z_]+)\s*\(", text)))


def make_params(p: dict) -> Params:
    s = Params()
    s.dim = int(p["dim"])
    s.visc_form = int(p.get("visc_form", 0))
    s.cont_form = int(p.get("cont_form", 0))
    s.renorm_every = int(p.get("renorm_every", 1))
    for k in ("h", "gamma", "delta_coef", "alpha_s", "skin_coef", "c_cfl", "c_force",
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


def _arrays(scene):
    params = (Params * scene.ninst)(*[make_params(p) for p in scene.params])
    nph = len(scene.phases[0])
    phases = (Phase * (scene.ninst * nph))()
    for b, phs in enumerate(scene.phases):
        if len(phs) != nph:
            raise ValueError("every instance needs the same number of phases")
        for q, (r0, nu, c0) in enumerate(phs):
            phases[b * nph + q].rho0, phases[b * nph + q].nu, phases[b * nph + q].c0 = r0, nu, c0
    counts = np.diff(scene.inst_offsets).astype(np.int64)
    return params, phases, nph, counts


def workspace_size(scene, precision=FP64) -> int:
    params, _, _, counts = _arrays(scene)
    return int(lib().sphx_workspace_size(precision, params, scene.ninst,
                                         counts.ctypes.data_as(C.c_void_p)))


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Sim:
    """One sphx context on one GPU: the state of every instance of a scene."""

    def __init__(self, scene, precision=FP64, device="cuda:0", graph=True, static_workspace=False,
                 tuned=True):
        import torch
        self.torch = torch
        self.scene = scene
        self.n = scene.n
        self.dim = scene.dim
        self.precision = precision
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)          # default priority
        params, phases, nph, counts = _arrays(scene)
        self._keep = (params, phases, counts)
        ctx = C.c_void_p()
        st = lib().sphx_create(precision, params, phases, nph, scene.ninst,
                               counts.ctypes.data_as(C.c_void_p),
                               C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        if st != 0:
            raise SphxError(st, "sphx_create", (lib().sphx_last_error(None) or b"").decode())
        self.ctx = ctx
        if static_workspace:
            # the library's own per-device workspace: nothing is allocated
            self.ws = None
            self._check(lib().sphx_bind_static_workspace(self.ctx), "sphx_bind_static_workspace")
        else:
            size = lib().sphx_workspace_size(precision, params, scene.ninst,
                                             counts.ctypes.data_as(C.c_void_p))
            with torch.cuda.device(self.device):
                self.ws = torch.empty(size + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            aligned = (base + 255) & ~255
            self._check(lib().sphx_bind_workspace(self.ctx, C.c_void_p(aligned), size),
                        "sphx_bind_workspace")
        if not graph:
            self.set_option(OPT_GRAPH, 0)
        # the autotuner's launch shape for scenes of this kind, when it has one (block
        # size and tile order only: results are bit-identical under any of them)
        self.tuned = None
        if tuned:
            from . import tune
            self.tuned = tune.best_for(scene.dim, scene.n, precision)
            if self.tuned:
                self.set_launch(**self.tuned)
        self.init_particles()

    # -- plumbing
    def _check(self, st, where):
        if st != 0:
            msg = lib().sphx_last_error(self.ctx) if getattr(self, "ctx", None) else b""
            raise SphxError(st, where, (msg or b"").decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            lib().sphx_destroy(self.ctx)
            self.ctx = None
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI, one method per entry point
    def init_particles(self, scene=None):
        """Upload a scene with this context's layout (default: the one it was made for)."""
        scene = self.scene if scene is None else scene
        x = np.ascontiguousarray(scene.x, np.float64)
        u = np.ascontiguousarray(scene.u, np.float64)
        rho = np.ascontiguousarray(scene.rho, np.float64)
        m = np.ascontiguousarray(scene.m, np.float64)
        ph = np.ascontiguousarray(scene.phase, np.uint8)
        kd = np.ascontiguousarray(scene.kind, np.uint8)
        self._check(lib().sphx_init_particles(self.ctx, _ptr(x), _ptr(u), _ptr(rho), _ptr(m),
                                              _ptr(ph), _ptr(kd)), "sphx_init_particles")

    def build_neighbors(self):
        self._check(lib().sphx_build_neighbors(self.ctx), "sphx_build_neighbors")

    def renormalize_density(self):
        self._check(lib().sphx_renormalize_density(self.ctx), "sphx_renormalize_density")

    def compute_forces(self):
        self._check(lib().sphx_compute_forces(self.ctx), "sphx_compute_forces")

    def integrate_step(self, dt: float = 0.0):
        self._check(lib().sphx_integrate_step(self.ctx, float(dt)), "sphx_integrate_step")

    def step(self, nsteps: int = 1):
        self._check(lib().sphx_step(self.ctx, int(nsteps)), "sphx_step")

    def set_moving(self, inst: int, disp, vel):
        dv = np.ascontiguousarray(disp, np.float64).reshape(3)
        vv = np.ascontiguousarray(vel, np.float64).reshape(3)
        self._check(lib().sphx_set_moving(self.ctx, int(inst), _ptr(dv), _ptr(vv)), "sphx_set_moving")

    def set_option(self, opt: int, value: int):
        self._check(lib().sphx_set_option(self.ctx, int(opt), int(value)), "sphx_set_option")

    def get_option(self, opt: int) -> int:
        v = C.c_int64()
        self._check(lib().sphx_get_option(self.ctx, int(opt), C.byref(v)), "sphx_get_option")
        return v.value

    def set_launch(self, block=None, xcd_remap=None, colour_in_predict=None):
        if block is not None:
            self.set_option(OPT_BLOCK, block)
        if xcd_remap is not None:
            self.set_option(OPT_XCD_REMAP, xcd_remap)
        if colour_in_predict is not None:
            self.set_option(OPT_COLOUR_IN_PREDICT, colour_in_predict)

    def launch_options(self) -> dict:
        """The launch shape in use: block size, tile order and where the colour pass at S*
        runs (what the tuner searches), and the lanes per particle of the Eq. (7) and force
        passes."""
        return dict(block=self.get_option(OPT_BLOCK), xcd_remap=self.get_option(OPT_XCD_REMAP),
                    colour_in_predict=self.get_option(OPT_COLOUR_IN_PREDICT),
                    lanes=self.get_option(OPT_LANES), force_lanes=self.get_option(OPT_FORCE_LANES))

    def sync(self):
        self._check(lib().sphx_sync(self.ctx), "sphx_sync")

    def stats(self) -> dict:
        s = Stats()
        self._check(lib().sphx_get_stats(self.ctx, C.byref(s)), "sphx_get_stats")
        return dict(steps=s.steps, t=s.t, dt=s.dt, interactions=s.interactions, ncells=s.ncells,
                    builds=s.builds, colour_particles=s.colour_particles, two_level_builds=s.two_level_builds,
                    phase_ms={k: s.phase_ms[q] for q, k in enumerate(PHASES)},
                    phase_launches={k: s.phase_launches[q] for q, k in enumerate(PHASES)})

    def reset_interactions(self):
        self._check(lib().sphx_reset_interactions(self.ctx), "sphx_reset_interactions")

    def get_field(self, field: int) -> np.ndarray:
        out = np.zeros((self.n, 3)) if field in _VEC else np.zeros(self.n)
        self._check(lib().sphx_get_field(self.ctx, int(field), _ptr(out)), "sphx_get_field")
        return out

    def get_neighbors(self):
        off = np.zeros(self.n + 1, np.int64)
        need = C.c_int64()
        self._check(lib().sphx_get_neighbors(self.ctx, _ptr(off), None, 0, C.byref(need)),
                    "sphx_get_neighbors")
        ids = np.zeros(max(need.value, 1), np.int32)
        self._check(lib().sphx_get_neighbors(self.ctx, _ptr(off), _ptr(ids), need.value,
                                             C.byref(need)), "sphx_get_neighbors")
        return off, ids[:need.value]

    def get_state(self) -> bytes:
        need = C.c_size_t()
        self._check(lib().sphx_get_state(self.ctx, None, 0, C.byref(need)), "sphx_get_state")
        buf = C.create_string_buffer(need.value)
        self._check(lib().sphx_get_state(self.ctx, buf, need.value, C.byref(need)),
                    "sphx_get_state")
        return buf.raw

    def set_state(self, blob: bytes):
        self._check(lib().sphx_set_state(self.ctx, blob, len(blob)), "sphx_set_state")
