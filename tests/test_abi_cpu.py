"""C-ABI checks that need no GPU: the library loads, exports every declared
entry point, sizes workspaces and rejects bad arguments before touching a device."""
import ctypes as C

import numpy as np
import pytest

from paper_1702_07760_amd import binding, inputs


def test_library_exports_every_header_symbol():
    L = binding.lib()
    names = binding.header_functions()
    assert len(names) >= 19
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def _header_structs():
    """Field (name, C type, array length) lists of the header's typedef structs."""
    import os
    import re
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sphx.h")
    text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    macros = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(\w+)\s+(\d+)", text)}
    out = {}
    for m in re.finditer(r"typedef struct\s*\{(.*?)\}\s*(\w+);", text, flags=re.S):
        fields = []
        for decl in filter(None, (d.strip() for d in m.group(1).split(";"))):
            ctype, rest = decl.split(None, 1)
            for v in rest.split(","):
                f = re.match(r"(\w+)(?:\[(\w+)\])?$", v.strip())
                n = f.group(2)
                fields.append((f.group(1), ctype, None if n is None else int(macros.get(n, n))))
        out[m.group(2)] = fields
    return out


@pytest.mark.parametrize("cname,cls", [("sphx_params", binding.Params), ("sphx_phase", binding.Phase),
                                       ("sphx_stats", binding.Stats)])
def test_binding_structs_match_the_header(cname, cls):
    # the ctypes mirrors have the header's fields, in its order, with its types and sizes
    ctypes_of = {"int32_t": C.c_int32, "int64_t": C.c_int64, "double": C.c_double}
    want = _header_structs()[cname]
    got = cls._fields_
    assert [f[0] for f in got] == [w[0] for w in want]
    for (name, ct), (_, ctype, n) in zip(got, want):
        base = ctypes_of[ctype]
        assert ct == (base if n is None else base * n), name


def test_workspace_size_scales_with_particles_and_precision():
    s = inputs.drop2d()
    w64 = binding.workspace_size(s, binding.FP64)
    w32 = binding.workspace_size(s, binding.FP32_CELLREL)
    assert w64 > 0 and w32 > 0 and w32 < w64
    big = inputs.concat("two", [s, s])
    assert binding.workspace_size(big, binding.FP64) > w64


def _create(scene, precision=0, mutate=None, nphase=None):
    params, phases, nph, counts = binding._arrays(scene)
    if mutate:
        mutate(params, phases, counts)
    ctx = C.c_void_p()
    st = binding.lib().sphx_create(precision, params, phases, nph if nphase is None else nphase,
                                   scene.ninst, counts.ctypes.data_as(C.c_void_p), None,
                                   C.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("case", ["gamma", "dim", "h", "skin", "phase_rho0", "precision",
                                  "nphase", "count", "count_max", "periodic_small", "lohi"])
def test_create_rejects_bad_arguments(case):
    s = inputs.drop2d()
    prec, nphase = 0, None

    def mut(p, ph, cnt):
        if case == "gamma":
            p[0].gamma = 1.4
        elif case == "dim":
            p[0].dim = 4
        elif case == "h":
            p[0].h = -1.0
        elif case == "skin":
            p[0].skin_coef = 0.0
        elif case == "phase_rho0":
            ph[1].rho0 = 0.0
        elif case == "count":
            cnt[0] = 0
        elif case == "count_max":
            cnt[0] = 1 << 25          # list entries hold 25-bit particle indices
        elif case == "periodic_small":
            p[0].periodic[0] = 1
            p[0].hi[0] = p[0].lo[0] + 4 * p[0].h
        elif case == "lohi":
            p[0].hi[1] = p[0].lo[1]
    if case == "precision":
        prec = 7
    if case == "nphase":
        nphase = 3
    st, ctx = _create(s, prec, mut, nphase)
    assert st == 1 and not ctx.value       # SPHX_E_ARG, no context


def test_workspace_size_rejects_bad_input():
    s = inputs.drop2d()
    params, _, _, counts = binding._arrays(s)
    assert binding.lib().sphx_workspace_size(3, params, 1, counts.ctypes.data_as(C.c_void_p)) == 0
    bad = np.zeros(1, np.int64)
    assert binding.lib().sphx_workspace_size(0, params, 1, bad.ctypes.data_as(C.c_void_p)) == 0


def test_create_without_gpu_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, ctx = _create(inputs.drop2d())
    assert st == 2 and not ctx.value       # SPHX_E_NODEV
    assert b"hipGetDevice" in binding.lib().sphx_last_error(None)   # why, for this thread


def test_create_failure_message_names_the_argument():
    s = inputs.drop2d()
    st, ctx = _create(s, mutate=lambda p, ph, c: setattr(p[0], "gamma", 5.0))
    assert st == 1 and b"gamma must be 7" in binding.lib().sphx_last_error(None)


def test_null_context_calls_are_argument_errors():
    L = binding.lib()
    assert L.sphx_step(None, 1) == 1
    assert L.sphx_sync(None) == 1
    assert L.sphx_compute_forces(None) == 1
    assert L.sphx_bind_static_workspace(None) == 1


def test_binding_constants_match_the_header():
    # status codes and option ids of the binding against the enums of include/sphx.h
    import re
    text = open(binding.HEADER).read()
    codes = {int(v): f"SPHX_{k}" for k, v in re.findall(r"SPHX_(OK|E_[A-Z]+)\s*=\s*(\d+)", text)}
    assert codes == binding.STATUS
    opts = {k: int(v) for k, v in re.findall(r"SPHX_OPT_([A-Z_]+)\s*=\s*(\d+)", text)}
    assert opts and all(getattr(binding, f"OPT_{k}") == v for k, v in opts.items())
