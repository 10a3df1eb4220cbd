"""CPU replay, in FP32, of the update sequences the compensated-integration GPU tests
check (``tests/test_gpu_kahan.py``): the same increments, the same compensated sum
(s, e) -> (t, yy - (t - s)) with yy = y + e, and the same re-celling of an offset
(TwoSum of o - sh s, plus the part of the cell size FP32 drops).  The compensated
replay stays within the GPU tests' bounds; the same sequence with plain FP32
additions misses them by more than a factor of 100.  That is what makes the GPU
bounds a test of the compensation rather than of FP32 itself.
"""
import numpy as np

import kahan_cases as K

f32 = np.float32


def _accumulate(s, y, n, kahan, cs=None, recell_every=4):
    """n steps of s += y (FP32 arrays); returns the represented value in FP64 (with the
    cell count times cs when cs is given)."""
    s = s.astype(f32)
    e = np.zeros_like(s)
    cells = np.zeros(s.shape, np.float64)
    y = y.astype(f32)
    if cs is not None:
        cs_f = f32(cs)
        cs_lo = f32(cs - float(cs_f))
    for k in range(n):
        if kahan:
            yy = (y + e).astype(f32)
            t = (s + yy).astype(f32)
            e = (yy - (t - s).astype(f32)).astype(f32)
            s = t
        else:
            s = (s + y).astype(f32)
        if cs is not None and k % recell_every == recell_every - 1:
            sh = np.floor(s / cs_f).astype(f32)
            b = (-sh * cs_f).astype(f32)
            sm = (s + b).astype(f32)
            if kahan:
                bv = (sm - s).astype(f32)
                err = ((s - (sm - bv).astype(f32)).astype(f32) + (b - bv).astype(f32)).astype(f32)
                e = (e + (err - (sh * cs_lo).astype(f32)).astype(f32)).astype(f32)
            s = sm
            cells += sh
    out = s.astype(np.float64) + e.astype(np.float64)
    if cs is not None:
        out += cells * cs
    return out


def _errors(start, step, bound_of, cs=None, n=K.NSTEPS):
    want = start + n * step.astype(np.float64)
    res = {}
    for kahan in (True, False):
        got = _accumulate(np.asarray(start, f32), step, n, kahan, cs)
        res[kahan] = float(np.abs(got - want).max())
    return res, bound_of(want)


def test_position_bound_needs_compensation():
    cs = K.cell_size()
    start = np.array([0.011, 0.0043, 0.017])     # offsets inside the first cell
    step = (f32(K.DT) * K.U0.astype(f32)).astype(f32)
    res, bound = _errors(start, step, lambda w: 4 * float(np.spacing(f32(cs))), cs=cs)
    assert res[True] <= bound
    assert res[False] > 100 * bound, res


def test_velocity_bound_needs_compensation():
    step = (f32(K.DT) * K.G0.astype(f32)).astype(f32)
    res, bound = _errors(K.U0, step, lambda w: 4 * float(np.spacing(f32(np.abs(w).max()))))
    assert res[True] <= bound
    assert res[False] > 100 * bound, res


def test_density_bound_needs_compensation():
    rate = np.float32([26.3, -17.9, 3.1])          # density rates of the size the GPU case has
    step = (f32(K.DT) * rate).astype(f32)
    res, bound = _errors(np.zeros(3), step, lambda w: 4 * float(np.spacing(f32(np.abs(w).max()))))
    assert res[True] <= bound
    assert res[False] > 100 * bound, res
