"""Error norms for comparing the GPU library with the FP64 oracle.

A rate f_i = sum_j t_ij is compared with the condition-aware E-norm
    e_f = max_i |f_i - f*_i| / max_i sum_j |t*_ij|
(the oracle's sum of absolute pair terms), which stays meaningful where the
terms cancel, as in hydrostatic balance.  Vectors use the Euclidean norm.
"""
import numpy as np


def enorm(f, fref, scale):
    f, fref = np.asarray(f), np.asarray(fref)
    diff = np.linalg.norm(f - fref, axis=1) if f.ndim == 2 else np.abs(f - fref)
    s = float(np.max(scale))
    return float(diff.max() / s) if s > 0 else float(diff.max())


def rel_to(f, fref, ref_scale):
    f, fref = np.asarray(f), np.asarray(fref)
    diff = np.linalg.norm(f - fref, axis=1) if f.ndim == 2 else np.abs(f - fref)
    return float(diff.max() / ref_scale)


def same_neighbours(off_a, ids_a, off_b, ids_b):
    return np.array_equal(off_a, off_b) and np.array_equal(ids_a, ids_b)
