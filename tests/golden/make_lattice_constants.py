"""Write lattice_constants.json: sums of the closed-form Wendland C2 kernel
(support 2h, h = 1.3 dx) over an infinite perfect square/cubic lattice, seen
from one lattice site.  Plain numpy over the closed form; it calls neither
the oracle nor the GPU library.

  partition   sum_j V W_ij              (j over all sites, i itself included)
  moment      sum_j V (x_j - x_i) (x) grad_i W_ij  = moment * I
  count       number of sites j != i with |x_i - x_j| < 2h
  m2, m4      kernel-weighted moments sum_j W_ij r_ij^k / sum_j W_ij, k = 2, 4 (i itself
              included, r in units of dx): the weights of Eq. (7) on a lattice
"""
import itertools
import json
import math
import os

import numpy as np

out = {"h_over_dx": 1.3, "note": "lattice sums of the closed-form Wendland C2 kernel"}
for dim in (2, 3):
    h = 1.3
    alpha = 7.0 / (4.0 * math.pi * h * h) if dim == 2 else 21.0 / (16.0 * math.pi * h ** 3)
    pts = np.array(list(itertools.product(range(-4, 5), repeat=dim)), float)
    r = np.sqrt((pts ** 2).sum(1))
    q = r / h
    inside = q < 2.0
    w = np.where(inside, alpha * (1 - q / 2) ** 4 * (2 * q + 1), 0.0)
    f = np.where(inside, -5.0 * alpha / h ** 2 * (1 - q / 2) ** 3, 0.0)
    grad = f[:, None] * (-pts)                    # r_ij = x_i - x_j = -pts
    mom = np.einsum("ja,jb->ab", pts, grad)
    out[f"{dim}d"] = {"partition": float(w.sum()), "moment": float(mom[0, 0]),
                      "count": int((inside & (r > 0)).sum()),
                      "m2": float((w * r ** 2).sum() / w.sum()),
                      "m4": float((w * r ** 4).sum() / w.sum())}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "lattice_constants.json"), "w") as fh:
    json.dump(out, fh, indent=1)
print(out)
