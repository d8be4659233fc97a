"""Structured test fields (inputs only: no evolution arithmetic).

Arrays use numpy shape reversed from the lattice shape, i.e. (ny, nx) in 2D
and (nz, ny, nx) in 3D, so that C order is the site order x-fastest.
"""
import math

import numpy as np


def coords(shape):
    """Integer coordinate grids (x, y[, z]) in numpy layout."""
    grids = np.meshgrid(*[np.arange(n) for n in reversed(shape)], indexing="ij")
    return list(reversed(grids))


def kink_pair(shape, W0, x1=None, x2=None):
    """Static wall pair along x: tanh(pi(x-x1)/W0) * tanh(pi(x2-x)/W0),
    uniform in the other directions.  Defaults x1 = N/4 - 1/2, x2 = 3N/4 - 1/2
    keep the profile exactly antisymmetric about both crossings."""
    nx = shape[0]
    x1 = nx / 4.0 - 0.5 if x1 is None else x1
    x2 = 3.0 * nx / 4.0 - 0.5 if x2 is None else x2
    x = coords(shape)[0].astype(np.float64)
    return np.tanh(math.pi * (x - x1) / W0) * np.tanh(math.pi * (x2 - x) / W0)


def cosine_mode(shape, ks, base=0.0, eps=1.0, dx=1.0):
    """base + eps * cos(sum_d k_d x_d dx) with integer wave numbers ks
    (k_d = 2 pi ks[d] / n_d)."""
    cs = coords(shape)
    phase = np.zeros(cs[0].shape)
    for d, kd in enumerate(ks):
        phase = phase + 2.0 * math.pi * kd * cs[d] / shape[d]
    return base + eps * np.cos(phase)


def signs_to_field(bits, shape):
    """+1/-1 field from a bit pattern (bit i set -> +1 at site i)."""
    n = int(np.prod(shape))
    v = np.array([1.0 if (bits >> i) & 1 else -1.0 for i in range(n)])
    return v.reshape(tuple(reversed(shape)))
