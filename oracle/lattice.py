"""D2Q9 and D3Q19 velocity sets.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3 (Fig. 1 and its caption) and Sec. 3.1: the velocities are xi * c with
c in {-1, 0, 1}^d; D3Q19 drops the eight corners, keeping |c1|+|c2|+|c3| <= 2.
The paper leaves the enumeration order open.  The order used here is the one
the library's public header documents (rest, then the axis pairs, then the
diagonal pairs, each pair being a velocity followed by its opposite), so that
fields can be compared index by index.  The tests check separately that the
set equals the definition above.
"""
import numpy as np

_D2Q9 = [
    (0, 0),
    (1, 0), (-1, 0), (0, 1), (0, -1),
    (1, 1), (-1, -1), (1, -1), (-1, 1),
]

_D3Q19 = [
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
]


def velocities(d):
    """Integer velocity set c_i, shape [Q, d], components ordered (x, y[, z])."""
    if d == 2:
        return np.array(_D2Q9, dtype=np.int64)
    if d == 3:
        return np.array(_D3Q19, dtype=np.int64)
    raise ValueError("d must be 2 or 3")


def velocity_class(c):
    """Number of nonzero components of each velocity (selects its weight)."""
    return np.count_nonzero(c, axis=1)


def opposite(c):
    """Index of -c_i for every i."""
    out = np.empty(len(c), dtype=np.int64)
    for i, ci in enumerate(c):
        (j,) = np.nonzero((c == -ci).all(axis=1))[0]
        out[i] = j
    return out
