"""Discrete velocity sets.

Sec. II C (phase-space discretization): velocities c_i with components c_ia in {-1, 0, 1},
the nearest-neighbour D3Q27 lattice in three dimensions; lattice speed of sound
varsigma = c / sqrt(3) with c = 1. The two-dimensional D2Q9 set is the restriction of the
same construction to the axes x and y (the product form is per axis).

Ordering (a reading, not fixed by the paper): i = (c_x+1) + 3 (c_y+1) [+ 9 (c_z+1)], so that
the opposite direction of i is Q-1-i.
"""
import itertools

import numpy as np

VARSIGMA2 = 1.0 / 3.0  # varsigma^2 = c^2/3, Sec. II C


def velocities(D):
    """Return c with shape (Q, D), Q = 3**D, in the ordering of the module docstring."""
    Q = 3 ** D
    c = np.zeros((Q, D), dtype=np.int64)
    for i in range(Q):
        r = i
        for a in range(D):
            c[i, a] = r % 3 - 1
            r //= 3
    return c


def opposite(D):
    """Index of -c_i for every i, found by search (not by the Q-1-i shortcut)."""
    c = velocities(D)
    opp = np.empty(len(c), dtype=np.int64)
    for i, ci in enumerate(c):
        for j, cj in enumerate(c):
            if np.all(cj == -ci):
                opp[i] = j
    return opp


def all_velocity_tuples(D):
    """Every element of {-1,0,1}^D, for set-equality checks."""
    return set(itertools.product((-1, 0, 1), repeat=D))
