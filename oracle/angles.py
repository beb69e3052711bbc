"""The 24-direction A4 angle set (oracle; test infrastructure only).

Sect. 3 names the A4 set of Carlson (1963) but does not print it.  Reading used:
the level-symmetric S4 construction.  In each octant the three permutations of
(mu1, mu1, mu2) with mu1 = 1/3 and mu2 = sqrt(1 - 2 mu1^2) = sqrt(7)/3, signs over
the 8 octants, all weights 1/24.
"""
from __future__ import annotations

import itertools

import numpy as np


def a4_directions():
    """(mu, w): mu of shape (24, 3) as unit vectors (x, y, z), weights of shape (24,).

    Ordered: the 12 upward directions (mu_z > 0) first, then their 12 reflections
    through the origin in the same order.
    """
    m1 = 1.0 / 3.0
    m2 = np.sqrt(1.0 - 2.0 * m1 * m1)
    base = [(m1, m1, m2), (m1, m2, m1), (m2, m1, m1)]
    up = []
    for sx, sy in itertools.product((1.0, -1.0), repeat=2):
        for b in base:
            up.append((sx * b[0], sy * b[1], b[2]))
    up = np.array(up)
    mu = np.concatenate([up, -up], axis=0)
    w = np.full(24, 1.0 / 24.0)
    return mu, w
