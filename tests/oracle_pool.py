"""The oracle's direction sums spread over forked worker processes (test infrastructure).

The oracle's formal solution and profile normalisation are sums over the 24 A4
directions; for grids where one process would take minutes, the directions are dealt
to forked workers, each computing its partial sums with the oracle's own functions, and
the parent adds them.  Only the order of that final addition differs from the serial
oracle (rounding at the 1e-16 level).  ``pooled(levels)`` installs the pooled formal
solution in the oracle's solver for the duration of a ``with`` block.
"""
from __future__ import annotations

import contextlib
import multiprocessing as mp
import os

import numpy as np

from oracle import formal as oformal
from oracle import solver as osolver

_STATE = {}


def workers():
    return max(1, min(16, os.cpu_count() or 1))


def _norm_part(dirs):
    return _STATE["lev"].norm_sum(dirs)


def _fs_part(dirs):
    return oformal.formal_solution(_STATE["lev"], _STATE["n"], dirs=dirs)


def _chunks(w):
    return [tuple(range(24))[i::w] for i in range(w)]


def _map(fn, w):
    with mp.get_context("fork").Pool(w) as pool:
        return pool.map(fn, _chunks(w))


def pooled_norm(lev, w=None):
    """Fill lev's profile normalisation from partial sums computed in parallel."""
    if lev._norm is None:
        w = w or workers()
        _STATE["lev"] = lev
        parts = _map(_norm_part, w)
        lev._norm = 1.0 / np.sum(parts, axis=0)
    return lev._norm


def pooled_formal_solution(lev, n, want_jbar=False, dirs=None):
    """(Jeff, 1 - L*) of the oracle, its direction sums computed by forked workers."""
    assert not want_jbar and dirs is None
    w = workers()
    pooled_norm(lev, w)
    _STATE["lev"], _STATE["n"] = lev, n
    parts = _map(_fs_part, w)
    return np.sum([p[0] for p in parts], axis=0), np.sum([p[1] for p in parts], axis=0)


@contextlib.contextmanager
def pooled():
    """Route the oracle solver's formal solutions through the worker pool."""
    saved = osolver.formal_solution
    osolver.formal_solution = pooled_formal_solution
    try:
        yield
    finally:
        osolver.formal_solution = saved
