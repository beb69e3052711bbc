"""MALI iteration, FAS V-cycle and full multigrid (oracle; test infrastructure only).

Follows Sect. 2.2 and 2.3 of the paper in its order and notation:

* MALI iteration (Sect. 2.1): a formal solution at the current populations, then the
  preconditioned rate equations solved per voxel with right-hand side f.
* Two-grid FAS step (Eqs. 6-12): nu_1 pre-smoothing iterations; the residual
  r^k = f^k - W*(n^k) with an extra formal solution at n^k (Eq. 7); restriction of n^k
  and r^k; the coarse right-hand side f^{k-1} = R r^k + W*(R n^k) (Eq. 10); nu_3 MALI
  iterations on the coarsest grid (or, recursively, a V-cycle on grid k-1 if it is
  not the coarsest); the relative correction e = (n_after - n_before) / n_before
  (Eq. 11) interpolated and applied as n_new = n_old (1 + I e) (Eq. 12); nu_2 post-
  smoothing iterations.
* The formal solution at R n^k that gives W*(R n^k) is the same computation as the
  first coarse iteration's formal solution and is reused (the results are identical).
* Negative-population repair (Sect. 4.10): where n_old (1 + I e) <= 0 the new value is
  10 % of the uncorrected population.
* nu_0 (Sect. 4.12): replaces nu_1 in the first V-cycle's finest-level pre-smoothing;
  nu_0 = 0 means no special first-cycle smoothing.
* Full multigrid (Sect. 2.3): zero-radiation populations of the coarsest level's own
  atmosphere, nu_FMG iterations there with f = [n_tot, 0, ...], then for every finer
  level the full approximation is interpolated (Eq. 14) and one V-cycle is applied on
  every intermediate level; at the finest level regular V-cycles follow.
* Convergence (Sect. 3.3): C_i = max |(n_i - n_{i-1}) / n_i| (Eq. 16) over all levels
  and voxels; for cycles it is taken between successive finest-level cycle ends.  The
  error estimate is E = rho / (1 - rho) C with rho = C_{i}/C_{i-1} (Eq. 18), which holds
  once the corrections are in their asymptotic linear regime; the first correction,
  made from the initial populations, is not, so rho is taken from the second
  correction on (three or more corrections before E is used).
* With a single grid a "cycle" is nu_1 (or nu_0) + nu_2 plain MALI iterations.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .formal import continuum_formal_solution, formal_solution
from .levels import Level, build_hierarchy
from .rates import apply_W, fine_rhs, max_rel_change, solve, zero_radiation
from .transfer import prolong, restrict


@dataclass
class Params:
    nlev: int = 3
    nu0: int = 0
    nu1: int = 2
    nu2: int = 2
    nu3: int = 32
    nu_fmg: int = 16
    repair_frac: float = 0.1
    max_cycles: int = 50
    max_iter: int = 2000
    tol_C: float | None = None
    E_target: float | None = 1.0e-3
    restriction: str = "full"      # populations and residuals (Sect. 4.4)
    interpolation: str = "trilinear"   # corrections and FMG full approximations (Sect. 4.5)
    sc_interp: str = "bilinear"        # upwind interpolation of the formal solution (Sect. 3)
    coarse_atmos: str = "full"     # coarse model atmospheres (Sect. 4.7)


@dataclass
class Stats:
    fs: dict = field(default_factory=dict)          # formal solutions per level index k
    solves: dict = field(default_factory=dict)      # rate solves per level index k
    repairs: int = 0
    C: list = field(default_factory=list)
    E_est: list = field(default_factory=list)

    def count_fs(self, k):
        self.fs[k] = self.fs.get(k, 0) + 1

    def count_solve(self, k):
        self.solves[k] = self.solves.get(k, 0) + 1

    def cost(self, levels):
        """Work in units of one finest-grid formal solution (Sect. 4.9)."""
        nf = levels[-1].nx * levels[-1].ny * levels[-1].nz
        return sum(c * (levels[k - 1].nx * levels[k - 1].ny * levels[k - 1].nz) / nf
                   for k, c in self.fs.items())


def _fs(lev, k, n, stats):
    """(Jeff, 1 - L*, continuum sums or None) of a formal solution at n."""
    if stats is not None:
        stats.count_fs(k)
    Jeff, omL = formal_solution(lev, n)
    cont = continuum_formal_solution(lev, n) if getattr(lev, "active_continua", False) else None
    return Jeff, omL, cont


def mali(lev, k, n, f, iters, stats=None, fs0=None):
    """``iters`` MALI iterations on level k; returns (n, C of the last iteration)."""
    C = None
    for it in range(iters):
        Jeff, omL, cont = fs0 if (it == 0 and fs0 is not None) else _fs(lev, k, n, stats)
        n_new = solve(lev, Jeff, omL, f, cont)
        if stats is not None:
            stats.count_solve(k)
        C = max_rel_change(n_new, n)
        n = n_new
    return n, C


def apply_correction(n_old, Ie, repair_frac):
    """The relative coarse-grid correction with the negative-population repair.

    Eq. 12: n_new = n_old (1 + I e), with I e the relative correction interpolated to
    this grid.  Sect. 4.10: where that value is not positive, the new population is
    ``repair_frac`` (10 %) of the uncorrected one instead (the equality case is repaired
    too, so that later relative corrections stay defined).  Returns (n_new, number of
    repaired entries).
    """
    n_new = n_old * (1.0 + Ie)
    bad = n_new <= 0.0
    n_new[bad] = repair_frac * n_old[bad]
    return n_new, int(np.count_nonzero(bad))


def vcycle(levels, k, n, f, p, first=False, stats=None, fs0=None):
    """One FAS V-cycle on levels k, k-1, ..., 1 with right-hand side f on level k."""
    lev = levels[k - 1]
    nu_pre = p.nu0 if (first and p.nu0 > 0) else p.nu1
    if k == 1:
        n, _ = mali(lev, k, n, f, nu_pre, stats, fs0)
        n, _ = mali(lev, k, n, f, p.nu2, stats)
        return n
    n, _ = mali(lev, k, n, f, nu_pre, stats, fs0)
    fs_n = fs0 if (nu_pre == 0 and fs0 is not None) else _fs(lev, k, n, stats)
    r = f - apply_W(lev, n, *fs_n)
    levc = levels[k - 2]
    nc = restrict(n, p.restriction)
    rc = restrict(r, p.restriction)
    fs_c = _fs(levc, k - 1, nc, stats)
    fc = rc + apply_W(levc, nc, *fs_c)
    n_before = nc.copy()
    if k - 1 == 1:
        nc, _ = mali(levc, k - 1, nc, fc, p.nu3, stats, fs_c)
    else:
        nc = vcycle(levels, k - 1, nc, fc, p, False, stats, fs_c)
    e = (nc - n_before) / n_before
    n, rep = apply_correction(n, prolong(e, lev.z, p.interpolation), p.repair_frac)
    if stats is not None:
        stats.repairs += rep
    n, _ = mali(lev, k, n, f, p.nu2, stats)
    return n


def _converged(hist, p):
    C = hist[-1]
    if p.tol_C is not None and C <= p.tol_C:
        return True
    if p.E_target is not None and len(hist) >= 3:
        rho = hist[-1] / hist[-2]
        if rho < 1.0 and rho / (1.0 - rho) * C <= p.E_target:
            return True
    return False


def _record(stats, hist):
    if len(hist) >= 3 and hist[-1] < hist[-2]:
        rho = hist[-1] / hist[-2]
        stats.E_est.append(rho / (1.0 - rho) * hist[-1])
    else:
        stats.E_est.append(float("inf"))


def solve_mali(atom, atmos, p, stats=None, n0=None, iters=None, top_I=None):
    """Plain MALI from zero-radiation populations until the stop rule (or ``iters``)."""
    stats = stats if stats is not None else Stats()
    lev = Level(atom, atmos, top_I=top_I, sc_interp=p.sc_interp)
    f = fine_rhs(lev)
    n = zero_radiation(lev) if n0 is None else np.array(n0, dtype=np.float64)
    count = iters if iters is not None else p.max_iter
    for _ in range(count):
        n, C = mali(lev, 1, n, f, 1, stats)
        stats.C.append(C)
        _record(stats, stats.C)
        if iters is None and _converged(stats.C, p):
            break
    return n, stats, lev


def solve_fas(atom, atmos, p, fmg=False, stats=None, cycles=None, levels=None):
    """FAS V-cycles (optionally preceded by full multigrid) until the stop rule."""
    stats = stats if stats is not None else Stats()
    levels = levels if levels is not None else build_hierarchy(atom, atmos, p.nlev, coarse_op=p.coarse_atmos,
                                                               sc_interp=p.sc_interp)
    L = len(levels)
    fine = levels[-1]
    f = fine_rhs(fine)
    if fmg:
        lev1 = levels[0]
        n = zero_radiation(lev1)
        n, _ = mali(lev1, 1, n, fine_rhs(lev1), p.nu_fmg, stats)
        for k in range(2, L + 1):
            n = prolong(n, levels[k - 1].z, p.interpolation)
            if k < L:
                n = vcycle(levels, k, n, fine_rhs(levels[k - 1]), p, False, stats)
        first = False
    else:
        n = zero_radiation(fine)
        first = True
    count = cycles if cycles is not None else p.max_cycles
    for _ in range(count):
        n_prev = n
        n = vcycle(levels, L, n, f, p, first, stats)
        first = False
        stats.C.append(max_rel_change(n, n_prev))
        _record(stats, stats.C)
        if cycles is None and _converged(stats.C, p):
            break
    return n, stats, levels
