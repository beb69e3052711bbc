"""Statistical equilibrium with the particle-conservation closure (oracle; test only).

Eq. (2): n_i sum_j P_ij - sum_j n_j P_ji = 0 with P the sum of radiative and
collisional rates; Eq. (3)/(5): the first rate equation (ground level, row 0) is
replaced by sum_i n_i = n_tot, so the right-hand side is f = [n_tot, 0, ..., 0].

Radiative rates use the preconditioned form of Rybicki & Hummer (1991) with a
diagonal operator (Sect. 2.1): for line i -> j
    upward   P_ij += B_ij Jeff
    downward P_ji += A_ji (1 - L*) + B_ji Jeff
so the net radiative term n_j A_ji - (n_i B_ij - n_j B_ji) Jbar with
Jbar = Jeff + L* S_l is linear in the new populations.  Built from a formal solution
at populations n, the same matrix applied to n gives W(n) (Eq. 4; Eq. 7 with the
"extra" formal solution at n), because (n_i B_ij - n_j B_ji) S_l = n_j A_ji.

Zero-radiation initialisation (Sect. 4.11): Jeff = 0 and 1 - L* = 1 (spontaneous
emission kept, fixed bound-free rates kept; active continua keep only their spontaneous
recombination F_t).
"""
from __future__ import annotations

import numpy as np


def rate_matrix(lev, Jeff, omL, cont=None):
    """P[i, j] (rate coefficient i -> j) per voxel, shape (N, N, nz, ny, nx).

    Active continua (cont = (U, G, L_.,0, ...) from formal.continuum_formal_solution, or
    None for no radiation) add upward U_t and downward G_t + F_t - L_t,c, c the continuum's
    own upper level; the terms in the populations of other upper levels are cross_terms()."""
    P = lev.fixed.copy()
    for l in range(lev.nline):
        Aji, Bij, Bji = lev.einstein[l]
        i, j = lev.lower[l], lev.upper[l]
        P[i, j] += Bij * Jeff[l]
        P[j, i] += Aji * omL[l] + Bji * Jeff[l]
    if getattr(lev, "active_continua", False):
        for t in range(lev.ncont):
            i, c = lev.cont_lower[t], lev.cont_upper[t]
            P[c, i] += lev.cont_F[t]
            if cont is not None:
                P[i, c] += cont[0, t]
                P[c, i] += cont[1, t] - cont[2 + lev.cont_uidx[t], t]
    return P


def cross_terms(lev, cont):
    """X[i, j] per voxel, shape (N, N, nz, ny, nx), added to the system matrix: the net
    upward rate of continuum t (lower l, upper c) holds n_u L_t,u for every upper level u
    of the continua; for u != c that is a flux l -> c proportional to n_u, which leaves l
    (X[l, u] += L_t,u) and enters c (X[c, u] -= L_t,u).  None when there is nothing to add."""
    if cont is None or not getattr(lev, "active_continua", False) or len(lev.cont_uppers) == 1:
        return None
    X = np.zeros((lev.N, lev.N) + cont.shape[2:])
    for t in range(lev.ncont):
        l, c = lev.cont_lower[t], lev.cont_upper[t]
        for u, lu in enumerate(lev.cont_uppers):
            if lu != c:
                X[l, lu] += cont[2 + u, t]
                X[c, lu] -= cont[2 + u, t]
    return X


def system_matrix(P, X=None):
    """A with A[i,i] = sum_{j!=i} P_ij, A[i,j] = -P_ji, plus X[i, j] if given, and row 0
    replaced by ones.

    Returned with the voxel axis first: shape (nvox, N, N)."""
    N = P.shape[0]
    Pv = P.reshape(N, N, -1)
    A = -np.transpose(Pv, (2, 1, 0)).copy()       # A[v, i, j] = -P[j, i]
    out = Pv.sum(axis=1) - np.einsum("iiv->iv", Pv)  # sum_{j != i} P_ij
    idx = np.arange(N)
    A[:, idx, idx] = out.T
    if X is not None:
        A += np.transpose(X.reshape(N, N, -1), (2, 0, 1))
    A[:, 0, :] = 1.0
    return A


def apply_W(lev, n, Jeff, omL, cont=None):
    """W(n) per level and voxel, shape (N, nz, ny, nx): row 0 = sum n, others stat. eq."""
    A = system_matrix(rate_matrix(lev, Jeff, omL, cont), cross_terms(lev, cont))
    N = n.shape[0]
    nv = n.reshape(N, -1).T
    return np.einsum("vij,vj->vi", A, nv).T.reshape(n.shape)


def solve(lev, Jeff, omL, f, cont=None):
    """Solve A n = f per voxel (LAPACK gesv, partial pivoting) and rescale so that
    sum_i n_i = f_0 exactly."""
    A = system_matrix(rate_matrix(lev, Jeff, omL, cont), cross_terms(lev, cont))
    N = f.shape[0]
    rhs = f.reshape(N, -1).T
    n = np.linalg.solve(A, rhs[..., None])[..., 0]
    n = n * (rhs[:, 0] / n.sum(axis=1))[:, None]
    return n.T.reshape(f.shape)


def fine_rhs(lev):
    """f = [n_tot, 0, ..., 0] (Eq. 5)."""
    f = np.zeros((lev.N,) + lev.ntot.shape)
    f[0] = lev.ntot
    return f


def zero_radiation(lev, f=None):
    """Populations from the rate equations with the radiation field set to zero."""
    shape = (lev.nline, lev.nz, lev.ny, lev.nx)
    return solve(lev, np.zeros(shape), np.ones(shape), fine_rhs(lev) if f is None else f)


def max_rel_change(n_new, n_old):
    """C = max |(n_new - n_old) / n_new| over levels and voxels (Eq. 16)."""
    return float(np.max(np.abs((n_new - n_old) / n_new)))


def source_function(lev, n):
    """Line source functions S_l = e_l / k_l per (line, voxel); NaN where k_l <= 0."""
    S = np.empty((lev.nline,) + n.shape[1:])
    for l in range(lev.nline):
        Aji, Bij, Bji = lev.einstein[l]
        i, j = lev.lower[l], lev.upper[l]
        k = n[i] * Bij - n[j] * Bji
        with np.errstate(divide="ignore", invalid="ignore"):
            S[l] = np.where(k > 0, n[j] * Aji / k, np.nan)
    return S
