"""Independent reference solutions used to pin the oracle (test helper, CPU only).

``exact_two_level_column`` solves the discretised two-level problem without
background directly: for a horizontally homogeneous atmosphere the source function
obeys S = (1 - eps)(L S + J_bc) + eps B, a linear system once the opacity is fixed.
The operator L is built column by column by sweeping a unit source function on one
plane at a time (brute force), and an outer fixed point updates the opacity from the
populations implied by S.  None of the oracle's MALI, rate-solve or multigrid code is
used; only its single-direction sweep and its profile are.

For a horizontally homogeneous, static column every direction with the same mu_z
gives the same plane-averaged intensity, so the helper sweeps one representative
per distinct mu_z and weights it by the number of directions that share it.
"""
import numpy as np

from oracle.formal import sweep
from oracle.levels import Level


def two_level_pops_from_S(lev, S):
    A, B12, B21 = lev.einstein[0]
    r = S * B12 / (A + S * B21)          # n2 / n1
    n1 = lev.ntot / (1.0 + r)
    return np.stack([n1, r * n1])


def _direction_classes(lev):
    mz = np.round(lev.mu[:, 2], 12)
    classes = []
    for v in np.unique(mz):
        idx = np.nonzero(mz == v)[0]
        classes.append((lev.mu[idx[0]], lev.wmu[idx].sum()))
    return classes


def column_operator(lev, n):
    """(L, J_bc): plane-to-plane mean-intensity operator of a homogeneous static column
    and the boundary contribution, for opacity from populations n."""
    assert np.all(lev.v == 0.0)
    kk, _ = lev.line_coefficients(n)
    norm = lev.norm()
    nz = lev.nz
    L = np.zeros((nz, nz))
    Jbc = np.zeros(nz)
    for mu, wsum in _direction_classes(lev):
        def local(k, mu=mu, wsum=wsum):
            phi = lev.profile(k, mu)[:, :1, :1]
            chi = kk[0, k, :1, :1][None] * phi
            S = np.zeros((nz + 1,) + chi.shape)
            S[k] = 1.0                            # batch b < nz: unit S on plane b
            wphi = wsum * lev.wnu[:, None, None] * phi * norm[0, k, :1, :1][None]
            return np.broadcast_to(chi, S.shape), S, wphi

        def bnd(k, mu=mu):
            I = np.zeros((nz + 1, lev.nf, 1, 1))
            if mu[2] > 0:
                I[nz] = lev.B[0, k, 0, 0]         # batch nz: boundary only, S = 0
            return I

        def acc(k, kind, data):
            if kind == "bc":
                I, wphi = data
            else:
                I, wphi = data[5], data[8]
            vals = (wphi[None] * I).sum(axis=1)[:, 0, 0]
            L[k, :] += vals[:nz]
            Jbc[k] += vals[nz]

        sweep(lev, mu, local, bnd, acc)
    return L, Jbc


def exact_two_level_column(atom, atmos, outer=60, tol=1e-14):
    lev = Level(atom, atmos)
    eps = atom["epsilon"]
    B = lev.B[0, :, 0, 0]
    S = B.copy()
    for _ in range(outer):
        n = two_level_pops_from_S(lev, np.broadcast_to(S[:, None, None], lev.T.shape))
        L, Jbc = column_operator(lev, n)
        S_new = np.linalg.solve(np.eye(lev.nz) - (1 - eps) * L, (1 - eps) * Jbc + eps * B)
        done = np.max(np.abs(S_new / S - 1.0)) < tol
        S = S_new
        if done:
            break
    n = two_level_pops_from_S(lev, np.broadcast_to(S[:, None, None], lev.T.shape))
    return S, n, lev
