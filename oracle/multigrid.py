"""Multigrid V-cycle, as an inner preconditioner P_1 ~ S_1 or P_K ~ K_m.

TEST INFRASTRUCTURE ONLY (see the package header).

Sec. 5.3 leaves P_1 and P_K free: any classical preconditioner of the
elliptic or parabolic block fits the block-LU framework of Def. 2, and the
paper names multigrid among them.  This module applies one symmetric
V-cycle from its definition, for a given hierarchy: level matrices A_l,
prolongations P_l (A_{l+1} = P_l^T A_l P_l), smoother data (D_l^-1 and the
interval [lo_l, hi_l] of D_l^-1 A_l) and the number m of smoother steps
(one count for all levels, or one per level).

With the smoother S_l = q_l(D_l^-1 A_l) D_l^-1, q_l the Chebyshev
polynomial of `chebyshev.q_polynomial` on [lo_l, hi_l], one cycle on level l
maps b to
    x1 = S_l b
    x2 = x1 + P_l B_{l+1} P_l^T (b - A_l x1)
    x  = x2 + S_l (b - A_l x2)
and the coarsest level is solved exactly (a dense solve of its matrix).  The
error propagator is then E_l = I - B_l A_l = (I - S_l A_l)(I - P_l B_{l+1}
P_l^T A_l)(I - S_l A_l).  Vertices with D^-1 = 0 (a grounded vertex) are
held at zero: the coarsest solve runs on the others only.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import chebyshev


def smooth(A, dinv, lo, hi, m, b):
    """x = q(D^-1 A) D^-1 b, the polynomial q from its closed form (Horner)."""
    c = chebyshev.q_polynomial(lo, hi, m)
    v = dinv * b
    x = c[-1] * v
    for j in range(m - 2, -1, -1):
        x = dinv * (A @ x) + c[j] * v
    return x


def coarse_solve(A, b, keep=None):
    """Dense solve of A x = b on the vertices in `keep` (the others stay 0)."""
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    n = Ad.shape[0]
    keep = np.ones(n, bool) if keep is None else keep
    x = np.zeros(n)
    x[keep] = sla.solve(Ad[np.ix_(keep, keep)], b[keep], assume_a="pos")
    return x


def vcycle(levels, m, b, level=0):
    """One V-cycle x = B b.  levels[l] = dict(A, P, dinv, lo, hi[, steps]);
    the last level has P = None and is solved exactly.  A level's smoother
    takes its own step count `steps` when given, else m.  On the finest level
    the vertices with D^-1 = 0 are held at zero."""
    L = levels[level]
    A = L["A"]
    if L["P"] is None:
        return coarse_solve(A, b, L["dinv"] != 0.0 if level == 0 else None)
    P = L["P"]
    ml = L.get("steps", m)
    x1 = smooth(A, L["dinv"], L["lo"], L["hi"], ml, b)
    e = vcycle(levels, m, P.T @ (b - A @ x1), level + 1)
    x2 = x1 + P @ e
    return x2 + smooth(A, L["dinv"], L["lo"], L["hi"], ml, b - A @ x2)
