"""Dense block algebra of Sec. 4 and the preconditioner of Sec. 5 (tiny
meshes only: everything here forms dense matrices).

  Def. 1   pseudo-inverses of S_1 and S_i: the inverse on the orthogonal of
           the constants, zero on the constants
  Prop. 2  Lambda = L U with the Schur complement
           K = gamma M_H + S_i - S_i Pi S_1^+ Pi^T S_i   (SPD)
  Rem. 1   K_0 = K - gamma M_H is the inverse of
           A = S_i^+ + Pi S_e^+ Pi^T on the orthogonal of 1_H
  Prop. 3  X = U^-1 L^+ Y solves Lambda X = Y for Y in the range
  Def. 2   P_Lambda = L_P U_P with preconditioners P_1 ~ S_1, P_K ~ K;
           its inverse applied as
             Z1 = P1^-1 Y1
             Z2 = PK^-1 (Y2 - S_i Pi Z1)
             X1 = Z1 - P1^-1 Pi^T S_i Z2,   X2 = Z2
  Sec. 5.2 monodomain approximation K_m = gamma M_H + S_m
"""
import numpy as np
import scipy.linalg as sla


def pinv_kernel1(S):
    """Pseudo-inverse (Def. 1) of a symmetric PSD matrix whose kernel is the
    constants: (S + e e^T)^-1 - e e^T with e = 1/sqrt(n)."""
    n = S.shape[0]
    e = np.full(n, 1.0 / np.sqrt(n))
    E = np.outer(e, e)
    return np.linalg.inv(S + E) - E


def dense_blocks(sysm):
    """Dense S1, Si, Se, Sm, M_H, Pi from an oracle System (heart-first)."""
    N, NH = sysm.N, sysm.NH
    Pi = np.zeros((NH, N))
    Pi[np.arange(NH), np.arange(NH)] = 1.0
    return dict(S1=sysm.S1.toarray(), Si=sysm.Si.toarray(),
                Se=sysm.Se.toarray(), Sm=sysm.Sm.toarray(),
                MH=np.diag(sysm.mH), Pi=Pi, gamma=sysm.gamma, N=N, NH=NH)


def schur_K(b):
    S1p = pinv_kernel1(b["S1"])
    Si, Pi = b["Si"], b["Pi"]
    return b["gamma"] * b["MH"] + Si - Si @ Pi @ S1p @ Pi.T @ Si


def K_monodomain(b):
    return b["gamma"] * b["MH"] + b["Sm"]


def LU_factors(b):
    S1p = pinv_kernel1(b["S1"])
    N, NH = b["N"], b["NH"]
    Si, Pi = b["Si"], b["Pi"]
    K = schur_K(b)
    L = np.block([[b["S1"], np.zeros((N, NH))], [Si @ Pi, K]])
    U = np.block([[np.eye(N), S1p @ Pi.T @ Si], [np.zeros((NH, N)), np.eye(NH)]])
    Kinv = np.linalg.inv(K)
    Lp = np.block([[S1p, np.zeros((N, NH))],
                   [-Kinv @ Si @ Pi @ S1p, Kinv]])
    Uinv = np.block([[np.eye(N), -S1p @ Pi.T @ Si],
                     [np.zeros((NH, N)), np.eye(NH)]])
    return L, U, Lp, Uinv, K


def grounded(S, k=None):
    """S with row and column k replaced by the unit vector e_k (k defaults to
    the last index).  It is SPD when the kernel of S is the constants."""
    n = S.shape[0]
    k = n - 1 if k is None else k
    G = S.copy()
    G[k, :] = 0.0
    G[:, k] = 0.0
    G[k, k] = 1.0
    return G


def grounded_solver(S, k=None):
    """Generalised inverse of a PSD S with kernel = constants, obtained by
    fixing unknown k to zero: y -> x with x_k = 0 and (S x)_i = y_i for
    i != k.  For y orthogonal to the constants the dropped equation k holds
    too (the rows of S sum to zero), so S x = y.  Written with the grounded
    matrix: zero entry k of y, solve, zero entry k of the result."""
    n = S.shape[0]
    k = n - 1 if k is None else k
    solve = chol_solver(grounded(S, k))

    def apply(y):
        y = y.copy()
        y[k] = 0.0
        x = solve(y)
        x[k] = 0.0
        return x
    return apply


def block_prec(b, P1inv, PKinv):
    """Return X = P_Lambda^-1 Y following Def. 2 / eq. (prec2)."""
    N = b["N"]
    Si, Pi = b["Si"], b["Pi"]

    def apply(Y):
        Y1, Y2 = Y[:N], Y[N:]
        Z1 = P1inv(Y1)
        Z2 = PKinv(Y2 - Si @ (Pi @ Z1))
        X1 = Z1 - P1inv(Pi.T @ (Si @ Z2))
        return np.concatenate([X1, Z2])
    return apply


def chol_solver(A):
    cf = sla.cho_factor(A, lower=True)
    return lambda y: sla.cho_solve(cf, y)


def pcg(A, Y, Pinv, x0=None, tol=1e-10, max_iter=500):
    """Preconditioned conjugate gradient with the stop |A x - Y| / |Y| <= tol
    (Euclidean norms, Sec. 6.2).  Returns (x, iterations, residual history)."""
    x = np.zeros_like(Y) if x0 is None else x0.copy()
    r = Y - A @ x
    ny = np.linalg.norm(Y)
    hist = [np.linalg.norm(r) / ny]
    if hist[-1] <= tol:
        return x, 0, hist
    z = Pinv(r)
    p = z.copy()
    rz = r @ z
    for it in range(1, max_iter + 1):
        q = A @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        hist.append(np.linalg.norm(r) / ny)
        if hist[-1] <= tol:
            return x, it, hist
        z = Pinv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_iter, hist
