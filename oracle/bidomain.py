"""Semi-implicit bidomain time step and the normalised linear solve.

Sec. 3.2 (scheme and resolution algorithm): with gamma = chi*c/dt,

  Step 1  Y = [0 ; M_H (gamma V^n - chi (I_ion(V^n, W^n) - I_st^n))]
  Step 2  Lambda X = Y, X = [U^{n+1}; V^{n+1}],
          Lambda = [[S_1, Pi^T S_i], [S_i Pi, gamma M_H + S_i]],
          normalised so that the integral of U^{n+1} over the thorax is 0
  Step 3  W^{n+1} = W^n + dt g(V^n, W^n)   (explicit on the reaction)

Vertices are reordered heart-first (assumption H1), so that Pi is the
truncation to the first N_H entries and Pi^T the zero padding.

Crank-Nicolson (the remark on the time discretisation after Prop. 3: another
scheme changes only Step 1 and the definition of K).  Reading: the diffusion
terms of the parabolic row are averaged over t^n and t^{n+1}, the reaction
stays explicit and the elliptic row holds at t^{n+1}:

  gamma M_H (V^{n+1} - V^n) + 1/2 S_i (V + Pi U)^{n+1} + 1/2 S_i (V + Pi U)^n
      = - chi M_H (I_ion(V^n, W^n) - I_st^n);

times 2 this is the system above with gamma replaced by 2 gamma (in Lambda
and in K) and

  Y = [0 ; M_H (2 gamma V^n - 2 chi (I_ion - I_st)) - S_i (V^n + Pi U^n)].

Strang operator splitting (named by the same remark): the reaction
c dV/dt = I_st - I_ion(V, W), dW/dt = g(V, W) and the diffusion are advanced
in turn, reaction over dt/2 (Heun's method, pointwise), diffusion over dt
(the Crank-Nicolson step above without the ionic term, from (U^n, V*)),
reaction over dt/2 again; second order in dt.  The diffusion step starts
from (U*, V*) with U* the potential the elliptic row gives V*
(S_1 U* = -Pi^T S_i V*): starting from U^n, which belongs to V^n, would
leave an O(dt) inconsistency and a first-order scheme.

`reaction=False` drops I_ion and I_st (the linear problem, for the
convergence-order pins).

Prop. 1: Lambda is symmetric positive semi-definite with kernel
1_Omega x {0}; for Y in its range the solution with (M U, 1) = 0 is unique,
obtained from any solution by U <- U - alpha 1 with
alpha = (M U, 1) / (M 1, 1).

The normalised solution is computed three independent ways:
  solve_dense   Cholesky of the SPD matrix Lambda + c w w^T, w = [M 1; 0]
  solve_sparse  sparse LU of Lambda with one u unknown fixed to 0, then the
                normalisation of Prop. 1
  solve_cg      Jacobi-preconditioned CG with a stop that accounts for the
                Lanczos estimate of the condition number, then normalisation
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, ionic


class System:
    """Assembled bidomain system for one mesh and one time step."""

    def __init__(self, cfg, dt=None, scheme="euler", reaction=True):
        if scheme not in ("euler", "cn", "strang"):
            raise ValueError("scheme is 'euler', 'cn' or 'strang'")
        self.cfg = cfg
        self.scheme = scheme
        self.reaction = reaction
        a = fem.assemble(cfg)
        self.N, self.NH = a["N"], a["NH"]
        self.hn = a["hn"]
        N, NH = self.N, self.NH
        is_h = np.zeros(N, dtype=bool)
        is_h[self.hn] = True
        self.torso = np.nonzero(~is_h)[0]
        # heart-first order: heart vertices (ascending id), then torso ones
        self.perm = np.concatenate([self.hn, self.torso])
        self.chi, self.cm = cfg["chi"], cfg["cm"]
        self.dt = cfg["dt"] if dt is None else dt
        self.gamma = self.chi * self.cm / self.dt
        # the coefficient of M_H in Lambda and K: gamma (Euler), 2 gamma (CN)
        self.gamma_eff = self.gamma * (1.0 if scheme == "euler" else 2.0)
        P = self.perm
        self.S1 = a["S1"][P][:, P].tocsr()
        self.Se = a["Se"][P][:, P].tocsr()
        self.Si, self.Sm = a["Si"], a["Sm"]
        self.m = a["m"][P]
        self.mH = a["mH"]
        Pi_T = sp.vstack([sp.identity(NH, format="csr"),
                          sp.csr_matrix((N - NH, NH))]).tocsr()
        self.PiT = Pi_T
        g = self.gamma_eff
        self.Lam = sp.bmat([[self.S1, Pi_T @ self.Si],
                            [self.Si @ Pi_T.T, g * sp.diags(self.mH) + self.Si]],
                           format="csr")
        stim = cfg["stim_mask"].astype(bool)[self.hn]
        self.stim_h = stim
        self.n0 = int(round(cfg["stim_t0"] / self.dt))
        self.n1 = int(round(cfg["stim_t1"] / self.dt))

    # ---- ordering helpers --------------------------------------------
    def to_global_u(self, Uperm):
        u = np.empty(self.N)
        u[self.perm] = Uperm
        return u

    def from_global_u(self, u):
        return u[self.perm]

    # ---- Step 1 and Step 3 --------------------------------------------
    def i_stim(self, n):
        amp = self.cfg["stim_amp"] if self.n0 <= n < self.n1 else 0.0
        return np.where(self.stim_h, amp, 0.0)

    def rhs(self, V, h, n, U=None, reaction=None):
        """Step 1: the right-hand side Y (heart-first order).  Crank-Nicolson
        also needs U^n (heart-first order; constants do not matter, S_i 1 = 0).
        reaction=False overrides the system's flag (the diffusion step of a
        splitting)."""
        react = self.reaction if reaction is None else reaction
        src = ionic.i_ion(V, h, self.cm) - self.i_stim(n) if react else np.zeros(self.NH)
        if self.scheme == "euler":
            Y2 = self.mH * (self.gamma * V - self.chi * src)
        else:
            if U is None:
                raise ValueError("the Crank-Nicolson right-hand side needs U^n")
            Y2 = self.mH * (2.0 * self.gamma * V - 2.0 * self.chi * src) - self.Si @ (V + U[:self.NH])
        return np.concatenate([np.zeros(self.N), Y2])

    def gate(self, V, h):
        """Step 3, forward Euler on the old state."""
        return h + self.dt * ionic.gate_rate(V, h) if self.reaction else h

    # ---- normalisation (Prop. 1) ---------------------------------------
    def normalise(self, X):
        X = X.copy()
        U = X[:self.N]
        alpha = np.dot(self.m, U) / np.sum(self.m)
        X[:self.N] = U - alpha
        return X

    # ---- Step 2: three solvers -----------------------------------------
    def solve_dense(self, Y):
        L = self.Lam.toarray()
        w = np.concatenate([self.m, np.zeros(self.NH)])
        c = np.abs(L).sum(axis=1).max() / np.dot(w, w)
        A = L + c * np.outer(w, w)
        cf = sla.cho_factor(A, lower=True)
        return sla.cho_solve(cf, Y)

    def solve_sparse(self, Y):
        n2 = self.N + self.NH
        k = self.N - 1                       # the u unknown fixed to 0
        keep = np.concatenate([np.arange(k), np.arange(k + 1, n2)])
        A = self.Lam[keep][:, keep].tocsc()
        lu = spla.splu(A, permc_spec="COLAMD")
        x = np.zeros(n2)
        x[keep] = lu.solve(Y[keep])
        # refine once against the full (consistent) system
        r = Y - self.Lam @ x
        x[keep] += lu.solve(r[keep])
        return self.normalise(x)

    def solve_cg(self, Y, x0=None, rtol=1e-12, kappa_rtol=1e-10,
                 max_iter=200000):
        """Jacobi-CG on the augmented matrix Lam + c w w^T of solve_dense
        (w = [M 1; 0]): symmetric positive definite, and its solution is the
        normalised one of Prop. 1.  On Lam itself the kernel (1, 0) made
        rounding show up as a Ritz value near zero, so the condition
        estimate of the stopping test never settled."""
        L = self.Lam
        w = np.concatenate([self.m, np.zeros(self.NH)])
        c = abs(L).sum(axis=1).max() / np.dot(w, w)

        class _Aug:
            def __matmul__(self, v):
                return L @ v + (c * np.dot(w, v)) * w
        A = _Aug()
        dinv = 1.0 / (L.diagonal() + c * w * w)
        x = np.zeros_like(Y) if x0 is None else x0.copy()
        r = Y - A @ x
        ny = np.linalg.norm(Y)
        z = dinv * r
        p = z.copy()
        rz = r @ z
        alphas, betas = [], []
        kappa = 1.0
        for it in range(max_iter):
            q = A @ p
            alpha = rz / (p @ q)
            x += alpha * p
            r -= alpha * q
            alphas.append(alpha)
            rel = np.linalg.norm(r) / ny
            if rel <= rtol and (it % 25 == 0 or rel * kappa <= kappa_rtol):
                kappa = _lanczos_kappa(alphas, betas)
                if rel * kappa <= kappa_rtol:
                    break
            z = dinv * r
            rz_new = r @ z
            beta = rz_new / rz
            betas.append(beta)
            rz = rz_new
            p = z + beta * p
        self.last_cg = dict(iters=it + 1, rel=rel, kappa=kappa)
        return self.normalise(x)

    def solve(self, Y, method="auto", x0=None):
        n2 = self.N + self.NH
        if method == "auto":
            method = "dense" if n2 <= 6000 else (
                "sparse" if self.cfg["dim"] == 2 else "cg")
        if method == "dense":
            return self.solve_dense(Y)
        if method == "sparse":
            return self.solve_sparse(Y)
        return self.solve_cg(Y, x0=x0)

    def elliptic_u(self, V):
        """A U with S_1 U = -Pi^T S_i V (the elliptic row for V; defined up
        to a constant, which S_i Pi ignores): the last u unknown fixed to 0,
        sparse LU of the rest."""
        N = self.N
        b = -(self.PiT @ (self.Si @ V))
        keep = np.arange(N - 1)
        A = self.S1[keep][:, keep].tocsc()
        U = np.zeros(N)
        U[keep] = spla.spsolve(A, b[keep])
        return U

    def reaction_half(self, V, h, n):
        """The reaction over dt/2 by Heun's method: with the rates
        f(V, W) = (I_st - I_ion(V, W)) / c and g(V, W),
        V1 = V + tau f, W1 = W + tau g at (V, W), then
        V* = V + tau/2 (f(V, W) + f(V1, W1)), likewise W* (tau = dt/2)."""
        tau = 0.5 * self.dt
        ist = self.i_stim(n) if self.reaction else np.zeros(self.NH)

        def rates(v, w):
            if not self.reaction:
                return np.zeros_like(v), np.zeros_like(w)
            return (ist - ionic.i_ion(v, w, self.cm)) / self.cm, ionic.gate_rate(v, w)
        f1, g1 = rates(V, h)
        f2, g2 = rates(V + tau * f1, h + tau * g1)
        return V + 0.5 * tau * (f1 + f2), h + 0.5 * tau * (g1 + g2)

    # ---- a full time step ------------------------------------------------
    def step(self, V, h, n, method="auto", U0=None):
        """Advance (V^n, h^n) -> (U^{n+1}, V^{n+1}, h^{n+1}).  U0: U^n in
        heart-first order (initial guess; required by Crank-Nicolson and the
        splitting)."""
        if self.scheme == "strang":
            if U0 is None:
                raise ValueError("the splitting's diffusion step needs U^n")
            Vs, hs = self.reaction_half(V, h, n)
            Us = self.elliptic_u(Vs)
            Y = self.rhs(Vs, hs, n, Us, reaction=False)
            X = self.solve(Y, method=method, x0=np.concatenate([U0, Vs]))
            V1, h1 = self.reaction_half(X[self.N:], hs, n)
            return X[:self.N], V1, h1
        Y = self.rhs(V, h, n, U0)
        x0 = None
        if U0 is not None:
            x0 = np.concatenate([U0, V])
        X = self.solve(Y, method=method, x0=x0)
        h1 = self.gate(V, h)
        return X[:self.N], X[self.N:], h1


def _lanczos_kappa(alphas, betas):
    """Condition-number estimate of the preconditioned operator from the CG
    coefficients (the Lanczos tridiagonal of the CG recurrences)."""
    k = len(alphas)
    a = np.asarray(alphas)
    b = np.asarray(betas[:k - 1]) if k > 1 else np.zeros(0)
    diag = 1.0 / a
    diag[1:] += b / a[:-1]
    off = np.sqrt(np.maximum(b, 0.0)) / a[:-1]
    ev = sla.eigh_tridiagonal(diag, off, eigvals_only=True)
    ev = ev[ev > 0]
    return float(ev.max() / ev.min()) if len(ev) else 1.0


def rel_err(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def sampled_residual(cfg, verts, Vn, hn, n, U1, V1):
    """Rows of Lambda X - Y at sampled vertices, for a full-size check that
    needs no global assembly: X = (U1, V1) is a computed solution of the
    semi-implicit step from (V^n, h^n) (U1 in global order, Vn, hn, V1 in
    heart-local order).  Each sampled row is assembled from the elements
    that hold its vertex (Sec. 3.1), with Y from Step 1 (Sec. 3.2):

      u row of g:  (S_1 U1)_g + (S_i V1)_g                  (0 in Y)
      v row of g:  (S_i (U1 + V1))_g + gamma m_g V1_g - m_g (gamma V^n_g
                   - chi (I_ion - I_st))_g

    Returns (r_u, r_v, y_v): the residual rows at the sampled vertices and
    the rows of Y_2 at the heart ones (r_v, y_v).  Only the semi-implicit
    scheme.
    """
    xyz, el = cfg["xyz"], cfg["elems"].astype(np.int64)
    N = len(xyz)
    hn_ids = fem.heart_nodes(cfg)
    loc = -np.ones(N, dtype=np.int64)
    loc[hn_ids] = np.arange(len(hn_ids))
    verts = np.asarray(verts, dtype=np.int64)
    want = np.zeros(N, dtype=bool)
    want[verts] = True
    touch = np.nonzero(want[el].any(axis=1))[0]
    sub = el[touch]
    vol, G = fem.element_geometry(xyz, sub)
    sig_i, _, sig_1, _, _ = fem.tensors(cfg, touch)
    heart_e = cfg["region"][touch] == fem.REGION_HEART
    K1 = vol[:, None, None] * np.einsum("eai,eij,ebj->eab", G, sig_1, G)
    Ki = vol[:, None, None] * np.einsum("eai,eij,ebj->eab", G, sig_i, G)
    k = sub.shape[1]
    vh = np.where(loc[sub] >= 0, V1[np.maximum(loc[sub], 0)], 0.0)     # V1 at the element's vertices
    u_e = U1[sub]
    su = np.einsum("eab,eb->ea", K1, u_e) + np.where(heart_e[:, None], np.einsum("eab,eb->ea", Ki, vh), 0.0)
    sv = np.where(heart_e[:, None], np.einsum("eab,eb->ea", Ki, u_e + vh), 0.0)
    mass = np.where(heart_e[:, None], np.repeat(vol[:, None] / k, k, axis=1), 0.0)
    ru = np.zeros(N)
    rv = np.zeros(N)
    mh = np.zeros(N)
    np.add.at(ru, sub.ravel(), su.ravel())
    np.add.at(rv, sub.ravel(), sv.ravel())
    np.add.at(mh, sub.ravel(), mass.ravel())
    gamma = cfg["chi"] * cfg["cm"] / cfg["dt"]
    n0 = int(round(cfg["stim_t0"] / cfg["dt"]))
    n1 = int(round(cfg["stim_t1"] / cfg["dt"]))
    amp = cfg["stim_amp"] if n0 <= n < n1 else 0.0
    ist = np.where(cfg["stim_mask"].astype(bool)[hn_ids], amp, 0.0)
    src = ionic.i_ion(Vn, hn, cfg["cm"]) - ist                        # heart-local
    hv = verts[loc[verts] >= 0]
    lv = loc[hv]
    r_v = rv[hv] + gamma * mh[hv] * V1[lv] - mh[hv] * (gamma * Vn[lv] - cfg["chi"] * src[lv])
    y_v = mh[hv] * (gamma * Vn[lv] - cfg["chi"] * src[lv])
    return ru[verts], r_v, y_v
