"""Recordings of a run: activation times and potentials at probe points.

TEST INFRASTRUCTURE ONLY (see the package header).

The test cases of Sec. 6 map the activation time of each point (the instant
at which the transmembrane potential reaches a fixed level during the
depolarisation) and record the potential u at body-surface electrodes at
every step (the ECG).  Written from those definitions:

  activation   the first time the potential of a vertex reaches v_act, with
               the potential taken linear in time over each step; a vertex
               already at or above the level at the start of a step gets the
               start time; -1 when never reached
  probe        u at a point of the mesh is the P1 interpolant: the
               barycentric combination of the vertex values of an element
               holding the point (the interpolant is continuous, so any such
               element gives the same value)
"""
import numpy as np


def activation_times(V_steps, t0, dt, v_act):
    """V_steps: potentials V^0, V^1, ... (one array per time level, V^k at
    time t0 + k dt).  Returns the activation time of each vertex."""
    act = np.full(len(V_steps[0]), -1.0)
    for k in range(len(V_steps) - 1):
        vo, vn = V_steps[k], V_steps[k + 1]
        tk = t0 + k * dt
        for i in range(len(act)):
            if act[i] >= 0 or vn[i] < v_act:
                continue
            act[i] = tk if vo[i] >= v_act else tk + dt * (v_act - vo[i]) / (vn[i] - vo[i])
    return act


def locate(xyz, elems, p):
    """An element holding point p and the barycentric coordinates there:
    solve [1 ... 1; vertices^T] lam = [1; p] element by element."""
    dim = xyz.shape[1]
    best, best_lam, best_min = -1, None, -np.inf
    for e, ids in enumerate(elems):
        A = np.vstack([np.ones(dim + 1), xyz[ids].T])
        try:
            lam = np.linalg.solve(A, np.concatenate([[1.0], p]))
        except np.linalg.LinAlgError:
            continue
        if lam.min() > best_min:
            best, best_lam, best_min = e, lam, lam.min()
    if best_min < -1e-9:
        raise ValueError("point outside the mesh")
    return best, best_lam


def probe_values(xyz, elems, u, points):
    out = []
    for p in points:
        e, lam = locate(xyz, elems, np.asarray(p, dtype=float))
        out.append(float(lam @ u[elems[e]]))
    return np.array(out)
