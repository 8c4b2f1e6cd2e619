"""Mitchell-Schaeffer two-current ionic model (pointwise, FP64).

The paper runs Luo-Rudy II (Sec. 6.1); the workloads of this project use the
Mitchell-Schaeffer model (Mitchell & Schaeffer, Bull. Math. Biol. 2003) with
its published constants.  Potentials are measured from rest in mV, with the
normalised potential vt = V / DV, DV = 100 mV.  In the paper's notation the
reaction enters as  chi (c dV/dt + I_ion - I_st) = div(...), so

    I_ion(V, h) = c * DV * ( -h vt^2 (1 - vt) / tau_in + vt / tau_out )
    g(V, h)     = (1 - h) / tau_open   if vt <  v_gate
                  -h / tau_close       otherwise

in uA/cm^2 and 1/ms.
"""
import numpy as np

TAU_IN = 0.3
TAU_OUT = 6.0
TAU_OPEN = 120.0
TAU_CLOSE = 150.0
V_GATE = 0.13
DV = 100.0


def i_ion(V, h, cm):
    vt = V / DV
    return cm * DV * (-h * vt * vt * (1.0 - vt) / TAU_IN + vt / TAU_OUT)


def gate_rate(V, h):
    vt = V / DV
    return np.where(vt < V_GATE, (1.0 - h) / TAU_OPEN, -h / TAU_CLOSE)
