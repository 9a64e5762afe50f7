"""Outflow functional of Model Problem 2 (oracle side).

Section 3.4 takes as quantity of interest the flux through the face x1 = 1,
M^(2)(p) = -int phi k grad p . n ds with a weight phi equal to 1 on x1 = 1
and 0 on x1 = 0.  For the discrete solution this is the sum of the
boundary-face fluxes on x1 = 1 (reading: phi is not specified; for the exact
discrete solution with f = 0 and no-flow sides every cross-section carries
the same total flux, so any such phi gives this value):

    Q_out = sum over cells P with i = m-1 of T_b,P (p_P - 0),  T_b = 2 k_P h^(d-2),
    Q_in  = sum over cells P with i = 0   of T_b,P (1 - p_P).

Q_in = Q_out is local mass conservation of the finite volume scheme.
"""
import numpy as np


def outflow(k, p):
    d = k.ndim
    m = k.shape[0]
    p = np.asarray(p).reshape(k.shape)
    scale = (1.0 / m) ** (d - 2)
    return float(np.sum(2.0 * k[..., m - 1] * scale * p[..., m - 1]))


def inflow(k, p):
    d = k.ndim
    m = k.shape[0]
    p = np.asarray(p).reshape(k.shape)
    scale = (1.0 / m) ** (d - 2)
    return float(np.sum(2.0 * k[..., 0] * scale * (1.0 - p[..., 0])))
