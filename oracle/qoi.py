"""Quantities of interest of Model Problems 1 and 2 (oracle side).

Section 3.4 takes as quantity of interest the flux through the face x1 = 1,
M^(2)(p) = -int phi k grad p . n ds with a weight phi equal to 1 on x1 = 1
and 0 on x1 = 0.  For the discrete solution this is the sum of the
boundary-face fluxes on x1 = 1 (reading: phi is not specified; for the exact
discrete solution with f = 0 and no-flow sides every cross-section carries
the same total flux, so any such phi gives this value):

    Q_out = sum over cells P with i = m-1 of T_b,P (p_P - 0),  T_b = 2 k_P h^(d-2),
    Q_in  = sum over cells P with i = 0   of T_b,P (1 - p_P).

Q_in = Q_out is local mass conservation of the finite volume scheme.

Model Problem 1 (Section 3.4) regularises a point value of the pressure by its
mean over a small subdomain D* around the point, M^(1)(p) = |D*|^-1 int_D* p.
The paper fixes neither the point nor D* (reading: x* = the centre of the unit
cube, D* = [1/2 - 1/16, 1/2 + 1/16]^d, the cell of the h = 1/8 grid centred
there).  The discrete pressure is constant on each cell, so

    M^(1) = sum over cells P of p_P |P cap D*| / |D*|,

with |P cap D*| the product over the axes of the overlaps of [i h, (i+1) h]
with [lo, hi].
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


MP1_BOX = (0.5 - 1.0 / 16.0, 0.5 + 1.0 / 16.0)


def axis_overlaps(m, lo, hi):
    """Length of [i h, (i+1) h] cap [lo, hi] for i = 0..m-1 (h = 1/m)."""
    edges = np.arange(m + 1) / m
    return np.clip(np.minimum(edges[1:], hi) - np.maximum(edges[:-1], lo), 0.0, None)


def box_average(p, lo=MP1_BOX[0], hi=MP1_BOX[1]):
    """M^(1): mean of the cell-wise constant pressure over D* = [lo, hi]^d.
    p has one axis per direction (shape (m,)*d)."""
    p = np.asarray(p)
    d = p.ndim
    w = axis_overlaps(p.shape[0], lo, hi)
    weight = w
    for _ in range(d - 1):
        weight = np.multiply.outer(w, weight)
    return float(np.sum(p * weight) / (hi - lo) ** d)
