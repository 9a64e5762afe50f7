"""Random layer partitions (oracle side).

Section 2 partitions the domain into random convex subdomains D_i(omega),
drawn independently of the permeability values.  Section 3.4 builds them
from straight random lines; the workloads here also use a single horizontal
interface and a piecewise-linear interface through equispaced random nodes.
The partition is evaluated at the cell centres x_ij of the finite volume
mesh of Section 3.1: x1 = (i + 1/2)/m, x2 = (j + 1/2)/m.

Every uniform comes from the geometry stream (tag 0) of the sample:
uniform number q is word q % 4 of block q // 4.

Conventions (readings where the paper or the workload is silent):
* layer 0 is the bottom layer; a centre lying exactly on an interface
  belongs to the upper layer (a measure-zero event);
* piecewise-linear nodes sit at x = q/(n-1), q = 0..n-1;
* in 3D the 2-D interfaces are extruded along x3, as the paper does in 3D;
* the tilted plane (3D workload) is x2 = a + (b - a) x1 + c (x3 - 1/2) with
  a, b ~ U(y_lo, y_hi) and c ~ U(-0.1, 0.1) (uniforms 0, 1, 2): the paper's
  straight line from (0, a) to (1, b), tilted along x3; x2 stays the
  vertical axis and x1 the flow direction.
"""
import numpy as np

from . import philox

HORIZONTAL = 0
PIECEWISE_LINEAR = 1
PAPER_TWO_LINES = 2
TILTED_PLANE = 3
NO_INTERFACE = 4


def geometry_uniforms(model, level, sample, count):
    nblk = (count + 3) // 4
    blk = philox.blocks(model.seed, sample, level, philox.TAG_GEOMETRY, np.arange(nblk))
    return philox.to_uniform(blk).reshape(-1)[:count]


def cell_centres(m):
    """Cell-centre coordinates (i + 1/2)/m, i = 0..m-1 (Section 3.1)."""
    return (np.arange(m, dtype=np.float64) + 0.5) / m


def interface_params(model, level, sample):
    """The random numbers that fix the partition of one sample."""
    kind = model.interface_kind
    if kind == HORIZONTAL:
        u = geometry_uniforms(model, level, sample, 1)
        return {"y0": model.y_lo + (model.y_hi - model.y_lo) * u[0]}
    if kind == PIECEWISE_LINEAR:
        n = model.n_nodes
        u = geometry_uniforms(model, level, sample, n)
        return {"nodes": model.y_lo + (model.y_hi - model.y_lo) * u}
    if kind == PAPER_TWO_LINES:
        # y1 ~ U(0.8, 0.9), y2 ~ U(0.6, 0.7), y3 ~ U(0.2, 0.3), y4 ~ U(0.4, 0.5)
        u = geometry_uniforms(model, level, sample, 4)
        lo = np.array([0.8, 0.6, 0.2, 0.4])
        return {"y": lo + 0.1 * u}
    if kind == TILTED_PLANE:
        u = geometry_uniforms(model, level, sample, 3)
        a = model.y_lo + (model.y_hi - model.y_lo) * u[0]
        b = model.y_lo + (model.y_hi - model.y_lo) * u[1]
        return {"a": a, "b": b, "c": -0.1 + 0.2 * u[2]}
    if kind == NO_INTERFACE:
        return {}
    raise ValueError("unknown interface kind %r" % kind)


def piecewise_linear(nodes, x):
    """Height of the interface through equispaced nodes at abscissae x."""
    n = len(nodes)
    s = np.minimum(np.floor((n - 1) * x), n - 2).astype(np.int64)
    t = (n - 1) * x - s
    return nodes[s] + t * (nodes[s + 1] - nodes[s])


def layer_ids(model, level, sample, m):
    """Layer index of every cell centre of an m^d grid; array indexed [..., x2, x1]."""
    d = model.dim
    x = cell_centres(m)
    x1 = x[None, :]
    x2 = x[:, None]
    prm = interface_params(model, level, sample)
    kind = model.interface_kind
    if kind == HORIZONTAL:
        lid = np.where(x2 < prm["y0"], 0, 1) + 0 * x1
    elif kind == PIECEWISE_LINEAR:
        yif = piecewise_linear(prm["nodes"], x)[None, :]
        lid = np.where(x2 < yif, 0, 1)
    elif kind == PAPER_TWO_LINES:
        y1, y2, y3, y4 = prm["y"]
        upper = y1 + x1 * (y2 - y1)
        lower = y3 + x1 * (y4 - y3)
        lid = np.where(x2 < lower, 0, np.where(x2 < upper, 1, 2))
    elif kind == TILTED_PLANE:
        a, b, c = prm["a"], prm["b"], prm["c"]
        if d == 3:
            x3 = x[:, None, None]
            plane = a + (b - a) * x[None, None, :] + c * (x3 - 0.5)
            return np.where(x[None, :, None] < plane, 0, 1).astype(np.int64)
        lid = np.where(x2 < a + (b - a) * x1, 0, 1)
    elif kind == NO_INTERFACE:
        lid = np.zeros((m, m), dtype=np.int64)
    lid = np.broadcast_to(lid, (m, m)).astype(np.int64)
    if d == 3:
        lid = np.broadcast_to(lid[None, :, :], (m, m, m)).copy()
    return lid
