"""Oracle pins for the 3-D path (CPU).

* tilted plane: on the slice x3 = 1/2 it is the straight line through the two
  random heights, i.e. the 2-node piecewise-linear interface; the fraction of
  bottom-layer cells tends to the volume under the plane, (a + b)/2, within
  the discretisation error 1/m;
* 3-D finite volume system: layers parallel to the flow (k depends on x2 only)
  give Q = mean of k over the rows, and layers across the flow (k depends on
  x1 only) give Q = the harmonic mean of the layer values (series resistances
  with half-cell Dirichlet faces); Q_in = Q_out; Q(c k) = c Q(k);
* the 3-D sample: the plain coarse companion takes the fine Gaussian values at
  even indices (checked on the composite k where both grids put a cell in the
  same layer), and the CGV sub-lattices tile the fine sample.
"""
import numpy as np
import pytest

import workloads as W
from oracle import field, fv, geometry, qoi, solve


def _solve_q(k):
    A, b = fv.assemble(k)
    p = solve.direct_solve(A, b)
    return qoi.outflow(k, p), qoi.inflow(k, p)


def test_tilted_plane_mid_slice_is_the_two_node_line():
    """On the slice x3 = 1/2 the tilt term vanishes: the partition there is the
    2-node piecewise-linear interface through the same two heights."""
    model = W.TILTED3
    flat = model.with_(interface_kind=W.PIECEWISE_LINEAR, n_nodes=2)
    m = 15                                   # odd: slice 7 has x3 = 1/2 exactly
    for sample in range(6):
        lid = geometry.layer_ids(model, 0, sample, m)
        ref = geometry.layer_ids(flat, 0, sample, m)
        np.testing.assert_array_equal(lid[m // 2], ref[m // 2])
        c = geometry.interface_params(model, 0, sample)["c"]
        if abs(c) > 0.05:                    # a visible tilt changes other slices
            assert not np.array_equal(lid[0], lid[-1])


def test_tilted_plane_bottom_fraction_is_volume_under_plane():
    model = W.TILTED3
    m = 64
    for sample in range(4):
        prm = geometry.interface_params(model, 0, sample)
        lid = geometry.layer_ids(model, 0, sample, m)
        frac = np.mean(lid == 0)
        assert abs(frac - 0.5 * (prm["a"] + prm["b"])) <= 1.0 / m, (frac, prm)
        assert -0.1 <= prm["c"] <= 0.1 and 0.3 <= prm["a"] <= 0.7


@pytest.mark.parametrize("m", [4, 6])
def test_3d_parallel_and_series_layers(m):
    rng = np.random.default_rng(m)
    kj = np.exp(rng.standard_normal(m))
    k = np.broadcast_to(kj[None, :, None], (m, m, m)).copy()     # depends on x2 only
    q_out, q_in = _solve_q(k)
    assert abs(q_out - kj.mean()) <= 1e-12 * kj.mean()
    assert abs(q_in - q_out) <= 1e-12 * q_out
    ki = np.exp(rng.standard_normal(m))
    k = np.broadcast_to(ki[None, None, :], (m, m, m)).copy()     # depends on x1 only
    q_out, q_in = _solve_q(k)
    # resistances in series: half cells at both ends, cell-to-cell harmonic faces
    h = 1.0 / m
    res = 0.5 * h / ki[0] + 0.5 * h / ki[-1] + sum(h / fv.harmonic(ki[i], ki[i + 1]) for i in range(m - 1))
    assert abs(q_out - 1.0 / res) <= 1e-12 / res
    assert abs(q_in - q_out) <= 1e-12 * q_out
    q2, _ = _solve_q(3.0 * k)
    assert abs(q2 - 3.0 * q_out) <= 1e-12 * q_out


def test_3d_sample_companions():
    model = W.TILTED3
    m = 8
    k, kc = field.sample_k(model, 1, 3, m, with_coarse=True)
    assert k.shape == (m, m, m) and kc.shape == (m // 2,) * 3
    lid = geometry.layer_ids(model, 1, 3, m)
    lid_c = geometry.layer_ids(model, 1, 3, m // 2)
    same = lid[::2, ::2, ::2] == lid_c
    assert same.mean() > 0.5
    np.testing.assert_array_equal(kc[same], k[::2, ::2, ::2][same])
    subs = field.cgv_sublattices(k)
    assert len(subs) == 8
    back = np.zeros_like(k)
    for j, s in enumerate(subs):
        a = [(j >> b) & 1 for b in range(3)]
        back[a[2]::2, a[1]::2, a[0]::2] = s
    np.testing.assert_array_equal(back, k)
