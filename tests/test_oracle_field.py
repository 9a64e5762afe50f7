"""Pins of the oracle's layer geometry and permeability samplers.

* Geometry: closed-form row counts for a horizontal interface; the
  piecewise-linear interface against numpy.interp; the ordering and
  parameter ranges of the paper's two random lines (Section 3.4).
* Example 1: the field takes exactly the layer values exp(mu_l + sigma_l z_l).
* Example 2 / circulant embedding: the sampler's linear map M (probed with
  unit noise vectors) has Re(M)Re(M)^T = Im(M)Im(M)^T = the covariance
  eq. (2.3) between grid points (evaluated directly from the distances, not
  through the torus) and Re(M)Im(M)^T = 0; the empirical covariance of real
  samples matches eq. (2.3); too-small embeddings are refused.
* Coarse samples: Coarse Grid Variates sub-lattices by index brute force
  (Section 4.1); the plain coarse sample equals direct evaluation on the
  coarse grid for piecewise constant layers.
"""
import numpy as np
import pytest

import workloads as W
from oracle import field, geometry


def test_horizontal_interface_row_count():
    m = 32
    for s in range(50):
        y0 = geometry.interface_params(W.PC2, 0, s)["y0"]
        assert 0.3 < y0 < 0.7
        lid = geometry.layer_ids(W.PC2, 0, s, m)
        below = int(np.sum(lid[:, 0] == 0))
        # rows j with (j + 1/2)/m < y0
        assert below == int(np.ceil(m * y0 - 0.5))
        assert np.all(lid == lid[:, :1])          # horizontal: rows are constant


def test_piecewise_linear_interface_matches_interp():
    model = W.CE2
    m = 64
    for s in range(20):
        nodes = geometry.interface_params(model, 1, s)["nodes"]
        assert np.all((nodes > 0.3) & (nodes < 0.7))
        x = (np.arange(m) + 0.5) / m
        yif = np.interp(x, np.linspace(0.0, 1.0, len(nodes)), nodes)
        assert np.allclose(geometry.piecewise_linear(nodes, x), yif, rtol=0, atol=1e-15)
        lid = geometry.layer_ids(model, 1, s, m)
        y = (np.arange(m) + 0.5) / m
        ref = np.where(y[:, None] < yif[None, :], 0, 1)
        # centres within rounding distance of the interface may go either way
        close = np.abs(y[:, None] - yif[None, :]) < 1e-14
        assert np.all((lid == ref) | close)


def test_paper_two_lines_ranges_and_order():
    model = W.PC2.with_(interface_kind=W.PAPER_TWO_LINES, n_layers=3)
    m = 32
    for s in range(30):
        y1, y2, y3, y4 = geometry.interface_params(model, 0, s)["y"]
        assert 0.8 < y1 < 0.9 and 0.6 < y2 < 0.7 and 0.2 < y3 < 0.3 and 0.4 < y4 < 0.5
        lid = geometry.layer_ids(model, 0, s, m)
        assert set(np.unique(lid)) == {0, 1, 2}
        assert np.all(np.diff(lid, axis=0) >= 0)   # layer index grows upwards in every column


def test_piecewise_constant_values():
    model = W.PC2
    for s in range(10):
        k = field.sample_k(model, 0, s, 16)
        z = field.layer_constants(model, 0, s)
        lid = geometry.layer_ids(model, 0, s, 16)
        assert np.array_equal(k, np.exp(z[lid]))
        assert len(np.unique(k)) == len(np.unique(lid))


def test_piecewise_constant_law_moments_at_general_variance():
    """Example 1 with unequal means and variances (sigma^2 = 3 and 0.5): over
    many samples log k of each layer has mean mu_l and variance sigma_l^2 (the
    sample mean within 5 standard errors, the sample variance within 5 of its
    standard errors sigma^2 sqrt(2 / (N - 1))), and the two layers are
    uncorrelated.  A law written with sigma^2 z instead of sigma z, or with the
    layers' parameters swapped, fails."""
    model = W.PC2.with_(mu=(-1.0, 2.0, 0.0, 0.0), sigma2=(3.0, 0.5, 1.0, 1.0), seed=11)
    n = 6000
    z = np.array([field.layer_constants(model, 0, s) for s in range(n)])
    for l in range(2):
        mu, s2 = model.mu[l], model.sigma2[l]
        assert abs(z[:, l].mean() - mu) <= 5.0 * np.sqrt(s2 / n), (l, z[:, l].mean())
        v = z[:, l].var(ddof=1)
        assert abs(v - s2) <= 5.0 * s2 * np.sqrt(2.0 / (n - 1)), (l, v)
    corr = np.corrcoef(z[:, 0], z[:, 1])[0, 1]
    assert abs(corr) <= 5.0 / np.sqrt(n)
    # the composite field takes exactly these values on its layers
    for s in range(3):
        k = field.sample_k(model, 0, s, 16)
        lid = geometry.layer_ids(model, 0, s, 16)
        assert np.allclose(np.log(k), z[s][lid], rtol=0, atol=1e-14)


def _ce_linear_map(n_ce, m, sigma2, lam, r, dim=2):
    lam_eig = field.ce_eigenvalues(n_ce, m, sigma2, lam, r, dim)
    npts = n_ce ** dim
    cols_re, cols_im = [], []
    for q in range(npts):
        for unit in (1.0, 1.0j):
            xi = np.zeros(npts, dtype=complex)
            xi[q] = unit
            re, im = field.ce_transform(xi.reshape((n_ce,) * dim), lam_eig, m)
            cols_re.append(re.ravel())
            cols_im.append(im.ravel())
    return np.array(cols_re).T, np.array(cols_im).T


def _direct_cov(m, sigma2, lam, r, dim=2):
    x = (np.arange(m) + 0.5) / m
    if dim == 2:
        pts = np.array([(xx, yy) for yy in x for xx in x])
    else:
        pts = np.array([(xx, yy, zz) for zz in x for yy in x for xx in x])
    diff = np.abs(pts[:, None, :] - pts[None, :, :])
    dist = diff.sum(-1) if r == 1 else np.sqrt((diff ** 2).sum(-1))
    return sigma2 * np.exp(-dist / lam)


@pytest.mark.parametrize("n_ce,m,sigma2,lam,r", [
    (8, 4, 1.0, 0.3, 1), (9, 4, 2.0, 0.5, 2), (15, 6, 1.0, 0.2, 2), (12, 5, 0.7, 0.4, 1)])
def test_ce_covariance_identity(n_ce, m, sigma2, lam, r):
    try:
        Mre, Mim = _ce_linear_map(n_ce, m, sigma2, lam, r)
    except ValueError:
        pytest.skip("embedding not valid for this size")
    C = _direct_cov(m, sigma2, lam, r)
    assert np.allclose(Mre @ Mre.T, C, rtol=0, atol=1e-12 * sigma2)
    assert np.allclose(Mim @ Mim.T, C, rtol=0, atol=1e-12 * sigma2)
    assert np.allclose(Mre @ Mim.T, 0.0, atol=1e-12 * sigma2)


def test_ce_covariance_identity_3d():
    n_ce, m = 6, 3
    Mre, Mim = _ce_linear_map(n_ce, m, 1.0, 0.3, 1, dim=3)
    C = _direct_cov(m, 1.0, 0.3, 1, dim=3)
    assert np.allclose(Mre @ Mre.T, C, atol=1e-12)
    assert np.allclose(Mre @ Mim.T, 0.0, atol=1e-12)


def test_ce_refuses_negative_embedding():
    with pytest.raises(ValueError):
        field.ce_eigenvalues(128, 64, 1.0, 0.3, 2)     # 2m is not enough at lambda = 0.3, r = 2
    assert field.min_embedding(64, 1.0, 0.3, 2) == 135


def test_workload_embedding_sizes_are_minimal_and_valid():
    for m, n in W.CE2.n_ce.items():
        assert field.min_embedding(m, 1.0, 0.3, 2) == n


def test_ce_empirical_covariance():
    model = W.STATIONARY_1NORM.with_(norm_r=2, lam=(0.3,) * 4, n_ce={16: 48})
    m, n_ce = 16, 48
    lam_eig = field.ce_eigenvalues(n_ce, m, 1.0, 0.3, 2)
    samples = []
    for s in range(1500):
        re, im = field.ce_pair_sample(model, 0, s, 0, m, n_ce, lam_eig)
        samples.append(re)
        samples.append(im)
    g = np.array(samples)
    N = g.shape[0]
    for lag in (0, 1, 5):
        emp = np.mean(g[:, 3, 2] * g[:, 3, 2 + lag])
        exact = np.exp(-lag / m / 0.3)
        sd = np.sqrt((1.0 + exact ** 2) / N)
        assert abs(emp - exact) < 5 * sd
    # Re and Im parts uncorrelated
    re = g[0::2, 4, 4]
    im = g[1::2, 4, 4]
    assert abs(np.mean(re * im)) < 5 / np.sqrt(re.size)


def test_cgv_sublattices_index_brute_force():
    m = 8
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    k = 1000.0 * j + i
    subs = field.cgv_sublattices(k)
    assert len(subs) == 4
    for idx, sub in enumerate(subs):
        a1, a2 = idx & 1, (idx >> 1) & 1
        for J in range(m // 2):
            for I in range(m // 2):
                assert sub[J, I] == 1000.0 * (2 * J + a2) + (2 * I + a1)
    k3 = np.arange(4 ** 3, dtype=float).reshape(4, 4, 4)   # [x3][x2][x1]
    subs3 = field.cgv_sublattices(k3)
    for idx, sub in enumerate(subs3):
        a = [(idx >> b) & 1 for b in range(3)]
        assert sub[1, 0, 1] == k3[2 + a[2], 0 + a[1], 2 + a[0]]


def test_plain_coarse_sample_piecewise_constant_is_direct_evaluation():
    for s in range(10):
        k, kc = field.sample_k(W.PC2, 2, s, 32, with_coarse=True)
        assert np.array_equal(kc, field.sample_k(W.PC2, 2, s, 16))


def test_plain_coarse_sample_correlated_uses_fine_sublattice():
    model = W.CE2
    m = 32
    k, kc = field.sample_k(model, 1, 3, m, with_coarse=True)
    lid_f = geometry.layer_ids(model, 1, 3, m)
    lid_c = geometry.layer_ids(model, 1, 3, m // 2)
    same = lid_c == lid_f[0::2, 0::2]
    assert np.array_equal(kc[same], k[0::2, 0::2][same])
    g = field.gaussian_layers(model, 1, 3, m)
    diff = ~same
    for l in range(2):
        sel = diff & (lid_c == l)
        assert np.allclose(kc[sel], np.exp(model.mu[l] + g[l][0::2, 0::2][sel]))
