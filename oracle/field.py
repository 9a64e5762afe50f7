"""Layered permeability samples at cell centres (oracle side).

* Example 1 (Section 2): on layer l the permeability is the constant
  exp(Z_l), Z_l ~ N(mu_l, sigma_l^2).  Z_l = mu_l + sqrt(sigma2_l) z_l with
  z_l the l-th normal of block 0 of the layer-constant stream (tag 1).
* Example 2 (Section 2, eq. (2.3)): on layer l the permeability is
  exp(g_l(x)), g_l a stationary Gaussian field with mean mu_l and covariance
  sigma_l^2 exp(-||x - y||_r / lambda_l).  Section 3.4 samples such fields by
  circulant embedding (Wood and Chan 1994; Dietrich and Newsam 1997), which
  is exact on a regular grid.  The method, in order:
    1. first row of the covariance matrix of the embedding torus of
       n_ce^d points with spacing h = 1/m, distance per axis min(a, n_ce-a) h;
    2. its eigenvalues Lambda = FFT(first row) (forward DFT, exp(-2 pi i jk/N));
    3. embedding check: min Lambda >= -1e-12 max Lambda, then Lambda <- max(Lambda, 0);
    4. white noise xi = xi_re + i xi_im on the n_ce^d frequencies;
    5. y = FFT(sqrt(Lambda / n_ce^d) * xi): Re y and Im y are two
       independent samples of the zero-mean field on the torus;
    6. keep the grid points [0, m)^d.
  Layers share embedding samples ("pairs") only when their (sigma^2, lambda)
  agree: layer l, in order, takes the Im part of the first earlier pair with
  its own (sigma^2, lambda) whose Im part is still free, and otherwise opens a
  new pair and takes its Re part.  Pair p draws its noise from stream tag
  2 + p and uses the eigenvalues of its own covariance (Section 3.4's three
  layers: bottom and top with lambda 0.3 share pair 0 as Re and Im, the middle
  layer with lambda 0.1 has pair 1).  Equal parameters give layers 2p, 2p+1
  the Re and Im parts of pair p.  Noise point (k2, k1) takes (z0, z1) of block
  (k2 // 2) n_ce + k1 when k2 is even and (z2, z3) of that block when k2 is
  odd (3-D: block ((k3 n_ce + k2) // 2) n_ce + k1 with the same parity rule
  on k3 n_ce + k2).  All layers share the norm r and the embedding size.
* The composite sample is k(x_ij) = exp(mu_l + g_l(x_ij)) with l the layer
  of the cell centre (Section 2: the partition is independent of k).
* Plain MLMC coarse sample (eq. (3.6): coarse and fine from the same omega):
  layer of each coarse centre re-evaluated on the coarse grid; piecewise
  constant layers keep their value; correlated layers take the Gaussian
  value of the fine cell (2I, 2J), i.e. the fine sub-lattice a = 0, which by
  stationarity is a valid coarse-grid sample of g.
* Coarse Grid Variates (Section 4.1, eq. (4.1)): the 2^d sub-lattices
  k^(a)(I) = k(2I + a), a in {0,1}^d, of the fine composite sample; sub-lattice
  index j = a1 + 2 a2 (+ 4 a3).
"""
import numpy as np

from . import geometry, philox

PIECEWISE_CONSTANT = 0
CORRELATED_CE = 1

EMBED_TOL = 1e-12


# ----------------------------------------------------------------- Example 1

def layer_constants(model, level, sample):
    """Gaussian layer values Z_l = mu_l + sqrt(sigma2_l) z_l (Example 1)."""
    blk = philox.blocks(model.seed, sample, level, philox.TAG_LAYER_CONST, [0])
    z = philox.normals_of_block(blk)[0]
    n = model.n_layers
    return np.array([model.mu[l] + np.sqrt(model.sigma2[l]) * z[l] for l in range(n)])


# ------------------------------------------------------------ Example 2 (CE)

def ce_first_row(n_ce, m, sigma2, lam, norm_r, dim):
    """Covariance eq. (2.3) between grid point 0 and every point of the torus."""
    h = 1.0 / m
    a = np.arange(n_ce)
    dist1 = np.minimum(a, n_ce - a) * h
    if dim == 2:
        dx = dist1[None, :]
        dy = dist1[:, None]
        if norm_r == 1:
            dist = dx + dy
        else:
            dist = np.sqrt(dx * dx + dy * dy)
    else:
        dx = dist1[None, None, :]
        dy = dist1[None, :, None]
        dz = dist1[:, None, None]
        if norm_r == 1:
            dist = dx + dy + dz
        else:
            dist = np.sqrt(dx * dx + dy * dy + dz * dz)
    return sigma2 * np.exp(-dist / lam)


def ce_eigenvalues(n_ce, m, sigma2, lam, norm_r, dim=2):
    """Eigenvalues of the circulant embedding; raises if the embedding is not
    non-negative definite (then the sampler would not be exact)."""
    c = ce_first_row(n_ce, m, sigma2, lam, norm_r, dim)
    lam_eig = np.fft.fftn(c).real
    lmax = lam_eig.max()
    if lam_eig.min() < -EMBED_TOL * lmax:
        raise ValueError("circulant embedding of size %d is not non-negative "
                         "(min/max = %.3e)" % (n_ce, lam_eig.min() / lmax))
    return np.maximum(lam_eig, 0.0)


def smooth_sizes(lo, hi):
    """Integers in [lo, hi] with no prime factor above 5, ascending."""
    out = []
    for n in range(lo, hi + 1):
        r = n
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            out.append(n)
    return out


def min_embedding(m, sigma2, lam, norm_r, dim=2, limit=12):
    """Smallest 5-smooth n_ce >= 2m whose embedding is non-negative."""
    for n in smooth_sizes(2 * m, limit * m):
        try:
            ce_eigenvalues(n, m, sigma2, lam, norm_r, dim)
            return n
        except ValueError:
            continue
    raise ValueError("no valid embedding up to %d m" % limit)


def ce_noise(model, level, sample, pair, n_ce, dim):
    """Complex white noise xi on the n_ce^d frequencies (layout [..., k2, k1])."""
    rows = n_ce ** (dim - 1)              # index of the line along x1: k2 (2-D), k3 n + k2 (3-D)
    row = np.arange(rows)[:, None]
    k1 = np.arange(n_ce)[None, :]
    b = (row // 2) * n_ce + k1
    nblk = ((rows + 1) // 2) * n_ce
    blk = philox.blocks(model.seed, sample, level, philox.TAG_CE_BASE + pair, np.arange(nblk))
    z = philox.normals_of_block(blk)
    even = (row % 2) == 0
    re = np.where(even, z[b, 0], z[b, 2])
    im = np.where(even, z[b, 1], z[b, 3])
    return (re + 1j * im).reshape((n_ce,) * dim)


def ce_transform(xi, lam_eig, m):
    """Circulant embedding sample (Section 3.4, covariance eq. (2.3)): the
    scaled noise sqrt(Lambda / n_ce^d) xi transformed by the forward DFT,
    y = FFT(sqrt(Lambda / n_ce^d) xi); Re y and Im y restricted to the grid
    points [0, m)^d."""
    dim = xi.ndim
    n_ce = xi.shape[0]
    y = np.fft.fftn(np.sqrt(lam_eig / float(n_ce ** dim)) * xi)
    sl = (slice(0, m),) * dim
    return y.real[sl].copy(), y.imag[sl].copy()


def ce_pair_sample(model, level, sample, pair, m, n_ce, lam_eig):
    """Two independent zero-mean Gaussian fields on [0, m)^d (Re and Im)."""
    xi = ce_noise(model, level, sample, pair, n_ce, model.dim)
    return ce_transform(xi, lam_eig, m)


def ce_pairs(model):
    """Embedding samples of a correlated model, in order: [sigma2, lambda,
    [layer taking Re, layer taking Im or None]] (rule in the module doc)."""
    pairs = []
    for l in range(model.n_layers):
        key = (float(model.sigma2[l]), float(model.lam[l]))
        for p in pairs:
            if (p[0], p[1]) == key and p[2][1] is None:
                p[2][1] = l
                break
        else:
            pairs.append([key[0], key[1], [l, None]])
    return pairs


def gaussian_layers(model, level, sample, m, n_ce=None, lam_eig=None):
    """Zero-mean Gaussian field of every layer at the m^d cell centres.
    lam_eig: eigenvalues for pairs with the covariance of layer 0 (optional)."""
    if n_ce is None:
        n_ce = model.n_ce[m]
    g = [None] * model.n_layers
    for p, (sigma2, lam, (l_re, l_im)) in enumerate(ce_pairs(model)):
        if lam_eig is not None and (sigma2, lam) == (model.sigma2[0], model.lam[0]):
            eig = lam_eig
        else:
            eig = ce_eigenvalues(n_ce, m, sigma2, lam, model.norm_r, model.dim)
        re, im = ce_pair_sample(model, level, sample, p, m, n_ce, eig)
        g[l_re] = re
        if l_im is not None:
            g[l_im] = im
    return g


def check_ce_model(model):
    if not 1 <= model.n_layers <= 4:
        raise ValueError("1 to 4 layers")


# ------------------------------------------------------------ composite k

def sample_k(model, level, sample, m, lam_eig=None, with_coarse=False):
    """Permeability at the cell centres of an m^d grid for sample (level, sample).

    Returns k, or (k, k_coarse_plain) when with_coarse is true (m even).
    """
    lid = geometry.layer_ids(model, level, sample, m)
    if model.field_kind == PIECEWISE_CONSTANT:
        z = layer_constants(model, level, sample)
        k = np.exp(z[lid])
        if not with_coarse:
            return k
        lid_c = geometry.layer_ids(model, level, sample, m // 2)
        return k, np.exp(z[lid_c])
    if model.field_kind == CORRELATED_CE:
        check_ce_model(model)
        g = gaussian_layers(model, level, sample, m, lam_eig=lam_eig)
        logk = np.zeros_like(g[0])
        for l in range(model.n_layers):
            logk = np.where(lid == l, model.mu[l] + g[l], logk)
        k = np.exp(logk)
        if not with_coarse:
            return k
        mc = m // 2
        lid_c = geometry.layer_ids(model, level, sample, mc)
        sub = (slice(0, m, 2),) * model.dim
        logk_c = np.zeros(lid_c.shape)
        for l in range(model.n_layers):
            logk_c = np.where(lid_c == l, model.mu[l] + g[l][sub], logk_c)
        return k, np.exp(logk_c)
    raise ValueError("unknown field kind %r" % model.field_kind)


def cgv_sublattices(k):
    """The 2^d coarse samples k^(a)(I) = k(2I + a) of eq. (4.1), a = bits of j."""
    d = k.ndim
    out = []
    for j in range(2 ** d):
        a = [(j >> b) & 1 for b in range(d)]          # a[0] along x1, a[1] along x2, ...
        sl = tuple(slice(a[ax], None, 2) for ax in reversed(range(d)))
        out.append(k[sl].copy())
    return out
