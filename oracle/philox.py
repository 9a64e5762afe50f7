"""Philox4x32-10 counter-based generator and Box-Muller normals (oracle side).

The paper draws standard normal variables for the layer values of Example 1
(Section 2; Section 3.4 takes three independent N(0,1) values) and complex
white noise for the circulant-embedding sampler of Example 2 (Section 3.4).
It names no generator.  This build uses Philox4x32-10 (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), restated here
from that definition:

* state: counter c = (c0, c1, c2, c3) of 32-bit words, key k = (k0, k1);
* one round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (64-bit products),
  c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
* between rounds the key is bumped by the Weyl constants W0, W1;
* ten rounds; the output block is the final counter value.

Counter layout used by the whole method (both sides follow it):
c0 = block index, c1 = sample index, c2 = level, c3 = stream tag;
key = (seed & 0xffffffff, seed >> 32).

Uniforms: u = (x + 1/2) * 2^-32, so u lies strictly inside (0, 1).
Normals: Box-Muller, (z0, z1) = sqrt(-2 ln u0) (cos 2 pi u1, sin 2 pi u1),
and (z2, z3) likewise from (u2, u3).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

# stream tags (counter word c3)
TAG_GEOMETRY = 0
TAG_LAYER_CONST = 1
TAG_CE_BASE = 2  # tag 2 + p for circulant-embedding noise of layer pair p

TWO_PI = 2.0 * np.pi


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on broadcastable uint32 counter words.

    Returns a (..., 4) uint32 array holding the output block.
    """
    c = [np.asarray(x, dtype=np.uint64) & MASK32 for x in (c0, c1, c2, c3)]
    c0, c1, c2, c3 = np.broadcast_arrays(*c)
    c0, c1, c2, c3 = (x.copy() for x in (c0, c1, c2, c3))
    key0 = int(k0) & 0xFFFFFFFF
    key1 = int(k1) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            key0 = (key0 + W0) & 0xFFFFFFFF
            key1 = (key1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(key0), lo1,
                          hi0 ^ c3 ^ np.uint64(key1), lo0)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def key_of_seed(seed):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def blocks(seed, sample, level, tag, block_ids):
    """Output blocks for the given block indices of one (sample, level, tag) stream."""
    k0, k1 = key_of_seed(seed)
    return philox4x32_10(np.asarray(block_ids, dtype=np.uint64), sample, level, tag, k0, k1)


def to_uniform(x):
    """uint32 -> double strictly inside (0, 1): (x + 1/2) 2^-32 (exact in FP64)."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def box_muller(u0, u1):
    """Two independent standard normals from two uniforms on (0, 1)."""
    r = np.sqrt(-2.0 * np.log(u0))
    theta = TWO_PI * u1
    return r * np.cos(theta), r * np.sin(theta)


def normals_of_block(blk):
    """(..., 4) uint32 block -> (..., 4) normals (z0, z1, z2, z3)."""
    u = to_uniform(blk)
    z0, z1 = box_muller(u[..., 0], u[..., 1])
    z2, z3 = box_muller(u[..., 2], u[..., 3])
    return np.stack([z0, z1, z2, z3], axis=-1)
