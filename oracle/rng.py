"""Random draws of the method from Philox4x64-10 (Salmon et al., SC 2011), FP64 (oracle).

The paper does not fix a generator.  Both the oracle and the GPU library draw from the
counter-based Philox4x64-10 so that the same counters give the same numbers on both
sides.  The oracle takes the block function from numpy's Philox bit generator (a library
implementation of the published definition); the GPU library implements it separately.

Key   = (seed, stream)                       two 64-bit words
Ctr   = (block, w1, purpose, step)            four 64-bit words; one block -> 4 words
purpose: PROBE = 1 (w1 = probe column), ULISSE = 2 (w1 = 2 * system + track),
         SGLD = 3 (w1 = 0)

Mappings of a 64-bit word x:
  uniform in [0, 1)      u = (x >> 11) * 2^-53
  uniform in (0, 1]      u = ((x >> 11) + 1) * 2^-53
  Rademacher             +1 if the top bit of x is 0 else -1
  Gaussian (Box-Muller)  from words (x_a, x_b): r = sqrt(-2 log u1) with u1 in (0, 1],
                         z_a = r cos(2 pi u2), z_b = r sin(2 pi u2) with u2 in [0, 1)
Element i of a stream uses block i // 4 and word i % 4; Gaussians pair words (0, 1) and
(2, 3) of each block.
"""
import numpy as np

PROBE, ULISSE, SGLD = 1, 2, 3
_TWO64 = 1 << 64
_TWO256 = 1 << 256


def blocks(seed, stream, w1, purpose, step, nblocks, first_block=0):
    """Raw Philox4x64-10 output for counters (first_block + b, w1, purpose, step)."""
    key = (int(seed) % _TWO64) | ((int(stream) % _TWO64) << 64)
    ctr = (int(first_block) | (int(w1) << 64) | (int(purpose) << 128)
           | ((int(step) % _TWO64) << 192))
    # numpy increments the counter before producing each block
    bg = np.random.Philox(key=key, counter=(ctr - 1) % _TWO256)
    return bg.random_raw(4 * int(nblocks)).astype(np.uint64).reshape(int(nblocks), 4)


def words(seed, stream, w1, purpose, step, count):
    nb = (int(count) + 3) // 4
    return blocks(seed, stream, w1, purpose, step, nb).reshape(-1)[:count]


def uniform_co(x):
    """[0, 1) from the top 53 bits."""
    return (np.asarray(x, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniform_oc(x):
    """(0, 1] from the top 53 bits."""
    return ((np.asarray(x, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53


def rademacher(x):
    return np.where((np.asarray(x, dtype=np.uint64) >> np.uint64(63)) == 0, 1.0, -1.0)


def box_muller(xa, xb):
    u1 = uniform_oc(xa)
    u2 = uniform_co(xb)
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)


def gaussians(seed, stream, w1, purpose, step, count):
    nb = (int(count) + 3) // 4
    blk = blocks(seed, stream, w1, purpose, step, nb)
    z = np.empty((nb, 4))
    z[:, 0], z[:, 1] = box_muller(blk[:, 0], blk[:, 1])
    z[:, 2], z[:, 3] = box_muller(blk[:, 2], blk[:, 3])
    return z.reshape(-1)[:count]


def probes(seed, stream, step, n, n_probes, kind):
    """Probe matrix R (n, n_probes): kind 0 Gaussian, kind 1 Rademacher (Sec. 2.1)."""
    R = np.empty((n, n_probes))
    for c in range(n_probes):
        if kind == 0:
            R[:, c] = gaussians(seed, stream, c, PROBE, step, n)
        elif kind == 1:
            R[:, c] = rademacher(words(seed, stream, c, PROBE, step, n))
        else:
            raise ValueError("probe kind must be 0 (Gaussian) or 1 (Rademacher)")
    return R


def ulisse_uniform(seed, stream, step, system, track, j):
    """u_j of Sec. 4 for one track of one system: word j of its stream, in [0, 1)."""
    blk = blocks(seed, stream, 2 * system + track, ULISSE, step, 1, first_block=j // 4)
    return float(uniform_co(blk[0, j % 4]))


def sgld_normals(seed, stream, step, count):
    """The standard normals xi of the SGLD noise eta = sqrt(eps) L xi."""
    return gaussians(seed, stream, 0, SGLD, step, count)
