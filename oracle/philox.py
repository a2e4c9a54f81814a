"""Philox4x32-10 and the Box-Muller transform, FP64 reference.  Test infrastructure only.

The paper only states that the Brownian increments are i.i.d. N(0, dt I)
(Sec. 2.3, eq. Xk).  It names no generator, so the scheme adopts a
counter-based one so that every increment can be regenerated on demand:

* Philox4x32-10 as defined by Salmon, Moraes, Dror and Shaw, "Parallel random
  numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter, a 2x32-bit key,
  ten rounds; each round multiplies counter words 0 and 2 by two fixed odd
  constants, splits the 64-bit products into high/low halves and permutes
  them with xors of the other two words and the round key; the key advances
  by the two Weyl constants (golden ratio and sqrt(3)-1 scaled to 32 bits)
  between rounds.
* Stream layout of the scheme: counter = (g, j, k, q) where g = floor(i/4)
  indexes groups of four coordinates, j the particle, k the time level of the
  increment (the step t_k -> t_{k+1}) and q the evaluation point
  (point_base + p) or 0xFFFFFFFF when increments are shared by all points;
  key = (seed_lo, seed_hi XOR instance).
* Each 32-bit word w maps to a uniform u = (w + 1/2) 2^-32 in (0, 1).
  Box-Muller (1958) turns the pair (u0, u1) into
  z0 = r cos(2 pi u1), z1 = r sin(2 pi u1) with r = sqrt(-2 ln u0), and the
  pair (u2, u3) likewise into z2, z3: coordinate 4g + m takes z_m.
"""
import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_MUL0 = np.uint64(0xD2511F53)
_MUL1 = np.uint64(0xCD9E8D57)
_WEYL0 = np.uint64(0x9E3779B9)
_WEYL1 = np.uint64(0xBB67AE85)
SHARED_STREAM = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 bijection on broadcastable uint32 arrays; returns 4 uint32 arrays."""
    c = [np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = np.broadcast_arrays(*c)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _WEYL0) & _MASK
            k1 = (k1 + _WEYL1) & _MASK
        prod0 = _MUL0 * c0
        prod1 = _MUL1 * c2
        hi0, lo0 = prod0 >> np.uint64(32), prod0 & _MASK
        hi1, lo1 = prod1 >> np.uint64(32), prod1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def key_of(seed, instance):
    """Key words (seed_lo, seed_hi ^ instance) of the scheme's stream layout."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, ((seed >> 32) ^ int(instance)) & 0xFFFFFFFF


def raw_words(seed, instance, stream, k, j, n_groups):
    """Philox words for particles j (array), groups 0..n_groups-1: uint32 [len(j), n_groups, 4]."""
    k0, k1 = key_of(seed, instance)
    jj = np.asarray(j, dtype=np.uint64)[:, None]
    gg = np.arange(n_groups, dtype=np.uint64)[None, :]
    w = philox4x32_10(gg, jj, np.uint64(k), np.uint64(stream), k0, k1)
    return np.stack(w, axis=-1)


def uniforms(words):
    """u = (w + 1/2) 2^-32, strictly inside (0, 1)."""
    return (words.astype(np.float64) + 0.5) * 2.0 ** -32


def box_muller(words):
    """Normals from Philox words [..., 4] -> [..., 4] (Box-Muller on pairs (0,1), (2,3))."""
    u = uniforms(words)
    r01 = np.sqrt(-2.0 * np.log(u[..., 0]))
    r23 = np.sqrt(-2.0 * np.log(u[..., 2]))
    a1 = 2.0 * np.pi * u[..., 1]
    a3 = 2.0 * np.pi * u[..., 3]
    return np.stack([r01 * np.cos(a1), r01 * np.sin(a1),
                     r23 * np.cos(a3), r23 * np.sin(a3)], axis=-1)


def normals(seed, instance, stream, k, M, d):
    """Standard normals xi[j, i] (j < M, i < d) of time level k on the given stream."""
    n_groups = (d + 3) // 4
    z = box_muller(raw_words(seed, instance, stream, k, np.arange(M), n_groups))
    return z.reshape(M, 4 * n_groups)[:, :d]
