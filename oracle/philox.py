"""Philox4x32-10 counter-based generator, vectorised in numpy.

Test infrastructure only (see the package docstring).

Definition (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11): a 4x32-bit counter and a 2x32-bit key; each of the ten
rounds multiplies counter words 0 and 2 by the constants 0xD2511F53 and
0xCD9E8D57 into 64-bit products, and forms the new counter from the high
halves xor-ed with the other two counter words and the key, and the low
halves.  The key is advanced by the Weyl constants 0x9E3779B9 and 0xBB67AE85
between rounds.

The PIC step keys every draw by the particle that makes it: counter =
(id low word, id high word, step, tag), key = (seed low word, seed high word).
One call yields two uniforms in [0, 1) with 53 random bits each:
u = ((w0 << 21) xor (w1 >> 11)) * 2^-53 and the same from (w2, w3).
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four 32-bit output words (as uint64 arrays) of Philox4x32-10.

    All arguments are integers or integer arrays holding 32-bit values; they
    are broadcast against each other.
    """
    c0, c1, c2, c3, k0, k1 = (np.asarray(v, dtype=np.uint64) & _LO
                              for v in (c0, c1, c2, c3, k0, k1))
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _LO
            k1 = (k1 + _W1) & _LO
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _LO
        hi1, lo1 = p1 >> _S32, p1 & _LO
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniforms(ids, step, tag, seed):
    """Two 53-bit uniforms in [0, 1) per id, for the given step and tag.

    ids: uint64 array (particle ids, or node index with bit 63 set for the
    per-node emission draws); step, tag, seed: integers.
    """
    ids = np.asarray(ids, dtype=np.uint64)
    seed = int(seed)
    w0, w1, w2, w3 = philox4x32_10(ids & _LO, ids >> _S32,
                                   np.uint64(step & 0xFFFFFFFF),
                                   np.uint64(tag & 0xFFFFFFFF),
                                   np.uint64(seed & 0xFFFFFFFF),
                                   np.uint64((seed >> 32) & 0xFFFFFFFF))
    s21, s11 = np.uint64(21), np.uint64(11)
    scale = 2.0 ** -53
    ua = ((w0 << s21) ^ (w1 >> s11)).astype(np.float64) * scale
    ub = ((w2 << s21) ^ (w3 >> s11)).astype(np.float64) * scale
    return ua, ub
