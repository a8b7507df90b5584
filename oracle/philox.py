"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy
as 1, 2, 3", SC'11), written from the published definition.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's stochastic rounding (Sec. III-A) needs one uniform draw per
quantized element.  The paper's own CPU code used XORShift (Sec. IV-C, CPU
implementation); we use a counter-based generator instead so that any element
can be drawn independently, in any order, by the CPU and the GPU alike.

Definition used here
--------------------
State: a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1), all
32-bit words.  One round:

    (hi0, lo0) = 0xD2511F53 * c0        (full 64-bit product)
    (hi1, lo1) = 0xCD9E8D57 * c2
    (c0, c1, c2, c3) <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)

and between rounds the key is bumped by the Weyl constants
(k0 += 0x9E3779B9, k1 += 0xBB67AE85, mod 2^32).  Ten rounds give four
output words.

Counter map for quantization (a reading, the paper fixes no generator):
element e of a stream uses counter (e >> 2 low word, e >> 2 high word,
stream, realization) with key (seed low word, seed high word) and takes
output word e & 3.
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(counters, key):
    """Apply ten Philox4x32 rounds.

    counters : (N, 4) array of uint32-valued integers (c0, c1, c2, c3).
    key      : pair (k0, k1) of 32-bit integers.
    returns  : (N, 4) uint32 array of output words.
    """
    ctr = np.asarray(counters, dtype=np.uint64).reshape(-1, 4)
    c0, c1, c2, c3 = (ctr[:, i].copy() for i in range(4))
    k0 = int(key[0]) & 0xFFFFFFFF
    k1 = int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0  # < 2^64: exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _LO
        hi1, lo1 = p1 >> _S32, p1 & _LO
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return np.stack([c0, c1, c2, c3], axis=1).astype(np.uint32)


def seed_key(seed):
    """Split a 64-bit seed into the Philox key (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def words(seed, stream, realization, e_begin, count):
    """The 32-bit draws for element indices e_begin .. e_begin+count-1.

    Element e uses output word (e & 3) of the block with counter
    (e >> 2, stream, realization).
    """
    count = int(count)
    if count <= 0:
        return np.zeros(0, dtype=np.uint32)
    e_begin = int(e_begin)
    b0 = e_begin >> 2
    b1 = (e_begin + count - 1) >> 2
    blocks = np.arange(b0, b1 + 1, dtype=np.uint64)
    ctr = np.empty((blocks.size, 4), dtype=np.uint64)
    ctr[:, 0] = blocks & _LO
    ctr[:, 1] = blocks >> _S32
    ctr[:, 2] = np.uint64(int(stream) & 0xFFFFFFFF)
    ctr[:, 3] = np.uint64(int(realization) & 0xFFFFFFFF)
    out = philox4x32_10(ctr, seed_key(seed)).reshape(-1)
    first = e_begin - 4 * b0
    return out[first:first + count]
