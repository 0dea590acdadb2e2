"""Philox4x32-10 counter-based generator (oracle side; test infrastructure only).

Written from the published definition in Salmon, Moraes, Dror & Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11 (the Philox-4x32 S-box and Weyl key schedule):

* state: four 32-bit counter words c0..c3 and two 32-bit key words k0, k1;
* one round: the two 64-bit products M0*c0 and M1*c2 are split into (hi, lo) halves and the new
  state is (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
* the key is bumped by the Weyl constants (W0, W1) between consecutive rounds;
* ten rounds.

How the field generator turns the output into Gaussian numbers (the stream layout is a reading,
since the paper delegates the initial conditions to an external generator): the 128-bit output
is read as two 64-bit words w_a = c1*2^32 + c0 and w_b = c3*2^32 + c2, and each gives the
uniform u = (2*(w >> 12) + 1) * 2^-53, which is exactly representable and lies strictly inside
(0, 1).
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on arrays of counters (any broadcastable shapes) and one key.

    Returns the four output words as uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd > 0:
            k0 = np.uint64((int(k0) + int(W0)) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + int(W1)) & 0xFFFFFFFF)
        p0 = c0 * M0          # < 2^64: both factors are below 2^32
        p1 = c2 * M1
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def uniforms_from_words(lo, hi):
    """(0,1) uniform from one 64-bit word given as two uint32 halves: (2*(w>>12)+1) * 2^-53."""
    w = (np.asarray(hi, dtype=np.uint64) << _S32) | np.asarray(lo, dtype=np.uint64)
    top = (w >> np.uint64(12)).astype(np.float64)       # < 2^52, exact in float64
    return (2.0 * top + 1.0) * 2.0 ** -53


def mode_uniforms(counter, seed):
    """Two uniforms per 64-bit counter value with the 64-bit seed as key.

    counter -> (c0, c1) = (low, high) 32-bit halves, c2 = c3 = 0; seed -> (k0, k1) likewise.
    """
    counter = np.asarray(counter, dtype=np.uint64)
    lo = counter & _MASK
    hi = counter >> _S32
    seed = int(seed)
    o0, o1, o2, o3 = philox4x32_10(lo, hi, 0, 0, seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return uniforms_from_words(o0, o1), uniforms_from_words(o2, o3)
