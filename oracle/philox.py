"""Philox4x32-10 counter-based random numbers (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), vectorised in numpy.

One block maps a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1) to
four 32-bit words through 10 rounds.  A round multiplies c0 and c2 by the
constants M0 = 0xD2511F53 and M1 = 0xCD9E8D57 into 64-bit products and mixes
    (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0));
between rounds the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85).

The paper draws scattering events with probability p_sc = Ndot dt per
particle and step (Sec. 3); this project keys every draw by (step, particle id,
stream) so that the draw of a particle does not depend on how the particle
arrays are laid out.  Pins: the published known-answer vectors and an
independent implementation (tests/test_oracle_philox.py).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)

# Stream tags: the fourth counter word of every draw of the method.
STREAM_INIT = 1       # initial positions / momenta
STREAM_RICS = 2       # scattering-event decision
STREAM_CHILD = 3      # ids of the pair created by a converting photon
STREAM_ATM_A = 4      # atmosphere: position and electron momentum
STREAM_ATM_B = 5      # atmosphere: ion momentum
STREAM_ATM_ID = 6     # atmosphere: ids of the injected electron and ion
STREAM_ANNIH = 7      # pair annihilation: ranking key of every e-/e+ in a cell over n_max

HASHED_ID_BIT = np.uint64(1) << np.uint64(63)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 block.  All inputs broadcast as uint32 arrays.

    Returns four uint32 arrays (the output words r0..r3).
    """
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        n0 = (p1 >> np.uint64(32)) ^ c1 ^ k0
        n1 = p1 & MASK32
        n2 = (p0 >> np.uint64(32)) ^ c3 ^ k1
        n3 = p0 & MASK32
        c0, c1, c2, c3 = n0, n1, n2, n3
        if r < 9:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def seed_key(seed):
    """Split a 64-bit seed into the two key words."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniform24(word):
    """U in [0, 1) from the top 24 bits of a word: (w >> 8) * 2^-24 (exact in float32)."""
    return (np.asarray(word, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) * 2.0 ** -24


def uniform24_open0(word):
    """U in (0, 1]: ((w >> 8) + 1) * 2^-24, for logarithms."""
    return ((np.asarray(word, dtype=np.uint32) >> np.uint32(8)).astype(np.float64) + 1.0) * 2.0 ** -24


def id_from_words(w_lo, w_hi):
    """A 64-bit particle id built from two output words, tagged with the top bit."""
    v = (np.asarray(w_hi, dtype=np.uint64) << np.uint64(32)) | np.asarray(w_lo, dtype=np.uint64)
    return v | HASHED_ID_BIT


def split_id(pid):
    pid = np.asarray(pid, dtype=np.uint64)
    return (pid & MASK32).astype(np.uint32), (pid >> np.uint64(32)).astype(np.uint32)
