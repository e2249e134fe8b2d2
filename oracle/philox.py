"""Counter-based random numbers for the oracle (test infrastructure only).

In the paper every random decision of a sweep comes from a counter-based
Philox generator whose key and counter combine the seed, the step, a stream
id per reaction and direction, and the two tags of a pair ordered by size
(Sec. 2.5).  The variant and the placement of these fields in key and
counter are left open; both sides here use:

* generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), 10 rounds,
  multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments
  0x9E3779B9 / 0xBB67AE85;
* key   = (seed, kind << 24 | reaction << 16 | replica);
* counter = (step_lo, step_hi, a, b) where (a, b) is (tag, 0) for per-site
  draws and (min tag, max tag) for per-pair draws; the initial velocities
  use step 0 of the INIT stream.

Everything here is plain integer arithmetic on numpy uint64 arrays holding
32-bit values, written from the published definition of the round function.
"""

import math

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

# Stream kinds: the per-reaction binding and unbinding streams of Sec. 2.5,
# plus one stream for each other random draw of the method.
KIND_THERMO = 1   # Langevin noise, per particle
KIND_ORDER = 2    # order in which reactions are processed in a sweep (Sec. 2.3)
KIND_MATCH = 3    # priority of a proposal in the matching phase
KIND_ON = 4       # acceptance draw of a claimed pair (Eq. pon)
KIND_OFF = 5      # breaking draw of an existing bond (Eq. pon, P_off)
KIND_INIT = 6     # initial Maxwell-Boltzmann velocities, per particle


def stream_key(seed, kind, reaction=0, replica=0):
    """Philox key (k0, k1) of one stream."""
    if not (0 <= reaction < 256 and 0 <= replica < 65536 and 0 <= kind < 256):
        raise ValueError("stream key field out of range")
    return (int(seed) & MASK32, (kind << 24) | (reaction << 16) | replica)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds, vectorised over numpy arrays.

    Inputs are integers or integer arrays (values < 2**32, broadcast against
    each other); returns four uint64 arrays holding the 32-bit output words.
    One round maps (c0, c1, c2, c3) with key (k0, k1) to
        (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))
    and the key is bumped by the Weyl constants between rounds.
    """
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & np.uint64(MASK32)
                      for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & np.uint64(MASK32)
    k1 = np.asarray(k1, dtype=np.uint64) & np.uint64(MASK32)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    w0, w1 = np.uint64(W0), np.uint64(W1)
    msk, sh = np.uint64(MASK32), np.uint64(32)
    for _ in range(10):
        p0 = m0 * c0          # < 2**64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> sh, p0 & msk
        hi1, lo1 = p1 >> sh, p1 & msk
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + w0) & msk
        k1 = (k1 + w1) & msk
    return c0, c1, c2, c3


def step_words(step):
    """Split a 64-bit time step into the two low counter words."""
    step = int(step)
    return step & MASK32, (step >> 32) & MASK32


def u53(w0, w1):
    """Uniform double in [0, 1) from two 32-bit words: 53 random bits."""
    w0 = np.asarray(w0, dtype=np.uint64)
    w1 = np.asarray(w1, dtype=np.uint64)
    bits = (w0 << np.uint64(21)) | (w1 >> np.uint64(11))
    return bits.astype(np.float64) * (2.0 ** -53)


def box_muller3(w0, w1, w2, w3):
    """Three standard normal deviates from one Philox block (Box-Muller).

    u1 = (w + 1) / 2**32 lies in (0, 1], u2 = w' / 2**32 in [0, 1);
    (g0, g1) come from (w0, w1) and g2 from (w2, w3) (its sine partner is
    discarded).
    """
    def pair(a, b):
        u1 = (np.asarray(a, dtype=np.float64) + 1.0) * (2.0 ** -32)
        u2 = np.asarray(b, dtype=np.float64) * (2.0 ** -32)
        rad = np.sqrt(-2.0 * np.log(u1))
        return rad * np.cos(2.0 * math.pi * u2), rad * np.sin(2.0 * math.pi * u2)
    g0, g1 = pair(w0, w1)
    g2, _ = pair(w2, w3)
    return g0, g1, g2


def reaction_order(seed, step, n_reactions):
    """Random processing order of the reactions for the sweep at ``step``.

    The paper redraws the order every sweep so that no reaction is favoured
    by its registration order (Sec. 2.3).  Reading: Fisher-Yates from the
    last position down, position k swapped with j = floor(w * (k+1) / 2**32)
    where w runs through the words of Philox blocks (step, 0, block) of the
    ORDER stream.
    """
    order = list(range(n_reactions))
    if n_reactions < 2:
        return order
    k0, k1 = stream_key(seed, KIND_ORDER)
    s_lo, s_hi = step_words(step)
    words = []
    block = 0
    while len(words) < n_reactions - 1:
        out = philox4x32_10(s_lo, s_hi, 0, block, k0, k1)
        words.extend(int(w) for w in out)
        block += 1
    wi = 0
    for k in range(n_reactions - 1, 0, -1):
        j = (words[wi] * (k + 1)) >> 32
        wi += 1
        order[k], order[j] = order[j], order[k]
    return order
