"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).

A block maps a 256-bit counter (four 64-bit words) and a 128-bit key (two
words) to four pseudo-random 64-bit words through ten rounds.  One round
multiplies counter words 0 and 2 by two fixed odd constants, keeps the 128-bit
products' high and low halves, and recombines them with words 1 and 3 and the
key; between rounds the key is advanced by two Weyl increments (the golden
ratio and sqrt(3) - 1 in 64-bit fixed point).

Stream layout used by the trajectory method (the paper only asks for uniform
r in [0, 1), Sec. 2.1, MCWF steps 2 and 5; the layout is this library's):

  counter = [ordinal n, iteration, direction (0 forward / 1 backward), 0]
  key     = [seed, (instance << 32) | trajectory]

Word 0 of block n gives the norm threshold r that ends waiting period n; word
1 of block n picks the jump operator of the jump that ends period n.  A 64-bit
word w maps to the uniform double (w >> 11) * 2^-53 in [0, 1).
"""

from __future__ import annotations

MASK64 = (1 << 64) - 1
MUL0 = 0xD2E7470EE14C6C93
MUL1 = 0xCA5A826395121157
WEYL0 = 0x9E3779B97F4A7C15
WEYL1 = 0xBB67AE8584CAA73B
ROUNDS = 10


def block(counter, key):
    """Return the four output words of Philox4x64-10 for (counter, key)."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in counter)
    k0, k1 = (int(x) & MASK64 for x in key)
    for rnd in range(ROUNDS):
        if rnd:
            k0 = (k0 + WEYL0) & MASK64
            k1 = (k1 + WEYL1) & MASK64
        p0 = MUL0 * c0
        p1 = MUL1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ c3 ^ k1, p0 & MASK64)
    return c0, c1, c2, c3


def to_unit(word: int) -> float:
    """Uniform double in [0, 1) from the top 53 bits of a 64-bit word."""
    return (int(word) >> 11) * (2.0 ** -53)


class TrajectoryStream:
    """Random numbers of one trajectory in one propagation pass."""

    def __init__(self, seed: int, trajectory: int, iteration: int, direction: int,
                 instance: int = 0):
        self.key = (seed, ((instance & 0xFFFFFFFF) << 32) | (trajectory & 0xFFFFFFFF))
        self.iteration = iteration
        self.direction = direction

    def _block(self, ordinal: int):
        return block((ordinal, self.iteration, self.direction, 0), self.key)

    def threshold(self, ordinal: int) -> float:
        """r for waiting period ``ordinal`` (MCWF steps 2 and 5)."""
        return to_unit(self._block(ordinal)[0])

    def choice(self, ordinal: int) -> float:
        """Uniform variate that selects L_l for the jump ending period ``ordinal``."""
        return to_unit(self._block(ordinal)[1])
