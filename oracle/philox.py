"""Philox4x32-10 counter-based generator (oracle), pure Python integers.

Written from its published definition (J. Salmon, M. Moraes, R. Dror,
D. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4x32-bit
counter is mixed with a 2x32-bit key over 10 rounds; each round multiplies
words 0 and 2 by the constants 0xD2511F53 and 0xCD9E8D57, keeps the high and
low halves of the 64-bit products, and XORs the high halves with the other
two counter words and the round key; the key is bumped by the Weyl
constants 0x9E3779B9 and 0xBB67AE85 between rounds.

Bond kinetics draw u = word0 * 2^-32 for counter (step, ligand, purpose,
instance) and key (seed low word, seed high word).
"""
from __future__ import annotations

MASK32 = 0xFFFFFFFF
M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = (int(v) & MASK32 for v in ctr)
    k0, k1 = (int(v) & MASK32 for v in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK32
        hi1, lo1 = p1 >> 32, p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & MASK32
        k1 = (k1 + W1) & MASK32
    return c0, c1, c2, c3


PURPOSE_FORM = 0
PURPOSE_RUPTURE = 1


def uniform(seed: int, step: int, ligand: int, purpose: int, instance: int = 0) -> float:
    """u in [0, 1): first output word scaled by 2^-32 (exact in FP64)."""
    w = philox4x32_10((step, ligand, purpose, instance), (seed & MASK32, (seed >> 32) & MASK32))
    return w[0] * (1.0 / 4294967296.0)
