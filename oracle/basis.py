"""Oracle basis: restricted Hilbert spaces by brute-force filtering.

Follows Sec. 3.1 of the paper: a configuration is a bit string (site i
is bit i, bit 0 least significant; for fermions orbital 2*site + sigma
with sigma = 0 up, 1 down, so a 4-ary site digit is split into two bits
with up in the low bit).  A canonical (restricted) space is the set of
configurations with a fixed total Sz (spins) or fixed particle numbers
(fermions), kept in ascending integer order as in the 4-site example of
Sec. 3.3.

The product path ranks through split lookup tables; the oracle instead
enumerates every bit string, filters, sorts and ranks by binary search,
plus an independent combinatorial-number-system rank for fixed-popcount
spaces too large to enumerate.
"""

from __future__ import annotations

from math import comb

import numpy as np

EVEN64 = np.uint64(0x5555555555555555)
ODD64 = np.uint64(0xAAAAAAAAAAAAAAAA)


def n_bits(desc) -> int:
    return desc.n_sites if desc.particle == "spin" else 2 * desc.n_sites


def in_sector(desc, states: np.ndarray) -> np.ndarray:
    """Boolean mask: which bit strings belong to the sector of desc."""
    s = np.asarray(states, dtype=np.uint64)
    if desc.sector == "none":
        return np.ones(s.shape, dtype=bool)
    if desc.particle == "spin":
        if desc.sector != "sz":
            raise ValueError("spin sector must be 'none' or 'sz'")
        n_up = (desc.n_sites + desc.two_sz) // 2
        return np.bitwise_count(s) == n_up
    if desc.sector == "nupndn":
        return (np.bitwise_count(s & EVEN64) == desc.n_up) & (np.bitwise_count(s & ODD64) == desc.n_dn)
    if desc.sector == "ntot":
        return np.bitwise_count(s) == desc.n_tot
    raise ValueError(f"bad sector {desc.sector!r}")


def states(desc) -> np.ndarray:
    """All configurations of the space, ascending (brute force over 2^nbits)."""
    nb = n_bits(desc)
    if nb > 28:
        raise ValueError("oracle enumeration limited to 28 bits; use cns_rank for sampled rows")
    allst = np.arange(1 << nb, dtype=np.uint64)
    if desc.sector == "none":
        return allst
    return np.sort(allst[in_sector(desc, allst)])


def rank(basis_states: np.ndarray, cfg: np.ndarray) -> np.ndarray:
    """Index of each configuration in the ascending list, -1 if absent."""
    cfg = np.asarray(cfg, dtype=np.uint64)
    idx = np.searchsorted(basis_states, cfg)
    idx_c = np.minimum(idx, len(basis_states) - 1)
    ok = basis_states[idx_c] == cfg
    return np.where(ok, idx_c, -1).astype(np.int64)


def dimension(desc) -> int:
    """Dimension from binomial counting."""
    n = desc.n_sites
    if desc.sector == "none":
        return 1 << n_bits(desc)
    if desc.particle == "spin":
        n_up = (n + desc.two_sz) // 2
        return comb(n, n_up) if 0 <= n_up <= n and (n + desc.two_sz) % 2 == 0 else 0
    if desc.sector == "nupndn":
        return comb(n, desc.n_up) * comb(n, desc.n_dn)
    return comb(2 * n, desc.n_tot)


# ----------------------------------------------------- combinatorial number system

def cns_rank(s: int) -> int:
    """Rank of s among all integers with the same popcount, ascending.

    With set-bit positions p_1 < p_2 < ... < p_k the rank is
    sum_i C(p_i, i): the count of same-popcount integers below s.
    """
    r = 0
    i = 0
    pos = 0
    while s:
        if s & 1:
            i += 1
            r += comb(pos, i)
        s >>= 1
        pos += 1
    return r


def cns_unrank(r: int, k: int, nbits: int) -> int:
    """Inverse of cns_rank for popcount k: greedy choice of the highest bit first."""
    s = 0
    for i in range(k, 0, -1):
        p = i - 1
        while p + 1 < nbits and comb(p + 1, i) <= r:
            p += 1
        r -= comb(p, i)
        s |= 1 << p
    if r != 0:
        raise ValueError("rank out of range")
    return s


# -------------------------------------------- sector rank by counting (any sector kind)

def _completions(desc, p: int, need) -> int:
    """Configurations of the p bits below position p holding the still-needed
    particles `need` (a count, or (up, down) for the interleaved fermion sector)."""
    if desc.sector == "nupndn":
        n_even = (p + 1) // 2          # even positions 0, 2, ... below p
        n_odd = p // 2
        return comb(n_even, need[0]) * comb(n_odd, need[1]) if need[0] >= 0 and need[1] >= 0 else 0
    return comb(p, need) if need >= 0 else 0


def _initial_need(desc):
    if desc.sector == "nupndn":
        return (desc.n_up, desc.n_dn)
    if desc.particle == "spin":
        return (desc.n_sites + desc.two_sz) // 2
    return desc.n_tot


def _take(desc, need, p):
    """Needs after placing a particle at position p."""
    if desc.sector == "nupndn":
        return (need[0] - 1, need[1]) if p % 2 == 0 else (need[0], need[1] - 1)
    return need - 1


def sector_rank(desc, s: int) -> int:
    """Index of configuration s in the ascending list of its sector (Sec. 3.1),
    by counting: for each set bit of s, from the top, the sector configurations
    that agree with s above it and have a 0 there."""
    if desc.sector == "none":
        return int(s)
    need = _initial_need(desc)
    r = 0
    for p in range(n_bits(desc) - 1, -1, -1):
        if (s >> p) & 1:
            r += _completions(desc, p, need)
            need = _take(desc, need, p)
    return r


def sector_unrank(desc, r: int) -> int:
    """Inverse of sector_rank: greedy from the top bit."""
    if desc.sector == "none":
        return int(r)
    need = _initial_need(desc)
    s = 0
    for p in range(n_bits(desc) - 1, -1, -1):
        zero = _completions(desc, p, need)
        if r >= zero:
            r -= zero
            s |= 1 << p
            need = _take(desc, need, p)
    if r != 0:
        raise ValueError("rank out of range")
    return s
