"""Block sampling for SPDHG.  Test infrastructure only.

The paper requires independent draws with p_i > 0 (Section 3, remark on sampling) and
uses uniform p_i = 1/n or balanced sampling (Section 4.2).  The random stream is the
SplitMix64 generator (G. Steele, D. Lea, C. Flood, OOPSLA 2014), used counter-style:
draw k (0-based) is mix(seed + (k + 1) * 0x9E3779B97F4A7C15 mod 2^64).  A draw maps to
u = (out >> 11) * 2^-53 in [0, 1) and block i = min{i : u < C_i}, with C the in-order
FP64 cumulative sum of p and the last entry set to 1.
"""
from __future__ import annotations

from typing import List

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64_output(state_after_increment: int) -> int:
    z = state_after_increment & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_stream(seed: int, n: int, start: int = 0) -> List[int]:
    """Outputs start .. start+n-1 of SplitMix64 seeded with `seed`."""
    return [splitmix64_output(seed + (k + 1) * GOLDEN) for k in range(start, start + n)]


def cumulative(p) -> List[float]:
    c, acc = [], 0.0
    for v in p:
        acc += float(v)
        c.append(acc)
    c[-1] = 1.0
    return c


def draw_blocks(seed: int, p, n: int, start: int = 0) -> List[int]:
    c = cumulative(p)
    out = []
    for z in splitmix64_stream(seed, n, start):
        u = (z >> 11) * (1.0 / 9007199254740992.0)
        i = 0
        while not (u < c[i]):
            i += 1
        out.append(i)
    return out


def uniform(n: int):
    return [1.0 / n] * n


def balanced(m: int, n_prior: int):
    """Data with probability 1/2 split uniformly over m subsets, prior with 1/2 split
    uniformly over the prior blocks (1/2 for one block; 1/4 each for TGV's two)."""
    if n_prior == 0:
        return uniform(m)
    return [1.0 / (2 * m)] * m + [0.5 / n_prior] * n_prior


def prior_share(m: int, n_prior: int, q: float, q_last: float = 0.0):
    """A constant tuned distribution (Discussion: optimising the sampling): the prior
    blocks together with probability q, the m data blocks uniformly with 1 - q.  With two
    prior blocks (TGV) the last gets q_last (0 < q_last < q) and the other q - q_last; q_last
    = 0 splits q equally.  q = 1/2 is the balanced sampling of Section 4.2."""
    if n_prior == 0:
        return uniform(m)
    if not 0.0 < q < 1.0:
        raise ValueError("prior share must be in (0, 1)")
    data = [(1.0 - q) / m] * m
    if n_prior == 1:
        return data + [q]
    if q_last == 0.0:
        return data + [q / 2.0, q / 2.0]
    if not 0.0 < q_last < q:
        raise ValueError("q_last must be in (0, q)")
    return data + [q - q_last, q_last]
