"""Block sampling: SplitMix64 against its published reference outputs, and the draw
frequencies against the probabilities of uniform and balanced sampling."""
import os

import numpy as np

from oracle import sampling as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")


def test_splitmix64_reference_outputs():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    for seed, idx, out in rows:
        assert S.splitmix64_stream(int(seed), 1, start=int(idx))[0] == int(out)


def test_balanced_probabilities():
    p = S.balanced(21, 1)
    assert abs(sum(p) - 1) < 1e-15 and abs(sum(p[:21]) - 0.5) < 1e-15 and p[-1] == 0.5
    p = S.balanced(10, 2)
    assert p[-1] == p[-2] == 0.25
    assert S.balanced(7, 0) == S.uniform(7)


def test_draw_frequencies():
    p = S.balanced(5, 1)
    draws = np.array(S.draw_blocks(123, p, 60000))
    freq = np.bincount(draws, minlength=len(p)) / len(draws)
    exp = np.array(p)
    chi2 = len(draws) * np.sum((freq - exp) ** 2 / exp)
    assert chi2 < 25.0  # 5 dof, p ~ 1e-4
    # counter-based: a stream resumed at k continues exactly
    a = S.draw_blocks(9, p, 100)
    assert S.draw_blocks(9, p, 40, start=60) == a[60:]


def test_prior_share_probabilities():
    """The tuned constant distribution: prior blocks together q, data 1 - q uniformly;
    q = 1/2 reproduces balanced sampling exactly; the draws follow it."""
    for m, npr in ((21, 1), (10, 2), (7, 0)):
        assert S.prior_share(m, npr, 0.5) == S.balanced(m, npr)
    p = S.prior_share(4, 2, 0.3, 0.05)
    assert abs(sum(p) - 1) < 1e-15
    assert p[-1] == 0.05 and abs(p[-2] - 0.25) < 1e-15 and p[0] == 0.7 / 4
    draws = np.array(S.draw_blocks(77, p, 60000))
    freq = np.bincount(draws, minlength=len(p)) / len(draws)
    chi2 = len(draws) * np.sum((freq - np.array(p)) ** 2 / np.array(p))
    assert chi2 < 25.0  # 5 dof
