"""Pins of the oracle's Philox4x32-10 and of the DE draw conventions.

Philox is pinned to the published known-answer vectors; the draw mapping
(indices of rand/1, crossover uniforms) to the properties DE/rand/1/bin
needs: distinct indices, uniform over the admissible members, uniforms in
(0, 1).
"""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            w = [int(v, 16) for v in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    assert oracle.philox4x32_10(ctr, key) == expect


def test_counter_words_all_matter():
    base = oracle.draw_words(7, 3, 1, 2, oracle.TAG_MUT, 0)
    assert oracle.draw_words(7, 3, 1, 2, oracle.TAG_MUT, 0) == base
    for alt in [(8, 3, 1, 2, oracle.TAG_MUT, 0), (7, 4, 1, 2, oracle.TAG_MUT, 0),
                (7, 3, 2, 2, oracle.TAG_MUT, 0), (7, 3, 1, 3, oracle.TAG_MUT, 0),
                (7, 3, 1, 2, oracle.TAG_XOVER, 0), (7, 3, 1, 2, oracle.TAG_MUT, 1),
                (7, 3 | (5 << 32), 1, 2, oracle.TAG_MUT, 0)]:
        assert oracle.draw_words(*alt) != base


@pytest.mark.parametrize("P", [4, 5, 8, 32, 40])
def test_mutation_indices_distinct(P):
    for g in range(1, 40):
        for i in range(P):
            r1, r2, r3, jr, U = oracle.de_draws(11, 0, g, i, P, 5)
            assert len({i, r1, r2, r3}) == 4
            assert all(0 <= r < P for r in (r1, r2, r3))
            assert 0 <= jr < 5
            assert np.all((U > 0) & (U < 1))


def test_mutation_indices_uniform():
    # For P = 6, target i = 2: r1 is uniform over the 5 others, and the
    # ordered triple (r1, r2, r3) is uniform over the 5*4*3 = 60 admissible ones.
    P, i, n = 6, 2, 12000
    counts1 = {}
    triples = {}
    for g in range(1, n + 1):
        r1, r2, r3, jr, _ = oracle.de_draws(5, 9, g, i, P, 4)
        counts1[r1] = counts1.get(r1, 0) + 1
        triples[(r1, r2, r3)] = triples.get((r1, r2, r3), 0) + 1
    assert set(counts1) == {0, 1, 3, 4, 5}
    assert len(triples) == 60
    exp1 = n / 5.0
    chi1 = sum((c - exp1) ** 2 / exp1 for c in counts1.values())
    exp3 = n / 60.0
    chi3 = sum((c - exp3) ** 2 / exp3 for c in triples.values())
    # 99.9 % quantiles of chi-square with 4 and 59 degrees of freedom
    assert chi1 < 18.47
    assert chi3 < 98.3


def test_crossover_uniforms_uniform():
    U = np.concatenate([oracle.de_draws(1, 2, g, 0, 8, 6)[4] for g in range(1, 4001)])
    hist, _ = np.histogram(U, bins=10, range=(0, 1))
    exp = U.size / 10
    assert ((hist - exp) ** 2 / exp).sum() < 27.88  # 99.9 % of chi-square(9)
    jr = [oracle.de_draws(1, 2, g, 0, 8, 5)[3] for g in range(1, 5001)]
    c = np.bincount(jr, minlength=5)
    assert ((c - 1000.0) ** 2 / 1000.0).sum() < 18.47
