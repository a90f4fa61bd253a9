"""Mutation test of the oracle's pins: each planted mistake in bbc_oracle.c
(built with -DORC_MUTANT=k) must make at least one pin fail. This shows that
the pins constrain every part of the oracle: the butterfly predicate, the
wedge type, C(n,3), the candidate prune, the class sum, the operands of the
intersection, the per-vertex attribution, the brute-force edge check and the
priority filter."""
import os
import tempfile

import numpy as np
import pytest

from paper_2605_03603_amd import generators as G
from tests import test_oracle_pins as P


def _pins(O):
    """A fast subset of the pins; returns the first failure (or None)."""
    checks = [
        ("fig2", lambda: P.test_fig2_butterfly_balance(O)),
        ("fig3b", lambda: P.test_fig3b_wedge_types(O)),
        ("fig1b", lambda: P.test_fig1b_signed_k44(O)),
        ("complete", lambda: P.test_complete_all_positive(O, 5, 6)),
        ("two_block", lambda: P.test_two_block_closed_form(O, 3, 4, 4, 3)),
        ("choose3", lambda: P.test_choose3_exact(O)),
        ("blocks", lambda: P.test_disjoint_planted_blocks_additive(O)),
    ]

    def tiny():
        rng = np.random.default_rng(11)
        for _ in range(400):
            g = G.tiny_random(rng, 7, 7)
            b, pu, pv = O.count_bruteforce(g, per_vertex=True)
            r0 = O.count_bbvp(g, 0, per_vertex=True)
            assert r0["total"] == b and (r0["per_vertex"] == pu).all()
            assert O.count_bbvp(g, 1)["total"] == b
    checks.append(("tiny", tiny))
    for name, fn in checks:
        try:
            fn()
        except AssertionError:
            return name
    return None


@pytest.mark.parametrize("mutant", list(range(1, 10)))
def test_every_mutant_is_caught(oracle, mutant):
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build(out=os.path.join(d, f"mut{mutant}.so"), mutant=mutant)
        oracle.use_library(path)
        try:
            caught = _pins(oracle)
        finally:
            oracle.use_library(None)
    assert caught is not None, f"mutant {mutant} passed every pin"


def test_unmutated_passes_subset(oracle):
    assert _pins(oracle) is None
