"""The oracle reproduces its stored regression values (written by
tests/golden/make_golden.py, which calls only the oracle)."""
import json
import os

import numpy as np
import pytest

from paper_2603_28907_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_bumps_oracle.json")


def test_oracle_matches_golden(oracle_mod):
    g = json.load(open(GOLDEN))
    sc = inputs.tiny_bumps(seed=0)
    counts = oracle_mod.make_counts(sc, seed=1)
    assert int(counts.sum()) == g["counts_sum"]
    assert counts.reshape(-1)[:8].tolist() == g["counts_first8"]
    sc.counts = counts
    prob = oracle_mod.OracleProblem(sc)
    O = prob.opacity(sc.truth)
    np.testing.assert_allclose(O[:32], g["opacity_truth_first32"], rtol=1e-13)
    assert prob.loglik(O) == pytest.approx(g["loglik_truth"], rel=1e-13)
    assert prob.log_prior(sc.truth) == pytest.approx(g["log_prior_truth"], rel=1e-13)
    st = inputs.init_states(sc, 4, seed=2)
    np.testing.assert_allclose(prob.logpost_batch(st), g["logpost_init4"], rtol=1e-13)
