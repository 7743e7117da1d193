"""Writes the stored expected values under tests/golden/ by calling only the
oracle (and the seeded input generators).  Run from the repository root:
    python tests/golden/make_golden.py
The paper prints no worked numerical example, so these fixtures are oracle
regression values on the small three-surface cave (16x16 grid over 100 m,
2 sensors x 32x32 pixels, seeds as below)."""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2603_28907_amd import inputs  # noqa: E402


def main():
    sc = inputs.tiny_bumps(seed=0)
    counts = oracle.make_counts(sc, seed=1)
    sc.counts = counts
    prob = oracle.OracleProblem(sc)
    states = inputs.init_states(sc, 4, seed=2)
    O_truth = prob.opacity(sc.truth)
    out = {
        "what": "oracle regression values, small three-surface cave (tiny_bumps seed 0, counts seed 1, "
                "init_states seed 2)",
        "counts_sum": int(counts.sum()),
        "counts_first8": counts.reshape(-1)[:8].tolist(),
        "opacity_truth_first32": O_truth[:32].tolist(),
        "loglik_truth": prob.loglik(O_truth),
        "log_prior_truth": prob.log_prior(sc.truth),
        "logpost_init4": prob.logpost_batch(states).tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_bumps_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
