"""Regression: the oracle and the seeded generator reproduce the stored fixture."""
import json
import os

import numpy as np

import oracle
from paper_1807_09932_amd import gen
from tests.golden.make_golden import digest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_uniform_1000x50_golden():
    ref = json.load(open(os.path.join(HERE, "golden", "uniform_1000x50_counts.json")))
    w, pop = gen.uniform_1000x50()
    offs, cols = gen.csr(pop)
    assert digest(w.X, offs, cols) == ref["inputs_sha256"]
    for key, run in ref["runs"].items():
        include = key.startswith("include")
        negative = key.endswith("neg")
        m, n, mm, nm = oracle.eval_population(w.X, offs, cols, include=include,
                                              negative=negative, masks=True)
        assert m.tolist() == run["matched"] and n.tolist() == run["negative"]
        assert digest(mm, nm) == run["masks_sha256"]
