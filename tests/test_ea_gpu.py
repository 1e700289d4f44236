"""The evaluation driven by the stand-in evolutionary loop: generation after
generation, the GPU counts of the evolving population equal the oracle's
(so both runs follow the same trajectory)."""
import numpy as np
import pytest

from paper_1807_09932_amd import ebic, gen
from tests.gpu_common import announce, oracle_eval, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("workload,include", [("methylation", False), ("missing", False),
                                              ("missing", True)])
def test_ea_trajectory_gpu_equals_oracle(workload, include):
    from paper_1807_09932_amd.ebic import Context
    w = (gen.methylation_436444x64()[0] if workload == "methylation"
         else gen.normal_missing_20000x200()[0])
    rows, n_cols = w.X.shape
    ctx = Context(0)
    mat = ctx.upload(w.X)
    ea = ebic.EA(n_cols, 400, 2, 30 if n_cols >= 30 else n_cols, seed=1000 + len(workload))
    for g in range(6):
        offs, cols, gno = ea.population()
        announce("ea generation", workload, include, gno)
        pop = ctx.population(offsets=offs, cols=cols)
        m, neg, _, _ = ctx.eval(mat, pop, include=include, negative=True)
        gm, gn = to_np(m), to_np(neg)
        om, on, _, _ = oracle_eval(w.X, offs, cols, include=include, negative=True, masks=False)
        assert np.array_equal(gm, om), f"generation {gno}: matched differs"
        assert np.array_equal(gn, on), f"generation {gno}: negative differs"
        ea.step(gm)
    ctx.close()
