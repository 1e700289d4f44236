"""Ingest to evaluation to export on the GPU: a matrix read from text is
uploaded column-major and evaluated; the counts equal the oracle's on the
original array, and the exported biclusters list the GPU masks' rows."""
import os

import numpy as np
import pytest

from paper_1807_09932_amd import ebic, gen
from tests.gpu_common import announce, assert_same, gpu_eval, oracle_eval
from tests.test_io import _parse_export, _write

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("delim,include", [(",", False), ("\t", True)])
def test_text_to_counts_to_export(tmp_path, delim, include):
    from paper_1807_09932_amd.ebic import Context
    w = gen.make_matrix(70, 5000, 120, "normal", 4, (100, 400), (4, 10), nan_fraction=0.05)
    pop = gen.make_population(70, 0, 120, 300, (2, 20), w.plants)
    offs, cols = gen.csr(pop)
    p = os.path.join(tmp_path, "m.txt")
    _write(p, w.X, delim, True, True)
    Y, rn, cn = ebic.read_delimited(p, threads=8)
    ctx = Context(0)
    mat = ctx.upload(Y)           # column-major source
    announce("io text->eval", delim, include)
    got = gpu_eval(ctx, mat, offs, cols, include=include, negative=True, masks=True)
    assert_same(got, oracle_eval(w.X, offs, cols, include=include, negative=True, masks=True),
                "text-ingested matrix")
    out = os.path.join(tmp_path, "bc.txt")
    ebic.write_biclusters(out, Y.shape[0], offs, cols, got[2], [0, 3], rn, cn)
    for (nr, k, rr, cc), i in zip(_parse_export(out), [0, 3]):
        bits = np.unpackbits(got[2][i].view(np.uint8), bitorder="little")[:Y.shape[0]]
        assert nr == got[0][i] and rr == [rn[r] for r in np.nonzero(bits)[0]]
    ctx.close()
