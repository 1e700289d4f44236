"""Which rank-code sets a resident matrix holds: the upload builds the SWAR
codes its default plan stages (bytes up to 128 columns, 10-bit codes up to
512), plus the FP16 codes exclude mode needs when cells are missing; the
other code sets (FP16, 16-bit) are built on first use, and results stay
bit-exact."""
import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, gpu_eval, oracle_eval

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_09932_amd.ebic import Context
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("cols,swar", [(64, 8), (200, 10), (400, 10), (600, 0)])
def test_upload_builds_only_what_the_plan_stages(ctx, cols, swar):
    from paper_1807_09932_amd import ebic
    rows = 5_000
    rng = np.random.default_rng(cols)
    X = rng.standard_normal((rows, cols)).astype(np.float32)
    mat = ctx.upload(X)
    st = ctx.stats(mat)
    ld = (rows + 63) // 64 * 64
    assert st["value_bytes"] == ld * cols * 4
    want_sets = {8: ebic.SET_U8, 10: ebic.SET_U10, 0: 0}[swar]
    assert st["code_sets"] == want_sets, st
    assert st["has_missing"] == (0 if swar else -1)
    if swar == 8:
        # whole 512-row units plus one (a 1024-row chunk may start at any unit)
        ldb = ((rows + 511) // 512 + 1) * 512
        assert st["code_bytes"] == ldb * cols + 256 + 4 * (ldb // 512)
        assert st["swar_chunks"] == (rows + 511) // 512
    if swar == 10:
        groups = (rows + 191) // 192
        padded = (groups + 1) // 2 * 2  # (an even count: two-group chunks)
        assert st["code_bytes"] == padded * 256 * cols + 256 + 4 * padded
        assert st["swar_chunks"] == groups
    ctx.release(mat)


def test_16bit_codes_built_on_first_use(ctx):
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(5)
    X = np.round(rng.standard_normal((3_001, 200)), 1).astype(np.float32)
    offs, cols = gen.csr([rng.permutation(200)[: int(rng.integers(1, 25))].astype(np.int32) for _ in range(90)])
    mat = ctx.upload(X)
    assert not ctx.stats(mat)["code_sets"] & ebic.SET_U16
    ctx.set_launch_shape(2, 8, 64, ebic.STAGE_HALVES, 0)
    try:
        assert ebic.ebic_plan_shape(ctx.handle, mat, 90)[3] == ebic.STAGE_HALVES
        got = gpu_eval(ctx, mat, offs, cols)
        assert_same(got, oracle_eval(X, offs, cols), "16-bit codes on first use")
        assert ctx.stats(mat)["code_sets"] & ebic.SET_U16
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_codes_built_on_first_use_and_exact(ctx):
    from paper_1807_09932_amd import ebic
    w = gen.make_matrix(41, 6_007, 64, "normal", 3, (100, 500), (4, 8), nan_fraction=0.0)
    X = w.X
    offs, cols = gen.csr(gen.make_population(41, 1, 64, 150, (1, 15), w.plants))
    mat = ctx.upload(X, fill=0.25, keep_fill_copy=True)
    st = ctx.stats(mat)
    assert st["code_sets"] == ebic.SET_U8 | ebic.SET_FILL_COPY, st
    before = st["code_bytes"]
    ctx.set_launch_shape(4, 8, 64, ebic.STAGE_CODES, 0)
    try:
        # plan reports do not build
        assert ebic.ebic_plan_shape(ctx.handle, mat, 150)[3] == ebic.STAGE_CODES
        assert ctx.stats(mat)["code_sets"] == st["code_sets"]
        for include, built in ((False, ebic.SET_FP16), (True, ebic.SET_FP16_FILL)):
            announce("codes on first use", include)
            got = gpu_eval(ctx, mat, offs, cols, include=include)
            assert_same(got, oracle_eval(X, offs, cols, include=include, fill=0.25), f"include={include}")
            assert ctx.stats(mat)["code_sets"] & built
        after = ctx.stats(mat)["code_bytes"]
        assert after == before + 2 * ((6_007 + 63) // 64 * 64) * 64 * 2
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_missing_cells_get_fp16_codes_at_upload(ctx):
    from paper_1807_09932_amd import ebic
    w = gen.make_matrix(42, 4_001, 64, "normal", 2, (100, 400), (4, 8), nan_fraction=0.05)
    offs, cols = gen.csr(gen.make_population(42, 1, 64, 100, (1, 15), w.plants))
    mat = ctx.upload(w.X)
    st = ctx.stats(mat)
    assert st["has_missing"] == 1
    assert st["code_sets"] == ebic.SET_U8 | ebic.SET_FP16, st
    # a shape asking for byte codes: exclude mode stages the FP16 codes (the
    # byte codes hold the fill value)
    ctx.set_launch_shape(8, 16, 200, ebic.STAGE_BYTES, 0)
    try:
        assert ebic.ebic_plan_shape(ctx.handle, mat, 100)[3] == ebic.STAGE_CODES
        for include in (False, True):
            got = gpu_eval(ctx, mat, offs, cols, include=include)
            assert_same(got, oracle_eval(w.X, offs, cols, include=include), f"include={include}")
    finally:
        ctx.set_launch_shape()
    ctx.release(mat)
