"""Parity of the HIP path with the CPU oracle, bit-exact (tolerance 0: the
outputs are integers decided by exact FP32 compares), through the C ABI."""
import numpy as np
import pytest

from paper_1807_09932_amd import gen
from tests.gpu_common import announce, assert_same, gpu_eval, oracle_eval, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1807_09932_amd.ebic import Context
    c = Context(0)
    yield c
    c.close()


def _special(rng, shape, nan_frac=0.0):
    alpha = np.array([-np.inf, -1.0, -0.0, 0.0, 1.4e-45, 2.8e-45, 1.0, 2.0, np.inf],
                     dtype=np.float32)
    X = alpha[rng.integers(0, alpha.size, size=shape)]
    if nan_frac:
        X[rng.random(shape) < nan_frac] = np.float32(np.nan)
    return X


def _random_pop(rng, ncols, n, kmax, dup=0.0, bad=0.0):
    inds = []
    for _ in range(n):
        k = int(rng.integers(1, kmax + 1))
        if rng.random() < dup:
            ind = rng.integers(0, ncols, size=k)
        else:
            ind = rng.permutation(ncols)[:min(k, ncols)]
        if rng.random() < bad:
            ind = np.append(ind, ncols + int(rng.integers(0, 3)))
        inds.append(np.asarray(ind, np.int32))
    return gen.csr(inds)


@pytest.mark.parametrize("include", [False, True])
@pytest.mark.parametrize("negative", [False, True])
def test_uniform_1000x50_plain(ctx, include, negative):
    w, pop = gen.uniform_1000x50()
    offs, cols = gen.csr(pop)
    mat = ctx.upload(w.X)
    announce("uniform_1000x50", include, negative)
    got = gpu_eval(ctx, mat, offs, cols, include=include, negative=negative)
    want = oracle_eval(w.X, offs, cols, include=include, negative=negative)
    assert_same(got, want, "uniform_1000x50")
    ctx.release(mat)


@pytest.fixture(scope="module")
def cfg2():
    return gen.normal_missing_20000x200()


@pytest.mark.parametrize("include,fill", [(False, 0.0), (True, 0.0), (True, 999.0)])
def test_normal_missing_values(ctx, cfg2, include, fill):
    w, pop = cfg2
    offs, cols = gen.csr(pop)
    mat = ctx.upload(w.X, fill=fill)
    announce("normal_missing_20000x200", include, fill)
    got = gpu_eval(ctx, mat, offs, cols, include=include)
    want = oracle_eval(w.X, offs, cols, include=include, fill=fill)
    assert_same(got, want, f"normal_missing_20000x200 include={include} fill={fill}")
    ctx.release(mat)


def test_methylation_436444x64_full(ctx):
    """436,444 rows x 64 columns, 800 individuals: every count and every mask
    word against the oracle, in the launch shape the benchmark uses."""
    w, pop = gen.methylation_436444x64()
    offs, cols = gen.csr(pop)
    mat = ctx.upload(w.X)
    announce("methylation_436444x64 full")
    got = gpu_eval(ctx, mat, offs, cols, negative=True, masks=True)
    want = oracle_eval(w.X, offs, cols, negative=True, masks=True)
    assert_same(got, want, "methylation_436444x64")
    # planted trends are recovered in full
    mm = got[2]
    for i, p in enumerate(w.plants):
        bits = np.unpackbits(mm[i].view(np.uint8), bitorder="little")[: w.X.shape[0]]
        assert bits[p.rows].all()
    announce("methylation_436444x64 positive only")
    got = gpu_eval(ctx, mat, offs, cols, negative=False, masks=False)
    want = oracle_eval(w.X, offs, cols, negative=False, masks=False)
    assert_same(got, want, "methylation_436444x64 pos")
    ctx.release(mat)


SHAPES = [  # tiles_per_wave, waves_per_block, individuals_per_group, staging, blocks
    (1, 1, 1, 0, 0), (1, 4, 7, 0, 3), (2, 8, 64, 0, 0), (4, 16, 1000, 0, 0), (4, 3, 33, 0, 1),
    (2, 5, 200, 0, 7), (1, 8, 1000, 1, 0), (2, 4, 13, 1, 2), (4, 8, 300, 1, 0), (4, 1, 5, 1, 0),
    # staging 2: the FP16 rank codes
    (2, 8, 64, 2, 0), (4, 16, 1000, 2, 0), (4, 3, 33, 2, 1), (2, 5, 200, 2, 7), (1, 8, 100, 2, 0),
    # staging 3: the byte rank codes (include mode here; exclude mode falls
    # back, the matrix has missing cells)
    (4, 8, 64, 3, 0), (4, 16, 1000, 3, 0), (4, 3, 33, 3, 1), (4, 5, 200, 3, 7), (2, 8, 100, 3, 0),
    (8, 16, 400, 3, 0), (8, 4, 33, 3, 2), (8, 7, 150, 3, 5),
    # byte codes with a multiple of 8 tile ranges per group (the XCD-aware
    # block placement; 10 and 5 groups, more ranges than chunks)
    (8, 4, 33, 3, 8), (4, 8, 64, 3, 16),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "L{}W{}P{}S{}B{}".format(*s))
def test_launch_shapes_agree(ctx, shape):
    rng = np.random.default_rng(101)
    rows, ncols = 5000 + 37, 48
    X = rng.integers(0, 6, size=(rows, ncols)).astype(np.float32)  # many ties
    X[rng.random((rows, ncols)) < 0.03] = np.float32(np.nan)
    offs, cols = _random_pop(rng, ncols, 301, 12, dup=0.05, bad=0.03)
    # (the fill copy also gives include mode its rank codes)
    mat = ctx.upload(X, fill=2.5, keep_fill_copy=shape[3] == 2)
    try:
        ctx.set_launch_shape(*shape)
        for include in (False, True):
            announce("shape", shape, include)
            got = gpu_eval(ctx, mat, offs, cols, include=include)
            want = oracle_eval(X, offs, cols, include=include, fill=2.5)
            assert_same(got, want, f"shape {shape} include={include}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("rows", [1, 2, 63, 64, 65, 127, 129, 255, 257, 4095])
def test_edge_rows(ctx, rows):
    rng = np.random.default_rng(200 + rows)
    X = _special(rng, (rows, 9), nan_frac=0.05)
    offs, cols = _random_pop(rng, 9, 60, 7, dup=0.1)
    mat = ctx.upload(X, fill=-0.0)
    for include in (False, True):
        announce("rows", rows, include)
        got = gpu_eval(ctx, mat, offs, cols, include=include)
        want = oracle_eval(X, offs, cols, include=include, fill=-0.0)
        assert_same(got, want, f"rows={rows}")
    ctx.release(mat)


@pytest.mark.parametrize("ncols", [1, 2, 3, 64, 65, 256, 310, 700])
def test_edge_cols(ctx, ncols):
    rng = np.random.default_rng(300 + ncols)
    rows = 700
    X = rng.standard_normal((rows, ncols)).astype(np.float32)
    X[:, ::3] = np.round(X[:, ::3])  # ties
    X[rng.random((rows, ncols)) < 0.02] = np.float32(np.nan)
    offs, cols = _random_pop(rng, ncols, 120, min(ncols, 25), dup=0.05)
    mat = ctx.upload(X, fill=0.0)
    for include in (False, True):
        announce("cols", ncols, include)
        got = gpu_eval(ctx, mat, offs, cols, include=include)
        want = oracle_eval(X, offs, cols, include=include)
        assert_same(got, want, f"cols={ncols}")
    ctx.release(mat)


@pytest.mark.parametrize("ncols,L", [(9, 2), (9, 4), (100, 4), (310, 2), (384, 2)])
def test_rank_codes_special_values(ctx, ncols, L):
    """FP16 rank-code staging on the special values (+-inf, +-0, denormals,
    ties, NaN), in both modes, at widths up to the largest with codes."""
    rng = np.random.default_rng(900 + ncols)
    X = _special(rng, (777, ncols), nan_frac=0.04)
    offs, cols = _random_pop(rng, ncols, 150, min(ncols, 14), dup=0.1, bad=0.02)
    mat = ctx.upload(X, fill=-0.0, keep_fill_copy=True)
    try:
        ctx.set_launch_shape(L, 8, 64, 2, 0)
        for include in (False, True):
            announce("rank codes", ncols, L, include)
            got = gpu_eval(ctx, mat, offs, cols, include=include)
            want = oracle_eval(X, offs, cols, include=include, fill=-0.0)
            assert_same(got, want, f"codes cols={ncols} L={L} include={include}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("tiles", [4, 8])
@pytest.mark.parametrize("ncols", [2, 9, 64, 128])
@pytest.mark.parametrize("rows", [1, 255, 257, 777, 3001])
def test_byte_codes_special_values(ctx, ncols, rows, tiles):
    """Byte rank-code staging (four rows per 32-bit lane word) on the special
    values (+-inf, +-0, denormals, ties): both modes and both trend settings
    on a matrix without missing cells, where both modes stage the byte
    codes; with missing cells, include mode stages them and exclude mode
    falls back to another staging. Individuals of up to 30 columns reach
    past the 8-column window. tiles = 64-row sub-tiles per chunk (one or two
    256-row groups)."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(1100 + 7 * ncols + rows + tiles)
    X = _special(rng, (rows, ncols))
    Xn = X.copy()
    Xn[rng.random(X.shape) < 0.04] = np.float32(np.nan)
    offs, cols = _random_pop(rng, ncols, 150, min(ncols, 30), dup=0.1, bad=0.02)
    for name, A in (("no missing", X), ("missing", Xn)):
        mat = ctx.upload(A, fill=-0.0)
        try:
            ctx.set_launch_shape(tiles, 8, 64, ebic.STAGE_BYTES, 0)
            plan = ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1, int(offs[-1]))
            assert (plan[3] == ebic.STAGE_BYTES) == (not np.isnan(A).any())
            if plan[3] == ebic.STAGE_BYTES:
                assert plan[0] == tiles
            for include in (False, True):
                for negative in (False, True):
                    announce("byte codes", rows, ncols, tiles, name, include, negative)
                    got = gpu_eval(ctx, mat, offs, cols, include=include, negative=negative)
                    want = oracle_eval(A, offs, cols, include=include, negative=negative, fill=-0.0)
                    assert_same(got, want, f"bytes {rows}x{ncols} {name} include={include} "
                                           f"negative={negative}")
        finally:
            ctx.set_launch_shape()
            ctx.release(mat)


@pytest.mark.parametrize("tiles", [2, 4])
@pytest.mark.parametrize("ncols", [129, 256, 384])
@pytest.mark.parametrize("rows", [1, 257, 777, 3001])
def test_halves_special_values(ctx, ncols, rows, tiles):
    """16-bit SWAR codes (two rows per 32-bit lane word, matrices of 129 to
    384 columns; one word per row of a 128-row chunk, or two of a 256-row
    chunk) on the special values (+-inf, +-0, denormals, ties): both modes
    and trend settings without missing cells; with them, include mode uses
    the codes and exclude mode falls back. Individuals of up to 30 columns
    reach past the 8-column window."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(1300 + ncols + rows)
    X = _special(rng, (rows, ncols))
    Xn = X.copy()
    Xn[rng.random(X.shape) < 0.04] = np.float32(np.nan)
    offs, cols = _random_pop(rng, ncols, 120, 30, dup=0.1, bad=0.02)
    for name, A in (("no missing", X), ("missing", Xn)):
        mat = ctx.upload(A, fill=-0.0)
        try:
            ctx.set_launch_shape(tiles, 8, 64, ebic.STAGE_HALVES, 0)
            plan = ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1, int(offs[-1]))
            if np.isnan(A).any():
                assert plan[3] != ebic.STAGE_HALVES
            else:
                assert plan[3] == ebic.STAGE_HALVES
                # a four-tile chunk of 384 columns does not fit the LDS: one word per row
                assert plan[0] == (2 if ncols > 256 else tiles)
            for include in (False, True):
                for negative in (False, True):
                    announce("halves", rows, ncols, tiles, name, include, negative)
                    got = gpu_eval(ctx, mat, offs, cols, include=include, negative=negative)
                    want = oracle_eval(A, offs, cols, include=include, negative=negative, fill=-0.0)
                    assert_same(got, want, f"halves {rows}x{ncols} {name} include={include} "
                                           f"negative={negative}")
        finally:
            ctx.set_launch_shape()
            ctx.release(mat)


@pytest.mark.parametrize("shape", [(4, 16, 400, 4, 0), (4, 3, 33, 4, 1), (4, 5, 200, 4, 7),
                                   (2, 8, 64, 4, 0)], ids=lambda s: "L{}W{}P{}S{}B{}".format(*s))
def test_halves_launch_shapes(ctx, shape):
    """16-bit SWAR codes on a 200-column matrix with many ties (integers
    0..5) and missing cells, in several launch shapes."""
    rng = np.random.default_rng(1400)
    rows, ncols = 5000 + 37, 200
    X = rng.integers(0, 6, size=(rows, ncols)).astype(np.float32)
    X[rng.random((rows, ncols)) < 0.03] = np.float32(np.nan)
    offs, cols = _random_pop(rng, ncols, 301, 14, dup=0.05, bad=0.03)
    mat = ctx.upload(X, fill=2.5)
    try:
        ctx.set_launch_shape(*shape)
        for include in (False, True):
            announce("halves shape", shape, include)
            got = gpu_eval(ctx, mat, offs, cols, include=include)
            want = oracle_eval(X, offs, cols, include=include, fill=2.5)
            assert_same(got, want, f"halves shape {shape} include={include}")
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


def test_invalid_and_degenerate_individuals(ctx):
    rng = np.random.default_rng(400)
    X = rng.standard_normal((1000, 10)).astype(np.float32)
    inds = [[0, 1], [], [0, 10], [-1, 2], [3], [2, 2, 2], [9, 8, 7, 6, 5, 4, 3, 2, 1, 0],
            [5, 5], [0], list(range(10)), [4, 11, 2]]
    offs, cols = gen.csr(inds)
    mat = ctx.upload(X)
    announce("invalid individuals")
    got = gpu_eval(ctx, mat, offs, cols)
    want = oracle_eval(X, offs, cols)
    assert_same(got, want, "invalid")
    assert list(got[0][[1, 2, 3, 10]]) == [-1, -1, -1, -1]
    assert not got[2][[1, 2, 3, 10]].any()
    # a population with zero individuals is a no-op
    import torch
    from paper_1807_09932_amd.ebic import ebic_eval_population
    ebic_eval_population(ctx.handle, mat, 0, 0, 0, 2, 0, None, None, None, 0)
    torch.cuda.synchronize()
    ctx.release(mat)


def test_sentinel_and_fill_copy(ctx):
    rng = np.random.default_rng(500)
    X = rng.integers(-3, 4, size=(3000, 12)).astype(np.float32)
    X[rng.random(X.shape) < 0.05] = np.float32(999.0)
    X[rng.random(X.shape) < 0.02] = np.float32(np.nan)
    X[rng.random(X.shape) < 0.02] = np.float32(-0.0)
    offs, cols = _random_pop(rng, 12, 200, 8)
    for sentinel in (999.0, 0.0):
        for keep in (False, True):
            mat = ctx.upload(X, sentinel=sentinel, fill=7.0, keep_fill_copy=keep)
            for staging in (0, 1):
                ctx.set_launch_shape(2, 4, 64, staging, 0)
                for include in (False, True):
                    announce("sentinel", sentinel, keep, staging, include)
                    got = gpu_eval(ctx, mat, offs, cols, include=include)
                    want = oracle_eval(X, offs, cols, include=include, sentinel=sentinel, fill=7.0)
                    assert_same(got, want, f"sentinel={sentinel} keep={keep} staging={staging}")
            ctx.set_launch_shape()
            ctx.release(mat)


def test_upload_layouts(ctx):
    import torch
    rng = np.random.default_rng(600)
    base = rng.standard_normal((900, 40)).astype(np.float32)
    X = base[:, 3:33]                       # row-major view with row stride 40
    offs, cols = _random_pop(rng, 30, 80, 10)
    want = oracle_eval(np.ascontiguousarray(X), offs, cols)
    variants = {
        "host_rowmajor_strided": torch.from_numpy(base)[:, 3:33],
        "host_colmajor": torch.from_numpy(np.asfortranarray(X)).t().contiguous().t(),
        "device_rowmajor": torch.from_numpy(np.ascontiguousarray(X)).cuda(),
        "device_colmajor": torch.from_numpy(np.ascontiguousarray(X.T)).cuda().t(),
    }
    for name, src in variants.items():
        mat = ctx.upload(src)
        announce("upload", name)
        got = gpu_eval(ctx, mat, offs, cols)
        assert_same(got, want, name)
        ctx.release(mat)


def test_repeat_is_deterministic(ctx):
    w, pop = gen.uniform_1000x50()
    offs, cols = gen.csr(pop)
    mat = ctx.upload(w.X)
    announce("repeat")
    a = gpu_eval(ctx, mat, offs, cols)
    b = gpu_eval(ctx, mat, offs, cols)
    assert_same(a, b, "repeat")
    ctx.release(mat)


def test_error_paths(ctx):
    from paper_1807_09932_amd import ebic
    X = np.ones((10, 3), np.float32)
    with pytest.raises(ebic.EbicError) as e:
        ctx.upload(X, fill=float("nan"))
    assert e.value.status == ebic.EBIC_EINVAL
    mat = ctx.upload(X)
    pop = ctx.population([[0, 1]])
    out = ctx.outputs(mat, 1)
    with pytest.raises(ebic.EbicError) as e:
        ebic.ebic_eval_population(ctx.handle, 12345, 1, pop.offsets.data_ptr(), pop.cols.data_ptr(),
                                  0, out[0].data_ptr(), None, None, None, 0)
    assert e.value.status == ebic.EBIC_ENOENT
    with pytest.raises(ebic.EbicError) as e:
        ebic.ebic_eval_population(ctx.handle, mat, 1, pop.offsets.data_ptr(), pop.cols.data_ptr(),
                                  64, out[0].data_ptr(), None, None, None, 0)
    assert e.value.status == ebic.EBIC_EINVAL
    with pytest.raises(ebic.EbicError) as e:
        ebic.ebic_eval_population(ctx.handle, mat, 1, 0, 0, 0, 0, None, None, None, 0)
    assert e.value.status == ebic.EBIC_EINVAL
    with pytest.raises(ValueError):
        ctx.population(offsets=np.array([0, 5], np.int32), cols=np.array([1, 2], np.int32))
    ctx.release(mat)
    with pytest.raises(ebic.EbicError) as e:
        ctx.release(mat)
    assert e.value.status == ebic.EBIC_ENOENT


@pytest.mark.parametrize("tiles_per_wave,staging", [(1, 0), (2, 0), (4, 0), (2, 2), (4, 2), (4, 3), (8, 3),
                                                    (4, 4)])
def test_measurement_variant_agrees(ctx, tiles_per_wave, staging):
    """The step-counting kernel variant (profiling mode 2) computes the same
    outputs as the timed one, and counts a positive number of steps."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(700 + tiles_per_wave)
    ncols = 150 if staging == ebic.STAGE_HALVES else 30  # (16-bit codes: over 128 columns)
    X = rng.integers(0, 5, size=(3000, ncols)).astype(np.float32)
    if staging < ebic.STAGE_BYTES:  # (SWAR codes serve exclude mode without missing cells)
        X[rng.random(X.shape) < 0.02] = np.float32(np.nan)
    offs, cols = _random_pop(rng, ncols, 150, 20, dup=0.05, bad=0.02)
    mat = ctx.upload(X, keep_fill_copy=True)
    try:
        ctx.set_launch_shape(tiles_per_wave, 4, 50, staging, 0)
        ebic.ebic_set_profiling(ctx.handle, 3)
        for include in (False, True):
            for negative in (False, True):
                announce("counting variant", tiles_per_wave, include, negative)
                got = gpu_eval(ctx, mat, offs, cols, include=include, negative=negative)
                want = oracle_eval(X, offs, cols, include=include, negative=negative)
                assert_same(got, want, f"counting L={tiles_per_wave}")
        launches, ms, steps = ebic.ebic_read_profile(ctx.handle)
        assert launches == 4 and ms > 0 and steps > 0
    finally:
        ebic.ebic_set_profiling(ctx.handle, 0)
        ctx.set_launch_shape()
        ctx.release(mat)


def test_halves_tall_ranges(ctx):
    """16-bit SWAR codes keep a block's counts in 16 bits, so the planner
    keeps every tile range below 65,536 rows: a 140,000-row matrix with one
    range per group forced is split into ranges that fit, and the counts
    (some individuals match most rows) stay exact."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(1500)
    rows, ncols = 140000, 160
    X = rng.standard_normal((rows, ncols)).astype(np.float32)
    X[:, 1] = X[:, 0] + 1.0  # columns 0, 1 rise on every row
    inds = [np.array([0, 1]), np.array([1, 0]), np.array([0, 1, 5]), np.array([3])] + \
        [rng.choice(ncols, size=int(rng.integers(2, 12)), replace=False) for _ in range(60)]
    offs, cols = gen.csr(inds)
    mat = ctx.upload(X)
    try:
        ctx.set_launch_shape(2, 16, 64, ebic.STAGE_HALVES, 1)
        plan = ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1, int(offs[-1]))
        assert plan[3] == ebic.STAGE_HALVES
        chunks = -(-rows // (plan[0] * 64))
        assert -(-chunks // plan[4]) * plan[0] * 64 <= 65535, plan
        announce("halves tall", plan)
        got = gpu_eval(ctx, mat, offs, cols, negative=True)
        want = oracle_eval(X, offs, cols, negative=True)
        assert_same(got, want, "halves 140000 rows")
        assert got[0][0] == rows and got[0][3] == rows  # every row matches
    finally:
        ctx.set_launch_shape()
        ctx.release(mat)


@pytest.mark.parametrize("tiles", [3, 6])
@pytest.mark.parametrize("ncols", [129, 300, 512])
@pytest.mark.parametrize("rows", [1, 193, 385, 3001])
def test_t10_special_values(ctx, ncols, rows, tiles):
    """10-bit rank codes (three rows per lane word) on the special values
    (+-inf, +-0, denormals, ties), both modes and trend settings, without
    and with missing cells (exclude mode then stages something else), one
    and two lane words per chunk."""
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(2100 + 7 * ncols + rows + tiles)
    X = _special(rng, (rows, ncols))
    Xn = X.copy()
    Xn[rng.random(X.shape) < 0.04] = np.float32(np.nan)
    offs, cols = _random_pop(rng, ncols, 120, 30, dup=0.1, bad=0.02)
    for name, A in (("no missing", X), ("missing", Xn)):
        mat = ctx.upload(A, fill=-0.0)
        try:
            ctx.set_launch_shape(tiles, 8, 64, ebic.STAGE_T10, 0)
            plan = ebic.ebic_plan_shape(ctx.handle, mat, offs.size - 1, int(offs[-1]))
            assert (plan[3] == ebic.STAGE_T10) == (not np.isnan(A).any())
            for include in (False, True):
                for negative in (False, True):
                    announce("t10 special", rows, ncols, tiles, name, include, negative)
                    got = gpu_eval(ctx, mat, offs, cols, include=include, negative=negative)
                    want = oracle_eval(A, offs, cols, include=include, negative=negative, fill=-0.0)
                    assert_same(got, want, f"t10 {rows}x{ncols} {name} include={include} "
                                           f"negative={negative}")
        finally:
            ctx.set_launch_shape()
            ctx.release(mat)


def test_library_allocator_without_torch():
    """A context that allocates with hipMalloc itself (no torch allocator
    hook): upload, plain and batched evaluation, release and destroy, with
    the oracle's counts."""
    import torch
    from paper_1807_09932_amd import ebic
    rng = np.random.default_rng(77)
    X = _special(rng, (2_001, 96))
    offs, cols = _random_pop(rng, 96, 200, 20, dup=0.05, bad=0.02)
    c = ebic.Context(0, torch_allocator=False)
    try:
        mat = c.upload(X)
        announce("own allocator")
        got = gpu_eval(c, mat, offs, cols, negative=True, masks=True)
        assert_same(got, oracle_eval(X, offs, cols, negative=True, masks=True), "own allocator plain")
        p = c.population(offsets=offs, cols=cols)
        o = c.outputs(mat, p.n)
        c.eval_batch([c.request(mat, p, o)])
        torch.cuda.synchronize()
        want = oracle_eval(X, offs, cols, negative=True, masks=False)
        assert np.array_equal(to_np(o[0]), want[0]) and np.array_equal(to_np(o[1]), want[1])
        c.release(mat)
    finally:
        c.close()
