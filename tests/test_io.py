"""Ingest (delimited text -> column-major FP32) and export (biclusters as
text) of the library, on the CPU. Values are written with Python's shortest
round-trip repr, so every parsed value must equal the original bit for bit."""
import os

import numpy as np
import pytest

import oracle
from paper_1807_09932_amd import ebic, gen


def _values(seed, rows, cols):
    rng = np.random.default_rng(seed)
    X = gen.draw_values(rng, "normal", (rows, cols)) * np.float32(1e3)
    X[0, 0] = np.float32(1e-41)       # denormal
    X[0, 1] = np.float32(-0.0)
    X[1, 0] = np.float32(3.4e38)
    X.reshape(-1)[rng.choice(X.size, X.size // 20, replace=False)] = np.nan
    return X


def _write(path, X, delim, header, names, crlf=False, upper_left=True, missing="NA"):
    rows, cols = X.shape
    eol = "\r\n" if crlf else "\n"
    lines = []
    if header:
        h = [f"s{j}" for j in range(cols)]
        if names and upper_left:
            h = ["gene"] + h
        lines.append(delim.join(h))
    for r in range(rows):
        f = [missing if np.isnan(v) else repr(float(v)) for v in X[r]]
        if names:
            f = [f"g{r}"] + f
        lines.append(delim.join(f))
    with open(path, "w", newline="") as fh:
        fh.write(eol.join(lines) + eol)


def _same(a, b):
    return np.array_equal(np.isnan(a), np.isnan(b)) and \
        np.array_equal(a[~np.isnan(a)].view(np.uint32), b[~np.isnan(b)].view(np.uint32))


@pytest.mark.parametrize("delim", [",", "\t", ";"])
@pytest.mark.parametrize("header,names,upper_left", [(False, False, True), (True, False, True),
                                                     (True, True, True), (True, True, False),
                                                     (False, True, True)])
def test_round_trip_bit_exact(tmp_path, delim, header, names, upper_left):
    X = _values(1, 57, 9)
    p = os.path.join(tmp_path, "m.txt")
    _write(p, X, delim, header, names, crlf=(delim == ";"), upper_left=upper_left)
    Y, rn, cn = ebic.read_delimited(p, threads=3)
    assert Y.shape == X.shape and Y.flags["F_CONTIGUOUS"]
    assert _same(np.ascontiguousarray(Y), X)
    assert (rn == [f"g{r}" for r in range(57)]) if names else rn is None
    assert (cn == [f"s{j}" for j in range(9)]) if header else cn is None


@pytest.mark.parametrize("token", ["", "NA", "NaN", "nan", "?"])
def test_missing_tokens(tmp_path, token):
    X = _values(2, 20, 5)
    p = os.path.join(tmp_path, "m.csv")
    _write(p, X, ",", True, True, missing=token)
    Y, _, _ = ebic.read_delimited(p)
    assert _same(np.ascontiguousarray(Y), X)


def test_threads_do_not_change_values(tmp_path):
    X = _values(3, 1000, 12)
    p = os.path.join(tmp_path, "m.tsv")
    _write(p, X, "\t", False, False)
    a = ebic.read_delimited(p, threads=1)[0]
    b = ebic.read_delimited(p, threads=7)[0]
    assert _same(np.ascontiguousarray(a), np.ascontiguousarray(b))


def test_errors(tmp_path):
    p = os.path.join(tmp_path, "bad.csv")
    with open(p, "w") as f:
        f.write("1,2,3\n4,5\n")
    with pytest.raises(ebic.EbicError) as e:
        ebic.read_delimited(p)
    assert e.value.status == ebic.EBIC_EINVAL and "line 2" in str(e.value)
    with open(p, "w") as f:
        f.write("1,2,3\n4,x5,6\n")
    with pytest.raises(ebic.EbicError) as e:
        ebic.read_delimited(p, header=0, row_names=0)
    assert "not a number" in str(e.value)
    with pytest.raises(ebic.EbicError) as e:
        ebic.read_delimited(os.path.join(tmp_path, "missing.csv"))
    assert e.value.status == ebic.EBIC_ENOENT


def _parse_export(path):
    out = []
    with open(path) as f:
        lines = f.read().splitlines()
    assert lines[0].startswith("# EBIC biclusters:")
    for i in range(1, len(lines), 3):
        head, rows, cols = (l.split("\t") for l in lines[i:i + 3])
        assert head[0] == "bicluster" and rows[0] == "rows" and cols[0] == "cols"
        out.append((int(head[2]), int(head[3]), rows[1:], cols[1:]))
    return out


def test_export_matches_masks(tmp_path):
    w, pop = gen.uniform_1000x50()
    offs, cols = gen.csr(pop)
    rows = w.X.shape[0]
    m, _, mm, _ = oracle.eval_population(w.X, offs, cols, negative=True, masks=True, threads=4)
    which = [0, 1, 2, 17]
    p = os.path.join(tmp_path, "bc.txt")
    ebic.write_biclusters(p, rows, offs, cols, mm, which)
    got = _parse_export(p)
    assert len(got) == len(which)
    for (nr, k, rr, cc), i in zip(got, which):
        bits = np.unpackbits(mm[i].view(np.uint8), bitorder="little")[:rows]
        want_rows = [str(r + 1) for r in np.nonzero(bits)[0]]
        assert nr == m[i] == len(rr) and rr == want_rows
        assert k == offs[i + 1] - offs[i]
        assert cc == [str(c + 1) for c in cols[offs[i]:offs[i + 1]]]
    # with names
    rn = [f"r{r}" for r in range(rows)]
    cn = [f"c{j}" for j in range(w.X.shape[1])]
    ebic.write_biclusters(p, rows, offs, cols, mm, [5], rn, cn)
    (nr, k, rr, cc), = _parse_export(p)
    bits = np.unpackbits(mm[5].view(np.uint8), bitorder="little")[:rows]
    assert rr == [rn[r] for r in np.nonzero(bits)[0]]
    assert cc == [cn[c] for c in cols[offs[5]:offs[6]]]
    with pytest.raises(ebic.EbicError):
        ebic.write_biclusters(p, rows, offs, cols, mm, [len(pop)])


def test_names_that_are_not_utf8_round_trip(tmp_path):
    """Row and column names are the file's bytes: names that are not UTF-8
    are read (as escapes) and written back as the same bytes."""
    p = tmp_path / "latin1.tsv"
    p.write_bytes(b"gene\tca\xe9\tcb\nr\xf61\t1.5\t2\nr2\t3\t-4\n")
    X, rn, cn = ebic.read_delimited(str(p), "\t")
    assert X.shape == (2, 2) and X[0, 0] == np.float32(1.5) and X[1, 1] == np.float32(-4)
    assert cn[0].encode("utf-8", "surrogateescape") == b"ca\xe9"
    assert rn[0].encode("utf-8", "surrogateescape") == b"r\xf61"
    offs, cols = gen.csr([np.array([0, 1], np.int32)])
    mask = np.array([[3]], dtype=np.uint64).view(np.int64)
    out = tmp_path / "out.txt"
    ebic.write_biclusters(str(out), 2, offs, cols, mask, [0], row_names=rn, col_names=cn)
    data = out.read_bytes()
    assert b"r\xf61" in data and b"ca\xe9" in data
