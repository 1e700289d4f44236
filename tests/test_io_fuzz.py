"""Random and byte-mutated delimited texts through the library's reader:
every input either parses into a finite-shaped matrix or raises EbicError
(never a crash or another exception). Seeded; small enough for the CPU
suite. (The same loop, longer, was also run against a build of the host
code with AddressSanitizer.)"""
import random

import numpy as np
import pytest

from paper_1807_09932_amd import ebic

TOKENS = ["1", "-2.5", "3e5", "nan", "NA", "?", "", "inf", "-0", "1e-45", "x", "\"q\"", "0x10", "1.", ".5",
          "+7", "1e999"]
SEPS = [",", "\t", ";", " ", ""]


def _text(rng):
    rows, cols = rng.randint(0, 6), rng.randint(0, 5)
    sep = rng.choice(SEPS[:3])
    lines = []
    if rng.random() < 0.5:
        lines.append(sep.join(f"h{j}" for j in range(cols + rng.randint(0, 1))))
    for r in range(rows):
        n = cols + (rng.randint(-1, 1) if rng.random() < 0.2 else 0)
        f = [rng.choice(TOKENS) for _ in range(max(0, n))]
        if rng.random() < 0.3:
            f = [f"r{r}"] + f
        lines.append(rng.choice([sep, rng.choice(SEPS)]).join(f))
    data = rng.choice(["\n", "\r\n"]).join(lines).encode() + (b"\n" if rng.random() < 0.3 else b"")
    if rng.random() < 0.15:
        b = bytearray(data)
        for _ in range(rng.randint(1, 5)):
            if b:
                b[rng.randrange(len(b))] = rng.randrange(256)
        data = bytes(b)
    return data


@pytest.mark.parametrize("seed", range(3))
def test_reader_parses_or_rejects(tmp_path, seed):
    rng = random.Random(seed)
    p = tmp_path / "m.txt"
    parsed = 0
    for _ in range(400):
        p.write_bytes(_text(rng))
        try:
            X, rn, cn = ebic.read_delimited(str(p), rng.choice(["", ",", "\t", ";"]), rng.choice([-1, 0, 1]),
                                            rng.choice([-1, 0, 1]), threads=rng.randint(1, 4))
        except ebic.EbicError:
            continue
        parsed += 1
        assert X.dtype == np.float32 and X.ndim == 2
        assert rn is None or len(rn) == X.shape[0]
        assert cn is None or len(cn) == X.shape[1]
    assert parsed > 0
