"""Writes tests/golden/uniform_1000x50_counts.json from the CPU oracle alone.

Regression fixture: the counts of the 1,000 x 50 plain-evaluation workload
(seeded generator) in both missing-value modes, with and without the
negative trend, plus a digest of the generated inputs. Run from the repo
root: ``python tests/golden/make_golden.py``. It calls only ``oracle`` and
the seeded generator.
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1807_09932_amd import gen  # noqa: E402


def digest(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(a.tobytes())
    return h.hexdigest()


def main():
    w, pop = gen.uniform_1000x50()
    offs, cols = gen.csr(pop)
    out = {"workload": "1000x50 U[0,1), 3 planted 50x8, 100 individuals of 3-8 columns",
           "inputs_sha256": digest(w.X, offs, cols), "runs": {}}
    for include in (False, True):
        for negative in (False, True):
            m, n, mm, nm = oracle.eval_population(w.X, offs, cols, include=include,
                                                  negative=negative, masks=True)
            key = f"{'include' if include else 'exclude'}_{'neg' if negative else 'pos'}"
            out["runs"][key] = {"matched": m.tolist(), "negative": n.tolist(),
                                "masks_sha256": digest(mm, nm)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "uniform_1000x50_counts.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
