#!/usr/bin/env python3
"""Write ``oracle_regression.json``: oracle outputs on small seeded inputs.

Calls only the oracle (``oracle/``) and the seeded generators.  The stored
values guard the oracle against unintended changes; a change to them must name,
in its commit message, the passage of the paper (or the reading of it) that
justifies it.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2510_02894_amd import synth  # noqa: E402


def cases():
    g = np.random.default_rng(2510)
    out = []
    for i in range(4):
        shape = tuple(int(x) for x in g.integers(5, 14, size=3))
        sp = tuple(float(x) for x in np.round(g.uniform(0.5, 1.5, size=3), 3))
        out.append(("random_%d" % i, synth.random_mask(shape, 0.45, g), sp))
    m, sp = synth.single_roi(0, shape=(40, 40, 40))
    out.append(("ellipsoid_40", m, sp))
    p, sp = synth.differentiable_small(0, shape=(20, 20, 20))
    out.append(("soft_20", p, (1.0, 0.9, 1.2)))
    return out


def main():
    rec = {}
    for name, vol, sp in cases():
        r = O.shape3d(vol, sp)
        rec[name] = dict(shape=list(vol.shape), dtype=str(vol.dtype), spacing=list(sp),
                         V=r["V"], T=r["T"], features=[float(x) for x in r["features"]],
                         pair_ids=r["pair_ids"].tolist())
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_regression.json")
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
