"""Writes tests/golden/oracle_c1.json: regression values of the FP64 oracle on
the 4,096-leaf scene (cut sizes, blended pair counts and sampled pixels at
tau = 1, 4, 16 px).  The paper prints no worked numeric example, so these
are not the paper's numbers: they freeze the oracle's own output, computed
by this script from ``oracle/`` alone, so that an unintended change of its
arithmetic shows up.  Run from the repository root:
    python tests/golden/make_golden.py
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2406_12080_amd import synth  # noqa: E402

PIXELS = [0, 255, 32896, 33000, 40000, 50000, 65535, 21000, 30000, 45123]


def compute() -> dict:
    h = synth.make_scene(1)
    out = {"scene": "config 1: 4,096 leaves, one 256x256 view at distance 3", "taus": {}}
    for tau in (1.0, 4.0, 16.0):
        v = synth.make_views(1, tau=tau)[0]
        ids, t = O.cut(h, v)
        r = O.render(h, v, ids, t, pix=np.array(PIXELS, np.int64), alternatives=False)
        full = O.render(h, v, ids, t, alternatives=False)
        out["taus"][str(tau)] = dict(cut=int(ids.shape[0]), cut_id_sum=int(ids.astype(np.int64).sum()),
                                     t_sum=float(t.sum()), blended=int(full["blended"]),
                                     pixels=PIXELS, rgb=r["rgb"].tolist(), T=r["T"].tolist())
    return out


if __name__ == "__main__":
    json.dump(compute(), open(os.path.join(HERE, "oracle_c1.json"), "w"), indent=1)
    print("wrote", os.path.join(HERE, "oracle_c1.json"))
