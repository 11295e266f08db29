"""Write tests/golden/fp64_small.json from the FP64 oracle (and the seeded generator) only.

The paper prints no worked numeric example; these stored values pin the
oracle against later drift.  Workload: Nt=32, Nd=16, Nm=64, F_k = N(0,1)
exp(-k/8), m and d ~ N(0,1), H = F^T F + I.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    w = synth.WORKLOADS["fp64-small"]
    blocks = synth.blocks(w["Nt"], w["Nd"], w["Nm"], w["tau"])
    m = synth.vectors(1, w["Nt"], w["Nm"], synth.STREAM_M)[0]
    d = synth.vectors(1, w["Nt"], w["Nd"], synth.STREAM_D)[0]
    out = {"workload": "fp64-small", "generator": "synth SplitMix64/Box-Muller seed 13066"}
    vals = {"Fm": oracle.apply_F(blocks, m).ravel(),
            "FTd": oracle.apply_FT(blocks, d).ravel(),
            "Hm": oracle.apply_H(blocks, m, w["noise_prec"], w["prior_prec"]).ravel()}
    rng = np.random.default_rng(2407)
    for name, v in vals.items():
        idx = np.sort(rng.choice(v.size, 48, replace=False))
        idx = np.unique(np.concatenate([[0, v.size - 1], idx]))
        out[name] = {"index": idx.tolist(), "value": [float(repr_) for repr_ in v[idx]],
                     "norm": float(np.linalg.norm(v))}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fp64_small.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
