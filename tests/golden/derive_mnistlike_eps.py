"""Derive eps for the 784-d quantised-image workload from the oracle.

eps sits at the 1st percentile of the sampled squared distances D (all
non-self slots, sampler seed 3): with the non-self values sorted, take index
k = floor(0.01 * (N - 1)), then place eps^2 at the midpoint between q_k and the
next larger distinct value, so no sampled pair lies exactly on the threshold.
Writes mnistlike_eps.json next to this file. Calls only the oracle.
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2006_06743_amd.workloads import mnistlike_784d  # noqa: E402


def derive():
    W = mnistlike_784d()
    m = oracle.samples_per_point(W.s, W.n)
    D = oracle.slot_sqdist(W.X, m, W.seed).ravel()
    D = np.sort(D[D >= 0.0])
    k = int(math.floor(0.01 * (D.size - 1)))
    qk = float(D[k])
    nxt = float(D[np.searchsorted(D, qk, side="right")])
    eps = math.sqrt(0.5 * (qk + nxt))
    e2 = eps * eps
    assert qk < e2 < nxt, (qk, e2, nxt)
    return {"eps": repr(eps), "eps2": repr(e2), "q_k": repr(qk), "q_next": repr(nxt),
            "k": k, "N": int(D.size), "m": m, "seed": W.seed}


if __name__ == "__main__":
    out = derive()
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mnistlike_eps.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)
