"""Pins for the oracle's post-processing (Algorithm 1: core points,
components of the core-induced subgraph, border assignment) on hand-built
graphs whose expected degrees and labels were written by hand."""
import json
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hand_graphs.json")
CASES = json.load(open(GOLD))["cases"]


@pytest.mark.parametrize("case", CASES, ids=[c["name"] for c in CASES])
def test_hand_graph(orc, case):
    if case.get("invalid"):
        with pytest.raises(orc.OracleError):
            orc.graph(case["n"], case["edges"], case["min_pts"])
        return
    r = orc.graph(case["n"], case["edges"] or np.zeros((0, 2), np.int64), case["min_pts"])
    assert r.deg.tolist() == case["deg"]
    assert r.labels.tolist() == case["labels"]
    core = np.array(case["deg"], np.int64) >= case["min_pts"]
    assert r.n_core == int(core.sum())
    assert r.n_noise == case["labels"].count(-1)
    assert r.n_clusters == len({l for l, c in zip(case["labels"], core) if c})
