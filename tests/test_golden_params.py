"""The solver defaults match the paper's parameter table (Tab. 1)."""
import os

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    out = {}
    with open(os.path.join(HERE, "golden", "tab1_defaults.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = v
    return out


def test_defaults_match_table1():
    g = _golden()
    p = W.DEFAULT_PARAMS
    for k in ("n_inv", "nkv", "mu", "nu", "mr_iters", "kc_len", "kc_restarts"):
        assert p[k] == int(g[k]), k
    for k in ("coarse_eps", "tol", "kc_tol"):
        assert p[k] == float(g[k]), k
    assert p["sap_block"] == tuple(int(x) for x in g["sap_block"].split(","))
    big = W.CONFIGS["clover16x32_3lvl"]
    assert big["agg"][0] == tuple(int(x) for x in g["agg_level1"].split(","))
    assert big["agg"][1] == tuple(int(x) for x in g["agg_coarser"].split(","))
    assert big["ntv"][0] == int(g["ntv"])


def test_input_generators_chunked_and_parallel_agree():
    """The streaming field generator and the multi-process link generator
    give the same values as the one-shot generators."""
    import numpy as np
    import workloads as W
    dims = (4, 4, 4, 8)
    full = W.test_vectors(dims, 12, 3, 99)
    parts = np.stack(list(W.gaussian_fields_iter(dims, 12, 3, 99)))
    assert np.array_equal(full, parts)
    assert np.array_equal(W.links(dims, 0.5, 98, workers=1), W.links(dims, 0.5, 98, workers=3))
