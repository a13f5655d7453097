"""The stored oracle values (tests/golden/*.json, written by make_golden.py
from the CPU oracle only) are internally consistent and match the configs:
the per-shift residuals of the oracle's unrestarted multishift FOM are at
rounding level, the deflated eigenpairs are accurate and biorthonormal,
the pole scale is the two-circle rule c = (a b)^{-1/2} (Sect. 6) to the
four digits the configs record, the stored full x* agrees with the
stored sample, and where the pole order was doubled the change of x*
is consistent with the Kenney-Laub error bound of the order."""
import glob
import json
import os

import pytest

from skinputs.configs import CONFIGS

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FILES = sorted(glob.glob(os.path.join(HERE, "*.json")))


def test_there_are_stored_values_for_every_large_config():
    names = {os.path.basename(f) for f in FILES}
    for must in ["c6_mu0.3.json", "c2_mu0.3.json", "c3_mu0.3.json", "cg_mu0.3.json", "c2_mu0.1.json",
                 "c3_mu0.1.json", "c3_mu0.5.json", "c3s_mu0.3.json"]:
        assert must in names


@pytest.mark.parametrize("path", FILES, ids=[os.path.basename(f) for f in FILES])
def test_stored_oracle_values(path):
    g = json.load(open(path))
    cfg = CONFIGS[g["config"]]
    assert tuple(g["dims"]) == cfg.dims and g["eps"] == cfg.eps
    assert max(g["shift_residuals"]) <= 1e-12
    assert g["c"] == float(f"{(g['a_next'] * g['lambda_max']) ** -0.5:.4g}")
    assert cfg.scales[g["mu"]] == g["c"]
    n = len(g["sample_index"])
    assert n == len(g["x_re"]) == len(g["x_im"]) and n > 1000
    if cfg.m > 0:
        assert len(g["eig_re"]) == cfg.m
        assert g["eig_res_right"] <= 1e-10 and g["eig_res_left"] <= 1e-10
        assert g["biorth"] <= 1e-12
        # the next eigenvalue is beyond the m deflated ones (selection gap)
        import numpy as np
        lam = np.abs(np.array(g["eig_re"]) + 1j * np.array(g["eig_im"]))
        assert g["a_next"] > lam.max()

    import numpy as np
    full = path[:-5] + "_x.npy"
    if os.path.exists(full):
        x = np.load(full)
        assert x.shape == (cfg.n,) and x.dtype == np.complex128
        idx = np.array(g["sample_index"])
        assert np.array_equal(x[idx], np.array(g["x_re"]) + 1j * np.array(g["x_im"]))
        assert abs(np.linalg.norm(x) - g["x_norm"]) <= 1e-12 * g["x_norm"]
    if "order_check" in g:
        oc = g["order_check"]
        assert oc["s2"] == 2 * cfg.s and oc["max_shift_residual_s2"] <= 1e-12
        # ||x*(s) - x*(2s)|| is the approximation error of order s to within
        # that of order 2s; it must not exceed the scalar bound by much (the
        # deflated operator is not normal, so allow a modest factor) and must
        # be well above the order-2s bound
        assert oc["rel_diff"] <= 100 * g["kl_bound"]
        assert oc["rel_diff"] >= 10 * oc["kl_bound_s2"] or oc["rel_diff"] < 1e-12
