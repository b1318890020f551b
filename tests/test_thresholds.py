"""The frozen thresholds the package uses are the ones the committed oracle
script wrote, and the C1 entry is reproducible here in seconds."""
import json
import os

import numpy as np

from paper_2603_13618_amd import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "thresholds.json")


def test_package_thresholds_match_golden():
    data = json.load(open(GOLDEN))
    for key, wl in (("C1", workloads.DOUBLE_SHEAR_128), ("C2", workloads.SMOOTH_4096),
                    ("C3", workloads.RIEMANN_2048)):
        rows = np.asarray(data[key])
        np.testing.assert_array_equal(np.asarray(wl["thr"])[: rows.shape[0]], rows)
    # the double distribution: four base rows, then the quasi-equilibrium sensor
    rows = np.asarray(data["C4"])
    wl = workloads.RIEMANN_2048_DDF
    np.testing.assert_array_equal(np.vstack([wl["thr"], [wl["thr_qe"]]]), rows)


def test_c1_thresholds_reproduce():
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_thresholds", os.path.join(os.path.dirname(GOLDEN), "make_thresholds.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    data = json.load(open(GOLDEN))
    assert mod.c1() == data["C1"]
