"""Oracle regression lock (tests/golden) and the oracle/product separation."""
import json
import os
import re

import numpy as np

import oracle
from paper_1912_05529_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_matches_golden_lock(cfg1, cfg1_table):
    with open(os.path.join(ROOT, "tests", "golden", "config1_oracle.json")) as f:
        g = json.load(f)
    tab, mg, pe, _ = cfg1_table
    for j, row in g["table_rows"].items():
        ref = np.array([complex(a, b) for a, b in row])
        assert np.abs(tab[int(j)] - ref).max() <= 1e-12
        assert abs(mg[int(j)] - g["maxgain"][j]) <= 1e-12
        assert abs(pe[int(j)] - g["passerr"][j]) <= 1e-12
    img = oracle.migrate(cfg1.desc, tab, cfg1.omega, cfg1.vel, cfg1.data)
    for iz, ix, v in g["image_samples"]:
        assert abs(img[iz, ix] - v) <= 1e-10 * g["image_l2"]
    assert abs(np.linalg.norm(img) - g["image_l2"]) <= 1e-10 * g["image_l2"]


def _sources(folder, exts):
    for dp, _, fs in os.walk(os.path.join(ROOT, folder)):
        if "__pycache__" in dp:
            continue
        for f in fs:
            if f.endswith(exts):
                yield os.path.join(dp, f)


def test_oracle_does_not_touch_product_and_vice_versa():
    for p in _sources("oracle", (".c", ".h", ".py")):
        txt = open(p).read()
        assert "paper_1912_05529_amd" not in txt, p
        assert "mig.h" not in txt and "libmig" not in txt, p
    for p in _sources("paper_1912_05529_amd", (".py", ".hip", ".cpp", ".h", ".hpp")):
        txt = open(p).read()
        assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), p
        assert "liboracle" not in txt and "oracle.h" not in txt, p
    for p in _sources("include", (".h",)):
        assert "oracle" not in open(p).read(), p


def test_generators_are_seeded_and_deterministic():
    a = synth.config1(seed=7)
    b = synth.config1(seed=7)
    assert np.array_equal(a.data, b.data) and np.array_equal(a.vel, b.vel)
    c = synth.random_case(3, 20, 6, 4)
    d = synth.random_case(3, 20, 6, 4)
    assert np.array_equal(c.data, d.data) and np.array_equal(c.vel, d.vel)
    m = synth.config2(with_data=False)
    v = m.vel.astype(np.float64) * 2.0
    assert v.min() >= 1500.0 and v.max() == 4800.0
    assert 7 <= np.unique(v).size <= 12
