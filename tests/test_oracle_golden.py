"""The oracle still reproduces its frozen outputs (tests/golden/*.txt,
written by tests/golden/make_golden.py from the oracle alone)."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))


def test_golden_accel(oracle_mod):
    import make_golden
    pos, mass, p = make_golden.small_box()
    r = oracle_mod.accel(pos, mass, p)
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "oracle_accel_48.txt")) if not l.startswith("#")]
    for row in rows:
        i = int(row[0])
        assert r["n_inter"][i] == int(row[1])
        ref = np.array([float(v) for v in row[2:5]])
        assert np.allclose(r["acc"][:, i], ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())


def test_golden_keys_leaves(oracle_mod):
    import make_golden
    pos, mass, p = make_golden.small_box()
    st = oracle_mod.structure(pos, p)
    keys, leaves = {}, []
    for l in open(os.path.join(HERE, "golden", "oracle_keys_leaves_48.txt")):
        t = l.split()
        if t[0] == "K":
            keys[int(t[1])] = int(t[2])
        elif t[0] == "F":
            leaves.append(tuple(int(v) for v in t[1:]))
    assert [int(k) for k in st["keys"]] == [keys[i] for i in range(len(keys))]
    lv = st["leaves"]
    got = [(int(lv["begin"][a]), int(lv["count"][a]), int(lv["level"][a]), int(lv["prefix"][a]))
           for a in range(lv["begin"].size)]
    assert got == leaves
