"""Write the oracle regression fixtures in this folder.

Calls only the CPU oracle (never the HIP library).  The paper prints no
worked numerical example for the short-range sum, the keys or the leaves, so
these fixtures freeze the oracle's own outputs on tiny seeded inputs; they
guard the oracle against unnoticed change, while the physics pins live in
tests/test_oracle_*.py.

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from workloads import BoxParams  # noqa: E402


def small_box():
    rng = np.random.Generator(np.random.PCG64(20180226))
    L = 10.0
    pos = rng.random((3, 48)) * L
    pos[:, :16] = np.mod(2.0 + 0.3 * rng.standard_normal((3, 16)), L)
    mass = rng.uniform(0.5, 1.5, 48)
    return pos, mass, BoxParams(L=L, rs=0.5, rcut=2.25, eps=0.02, G=1.0, leaf_max=4)


def main():
    pos, mass, p = small_box()
    r = oracle.accel(pos, mass, p)
    with open(os.path.join(HERE, "oracle_accel_48.txt"), "w") as f:
        f.write("# Short-range accelerations (sec. 3.1 Eq. equ:split; direct sum within r_cut)\n")
        f.write("# of the 48-particle box of make_golden.small_box(); written by make_golden.py from the oracle.\n")
        f.write("# columns: index n_inter ax ay az (%.17e)\n")
        for i in range(pos.shape[1]):
            f.write(f"{i} {r['n_inter'][i]} {r['acc'][0, i]:.17e} {r['acc'][1, i]:.17e} {r['acc'][2, i]:.17e}\n")
    st = oracle.structure(pos, p)
    with open(os.path.join(HERE, "oracle_keys_leaves_48.txt"), "w") as f:
        f.write("# Peano-Hilbert keys (sec. 4.1, 21 bits per axis) and leaves (sec. 3.2-3.3, leaf_max 4)\n")
        f.write("# of the same box; written by make_golden.py from the oracle.\n")
        f.write("# key lines: K index key ; leaf lines: F begin count level prefix\n")
        for i, k in enumerate(st["keys"]):
            f.write(f"K {i} {int(k)}\n")
        lv = st["leaves"]
        for a in range(lv["begin"].size):
            f.write(f"F {lv['begin'][a]} {lv['count'][a]} {lv['level'][a]} {int(lv['prefix'][a])}\n")


if __name__ == "__main__":
    main()
