"""Writes oracle_regression.txt from the FP64 oracle only (no GPU code involved).

The fixture freezes the oracle's output on two tiny seeded scenes so that any
later change to the oracle's arithmetic shows up as a failing regression test
(the change then has to name the passage of the paper that justifies it).
Run:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import oracle  # noqa: E402
from helpers import tiny_scene  # noqa: E402

CASES = {
    "static-uniform": dict(n_balls=4, n_sensors=3, seed=101),
    "fourier-add-uniform": dict(n_balls=4, n_sensors=3, n_frames=3, basis=1, seed=102),
    "gaussbasis-mul-gauss": dict(n_balls=3, n_sensors=2, n_frames=2, basis=2, pos_mode=1,
                                 kernel=1, seed=103),
}


def rows():
    out = []
    for name, kw in CASES.items():
        wl = tiny_scene(**kw)
        y = oracle.forward(wl)
        rng = np.random.default_rng(7)
        res = rng.normal(size=y.shape)
        gb, gd = oracle.adjoint(wl, res)
        out.append((name, "signal_sum_abs", float(np.abs(y).sum())))
        out.append((name, "signal_sum_sq", float((y * y).sum())))
        out.append((name, "grad_balls_l1", float(np.abs(gb).sum())))
        out.append((name, "grad_balls_dot_index", float((gb * np.arange(gb.size).reshape(gb.shape)).sum())))
        if gd is not None:
            out.append((name, "grad_deform_l1", float(np.abs(gd).sum())))
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_regression.txt"), "w") as f:
        f.write("# FP64 oracle regression values (written by tests/golden/make_golden.py from oracle/ only)\n")
        for name, key, val in rows():
            f.write(f"{name} {key} {val!r}\n")
