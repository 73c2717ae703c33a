"""Readers for the small text fixtures under tests/golden/."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line


def eq1_factors():
    """dict name -> 4x4 complex matrix, in the printed left-to-right order."""
    mats, order, cur = {}, [], None
    for line in _lines("eq1_factors.txt"):
        if line.startswith("matrix "):
            cur = line.split()[1]
            order.append(cur)
            mats[cur] = []
        else:
            mats[cur].append([complex(t) for t in line.split()])
    return [(k, np.array(mats[k], dtype=np.complex128)) for k in order]


def listing1_input():
    vals = {}
    for line in _lines("listing1_input.txt"):
        key, *nums = line.split()
        vals[key] = [float(t) for t in nums]
    return np.array(vals["real"]) + 1j * np.array(vals["imag"])
