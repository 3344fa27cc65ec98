"""Reader of the hand-worked text fixtures under tests/golden/."""
from __future__ import annotations

import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_handworked(name: str):
    """Returns (n, src list, dst list, [(root, expected depth list), ...])."""
    n, src, dst, cases = None, [], [], []
    root = None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, *vals = line.split()
            if tag == "n":
                n = int(vals[0])
            elif tag == "e":
                src.append(int(vals[0]))
                dst.append(int(vals[1]))
            elif tag == "root":
                root = int(vals[0])
            elif tag == "depth":
                cases.append((root, [int(x) for x in vals]))
    return n, src, dst, cases
