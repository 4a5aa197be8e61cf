"""Readers for the text fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def key_values(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()[:2]
            out[k] = float(v)
    return out


def morton_sets():
    sets = {}
    cur = None
    with open(os.path.join(GOLDEN, "morton_examples.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("set "):
                cur = line.split()[1]
                sets[cur] = []
                continue
            x, y, z, k = line.split()
            sets[cur].append(((float(x), float(y), float(z)), int(k)))
    return sets
