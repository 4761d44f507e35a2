import os

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    """Read a 'key value' fixture (lines starting with '#' are citations)."""
    out = {}
    with open(os.path.join(HERE, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[k] = float(v)
    return out
