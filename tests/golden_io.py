"""Reader for the hand-derived fixtures in tests/golden/ (key: value lines)."""
import glob
import os

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(path):
    d = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    d["_name"] = os.path.basename(path)
    if "bytes" in d:
        d["bytes"] = bytes(int(x, 16) for x in d["bytes"].split())
    return d


def fixtures(kind_prefix):
    out = []
    for p in sorted(glob.glob(os.path.join(HERE, "*.txt"))):
        d = load(p)
        if d.get("kind", "").startswith(kind_prefix):
            out.append(d)
    return out
