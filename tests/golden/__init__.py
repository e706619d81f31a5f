"""Values the paper prints (tests/golden/*.txt), each file citing its
passage.  A line is `name value  # comment`."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name):
    out = {}
    for line in open(os.path.join(HERE, name)):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, val = line.split()
        out[key] = float(val)
    return out
