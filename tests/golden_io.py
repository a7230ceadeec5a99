"""Reader for the hand-worked fixtures under tests/golden/ (plain text:
"[name]" opens a case, "key = values" lines, "|" separates table rows, "#"
starts a comment)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
INTS = ("E", "tau", "Tp", "k", "excl", "E_max", "E_opt")


def load(name="worked_examples.txt"):
    cases, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = cases.setdefault(line[1:-1], {})
                continue
            key, val = (s.strip() for s in line.split("=", 1))
            if key in INTS:
                cur[key] = int(val)
            elif "|" in val:
                cur[key] = np.array([[float(t) for t in row.split()] for row in val.split("|")])
            else:
                cur[key] = np.array([float(t) for t in val.split()])
    return cases
