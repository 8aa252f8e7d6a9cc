"""Readers for the paper-value fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield line.split()


def paper_values():
    return {k: float(v) for k, v in _lines("paper_values.txt")}


def table2():
    return [(float(h), (None if it == "NaN" else int(it))) for h, it in _lines("table2_search_length.txt")]


def table3():
    grids, cur = {}, None
    for tok in _lines("table3_metric_grid.txt"):
        if tok[0] == "grid":
            cur = {"kernel": 0 if tok[2] == "conon" else 1, "n": int(tok[3]), "rows": []}
            grids[tok[1]] = cur
        else:
            cur["rows"].append((float(tok[0]), [None if c == "x" else int(c) for c in tok[1:]]))
    return grids
