"""Loader of the golden fixtures under tests/golden/ (plain text)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sections(path):
    out = {}
    cur = None
    for raw in open(path, encoding="utf-8"):
        line = raw.split("#", 1)[0].rstrip() if raw.lstrip().startswith("#") else raw.rstrip()
        if not line.strip():
            continue
        if line.startswith("["):
            name, _, rest = line.partition("]")
            cur = name[1:]
            out[cur] = {"header": rest.split(), "rows": []}
            continue
        words = line.split()
        if words and words[-1] == "decoy":
            words = words[:-1]
        out[cur]["rows"].append(words)
    return out


def load_table1():
    """Table 1 of the paper: dictionary, store, patterns and expected tables as IDs."""
    sec = _sections(os.path.join(GOLDEN, "table1.txt"))
    d = {w[0]: int(w[1]) for w in sec["dict"]["rows"]}
    store = np.array([[d[t] for t in row] for row in sec["store"]["rows"]], dtype=np.int32)
    var_no = {"?person": 0, "?job": 1}

    def tab(name):
        return [tuple(d[t] for t in r) for r in sec[name]["rows"]], [var_no[v] for v in sec[name]["header"]]

    return {
        "dict": d,
        "s": store[:, 0].copy(),
        "p": store[:, 1].copy(),
        "o": store[:, 2].copy(),
        "P1": (-1, d["hasJob"], -2),          # ?person hasJob ?job
        "P2": (-2, d["workAt"], d['"Hospital"']),  # ?job workAt "Hospital"
        "Tp1": tab("Tp1"),
        "Tp2": tab("Tp2"),
        "RS": tab("RS"),
        "SELECT": tab("SELECT"),
    }
