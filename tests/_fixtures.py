"""Helpers shared by the tests: golden-file parsers and cached scenes."""
import functools
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def parse_aggregation_cases(name="aggregation_hand.txt"):
    cases, cur = [], None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = {"name": tok[1], "edges": []}
        elif tok[0] == "diag":
            cur["diag"] = [int(v) for v in tok[1:]]
        elif tok[0] == "edge":
            cur["edges"].append(tuple(int(v) for v in tok[1:]))
        elif tok[0] == "expect":
            cur["expect"] = [int(v) for v in tok[1:]]
        elif tok[0] == "end":
            cases.append(cur)
    return cases


def case_matrix(case):
    n = len(case["diag"])
    W = np.diag(case["diag"]).astype(np.int64)
    for i, j, w in case["edges"]:
        W[i, j] = W[j, i] = w
    return W


def projection_cases(name="projection_hand.txt"):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=2)


@functools.lru_cache(maxsize=None)
def scene(name):
    from scenes import make_scene
    return make_scene(name)
