"""Hand-worked cases of the method (tests/golden/*.txt, each derived in its
header from the definitions of Alg. 2 and the tie rules): the oracle must
reproduce them exactly.  The GPU path is compared with the same files in
tests/test_gpu_parity.py."""
import glob
import os

import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_case(path):
    """Graph, seeds and expected result of one fixture: lines `n N`, `edge u v w`, `seeds s...`, `code C`,
    `tree a b w` (canonical: a < b, sorted) and `D total`; `#` starts a comment."""
    n, edges, seeds, code, tree, total = None, [], [], 0, [], None
    for line in open(path):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        tag, vals = line[0], [int(x) for x in line[1:]]
        if tag == "n":
            n = vals[0]
        elif tag == "edge":
            edges.append(tuple(vals))
        elif tag == "seeds":
            seeds = vals
        elif tag == "code":
            code = vals[0]
        elif tag == "tree":
            tree.append(tuple(vals))
        elif tag == "D":
            total = vals[0]
        else:
            raise ValueError(f"{path}: unknown line {line}")
    return W.from_edges(n, edges), seeds, code, sorted(tree), total


CASES = sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))


def test_cases_present():
    assert len(CASES) >= 7


@pytest.mark.parametrize("path", CASES, ids=[os.path.basename(p)[:-4] for p in CASES])
def test_oracle_matches_hand_worked_case(path):
    g, seeds, code, tree, total = load_case(path)
    sol = O.solve(g, seeds)
    assert sol.code == code
    if code == O.OK:
        assert sorted(sol.edges) == tree
        assert sol.total == total
