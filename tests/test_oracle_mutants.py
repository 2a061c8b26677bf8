"""Plants plausible mistakes in a private copy of the oracle (on the CPU) and
checks that the pins catch every one of them: a pin suite that a dropped
term, a wrong sign or a swapped operand survives would not pin anything."""
import os

import pytest

import oracle as O
import pins

SRC = os.path.join(os.path.dirname(O.__file__), "oracle.c")

MUTANTS = [
    ("voronoi ignores the seed-index tie rule",
     "return a.d < b.d || (a.d == b.d && a.i < b.i);", "return a.d < b.d;"),
    ("voronoi off-by-one relaxation",
     "hitem cand = {x.d + w[e], x.i, u};", "hitem cand = {x.d + w[e] + (w[e] > 1), x.i, u};"),
    ("pred accepts any neighbour in the cell",
     "src[u] == src[v] && dist[u] + w[e] == dist[v]", "src[u] == src[v] && dist[u] < dist[v]"),
    ("pred ignores the cell",
     "src[u] == src[v] && dist[u] + w[e] == dist[v]", "dist[u] + w[e] == dist[v]"),
    ("pred takes the last qualifying entry",
     "                pred[v] = u;\n                break;", "                pred[v] = u;"),
    ("boundary drops the far endpoint's distance",
     "x.bsum = dist[a] + (uint64_t)w[e] + dist[b];", "x.bsum = dist[a] + (uint64_t)w[e];"),
    ("boundary keeps the largest edge id on ties",
     "if (a->e != b->e) return a->e < b->e ? -1 : 1;", "if (a->e != b->e) return a->e < b->e ? 1 : -1;"),
    ("boundary keeps the worst edge per pair",
     "if (a->bsum != b->bsum) return a->bsum < b->bsum ? -1 : 1;\n    if (a->e",
     "if (a->bsum != b->bsum) return a->bsum < b->bsum ? 1 : -1;\n    if (a->e"),
    ("mst ignores the pair-index tie rule",
     "    if (a->i != b->i) return a->i < b->i ? -1 : 1;\n    if (a->j != b->j) return a->j < b->j ? -1 : 1;\n    return 0;\n}\n\nstatic uint32_t dsu_find",
     "    return 0;\n}\n\nstatic uint32_t dsu_find"),
    ("mst orders by the larger weight first",
     "    if (a->bsum != b->bsum) return a->bsum < b->bsum ? -1 : 1;\n    if (a->i != b->i) return a->i < b->i ? -1 : 1;\n    if (a->j != b->j) return a->j < b->j ? -1 : 1;\n    return 0;\n}\n\nstatic uint32_t dsu_find",
     "    if (a->bsum != b->bsum) return a->bsum < b->bsum ? 1 : -1;\n    if (a->i != b->i) return a->i < b->i ? -1 : 1;\n    if (a->j != b->j) return a->j < b->j ? -1 : 1;\n    return 0;\n}\n\nstatic uint32_t dsu_find"),
    ("expand walks only one endpoint",
     "for (int s = 0; s < 2; s++) {", "for (int s = 0; s < 1; s++) {"),
    ("expand uses the wrong path-edge weight",
     "ADD_EDGE(x, p, (uint32_t)(dist[x] - dist[p]));", "ADD_EDGE(x, p, (uint32_t)(dist[x]));"),
    ("expand omits the cross-cell edge",
     "        ADD_EDGE(a, b, w[e]);\n", ""),
    ("overflow limit off by one",
     "#define DIST32_LIMIT 0xFFFFFFFFULL", "#define DIST32_LIMIT 0xFFFFFFFEULL"),
]


def run_overflow_pins(lib):
    """The overflow cases of test_overflow_rules, callable on any build."""
    import numpy as np
    import workloads as W
    g = W.from_edges(2, [(0, 1, 0xFFFFFFFE)])
    dist, _ = O.voronoi(g, np.array([0], dtype=np.uint32), lib)
    assert O.check_dist(dist, lib) == O.OK


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_kill_mutant(tmp_path, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor not unique for: {name}"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = O.load(O.build(str(src), str(tmp_path / "libmutant.so")))
    with pytest.raises(AssertionError):
        pins.run_all(lib, seed=2, count=120)
        run_overflow_pins(lib)
