"""The property verifier accepts the oracle's Voronoi keys and G'1 and rejects
small corruptions of them (CPU)."""
import numpy as np

import props
import oracle as O
import workloads as W


def _dense(k, pi, pj, pb, pe):
    pt = np.full(k * (k - 1) // 2, np.iinfo(np.uint64).max, dtype=np.uint64)
    idx = pj.astype(np.uint64) * (pj.astype(np.uint64) - 1) // 2 + pi
    pt[idx] = (pb.astype(np.uint64) << np.uint64(32)) | pe.astype(np.uint64)
    return pt


def test_verifier_accepts_oracle_and_rejects_corruptions():
    for g, k in ((W.rmat(11, 8, wlo=1, whi=50, master=3), 40), (W.grid(30, 31, 1, 4, 5), 25),
                 (W.er(2000, 6000, 1, 1, 6), 60)):
        _, S = O.canon_seeds(g.n, W.sample(W.lcc(g), k, master=2))
        dist, src = O.voronoi(g, S)
        key = O.packed_key(dist, src)
        assert props.voronoi_fixed_point(g, S, key) == -1
        rc, pi, pj, pb, pe = O.boundary(g, dist, src, len(S))
        pt = _dense(len(S), pi, pj, pb, pe)
        assert props.boundary_exact(g, key, len(S), pt) == 0
        # a vertex one too far, one too near, or in the wrong cell
        reached = np.nonzero((dist != np.iinfo(np.uint64).max) & (dist > 0))[0]
        v = int(reached[len(reached) // 2])
        for delta_key in ((1 << 32), -(1 << 32), 1):
            bad = key.copy()
            bad[v] = np.uint64(int(bad[v]) + delta_key)
            assert props.voronoi_fixed_point(g, S, bad) != -1
        # a pair entry too large (not attained), too small (below a candidate), or an extra pair
        p0 = int(np.nonzero(pt != np.iinfo(np.uint64).max)[0][0])
        for val in (int(pt[p0]) + 1, int(pt[p0]) - 1):
            bad = pt.copy()
            bad[p0] = np.uint64(val)
            assert props.boundary_exact(g, key, len(S), bad) != 0
        empty = np.nonzero(pt == np.iinfo(np.uint64).max)[0]
        if len(empty):
            bad = pt.copy()
            bad[empty[0]] = np.uint64(5)
            assert props.boundary_exact(g, key, len(S), bad) != 0
