"""Mesh bookkeeping of the oracle pinned by brute-force enumeration (Points class)."""

import itertools

import numpy as np

from oracle import mesh


def test_ordering_last_coordinate_fastest():
    n = (3, 4, 5)
    brute = list(itertools.product(range(3), range(4), range(5)))
    t = mesh.mesh_triples(n)
    assert [tuple(x) for x in t] == brute
    for i, tr in enumerate(brute):
        assert mesh.linear_index(tr, n) == i
        assert mesh.triple_of(i, n) == tr
    p = mesh.mesh_points(n)
    assert np.allclose(p[7], np.array(brute[7]) / np.array(n))


def test_sum_index_folds_per_axis():
    n = (3, 2, 4)
    pts = list(itertools.product(range(3), range(2), range(4)))
    tab = mesh.sum_index_table(list(range(len(pts))), n)
    for ik, a in enumerate(pts):
        for iq, b in enumerate(pts):
            c = tuple((a[d] + b[d]) % n[d] for d in range(3))
            j = pts.index(c)
            assert tab[ik, iq] == j
            assert mesh.sum_index(ik, iq, n) == j
