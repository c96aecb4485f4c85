"""Uniform-mesh bookkeeping (Computational structure, Points class).

A Monkhorst-Pack mesh N = (N0, N1, N2) is an implicit, sorted list of points:
the paper increments the third coordinate fastest, then the second, then the
first.  Point (i0, i1, i2) has crystal coordinates (i0/N0, i1/N1, i2/N2) and
linear index (i0*N1 + i1)*N2 + i2; the lookup of a mesh point is O(1) by that
formula.  On a mesh, k + q is again a mesh point: per axis (i + j) mod N.
"""

import numpy as np


def mesh_triples(n):
    """Integer coordinates of every mesh point, in linear-index order ([N, 3] int64)."""
    n0, n1, n2 = (int(x) for x in n)
    out = np.empty((n0 * n1 * n2, 3), dtype=np.int64)
    idx = 0
    for i0 in range(n0):
        for i1 in range(n1):
            for i2 in range(n2):
                out[idx] = (i0, i1, i2)
                idx += 1
    return out


def mesh_points(n):
    """Crystal coordinates of every mesh point, in linear-index order ([N, 3] float64)."""
    t = mesh_triples(n)
    return t / np.asarray(n, dtype=np.float64)[None, :]


def linear_index(triple, n):
    i0, i1, i2 = (int(x) for x in triple)
    return (i0 * int(n[1]) + i1) * int(n[2]) + i2


def triple_of(index, n):
    index = int(index)
    i2 = index % int(n[2])
    index //= int(n[2])
    i1 = index % int(n[1])
    i0 = index // int(n[1])
    return (i0, i1, i2)


def sum_index(ik, iq, n):
    """Linear index of k + q folded back onto the mesh."""
    a = triple_of(ik, n)
    b = triple_of(iq, n)
    return linear_index(tuple((a[d] + b[d]) % int(n[d]) for d in range(3)), n)


def sum_index_table(k_index, n):
    """[len(k_index), N] table of linear indices of k + q for every mesh q."""
    tq = mesh_triples(n)
    out = np.empty((len(k_index), tq.shape[0]), dtype=np.int64)
    nn = np.asarray(n, dtype=np.int64)
    for a, ik in enumerate(k_index):
        tk = np.asarray(triple_of(ik, n), dtype=np.int64)
        s = (tq + tk[None, :]) % nn[None, :]
        out[a] = (s[:, 0] * nn[1] + s[:, 1]) * nn[2] + s[:, 2]
    return out
