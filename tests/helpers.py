"""Shared test helpers: gauge-invariant comparisons of couplings."""

import numpy as np


def degenerate_groups(e, tol=1e-6):
    """Group labels of an ascending-ish energy vector: |diff| < tol joins a group."""
    order = np.argsort(e, kind="stable")
    labels = np.empty(len(e), dtype=np.int64)
    g = 0
    prev = None
    for i in order:
        if prev is not None and abs(e[i] - e[prev]) >= tol:
            g += 1
        labels[i] = g
        prev = i
    return labels


def group_sum_g2(g, eps_n, eps_m, omega, tol=1e-6):
    """|g_{nu n m}|^2 summed over degenerate groups of n, m and nu.

    g [nu, n, m]; returns an array of the same shape holding, at each entry,
    the sum of |g|^2 over the degenerate group the entry belongs to.  This is
    invariant under any unitary mixing inside degenerate subspaces.
    """
    g2 = np.abs(g) ** 2
    ln = degenerate_groups(eps_n, tol)
    lm = degenerate_groups(eps_m, tol)
    lv = degenerate_groups(omega, tol)
    if len(np.unique(ln)) == len(ln) and len(np.unique(lm)) == len(lm) and \
            len(np.unique(lv)) == len(lv):
        return g2  # no degeneracy: every group is one entry
    out = np.zeros_like(g2)
    for a in np.unique(lv):
        va = lv == a
        for b in np.unique(ln):
            nb = ln == b
            for c in np.unique(lm):
                mc = lm == c
                s = g2[np.ix_(va, nb, mc)].sum()
                out[np.ix_(va, nb, mc)] = s
    return out


def random_unitary(rng, n):
    a = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(2)
    q, r = np.linalg.qr(a)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def random_rotation(rng):
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q
