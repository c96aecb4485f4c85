"""Pins of the oracle's Philox stream, network initialisation and training-set builder."""

import numpy as np

from oracle import mlp, rng


def test_block_matches_numpy_philox():
    # numpy's Philox bit generator is an independent implementation of the same
    # block function; it advances its counter before each block
    for ctr, key in [(0, 0), (3, 5), (2 ** 63 + 11, 2 ** 64 - 7), (123456789, 42)]:
        bg = np.random.Philox(key=np.array([key, 0], dtype=np.uint64),
                              counter=np.array([ctr, 0, 0, 0], dtype=np.uint64))
        ref = [int(x) for x in bg.random_raw(4)]
        assert rng.philox4x64_int([ctr + 1, 0, 0, 0], [key, 0]) == ref
        words = rng.philox4x64(np.array([ctr + 1], dtype=np.uint64), key)
        assert [int(w[0]) for w in words] == ref


def test_zero_block_known_answer():
    # the published known-answer block of Philox-4x64-10 for zero counter and key
    assert rng.philox4x64_int([0, 0, 0, 0], [0, 0]) == [
        0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


def test_vectorised_equals_integer_form():
    c = np.array([0, 1, 2 ** 32 - 1, 2 ** 32, 2 ** 64 - 1, 987654321987], dtype=np.uint64)
    w = rng.philox4x64(c, 77)
    for i, ci in enumerate(c):
        ref = rng.philox4x64_int([int(ci), 0, 0, 0], [77, 0])
        assert [int(w[j][i]) for j in range(4)] == ref


def test_uniform_stream_properties():
    u = rng.uniform(9, 0, 200_000)
    assert u.min() >= 0.0 and u.max() < 1.0
    # mean and variance of U[0, 1) within 5 standard errors
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / u.size)
    # offsets index the same stream
    assert np.array_equal(rng.uniform(9, 1000, 50), u[1000:1050])
    # 53-bit values: u * 2^53 is an integer
    assert np.all(np.floor(u[:1000] * 2 ** 53) == u[:1000] * 2 ** 53)
    r = rng.randint(9, 0, 200_000, 7)
    assert r.min() == 0 and r.max() == 6
    counts = np.bincount(r, minlength=7)
    assert np.all(np.abs(counts - r.size / 7) < 5 * np.sqrt(r.size / 7))


def test_init_layout_and_range():
    n_in, width, depth = 5, 8, 2
    th = mlp.init_params_philox(3, n_in, width, depth)
    assert th.size == mlp.n_params(n_in, width, depth)
    for (W, b), (o, i) in zip(mlp.unpack(th, n_in, width, depth), mlp.layer_shapes(n_in, width, depth)):
        assert np.all(b == 0.0)
        assert np.all(np.abs(W) < 1.0 / np.sqrt(i))
    # weight j is (2 u_j - 1)/sqrt(in) of the stream element at its packed position
    u = rng.uniform(3, 0, th.size)
    assert th[7] == (2 * u[7] - 1) / np.sqrt(n_in)


def test_training_set_by_brute_force():
    g = np.random.default_rng(4)
    ns, nq, nm = 3, 11, 4
    D = g.exponential(size=(ns, nq, nm)) * (g.uniform(size=(ns, nq, nm)) > 0.3)
    T = D * g.lognormal(size=D.shape)
    thr, cf = 0.05, 1e-3
    st, q, nu, y, c = mlp.training_set(T, D, thr, cf, max_samples=10 ** 9, seed=1)
    # everything selected is kept when max_samples is large; explicit loops
    sel = []
    for s in range(ns):
        dm = D[s].max()
        for a in range(nq):
            for v in range(nm):
                if D[s, a, v] > thr * dm:
                    sel.append((s, a, v))
    assert list(zip(st, q, nu)) == sel
    ratios = np.array([T[s, a, v] / D[s, a, v] for s, a, v in sel])
    assert np.isclose(c, cf * ratios.mean(), rtol=1e-14)
    assert np.allclose(y, np.log(ratios + c), rtol=1e-14)
    # subsampling keeps a Philox-decided subset of about the requested size
    st2, q2, nu2, y2, _ = mlp.training_set(T, D, thr, cf, max_samples=len(sel) // 2, seed=1)
    assert set(zip(st2, q2, nu2)) <= set(sel)
    assert abs(len(st2) - len(sel) / 2) < 5 * np.sqrt(len(sel) / 4)
