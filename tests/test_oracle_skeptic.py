"""Pins of the Skeptic oracle: the paper's worked example (ranks exactly, the
transformed values and the sparse + rank-one split to the two printed
decimals), the rank definition by brute force, and the split identity."""
import json
import os

import numpy as np

from oracle import skeptic as SK

GOLD = os.path.join(os.path.dirname(__file__), "golden", "skeptic_worked_example.json")


def test_paper_worked_example():
    g = json.load(open(GOLD))
    X = np.asarray(g["data"], dtype=np.float64).T          # variables are the example's rows
    F = SK.skeptic_dense(X)
    np.testing.assert_allclose(F.T, np.asarray(g["transformed_2dp"]), atol=0.006)
    n = X.shape[0]
    R = np.round((n + 1) * 0.5 * (1 + np.vectorize(__import__("math").erf)(F / np.sqrt(2.0)))).T
    np.testing.assert_array_equal(R, np.asarray(g["ranks"]))
    S, z = SK.skeptic_split(X)
    np.testing.assert_allclose(z, np.asarray(g["split_z_2dp"]), atol=0.006)
    np.testing.assert_allclose(S.T, np.asarray(g["split_sparse_2dp"]), atol=0.011)


def test_rank_definition_brute_force():
    rng = np.random.default_rng(3)
    X = rng.integers(-3, 4, size=(23, 6)).astype(np.float64)
    X[rng.random(X.shape) < 0.4] = 0.0
    F = SK.skeptic_dense(X)
    n = X.shape[0]
    for g in range(X.shape[1]):
        for i in range(n):
            rank = 1 + sum(1 for t in range(n) if X[t, g] < X[i, g])
            q = rank / (n + 1.0)
            # Phi(F) == q, through the erf closed form
            assert abs(0.5 * (1 + __import__("math").erf(F[i, g] / np.sqrt(2.0))) - q) < 1e-12


def test_split_identity_and_pattern():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((50, 9))
    X[rng.random(X.shape) < 0.7] = 0.0
    X[:, 3] = 0.0                                          # an all-zero column
    S, z = SK.skeptic_split(X)
    np.testing.assert_allclose(S + z[None, :], SK.skeptic_dense(X), atol=1e-14)
    assert np.all(S[X == 0.0] == 0.0)
    # monotone: order within a column is kept, ties stay tied
    F = SK.skeptic_dense(X)
    for g in range(X.shape[1]):
        o = np.argsort(X[:, g], kind="stable")
        assert np.all(np.diff(F[o, g]) >= 0)
