"""Pins for the oracle's model generators (Eq. A_def with the model rates).

Checked by brute force (a dense matrix assembled reaction by reaction), by the
structural counts of the two workload grids, by the generator properties the
paper states (non-negative off-diagonals, rows of A summing to 0 so rows of B
sum to 1, Eq. B_def) and by the birth-death exit-rate formula the paper prints
(Sec. 3.1.1).
"""
import json
import os

import numpy as np
import pytest

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def dense_from_reactions(model, theta, dims, leaky):
    """Assemble A densely by walking states and reactions (independent of the
    CSR builder's loop structure)."""
    if model == 0:
        (N,) = dims[:1]
        beta, gamma = theta
        A = np.zeros((N, N))
        for n in range(N):
            for dn, rate in ((+1, beta), (-1, gamma * n)):
                m = n + dn
                if rate == 0:
                    continue
                if 0 <= m < N:
                    A[n, m] += rate
                    A[n, n] -= rate
                elif leaky:
                    A[n, n] -= rate
        return A
    S1, S2 = dims
    k1, g1, k2, g2 = theta
    N = S1 * S2
    A = np.zeros((N, N))
    for n2 in range(S2):
        for n1 in range(S1):
            n = n1 + S1 * n2
            for (d1, d2), rate in (((1, 0), k1), ((-1, 0), g1 * n1), ((0, 1), k2 * n1), ((0, -1), g2 * n2)):
                if rate == 0:
                    continue
                m1, m2 = n1 + d1, n2 + d2
                if 0 <= m1 < S1 and 0 <= m2 < S2:
                    A[n, m1 + S1 * m2] += rate
                    A[n, n] -= rate
                elif leaky:
                    A[n, n] -= rate
    return A


@pytest.mark.parametrize("leaky", [False, True])
def test_bd_dense_bruteforce(orc, leaky):
    A = orc.model_generator(0, [7.5, 1.3], [12], leaky=leaky)
    ref = dense_from_reactions(0, [7.5, 1.3], [12], leaky)
    assert np.array_equal(A.dense(), ref)


@pytest.mark.parametrize("leaky", [False, True])
def test_cascade2_dense_bruteforce(orc, leaky):
    th = [3.0, 0.7, 0.4, 0.9]
    A = orc.model_generator(1, th, [6, 5], leaky=leaky)
    ref = dense_from_reactions(1, th, [6, 5], leaky)
    assert np.allclose(A.dense(), ref, rtol=0, atol=1e-14)


def test_generator_properties(orc):
    for model, th, dims in ((0, [500, 1], [1000]), (1, [200, 1, 0.5, 0.5], [60, 70])):
        A = orc.model_generator(model, th, dims)
        D = A.dense() if A.n <= 5000 else None
        rows = np.add.reduceat(A.val, A.row_ptr[:-1])
        assert np.abs(rows).max() < 1e-9
        r = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
        off = A.col != r
        assert (A.val[off] > 0).all()
        assert (A.val[~off] <= 0).all()
        # each row sorted by column, one diagonal entry
        for i in range(0, A.n, max(1, A.n // 50)):
            c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
            assert (np.diff(c) > 0).all() and (c == i).sum() == 1
        if D is not None:
            assert np.allclose(D.sum(1), 0, atol=1e-9)


def test_bd_max_exit_rate_matches_paper(orc):
    """Sec. 3.1.1: max_n |a_nn| = beta + gamma (N-1) when the birth out of the
    top state still counts (the leaky reading)."""
    assert GOLDEN["bd_max_exit_rate"]["formula"] == "beta + gamma*(N-1)"
    for beta, gamma, N in ((500.0, 1.0, 1000), (50.0, 2.0, 77)):
        A = orc.model_generator(0, [beta, gamma], [N], leaky=True)
        diag = A.val[A.col == np.repeat(np.arange(A.n), np.diff(A.row_ptr))]
        assert np.max(np.abs(diag)) == beta + gamma * (N - 1)
        A = orc.model_generator(0, [beta, gamma], [N], leaky=False)
        diag = A.val[A.col == np.repeat(np.arange(A.n), np.diff(A.row_ptr))]
        assert np.max(np.abs(diag)) == max(beta + gamma * (N - 2), gamma * (N - 1))


def test_workload_grid_counts(orc):
    """Stored entries of the cascade generator on an S1 x S2 grid:
    S1*S2 diagonals + (S1-1)*S2 births and (S1-1)*S2 deaths of species 1
    + (S1-1)*(S2-1) births of species 2 (rate k2*n1 vanishes at n1 = 0)
    + S1*(S2-1) deaths of species 2."""
    for S1, S2 in ((300, 300), (1000, 1000), (7, 11)):
        A = orc.model_generator(1, [200, 1, 0.5, 0.5], [S1, S2])
        expect = S1 * S2 + 2 * (S1 - 1) * S2 + (S1 - 1) * (S2 - 1) + S1 * (S2 - 1)
        assert A.nnz == expect
    assert orc.model_generator(1, [200, 1, 0.5, 0.5], [300, 300]).nnz == 448501
    assert orc.model_generator(0, [500, 1], [1000]).nnz == 2998


def test_dense_memory_wall_claim():
    """Sec. 1: a dense FP64 matrix at N = 44722 exceeds 16 GB (and N = 44721
    would not): a consistency check of how the paper counts bytes."""
    g = GOLDEN["dense_memory_wall"]
    assert g["N"] ** 2 * 8 > g["bytes_exceed"] >= (g["N"] - 1) ** 2 * 8
