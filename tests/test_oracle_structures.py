"""Pins of the oracle's reference vectors (R1) and neighbourhoods (R2)."""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("m,n_req,H,n_eff", [(2, 100, 99, 100), (3, 1000, 44, 1035),
                                             (3, 100000, 446, 100128), (2, 2, 1, 2),
                                             (3, 91, 12, 91), (3, 92, 13, 105)])
def test_das_dennis_sizes(oracle_core, m, n_req, H, n_eff):
    assert oracle_core.dd_H(m, n_req) == H
    assert oracle_core.dd_count(m, H) == n_eff == math.comb(H + m - 1, m - 1)
    # H is the smallest such value
    assert H == 1 or math.comb(H - 1 + m - 1, m - 1) < n_req


@pytest.mark.parametrize("m,H", [(2, 9), (3, 12), (4, 5)])
def test_das_dennis_lattice(oracle_core, m, H):
    K = oracle_core.dd_lattice(m, H)
    assert K.shape == (math.comb(H + m - 1, m - 1), m)
    assert np.all(K >= 0) and np.all(K.sum(1) == H)
    # distinct rows in ascending lexicographic order of the leading m-1 entries
    lead = [tuple(r[:-1]) for r in K]
    assert lead == sorted(lead) and len(set(lead)) == len(lead)
    # every composition of H into m parts appears (brute force)
    import itertools
    allc = [c for c in itertools.product(range(H + 1), repeat=m) if sum(c) == H]
    assert sorted(map(tuple, K)) == sorted(allc)


def _knn_brute(K, t):
    """Independent kNN: full sort by (squared distance, index)."""
    K = K.astype(np.int64)
    out = []
    for i in range(K.shape[0]):
        d = ((K - K[i]) ** 2).sum(1)
        order = np.lexsort((np.arange(K.shape[0]), d))
        out.append(order[:t])
    return np.array(out, dtype=np.int32)


@pytest.mark.parametrize("m,H,t", [(2, 99, 10), (2, 99, 40), (3, 12, 5), (3, 12, 20), (3, 20, 64)])
def test_knn_against_full_sort(oracle_core, m, H, t):
    K = oracle_core.dd_lattice(m, H)
    B = oracle_core.knn(K, t)
    assert np.array_equal(B, _knn_brute(K, t))
    assert np.all(B[:, 0] == np.arange(K.shape[0]))           # self first
    assert all(len(set(r)) == t for r in B)                    # distinct


def test_reverse_lists(oracle_core):
    K = oracle_core.dd_lattice(3, 15)
    N = K.shape[0]
    t = 16
    B = oracle_core.knn(K, t)
    rev = [[] for _ in range(N)]
    for i in range(N):
        for j in B[i]:
            rev[j].append(i)
    assert sum(len(r) for r in rev) == N * t
    for j in range(N):
        for i in rev[j]:
            assert j in B[i]
    for i in range(N):
        for j in B[i]:
            assert i in rev[j]
