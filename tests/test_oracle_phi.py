"""Pins for the oracle's MMPM rotation Phi (Sec. 3).

Phi(1) is checked against the matrix printed in Example 1 (golden file); every
other Phi(c) is then pinned by the group law Phi(c) = Phi(1)^c computed with a
generic monomial-matrix product, by Phi(r) = x I, Phi(Nr) = -I (Lemma 6), the
order 2Nr (Lemma 4), the r = 1 and x = 1 special cases of Example 1, and by
the interleaved reading Y^c in Z[Y]/(Y^(Nr)+1), Y^r = x.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from helpers import Q, dense_matvec, monomial_matrix_mul

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def phi_rows(N, r, c):
    rows = []
    for j in range(r):
        col, e = oracle.phi_entry(N, r, c, j)
        sign = 1
        e %= 2 * N
        if e >= N:
            e -= N
            sign = -1
        rows.append((col, sign, e))
    return rows


def test_generator_matches_example_1():
    rows = {}
    for line in open(os.path.join(GOLD, "phi_generator.txt")):
        if line.startswith("#") or not line.strip():
            continue
        r, j, col, e = map(int, line.split())
        rows.setdefault(r, {})[j] = (col, e)
    for r, entries in rows.items():
        for N in (2, 4, 8):
            for j, (col, e) in entries.items():
                assert oracle.phi_entry(N, r, 1, j) == (col, e), (r, N, j)


@pytest.mark.parametrize("N,r", [(1, 1), (2, 1), (4, 1), (2, 2), (4, 3), (4, 4), (8, 4), (2, 5)])
def test_group_law_exhaustive(N, r):
    """Phi(u) Phi(v) = Phi(u + v) for all u, v in Z_{2Nr}, and Phi(c) = Phi(1)^c."""
    M = 2 * N * r
    table = [phi_rows(N, r, c) for c in range(M)]
    gen = table[1]
    power = [(j, 1, 0) for j in range(r)]  # identity
    for c in range(M):
        assert table[c] == power, (N, r, c)
        power = monomial_matrix_mul(power, gen, N)
    assert power == table[0]
    for u, v in itertools.product(range(M), repeat=2):
        assert monomial_matrix_mul(table[u], table[v], N) == table[(u + v) % M]


@pytest.mark.parametrize("N,r", [(4, 1), (4, 3), (8, 4), (16, 2)])
def test_special_elements_and_order(N, r):
    ident = [(j, 1, 0) for j in range(r)]
    assert phi_rows(N, r, r) == [(j, 1, 1) for j in range(r)]            # Phi(r) = x I
    assert phi_rows(N, r, N * r) == [(j, -1, 0) for j in range(r)]       # Phi(Nr) = -I
    M = 2 * N * r
    assert phi_rows(N, r, M) == ident
    assert all(phi_rows(N, r, c) != ident for c in range(1, M))           # ord = 2Nr


def test_r1_is_monomial_and_x1_is_cyclic_shift():
    N = 8
    for c in range(2 * N):  # r = 1: Phi(c) = x^c
        col, e = oracle.phi_entry(N, 1, c, 0)
        assert col == 0 and e == c
    r = 5  # x = 1: the index part is the AP14 cyclic shift by c mod r
    for c in range(2 * N * r):
        for j in range(r):
            col, _ = oracle.phi_entry(N, r, c, j)
            assert col == (j - c) % r


@pytest.mark.parametrize("N,r", [(4, 3), (8, 4), (8, 1), (4, 5)])
def test_rotate_equals_matrix_vector_product(N, r):
    rng = np.random.default_rng(7)
    v = rng.integers(0, Q, size=(r, N), dtype=np.uint32)
    for c in range(0, 2 * N * r, max(1, (2 * N * r) // 23)):
        got = oracle.rotate(v, c, Q)
        want = dense_matvec(phi_rows(N, r, c), v)
        np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("N,r", [(4, 3), (8, 4), (16, 2)])
def test_rotate_is_interleaved_negacyclic_shift(N, r):
    """W[alpha r + beta] = v_beta[alpha]; Phi(c) acts as Y^c in Z_Q[Y]/(Y^(Nr)+1)."""
    rng = np.random.default_rng(11)
    v = rng.integers(0, Q, size=(r, N), dtype=np.uint32)
    W = v.T.reshape(-1)
    L = N * r
    for c in range(2 * L):
        out = np.zeros(L, dtype=np.int64)
        for p in range(L):
            k = p + c
            sign = 1
            k %= 2 * L
            if k >= L:
                k -= L
                sign = -1
            out[k] = W[p] if sign > 0 else (Q - int(W[p])) % Q
        want = out.reshape(N, r).T
        np.testing.assert_array_equal(oracle.rotate(v, c, Q), want)
