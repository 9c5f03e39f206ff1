"""Pins for the test polynomial vector and the look-up property (Sec. 3, Example 2).

* Layout: entry b, coefficient a of v_test holds f'(-(a r + b)) (golden file
  transcribed from eq. (equ:test-use)).
* The nega-cyclic extension: f'(m Delta + e) = f(m) for 2|e| < Delta and
  f'(x + Nr) = -f'(x) (Sec. 2 item (7)).
* Eq. (equ:ex): for every m, Phi(m) v_test has f'(m - a r - d) at entry d,
  coefficient a -- so the constant term of entry 0 is f'(m) (Lemma 7).
"""
import os

import numpy as np
import pytest

import oracle
from helpers import Q

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def decode(v, t_out):
    """Nearest multiple of floor(Q/t') -> residue mod t'."""
    dq = Q // t_out
    return ((np.asarray(v, np.int64) + dq // 2) // dq) % t_out


def test_layout_matches_example_2():
    rows = [tuple(map(int, s.split())) for s in open(os.path.join(GOLD, "test_vector_layout.txt"))
            if s.strip() and not s.startswith("#")]
    r, N = 3, 4
    M = 2 * N * r
    t = M  # Delta = 1: f' = f, every index distinct
    f = np.array([(7 * i + 3) % 97 for i in range(t // 2)], dtype=np.int64)
    f = np.concatenate([f, (-f) % 128]).astype(np.uint32)
    V = oracle.test_vector(N, r, Q, t, 128, f)
    dec = decode(V, 128)
    for b, a, idx in rows:
        assert dec[b, a] == f[idx] % 128, (b, a, idx)


@pytest.mark.parametrize("N,r,t,t_out", [(8, 2, 16, 16), (8, 3, 12, 32), (16, 4, 8, 8), (4, 1, 8, 64)])
def test_extension_properties(N, r, t, t_out):
    M = 2 * N * r
    D = M // t
    rng = np.random.default_rng(N * 100 + r)
    half = rng.integers(0, t_out, size=t // 2)
    f = np.concatenate([half, (-half) % t_out]).astype(np.uint32)
    V = oracle.test_vector(N, r, Q, t, t_out, f)
    # f'(x) read back from V through the layout: f'(-(a r + b)) at (b, a)
    fext = {}
    for b in range(r):
        for a in range(N):
            fext[(-(a * r + b)) % M] = int(decode(V[b, a], t_out))
    for x, val in fext.items():
        m, e = divmod(x + D // 2, D)  # nearest multiple of Delta, half up
        e -= D // 2
        assert 2 * abs(e) <= D
        if 2 * abs(e) < D:
            assert val == f[m % t], (x, m, e)
    # nega-cyclic: the stored half [0, Nr) of -index range and its negation
    for x in range(M):
        if x in fext and (x + N * r) % M in fext:
            assert (fext[x] + fext[(x + N * r) % M]) % t_out == 0


@pytest.mark.parametrize("N,r,t,t_out", [(8, 2, 16, 16), (8, 3, 12, 32), (4, 4, 32, 64), (16, 1, 8, 8)])
def test_rotated_test_vector_equation_ex(N, r, t, t_out):
    M = 2 * N * r
    D = M // t
    rng = np.random.default_rng(3 + N + r)
    half = rng.integers(0, t_out, size=t // 2)
    f = np.concatenate([half, (-half) % t_out]).astype(np.uint32)

    def fprime(x):  # nega-cyclic extension to Z_M
        m = ((x % M) + D // 2) // D
        return int(f[m % t])

    V = oracle.test_vector(N, r, Q, t, t_out, f)
    for m in range(M):
        R = decode(oracle.rotate(V, m, Q), t_out)
        want = np.array([[fprime(m - a * r - d) for a in range(N)] for d in range(r)])
        np.testing.assert_array_equal(R, want % t_out)
        assert R[0, 0] == fprime(m)  # Lemma 7: f'(m) lands in the constant term of entry 0
