"""Independent brute-force arithmetic used by the pins (no oracle code here)."""
from __future__ import annotations

import numpy as np

Q = 2147352577


def nega_mul(a, b, q: int = Q) -> np.ndarray:
    """a * b in Z_q[x]/(x^N+1) via Python big ints: full convolution, then fold
    the upper half with a minus sign (x^N = -1)."""
    a = [int(v) for v in a]
    b = [int(v) for v in b]
    N = len(a)
    full = [0] * (2 * N)
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j, bj in enumerate(b):
            full[i + j] += ai * bj
    return np.array([(full[k] - full[k + N]) % q for k in range(N)], dtype=np.uint32)


def nega_mul_np(a, b, q: int = Q) -> np.ndarray:
    """Same product with numpy object arithmetic split to stay exact: b is split
    into 16-bit halves so each float-free int64 convolution stays below 2^63."""
    a = np.asarray(a, dtype=np.int64) % q
    b = np.asarray(b, dtype=np.int64) % q
    N = a.size
    out = np.zeros(N, dtype=object)
    for shift in (0, 16):
        part = (b >> shift) & 0xFFFF
        full = np.convolve(a.astype(object), part.astype(object))
        full = np.concatenate([full, np.zeros(2 * N - full.size, dtype=object)])
        out = out + (full[:N] - full[N:]) * (1 << shift)
    return np.array([int(v) % q for v in out], dtype=np.uint32)


def poly_sub(a, b, q: int = Q) -> np.ndarray:
    return ((np.asarray(a, np.int64) - np.asarray(b, np.int64)) % q).astype(np.uint32)


def rlwe_phase(a, b, z, q: int = Q) -> np.ndarray:
    """b - a z for one RLWE pair."""
    return poly_sub(b, nega_mul_np(a, z, q), q)


def primitive_root_2n(N: int, q: int = Q) -> int:
    """A primitive 2N-th root of unity mod prime q (q = 1 mod 2N)."""
    assert (q - 1) % (2 * N) == 0
    for g in range(2, 10_000):
        psi = pow(g, (q - 1) // (2 * N), q)
        if pow(psi, N, q) == q - 1:
            return psi
    raise ValueError("no root")


def evaluate_at_odd_roots(p, psi: int, q: int = Q) -> list[int]:
    """p(psi^(2k+1)) for k < N: the roots of x^N + 1 (definition of the
    negacyclic transform)."""
    N = len(p)
    out = []
    for k in range(N):
        w = pow(psi, 2 * k + 1, q)
        acc, x = 0, 1
        for c in p:
            acc = (acc + int(c) * x) % q
            x = (x * w) % q
        out.append(acc)
    return out


def monomial_matrix_mul(A, B, N: int):
    """Product of two r x r monomial-permutation matrices given as lists of
    (col, sign, exp) per row: (AB)(i, k) = sum_j A(i, j) B(j, k)."""
    r = len(A)
    out = []
    for i in range(r):
        ca, sa, ea = A[i]
        cb, sb, eb = B[ca]
        e = ea + eb
        sign = sa * sb
        e %= 2 * N
        if e >= N:
            e -= N
            sign = -sign
        out.append((cb, sign, e))
    return out


def dense_matvec(rows, v, q: int = Q):
    """rows: per row (col, sign, exp) of a monomial matrix over Z_q[x]/(x^N+1);
    v: (r, N).  Computes the matrix-vector product with the generic product."""
    r, N = v.shape
    out = np.zeros_like(v)
    for i, (col, sign, e) in enumerate(rows):
        mono = np.zeros(N, dtype=np.int64)
        mono[e] = 1 if sign > 0 else q - 1
        out[i] = nega_mul(mono, v[col], q)
    return out
