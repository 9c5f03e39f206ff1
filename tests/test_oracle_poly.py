"""Pins for negacyclic products, the gadget and the external product.

* Schoolbook product vs. evaluation at the roots of x^N + 1 (the definition of
  the negacyclic NTT) and vs. an exact big-integer convolution.
* x^N = -1 and x^(2N) = 1 for the monomial product.
* Gadget decomposition: digit ranges, the reconstruction error bound
  |x - sum d_u g_u| <= 2^(sg-1) (exact when sg = 0), on the extreme residues and
  a large random sample (the exhaustive sweep over [0, Q) is the slow test).
* External product with a trivial RGSW m diag(g, g) (Sec. 2 item (14)) returns
  m times its input exactly; with a real noise-free key its phase is m times
  the input phase.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
from helpers import Q, evaluate_at_odd_roots, nega_mul, nega_mul_np, primitive_root_2n, rlwe_phase


@pytest.mark.parametrize("N", [8, 32])
def test_schoolbook_vs_root_evaluation(N):
    rng = np.random.default_rng(N)
    a = rng.integers(0, Q, N, dtype=np.uint32)
    b = rng.integers(0, Q, N, dtype=np.uint32)
    c = oracle.poly_mul(a, b, Q)
    psi = primitive_root_2n(N)
    ea, eb, ec = (evaluate_at_odd_roots(p, psi) for p in (a, b, c))
    assert [x * y % Q for x, y in zip(ea, eb)] == ec


@pytest.mark.parametrize("N", [16, 256])
def test_schoolbook_vs_bigint(N):
    rng = np.random.default_rng(N + 1)
    a = rng.integers(0, Q, N, dtype=np.uint32)
    b = rng.integers(0, Q, N, dtype=np.uint32)
    np.testing.assert_array_equal(oracle.poly_mul(a, b, Q), nega_mul(a, b))
    np.testing.assert_array_equal(nega_mul_np(a, b), nega_mul(a, b))


def test_monomial_identities():
    N = 64
    rng = np.random.default_rng(5)
    p = rng.integers(0, Q, N, dtype=np.uint32)
    neg = ((Q - p.astype(np.int64)) % Q).astype(np.uint32)
    np.testing.assert_array_equal(oracle.monomial_mul(p, N, Q), neg)
    np.testing.assert_array_equal(oracle.monomial_mul(p, 2 * N, Q), p)
    for e in (1, 7, N - 1, N + 3):
        mono = np.zeros(N, dtype=np.uint32)
        if e < N:
            mono[e] = 1
        else:
            mono[e - N] = Q - 1
        np.testing.assert_array_equal(oracle.monomial_mul(p, e, Q), nega_mul(mono, p))


def _check_digits(x, log2_B, l):
    sg = oracle.gadget_shift(Q, log2_B, l)
    d = oracle.decompose(x, Q, log2_B, l).astype(np.int64)
    B = 1 << log2_B
    assert np.all(np.abs(d[:-1]) <= B // 2) and np.all(d[:-1] >= -B // 2) and np.all(d[:-1] < B // 2)
    assert abs(d[-1]) <= B // 2
    recon = sum(int(d[u]) << (sg + u * log2_B) for u in range(l))
    xc = x if x <= (Q - 1) // 2 else x - Q
    err = xc - recon
    assert abs(err) <= (1 << (sg - 1) if sg else 0), (x, d, err)
    return d


@pytest.mark.parametrize("log2_B,l,sg", [(8, 3, 7), (7, 4, 3), (8, 4, 0), (6, 5, 1), (10, 3, 1)])
def test_decompose_edges_and_sample(log2_B, l, sg):
    assert oracle.gadget_shift(Q, log2_B, l) == sg
    g = oracle.gadget(Q, log2_B, l)
    assert all(int(g[u]) == pow(2, sg + u * log2_B, Q) for u in range(l))
    edges = [0, 1, 2, (Q - 1) // 2 - 1, (Q - 1) // 2, (Q + 1) // 2, Q - 2, Q - 1]
    edges += [(1 << k) + o for k in range(31) for o in (-1, 0, 1) if 0 <= (1 << k) + o < Q]
    rng = np.random.default_rng(log2_B * 10 + l)
    for x in edges + [int(v) for v in rng.integers(0, Q, 3000)]:
        _check_digits(int(x), log2_B, l)


def test_top_digit_reaches_half_base():
    """With this Q the carry lands in the top digit at exactly B/2 (so it must be kept)."""
    seen = set()
    for log2_B, l in ((8, 3), (7, 4)):
        sg = oracle.gadget_shift(Q, log2_B, l)
        xmax = (Q - 1) // 2
        seen.add(int(_check_digits(xmax, log2_B, l)[-1]))
        # the largest centred values round up into the top digit
        assert int(oracle.decompose(xmax, Q, log2_B, l)[-1]) == (1 << (log2_B - 1)), (log2_B, l, sg)


@pytest.mark.slow
def test_decompose_exhaustive(tmp_path):
    """Every x in [0, Q): digit ranges and error bound (C checker linked to the oracle)."""
    src = os.path.join(os.path.dirname(__file__), "c", "decomp_exhaustive.c")
    exe = tmp_path / "decomp_exhaustive"
    libdir = os.path.dirname(oracle.lib()._name)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-o", str(exe), src, "-L" + libdir, "-loracle",
                    "-Wl,-rpath," + libdir], check=True)
    for log2_B, l in ((8, 3), (7, 4), (8, 4)):
        out = subprocess.run([str(exe), str(Q), str(log2_B), str(l)], check=True,
                             capture_output=True, text=True).stdout
        assert "OK" in out, out


def _trivial_rgsw(m, N, log2_B, l):
    sg = oracle.gadget_shift(Q, log2_B, l)
    C = np.zeros((2 * l, 2, N), dtype=np.uint32)
    for u in range(l):
        g = pow(2, sg + u * log2_B, Q)
        C[u, 1, 0] = m * g % Q       # b column of the first l rows
        C[l + u, 0, 0] = m * g % Q   # a column of the last l rows
    return C


@pytest.mark.parametrize("m", [0, 1])
def test_external_product_trivial_rgsw_exact(m):
    N, log2_B, l = 64, 8, 4  # l log2 B = 32 >= 31 bits: exact gadget
    rng = np.random.default_rng(9 + m)
    ct = rng.integers(0, Q, size=(2, N), dtype=np.uint32)
    out = oracle.external_product(_trivial_rgsw(m, N, log2_B, l), ct, Q, log2_B, l)
    np.testing.assert_array_equal(out, ct if m else np.zeros_like(ct))


def test_external_product_real_key_phase():
    """Noise-free RGSW_z(m), exact gadget: phase(out) = m * phase(in)."""
    from synth import Params, key_draws
    p = Params(n=2, N=64, log2_B=8, l=4, sigma=0.0, sigma_ks=0.0)
    dr = key_draws(p, seed=21)
    dr["s"][:] = [1, 0]
    bsk = oracle.keygen_bsk(p, dr)
    rng = np.random.default_rng(4)
    ct = rng.integers(0, Q, size=(2, p.N), dtype=np.uint32)
    ph = rlwe_phase(ct[0], ct[1], dr["z"])
    for i, m in ((0, 1), (1, 0)):
        out = oracle.external_product(bsk[i], ct, Q, p.log2_B, p.l)
        np.testing.assert_array_equal(rlwe_phase(out[0], out[1], dr["z"]), ph if m else np.zeros_like(ph))
