"""Pins for the oracle at a wide ring modulus (the parameters of the experiments
in Sec. 5: log Q = 54, gadget base 2^15, 2Nr/t = 128).

* Products, rotations and the decomposition against Python big integers.
* Every wide function at a modulus below 2^31 equals the 32-bit oracle (pinned
  on its own in the other files), and reduction mod a factor of Q commutes
  with the ring operations.
* Keys: RGSW rows carry the phases Sec. 2 item (14) states.
* External product with noise-free keys and an exact gadget: the phase is
  multiplied by the key's bit exactly (eq. def:gsw).
* Blind rotation with noise-free keys: the accumulator's phase is
  Phi(b' - sum a'_i s_i)(0, V) exactly (Alg. 1, Theorem 2).
* The rounding switch Q_w -> Q_ks against exact rational rounding.
* End to end with noisy keys and noisy inputs at 2Nr/t = 128: every message
  decrypts to f(m) (Definition 1), the point of the wide modulus.
"""
from dataclasses import replace
from fractions import Fraction

import numpy as np
import pytest

import oracle
from helpers import Q
from synth import Q2_DEFAULT, Params, enc_draws, key_draws, messages, negacyclic_table

QW = Q * Q2_DEFAULT


def big_nega_mul(a, b, q):
    """a * b in Z_q[x]/(x^N+1) with Python integers (brute force)."""
    a = [int(v) for v in a]
    b = [int(v) for v in b]
    N = len(a)
    full = [0] * (2 * N)
    for i, ai in enumerate(a):
        if ai:
            for j, bj in enumerate(b):
                full[i + j] += ai * bj
    return [(full[k] - full[k + N]) % q for k in range(N)]


def big_phase(a, b, z, q):
    az = big_nega_mul(a, z, q)
    return [(int(bv) - av) % q for bv, av in zip(b, az)]


def wide(n, N, r=None, **kw):
    return Params(n=n, N=N, log2_B=kw.pop("log2_B", 15), l=kw.pop("l", 4), Q2=Q2_DEFAULT, **kw)


def test_wide_modulus_is_54_bits_and_prime_factors_are_ntt_friendly():
    assert QW.bit_length() == 54
    for q, twoN in ((Q, 1 << 17), (Q2_DEFAULT, 1 << 13)):
        assert (q - 1) % twoN == 0
        assert all(q % d for d in range(2, int(q ** 0.5) + 1))


@pytest.mark.parametrize("N", [1, 2, 8, 16])
def test_w_poly_mul_brute_force_and_crt(N):
    rng = np.random.default_rng(N)
    a = rng.integers(0, QW, N, dtype=np.uint64)
    b = rng.integers(0, QW, N, dtype=np.uint64)
    a[0] = QW - 1
    got = oracle.w_poly_mul(a, b, QW)
    assert [int(v) for v in got] == big_nega_mul(a, b, QW)
    # reduction mod the factor Q commutes with the product
    np.testing.assert_array_equal((got % Q).astype(np.uint32),
                                  oracle.poly_mul((a % Q).astype(np.uint32), (b % Q).astype(np.uint32), Q))


def test_w_rotate_is_a_group_action_and_reduces_mod_q():
    N, r = 8, 3
    M = 2 * N * r
    rng = np.random.default_rng(3)
    v = rng.integers(0, QW, (r, N), dtype=np.uint64)
    for c1, c2 in ((1, 2), (5, M - 1), (N * r, N * r), (17, 40)):
        np.testing.assert_array_equal(oracle.w_rotate(oracle.w_rotate(v, c1, QW), c2, QW),
                                      oracle.w_rotate(v, c1 + c2, QW))
        np.testing.assert_array_equal((oracle.w_rotate(v, c1, QW) % Q).astype(np.uint32),
                                      oracle.rotate((v % Q).astype(np.uint32), c1, Q))
    # Phi(Nr) = -I
    np.testing.assert_array_equal(oracle.w_rotate(v, N * r, QW), (QW - v) % QW)


@pytest.mark.parametrize("log2_B,l", [(15, 4), (10, 4), (13, 3), (7, 8)])
def test_w_decompose_recomposes_within_the_truncation(log2_B, l):
    sg = oracle.w_gadget_shift(QW, log2_B, l)
    assert sg == max(0, 54 - l * log2_B)
    g = oracle.w_gadget(QW, log2_B, l)
    assert g == [pow(2, sg + u * log2_B, QW) for u in range(l)]
    B = 1 << log2_B
    rng = np.random.default_rng(log2_B * 10 + l)
    xs = [0, 1, QW - 1, (QW - 1) // 2, (QW + 1) // 2, QW // 3] + [int(v) for v in rng.integers(0, QW, 3000, dtype=np.uint64)]
    for x in xs:
        d = [int(v) for v in oracle.w_decompose(x, QW, log2_B, l)]
        for u in range(l - 1):
            assert -B // 2 <= d[u] < B // 2
        rec = sum(du * (1 << (sg + u * log2_B)) for u, du in enumerate(d))
        xc = x - QW if x > (QW - 1) // 2 else x
        err = xc - rec
        # round half up: err in [-2^(sg-1), 2^(sg-1))
        assert (-(1 << sg) // 2 <= err < (1 << sg) // 2) if sg else err == 0, (x, d, err)


def test_w_decompose_equals_the_32bit_decomposition_below_2_31():
    rng = np.random.default_rng(5)
    for log2_B, l in ((7, 4), (8, 3), (15, 2)):
        for x in [0, 1, Q - 1, (Q - 1) // 2, (Q + 1) // 2] + [int(v) for v in rng.integers(0, Q, 500)]:
            np.testing.assert_array_equal(oracle.w_decompose(x, Q, log2_B, l),
                                          oracle.decompose(x, Q, log2_B, l).astype(np.int64))


def test_w_test_vector_scales_the_same_table_by_floor_q_over_t():
    N, r, t, t_out = 16, 4, 32, 32
    f = negacyclic_table(t, t_out, 9)
    Vw = oracle.w_test_vector(N, r, QW, t, t_out, f)
    V32 = oracle.test_vector(N, r, Q, t, t_out, f)
    unscaled = V32.astype(np.uint64) // (Q // t_out)
    assert np.all(V32.astype(np.uint64) == unscaled * (Q // t_out))
    np.testing.assert_array_equal(Vw, unscaled * np.uint64(QW // t_out))


def test_w_bsk_rows_have_the_stated_phase():
    p = wide(2, 16)
    dr = key_draws(p, seed=4)
    assert dr["bsk_a"].dtype == np.uint64 and int(dr["bsk_a"].max()) < QW
    bsk = oracle.w_keygen_bsk(p, dr)
    g = oracle.w_gadget(QW, p.log2_B, p.l)
    z = [int(v) for v in dr["z"]]
    for i in range(p.n):
        s = int(dr["s"][i])
        for row in range(2 * p.l):
            ph = big_phase(bsk[i, row, 0], bsk[i, row, 1], z, QW)
            e = [int(v) for v in dr["bsk_e"][i, row]]
            u = row % p.l
            if row < p.l:
                msg = [s * g[u]] + [0] * (p.N - 1)
            else:
                msg = [-s * g[u] * zk for zk in z]
            assert ph == [(ek + mk) % QW for ek, mk in zip(e, msg)], (i, row)


@pytest.mark.parametrize("log2_B,l", [(15, 4), (10, 4)])
def test_w_external_product_multiplies_the_phase(log2_B, l):
    p = replace(wide(2, 16, log2_B=log2_B, l=l), sigma=0.0)
    dr = key_draws(p, seed=6)
    bsk = oracle.w_keygen_bsk(p, dr)
    z = [int(v) for v in dr["z"]]
    sg = oracle.w_gadget_shift(QW, log2_B, l)
    rng = np.random.default_rng(7)
    for i in range(p.n):
        m = int(dr["s"][i])
        rl = rng.integers(0, QW, (2, p.N), dtype=np.uint64)
        out = oracle.w_external_product(bsk[i], rl, QW, log2_B, l)
        mu = big_phase(rl[0], rl[1], z, QW)
        got = big_phase(out[0], out[1], z, QW)
        if sg == 0:
            assert got == [(m * v) % QW for v in mu]
        else:
            bound = (1 << (sg - 1)) * (1 + p.N)
            for gv, mv in zip(got, mu):
                diff = (gv - m * mv) % QW
                diff = diff - QW if diff > QW // 2 else diff
                assert abs(diff) <= bound


@pytest.mark.parametrize("ternary", [False, True])
def test_w_blind_rotate_noise_free_phase(ternary):
    """With noise-free keys and an exact gadget the accumulator phase is exactly
    Phi(b' - <a', s>)(0, V)."""
    p = replace(wide(6, 16, ternary=ternary), sigma=0.0)
    r, t = 2, 16
    M = 2 * p.N * r
    dr = key_draws(p, seed=8 + ternary)
    bsk = oracle.w_keygen_bsk(p, dr)
    f = negacyclic_table(t, t, 10)
    V = oracle.w_test_vector(p.N, r, QW, t, t, f)
    rng = np.random.default_rng(11)
    z = [int(v) for v in dr["z"]]
    for _ in range(3):
        ct = rng.integers(0, M, p.n + 1).astype(np.uint32)
        acc = oracle.w_blind_rotate(p, r, bsk, V, ct)
        ph = (int(ct[p.n]) - sum(int(a) * int(s) for a, s in zip(ct[:p.n], dr["s"]))) % M
        want = oracle.w_rotate(V, ph, QW)
        for j in range(r):
            assert big_phase(acc[j, 0], acc[j, 1], z, QW) == [int(v) for v in want[j]]


def test_w_modswitch_rounds_half_up_without_ties():
    rng = np.random.default_rng(12)
    xs = [0, 1, QW - 1, Q2_DEFAULT // 2, Q2_DEFAULT // 2 + 1] + [int(v) for v in rng.integers(0, QW, 2000, dtype=np.uint64)]
    got = oracle.w_modswitch(np.array(xs, dtype=np.uint64), QW, Q)
    for x, g in zip(xs, got):
        exact = Fraction(x * Q, QW)
        assert exact.denominator != 2 or exact.numerator % 2 == 0  # never a tie
        assert int(g) == int(exact + Fraction(1, 2)) % Q


def test_w_sample_extract_keeps_the_constant_phase():
    N = 16
    rng = np.random.default_rng(13)
    z = rng.integers(0, 2, N).astype(np.uint32)
    rl = rng.integers(0, QW, (2, N), dtype=np.uint64)
    lwe = oracle.w_sample_extract(rl, QW)
    ph = big_phase(rl[0], rl[1], [int(v) for v in z], QW)[0]
    assert (int(lwe[N]) - sum(int(a) * int(zz) for a, zz in zip(lwe[:N], z))) % QW == ph


@pytest.mark.parametrize("ternary", [False, True])
def test_w_functions_equal_the_32bit_oracle_below_2_31(ternary):
    """At a ring modulus below 2^31 the wide oracle and the 32-bit one give the same bits."""
    p = Params(n=8, N=32, log2_B=7, l=4, ternary=ternary)
    dr = key_draws(p, seed=14)
    bsk32 = oracle.keygen_bsk(p, dr)
    drw = dict(dr, bsk_a=dr["bsk_a"].astype(np.uint64))
    bskw = oracle.w_keygen_bsk(p, drw)
    np.testing.assert_array_equal(bskw, bsk32.astype(np.uint64))
    ksk = oracle.keygen_ksk(p, dr)
    r, t = 2, 32
    q = 2 * p.N * r
    f = negacyclic_table(t, t, 15)
    V32 = oracle.test_vector(p.N, r, Q, t, t, f)
    Vw = oracle.w_test_vector(p.N, r, Q, t, t, f)
    np.testing.assert_array_equal(Vw, V32.astype(np.uint64))
    s = dr["s"]
    ed = enc_draws(p.n, q, 4, 16)
    ct = oracle.encrypt(p.n, q, t, s, messages(t, 4, 17), ed["a"], ed["e"])
    np.testing.assert_array_equal(oracle.w_blind_rotate(p, r, bskw, Vw, ct[0], 5),
                                  oracle.blind_rotate(p, r, bsk32, V32, ct[0], 5).astype(np.uint64))
    # with Q_ks = Q_w the switch after extraction is the identity
    np.testing.assert_array_equal(oracle.w_bootstrap_many(p, r, bskw, ksk, Vw, q, q, ct),
                                  oracle.bootstrap_many(p, r, bsk32, ksk, V32, q, q, ct))


@pytest.mark.parametrize("r,seed", [(1, 20), (4, 21)])
def test_w_noisy_inputs_decrypt_at_delta_128(r, seed):
    """Noisy keys (sigma 3.2) and fresh noisy encryptions at q = 2Nr, t = 2Nr/128:
    every message bootstraps to f(m)."""
    p = wide(24, 256)
    t = 2 * p.N * r // 128
    q = 2 * p.N * r
    dr = key_draws(p, seed)
    keys = oracle.KeySetWide(p, dr)
    f = negacyclic_table(t, t, seed + 1)
    V = oracle.w_test_vector(p.N, r, QW, t, t, f)
    m = np.arange(t, dtype=np.uint32)
    ed = enc_draws(p.n, q, t, seed + 2, sigma=3.2)
    ct = oracle.encrypt(p.n, q, t, keys.s, m, ed["a"], ed["e"])
    assert np.any(ed["e"] != 0)
    out = oracle.w_bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(oracle.decrypt(p.n, q, t, keys.s, out), f[m])
    # the output noise stays well inside Delta / 2 = 64
    ph = oracle.lwe_phase(p.n, q, keys.s, out).astype(np.int64)
    err = (ph - f[m].astype(np.int64) * (q // t)) % q
    err = np.where(err > q // 2, err - q, err)
    assert np.max(np.abs(err)) < 32


def test_w_bootstrap_single_equals_many_and_extracts_at_q():
    p = wide(8, 64)
    r, t = 2, 2
    q = 2 * p.N * r
    dr = key_draws(p, 30)
    keys = oracle.KeySetWide(p, dr)
    f = negacyclic_table(t, t, 31)
    V = oracle.w_test_vector(p.N, r, QW, t, t, f)
    ed = enc_draws(p.n, q, 3, 32)
    ct = oracle.encrypt(p.n, q, t, keys.s, messages(t, 3, 33), ed["a"], ed["e"])
    many = oracle.w_bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, ct)
    for k in range(3):
        one, ext = oracle.w_bootstrap(p, r, keys.bsk, keys.ksk, V, q, q, ct[k], ext_out=True)
        np.testing.assert_array_equal(one, many[k])
        assert ext.max() < Q


def test_w_general_equals_the_32bit_general_below_2_31():
    p = Params(n=8, N=32, log2_B=7, l=4)
    dr = key_draws(p, 40)
    keys = oracle.KeySet(p, dr)
    bskw = oracle.w_keygen_bsk(p, dict(dr, bsk_a=dr["bsk_a"].astype(np.uint64)))
    r, t = 2, 8
    q = 2 * p.N * r
    f = np.arange(t, dtype=np.uint32)[::-1].copy()
    g, F = oracle.general_tables(t, t, f)
    Vg, VF = oracle.test_vector(p.N, r, Q, 2 * t, 2 * t, g), oracle.test_vector(p.N, r, Q, 2 * t, t, F)
    ed = enc_draws(p.n, q, 3, 41)
    ct = oracle.encrypt(p.n, q, 2 * t, keys.s, messages(t, 3, 42), ed["a"], ed["e"])
    want = np.stack([oracle.bootstrap_general(p, r, keys.bsk, keys.ksk, Vg, VF, q, t, q, ct[k]) for k in range(3)])
    got = oracle.w_bootstrap_general(p, r, bskw, keys.ksk, Vg.astype(np.uint64), VF.astype(np.uint64), q, t, q, ct)
    np.testing.assert_array_equal(got, want)


def test_w_identity_function_by_two_bootstraps_decrypts_at_delta_128():
    """The workload of the experiments in Sec. 5: f(x) = x (not nega-cyclic), two
    bootstraps; noisy inputs at plaintext modulus 2t with 2Nr/(2t) = 128."""
    p = wide(24, 256)
    r = 4
    t = 2 * p.N * r // 128 // 2  # the input carries m + b t in Z_2t
    q = 2 * p.N * r
    dr = key_draws(p, 43)
    keys = oracle.KeySetWide(p, dr)
    f = np.arange(t, dtype=np.uint32)
    g, F = oracle.general_tables(t, t, f)
    Vg = oracle.w_test_vector(p.N, r, QW, 2 * t, 2 * t, g)
    VF = oracle.w_test_vector(p.N, r, QW, 2 * t, t, F)
    m = np.arange(t, dtype=np.uint32)
    ed = enc_draws(p.n, q, t, 44, sigma=3.2)
    ct = oracle.encrypt(p.n, q, 2 * t, keys.s, m, ed["a"], ed["e"])
    out = oracle.w_bootstrap_general(p, r, keys.bsk, keys.ksk, Vg, VF, q, t, q, ct)
    np.testing.assert_array_equal(oracle.decrypt(p.n, q, t, keys.s, out), m)


def test_w_switch_after_extraction_scales_the_phase():
    """After extraction each coefficient is switched Q_w -> Q by rounding, so the
    sample's phase at Q is the accumulator's constant phase at Q_w times Q / Q_w,
    up to the rounding of N + 1 terms: |err| <= (||z||_1 + 1) / 2 (Sec. 2 item (9))."""
    p = wide(6, 32)
    r, t = 2, 4
    q = 2 * p.N * r
    dr = key_draws(p, 50)
    keys = oracle.KeySetWide(p, dr)
    f = negacyclic_table(t, t, 51)
    V = oracle.w_test_vector(p.N, r, QW, t, t, f)
    z = [int(v) for v in dr["z"]]
    ed = enc_draws(p.n, q, 4, 52)
    cts = oracle.encrypt(p.n, q, t, keys.s, messages(t, 4, 53), ed["a"], ed["e"])
    for ct in cts:
        acc = oracle.w_blind_rotate(p, r, keys.bsk, V, ct)
        ph_w = big_phase(acc[0, 0], acc[0, 1], z, QW)[0]
        _, ext = oracle.w_bootstrap(p, r, keys.bsk, keys.ksk, V, q, q, ct, ext_out=True)
        ph_q = (int(ext[p.N]) - sum(int(a) * zk for a, zk in zip(ext[:p.N], z))) % Q
        want = Fraction(ph_w * Q, QW)
        diff = (ph_q - want) % Q
        diff = diff - Q if diff > Q // 2 else diff
        assert abs(diff) <= Fraction(sum(z) + 1, 2), (ph_w, ph_q, float(diff))
