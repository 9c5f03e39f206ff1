"""Pins for the oracle's keys, blind rotation, extraction, key switch and the
whole of Algorithm 1.

* Key phases: RGSW rows carry e_u + s_i g_u and e - s_i g_u z; KSK rows carry
  e + v z_i B_ks^j (Sec. 2 items (11), (14)).
* Encrypt/decrypt round trip and the BFV phase (Sec. 2 item (8)).
* Blind rotation with a trivial key (z = 0, no noise, exact gadget): the
  accumulator's b part is exactly Phi(phase') (0, V) -- the closed form of the
  phase accumulation (Alg. 1 and the first step of Theorem 2's proof).
* Sample extraction keeps the constant coefficient of the RLWE phase.
* The key switch keeps the phase exactly when its keys are noise-free and the
  digits are exact (l_ks log2 B_ks >= 31).
* End to end: decrypt(bootstrap(Enc(m))) = f(m) for every m at the tiny size
  and several key seeds (Definition 1).
* Key sizes reproduce the printed sizes of Tables 1 and 2 (golden file).
"""
import os

import numpy as np
import pytest

import oracle
from helpers import Q, nega_mul_np, rlwe_phase
from synth import PRESETS, Params, enc_draws, key_draws, messages, negacyclic_table

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_bsk_rows_have_the_stated_phase():
    p = Params(n=3, N=32, log2_B=7, l=4)
    dr = key_draws(p, seed=1)
    bsk = oracle.keygen_bsk(p, dr)
    g = oracle.gadget(Q, p.log2_B, p.l)
    for i in range(p.n):
        s = int(dr["s"][i])
        for row in range(2 * p.l):
            ph = rlwe_phase(bsk[i, row, 0], bsk[i, row, 1], dr["z"]).astype(np.int64)
            e = dr["bsk_e"][i, row].astype(np.int64)
            u = row % p.l
            msg = np.zeros(p.N, dtype=np.int64)
            if row < p.l:
                msg[0] = s * int(g[u])
            elif s:
                gz = np.zeros(p.N, dtype=np.int64)
                gz[0] = int(g[u])
                msg = -nega_mul_np(gz, dr["z"]).astype(np.int64)
            np.testing.assert_array_equal(ph, (e + msg) % Q)
            if row < p.l:
                np.testing.assert_array_equal(bsk[i, row, 0], dr["bsk_a"][i, row])


def test_ksk_rows_have_the_stated_phase():
    p = Params(n=5, N=8, log2_Bks=4, l_ks=8)
    dr = key_draws(p, seed=2)
    ksk = oracle.keygen_ksk(p, dr)
    s = dr["s"].astype(np.int64)
    for i in range(p.N):
        for j in range(p.l_ks):
            for v in range(p.B_ks):
                row = ksk[i, j, v].astype(np.int64)
                ph = (row[p.n] - row[:p.n] @ s) % Q
                want = (int(dr["ksk_e"][i, j, v]) + v * int(dr["z"][i]) * pow(16, j, Q)) % Q
                assert ph == want


@pytest.mark.parametrize("q,t", [(1024, 16), (8192, 4096), (Q, 4096)])
def test_encrypt_decrypt_roundtrip(q, t):
    n = 40
    dr = key_draws(Params(n=n, N=8), seed=3)
    m = messages(t, 200, seed=4)
    ed = enc_draws(n, q, 200, seed=5, sigma=3.2 if q // t > 64 else 0.0)
    ct = oracle.encrypt(n, q, t, dr["s"], m, ed["a"], ed["e"])
    ph = (ct[:, n].astype(np.int64) - ct[:, :n].astype(np.int64) @ dr["s"].astype(np.int64)) % q
    np.testing.assert_array_equal(ph, (m.astype(np.int64) * (q // t) + ed["e"]) % q)
    np.testing.assert_array_equal(oracle.decrypt(n, q, t, dr["s"], ct), m)


def trivial_bsk(p, s, rng):
    """RGSW_z(s_i) with z = 0, no noise: random a, b = m g on rows u < l."""
    sg = oracle.gadget_shift(Q, p.log2_B, p.l)
    bsk = np.zeros((p.n, 2 * p.l, 2, p.N), dtype=np.uint32)
    bsk[:, :, 0, :] = rng.integers(0, Q, size=(p.n, 2 * p.l, p.N), dtype=np.uint32)
    for i in range(p.n):
        for u in range(p.l):
            g = pow(2, sg + u * p.log2_B, Q)
            bsk[i, u, 1, 0] = int(s[i]) * g % Q
            bsk[i, p.l + u, 0, 0] = (int(bsk[i, p.l + u, 0, 0]) + int(s[i]) * g) % Q
    return bsk


@pytest.mark.parametrize("N,r,n", [(16, 3, 9), (32, 2, 20), (8, 1, 12), (16, 5, 7)])
def test_blind_rotation_trivial_key_closed_form(N, r, n):
    p = Params(n=n, N=N, log2_B=8, l=4)  # exact gadget
    rng = np.random.default_rng(N + r + n)
    s = rng.integers(0, 2, n)
    bsk = trivial_bsk(p, s, rng)
    M = 2 * N * r
    t = 2 * r * N // 2
    f = negacyclic_table(t, 64, seed=N)
    V = oracle.test_vector(N, r, Q, t, 64, f)
    for trial in range(4):
        ct_ms = rng.integers(0, M, n + 1, dtype=np.uint32)
        acc = oracle.blind_rotate(p, r, bsk, V, ct_ms)
        phase = (int(ct_ms[n]) - int(ct_ms[:n].astype(np.int64) @ s)) % M
        np.testing.assert_array_equal(acc[:, 1, :], oracle.rotate(V, phase, Q))
        # stopping after k steps gives the partial phase
        k = int(rng.integers(0, n))
        acc_k = oracle.blind_rotate(p, r, bsk, V, ct_ms, steps=k)
        phase_k = (int(ct_ms[n]) - int(ct_ms[:k].astype(np.int64) @ s[:k])) % M
        np.testing.assert_array_equal(acc_k[:, 1, :], oracle.rotate(V, phase_k, Q))


def test_sample_extract_keeps_constant_term():
    N = 64
    rng = np.random.default_rng(17)
    z = rng.integers(0, 2, N).astype(np.uint32)
    for _ in range(5):
        rl = rng.integers(0, Q, size=(2, N), dtype=np.uint32)
        lwe = oracle.sample_extract(rl, Q)
        ph_lwe = (int(lwe[N]) - int(lwe[:N].astype(np.int64) @ z.astype(np.int64))) % Q
        assert ph_lwe == int(rlwe_phase(rl[0], rl[1], z)[0])


def test_keyswitch_preserves_phase_noise_free():
    p = Params(n=20, N=32, log2_Bks=4, l_ks=8).noise_free()
    dr = key_draws(p, seed=8)
    ksk = oracle.keygen_ksk(p, dr)
    rng = np.random.default_rng(1)
    z = dr["z"].astype(np.int64)
    s = dr["s"].astype(np.int64)
    for _ in range(10):
        c = rng.integers(0, Q, p.N + 1, dtype=np.uint32)
        out = oracle.keyswitch(p, ksk, c)
        ph_in = (int(c[p.N]) - int(c[:p.N].astype(np.int64) @ z)) % Q
        ph_out = (int(out[p.n]) - int(out[:p.n].astype(np.int64) @ s)) % Q
        assert ph_in == ph_out


def _tiny_case(seed):
    pre = PRESETS["tiny"]
    p, t, t_out, r = pre["params"], pre["t"], pre["t_out"], pre["r"]
    keys = oracle.KeySet(p, key_draws(p, seed))
    f = negacyclic_table(t, t_out, seed + 1000)
    V = oracle.test_vector(p.N, r, Q, t, t_out, f)
    q = 2 * p.N * r
    m = np.arange(t, dtype=np.uint32)
    ed = enc_draws(p.n, q, t, seed + 2000)
    ct = oracle.encrypt(p.n, q, t, keys.s, m, ed["a"], ed["e"])
    return p, keys, f, V, q, t, t_out, r, m, ct


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_end_to_end_tiny_exhaustive(seed):
    p, keys, f, V, q, t, t_out, r, m, ct = _tiny_case(seed)
    out = oracle.bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(oracle.decrypt(p.n, q, t_out, keys.s, out), f[m])


@pytest.mark.slow
def test_end_to_end_tiny_many_seeds():
    for seed in range(3, 103):
        p, keys, f, V, q, t, t_out, r, m, ct = _tiny_case(seed)
        out = oracle.bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, ct)
        np.testing.assert_array_equal(oracle.decrypt(p.n, q, t_out, keys.s, out), f[m])


def test_end_to_end_intermediates_consistent():
    p, keys, f, V, q, t, t_out, r, m, ct = _tiny_case(5)
    out, acc, ext, ks = keys.bootstrap(r, V, q, q, ct[3], intermediates=True)
    np.testing.assert_array_equal(ext, oracle.sample_extract(acc[0], Q))
    np.testing.assert_array_equal(ks, oracle.keyswitch(p, keys.ksk, ext))
    np.testing.assert_array_equal(out, oracle.modswitch(ks, Q, q))
    # decrypting the extracted sample under z and the switched one under s at Q
    assert oracle.decrypt(p.N, Q, t_out, keys.z, ext)[0] == f[3]
    assert oracle.decrypt(p.n, Q, t_out, keys.s, ks)[0] == f[3]


def _parse_size(txt):
    for unit, scale in (("GB", 2 ** 30), ("MB", 2 ** 20)):
        if txt.endswith(unit):
            return float(txt[:-2]), scale
    raise ValueError(txt)


def test_key_sizes_match_tables():
    for line in open(os.path.join(GOLD, "key_sizes.txt")):
        if line.startswith("#") or not line.strip():
            continue
        _, scheme, logn, logN, bsk_txt, ksk_txt = line.split()
        n, N = 1 << int(logn), 1 << int(logN)
        lB, B_ks, l_ks = 4, 25, 12
        bsk = oracle.bsk_bytes(n, N, lB, word_bytes=8, keys_per_coord=2)
        ksk = oracle.ksk_bytes(n, N, B_ks, l_ks, word_bytes=8)
        for got, txt in ((bsk, bsk_txt), (ksk, ksk_txt)):
            val, scale = _parse_size(txt)
            digits = len(txt[:-2].split(".")[1]) if "." in txt else 0
            assert round(got / scale, digits) == pytest.approx(val), (line, got / scale)


@pytest.mark.parametrize("q_from,q_to", [(Q, 8192), (Q, 1024), (8192, 8192), (1 << 20, 2048), (Q, 16384)])
def test_modswitch_is_nearest_integer(q_from, q_to):
    """|x q'/q - out| <= 1/2 with exact rationals (Sec. 2 item (9)), ties upward."""
    from fractions import Fraction
    rng = np.random.default_rng(q_to)
    xs = np.concatenate([rng.integers(0, q_from, 2000), [0, 1, q_from - 1, q_from // 2]]).astype(np.uint32)
    out = oracle.modswitch(xs, q_from, q_to)
    for x, o in zip(xs.tolist(), out.tolist()):
        exact = Fraction(x * q_to, q_from)
        hi = exact + Fraction(1, 2)
        k = hi.numerator // hi.denominator  # floor(exact + 1/2): nearest integer, ties upward
        assert o == k % q_to, (x, o, exact)


def _general_case(seed, t=8, t_out=16, identity=False):
    from synth import Params
    p = Params(n=64, N=256, log2_B=8, l=3)
    r = 2
    keys = oracle.KeySet(p, key_draws(p, seed))
    rng = np.random.default_rng(seed)
    f = np.arange(t, dtype=np.uint32) % t_out if identity else rng.integers(0, t_out, t).astype(np.uint32)
    g, F = oracle.general_tables(t, t_out, f)
    Vg = oracle.test_vector(p.N, r, Q, 2 * t, 2 * t, g)
    VF = oracle.test_vector(p.N, r, Q, 2 * t, t_out, F)
    q = 2 * p.N * r
    m = np.repeat(np.arange(t, dtype=np.uint32), 2)
    b = np.tile(np.array([0, 1], dtype=np.uint32), t)  # unknown top bit of the Z_2t plaintext
    ed = enc_draws(p.n, q, m.size, seed + 7)
    ct = oracle.encrypt(p.n, q, 2 * t, keys.s, m + b * t, ed["a"], ed["e"])
    return p, r, keys, f, Vg, VF, q, t, t_out, m, ct


def test_general_tables_are_negacyclic():
    f = np.array([3, 0, 7, 7, 1, 5, 2, 6], dtype=np.uint32)
    g, F = oracle.general_tables(8, 8, f)
    np.testing.assert_array_equal(F[:8], f)
    assert all((int(F[x]) + int(F[x + 8])) % 8 == 0 for x in range(8))
    assert all((int(g[x]) + int(g[x + 8])) % 16 == 0 for x in range(8))
    assert set(g[:8].tolist()) == {4}


@pytest.mark.parametrize("seed,identity", [(0, False), (1, False), (2, True)])
def test_general_function_two_bootstraps(seed, identity):
    """A function that is not nega-cyclic, on Z_2t inputs with an unknown top
    bit: MSB removal by a sign bootstrap, then the nega-cyclic extension of f
    (Sec. 4, end; identity f is the workload of Tables 1-2)."""
    p, r, keys, f, Vg, VF, q, t, t_out, m, ct = _general_case(seed, identity=identity)
    for c in range(ct.shape[0]):
        out = oracle.bootstrap_general(p, r, keys.bsk, keys.ksk, Vg, VF, q, t, q, ct[c])
        assert oracle.decrypt(p.n, q, t_out, keys.s, out)[0] == f[m[c]], (c, m[c])


# ---------------------------------------------------------------- ternary secret (Alg. 1 as printed)

def test_ternary_bsk_encrypts_s_plus_and_s_minus():
    p = Params(n=6, N=32, log2_B=7, l=4, ternary=True)
    dr = key_draws(p, 40)
    assert set(dr["s"].tolist()) <= {-1, 0, 1}
    bsk = oracle.keygen_bsk(p, dr)
    g = oracle.gadget(Q, p.log2_B, p.l)
    for i in range(p.n):
        for key, m in ((0, max(int(dr["s"][i]), 0)), (1, max(-int(dr["s"][i]), 0))):
            row = 0  # row u = 0 carries m g_0 on b
            ph = rlwe_phase(bsk[2 * i + key, row, 0], bsk[2 * i + key, row, 1], dr["z"]).astype(np.int64)
            want = dr["bsk_e"][2 * i + key, row].astype(np.int64)
            want[0] += m * int(g[0])
            np.testing.assert_array_equal(ph, want % Q)


@pytest.mark.parametrize("N,r,n", [(16, 3, 9), (8, 2, 14)])
def test_ternary_blind_rotation_trivial_key_closed_form(N, r, n):
    """With trivial keys, ACC.b = Phi(b' - sum a'_i s_i) V for s in {-1, 0, 1}^n (eq. cmux:BP)."""
    p = Params(n=n, N=N, log2_B=8, l=4, ternary=True)
    rng = np.random.default_rng(N * r + n)
    s = rng.integers(-1, 2, n)
    sg = oracle.gadget_shift(Q, p.log2_B, p.l)
    bsk = np.zeros((2 * n, 2 * p.l, 2, N), dtype=np.uint32)
    bsk[:, :, 0, :] = rng.integers(0, Q, size=(2 * n, 2 * p.l, N), dtype=np.uint32)
    for i in range(n):
        for key, m in ((0, max(int(s[i]), 0)), (1, max(-int(s[i]), 0))):
            for u in range(p.l):
                gu = pow(2, sg + u * p.log2_B, Q)
                bsk[2 * i + key, u, 1, 0] = m * gu % Q
                bsk[2 * i + key, p.l + u, 0, 0] = (int(bsk[2 * i + key, p.l + u, 0, 0]) + m * gu) % Q
    M = 2 * N * r
    t = N * r
    f = negacyclic_table(t, 64, seed=N)
    V = oracle.test_vector(N, r, Q, t, 64, f)
    for _ in range(3):
        ct_ms = rng.integers(0, M, n + 1, dtype=np.uint32)
        acc = oracle.blind_rotate(p, r, bsk, V, ct_ms)
        phase = (int(ct_ms[n]) - int(ct_ms[:n].astype(np.int64) @ s)) % M
        np.testing.assert_array_equal(acc[:, 1, :], oracle.rotate(V, phase, Q))


@pytest.mark.parametrize("seed", [0, 1])
def test_ternary_end_to_end_tiny(seed):
    from dataclasses import replace
    pre = PRESETS["tiny"]
    p = replace(pre["params"], ternary=True)
    t, t_out, r = pre["t"], pre["t_out"], pre["r"]
    keys = oracle.KeySet(p, key_draws(p, seed + 50))
    f = negacyclic_table(t, t_out, seed + 60)
    V = oracle.test_vector(p.N, r, Q, t, t_out, f)
    q = 2 * p.N * r
    m = np.arange(t, dtype=np.uint32)
    ed = enc_draws(p.n, q, t, seed + 70)
    ct = oracle.encrypt(p.n, q, t, keys.s, m, ed["a"], ed["e"])
    out = oracle.bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(oracle.decrypt(p.n, q, t_out, keys.s, out), f[m])


def test_ternary_keyswitch_preserves_phase():
    p = Params(n=20, N=32, ternary=True).noise_free()
    dr = key_draws(p, 41)
    ksk = oracle.keygen_ksk(p, dr)
    rng = np.random.default_rng(2)
    z = dr["z"].astype(np.int64)
    s = dr["s"].astype(np.int64)
    for _ in range(5):
        c = rng.integers(0, Q, p.N + 1, dtype=np.uint32)
        out = oracle.keyswitch(p, ksk, c)
        assert (int(c[p.N]) - int(c[:p.N].astype(np.int64) @ z)) % Q == (int(out[p.n]) - int(out[:p.n].astype(np.int64) @ s)) % Q
