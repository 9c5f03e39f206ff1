"""Statistical pins for the oracle's noise (Sec. 4).

The paper's error analysis gives variance proxies: 2 N l_B B^2 sigma^2 added per
external product (the bound (GSW:error)), beta^2 + 4 N l_B B^2 sigma^2 for the CMux
of Lemma 8, and for the whole bootstrap Theorem 2's three terms: the phase
accumulation, N l_KS sigma_KS^2 for the key switch, and (||s||^2 + 1) / 12 for the
last modulus switch, each scaled by (q/Q)^2 where it applies.  Specialised to
what the oracle computes (a binary secret, so one external product per step;
balanced digits; a truncated gadget), the expected squared error has a closed form:

* per blind-rotation step with a'_i != 0: E[d^2] ||e||^2 summed over the 2l key
  rows, with E[d^2] = (B^2 + 2)/12 for digits uniform on [-B/2, B/2), plus, when
  s_i = 1, the gadget's rounding error eps (uniform on [-2^(sg-1), 2^(sg-1)),
  mean -1/2, variance (4^sg - 1)/12) on b and through z on a;
* per key switch: N l_KS sigma_KS^2;
* per modulus switch: (||s||^2 + 1)/12.

Each check compares a mean square over a few thousand samples with its
prediction (relative standard error about 2-3 %; the bands are about 4 of
those); the blind rotation's also stays under the paper's proxy, and a
zero-mask key switch gives its error exactly.  Unbalanced digits
(4x), a gadget shift off by one (4x on the rounding term), a key switch
that skips the v = 0 rows or a modulus switch that truncates (mean -1/2, not 0)
all fall outside the bands.
"""
import numpy as np
import pytest

import oracle
from helpers import Q
from synth import Params, enc_draws, key_draws, negacyclic_table


def _nega_matrix(z):
    """Integer matrix M with M @ a = a * z in Z[x]/(x^N + 1)."""
    N = z.size
    M = np.zeros((N, N), dtype=np.int64)
    for j in range(N):
        for k in range(N):
            M[j, k] = z[j - k] if k <= j else -z[j - k + N]
    return M


def _centred(x, q):
    x = np.asarray(x, dtype=np.int64) % q
    return np.where(x > q // 2, x - q, x)


def _acc_errors(acc, z_mat, want_b):
    """Phase error of every coefficient of every component: (b - a z) - want."""
    a = acc[:, 0, :].astype(np.int64)
    b = acc[:, 1, :].astype(np.int64)
    ph = (b - (a @ z_mat.T)) % Q
    return _centred(ph - want_b.astype(np.int64), Q)


def _phi(v, c):
    """Phi(c) on integer (r, N) arrays: multiplication by Y^c in Z[Y]/(Y^(Nr) + 1)
    of the interleaved vector W[alpha r + beta] = v[beta][alpha] (Sec. 3)."""
    r, N = v.shape
    W = v.T.reshape(-1)
    src = (np.arange(N * r) - c) % (2 * N * r)
    out = np.where(src < N * r, W[src % (N * r)], -W[src % (N * r)])
    return out.reshape(N, r).T


def _blind_rotation_errors(p, r, draws, cts):
    """Error that steps 1 .. n-1 add, per coefficient and component.  A step with
    s_i = 1 rotates the error it receives by Phi(-a'_i), so the first step's error
    (made while the accumulator's mask is still zero) reaches the end rotated by
    Phi(-sum_{i>=1} a'_i s_i); it is taken off in that form.  Rotations keep the
    sum of squares, so the rest has the per-step variance summed over the steps."""
    bsk = oracle.keygen_bsk(p, draws)
    M = 2 * p.N * r
    t = 2 * r
    f = negacyclic_table(t, t, seed=5)
    V = oracle.test_vector(p.N, r, Q, t, t, f)
    z_mat = _nega_matrix(draws["z"].astype(np.int64))
    s = draws["s"].astype(np.int64)
    errs, steps_on = [], []
    for ct in cts:
        a = ct[:p.n].astype(np.int64)
        phase = (int(ct[p.n]) - int(a @ s)) % M
        phase_1 = (int(ct[p.n]) - int(a[0] * s[0])) % M
        e_n = _acc_errors(oracle.blind_rotate(p, r, bsk, V, ct), z_mat, oracle.rotate(V, phase, Q))
        e_1 = _acc_errors(oracle.blind_rotate(p, r, bsk, V, ct, steps=1), z_mat, oracle.rotate(V, phase_1, Q))
        errs.append(e_n - _phi(e_1, int(-(a[1:] @ s[1:])) % M))
        steps_on.append(ct[1:p.n] % M != 0)
    return np.array(errs), np.array(steps_on)


def _rounding_var(p, s, steps_on, z):
    """Variance of the gadget-rounding part per coefficient, per ciphertext: the
    term s_i (eps_b - z * eps_a) of each step with D != 0.  (eps has mean -1/2; the
    squared mean it adds is below 0.1 % of this at the shifts used here.)"""
    sg = oracle.gadget_shift(Q, p.log2_B, p.l)
    var_eps = (4.0 ** sg - 1) / 12
    k = (s[1:p.n] == 1)[None, :] & steps_on
    return k.sum(axis=1) * (1 + int(z.sum())) * var_eps, var_eps


def test_blind_rotation_error_matches_the_digit_and_key_variance():
    p = Params(n=32, N=64, log2_B=8, l=3)  # gadget shift 7
    r = 2
    draws = key_draws(p, seed=31)
    rng = np.random.default_rng(32)
    M = 2 * p.N * r
    cts = rng.integers(0, M, size=(32, p.n + 1), dtype=np.uint32)
    err, on = _blind_rotation_errors(p, r, draws, cts)
    B = 1 << p.log2_B
    e2 = draws["bsk_e"].astype(np.float64) ** 2          # (n, 2l, N)
    key_energy = e2.sum(axis=(1, 2))[1:]                # per step i >= 1
    gauss = (on * key_energy[None, :]).sum(axis=1) * (B * B + 2) / 12  # per ciphertext
    rnd, _ = _rounding_var(p, draws["s"], on, draws["z"])
    pred = (gauss + rnd) * r * p.N                      # summed over components and coefficients
    ratio = float((err.astype(np.float64) ** 2).sum() / pred.sum())
    assert 0.9 < ratio < 1.1, ratio
    # the paper's proxy for the same steps is an upper bound (12x looser for balanced digits)
    proxy = (p.n - 1) * 2 * p.N * p.l * B * B * p.sigma ** 2
    assert float((err.astype(np.float64) ** 2).mean()) < proxy / 8


def test_gadget_rounding_error_alone():
    # noise-free keys: what remains is s_i times the truncated gadget's rounding error
    p = Params(n=32, N=64, log2_B=7, l=3).noise_free()  # gadget shift 10
    r = 2
    draws = key_draws(p, seed=41)
    rng = np.random.default_rng(42)
    cts = rng.integers(0, 2 * p.N * r, size=(32, p.n + 1), dtype=np.uint32)
    err, on = _blind_rotation_errors(p, r, draws, cts)
    pred, var_eps = _rounding_var(p, draws["s"], on, draws["z"])
    ratio = float((err.astype(np.float64) ** 2).sum() / (pred * r * p.N).sum())
    assert 0.9 < ratio < 1.1, ratio
    assert var_eps == (4.0 ** 10 - 1) / 12


def test_keyswitch_error_variance():
    p = Params(n=48, N=128)
    draws = key_draws(p, seed=51)
    ksk = oracle.keygen_ksk(p, draws)
    rng = np.random.default_rng(52)
    count = 3000
    z = draws["z"].astype(np.int64)
    s = draws["s"].astype(np.int64)
    A = rng.integers(0, Q, size=(count, p.N), dtype=np.uint32)
    msg = rng.integers(0, Q, size=count, dtype=np.int64)
    lwe = np.concatenate([A, ((A.astype(np.int64) @ z + msg) % Q).astype(np.uint32)[:, None]], axis=1)
    out = np.array([oracle.keyswitch(p, ksk, c) for c in lwe])
    ph = (out[:, p.n].astype(np.int64) - (out[:, :p.n].astype(np.int64) @ s) % Q) % Q
    err = _centred(ph - msg, Q).astype(np.float64)
    # Theorem 2's second term at q = Q is N l_KS sigma_KS^2; for the realised key the
    # error is minus one row error per (i, j), picked by a digit uniform on its range
    # (the top digit of a value below Q < 2^31 takes 8 values, the others B_ks)
    e = draws["ksk_e"].astype(np.float64)
    m1 = np.zeros(e.shape[:2])
    m2 = np.zeros(e.shape[:2])
    for j in range(p.l_ks):
        vals = min(p.B_ks, ((Q - 1) >> (p.log2_Bks * j)) + 1)
        m1[:, j] = e[:, j, :vals].mean(axis=1)
        m2[:, j] = (e[:, j, :vals] ** 2).mean(axis=1)
    var = float((m2 - m1 ** 2).sum())
    mean = -float(m1.sum())
    # averaged over keys, var + mean^2 is N l_KS sigma_KS^2 (each row error has
    # variance sigma^2): Theorem 2's term; for one key the split between the two varies
    assert 0.9 < float((err ** 2).mean()) / (var + mean ** 2) < 1.1
    assert abs(float(err.mean()) - mean) < 4 * np.sqrt(var / count)
    # a zero mask selects the v = 0 row of every (i, j): the error is exactly minus their sum
    zero = np.zeros(p.N + 1, dtype=np.uint32)
    zero[p.N] = 12345
    o = oracle.keyswitch(p, ksk, zero).astype(np.int64)
    got = int(_centred((o[p.n] - o[:p.n] @ s) - 12345, Q))
    assert got == -int(draws["ksk_e"][:, :, 0].astype(np.int64).sum())


@pytest.mark.parametrize("q_to", [1024, 4096])
def test_modswitch_rounding_variance(q_to):
    n = 64
    rng = np.random.default_rng(q_to)
    s = rng.integers(0, 2, n).astype(np.int64)
    count = 6000
    ct = rng.integers(0, Q, size=(count, n + 1), dtype=np.uint32)
    out = oracle.modswitch(ct, Q, q_to).astype(np.int64)
    phase_Q = (ct[:, n].astype(np.int64) - (ct[:, :n].astype(np.int64) @ s) % Q) % Q
    phase_q = (out[:, n] - out[:, :n] @ s) % q_to
    # error of the switched phase against the exact rational (q/Q) phase, centred mod q
    err = phase_q - phase_Q.astype(np.float64) * q_to / Q
    err = (err + q_to / 2) % q_to - q_to / 2
    pred = (float(s @ s) + 1) / 12                      # Theorem 2's third term
    assert 0.9 < float((err ** 2).mean()) / pred < 1.1
    assert abs(float(err.mean())) < 4 * np.sqrt(pred / count)
