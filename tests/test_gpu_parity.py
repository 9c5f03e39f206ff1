"""GPU parity: every row of the hot path through the C ABI against the oracle.

The HIP library and the oracle build their keys, test vectors and ciphertexts
from the same draws (synth) independently; every comparison is bit-exact
(tolerance 0), since the whole path is exact integer arithmetic.
"""
import os

import numpy as np
import pytest

import oracle
from synth import CLASS_MIX, PRESETS, Params, class_mix, enc_draws, key_draws, messages, negacyclic_table

pytestmark = pytest.mark.gpu
Q = 2147352577


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_12441_amd import binding
    return binding


class Case:
    """Product context + oracle keys for one parameter set."""

    def __init__(self, p, seed):
        b = _gpu()
        self.p = p
        self.draws = key_draws(p, seed)
        self.ctx = b.Context(p, self.draws)
        self.keys = oracle.KeySet(p, self.draws)
        self.ctx.device_init(0)

    def table(self, t, t_out, r, seed, q_in=0):
        f = negacyclic_table(t, t_out, seed)
        tid = self.ctx.table_create(t, t_out, r, f, q_in)
        V = oracle.test_vector(self.p.N, r, Q, t, t_out, f)
        return tid, f, V

    def encrypt(self, q, t, m, seed, sigma=3.2):
        ed = enc_draws(self.p.n, q, len(m), seed, sigma)
        return oracle.encrypt(self.p.n, q, t, self.keys.s, m, ed["a"], ed["e"])


@pytest.fixture(scope="module")
def tiny():
    return Case(PRESETS["tiny"]["params"], 11)


@pytest.fixture(scope="module")
def paper():
    return Case(PRESETS["paper_shaped"]["params"], 12)


def say(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------- single rows

@pytest.mark.parametrize("q_from,q_to", [(Q, 8192), (8192, 8192), (1 << 20, 2048), (Q, 1024)])
def test_modswitch(tiny, q_from, q_to):
    say("modswitch", q_from, q_to)
    rng = np.random.default_rng(q_to)
    x = rng.integers(0, q_from, 5000, dtype=np.uint32)
    np.testing.assert_array_equal(tiny.ctx.modswitch(x, q_from, q_to), oracle.modswitch(x, q_from, q_to))


@pytest.mark.parametrize("which", ["tiny", "paper"])
@pytest.mark.parametrize("count", [1, 5, 33])
def test_negacyclic_mul(request, which, count):
    case = request.getfixturevalue(which)
    say("negacyclic_mul", which, count)
    N = case.p.N
    rng = np.random.default_rng(count + N)
    a = rng.integers(0, Q, (count, N), dtype=np.uint32)
    b = rng.integers(0, Q, (count, N), dtype=np.uint32)
    got = case.ctx.negacyclic_mul(a, b)
    for c in range(count):
        np.testing.assert_array_equal(got[c], oracle.poly_mul(a[c], b[c], Q), err_msg=f"poly {c}")


def test_negacyclic_mul_edges(paper):
    N = paper.p.N
    a = np.zeros((4, N), np.uint32)
    b = np.zeros((4, N), np.uint32)
    a[0, 0] = 1
    b[0] = np.arange(N)
    a[1, N - 1] = 1  # x^(N-1) * x = -1
    b[1, 1] = 1
    a[2] = Q - 1
    b[2] = Q - 1
    a[3, 5] = 7
    b[3, N - 3] = Q - 2
    got = paper.ctx.negacyclic_mul(a, b)
    for c in range(4):
        np.testing.assert_array_equal(got[c], oracle.poly_mul(a[c], b[c], Q))


@pytest.mark.parametrize("which", ["tiny", "paper"])
def test_external_product(request, which):
    case = request.getfixturevalue(which)
    say("external_product", which)
    N = case.p.N
    rng = np.random.default_rng(3)
    count = 9
    rl = rng.integers(0, Q, (count, 2, N), dtype=np.uint32)
    rl[0] = 0
    rl[1] = Q - 1
    for i in (0, 1, case.p.n - 1):
        got = case.ctx.external_product(i, rl)
        for c in range(count):
            want = oracle.external_product(case.keys.bsk[i], rl[c], Q, case.p.log2_B, case.p.l)
            np.testing.assert_array_equal(got[c], want, err_msg=f"key {i} pair {c}")


def test_sample_extract(paper):
    N = paper.p.N
    rng = np.random.default_rng(4)
    rl = rng.integers(0, Q, (6, 2, N), dtype=np.uint32)
    got = paper.ctx.sample_extract(rl)
    for c in range(6):
        np.testing.assert_array_equal(got[c], oracle.sample_extract(rl[c], Q))


@pytest.mark.parametrize("count", [1, 3, 70])
def test_keyswitch(paper, count):
    say("keyswitch", count)
    rng = np.random.default_rng(count)
    lw = rng.integers(0, Q, (count, paper.p.N + 1), dtype=np.uint32)
    got = paper.ctx.keyswitch(lw)
    for c in range(count):
        np.testing.assert_array_equal(got[c], oracle.keyswitch(paper.p, paper.keys.ksk, lw[c]))


# ---------------------------------------------------------------- blind rotation

@pytest.mark.parametrize("steps", [0, 1, 2, 5, 64])
def test_blind_rotate_tiny_steps(tiny, steps):
    say("blind_rotate tiny steps", steps)
    tid, f, V = tiny.table(16, 16, 2, 5)
    q = 2 * tiny.p.N * 2
    m = messages(16, 4, 7)
    ct = tiny.encrypt(q, 16, m, 8)
    got = tiny.ctx.blind_rotate([tid] * 4, ct, steps).reshape(4, 2, 2, tiny.p.N)
    for c in range(4):
        want = oracle.blind_rotate(tiny.p, 2, tiny.keys.bsk, V, ct[c], steps)
        np.testing.assert_array_equal(got[c], want, err_msg=f"ct {c}")


@pytest.mark.parametrize("steps", [1, 3])
def test_blind_rotate_paper_mixed_r(paper, steps):
    """r = 1, 2, 4, 8 in one launch (components packed into shared workgroups)."""
    say("blind_rotate paper mixed steps", steps)
    ids, cts, Vs, rs = [], [], [], []
    for k, (t, r) in enumerate(CLASS_MIX):
        tid, f, V = paper.table(t, t, r, 20 + k)
        q = 2 * paper.p.N * r
        ct = paper.encrypt(q, t, messages(t, 2, 30 + k), 40 + k)
        for c in range(2):
            ids.append(tid)
            cts.append(ct[c])
            Vs.append(V)
            rs.append(r)
    got = paper.ctx.blind_rotate(ids, np.array(cts), steps)
    off = 0
    for c in range(len(ids)):
        r = rs[c]
        size = r * 2 * paper.p.N
        want = oracle.blind_rotate(paper.p, r, paper.keys.bsk, Vs[c], cts[c], steps)
        np.testing.assert_array_equal(got[off:off + size].reshape(r, 2, paper.p.N), want, err_msg=f"ct {c} r {r}")
        off += size


# ---------------------------------------------------------------- whole bootstrap

@pytest.mark.parametrize("plain", [False, True])
def test_bootstrap_tiny_all_messages(tiny, plain):
    say("bootstrap tiny plain", plain)
    tid, f, V = tiny.table(16, 16, 2, 6)
    q = 2 * tiny.p.N * 2
    m = np.arange(16, dtype=np.uint32)
    ct = tiny.encrypt(q, 16, m, 9)
    got = tiny.ctx.bootstrap([tid] * 16, ct, plain=plain)
    want = oracle.bootstrap_many(tiny.p, 2, tiny.keys.bsk, tiny.keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(oracle.decrypt(tiny.p.n, q, 16, tiny.keys.s, got), f[m])


def test_bootstrap_tiny_correct_many_seeds():
    """decrypt(bootstrap(Enc(m))) = f(m) for every m, fresh keys per seed (Definition 1)."""
    b = _gpu()
    pre = PRESETS["tiny"]
    p = pre["params"]
    for seed in range(100, 112):
        dr = key_draws(p, seed)
        ctx = b.Context(p, dr)
        f = negacyclic_table(16, 16, seed)
        tid = ctx.table_create(16, 16, 2, f)
        q = 2 * p.N * 2
        m = np.tile(np.arange(16, dtype=np.uint32), 4)
        ed = enc_draws(p.n, q, m.size, seed)
        ct = ctx.encrypt(q, 16, m, ed["a"], ed["e"])
        out = ctx.bootstrap([tid] * m.size, ct)
        np.testing.assert_array_equal(ctx.decrypt(q, 16, out), f[m], err_msg=f"seed {seed}")
        ctx.close()


@pytest.mark.parametrize("q_out", [0, Q, 4096])
def test_bootstrap_paper_single(paper, q_out):
    say("bootstrap paper single q_out", q_out)
    tid, f, V = paper.table(4096, 4096, 4, 7)
    q = 8192
    ct = paper.encrypt(q, 4096, messages(4096, 2, 10), 11)
    got_plain = paper.ctx.bootstrap([tid] * 2, ct, q_out=q_out, plain=True)
    got_batch = paper.ctx.bootstrap([tid] * 2, ct, q_out=q_out)
    np.testing.assert_array_equal(got_plain, got_batch)
    qo = q if q_out == 0 else q_out
    want = oracle.bootstrap_many(paper.p, 4, paper.keys.bsk, paper.keys.ksk, V, q, qo, ct)
    np.testing.assert_array_equal(got_plain, want)


def test_bootstrap_mixed_batch_equals_alone(paper):
    """Uneven (t, r) batch: every output equals the oracle and the same ciphertext run alone."""
    say("bootstrap mixed batch")
    tabs = []
    for k, (t, r) in enumerate(CLASS_MIX):
        tid, f, V = paper.table(t, t, r, 50 + k)
        tabs.append((tid, t, r, V))
    cls = class_mix(24, 3)
    ids, cts = [], []
    for c, k in enumerate(cls):
        tid, t, r, V = tabs[k]
        ids.append(tid)
        cts.append(paper.encrypt(2 * paper.p.N * r, t, messages(t, 1, 100 + c), 200 + c)[0])
    cts = np.array(cts)
    got = paper.ctx.bootstrap(ids, cts)
    alone = paper.ctx.bootstrap(ids, cts, plain=True)
    np.testing.assert_array_equal(got, alone)
    # the first ciphertext of every class, and every sixth
    picks = sorted({int(np.where(cls == k)[0][0]) for k in range(len(CLASS_MIX))} | set(range(0, len(ids), 6)))
    for c in picks:
        tid, t, r, V = tabs[cls[c]]
        q = 2 * paper.p.N * r
        want = oracle.bootstrap(paper.p, r, paper.keys.bsk, paper.keys.ksk, V, q, q, cts[c])
        np.testing.assert_array_equal(got[c], want, err_msg=f"ct {c} class {cls[c]}")


def test_bootstrap_noise_free_all_messages_decode_at_Q():
    """sigma = 0 keys and inputs: every m in Z_4096 decodes from the output at Q."""
    b = _gpu()
    p = PRESETS["paper_shaped"]["params"].noise_free()
    dr = key_draws(p, 77)
    ctx = b.Context(p, dr)
    f = negacyclic_table(4096, 4096, 77)
    tid = ctx.table_create(4096, 4096, 4, f)
    m = np.arange(4096, dtype=np.uint32)
    ed = enc_draws(p.n, 8192, 4096, 78, sigma=0.0)
    ct = ctx.encrypt(8192, 4096, m, ed["a"], ed["e"])
    out = ctx.bootstrap([tid] * 4096, ct, q_out=Q)
    np.testing.assert_array_equal(ctx.decrypt(Q, 4096, out), f[m])
    # a sample against the oracle at full batch size
    keys = oracle.KeySet(p, dr)
    V = oracle.test_vector(p.N, 4, Q, 4096, 4096, f)
    pick = np.array([0, 1, 2047, 4095])
    want = oracle.bootstrap_many(p, 4, keys.bsk, keys.ksk, V, 8192, Q, ct[pick])
    np.testing.assert_array_equal(out[pick], want)
    ctx.close()


def test_bootstrap_device_pointers(paper):
    import torch
    tid, f, V = paper.table(4096, 4096, 4, 8)
    ct = paper.encrypt(8192, 4096, messages(4096, 3, 12), 13)
    host = paper.ctx.bootstrap([tid] * 3, ct)
    dev_in = torch.from_numpy(ct.view(np.int32)).cuda()
    dev_out = paper.ctx.bootstrap([tid] * 3, dev_in)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dev_out.cpu().numpy().view(np.uint32), host)


def test_keyswitch_tiled_batch(paper):
    """Large batches take the LDS-tiled key switch."""
    say("keyswitch tiled 300")
    rng = np.random.default_rng(300)
    lw = rng.integers(0, Q, (300, paper.p.N + 1), dtype=np.uint32)
    got = paper.ctx.keyswitch(lw)
    for c in (0, 1, 150, 299):
        np.testing.assert_array_equal(got[c], oracle.keyswitch(paper.p, paper.keys.ksk, lw[c]))


def test_keyswitch_tiled_rows_not_multiple_of_4():
    """Key-switch base 2 with 31 digits (l_ks B_ks = 62 candidate rows per
    coordinate, not a multiple of 4, an odd digit count): both LDS-staged
    kernels stage every row and take every digit, at their default tilings
    (300 and 600 samples) and at every tiling a bootstrap batch of 300 may use
    (eq. equ-key-swi)."""
    p = Params(n=16, N=256, log2_B=8, l=3, log2_Bks=1, l_ks=31)
    c = Case(p, 31)
    rng = np.random.default_rng(31)
    for cnt in (300, 600):
        lw = rng.integers(0, Q, (cnt, p.N + 1), dtype=np.uint32)
        say("keyswitch base 2, 31 digits,", cnt, "samples")
        got = c.ctx.keyswitch(lw)
        for k in (0, 1, 150, 298, cnt - 1):
            np.testing.assert_array_equal(got[k], oracle.keyswitch(p, c.keys.ksk, lw[k]), err_msg=f"sample {k}")
    tid, f, V = c.table(16, 16, 2, 32)
    q = 2 * p.N * 2
    cts = c.encrypt(q, 16, messages(16, 300, 33), 34)
    ids = np.full(300, tid, np.int32)
    want = oracle.bootstrap_many(p, 2, c.keys.bsk, c.keys.ksk, V, q, q, cts)
    n = c.ctx.schedule_count(ids)
    kinds = {c.ctx.schedule_describe(ids, k)[4] for k in range(n)}
    assert kinds == {1, 2}, kinds  # both LDS-staged key switches among the candidates
    for choice in range(n):
        c.ctx.set_schedule(ids, choice)
        np.testing.assert_array_equal(c.ctx.bootstrap(ids, cts), want, err_msg=f"schedule {choice}")
    c.ctx.close()


def test_every_schedule_gives_the_same_bits(paper):
    """All candidate schedules (4- and 8-wave groups, key-switch tilings) agree bit for bit."""
    tabs = []
    for k, (t, r) in enumerate(CLASS_MIX[:3]):  # r <= 4 admits 4-wave groups
        tid, f, V = paper.table(t, t, r, 70 + k)
        tabs.append((tid, t, r, V))
    cls = class_mix(300, 9) % 3
    ids = np.array([tabs[k][0] for k in cls], np.int32)
    cts = np.array([paper.encrypt(2 * paper.p.N * tabs[k][2], tabs[k][1], messages(tabs[k][1], 1, 500 + c),
                                  600 + c)[0] for c, k in enumerate(cls)])
    n = paper.ctx.schedule_count(ids)
    say("schedules", n)
    assert n >= 4
    # 2-wave component slots are among the candidates (N = 1024, r <= 4), the
    # global-accumulator shape with 2 and 4 waves per component, and both LDS-staged
    # key switches
    assert {paper.ctx.schedule_describe(ids, k)[3] for k in range(n)} == {1, 2, 4}
    assert {paper.ctx.schedule_describe(ids, k)[0] for k in range(n)} == {0, 4, 8}
    assert {paper.ctx.schedule_describe(ids, k)[4] for k in range(n)} == {1, 2}
    # the three NTT stage schedules (LDS lockstep, lane swaps, staggered LDS) and the
    # global shape's two digit groups
    assert {paper.ctx.schedule_describe(ids, k)[5] for k in range(n)} == {0, 1, 2, 4}
    ref = None
    for choice in range(n):
        paper.ctx.set_schedule(ids, choice)
        out = paper.ctx.bootstrap(ids, cts)
        if ref is None:
            ref = out
        np.testing.assert_array_equal(out, ref, err_msg=f"schedule {choice}")
    for c in (0, 299):
        tid, t, r, V = tabs[cls[c]]
        q = 2 * paper.p.N * r
        np.testing.assert_array_equal(ref[c], oracle.bootstrap(paper.p, r, paper.keys.bsk, paper.keys.ksk, V, q, q,
                                                               cts[c]))
    choice = paper.ctx.autotune(ids, cts)
    assert 0 <= choice < n
    np.testing.assert_array_equal(paper.ctx.bootstrap(ids, cts), ref)


@pytest.mark.parametrize("identity,plain", [(False, False), (True, False), (False, True)])
def test_general_function_tiny(tiny, identity, plain):
    """An arbitrary f (or the identity) by two bootstraps: every m with both values of the top bit."""
    say("general f tiny identity", identity, "plain", plain)
    t, t_out, r = 8, 16, 2
    rng = np.random.default_rng(41)
    f = (np.arange(t) % t_out if identity else rng.integers(0, t_out, t)).astype(np.uint32)
    tid = tiny.ctx.table_create_general(t, t_out, r, f)
    g, F = oracle.general_tables(t, t_out, f)
    Vg = oracle.test_vector(tiny.p.N, r, Q, 2 * t, 2 * t, g)
    VF = oracle.test_vector(tiny.p.N, r, Q, 2 * t, t_out, F)
    q = 2 * tiny.p.N * r
    m = np.repeat(np.arange(t, dtype=np.uint32), 2)
    b = np.tile(np.array([0, 1], dtype=np.uint32), t)
    ct = tiny.encrypt(q, 2 * t, m + b * t, 77)
    got = tiny.ctx.bootstrap([tid] * m.size, ct, plain=plain)
    for c in range(m.size):
        want = oracle.bootstrap_general(tiny.p, r, tiny.keys.bsk, tiny.keys.ksk, Vg, VF, q, t, q, ct[c])
        np.testing.assert_array_equal(got[c], want, err_msg=f"ct {c}")
    np.testing.assert_array_equal(oracle.decrypt(tiny.p.n, q, t_out, tiny.keys.s, got), f[m])


def test_general_function_paper(paper):
    t, r = 2048, 4
    rng = np.random.default_rng(42)
    f = rng.integers(0, t, t).astype(np.uint32)
    tid = paper.ctx.table_create_general(t, t, r, f)
    g, F = oracle.general_tables(t, t, f)
    Vg = oracle.test_vector(paper.p.N, r, Q, 2 * t, 2 * t, g)
    VF = oracle.test_vector(paper.p.N, r, Q, 2 * t, t, F)
    q = 2 * paper.p.N * r
    ct = paper.encrypt(q, 2 * t, np.array([5, 2047 + 2048], np.uint32), 79)
    got = paper.ctx.bootstrap([tid] * 2, ct)
    for c in range(2):
        want = oracle.bootstrap_general(paper.p, r, paper.keys.bsk, paper.keys.ksk, Vg, VF, q, t, q, ct[c])
        np.testing.assert_array_equal(got[c], want)


# ---------------------------------------------------------------- ternary secret (Alg. 1 as printed)

@pytest.fixture(scope="module")
def tiny_ternary():
    from dataclasses import replace
    return Case(replace(PRESETS["tiny"]["params"], ternary=True), 13)


@pytest.mark.parametrize("plain", [False, True])
def test_ternary_tiny_all_messages(tiny_ternary, plain):
    case = tiny_ternary
    say("ternary tiny plain", plain)
    tid, f, V = case.table(16, 16, 2, 16)
    q = 2 * case.p.N * 2
    m = np.arange(16, dtype=np.uint32)
    ct = case.encrypt(q, 16, m, 17)
    got = case.ctx.bootstrap([tid] * 16, ct, plain=plain)
    want = oracle.bootstrap_many(case.p, 2, case.keys.bsk, case.keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(oracle.decrypt(case.p.n, q, 16, case.keys.s, got), f[m])


def test_ternary_every_schedule():
    """Ternary secret at the paper-shaped ring (N = 1024, n = 10, r = 4): every
    candidate schedule -- group widths, two-wave slots, the three NTT stage
    schedules, key-switch kernels -- gives the oracle's bits."""
    from dataclasses import replace
    case = Case(replace(PRESETS["paper_shaped"]["params"], n=10, ternary=True), 15)
    tid, f, V = case.table(4096, 4096, 4, 25)
    ct = case.encrypt(8192, 4096, messages(4096, 40, 26), 27)
    ids = np.full(40, tid, np.int32)
    want = oracle.bootstrap_many(case.p, 4, case.keys.bsk, case.keys.ksk, V, 8192, 8192, ct)
    n = case.ctx.schedule_count(ids)
    assert {case.ctx.schedule_describe(ids, k)[5] for k in range(n)} == {0, 1, 2, 4}
    for choice in range(n):
        case.ctx.set_schedule(ids, choice)
        np.testing.assert_array_equal(case.ctx.bootstrap(ids, ct), want, err_msg=f"schedule {choice}")
    case.ctx.close()


@pytest.mark.parametrize("steps", [1, 4])
def test_ternary_blind_rotate_steps(tiny_ternary, steps):
    case = tiny_ternary
    tid, f, V = case.table(16, 16, 2, 18)
    q = 2 * case.p.N * 2
    ct = case.encrypt(q, 16, messages(16, 3, 19), 20)
    got = case.ctx.blind_rotate([tid] * 3, ct, steps).reshape(3, 2, 2, case.p.N)
    for c in range(3):
        np.testing.assert_array_equal(got[c], oracle.blind_rotate(case.p, 2, case.keys.bsk, V, ct[c], steps))


def test_ternary_external_product_second_key(tiny_ternary):
    case = tiny_ternary
    rng = np.random.default_rng(21)
    rl = rng.integers(0, Q, (3, 2, case.p.N), dtype=np.uint32)
    for idx in (0, 1, 2 * case.p.n - 1):
        got = case.ctx.external_product(idx, rl)
        for c in range(3):
            want = oracle.external_product(case.keys.bsk[idx], rl[c], Q, case.p.log2_B, case.p.l)
            np.testing.assert_array_equal(got[c], want)


def test_ternary_paper_shaped_single():
    from dataclasses import replace
    say("ternary paper single")
    case = Case(replace(PRESETS["paper_shaped"]["params"], ternary=True), 14)
    tid, f, V = case.table(4096, 4096, 4, 22)
    ct = case.encrypt(8192, 4096, messages(4096, 2, 23), 24)
    got = case.ctx.bootstrap([tid] * 2, ct)
    want = oracle.bootstrap_many(case.p, 4, case.keys.bsk, case.keys.ksk, V, 8192, 8192, ct)
    np.testing.assert_array_equal(got, want)
    case.ctx.close()


@pytest.fixture(scope="module")
def bench_keys():
    """The key set of the benchmark (paper-shaped parameters, key seed 1)."""
    b = _gpu()
    p = PRESETS["paper_shaped"]["params"]
    dr = key_draws(p, 1)
    ctx = b.Context(p, dr)
    ctx.device_init(0)
    yield ctx, oracle.KeySet(p, dr), p
    ctx.close()


def test_full_batch_bench_configuration_sampled(bench_keys):
    """The timed workload itself: 4096 paper-shaped ciphertexts (sigma = 3.2, the bench
    seeds), autotuned schedule, one batched launch; 64 outputs spread over the batch
    equal the oracle's."""
    ctx, keys, p = bench_keys
    f = negacyclic_table(4096, 4096, 2)
    tid = ctx.table_create(4096, 4096, 4, f)
    m = messages(4096, 4096, 3)
    ed = enc_draws(p.n, 8192, 4096, 4)
    ct = ctx.encrypt(8192, 4096, m, ed["a"], ed["e"])
    ids = np.full(4096, tid, np.int32)
    say("bench configuration: autotune + batch of 4096")
    np.testing.assert_array_equal(ct, oracle.encrypt(p.n, 8192, 4096, keys.s, m, ed["a"], ed["e"]))
    ctx.autotune(ids, ct)
    out = ctx.bootstrap(ids, ct)
    V = oracle.test_vector(p.N, 4, Q, 4096, 4096, f)
    pick = np.unique(np.concatenate([[0, 1, 2, 1023, 2048, 3071, 4094, 4095], np.linspace(0, 4095, 60).astype(int)]))
    say("oracle on", pick.size, "samples")
    want = oracle.bootstrap_many(p, 4, keys.bsk, keys.ksk, V, 8192, 8192, ct[pick])
    np.testing.assert_array_equal(out[pick], want)


def test_mixed_bench_configuration_sampled_per_class(bench_keys):
    """The uneven batch the benchmark times: 2048 paper-shaped ciphertexts, class
    (t, r) drawn uniformly from {(2^8,1), (2^10,2), (2^12,4), (2^14,8)} with the
    bench's seeds, autotuned schedule, one launch; 16 outputs of every class equal
    the oracle's."""
    ctx, keys, p = bench_keys
    M = 2048
    cls = class_mix(M, 8)
    cts = np.empty((M, p.n + 1), np.uint32)
    tabs = []
    for k, (t, r) in enumerate(CLASS_MIX):
        f = negacyclic_table(t, t, 100 + k)
        tabs.append((ctx.table_create(t, t, r, f), t, r, oracle.test_vector(p.N, r, Q, t, t, f)))
        sel = np.where(cls == k)[0]
        q = 2 * p.N * r
        ed = enc_draws(p.n, q, sel.size, 400 + k)
        mk = messages(t, sel.size, 500 + k)
        cts[sel] = oracle.encrypt(p.n, q, t, keys.s, mk, ed["a"], ed["e"])
        np.testing.assert_array_equal(ctx.encrypt(q, t, mk, ed["a"], ed["e"]), cts[sel])
    ids = np.array([tabs[k][0] for k in cls], np.int32)
    say("uneven batch of", M, "autotuned")
    ctx.autotune(ids, cts)
    out = ctx.bootstrap(ids, cts)
    for k, (tid, t, r, V) in enumerate(tabs):
        sel = np.where(cls == k)[0]
        pick = sel[np.linspace(0, sel.size - 1, 16).astype(int)]
        q = 2 * p.N * r
        say("oracle on 16 of class", (t, r))
        want = oracle.bootstrap_many(p, r, keys.bsk, keys.ksk, V, q, q, cts[pick])
        np.testing.assert_array_equal(out[pick], want, err_msg=f"class {(t, r)}")


def test_batch_three_times_the_bench_sampled(paper):
    """12,288 paper-shaped ciphertexts in one launch (49,152 components: 24 groups per
    persistent workgroup, workspaces three times the timed batch's); the first 4096
    equal the same ciphertexts bootstrapped as a batch of their own, and sampled
    outputs across the whole batch equal the oracle's."""
    B = 3 * 4096
    tid, f, V = paper.table(4096, 4096, 4, 41)
    ct = paper.encrypt(8192, 4096, messages(4096, B, 42), 43)
    say("batch of", B)
    out = paper.ctx.bootstrap([tid] * B, ct)
    np.testing.assert_array_equal(paper.ctx.bootstrap([tid] * 4096, ct[:4096]), out[:4096])
    pick = np.array([0, 4095, 4096, 8191, 8192, B - 1])
    say("oracle on", pick.size, "samples")
    want = oracle.bootstrap_many(paper.p, 4, paper.keys.bsk, paper.keys.ksk, V, 8192, 8192, ct[pick])
    np.testing.assert_array_equal(out[pick], want)


def test_empty_and_ragged_batches(paper):
    """count = 0 is a no-op; ragged batch sizes give the same bits as one larger batch."""
    tid, f, V = paper.table(4096, 4096, 4, 15)
    ct = paper.encrypt(8192, 4096, messages(4096, 131, 16), 17)
    empty = paper.ctx.bootstrap(np.zeros(0, np.int32), ct[:0])
    assert empty.shape == (0, paper.p.n + 1)
    full = paper.ctx.bootstrap([tid] * 131, ct)
    for cnt in (1, 3, 64, 129):
        np.testing.assert_array_equal(paper.ctx.bootstrap([tid] * cnt, ct[:cnt]), full[:cnt], err_msg=f"count {cnt}")
    np.testing.assert_array_equal(full[130], oracle.bootstrap(paper.p, 4, paper.keys.bsk, paper.keys.ksk, V, 8192,
                                                              8192, ct[130]))


@pytest.mark.parametrize("N,ternary", [(1024, False), (1024, True), (512, False), (512, True)])
def test_two_wave_slots_small_batches(N, ternary):
    """Batches too small to fill the device: their default at N = 1024 is the
    global-accumulator shape (a compute unit per component), and the fused kernel's schedule with each
    component on two waves (N = 512, 1024, r <= 4) is among the candidates; blind
    rotation and bootstrap against the oracle, and every schedule gives the same bits.
    r = 8 does not fit two-wave slots: its fused schedules run one wave per component."""
    from dataclasses import replace
    say("two-wave slots N", N, "ternary", ternary)
    p = replace(Params(n=12, N=N, log2_B=7, l=4), ternary=ternary)
    c = Case(p, 1500 + N + ternary)
    tid, f, V = c.table(2 * N, 2 * N, 4, 31)  # r = 4, t = 2N
    tid8, f8, V8 = c.table(64, 64, 8, 32)     # r = 8 does not fit 2-wave slots
    q = 2 * N * 4
    ct = c.encrypt(q, 2 * N, messages(2 * N, 3, 33), 34)
    ids = np.full(3, tid, np.int32)
    ids8 = np.full(3, tid8, np.int32)
    if N == 1024:  # the default there: the global-accumulator shape, four waves per component
        assert c.ctx.schedule_describe(ids)[0] == 0 and c.ctx.schedule_describe(ids8)[0] == 0
    else:  # N = 512: the fused kernel, two-wave slots for r = 4
        assert c.ctx.schedule_describe(ids)[:1] == (8,) and c.ctx.schedule_describe(ids)[3] == 2
    desc = [c.ctx.schedule_describe(ids, k) for k in range(c.ctx.schedule_count(ids))]
    assert any(d[0] == 8 and d[3] == 2 for d in desc)  # two-wave slots
    desc8 = [c.ctx.schedule_describe(ids8, k) for k in range(c.ctx.schedule_count(ids8))]
    assert all(d[3] == 1 for d in desc8 if d[0] != 0)
    acc = c.ctx.blind_rotate(ids, ct, 5)
    for j in range(3):
        np.testing.assert_array_equal(acc[j * 4 * 2 * N:(j + 1) * 4 * 2 * N].reshape(4, 2, N),
                                      oracle.blind_rotate(p, 4, c.keys.bsk, V, ct[j], 5))
    out = c.ctx.bootstrap(ids, ct)
    np.testing.assert_array_equal(out, oracle.bootstrap_many(p, 4, c.keys.bsk, c.keys.ksk, V, q, q, ct))
    np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct, plain=True), out)
    n = c.ctx.schedule_count(ids)
    for k in range(n):
        c.ctx.set_schedule(ids, k)
        np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct), out, err_msg=f"schedule {k}")
    q8 = 2 * N * 8
    ct8 = c.encrypt(q8, 64, messages(64, 2, 35), 36)
    want8 = oracle.bootstrap_many(p, 8, c.keys.bsk, c.keys.ksk, V8, q8, q8, ct8)
    ids8 = np.full(2, tid8, np.int32)
    for k in range(c.ctx.schedule_count(ids8)):
        c.ctx.set_schedule(ids8, k)
        np.testing.assert_array_equal(c.ctx.bootstrap(ids8, ct8), want8, err_msg=f"r = 8, schedule {k}")
    c.ctx.close()


@pytest.mark.parametrize("l,log2_B,ternary", [(4, 7, False), (3, 10, False), (3, 10, True), (5, 6, True),
                                               (1, 15, False)])
def test_two_digit_groups(l, log2_B, ternary):
    """NTT schedule 4 of the global-accumulator shape at N = 1024: two groups of four
    waves per component, each taking every other gadget digit (odd l: the second
    group transforms zeros on its last pass) and one part's inverse NTT.  One
    ciphertext, a batch of mixed r and a batch spanning every compute unit several
    times against the oracle."""
    from dataclasses import replace
    say("two digit groups l", l, "log2_B", log2_B, "ternary", ternary)
    p = replace(Params(n=12, N=1024, log2_B=log2_B, l=l), ternary=ternary)
    c = Case(p, 1700 + 10 * l + ternary)
    tid, f, V = c.table(2048, 2048, 4, 41)
    tid8, f8, V8 = c.table(64, 64, 8, 42)
    for cnt, mixed in ((1, False), (7, True), (700, False)):
        say("  count", cnt, "mixed", mixed)
        r_of = [8 if mixed and j % 3 == 1 else 4 for j in range(cnt)]
        ids = np.array([tid8 if r == 8 else tid for r in r_of], np.int32)
        ct = np.array([c.encrypt(2 * 1024 * r, 64 if r == 8 else 2048,
                                 messages(64 if r == 8 else 2048, 1, 43 + j), 44 + j)[0] for j, r in enumerate(r_of)])
        n = c.ctx.schedule_count(ids)
        dg = [k for k in range(n) if c.ctx.schedule_describe(ids, k)[5] == 4]
        assert dg and all(c.ctx.schedule_describe(ids, k)[:1] == (0,) and c.ctx.schedule_describe(ids, k)[3] == 4
                          for k in dg)
        c.ctx.set_schedule(ids, dg[0])
        out = c.ctx.bootstrap(ids, ct)
        picks = range(cnt) if cnt < 10 else (0, 1, cnt // 2, cnt - 1)
        for j in picks:
            r = r_of[j]
            q = 2 * 1024 * r
            np.testing.assert_array_equal(out[j], oracle.bootstrap(p, r, c.keys.bsk, c.keys.ksk, V8 if r == 8 else V,
                                                                   q, q, ct[j]), err_msg=f"ciphertext {j}")
        if cnt >= 10:
            c.ctx.set_schedule(ids, [k for k in range(n) if c.ctx.schedule_describe(ids, k)[5] != 4][0])
            np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct), out)
    c.ctx.close()


@pytest.mark.parametrize("q_in", [2 ** 31, 12289, 196611])
@pytest.mark.parametrize("plain", [False, True])
def test_bootstrap_first_switch_not_identity(tiny, q_in, plain):
    """Ciphertexts at a modulus q_in other than 2Nr: the first modulus switch of
    Alg. 1 (round(a 2Nr / q_in), ties upward) runs inside the blind rotation."""
    say("q_in", q_in, "plain", plain)
    t, r = 16, 2
    tid, f, V = tiny.table(t, t, r, 140, q_in=q_in)
    m = np.arange(t, dtype=np.uint32)
    ct = tiny.encrypt(q_in, t, m, 141)
    got = tiny.ctx.bootstrap([tid] * t, ct, plain=plain)
    want = oracle.bootstrap_many(tiny.p, r, tiny.keys.bsk, tiny.keys.ksk, V, q_in, q_in, ct)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(oracle.decrypt(tiny.p.n, q_in, t, tiny.keys.s, got), f[m])


def test_two_entry_table(tiny):
    """t = 2, the smallest nega-cyclic table (f(1) = -f(0) mod t')."""
    t, t_out, r = 2, 16, 2
    tid, f, V = tiny.table(t, t_out, r, 142)
    q = 2 * tiny.p.N * r
    m = np.array([0, 1, 1, 0], dtype=np.uint32)
    ct = tiny.encrypt(q, t, m, 143)
    got = tiny.ctx.bootstrap([tid] * 4, ct)
    np.testing.assert_array_equal(got, oracle.bootstrap_many(tiny.p, r, tiny.keys.bsk, tiny.keys.ksk, V, q, q, ct))
