"""GPU parity at ring degrees above 1024, where one polynomial spans several
waves (N / 1024 of them) and the NTT relayouts synchronise the workgroup, and
on the global-accumulator path (components beyond one workgroup, N = 16384).

N = 2048, 4096, 8192 with r = 1 is the TFHE-shaped comparison point of
Sec. 5 (one ring of degree N r instead of r components of degree N); MMPM
tables with r > 1 at N = 2048 and 4096 run through the same kernels.  Every
comparison is bit-exact against the oracle on the same draws.
"""
import numpy as np
import pytest

import oracle
from synth import PRESETS, Params, enc_draws, key_draws, messages, negacyclic_table

pytestmark = pytest.mark.gpu
Q = 2147352577


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_12441_amd import binding
    return binding


def say(*a):
    print(*a, flush=True)


class Case:
    def __init__(self, p, seed):
        b = _gpu()
        self.p = p
        self.draws = key_draws(p, seed)
        self.ctx = b.Context(p, self.draws)
        self.keys = oracle.KeySet(p, self.draws)
        self.ctx.device_init(0)

    def table(self, t, t_out, r, seed):
        f = negacyclic_table(t, t_out, seed)
        tid = self.ctx.table_create(t, t_out, r, f)
        return tid, f, oracle.test_vector(self.p.N, r, Q, t, t_out, f)

    def encrypt(self, q, t, m, seed, sigma=3.2):
        ed = enc_draws(self.p.n, q, len(m), seed, sigma)
        return oracle.encrypt(self.p.n, q, t, self.keys.s, m, ed["a"], ed["e"])


_cases = {}


def case(N, n=16):
    key = (N, n)
    if key not in _cases:
        say("keygen N", N, "n", n)
        _cases[key] = Case(Params(n=n, N=N, log2_B=7, l=4), 900 + N + n)
    return _cases[key]


@pytest.mark.parametrize("N", [2048, 4096, 8192])
@pytest.mark.parametrize("count", [1, 3])
def test_negacyclic_mul_large(N, count):
    say("negacyclic_mul N", N, "count", count)
    c = case(N)
    rng = np.random.default_rng(N + count)
    a = rng.integers(0, Q, (count, N), dtype=np.uint32)
    b = rng.integers(0, Q, (count, N), dtype=np.uint32)
    a[0, :3] = [0, 1, Q - 1]
    got = c.ctx.negacyclic_mul(a, b)
    for k in range(count):
        np.testing.assert_array_equal(got[k], oracle.poly_mul(a[k], b[k], Q), err_msg=f"poly {k}")


def test_negacyclic_mul_monomials_8192():
    """x^(N-1) x = -1 and x^i x^j = x^(i+j) across the wave boundaries of one polynomial."""
    c = case(8192)
    N = 8192
    a = np.zeros((3, N), np.uint32)
    b = np.zeros((3, N), np.uint32)
    a[0, N - 1] = 1
    b[0, 1] = 1
    a[1, 1023] = 5
    b[1, 1025] = 3
    a[2, 4095] = Q - 1
    b[2, 6000] = 2
    got = c.ctx.negacyclic_mul(a, b)
    for k in range(3):
        np.testing.assert_array_equal(got[k], oracle.poly_mul(a[k], b[k], Q))
    assert got[0, 0] == Q - 1 and np.count_nonzero(got[0]) == 1
    assert got[1, 2048] == 15 and np.count_nonzero(got[1]) == 1


@pytest.mark.parametrize("N", [2048, 4096, 8192])
def test_external_product_large(N):
    say("external_product N", N)
    c = case(N)
    rng = np.random.default_rng(7 + N)
    count = 3
    rl = rng.integers(0, Q, (count, 2, N), dtype=np.uint32)
    rl[0] = Q - 1
    for i in (0, c.p.n - 1):
        got = c.ctx.external_product(i, rl)
        for k in range(count):
            want = oracle.external_product(c.keys.bsk[i], rl[k], Q, c.p.log2_B, c.p.l)
            np.testing.assert_array_equal(got[k], want, err_msg=f"key {i} pair {k}")


@pytest.mark.parametrize("N,rs,steps", [(2048, (1, 2, 4), 3), (4096, (1, 2), 3), (8192, (1,), 2)])
def test_blind_rotate_large_steps(N, rs, steps):
    """Mixed r in one launch at N > 1024 (component slots of N / 1024 waves)."""
    say("blind_rotate N", N, "rs", rs, "steps", steps)
    c = case(N)
    ids, cts, Vs, rr = [], [], [], []
    for k, r in enumerate(rs):
        t = 2 * N * r // 4  # Delta = 4
        tid, f, V = c.table(t, t, r, 30 + k)
        ct = c.encrypt(2 * N * r, t, messages(t, 2, 40 + k), 50 + k)
        for j in range(2):
            ids.append(tid)
            cts.append(ct[j])
            Vs.append(V)
            rr.append(r)
    got = c.ctx.blind_rotate(ids, np.array(cts), steps)
    off = 0
    for j in range(len(ids)):
        r = rr[j]
        size = r * 2 * N
        want = oracle.blind_rotate(c.p, r, c.keys.bsk, Vs[j], cts[j], steps)
        np.testing.assert_array_equal(got[off:off + size].reshape(r, 2, N), want, err_msg=f"ct {j} r {r}")
        off += size


@pytest.mark.parametrize("plain", [False, True])
def test_bootstrap_tfhe_shaped_small(plain):
    """r = 1 at N = 2048, t = 16: every message, against the oracle, and decrypts to f(m)."""
    say("bootstrap N=2048 r=1 plain", plain)
    c = case(2048, n=24)
    tid, f, V = c.table(16, 16, 1, 61)
    q = 2 * 2048
    m = np.arange(16, dtype=np.uint32)
    ct = c.encrypt(q, 16, m, 62)
    got = c.ctx.bootstrap([tid] * 16, ct, plain=plain)
    want = oracle.bootstrap_many(c.p, 1, c.keys.bsk, c.keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(oracle.decrypt(c.p.n, q, 16, c.keys.s, got), f[m])


@pytest.mark.parametrize("plain", [False, True])
def test_bootstrap_8192_end_to_end(plain):
    """r = 1 at N = 8192 (one polynomial over 8 waves), t = 2^14: the whole
    bootstrap -- n CMux steps, extraction of an 8193-word sample, its key switch
    over 65,536 key rows and the final switch -- against the oracle."""
    say("bootstrap N=8192 r=1 n=12 plain", plain)
    c = case(8192, n=12)
    t = 16384
    tid, f, V = c.table(t, t, 1, 63)
    q = 2 * 8192
    ct = c.encrypt(q, t, messages(t, 3, 64), 65)
    got = c.ctx.bootstrap([tid] * 3, ct, plain=plain)
    want = oracle.bootstrap_many(c.p, 1, c.keys.bsk, c.keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(got, want)
    # the same at Q, before the last modulus switch
    np.testing.assert_array_equal(c.ctx.bootstrap([tid] * 3, ct, q_out=Q, plain=plain),
                                  oracle.bootstrap_many(c.p, 1, c.keys.bsk, c.keys.ksk, V, q, Q, ct))


def test_bootstrap_tfhe_shaped_8192_bench_batch_sampled():
    """The TFHE-shaped comparison point for t = 2^14 exactly as the benchmark times
    it: n = 630, N = 8192, r = 1, its key, table and encryption seeds, a batch of
    4096 in one autotuned launch; sampled outputs equal the oracle's, stored by
    tests/golden/make_oracle_expected.py (the oracle takes minutes per ciphertext
    at this size)."""
    import importlib.util
    import os
    b = _gpu()
    spec_path = os.path.join(os.path.dirname(__file__), "golden", "make_oracle_expected.py")
    sp = importlib.util.spec_from_file_location("make_oracle_expected", spec_path)
    gold = importlib.util.module_from_spec(sp)
    sp.loader.exec_module(gold)
    spec = gold.SETS["tfhe_shaped_8192"]
    expected = gold.load("tfhe_shaped_8192")
    p, t, r = spec["params"], spec["t"], spec["r"]
    say("tfhe-shaped 8192 keygen (n = 630)")
    dr = key_draws(p, spec["key_seed"])
    ctx = b.Context(p, dr)
    ctx.device_init(0)
    tid = ctx.table_create(t, t, r, negacyclic_table(t, t, spec["table_seed"]))
    q, m, ct = gold.inputs(spec, dr["s"])
    ed = enc_draws(p.n, q, spec["batch"], spec["enc_seed"])
    np.testing.assert_array_equal(ctx.encrypt(q, t, m, ed["a"], ed["e"]), ct)
    ids = np.full(spec["batch"], tid, np.int32)
    say("autotune + batch of", spec["batch"])
    ctx.autotune(ids, ct)
    out = ctx.bootstrap(ids, ct)
    assert sorted(expected) == sorted(spec["pick"])
    for i, want in expected.items():
        np.testing.assert_array_equal(out[i], want, err_msg=f"ciphertext {i}")
    ctx.close()


def test_bootstrap_mmpm_r2_at_4096_and_schedules():
    """r = 2 at N = 4096 (one 8-wave group per ciphertext); every schedule gives the same bits."""
    c = case(4096, n=12)
    tid, f, V = c.table(4096, 4096, 2, 71)
    q = 2 * 4096 * 2
    ct = c.encrypt(q, 4096, messages(4096, 5, 72), 73)
    ids = np.full(5, tid, np.int32)
    n = c.ctx.schedule_count(ids)
    say("N=4096 r=2 schedules", n)
    ref = None
    for choice in range(n):
        c.ctx.set_schedule(ids, choice)
        out = c.ctx.bootstrap(ids, ct)
        if ref is None:
            ref = out
        np.testing.assert_array_equal(out, ref, err_msg=f"schedule {choice}")
    want = oracle.bootstrap_many(c.p, 2, c.keys.bsk, c.keys.ksk, V, q, q, ct[:2])
    np.testing.assert_array_equal(ref[:2], want)


def test_r_too_wide_for_a_workgroup_runs_the_global_path():
    """r = 4 at N = 4096 needs 16 waves, more than one fused workgroup holds: the
    batch (with an r = 1 ciphertext beside it) runs the global-accumulator path,
    accumulators in device memory and one launch per CMux step, bit-exact."""
    b = _gpu()
    c = case(4096, n=6)
    tid, f, V = c.table(64, 64, 4, 81)
    tid1, f1, V1 = c.table(64, 64, 1, 84)
    ct = c.encrypt(2 * 4096 * 4, 64, messages(64, 2, 82), 83)
    ct1 = c.encrypt(2 * 4096, 64, messages(64, 1, 85), 86)
    cts = np.concatenate([ct, ct1])
    ids = [tid, tid, tid1]
    say("global path N=4096 r=4 + r=1: 3 steps")
    got = c.ctx.blind_rotate(ids, cts, 3)
    size4 = 4 * 2 * 4096
    for j in range(2):
        np.testing.assert_array_equal(got[j * size4:(j + 1) * size4].reshape(4, 2, 4096),
                                      oracle.blind_rotate(c.p, 4, c.keys.bsk, V, ct[j], 3), err_msg=f"ct {j}")
    np.testing.assert_array_equal(got[2 * size4:].reshape(1, 2, 4096),
                                  oracle.blind_rotate(c.p, 1, c.keys.bsk, V1, ct1[0], 3))
    out = c.ctx.bootstrap(ids, cts)
    np.testing.assert_array_equal(c.ctx.bootstrap(ids, cts, plain=True), out)
    q = 2 * 4096 * 4
    np.testing.assert_array_equal(out[:2], oracle.bootstrap_many(c.p, 4, c.keys.bsk, c.keys.ksk, V, q, q, ct))
    np.testing.assert_array_equal(out[2:], oracle.bootstrap_many(c.p, 1, c.keys.bsk, c.keys.ksk, V1, 2 * 4096,
                                                                 2 * 4096, ct1))
    n = c.ctx.schedule_count(ids)  # one blind-rotation shape: key-switch candidates only
    assert all(c.ctx.schedule_describe(ids, k)[0] == 0 for k in range(n))
    for k in range(n):
        c.ctx.set_schedule(ids, k)
        np.testing.assert_array_equal(c.ctx.bootstrap(ids, cts), out, err_msg=f"schedule {k}")


@pytest.mark.parametrize("ternary,r", [(False, 16), (True, 12)])
def test_mmpm_more_components_than_a_workgroup(ternary, r):
    """MMPM with r = 16 at N = 1024 (the t = 2^15 class: 2Nr = t) and, ternary,
    r = 12: more components than the 8 slots of a fused workgroup, through the
    global-accumulator path; whole bootstraps against the oracle."""
    from dataclasses import replace
    p = replace(Params(n=8, N=1024, log2_B=7, l=4), ternary=ternary)
    c = Case(p, 970 + r)
    t = 2 * 1024 * r if not ternary else 1024 * r // 2  # 2Nr / t = 1 or 4
    tid, f, V = c.table(t, t, r, 99)
    q = 2 * 1024 * r
    ct = c.encrypt(q, t, messages(t, 3, 100), 101)
    say("global path N=1024 r", r, "ternary", ternary)
    got = c.ctx.bootstrap([tid] * 3, ct)
    np.testing.assert_array_equal(got, oracle.bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct))
    got2 = c.ctx.blind_rotate([tid], ct[:1], 2)
    np.testing.assert_array_equal(got2.reshape(r, 2, 1024), oracle.blind_rotate(c.p, r, c.keys.bsk, V, ct[0], 2))
    c.ctx.close()


@pytest.mark.parametrize("plain", [False, True])
def test_bootstrap_16384(plain):
    """N = 16384, r = 1, t = 2^15 (the TFHE-shaped point for t = 2^15): one
    polynomial over 16 waves on the global-accumulator path; the accumulator
    after 2 steps and whole bootstraps (at q and at Q) against the oracle."""
    b = _gpu()
    c = case(16384, n=4)
    t = 32768
    tid, f, V = c.table(t, t, 1, 111)
    q = 2 * 16384
    ct = c.encrypt(q, t, messages(t, 2, 112), 113)
    say("N=16384 plain", plain)
    if not plain:
        got = c.ctx.blind_rotate([tid] * 2, ct, 2)
        for j in range(2):
            np.testing.assert_array_equal(got[j * 2 * 16384:(j + 1) * 2 * 16384].reshape(1, 2, 16384),
                                          oracle.blind_rotate(c.p, 1, c.keys.bsk, V, ct[j], 2), err_msg=f"ct {j}")
    out = c.ctx.bootstrap([tid] * 2, ct, plain=plain)
    np.testing.assert_array_equal(out, oracle.bootstrap_many(c.p, 1, c.keys.bsk, c.keys.ksk, V, q, q, ct))
    if not plain:
        # both blind-rotation shapes of this ring (one 16-wave workgroup per component,
        # or two sub-rings of 8192) with every key switch give the same bits
        ids = np.full(2, tid, np.int32)
        n = c.ctx.schedule_count(ids)
        shapes = {c.ctx.schedule_describe(ids, k)[5] for k in range(n)}
        assert shapes == {0, 3}
        for k in range(n):
            c.ctx.set_schedule(ids, k)
            np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct), out, err_msg=f"schedule {k}")
            np.testing.assert_array_equal(c.ctx.blind_rotate(ids, ct, 2), got, err_msg=f"schedule {k}")
        c.ctx.autotune(ids, ct)
        np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct), out)
        # served on the global-accumulator path (chunk 3 does not divide n = 4)
        srv = c.ctx.server_start(64 << 20, chunk_steps=3)
        try:
            got, lat = srv.replay(np.full(2, tid, np.int32), ct, np.array([0, 1000000], np.int64))
        finally:
            srv.stop()
        np.testing.assert_array_equal(got, out)
    np.testing.assert_array_equal(c.ctx.bootstrap([tid] * 2, ct, q_out=Q, plain=plain),
                                  oracle.bootstrap_many(c.p, 1, c.keys.bsk, c.keys.ksk, V, q, Q, ct))


@pytest.mark.parametrize("N,r,ternary", [(32768, 1, False), (65536, 1, False), (32768, 2, True)])
def test_split_ring(N, r, ternary):
    """Rings of 32768 and 65536 coefficients (the TFHE-shaped points t = 2^16 and 2^17)
    split into sub-rings of 8192: the stages that mix sub-rings run column by column
    through device memory, each sub-ring's NTT, product and inverse in one workgroup.
    The accumulator after 2 CMux steps and whole bootstraps (at q and at Q) against
    the oracle; r = 2 with a ternary secret covers the rotation between components and
    both CMux terms."""
    from dataclasses import replace
    c = case(N, n=3) if not ternary else None
    if ternary:
        key = (N, 3, "ternary")
        if key not in _cases:
            say("keygen N", N, "ternary")
            _cases[key] = Case(replace(Params(n=3, N=N, log2_B=7, l=4), ternary=True), 950 + N)
        c = _cases[key]
    t = 2 * N * r // 4
    tid, f, V = c.table(t, t, r, 131)
    q = 2 * N * r
    ct = c.encrypt(q, t, messages(t, 2, 132), 133)
    ids = np.full(2, tid, np.int32)
    assert c.ctx.schedule_describe(ids)[5] == 3  # the split ring
    say("split ring N", N, "r", r, "ternary", ternary)
    got = c.ctx.blind_rotate(ids, ct, 2)
    size = r * 2 * N
    for j in range(2):
        np.testing.assert_array_equal(got[j * size:(j + 1) * size].reshape(r, 2, N),
                                      oracle.blind_rotate(c.p, r, c.keys.bsk, V, ct[j], 2), err_msg=f"ct {j}")
    out = c.ctx.bootstrap(ids, ct)
    np.testing.assert_array_equal(out, oracle.bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct))
    np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct, plain=True), out)
    np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct, q_out=Q),
                                  oracle.bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, Q, ct))
    c.ctx.close()
    _cases.pop(next(k for k, v in _cases.items() if v is c))


def test_serving_at_2048_matches_alone():
    c = case(2048)
    tid, f, V = c.table(1024, 1024, 2, 91)
    q = 2 * 2048 * 2
    ct = c.encrypt(q, 1024, messages(1024, 6, 92), 93)
    wide = c.table(64, 64, 8, 94)[0]  # r = 8 at N = 2048 needs 16 waves
    alone = c.ctx.bootstrap([tid] * 6, ct)
    srv = c.ctx.server_start(64 << 20, chunk_steps=5)
    try:
        out, lat = srv.replay(np.full(6, tid, np.int32), ct, np.arange(6, dtype=np.int64) * 200000)
        with pytest.raises(Exception):
            srv.submit(wide, ct[0])
    finally:
        srv.stop()
    np.testing.assert_array_equal(out, alone)


@pytest.mark.parametrize("N,r", [(2048, 2), (4096, 1)])
def test_ternary_at_large_ring(N, r):
    """Ternary secret (two keys, both CMux terms per step) with polynomials spanning several waves."""
    from dataclasses import replace
    say("ternary N", N, "r", r)
    p = replace(Params(n=10, N=N, log2_B=7, l=4), ternary=True)
    c = Case(p, 950 + N)
    t = 2 * N * r // 8
    tid, f, V = c.table(t, t, r, 96)
    q = 2 * N * r
    ct = c.encrypt(q, t, messages(t, 3, 97), 98)
    got = c.ctx.blind_rotate([tid] * 3, ct, 4)
    size = r * 2 * N
    for j in range(3):
        want = oracle.blind_rotate(c.p, r, c.keys.bsk, V, ct[j], 4)
        np.testing.assert_array_equal(got[j * size:(j + 1) * size].reshape(r, 2, N), want, err_msg=f"ct {j}")
    out = c.ctx.bootstrap([tid] * 3, ct)
    np.testing.assert_array_equal(out, oracle.bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct))
    c.ctx.close()


@pytest.fixture(scope="module")
def tfhe_paper():
    pre = PRESETS["tfhe_shaped"]
    return Case(pre["params"], 13), pre


def test_bootstrap_tfhe_paper_shaped(tfhe_paper):
    """n = 630, N = 4096, r = 1, t = 2^12: the TFHE counterpart of the paper-shaped MMPM workload."""
    c, pre = tfhe_paper
    t, r = pre["t"], pre["r"]
    tid, f, V = c.table(t, t, r, 7)
    q = 2 * c.p.N * r
    ct = c.encrypt(q, t, messages(t, 2, 10), 11)
    say("bootstrap tfhe-shaped batched + plain")
    got = c.ctx.bootstrap([tid] * 2, ct)
    np.testing.assert_array_equal(c.ctx.bootstrap([tid] * 2, ct, plain=True), got)
    say("oracle")
    want = oracle.bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(got, want)


def test_bootstrap_tfhe_noise_free_all_messages_decode_at_Q():
    """sigma = 0: every m in Z_4096 decodes from the TFHE-shaped output at Q."""
    b = _gpu()
    pre = PRESETS["tfhe_shaped"]
    p = pre["params"].noise_free()
    dr = key_draws(p, 78)
    ctx = b.Context(p, dr)
    f = negacyclic_table(4096, 4096, 78)
    tid = ctx.table_create(4096, 4096, 1, f)
    m = np.arange(4096, dtype=np.uint32)
    ed = enc_draws(p.n, 8192, 4096, 79, sigma=0.0)
    ct = ctx.encrypt(8192, 4096, m, ed["a"], ed["e"])
    say("noise-free tfhe-shaped 4096")
    out = ctx.bootstrap([tid] * 4096, ct, q_out=Q)
    np.testing.assert_array_equal(ctx.decrypt(Q, 4096, out), f[m])
    ctx.close()
