"""GPU parity of the blind rotation at a wide ring modulus Q Q2 (54 bits, gadget
2^15 x 4: the parameters of the experiments in Sec. 5), bit-exact against the
oracle's uint64 statement of the same steps.

The accumulator lives in device memory and each CMux step is one launch, so r
is no longer bounded by a workgroup: the cases cover r from 1 to 128, mixed r
in one call, N from 256 to 2048 (one polynomial over two waves at 2048), both
secret types, the plain and the batched path, and, at the full paper-margin
size (n = 512, N = 2048, r = 128, t = 2^12), the first steps against the oracle
and correct decryption of noisy inputs for a whole batch.
"""
from dataclasses import replace

import numpy as np
import pytest

import oracle
from synth import PRESETS, Q2_DEFAULT, Params, enc_draws, key_draws, messages, negacyclic_table

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_12441_amd import binding
    return binding


def say(*a):
    print(*a, flush=True)


class WideCase:
    def __init__(self, p, seed):
        b = _gpu()
        self.p = p
        self.draws = key_draws(p, seed)
        self.ctx = b.Context(p, self.draws)
        self.keys = oracle.KeySetWide(p, self.draws)
        self.ctx.device_init(0)

    def table(self, t, r, seed):
        f = negacyclic_table(t, t, seed)
        tid = self.ctx.table_create(t, t, r, f)
        return tid, f, oracle.w_test_vector(self.p.N, r, self.p.Q_ring, t, t, f)

    def encrypt(self, q, t, m, seed, sigma=3.2):
        ed = enc_draws(self.p.n, q, len(m), seed, sigma)
        return oracle.encrypt(self.p.n, q, t, self.keys.s, m, ed["a"], ed["e"])


_cases = {}


def case(N, n, ternary=False):
    key = (N, n, ternary)
    if key not in _cases:
        say("wide keygen N", N, "n", n, "ternary", ternary)
        p = Params(n=n, N=N, log2_B=15, l=4, Q2=Q2_DEFAULT, ternary=ternary)
        _cases[key] = WideCase(p, 1300 + N + n + ternary)
    return _cases[key]


@pytest.mark.parametrize("N,rs,steps", [(256, (1, 3, 8), 3), (256, (64,), 2), (512, (2, 5), 4),
                                        (1024, (4,), 2), (2048, (1, 2), 2)])
def test_wide_blind_rotate_steps(N, rs, steps):
    say("wide blind_rotate N", N, "rs", rs, "steps", steps)
    c = case(N, 8)
    ids, cts, Vs, rr = [], [], [], []
    for k, r in enumerate(rs):
        t = max(2, 2 * N * r // 128)
        tid, f, V = c.table(t, r, 40 + k)
        ct = c.encrypt(2 * N * r, t, messages(t, 2, 50 + k), 60 + k)
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
        want = oracle.w_blind_rotate(c.p, r, c.keys.bsk, Vs[j], cts[j], steps)
        np.testing.assert_array_equal(got[off:off + size].reshape(r, 2, N), want, err_msg=f"ct {j} r {r}")
        off += size
    assert off == got.size


@pytest.mark.parametrize("N,r", [(256, 4), (256, 1), (512, 2)])
def test_wide_bootstrap_matches_oracle_and_decrypts(N, r):
    say("wide bootstrap N", N, "r", r)
    c = case(N, 16)
    t = 2 * N * r // 128
    q = 2 * N * r
    tid, f, V = c.table(t, r, 70 + r)
    m = np.arange(t, dtype=np.uint32)
    ct = c.encrypt(q, t, m, 71 + r)
    got = c.ctx.bootstrap([tid] * t, ct)
    want = oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(oracle.decrypt(c.p.n, q, t, c.keys.s, got), f[m])
    np.testing.assert_array_equal(c.ctx.bootstrap([tid] * t, ct, plain=True), got)


def test_wide_bootstrap_mixed_r_and_q_out():
    c = case(256, 16)
    rs = (1, 2, 8)
    tids, cts, want = [], [], []
    for k, r in enumerate(rs):
        t = 2 * 256 * r // 128
        q = 2 * 256 * r
        tid, f, V = c.table(t, r, 80 + k)
        ct = c.encrypt(q, t, messages(t, 2, 81 + k), 82 + k)
        tids += [tid] * 2
        cts.append(ct)
        want.append(oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, c.p.Q, ct))
    got = c.ctx.bootstrap(tids, np.concatenate(cts), q_out=c.p.Q)
    np.testing.assert_array_equal(got, np.concatenate(want))


def test_wide_ternary():
    c = case(512, 6, ternary=True)
    r, t = 2, 16
    q = 2 * 512 * r
    tid, f, V = c.table(t, r, 90)
    ct = c.encrypt(q, t, messages(t, 3, 91), 92)
    got = c.ctx.blind_rotate([tid] * 3, ct, 3)
    for j in range(3):
        want = oracle.w_blind_rotate(c.p, r, c.keys.bsk, V, ct[j], 3)
        np.testing.assert_array_equal(got[j * r * 2 * 512:(j + 1) * r * 2 * 512].reshape(r, 2, 512), want)
    out = c.ctx.bootstrap([tid] * 3, ct)
    np.testing.assert_array_equal(out, oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct))


@pytest.mark.parametrize("plain", [False, True])
def test_wide_ternary_2048_end_to_end(plain):
    """The ternary wide-modulus kernel the paper-margin rows time (N = 2048, two
    waves per polynomial, both CMux terms per step), over a whole bootstrap at
    small n, r = 2, 2Nr/t = 128: against the oracle, and the outputs decrypt."""
    c = case(2048, 8, ternary=True)
    r = 2
    t = 2 * 2048 * r // 128
    q = 2 * 2048 * r
    tid, f, V = c.table(t, r, 93)
    m = messages(t, 3, 94)
    ct = c.encrypt(q, t, m, 95)
    say("wide ternary N=2048 bootstrap plain", plain)
    got = c.ctx.bootstrap([tid] * 3, ct, plain=plain)
    np.testing.assert_array_equal(got, oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct))
    np.testing.assert_array_equal(oracle.decrypt(c.p.n, q, t, c.keys.s, got), f[m])


@pytest.mark.parametrize("ternary", [False, True])
def test_wide_blind_rotate_4096(ternary):
    """N = 4096 at the wide modulus (8 waves per polynomial; the largest ring the
    second prime carries): three CMux steps for mixed r against the oracle, and
    a whole bootstrap at small n."""
    c = case(4096, 4, ternary=ternary)
    ids, cts, Vs, rr = [], [], [], []
    for k, r in enumerate((1, 2)):
        t = 2 * 4096 * r // 128
        tid, f, V = c.table(t, r, 130 + k)
        ct = c.encrypt(2 * 4096 * r, t, messages(t, 1, 131 + k), 132 + k)
        ids.append(tid)
        cts.append(ct[0])
        Vs.append(V)
        rr.append(r)
    say("wide N=4096 ternary", ternary, "3 steps")
    got = c.ctx.blind_rotate(ids, np.array(cts), 3)
    off = 0
    for j, r in enumerate(rr):
        size = r * 2 * 4096
        want = oracle.w_blind_rotate(c.p, r, c.keys.bsk, Vs[j], cts[j], 3)
        np.testing.assert_array_equal(got[off:off + size].reshape(r, 2, 4096), want, err_msg=f"ct {j} r {r}")
        off += size
    q = 2 * 4096
    out = c.ctx.bootstrap([ids[0]], np.array(cts[:1]))
    np.testing.assert_array_equal(out, oracle.w_bootstrap_many(c.p, 1, c.keys.bsk, c.keys.ksk, Vs[0], q, q,
                                                               np.array(cts[:1])))


def test_wide_bootstrap_2048():
    c = case(2048, 8)
    r = 2
    t = 2 * 2048 * r // 128
    q = 2 * 2048 * r
    tid, f, V = c.table(t, r, 95)
    ct = c.encrypt(q, t, messages(t, 2, 96), 97)
    got = c.ctx.bootstrap([tid] * 2, ct)
    np.testing.assert_array_equal(got, oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct))


@pytest.mark.parametrize("N,r", [(256, 4), (2048, 2)])
def test_wide_identity_function_two_bootstraps(N, r):
    """f(x) = x, not nega-cyclic: the sign bootstrap, the top-bit removal and the
    second bootstrap, at the wide modulus, against the oracle; noisy inputs decrypt."""
    c = case(N, 16)
    t = 2 * N * r // 128 // 2
    q = 2 * N * r
    f = np.arange(t, dtype=np.uint32)
    tid = c.ctx.table_create_general(t, t, r, f)
    g, F = oracle.general_tables(t, t, f)
    Vg = oracle.w_test_vector(N, r, c.p.Q_ring, 2 * t, 2 * t, g)
    VF = oracle.w_test_vector(N, r, c.p.Q_ring, 2 * t, t, F)
    m = messages(t, 16 if N <= 512 else 4, 110 + r)
    ct = c.encrypt(q, 2 * t, m, 111 + r)
    got = c.ctx.bootstrap([tid] * len(m), ct)
    np.testing.assert_array_equal(got, oracle.w_bootstrap_general(c.p, r, c.keys.bsk, c.keys.ksk, Vg, VF, q, t, q, ct))
    np.testing.assert_array_equal(oracle.decrypt(c.p.n, q, t, c.keys.s, got), m)


def test_wide_empty_and_rejected_calls():
    b = _gpu()
    c = case(256, 8)
    tid, f, V = c.table(8, 4, 99)
    assert c.ctx.bootstrap(np.zeros(0, np.int32), np.zeros((0, 9), np.uint32)).shape == (0, 9)
    with pytest.raises(b.MMError):
        c.ctx.table_create(8, 8, 2048, np.zeros(8, np.uint32))  # r above 1024
    with pytest.raises(b.MMError):
        c.ctx.external_product(0, np.zeros((1, 2, 256), np.uint32))
    with pytest.raises(b.MMError):
        c.ctx.server_start(1 << 10)  # below one component's two accumulators


@pytest.mark.parametrize("N,ternary,r,count", [(256, False, 2, 70), (2048, True, 1, 3), (512, True, 4, 80),
                                                (1024, False, 3, 12), (1024, True, 1, 2)])
def test_wide_schedules_give_the_same_bits_and_autotune(N, ternary, r, count):
    """At the wide modulus the blind rotation has two shapes (reported as 0 waves per
    fused group, one workgroup of N / 512 waves per component): one workgroup per
    component (NTT schedule 0) or one per component and prime (5, the default up to 16
    components per compute unit; 6, of two digit groups, at N = 1024 and 2048); the schedules
    also differ in the key switch, every one gives the oracle's bits, and autotuning
    picks one of them."""
    say("wide schedules N", N, "ternary", ternary, "r", r, "count", count)
    c = case(N, 8, ternary)
    t = 16
    q = 2 * N * r
    tid, f, V = c.table(t, r, 31)
    ct = c.encrypt(q, t, messages(t, count, 32), 33)
    ids = np.full(len(ct), tid, np.int32)
    n = c.ctx.schedule_count(ids)
    desc = [c.ctx.schedule_describe(ids, k) for k in range(n)]
    say("wide schedules:", desc)
    assert n >= 2 and all(d[0] == 0 and d[3] == max(1, N // 512) for d in desc)
    assert {d[5] for d in desc} == ({0, 5, 6} if N in (1024, 2048) else {0, 5})
    # the defaults: per-prime workgroups up to 16 components per compute unit, of two digit
    # groups where both primes' workgroups fit one per compute unit (N = 1024, 2048)
    assert c.ctx.schedule_describe(ids)[5] == (6 if N in (1024, 2048) and 2 * count * r <= 256 else 5)
    if count >= 64:
        assert {d[4] for d in desc} >= {0, 1}  # i-split and LDS-tiled key switches
    want = oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct)
    for k in range(n):
        c.ctx.set_schedule(ids, k)
        np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct), want, err_msg=f"schedule {k}")
        if desc[k][5] in (5, 6):
            np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct, plain=True), want, err_msg=f"plain, schedule {k}")
    choice = c.ctx.autotune(ids, ct)
    assert 0 <= choice < n
    assert c.ctx.schedule_describe(ids) == desc[choice]
    np.testing.assert_array_equal(c.ctx.bootstrap(ids, ct), want)


@pytest.mark.parametrize("N,ternary", [(256, False), (512, True)])
def test_wide_serving_matches_alone_and_oracle(N, ternary):
    """Continuous batching at the wide modulus: a Poisson trace over tables of r = 1, 3
    and 16 through a server whose budget holds fewer components than arrive, so requests
    wait for memory and join running ticks; chunk_steps = 3 does not divide n = 8, so
    ciphertexts finish inside a tick.  Every result equals the same ciphertext
    bootstrapped alone and, for two per table, the oracle's."""
    from synth import poisson_arrivals
    c = case(N, 8, ternary)
    tabs = []
    for k, r in enumerate((1, 3, 16)):
        t = max(2, 2 * N * r // 128)
        tid, f, V = c.table(t, r, 140 + k)
        q = 2 * N * r
        tabs.append((tid, t, r, q, V, c.encrypt(q, t, messages(t, 12, 150 + k), 160 + k)))
    order = np.random.default_rng(170).permutation(36)
    ids = np.array([tabs[k // 12][0] for k in order], np.int32)
    cts = np.stack([tabs[k // 12][5][k % 12] for k in order])
    per_comp = 2 * 2 * 2 * N * 4  # two arenas x (a, b) x two residues
    budget = 40 * (per_comp + (9 + N + 1) * 4 + 9 * 8)  # 40 components for 36 requests of up to 16
    srv = c.ctx.server_start(budget, chunk_steps=3)
    try:
        say("wide serving N", N, "ternary", ternary)
        out, lat = srv.replay(ids, cts, poisson_arrivals(2000.0, len(ids), 171))
        st = srv.stats()
    finally:
        srv.stop()
    assert st["completed"] == len(ids) and np.all(lat > 0)
    for tid, t, r, q, V, ct in tabs:
        sel = ids == tid
        np.testing.assert_array_equal(out[sel], c.ctx.bootstrap(ids[sel], cts[sel]), err_msg=f"r = {r}")
        np.testing.assert_array_equal(out[sel][:2], oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q,
                                                                          cts[sel][:2]), err_msg=f"oracle r = {r}")


@pytest.fixture(scope="module")
def margin():
    pre = PRESETS["paper_margin"]
    say("paper-margin keygen (n = 512, N = 2048)")
    return WideCase(pre["params"], 21), pre


@pytest.mark.parametrize("steps", [1, 3])
def test_paper_margin_first_steps(margin, steps):
    """n = 512, N = 2048, r = 128, ternary: the accumulator after the
    initialisation and the first CMux steps, against the oracle, for one
    ciphertext (every component)."""
    c, pre = margin
    t, r = pre["t"], pre["r"]
    q = 2 * c.p.N * r
    tid, f, V = c.table(t, r, 22)
    ct = c.encrypt(q, t, messages(t, 1, 23), 24)
    got = c.ctx.blind_rotate([tid], ct, steps).reshape(r, 2, c.p.N)
    say("oracle,", steps, "steps at r = 128")
    want = oracle.w_blind_rotate(c.p, r, c.keys.bsk, V, ct[0], steps)
    np.testing.assert_array_equal(got, want)


def test_paper_margin_r_1024_two_steps(margin):
    """The largest table of the sweep (log t = 15: r = 1024 at N = 2048, Table 2),
    ternary, 54-bit ring: two CMux steps against the oracle."""
    c, pre = margin
    r, t = 1024, 1 << 15
    q = 2 * c.p.N * r
    tid, f, V = c.table(t, r, 28)
    ct = c.encrypt(q, t, messages(t, 1, 29), 30)
    got = c.ctx.blind_rotate([tid], ct, 2).reshape(r, 2, c.p.N)
    say("oracle, two steps at r = 1024")
    want = oracle.w_blind_rotate(c.p, r, c.keys.bsk, V, ct[0], 2)
    np.testing.assert_array_equal(got, want)


def test_paper_margin_noisy_batch_decrypts_at_t_4096(margin):
    """A batch of noisy encryptions (sigma 3.2) at t = 2^12, 2Nr/t = 128: every
    output decrypts to f(m), with the output noise well inside Delta/2."""
    c, pre = margin
    t, r = pre["t"], pre["r"]
    q = 2 * c.p.N * r
    tid, f, V = c.table(t, r, 25)
    m = messages(t, 64, 26)
    ct = c.encrypt(q, t, m, 27)
    say("paper-margin bootstrap of 64")
    out = c.ctx.bootstrap([tid] * 64, ct)
    np.testing.assert_array_equal(oracle.decrypt(c.p.n, q, t, c.keys.s, out), f[m])
    ph = oracle.lwe_phase(c.p.n, q, c.keys.s, out).astype(np.int64)
    err = (ph - f[m].astype(np.int64) * (q // t)) % q
    err = np.where(err > q // 2, err - q, err)
    assert np.max(np.abs(err)) < 32


def test_paper_margin_serving_matches_alone_and_decrypts(margin):
    """The paper-margin shape served: noisy requests at t = 2^12 (r = 128, n = 512,
    N = 2048, ternary, 54-bit ring) through the server in ticks of 64 CMux steps;
    every result equals the batched bootstrap of the same ciphertexts and decrypts."""
    from synth import poisson_arrivals
    c, pre = margin
    t, r = pre["t"], pre["r"]
    q = 2 * c.p.N * r
    tid, f, V = c.table(t, r, 35)
    m = messages(t, 6, 36)
    ct = c.encrypt(q, t, m, 37)
    ids = np.full(len(m), tid, np.int32)
    srv = c.ctx.server_start(256 << 20, chunk_steps=64)
    try:
        say("paper-margin serving of", len(m))
        out, lat = srv.replay(ids, ct, poisson_arrivals(100.0, len(m), 38))
    finally:
        srv.stop()
    say("latency ms", np.round(lat, 1))
    np.testing.assert_array_equal(out, c.ctx.bootstrap(ids, ct))
    np.testing.assert_array_equal(oracle.decrypt(c.p.n, q, t, c.keys.s, out), f[m])


def test_wide_maximum_r_1024():
    """r = 1024 (the largest table) at N = 256: two CMux steps against the oracle."""
    c = case(256, 8)
    r = 1024
    t = 2 * 256 * r // 128
    tid, f, V = c.table(t, r, 120)
    ct = c.encrypt(2 * 256 * r, t, messages(t, 1, 121), 122)
    say("wide r = 1024, 2 steps")
    got = c.ctx.blind_rotate([tid], ct, 2).reshape(r, 2, 256)
    np.testing.assert_array_equal(got, oracle.w_blind_rotate(c.p, r, c.keys.bsk, V, ct[0], 2))


def test_wide_ragged_batches_and_device_pointers():
    """Batch sizes 1, 3, 17, 64 give the bits of one batch of 65; device tensors in and out
    give the bits of host buffers (bootstrap and blind rotation)."""
    import torch
    c = case(256, 16)
    r = 2
    t = 2 * 256 * r // 128
    q = 2 * 256 * r
    tid, f, V = c.table(t, r, 123)
    ct = c.encrypt(q, t, messages(t, 65, 124), 125)
    full = c.ctx.bootstrap([tid] * 65, ct)
    for cnt in (1, 3, 17, 64):
        np.testing.assert_array_equal(c.ctx.bootstrap([tid] * cnt, ct[:cnt]), full[:cnt], err_msg=f"count {cnt}")
    np.testing.assert_array_equal(full[64], oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q, q, ct[64:]).reshape(-1))
    din = torch.from_numpy(ct.view(np.int32)).cuda()
    dout = c.ctx.bootstrap([tid] * 65, din)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dout.cpu().numpy().view(np.uint32), full)
    host_acc = c.ctx.blind_rotate([tid] * 3, ct[:3], 4)
    dev_acc = c.ctx.blind_rotate([tid] * 3, din[:3].contiguous(), 4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(dev_acc.cpu().numpy().view(np.uint64).reshape(-1), host_acc.reshape(-1))


def test_wide_general_function_plain_at_r_256():
    """A general f with r = 256 (t = 512 at N = 256) by the plain path, against the batched
    path and the oracle for one ciphertext."""
    c = case(256, 16)
    r = 256
    t = 2 * 256 * r // 128 // 2
    q = 2 * 256 * r
    rng = np.random.default_rng(126)
    f = rng.integers(0, t, t).astype(np.uint32)
    tid = c.ctx.table_create_general(t, t, r, f)
    m = messages(t, 2, 127)
    ct = c.encrypt(q, 2 * t, m, 128)
    batched = c.ctx.bootstrap([tid] * 2, ct)
    np.testing.assert_array_equal(c.ctx.bootstrap([tid] * 2, ct, plain=True), batched)
    np.testing.assert_array_equal(oracle.decrypt(c.p.n, q, t, c.keys.s, batched), f[m])
    g, F = oracle.general_tables(t, t, f)
    Vg = oracle.w_test_vector(256, r, c.p.Q_ring, 2 * t, 2 * t, g)
    VF = oracle.w_test_vector(256, r, c.p.Q_ring, 2 * t, t, F)
    np.testing.assert_array_equal(batched[:1], oracle.w_bootstrap_general(c.p, r, c.keys.bsk, c.keys.ksk, Vg, VF, q,
                                                                           t, q, ct[:1]))


@pytest.mark.parametrize("q_in", [2 ** 31, 12289])
def test_wide_first_switch_not_identity(q_in):
    """Ciphertexts at q_in other than 2Nr on the wide path (the switch runs in the
    accumulator initialisation and in every step)."""
    c = case(256, 16)
    r, t = 4, 16
    f = negacyclic_table(t, t, 130)
    tid = c.ctx.table_create(t, t, r, f, q_in)
    V = oracle.w_test_vector(256, r, c.p.Q_ring, t, t, f)
    m = np.arange(t, dtype=np.uint32)
    ct = c.encrypt(q_in, t, m, 131)
    got = c.ctx.bootstrap([tid] * t, ct)
    np.testing.assert_array_equal(got, oracle.w_bootstrap_many(c.p, r, c.keys.bsk, c.keys.ksk, V, q_in, q_in, ct))
    np.testing.assert_array_equal(oracle.decrypt(c.p.n, q_in, t, c.keys.s, got), f[m])
