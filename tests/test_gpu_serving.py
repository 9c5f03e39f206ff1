"""Serving (continuous batching) on the GPU: requests of mixed (t, r) that
arrive while others run are admitted at tick boundaries, and every result is
bit-identical to the same ciphertext bootstrapped alone."""
import time

import numpy as np
import pytest

import oracle
from synth import CLASS_MIX, PRESETS, class_mix, enc_draws, key_draws, messages, negacyclic_table, poisson_arrivals

pytestmark = pytest.mark.gpu
Q = 2147352577


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_12441_amd import binding
    p = PRESETS["paper_shaped"]["params"]
    draws = key_draws(p, 31)
    ctx = binding.Context(p, draws)
    ctx.device_init(0)
    tabs = []
    for k, (t, r) in enumerate(CLASS_MIX):
        f = negacyclic_table(t, t, 60 + k)
        tabs.append((ctx.table_create(t, t, r, f), t, r, f))
    keys = oracle.KeySet(p, draws)
    yield p, ctx, tabs, keys, binding
    ctx.close()


def _requests(p, keys, tabs, count, seed):
    cls = class_mix(count, seed)
    ids, cts = [], []
    for c, k in enumerate(cls):
        tid, t, r, f = tabs[k]
        q = 2 * p.N * r
        ed = enc_draws(p.n, q, 1, seed * 1000 + c)
        cts.append(oracle.encrypt(p.n, q, t, keys.s, messages(t, 1, seed * 1000 + c), ed["a"], ed["e"])[0])
        ids.append(tid)
    return np.array(ids, np.int32), np.array(cts, np.uint32), cls


def test_submit_poll_matches_alone(setup):
    p, ctx, tabs, keys, b = setup
    ids, cts, cls = _requests(p, keys, tabs, 40, 1)
    srv = ctx.server_start(256 << 20, chunk_steps=90)
    tickets = []
    for k in range(len(ids)):
        tickets.append(srv.submit(int(ids[k]), cts[k]))
        if k % 10 == 9:
            time.sleep(0.003)  # later requests arrive while earlier ones run
    got = [None] * len(ids)
    deadline = time.time() + 60
    while any(g is None for g in got) and time.time() < deadline:
        for k, tk in enumerate(tickets):
            if got[k] is None:
                got[k] = srv.poll(tk)
        time.sleep(0.002)
    if got[0] is not None:
        with pytest.raises(b.MMError):
            srv.poll(tickets[0])  # collected already: an error, not "not ready" forever
    st = srv.stats()
    srv.stop()
    assert all(g is not None for g in got)
    alone = ctx.bootstrap(ids, cts, plain=True)
    np.testing.assert_array_equal(np.array(got), alone)
    assert st["completed"] == len(ids)
    # one per class against the oracle
    for k in range(4):
        c = int(np.where(cls == k)[0][0])
        tid, t, r, f = tabs[k]
        V = oracle.test_vector(p.N, r, Q, t, t, f)
        q = 2 * p.N * r
        np.testing.assert_array_equal(got[c], oracle.bootstrap(p, r, keys.bsk, keys.ksk, V, q, q, cts[c]))


def test_replay_poisson_trace_small_budget(setup):
    """A budget of a few hundred slots forces admission to wait for completions."""
    p, ctx, tabs, keys, b = setup
    ids, cts, cls = _requests(p, keys, tabs, 600, 2)
    arrivals = poisson_arrivals(3000.0, len(ids), 5)
    srv = ctx.server_start(24 << 20, chunk_steps=63)
    out, lat = srv.replay(ids, cts, arrivals)
    st = srv.stats()
    srv.stop()
    np.testing.assert_array_equal(out, ctx.bootstrap(ids, cts))
    assert np.all(lat > 0) and st["completed"] == len(ids)
    assert st["p99_ms"] >= st["p50_ms"] > 0
    print("serving p50 %.2f ms p99 %.2f ms, %.0f boots/s" % (st["p50_ms"], st["p99_ms"], st["boots_per_s"]))


def test_admission_sheds_load_and_admitted_results_are_exact(setup):
    """Arrivals far above capacity with admission by expected latency on:
    some requests are refused (latency -1, zero output, counted by the server),
    every admitted one equals the same ciphertext bootstrapped alone."""
    p, ctx, tabs, keys, b = setup
    ids, cts, cls = _requests(p, keys, tabs, 3000, 6)
    arrivals = poisson_arrivals(50000.0, len(ids), 7)
    srv = ctx.server_start(24 << 20, chunk_steps=63)
    with pytest.raises(b.MMError):
        srv.set_admission(-1.0)
    srv.set_admission(40.0)
    out, lat = srv.replay(ids, cts, arrivals)
    st = srv.stats()
    refused = srv.refused()
    srv.stop()
    shed = lat < 0
    print("admission: %d of %d refused; admitted p50 %.2f ms p99 %.2f ms" %
          (shed.sum(), len(ids), np.percentile(lat[~shed], 50), np.percentile(lat[~shed], 99)))
    assert shed.sum() == refused > 0
    assert st["completed"] == len(ids) - refused
    assert np.all(out[shed] == 0)
    np.testing.assert_array_equal(out[~shed], ctx.bootstrap(ids[~shed], cts[~shed]))


def test_ticks_switch_between_fused_and_global_kernels(setup):
    """A burst of 1500 requests (ticks of many components per compute unit: the fused
    kernel) followed by sparse arrivals (light ticks: the global-accumulator kernel with
    four waves per component): ciphertexts change kernels between ticks, and every result
    equals the same ciphertext bootstrapped alone."""
    p, ctx, tabs, keys, b = setup
    ids, cts, cls = _requests(p, keys, tabs, 1700, 11)
    arrivals = np.concatenate([np.zeros(1500, np.int64),
                               np.sort(np.random.default_rng(12).integers(0, 300_000_000, 200)) + 1000])
    srv = ctx.server_start(1 << 30, chunk_steps=63)
    out, lat = srv.replay(ids, cts, arrivals)
    st = srv.stats()
    srv.stop()
    print("burst then sparse: p50 %.1f ms p99 %.1f ms; sparse part p50 %.1f ms" %
          (np.percentile(lat, 50), np.percentile(lat, 99), np.percentile(lat[1500:], 50)))
    assert st["completed"] == len(ids) and np.all(lat > 0)
    np.testing.assert_array_equal(out, ctx.bootstrap(ids, cts))


def test_server_errors(setup):
    p, ctx, tabs, keys, b = setup
    with pytest.raises(b.MMError):
        ctx.server_start(1 << 10)  # budget too small
    srv = ctx.server_start(64 << 20)
    with pytest.raises(b.MMError):
        srv.submit(99, np.zeros(p.n + 1, np.uint32))  # unknown table
    with pytest.raises(b.MMError):
        ctx.server_start(64 << 20)  # one server per context
    srv.stop()


def test_server_refuses_after_stop_and_tickets_never_issued(setup):
    p, ctx, tabs, keys, b = setup
    srv = ctx.server_start(64 << 20)
    with pytest.raises(b.MMError):
        srv.poll(12345)  # never issued
    srv.stop()
    with pytest.raises(Exception):
        srv.submit(tabs[0][0], np.zeros(p.n + 1, np.uint32))
