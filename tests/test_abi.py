"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side calls (key generation, test vectors, encryption) agree bit
for bit with the oracle on the same draws.  No device compute runs here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from synth import PRESETS, Params, enc_draws, key_draws, messages, negacyclic_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _binding():
    from paper_2310_12441_amd import binding
    return binding


def test_header_symbols_exported():
    b = _binding()
    hdr = open(os.path.join(ROOT, "include", "mmpm.h")).read()
    declared = sorted(set(re.findall(r"\b(mm_[a-z_]+)\s*\(", hdr)))
    assert declared, "no declarations found"
    so = ctypes.CDLL(b.LIB_PATH)
    missing = [s for s in declared if not hasattr(so, s)]
    assert not missing, missing
    assert sorted(b.SYMBOLS) == declared


@pytest.mark.parametrize("preset,seed", [("tiny", 0), ("tiny", 9)])
def test_keygen_matches_oracle(preset, seed):
    b = _binding()
    p = PRESETS[preset]["params"]
    dr = key_draws(p, seed)
    ctx = b.Context(p, dr)
    np.testing.assert_array_equal(ctx.export_bsk(), oracle.keygen_bsk(p, dr))
    np.testing.assert_array_equal(ctx.export_ksk(), oracle.keygen_ksk(p, dr))


def test_keygen_matches_oracle_paper_shaped_bsk():
    b = _binding()
    p = PRESETS["paper_shaped"]["params"]
    small = Params(n=24, N=p.N, log2_B=p.log2_B, l=p.l)  # full ring, fewer LWE coordinates
    dr = key_draws(small, 5)
    ctx = b.Context(small, dr)
    np.testing.assert_array_equal(ctx.export_bsk(), oracle.keygen_bsk(small, dr))
    np.testing.assert_array_equal(ctx.export_ksk(), oracle.keygen_ksk(small, dr))


@pytest.mark.parametrize("N,r,t,t_out", [(256, 2, 16, 16), (1024, 4, 4096, 4096), (1024, 1, 256, 256),
                                         (1024, 8, 16384, 16384), (256, 3, 24, 32)])
def test_test_vector_matches_oracle(N, r, t, t_out):
    b = _binding()
    p = Params(n=4, N=N)
    ctx = b.Context(p, key_draws(p, 1))
    f = negacyclic_table(t, t_out, 7)
    tid = ctx.table_create(t, t_out, r, f)
    np.testing.assert_array_equal(ctx.table_export(tid), oracle.test_vector(N, r, p.Q, t, t_out, f))
    assert ctx.table_info(tid) == (t, t_out, r, 2 * N * r)


@pytest.mark.parametrize("q,t", [(1024, 16), (8192, 4096), (2147352577, 4096), (16384, 16384)])
def test_encrypt_decrypt_match_oracle(q, t):
    b = _binding()
    p = Params(n=37, N=256)
    dr = key_draws(p, 2)
    ctx = b.Context(p, dr)
    m = messages(t, 300, 3)
    ed = enc_draws(p.n, q, 300, 4)
    ct = ctx.encrypt(q, t, m, ed["a"], ed["e"])
    np.testing.assert_array_equal(ct, oracle.encrypt(p.n, q, t, dr["s"], m, ed["a"], ed["e"]))
    np.testing.assert_array_equal(ctx.decrypt(q, t, ct), oracle.decrypt(p.n, q, t, dr["s"], ct))


def test_error_paths():
    b = _binding()
    p = Params(n=4, N=256)
    dr = key_draws(p, 1)
    with pytest.raises(b.MMError) as e:
        b.Context(Params(n=4, N=256, Q=2147352579), dr)  # not prime
    assert e.value.code == b.MM_EINVAL
    with pytest.raises(b.MMError):
        b.Context(Params(n=4, N=256, log2_Bks=4, l_ks=6), key_draws(Params(n=4, N=256, l_ks=6), 1))
    ctx = b.Context(p, dr)
    f = negacyclic_table(16, 16, 1)
    with pytest.raises(b.MMError):
        ctx.table_create(16, 16, 2, np.arange(16))  # not nega-cyclic
    with pytest.raises(b.MMError):
        ctx.table_create(12, 16, 2, negacyclic_table(12, 16, 1))  # 12 does not divide 2Nr = 1024
    with pytest.raises(b.MMError):
        ctx.table_create(16, 16, 1025, f)  # r > 1024
    assert ctx.table_create(16, 16, 9, f) >= 0  # r = 9 runs the global-accumulator path
    bad = dict(dr)
    bad["s"] = dr["s"] + 2
    with pytest.raises(b.MMError):
        b.Context(p, bad)


def test_device_calls_fail_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    b = _binding()
    p = PRESETS["tiny"]["params"]
    ctx = b.Context(p, key_draws(p, 1))
    tid = ctx.table_create(16, 16, 2, negacyclic_table(16, 16, 1))
    with pytest.raises(b.MMError) as e:
        ctx.bootstrap([tid], np.zeros((1, p.n + 1), np.uint32))
    assert e.value.code == b.MM_EDEVICE


def test_ternary_keygen_and_encryption_match_oracle():
    from dataclasses import replace
    b = _binding()
    p = replace(PRESETS["tiny"]["params"], ternary=True)
    dr = key_draws(p, 3)
    ctx = b.Context(p, dr)
    np.testing.assert_array_equal(ctx.export_bsk(), oracle.keygen_bsk(p, dr))
    np.testing.assert_array_equal(ctx.export_ksk(), oracle.keygen_ksk(p, dr))
    q, t = 1024, 16
    m = messages(t, 100, 4)
    ed = enc_draws(p.n, q, 100, 5)
    ct = ctx.encrypt(q, t, m, ed["a"], ed["e"])
    np.testing.assert_array_equal(ct, oracle.encrypt(p.n, q, t, dr["s"], m, ed["a"], ed["e"]))
    np.testing.assert_array_equal(ctx.decrypt(q, t, ct), m)


@pytest.mark.parametrize("N", [2048, 8192])
def test_keygen_and_test_vector_match_oracle_large_ring(N):
    """Rings above 1024 (the TFHE-shaped comparison point): keys and an r = 1 test vector."""
    b = _binding()
    p = Params(n=6, N=N, log2_B=7, l=4)
    dr = key_draws(p, 21)
    ctx = b.Context(p, dr)
    np.testing.assert_array_equal(ctx.export_bsk(), oracle.keygen_bsk(p, dr))
    np.testing.assert_array_equal(ctx.export_ksk(), oracle.keygen_ksk(p, dr))
    f = negacyclic_table(4096, 4096, 22)
    tid = ctx.table_create(4096, 4096, 1, f)
    np.testing.assert_array_equal(ctx.table_export(tid), oracle.test_vector(N, 1, p.Q, 4096, 4096, f))


def test_ring_degree_limits():
    b = _binding()
    for N in (32, 131072):
        p = Params(n=4, N=N)
        with pytest.raises(b.MMError) as e:
            b.Context(p, key_draws(p, 1))
        assert e.value.code == b.MM_EINVAL
    # 65536 is the largest ring (the global-accumulator path, split into sub-rings of 8192;
    # 2N divides Q - 1 = 2^17 (2^14 - 1))
    p = Params(n=2, N=65536)
    dr = key_draws(p, 1)
    ctx = b.Context(p, dr)
    np.testing.assert_array_equal(ctx.export_bsk(), oracle.keygen_bsk(p, dr))


@pytest.mark.parametrize("N,ternary", [(256, False), (2048, True)])
def test_wide_keygen_and_test_vector_match_oracle(N, ternary):
    """A 54-bit ring modulus Q Q2: the library keeps two residues per coefficient
    and exports uint64 values equal to the oracle's."""
    from synth import Q2_DEFAULT
    b = _binding()
    p = Params(n=3, N=N, log2_B=15, l=4, Q2=Q2_DEFAULT, ternary=ternary)
    dr = key_draws(p, 23)
    ctx = b.Context(p, dr)
    np.testing.assert_array_equal(ctx.export_bsk(), oracle.w_keygen_bsk(p, dr))
    np.testing.assert_array_equal(ctx.export_ksk(), oracle.keygen_ksk(p, dr))
    for t, r in ((16, 1), (4096, 128), (24, 3)):
        f = negacyclic_table(t, t, 24 + r)
        tid = ctx.table_create(t, t, r, f)
        assert ctx.table_info(tid) == (t, t, r, 2 * N * r)
        np.testing.assert_array_equal(ctx.table_export(tid), oracle.w_test_vector(N, r, p.Q_ring, t, t, f))


def test_wide_parameter_limits():
    from dataclasses import replace
    from synth import Q2_DEFAULT
    b = _binding()
    p = Params(n=3, N=256, log2_B=15, l=4, Q2=Q2_DEFAULT)
    dr = key_draws(p, 25)
    bad = [dict(Q2=p.Q), dict(Q2=Q2_DEFAULT - 1), dict(Q2=2013265921),  # Q + 2 Q2 >= 2^32
           dict(log2_B=17), dict(l=5, log2_B=13), dict(Q2=12289, log2_B=15)]  # 2B >= Q2
    for kw in bad:
        with pytest.raises(b.MMError) as e:
            b.Context(replace(p, **kw), dr)
        assert e.value.code == b.MM_EINVAL, kw
    ctx = b.Context(p, dr)
    with pytest.raises(b.MMError):
        ctx.table_create(8, 8, 2048, np.zeros(8, np.uint32))
