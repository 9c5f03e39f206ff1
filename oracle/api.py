"""numpy-facing wrappers over the C oracle, plus the key-size formulas.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .build import ensure_built

__all__ = [
    "lib", "num_threads", "modswitch", "poly_mul", "monomial_mul", "phi_entry", "rotate",
    "test_vector", "gadget_shift", "gadget", "decompose", "keygen_bsk", "keygen_ksk",
    "encrypt", "decrypt", "lwe_phase", "external_product", "blind_rotate", "sample_extract",
    "keyswitch", "bootstrap", "bootstrap_many", "KeySet", "bsk_bytes", "ksk_bytes",
    "general_tables", "bootstrap_general",
    "w_poly_mul", "w_rotate", "w_test_vector", "w_gadget_shift", "w_gadget", "w_decompose", "w_keygen_bsk",
    "w_external_product", "w_blind_rotate", "w_modswitch", "w_sample_extract", "w_bootstrap", "w_bootstrap_many",
    "KeySetWide", "w_bootstrap_general",
]

_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32 = C.c_uint32
_u64 = C.c_uint64

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(ensure_built())
        sig = {
            "orc_num_threads": (C.c_int, []),
            "orc_modswitch_vec": (None, [_u32p, _u64, _u32, _u32, _u32p]),
            "orc_poly_mul": (None, [_u32, _u32, _u32p, _u32p, _u32p]),
            "orc_monomial_mul": (None, [_u32, _u32, _u64, _u32p, _u32p]),
            "orc_phi_entry": (_u32, [_u32, _u32, _u64, _u32, C.POINTER(_u64)]),
            "orc_rotate": (None, [_u32, _u32, _u32, _u64, _u32p, _u32p]),
            "orc_test_vector": (None, [_u32, _u32, _u32, _u32, _u32, _u32p, _u32p]),
            "orc_gadget_shift": (_u32, [_u32, _u32, _u32]),
            "orc_gadget": (_u32, [_u32, _u32, _u32, _u32]),
            "orc_decompose": (None, [_u32, _u32, _u32, _u32, _i32p]),
            "orc_keygen_bsk": (None, [_u32, _u32, _u32, _u32, _u32, _u32, _i32p, _u32p, _u32p, _i32p, _u32p]),
            "orc_keygen_ksk": (None, [_u32, _u32, _u32, _u32, _u32, _i32p, _u32p, _u32p, _i32p, _u32p]),
            "orc_encrypt": (None, [_u32, _u32, _u32, _i32p, _u32p, _u32p, _i32p, _u64, _u32p]),
            "orc_decrypt": (None, [_u32, _u32, _u32, _i32p, _u32p, _u64, _u32p]),
            "orc_lwe_phase": (None, [_u32, _u32, _i32p, _u32p, _u64, _u32p]),
            "orc_external_product": (None, [_u32, _u32, _u32, _u32, _u32p, _u32p, _u32p]),
            "orc_blind_rotate": (None, [_u32] * 7 + [_u32p, _u32p, _u32p, _u32, _u32p]),
            "orc_sample_extract": (None, [_u32, _u32, _u32p, _u32p]),
            "orc_keyswitch": (None, [_u32, _u32, _u32, _u32, _u32, _u32p, _u32p, _u32p]),
            "orc_bootstrap": (None, [_u32] * 9 + [_u32p, _u32p, _u32p, _u32, _u32, _u32p, _u32p,
                                                 C.c_void_p, C.c_void_p, C.c_void_p]),
            "orc_bootstrap_many": (None, [_u32] * 9 + [_u32p, _u32p, _u32p, _u32, _u32, _u32p, _u64, _u32p]),
            "orc_general_tables": (None, [_u32, _u32, _u32p, _u32p, _u32p]),
            "orc_bootstrap_general": (None, [_u32] * 9 + [_u32p, _u32p, _u32p, _u32p, _u32, _u32, _u32,
                                                         _u32p, _u32p]),
            "orc_w_poly_mul": (None, [_u32, _u64, _u64p, _u64p, _u64p]),
            "orc_w_rotate": (None, [_u32, _u32, _u64, _u64, _u64p, _u64p]),
            "orc_w_test_vector": (None, [_u32, _u32, _u64, _u32, _u32, _u32p, _u64p]),
            "orc_w_gadget_shift": (_u32, [_u64, _u32, _u32]),
            "orc_w_gadget": (_u64, [_u64, _u32, _u32, _u32]),
            "orc_w_decompose": (None, [_u64, _u32, _u32, _u64, _i64p]),
            "orc_w_keygen_bsk": (None, [_u32, _u32, _u64, _u32, _u32, _u32, _i32p, _u32p, _u64p, _i32p, _u64p]),
            "orc_w_external_product": (None, [_u32, _u64, _u32, _u32, _u64p, _u64p, _u64p]),
            "orc_w_blind_rotate": (None, [_u32, _u32, _u64, _u32, _u32, _u32, _u32, _u64p, _u64p, _u32p, _u32,
                                          _u64p]),
            "orc_w_modswitch": (_u64, [_u64, _u64, _u64]),
            "orc_w_sample_extract": (None, [_u32, _u64, _u64p, _u64p]),
            "orc_w_bootstrap": (None, [_u32, _u32, _u64, _u32, _u32, _u32, _u32, _u32, _u32, _u32, _u64p, _u32p,
                                       _u64p, _u32, _u32, _u32p, _u32p, C.c_void_p]),
            "orc_w_bootstrap_many": (None, [_u32, _u32, _u64, _u32, _u32, _u32, _u32, _u32, _u32, _u32, _u64p,
                                            _u32p, _u64p, _u32, _u32, _u32p, _u64, _u32p]),
            "orc_w_bootstrap_general": (None, [_u32, _u32, _u64, _u32, _u32, _u32, _u32, _u32, _u32, _u32, _u64p,
                                               _u32p, _u64p, _u64p, _u32, _u32, _u32, _u32p, _u64, _u32p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _i(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def modswitch(x, q_from: int, q_to: int) -> np.ndarray:
    x = _u(x)
    out = np.empty_like(x)
    lib().orc_modswitch_vec(x.reshape(-1), x.size, q_from, q_to, out.reshape(-1))
    return out


def poly_mul(a, b, Q: int) -> np.ndarray:
    a, b = _u(a), _u(b)
    out = np.empty_like(a)
    lib().orc_poly_mul(a.size, Q, a, b, out)
    return out


def monomial_mul(p, e: int, Q: int) -> np.ndarray:
    p = _u(p)
    out = np.empty_like(p)
    lib().orc_monomial_mul(p.size, Q, e, p, out)
    return out


def phi_entry(N: int, r: int, c: int, j: int):
    """(column, exponent) of the only nonzero entry in row j of Phi(c)."""
    e = _u64(0)
    col = lib().orc_phi_entry(N, r, c, j, C.byref(e))
    return int(col), int(e.value)


def rotate(v, c: int, Q: int) -> np.ndarray:
    """Phi(c) v for v of shape (r, N)."""
    v = _u(v)
    r, N = v.shape
    out = np.empty_like(v)
    lib().orc_rotate(N, r, Q, c % (2 * N * r), v, out)
    return out


def test_vector(N: int, r: int, Q: int, t: int, t_out: int, f) -> np.ndarray:
    V = np.empty((r, N), dtype=np.uint32)
    lib().orc_test_vector(N, r, Q, t, t_out, _u(f), V)
    return V


def gadget_shift(Q: int, log2_B: int, l: int) -> int:
    return int(lib().orc_gadget_shift(Q, log2_B, l))


def gadget(Q: int, log2_B: int, l: int) -> np.ndarray:
    return np.array([lib().orc_gadget(Q, log2_B, l, u) for u in range(l)], dtype=np.uint64)


def decompose(x: int, Q: int, log2_B: int, l: int) -> np.ndarray:
    d = np.empty(l, dtype=np.int32)
    lib().orc_decompose(Q, log2_B, l, int(x), d)
    return d


def _keys(p) -> int:
    return 2 if getattr(p, "ternary", False) else 1


def keygen_bsk(p, draws) -> np.ndarray:
    """[n * K][2l][2][N]: key k of coordinate i at i K + k (K = 2 for a ternary secret)."""
    K = _keys(p)
    out = np.empty((p.n * K, 2 * p.l, 2, p.N), dtype=np.uint32)
    lib().orc_keygen_bsk(p.n, p.N, p.Q, p.log2_B, p.l, K, _i(draws["s"]), _u(draws["z"]),
                         _u(draws["bsk_a"]), _i(draws["bsk_e"]), out)
    return out


def keygen_ksk(p, draws) -> np.ndarray:
    out = np.empty((p.N, p.l_ks, p.B_ks, p.n + 1), dtype=np.uint32)
    lib().orc_keygen_ksk(p.n, p.N, p.Q, p.log2_Bks, p.l_ks, _i(draws["s"]), _u(draws["z"]),
                         _u(draws["ksk_a"]), _i(draws["ksk_e"]), out)
    return out


def encrypt(n: int, q: int, t: int, s, m, a, e) -> np.ndarray:
    m = _u(np.atleast_1d(m))
    ct = np.empty((m.size, n + 1), dtype=np.uint32)
    lib().orc_encrypt(n, q, t, _i(s), m, _u(a), _i(e), m.size, ct)
    return ct


def decrypt(n: int, q: int, t: int, s, ct) -> np.ndarray:
    ct = _u(ct).reshape(-1, n + 1)
    m = np.empty(ct.shape[0], dtype=np.uint32)
    lib().orc_decrypt(n, q, t, _i(s), ct, ct.shape[0], m)
    return m


def lwe_phase(n: int, q: int, s, ct) -> np.ndarray:
    ct = _u(ct).reshape(-1, n + 1)
    ph = np.empty(ct.shape[0], dtype=np.uint32)
    lib().orc_lwe_phase(n, q, _i(s), ct, ct.shape[0], ph)
    return ph


def external_product(rgsw, rlwe, Q: int, log2_B: int, l: int) -> np.ndarray:
    """g^{-1}(rlwe) * rgsw for rgsw (2l, 2, N) and rlwe (2, N) = (a, b)."""
    rgsw, rlwe = _u(rgsw), _u(rlwe)
    N = rlwe.shape[-1]
    out = np.empty((2, N), dtype=np.uint32)
    lib().orc_external_product(N, Q, log2_B, l, rgsw, rlwe, out)
    return out


def blind_rotate(p, r: int, bsk, V, ct_ms, steps=None) -> np.ndarray:
    acc = np.empty((r, 2, p.N), dtype=np.uint32)
    steps = p.n if steps is None else steps
    lib().orc_blind_rotate(p.n, p.N, p.Q, p.log2_B, p.l, r, _keys(p), _u(bsk), _u(V), _u(ct_ms), steps, acc)
    return acc


def sample_extract(rlwe, Q: int) -> np.ndarray:
    rlwe = _u(rlwe)
    N = rlwe.shape[-1]
    out = np.empty(N + 1, dtype=np.uint32)
    lib().orc_sample_extract(N, Q, rlwe, out)
    return out


def keyswitch(p, ksk, lwe_N) -> np.ndarray:
    out = np.empty(p.n + 1, dtype=np.uint32)
    lib().orc_keyswitch(p.n, p.N, p.Q, p.log2_Bks, p.l_ks, _u(ksk), _u(lwe_N), out)
    return out


def bootstrap(p, r: int, bsk, ksk, V, q_in: int, q_out: int, ct, intermediates=False):
    ct = _u(ct)
    out = np.empty(p.n + 1, dtype=np.uint32)
    acc = np.empty((r, 2, p.N), dtype=np.uint32) if intermediates else None
    ext = np.empty(p.N + 1, dtype=np.uint32) if intermediates else None
    ks = np.empty(p.n + 1, dtype=np.uint32) if intermediates else None
    lib().orc_bootstrap(p.n, p.N, p.Q, p.log2_B, p.l, p.log2_Bks, p.l_ks, r, _keys(p), _u(bsk), _u(ksk),
                        _u(V), q_in, q_out, ct, out, _ptr(acc), _ptr(ext), _ptr(ks))
    if intermediates:
        return out, acc, ext, ks
    return out


def bootstrap_many(p, r: int, bsk, ksk, V, q_in: int, q_out: int, cts) -> np.ndarray:
    cts = _u(cts).reshape(-1, p.n + 1)
    out = np.empty_like(cts)
    lib().orc_bootstrap_many(p.n, p.N, p.Q, p.log2_B, p.l, p.log2_Bks, p.l_ks, r, _keys(p), _u(bsk),
                             _u(ksk), _u(V), q_in, q_out, cts, cts.shape[0], out)
    return out


def general_tables(t: int, t_out: int, f):
    """(g, F): the two nega-cyclic tables on Z_2t for an arbitrary f: Z_t -> Z_t'."""
    g = np.empty(2 * t, dtype=np.uint32)
    F = np.empty(2 * t, dtype=np.uint32)
    lib().orc_general_tables(t, t_out, _u(f), g, F)
    return g, F


def bootstrap_general(p, r: int, bsk, ksk, Vg, VF, q: int, t: int, q_out: int, ct) -> np.ndarray:
    out = np.empty(p.n + 1, dtype=np.uint32)
    lib().orc_bootstrap_general(p.n, p.N, p.Q, p.log2_B, p.l, p.log2_Bks, p.l_ks, r, _keys(p), _u(bsk), _u(ksk),
                                _u(Vg), _u(VF), q, t, q_out, _u(ct), out)
    return out


class KeySet:
    """Keys the oracle builds for itself from the shared draws."""

    def __init__(self, p, draws):
        self.p = p
        self.s = _i(draws["s"])
        self.z = _u(draws["z"])
        self.bsk = keygen_bsk(p, draws)
        self.ksk = keygen_ksk(p, draws)

    def bootstrap(self, r, V, q_in, q_out, ct, intermediates=False):
        return bootstrap(self.p, r, self.bsk, self.ksk, V, q_in, q_out, ct, intermediates)


def bsk_bytes(n: int, N: int, l: int, word_bytes: int, keys_per_coord: int) -> int:
    """keys_per_coord RGSW keys per LWE coordinate, each 2l x 2 polys of N words
    (Sec. 5 item (1): 2n keys for a ternary secret, one per coordinate for binary)."""
    return keys_per_coord * n * 2 * l * 2 * N * word_bytes


def ksk_bytes(n: int, N: int, B_ks: int, l_ks: int, word_bytes: int) -> int:
    """LWE_{n,Q}(v z_i B_ks^j) for v < B_ks, i < N, j < l_ks (Sec. 5 item (2))."""
    return N * B_ks * l_ks * (n + 1) * word_bytes


# ---------------------------------------------------------------- wide ring modulus
# The same steps with the accumulator and the bootstrapping key modulo Q_w =
# p.Q_ring (up to 2^62, one uint64 per coefficient); the key switch stays at p.Q.


def _w(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


def w_poly_mul(a, b, Q: int) -> np.ndarray:
    a, b = _w(a), _w(b)
    out = np.empty_like(a)
    lib().orc_w_poly_mul(a.size, Q, a, b, out)
    return out


def w_rotate(v, c: int, Q: int) -> np.ndarray:
    v = _w(v)
    r, N = v.shape
    out = np.empty_like(v)
    lib().orc_w_rotate(N, r, Q, c % (2 * N * r), v, out)
    return out


def w_test_vector(N: int, r: int, Q: int, t: int, t_out: int, f) -> np.ndarray:
    V = np.empty((r, N), dtype=np.uint64)
    lib().orc_w_test_vector(N, r, Q, t, t_out, _u(f), V)
    return V


def w_gadget_shift(Q: int, log2_B: int, l: int) -> int:
    return int(lib().orc_w_gadget_shift(Q, log2_B, l))


def w_gadget(Q: int, log2_B: int, l: int) -> list:
    return [int(lib().orc_w_gadget(Q, log2_B, l, u)) for u in range(l)]


def w_decompose(x: int, Q: int, log2_B: int, l: int) -> np.ndarray:
    d = np.empty(l, dtype=np.int64)
    lib().orc_w_decompose(Q, log2_B, l, int(x), d)
    return d


def w_keygen_bsk(p, draws) -> np.ndarray:
    """[n * K][2l][2][N] uint64 at p.Q_ring."""
    K = _keys(p)
    out = np.empty((p.n * K, 2 * p.l, 2, p.N), dtype=np.uint64)
    lib().orc_w_keygen_bsk(p.n, p.N, p.Q_ring, p.log2_B, p.l, K, _i(draws["s"]), _u(draws["z"]),
                           _w(draws["bsk_a"]), _i(draws["bsk_e"]), out)
    return out


def w_external_product(rgsw, rlwe, Q: int, log2_B: int, l: int) -> np.ndarray:
    rgsw, rlwe = _w(rgsw), _w(rlwe)
    N = rlwe.shape[-1]
    out = np.empty((2, N), dtype=np.uint64)
    lib().orc_w_external_product(N, Q, log2_B, l, rgsw, rlwe, out)
    return out


def w_blind_rotate(p, r: int, bsk, V, ct_ms, steps=None) -> np.ndarray:
    acc = np.empty((r, 2, p.N), dtype=np.uint64)
    steps = p.n if steps is None else steps
    lib().orc_w_blind_rotate(p.n, p.N, p.Q_ring, p.log2_B, p.l, r, _keys(p), _w(bsk), _w(V), _u(ct_ms),
                             steps, acc)
    return acc


def w_modswitch(x, Q_from: int, q_to: int) -> np.ndarray:
    x = _w(np.atleast_1d(x))
    return np.array([lib().orc_w_modswitch(int(v), Q_from, q_to) for v in x.reshape(-1)],
                    dtype=np.uint64).reshape(x.shape)


def w_sample_extract(rlwe, Q: int) -> np.ndarray:
    rlwe = _w(rlwe)
    N = rlwe.shape[-1]
    out = np.empty(N + 1, dtype=np.uint64)
    lib().orc_w_sample_extract(N, Q, rlwe, out)
    return out


def w_bootstrap(p, r: int, bsk, ksk, V, q_in: int, q_out: int, ct, ext_out=False):
    """One ciphertext; with ext_out also the extracted sample after the switch to p.Q."""
    out = np.empty(p.n + 1, dtype=np.uint32)
    ext = np.empty(p.N + 1, dtype=np.uint32) if ext_out else None
    lib().orc_w_bootstrap(p.n, p.N, p.Q_ring, p.log2_B, p.l, p.Q, p.log2_Bks, p.l_ks, r, _keys(p), _w(bsk),
                          _u(ksk), _w(V), q_in, q_out, _u(ct), out, _ptr(ext))
    return (out, ext) if ext_out else out


def w_bootstrap_many(p, r: int, bsk, ksk, V, q_in: int, q_out: int, cts) -> np.ndarray:
    cts = _u(cts).reshape(-1, p.n + 1)
    out = np.empty_like(cts)
    lib().orc_w_bootstrap_many(p.n, p.N, p.Q_ring, p.log2_B, p.l, p.Q, p.log2_Bks, p.l_ks, r, _keys(p),
                               _w(bsk), _u(ksk), _w(V), q_in, q_out, cts, cts.shape[0], out)
    return out


def w_bootstrap_general(p, r: int, bsk, ksk, Vg, VF, q: int, t: int, q_out: int, cts) -> np.ndarray:
    """f(m) from Enc_{2t}(m + b t) by two bootstraps at the wide ring modulus."""
    cts = _u(cts).reshape(-1, p.n + 1)
    out = np.empty_like(cts)
    lib().orc_w_bootstrap_general(p.n, p.N, p.Q_ring, p.log2_B, p.l, p.Q, p.log2_Bks, p.l_ks, r, _keys(p),
                                  _w(bsk), _u(ksk), _w(Vg), _w(VF), q, t, q_out, cts, cts.shape[0], out)
    return out


class KeySetWide:
    """Keys at the wide ring modulus p.Q_ring (BSK) and at p.Q (KSK), built from the shared draws."""

    def __init__(self, p, draws):
        self.p = p
        self.s = _i(draws["s"])
        self.z = _u(draws["z"])
        self.bsk = w_keygen_bsk(p, draws)
        self.ksk = keygen_ksk(p, draws)
