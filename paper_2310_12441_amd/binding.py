"""ctypes binding of ``libmmpm.so`` (include/mmpm.h): argument marshalling only.

Every computation happens in the library.  Host arrays are numpy uint32/int32
arrays; device buffers are torch tensors on the GPU (their data pointers are
passed with MM_DEVICE_PTRS, on torch's current stream).  If the library is not
built this module raises at import time: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libmmpm.so")

MM_OK, MM_EINVAL, MM_ENOMEM, MM_EDEVICE, MM_EBUSY, MM_EAGAIN, MM_ESTATE = 0, -1, -2, -3, -4, -5, -6
MM_DEVICE_PTRS = 1
MM_PLAIN = 2

SYMBOLS = [
    "mm_keygen", "mm_free", "mm_last_error", "mm_get_params", "mm_export_bsk", "mm_export_ksk",
    "mm_device_init", "mm_table_create", "mm_table_create_general", "mm_table_info", "mm_table_export", "mm_encrypt", "mm_decrypt",
    "mm_bootstrap", "mm_modswitch", "mm_blind_rotate", "mm_external_product", "mm_sample_extract",
    "mm_keyswitch", "mm_keyswitch_noalloc", "mm_negacyclic_mul", "mm_set_timing", "mm_last_timing", "mm_autotune",
    "mm_schedule_count", "mm_set_schedule", "mm_schedule_describe", "mm_server_start", "mm_submit", "mm_poll",
    "mm_server_stats", "mm_server_stop", "mm_server_replay", "mm_server_set_admission", "mm_server_refused",
]


class MMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [(f, C.c_uint32) for f in ("n", "N", "Q", "log2_B", "l", "log2_Bks", "l_ks", "ternary", "Q2")]


class KeyDraws(C.Structure):
    _fields_ = [("s", C.c_void_p), ("z", C.c_void_p), ("bsk_a", C.c_void_p), ("bsk_e", C.c_void_p),
                ("ksk_a", C.c_void_p), ("ksk_e", C.c_void_p), ("bsk_a_wide", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2310_12441_amd.build.build() first")
    L = C.CDLL(LIB_PATH)
    vp, u32, i32, sz, u64 = C.c_void_p, C.c_uint32, C.c_int, C.c_size_t, C.c_uint64
    sig = {
        "mm_keygen": (i32, [C.POINTER(Params), C.POINTER(KeyDraws), C.POINTER(vp)]),
        "mm_free": (None, [vp]),
        "mm_last_error": (C.c_char_p, [vp]),
        "mm_get_params": (i32, [vp, C.POINTER(Params)]),
        "mm_export_bsk": (i32, [vp, vp, sz]),
        "mm_export_ksk": (i32, [vp, vp, sz]),
        "mm_device_init": (i32, [vp, i32]),
        "mm_table_create": (i32, [vp, u32, u32, u32, u32, vp, C.POINTER(i32)]),
        "mm_table_create_general": (i32, [vp, u32, u32, u32, u32, vp, C.POINTER(i32)]),
        "mm_table_info": (i32, [vp, i32, C.POINTER(u32), C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]),
        "mm_table_export": (i32, [vp, i32, vp, sz]),
        "mm_encrypt": (i32, [vp, u32, u32, vp, sz, vp, vp, vp]),
        "mm_decrypt": (i32, [vp, u32, u32, vp, sz, vp]),
        "mm_bootstrap": (i32, [vp, vp, vp, sz, vp, u32, u32, vp]),
        "mm_modswitch": (i32, [vp, vp, sz, u32, u32, vp, u32, vp]),
        "mm_blind_rotate": (i32, [vp, vp, vp, sz, u32, vp, u32, vp]),
        "mm_external_product": (i32, [vp, u32, vp, sz, vp, u32, vp]),
        "mm_sample_extract": (i32, [vp, vp, sz, vp, u32, vp]),
        "mm_keyswitch": (i32, [vp, vp, sz, vp, u32, vp]),
        "mm_negacyclic_mul": (i32, [vp, vp, vp, sz, vp, u32, vp]),
        "mm_keyswitch_noalloc": (i32, [vp, vp, sz, vp, vp]),
        "mm_set_timing": (i32, [vp, i32]),
        "mm_last_timing": (i32, [vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
        "mm_autotune": (i32, [vp, vp, vp, sz, C.POINTER(i32)]),
        "mm_schedule_count": (i32, [vp, vp, sz, C.POINTER(i32)]),
        "mm_set_schedule": (i32, [vp, vp, sz, i32]),
        "mm_schedule_describe": (i32, [vp, vp, sz, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32),
                                       C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]),
        "mm_server_start": (i32, [vp, sz, u32, C.POINTER(vp)]),
        "mm_submit": (i32, [vp, i32, vp, C.POINTER(u64)]),
        "mm_poll": (i32, [vp, u64, vp]),
        "mm_server_stats": (i32, [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(u64)]),
        "mm_server_stop": (i32, [vp]),
        "mm_server_replay": (i32, [vp, vp, vp, vp, sz, vp, vp]),
        "mm_server_set_admission": (i32, [vp, C.c_double]),
        "mm_server_refused": (i32, [vp, C.POINTER(C.c_uint64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _is_dev(x) -> bool:
    return hasattr(x, "is_cuda") and x.is_cuda


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Buf:
    """A host (numpy) or device (torch) uint32 buffer with its pointer."""

    def __init__(self, x, words=None, out=False):
        self.dev = _is_dev(x)
        if self.dev:
            import torch
            assert x.dtype in (torch.int32, torch.uint32) and x.is_contiguous(), "device buffers are contiguous int32"
            self.arr = x
            self.ptr = C.c_void_p(x.data_ptr())
        else:
            self.arr = x if out else _u32(x)
            assert self.arr.dtype == np.uint32 and self.arr.flags.c_contiguous
            self.ptr = self.arr.ctypes.data_as(C.c_void_p)
        n = self.arr.numel() if self.dev else self.arr.size
        if words is not None:
            assert n >= words, f"buffer holds {n} words, needs {words}"


class Context:
    """One key set (mm_ctx)."""

    def __init__(self, params, draws):
        self.wide = bool(getattr(params, "Q2", 0))
        p = Params(params.n, params.N, params.Q, params.log2_B, params.l, params.log2_Bks, params.l_ks,
                   1 if getattr(params, "ternary", False) else 0, getattr(params, "Q2", 0))
        self.params = params
        self._lib = lib  # held so that close() still works while the interpreter shuts down
        keep = {}
        for k, v in draws.items():
            if k == "bsk_a" and self.wide:
                keep["bsk_a_wide"] = np.ascontiguousarray(v, dtype=np.uint64)
            else:
                keep[k] = _i32(v) if k.endswith("_e") or k == "s" else _u32(v)
        self._keep = keep
        ptr = lambda k: keep[k].ctypes.data_as(C.c_void_p) if k in keep else None
        d = KeyDraws(*(ptr(k) for k in ("s", "z", "bsk_a", "bsk_e", "ksk_a", "ksk_e", "bsk_a_wide")))
        h = C.c_void_p()
        rc = lib.mm_keygen(C.byref(p), C.byref(d), C.byref(h))
        self._keep = None
        if rc != MM_OK:
            raise MMError(rc, lib.mm_last_error(None).decode())
        self.h = h

    def close(self):
        h = getattr(self, "h", None)
        if h:
            self.h = None
            self._lib.mm_free(h)

    def __del__(self):
        self.close()

    def _check(self, rc):
        if rc != MM_OK:
            raise MMError(rc, lib.mm_last_error(self.h).decode())

    # ---- keys, tables, host-side encryption
    def export_bsk(self):
        p = self.params
        K = 2 if getattr(p, "ternary", False) else 1
        out = np.empty((p.n * K, 2 * p.l, 2, p.N), dtype=np.uint64 if self.wide else np.uint32)
        self._check(lib.mm_export_bsk(self.h, out.ctypes.data_as(C.c_void_p), out.nbytes // 4))
        return out

    def export_ksk(self):
        p = self.params
        out = np.empty((p.N, p.l_ks, p.B_ks, p.n + 1), dtype=np.uint32)
        self._check(lib.mm_export_ksk(self.h, out.ctypes.data_as(C.c_void_p), out.size))
        return out

    def device_init(self, device: int = 0):
        self._check(lib.mm_device_init(self.h, device))

    def table_create(self, t, t_out, r, f, q_in=0) -> int:
        f = _u32(f)
        tid = C.c_int()
        self._check(lib.mm_table_create(self.h, t, t_out, r, q_in, f.ctypes.data_as(C.c_void_p), C.byref(tid)))
        return tid.value

    def table_create_general(self, t, t_out, r, f, q_in=0) -> int:
        f = _u32(f)
        tid = C.c_int()
        self._check(lib.mm_table_create_general(self.h, t, t_out, r, q_in, f.ctypes.data_as(C.c_void_p),
                                                C.byref(tid)))
        return tid.value

    def table_info(self, tid):
        v = [C.c_uint32() for _ in range(4)]
        self._check(lib.mm_table_info(self.h, tid, *(C.byref(x) for x in v)))
        return tuple(x.value for x in v)  # t, t_out, r, q_in

    def table_export(self, tid):
        r = self.table_info(tid)[2]
        V = np.empty((r, self.params.N), dtype=np.uint64 if self.wide else np.uint32)
        self._check(lib.mm_table_export(self.h, tid, V.ctypes.data_as(C.c_void_p), V.nbytes // 4))
        return V

    def encrypt(self, q, t, m, mask, err):
        m = _u32(np.atleast_1d(m))
        mask, err = _u32(mask), _i32(err)
        ct = np.empty((m.size, self.params.n + 1), dtype=np.uint32)
        self._check(lib.mm_encrypt(self.h, q, t, m.ctypes.data_as(C.c_void_p), m.size,
                                   mask.ctypes.data_as(C.c_void_p), err.ctypes.data_as(C.c_void_p),
                                   ct.ctypes.data_as(C.c_void_p)))
        return ct

    def decrypt(self, q, t, ct):
        ct = _u32(ct).reshape(-1, self.params.n + 1)
        m = np.empty(ct.shape[0], dtype=np.uint32)
        self._check(lib.mm_decrypt(self.h, q, t, ct.ctypes.data_as(C.c_void_p), ct.shape[0],
                                   m.ctypes.data_as(C.c_void_p)))
        return m

    # ---- the hot path
    def _io(self, inp, out_shape, out=None):
        """Input/output buffers: device tensors pass through; host arrays are numpy."""
        i = Buf(inp)
        if i.dev:
            import torch
            if out is None:
                out = torch.empty(out_shape, dtype=torch.int32, device=inp.device)
            o = Buf(out, out=True)
            return i, o, MM_DEVICE_PTRS, _stream()
        if out is None:
            out = np.empty(out_shape, dtype=np.uint32)
        return i, Buf(out, out=True), 0, None

    def bootstrap(self, table_ids, ct, q_out=0, plain=False, out=None):
        ids = _i32(np.atleast_1d(table_ids))
        W = self.params.n + 1
        cnt = ids.size
        i, o, flags, st = self._io(ct, (cnt, W), out)
        if plain:
            flags |= MM_PLAIN
        self._check(lib.mm_bootstrap(self.h, ids.ctypes.data_as(C.c_void_p), i.ptr, cnt, o.ptr, q_out, flags, st))
        return o.arr

    def modswitch(self, x, q_from, q_to, out=None):
        n = x.numel() if _is_dev(x) else np.asarray(x).size
        shape = tuple(x.shape)
        i, o, flags, st = self._io(x, shape, out)
        self._check(lib.mm_modswitch(self.h, i.ptr, n, q_from, q_to, o.ptr, flags, st))
        return o.arr

    def blind_rotate(self, table_ids, ct, steps=None, out=None):
        ids = _i32(np.atleast_1d(table_ids))
        steps = self.params.n if steps is None else steps
        words = sum(self.table_info(int(t))[2] * 2 * self.params.N for t in ids)
        if self.wide:
            words *= 2  # uint64 entries
        i, o, flags, st = self._io(ct, (words,), out)
        self._check(lib.mm_blind_rotate(self.h, ids.ctypes.data_as(C.c_void_p), i.ptr, ids.size, steps, o.ptr,
                                        flags, st))
        if self.wide and not o.dev:
            return o.arr.view(np.uint64)
        return o.arr

    def external_product(self, i_key, rlwe, out=None):
        N = self.params.N
        cnt = (rlwe.numel() if _is_dev(rlwe) else np.asarray(rlwe).size) // (2 * N)
        i, o, flags, st = self._io(rlwe, (cnt, 2, N), out)
        self._check(lib.mm_external_product(self.h, i_key, i.ptr, cnt, o.ptr, flags, st))
        return o.arr

    def sample_extract(self, rlwe, out=None):
        N = self.params.N
        cnt = (rlwe.numel() if _is_dev(rlwe) else np.asarray(rlwe).size) // (2 * N)
        i, o, flags, st = self._io(rlwe, (cnt, N + 1), out)
        self._check(lib.mm_sample_extract(self.h, i.ptr, cnt, o.ptr, flags, st))
        return o.arr

    def keyswitch(self, lwe_N, out=None):
        N = self.params.N
        cnt = (lwe_N.numel() if _is_dev(lwe_N) else np.asarray(lwe_N).size) // (N + 1)
        i, o, flags, st = self._io(lwe_N, (cnt, self.params.n + 1), out)
        self._check(lib.mm_keyswitch(self.h, i.ptr, cnt, o.ptr, flags, st))
        return o.arr

    def keyswitch_noalloc(self, lwe_N, out):
        """mm_keyswitch_noalloc on device tensors (int32 views of the words):
        lwe_N [count][N+1], out [count][n+1]; asynchronous on torch's current
        stream."""
        assert _is_dev(lwe_N) and _is_dev(out), "mm_keyswitch_noalloc takes device buffers"
        N, W = self.params.N, self.params.n + 1
        cnt = lwe_N.numel() // (N + 1)
        i, o = Buf(lwe_N, cnt * (N + 1)), Buf(out, cnt * W)
        self._check(lib.mm_keyswitch_noalloc(self.h, i.ptr, cnt, o.ptr, _stream()))
        return out

    def negacyclic_mul(self, a, b, out=None):
        N = self.params.N
        cnt = (a.numel() if _is_dev(a) else np.asarray(a).size) // N
        i, o, flags, st = self._io(a, (cnt, N), out)
        bb = Buf(b)
        self._check(lib.mm_negacyclic_mul(self.h, i.ptr, bb.ptr, cnt, o.ptr, flags, st))
        return o.arr

    def set_timing(self, enable: bool):
        self._check(lib.mm_set_timing(self.h, 1 if enable else 0))

    def last_timing(self):
        """(blind-rotation ms, key-switch ms) of the last batched bootstrap."""
        a, b = C.c_float(), C.c_float()
        self._check(lib.mm_last_timing(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def autotune(self, table_ids, ct) -> int:
        ids = _i32(np.atleast_1d(table_ids))
        ct = _u32(ct)
        ch = C.c_int()
        self._check(lib.mm_autotune(self.h, ids.ctypes.data_as(C.c_void_p), ct.ctypes.data_as(C.c_void_p), ids.size,
                                    C.byref(ch)))
        return ch.value

    def schedule_count(self, table_ids) -> int:
        ids = _i32(np.atleast_1d(table_ids))
        n = C.c_int()
        self._check(lib.mm_schedule_count(self.h, ids.ctypes.data_as(C.c_void_p), ids.size, C.byref(n)))
        return n.value

    def set_schedule(self, table_ids, choice: int):
        ids = _i32(np.atleast_1d(table_ids))
        self._check(lib.mm_set_schedule(self.h, ids.ctypes.data_as(C.c_void_p), ids.size, choice))

    def schedule_describe(self, table_ids, choice: int = -1):
        """(waves per blind-rotation workgroup (0: the global-accumulator path), key-switch ciphertexts per wave, key-switch splits,
        waves per ring component, key-switch kernel (0 i-split, 1 columns in lanes, 2 one ciphertext
        per lane), NTT schedule)."""
        ids = _i32(np.atleast_1d(table_ids))
        v = [C.c_int() for _ in range(6)]
        self._check(lib.mm_schedule_describe(self.h, ids.ctypes.data_as(C.c_void_p), ids.size, choice,
                                             *(C.byref(x) for x in v)))
        return tuple(x.value for x in v)

    # ---- serving
    def server_start(self, hbm_budget_bytes: int, chunk_steps: int = 32) -> "Server":
        h = C.c_void_p()
        self._check(lib.mm_server_start(self.h, hbm_budget_bytes, chunk_steps, C.byref(h)))
        return Server(self, h)


class Server:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def _check(self, rc):
        if rc not in (MM_OK,):
            raise MMError(rc, lib.mm_last_error(self.ctx.h).decode())

    def submit(self, table_id: int, ct) -> int:
        ct = _u32(ct)
        t = C.c_uint64()
        rc = lib.mm_submit(self.h, table_id, ct.ctypes.data_as(C.c_void_p), C.byref(t))
        if rc == MM_EBUSY:
            return -1
        self._check(rc)
        return t.value

    def poll(self, ticket: int):
        out = np.empty(self.ctx.params.n + 1, dtype=np.uint32)
        rc = lib.mm_poll(self.h, ticket, out.ctypes.data_as(C.c_void_p))
        if rc == MM_EAGAIN:
            return None
        self._check(rc)
        return out

    def stats(self):
        p50, p99, bps = C.c_double(), C.c_double(), C.c_double()
        done = C.c_uint64()
        self._check(lib.mm_server_stats(self.h, C.byref(p50), C.byref(p99), C.byref(bps), C.byref(done)))
        return {"p50_ms": p50.value, "p99_ms": p99.value, "boots_per_s": bps.value, "completed": done.value}

    def set_admission(self, max_latency_ms: float):
        """Refuse requests whose expected latency (queued and in-flight requests over the recent
        completion rate) exceeds max_latency_ms (0: off)."""
        self._check(lib.mm_server_set_admission(self.h, float(max_latency_ms)))

    def refused(self) -> int:
        n = C.c_uint64()
        self._check(lib.mm_server_refused(self.h, C.byref(n)))
        return n.value

    def replay(self, table_ids, cts, arrival_ns):
        ids = _i32(table_ids)
        cts = _u32(cts)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        out = np.empty_like(cts)
        lat = np.empty(ids.size, dtype=np.float64)
        self._check(lib.mm_server_replay(self.h, ids.ctypes.data_as(C.c_void_p), cts.ctypes.data_as(C.c_void_p),
                                         arr.ctypes.data_as(C.c_void_p), ids.size, out.ctypes.data_as(C.c_void_p),
                                         lat.ctypes.data_as(C.c_void_p)))
        return out, lat

    def stop(self):
        if self.h:
            self._check(lib.mm_server_stop(self.h))
            self.h = None
