"""ctypes binding of libpmk.so (include/pmk.h): argument marshalling only.

Every function of the C ABI appears here under the same name.  Device buffers
are passed as torch CUDA tensors (or raw integer device addresses); streams as
torch streams, raw hipStream_t integers, or None for the current torch stream.
All arithmetic happens in the library's HIP kernels; if libpmk.so has not been
built this module raises on first use instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmk.so")

PMK_OK = 0
PMK_EINVAL = -1
PMK_EKEY = -2
PMK_ERANGE = -3
PMK_ESIZE = -4
PMK_ENOMEM = -5
PMK_EDEVICE = -6
PMK_EBUSY = -7
PMK_EUNSUPPORTED = -8
PMK_EBLIND = -9

PMK_KERNEL_PACK = 0
PMK_KERNEL_ENCRYPT = 1
PMK_KERNEL_CRT_HALVES = 2
PMK_KERNEL_GARNER = 3
PMK_KERNEL_UNPACK = 4
PMK_KERNEL_BATCH = 5
KERNEL_NAMES = {0: "pack", 1: "encrypt", 2: "crt_halves", 3: "garner", 4: "unpack", 5: "batch"}

PMK_DEC_CHUNKS = 0
PMK_DEC_BLOCKS = 1

STATUS_NAMES = {0: "PMK_OK", -1: "PMK_EINVAL", -2: "PMK_EKEY", -3: "PMK_ERANGE", -4: "PMK_ESIZE",
                -5: "PMK_ENOMEM", -6: "PMK_EDEVICE", -7: "PMK_EBUSY", -8: "PMK_EUNSUPPORTED",
                -9: "PMK_EBLIND"}

U32P = C.POINTER(C.c_uint32)


class PmkError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class pmk_key(C.Structure):
    _fields_ = [("bits", C.c_uint32), ("n", U32P), ("n0inv", C.c_uint32), ("rr", U32P),
                ("e", U32P), ("e_limbs", C.c_uint32), ("p", U32P), ("q", U32P), ("dp", U32P),
                ("dq", U32P), ("qinv", U32P)]


class pmk_key_mp(C.Structure):
    _fields_ = [("bits", C.c_uint32), ("nprimes", C.c_uint32), ("n", U32P), ("primes", U32P), ("d", U32P)]


class pmk_server_cfg(C.Structure):
    _fields_ = [("staging_bytes", C.c_uint64), ("round_chunks", C.c_uint64), ("pipeline_depth", C.c_uint32)]


class pmk_request(C.Structure):
    _fields_ = [("op", C.c_int), ("in_", C.c_void_p), ("out", C.c_void_p), ("out_cap", C.c_uint64),
                ("msg_len", C.c_uint64), ("key_map", U32P), ("nchunks", C.c_uint64)]


class pmk_ticket_info(C.Structure):
    _fields_ = [("state", C.c_int), ("status", C.c_int), ("t_submit_ns", C.c_uint64),
                ("t_admit_ns", C.c_uint64), ("t_done_ns", C.c_uint64)]


class pmk_server_stats(C.Structure):
    _fields_ = [("requests_submitted", C.c_uint64), ("requests_done", C.c_uint64), ("rounds", C.c_uint64),
                ("chunks", C.c_uint64), ("busy_ns", C.c_uint64), ("queued", C.c_uint64)]


PMK_OP_ENCRYPT = 0
PMK_OP_DECRYPT = 1
PMK_REQ_QUEUED = 0
PMK_REQ_ADMITTED = 1
PMK_REQ_DONE = 2

_lib = None


def load_library(path: Optional[str] = None) -> C.CDLL:
    """Load libpmk.so (raises RuntimeError when it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build the HIP library first "
                           "(python -m paper_2111_11924_amd.build)")
    L = C.CDLL(p)
    vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
    sig = {
        "pmk_create": (C.c_int, [C.c_int, C.POINTER(vp)]),
        "pmk_destroy": (None, [vp]),
        "pmk_last_error": (C.c_char_p, [vp]),
        "pmk_keys_load": (C.c_int, [vp, C.POINTER(pmk_key), u32]),
        "pmk_key_check": (C.c_int, [C.POINTER(pmk_key), C.c_char_p, C.c_size_t]),
        "pmk_plan_validate": (C.c_int, [U32P, u32, U32P, u64, u64, C.POINTER(u64)]),
        "pmk_key_count": (u32, [vp]),
        "pmk_key_bits": (u32, [vp, u32]),
        "pmk_plan_create": (C.c_int, [vp, U32P, u64, u64, C.POINTER(vp), C.POINTER(u64)]),
        "pmk_plan_destroy": (None, [vp]),
        "pmk_plan_info": (C.c_int, [vp, C.POINTER(u64), C.POINTER(u64), C.POINTER(u64)]),
        "pmk_encrypt_plan": (C.c_int, [vp, vp, vp, vp]),
        "pmk_decrypt_plan": (C.c_int, [vp, vp, vp, vp]),
        "pmk_encrypt_blinded_plan": (C.c_int, [vp, vp, vp, vp, vp, vp]),
        "pmk_decrypt_blinded_plan": (C.c_int, [vp, vp, vp, vp, vp]),
        "pmk_encrypt_batch": (C.c_int, [vp, vp, vp, vp]),
        "pmk_decrypt_batch": (C.c_int, [vp, vp, vp, vp]),
        "pmk_set_window": (C.c_int, [vp, u32, C.c_int]),
        "pmk_get_window": (C.c_int, [vp, u32]),
        "pmk_set_grid_limit": (C.c_int, [vp, u32]),
        "pmk_set_lanes": (C.c_int, [vp, u32, C.c_int, C.c_int]),
        "pmk_get_lanes": (C.c_int, [vp, u32, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
        "pmk_autotune": (C.c_int, [vp, C.c_char_p, C.c_int]),
        "pmk_sieve": (C.c_int, [vp, u32, vp, u32, vp, vp]),
        "pmk_miller_rabin": (C.c_int, [vp, u32, vp, u32, vp, u32, vp, vp]),
        "pmk_server_start": (C.c_int, [vp, C.POINTER(pmk_server_cfg)]),
        "pmk_submit": (C.c_int, [vp, C.POINTER(pmk_request), C.POINTER(u64)]),
        "pmk_poll": (C.c_int, [vp, u64, C.POINTER(pmk_ticket_info)]),
        "pmk_wait": (C.c_int, [vp, u64, C.POINTER(pmk_ticket_info)]),
        "pmk_server_stats_get": (C.c_int, [vp, C.POINTER(pmk_server_stats)]),
        "pmk_server_stop": (C.c_int, [vp]),
        "pmk_plan_check": (C.c_int, [vp, vp]),
        "pmk_plan_set_decrypt_output": (C.c_int, [vp, C.c_int]),
        "pmk_plan_profile": (C.c_int, [vp, C.c_int]),
        "pmk_plan_kernel_time": (C.c_int, [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(u64)]),
        "pmk_encrypt": (C.c_int, [vp, vp, u64, U32P, u64, vp, u64, vp]),
        "pmk_decrypt": (C.c_int, [vp, vp, u64, U32P, u64, vp, u64, vp]),
        "pmk_encrypt_host": (C.c_int, [vp, vp, vp, u32]),
        "pmk_decrypt_noalloc": (C.c_int, [vp, vp, u64, U32P, u64, vp, u64, vp]),
        "pmk_decrypt_host": (C.c_int, [vp, vp, vp, u32]),
        "pmk_mp_key_check": (C.c_int, [C.POINTER(pmk_key_mp), C.c_char_p, C.c_size_t]),
        "pmk_mp_keys_load": (C.c_int, [vp, C.POINTER(pmk_key_mp), u32]),
        "pmk_mp_key_count": (u32, [vp]),
        "pmk_mp_decrypt": (C.c_int, [vp, vp, u64, U32P, u64, vp, u64, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = L
    return L


# ---------- marshalling helpers ------------------------------------------------------------

def _limbs(x: int, n: int) -> np.ndarray:
    if x < 0 or x.bit_length() > 32 * n:
        raise ValueError("value does not fit its field")
    return np.frombuffer(int(x).to_bytes(4 * n, "little"), dtype=np.uint32).copy()


class KeyArray:
    """pmk_key structs for a list of key objects with int fields
    (bits, n, n0inv, rr, e, p, q, dp, dq, qinv); keeps the limb arrays alive."""

    def __init__(self, keys: Sequence):
        self.count = len(keys)
        self.arr = (pmk_key * max(1, self.count))()
        self._keep: List[np.ndarray] = []
        for i, k in enumerate(keys):
            bits = int(k.bits)
            s, sh = bits // 32, bits // 64
            el = 1 if int(k.e) < (1 << 32) else 2
            fields = {"n": _limbs(k.n, s), "rr": _limbs(k.rr, s), "e": _limbs(k.e, el),
                      "p": _limbs(k.p, sh), "q": _limbs(k.q, sh), "dp": _limbs(k.dp, sh),
                      "dq": _limbs(k.dq, sh), "qinv": _limbs(k.qinv, sh)}
            st = self.arr[i]
            st.bits = bits
            st.n0inv = int(k.n0inv)
            st.e_limbs = el
            for f, a in fields.items():
                self._keep.append(a)
                setattr(st, f, a.ctypes.data_as(U32P))

    def ptr(self):
        return self.arr


class MpKeyArray:
    """pmk_key_mp structs for key objects with int fields bits, n and lists
    primes, exps (d_i = d mod (p_i - 1)); keeps the limb arrays alive."""

    def __init__(self, keys: Sequence):
        self.count = len(keys)
        self.arr = (pmk_key_mp * max(1, self.count))()
        self._keep: List[np.ndarray] = []
        for i, k in enumerate(keys):
            bits = int(k.bits)
            primes = np.concatenate([_limbs(int(p), 32) for p in k.primes]) if len(k.primes) else _limbs(0, 1)
            exps = np.concatenate([_limbs(int(d), 32) for d in k.exps]) if len(k.exps) else _limbs(0, 1)
            n = _limbs(int(k.n), bits // 32)
            st = self.arr[i]
            st.bits = bits
            st.nprimes = len(k.primes)
            for f, a in (("n", n), ("primes", primes), ("d", exps)):
                self._keep.append(a)
                setattr(st, f, a.ctypes.data_as(U32P))

    def ptr(self):
        return self.arr


def _map_array(key_map) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(key_map, dtype=np.uint32))


def _dev_ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(s) -> Optional[int]:
    if s is None:
        import torch

        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(s, int):
        return s
    return int(s.cuda_stream)


def _check(rc: int, ctx=None):
    if rc != PMK_OK:
        msg = pmk_last_error(ctx) if ctx else ""
        raise PmkError(rc, msg)


# ---------- the C ABI, one function each -------------------------------------------------

def pmk_create(device: int = 0) -> int:
    h = C.c_void_p()
    _check(load_library().pmk_create(int(device), C.byref(h)))
    return h.value


def pmk_destroy(ctx: int) -> None:
    load_library().pmk_destroy(ctx)


def pmk_last_error(ctx: int) -> str:
    r = load_library().pmk_last_error(ctx)
    return r.decode() if r else ""


def pmk_keys_load(ctx: int, keys: Sequence) -> None:
    ka = keys if isinstance(keys, KeyArray) else KeyArray(keys)
    _check(load_library().pmk_keys_load(ctx, ka.ptr(), ka.count), ctx)


def pmk_key_check(key) -> Tuple[int, str]:
    ka = KeyArray([key])
    buf = C.create_string_buffer(256)
    rc = load_library().pmk_key_check(ka.ptr(), buf, 256)
    return rc, buf.value.decode()


def pmk_plan_validate(key_bits: Sequence[int], key_map, msg_len: int) -> Tuple[int, int]:
    kb = np.ascontiguousarray(np.asarray(key_bits, dtype=np.uint32))
    km = _map_array(key_map)
    out = C.c_uint64(0)
    rc = load_library().pmk_plan_validate(kb.ctypes.data_as(U32P), len(kb), km.ctypes.data_as(U32P),
                                          len(km), int(msg_len), C.byref(out))
    return rc, out.value


def pmk_key_count(ctx: int) -> int:
    return load_library().pmk_key_count(ctx)


def pmk_key_bits(ctx: int, index: int) -> int:
    return load_library().pmk_key_bits(ctx, index)


def pmk_plan_create(ctx: int, key_map, msg_len: int) -> Tuple[int, int]:
    km = _map_array(key_map)
    h = C.c_void_p()
    ct = C.c_uint64(0)
    _check(load_library().pmk_plan_create(ctx, km.ctypes.data_as(U32P), len(km), int(msg_len),
                                          C.byref(h), C.byref(ct)), ctx)
    return h.value, ct.value


def pmk_plan_destroy(plan: int) -> None:
    load_library().pmk_plan_destroy(plan)


def pmk_plan_info(plan: int) -> Tuple[int, int, int]:
    a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
    _check(load_library().pmk_plan_info(plan, C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def pmk_encrypt_plan(plan: int, d_msg, d_ct, stream=None, ctx: Optional[int] = None) -> None:
    _check(load_library().pmk_encrypt_plan(plan, _dev_ptr(d_msg), _dev_ptr(d_ct), _stream(stream)), ctx)


def pmk_decrypt_plan(plan: int, d_ct, d_msg, stream=None, ctx: Optional[int] = None) -> None:
    _check(load_library().pmk_decrypt_plan(plan, _dev_ptr(d_ct), _dev_ptr(d_msg), _stream(stream)), ctx)


def pmk_encrypt_blinded_plan(plan: int, d_msg, d_r, d_ct_star, d_ct_r, stream=None, ctx: Optional[int] = None) -> None:
    _check(load_library().pmk_encrypt_blinded_plan(plan, _dev_ptr(d_msg), _dev_ptr(d_r), _dev_ptr(d_ct_star),
                                                   _dev_ptr(d_ct_r), _stream(stream)), ctx)


def pmk_decrypt_blinded_plan(plan: int, d_ct_star, d_ct_r, d_msg, stream=None, ctx: Optional[int] = None) -> None:
    _check(load_library().pmk_decrypt_blinded_plan(plan, _dev_ptr(d_ct_star), _dev_ptr(d_ct_r), _dev_ptr(d_msg),
                                                   _stream(stream)), ctx)


def pmk_encrypt_batch(plan: int, d_msg, d_ct, stream=None, ctx: Optional[int] = None) -> None:
    _check(load_library().pmk_encrypt_batch(plan, _dev_ptr(d_msg), _dev_ptr(d_ct), _stream(stream)), ctx)


def pmk_decrypt_batch(plan: int, d_ct, d_msg, stream=None, ctx: Optional[int] = None) -> None:
    _check(load_library().pmk_decrypt_batch(plan, _dev_ptr(d_ct), _dev_ptr(d_msg), _stream(stream)), ctx)


def pmk_set_window(ctx: int, bits: int, win: int) -> None:
    _check(load_library().pmk_set_window(ctx, int(bits), int(win)), ctx)


def pmk_get_window(ctx: int, bits: int) -> int:
    return load_library().pmk_get_window(ctx, int(bits))


def pmk_set_lanes(ctx: int, bits: int, fill_lanes: int, tail_lanes: int) -> None:
    _check(load_library().pmk_set_lanes(ctx, int(bits), int(fill_lanes), int(tail_lanes)), ctx)


def pmk_get_lanes(ctx: int, bits: int) -> Tuple[int, int]:
    """(fill_lanes, tail_lanes) of the class holding `bits`-bit moduli."""
    f, t = C.c_int(0), C.c_int(0)
    _check(load_library().pmk_get_lanes(ctx, int(bits), C.byref(f), C.byref(t)), ctx)
    return f.value, t.value


def pmk_set_grid_limit(ctx: int, waves: int) -> None:
    _check(load_library().pmk_set_grid_limit(ctx, int(waves)), ctx)


PMK_AUTOTUNE_FORCE = 1


def pmk_autotune(ctx: int, cache_path: Optional[str] = None, flags: int = 0) -> None:
    path = os.fsencode(cache_path) if cache_path else None
    _check(load_library().pmk_autotune(ctx, path, int(flags)), ctx)


def pmk_plan_check(plan: int, stream=None) -> int:
    return load_library().pmk_plan_check(plan, _stream(stream))


def pmk_plan_set_decrypt_output(plan: int, form: int) -> None:
    _check(load_library().pmk_plan_set_decrypt_output(plan, int(form)))


def pmk_plan_profile(plan: int, enable: bool) -> None:
    _check(load_library().pmk_plan_profile(plan, 1 if enable else 0))


def pmk_plan_kernel_time(plan: int, kind: int) -> Tuple[float, int]:
    ms, n = C.c_double(0.0), C.c_uint64(0)
    _check(load_library().pmk_plan_kernel_time(plan, int(kind), C.byref(ms), C.byref(n)))
    return ms.value, n.value


def pmk_encrypt(ctx: int, d_msg, msg_len: int, key_map, d_ct, ct_cap: int, stream=None) -> int:
    km = _map_array(key_map)
    return load_library().pmk_encrypt(ctx, _dev_ptr(d_msg), int(msg_len), km.ctypes.data_as(U32P), len(km),
                                      _dev_ptr(d_ct), int(ct_cap), _stream(stream))


def pmk_decrypt(ctx: int, d_ct, ct_len: int, key_map, d_msg, msg_len: int, stream=None) -> int:
    km = _map_array(key_map)
    return load_library().pmk_decrypt(ctx, _dev_ptr(d_ct), int(ct_len), km.ctypes.data_as(U32P), len(km),
                                      _dev_ptr(d_msg), int(msg_len), _stream(stream))


def pmk_decrypt_noalloc(ctx: int, d_ct, ct_len: int, key_map, d_msg, msg_len: int, stream=None) -> int:
    km = _map_array(key_map)
    return load_library().pmk_decrypt_noalloc(ctx, _dev_ptr(d_ct), int(ct_len), km.ctypes.data_as(U32P), len(km),
                                              _dev_ptr(d_msg), int(msg_len), _stream(stream))


def _host_ptr(x) -> Optional[int]:
    """Address of a host buffer: a numpy array, a CPU torch tensor, or an int."""
    if x is None or isinstance(x, int):
        return x
    if isinstance(x, np.ndarray):
        return int(x.ctypes.data)
    return int(x.data_ptr())


def pmk_encrypt_host(plan: int, msg, ct, slices: int = 0) -> int:
    return load_library().pmk_encrypt_host(plan, _host_ptr(msg), _host_ptr(ct), int(slices))


def pmk_decrypt_host(plan: int, ct, msg, slices: int = 0) -> int:
    return load_library().pmk_decrypt_host(plan, _host_ptr(ct), _host_ptr(msg), int(slices))


def pmk_mp_key_check(key) -> Tuple[int, str]:
    ka = MpKeyArray([key])
    buf = C.create_string_buffer(256)
    rc = load_library().pmk_mp_key_check(ka.ptr(), buf, 256)
    return rc, buf.value.decode()


def pmk_mp_keys_load(ctx: int, keys: Sequence) -> None:
    ka = keys if isinstance(keys, MpKeyArray) else MpKeyArray(keys)
    _check(load_library().pmk_mp_keys_load(ctx, ka.ptr(), ka.count), ctx)


def pmk_mp_key_count(ctx: int) -> int:
    return load_library().pmk_mp_key_count(ctx)


def pmk_mp_decrypt(ctx: int, d_ct, ct_len: int, key_map, d_msg, msg_len: int, stream=None) -> int:
    km = _map_array(key_map)
    return load_library().pmk_mp_decrypt(ctx, _dev_ptr(d_ct), int(ct_len), km.ctypes.data_as(U32P), len(km),
                                         _dev_ptr(d_msg), int(msg_len), _stream(stream))


def pmk_sieve(ctx: int, bits: int, d_cand, count: int, d_flags, stream=None) -> None:
    _check(load_library().pmk_sieve(ctx, int(bits), _dev_ptr(d_cand), int(count), _dev_ptr(d_flags),
                                    _stream(stream)), ctx)


def pmk_miller_rabin(ctx: int, bits: int, d_cand, count: int, d_bases, rounds: int, d_result, stream=None) -> None:
    _check(load_library().pmk_miller_rabin(ctx, int(bits), _dev_ptr(d_cand), int(count), _dev_ptr(d_bases),
                                           int(rounds), _dev_ptr(d_result), _stream(stream)), ctx)


def pmk_server_start(ctx: int, staging_bytes: int = 0, round_chunks: int = 0, pipeline_depth: int = 0) -> None:
    cfg = pmk_server_cfg(int(staging_bytes), int(round_chunks), int(pipeline_depth))
    _check(load_library().pmk_server_start(ctx, C.byref(cfg)), ctx)


def pmk_submit(ctx: int, op: int, data: np.ndarray, out: np.ndarray, msg_len: int, key_map) -> Tuple[int, int]:
    """(status, ticket).  data / out: host uint8 arrays that must stay alive
    until the ticket is reported done."""
    km = _map_array(key_map)
    req = pmk_request(int(op), data.ctypes.data if len(data) else None, out.ctypes.data if len(out) else None,
                      out.nbytes, int(msg_len), km.ctypes.data_as(U32P), len(km))
    t = C.c_uint64(0)
    rc = load_library().pmk_submit(ctx, C.byref(req), C.byref(t))
    return rc, t.value


def _info(i: pmk_ticket_info) -> dict:
    return {"state": i.state, "status": i.status, "t_submit_ns": i.t_submit_ns, "t_admit_ns": i.t_admit_ns,
            "t_done_ns": i.t_done_ns}


def pmk_poll(ctx: int, ticket: int) -> Tuple[int, dict]:
    info = pmk_ticket_info()
    rc = load_library().pmk_poll(ctx, int(ticket), C.byref(info))
    return rc, _info(info)


def pmk_wait(ctx: int, ticket: int) -> Tuple[int, dict]:
    info = pmk_ticket_info()
    rc = load_library().pmk_wait(ctx, int(ticket), C.byref(info))
    return rc, _info(info)


def pmk_server_stats_get(ctx: int) -> dict:
    st = pmk_server_stats()
    _check(load_library().pmk_server_stats_get(ctx, C.byref(st)), ctx)
    return {f: getattr(st, f) for f, _ in pmk_server_stats._fields_}


def pmk_server_stop(ctx: int) -> None:
    _check(load_library().pmk_server_stop(ctx), ctx)


# ---------- a small object layer over the same calls -------------------------------------

class Plan:
    """A chunk plan (pmk_plan_create) bound to its context."""

    def __init__(self, ctx: "Context", key_map, msg_len: int):
        self.ctx = ctx
        self.handle, self.ct_len = pmk_plan_create(ctx.handle, key_map, msg_len)
        self.msg_len = int(msg_len)

    def encrypt(self, msg, ct=None, stream=None, batch: bool = False):
        """Encrypt `msg` (device tensor) into `ct`; batch=True uses the
        graph-captured persistent path (pmk_encrypt_batch)."""
        import torch

        if ct is None:
            ct = torch.empty(max(self.ct_len, 4), dtype=torch.uint8, device=msg.device)
        fn = pmk_encrypt_batch if batch else pmk_encrypt_plan
        fn(self.handle, msg, ct, stream, self.ctx.handle)
        return ct

    def set_decrypt_output(self, form: int) -> None:
        """PMK_DEC_CHUNKS (msg_len bytes) or PMK_DEC_BLOCKS (every m in full, ct_len bytes)."""
        pmk_plan_set_decrypt_output(self.handle, form)
        self.dec_blocks = form == PMK_DEC_BLOCKS

    def _dec_len(self) -> int:
        return self.ct_len if getattr(self, "dec_blocks", False) else self.msg_len

    def decrypt(self, ct, msg=None, stream=None, batch: bool = False):
        """CRT-decrypt `ct` into `msg`; batch=True uses pmk_decrypt_batch."""
        import torch

        if msg is None:
            msg = torch.empty(max(self._dec_len(), 4), dtype=torch.uint8, device=ct.device)
        fn = pmk_decrypt_batch if batch else pmk_decrypt_plan
        fn(self.handle, ct, msg, stream, self.ctx.handle)
        return msg

    def encrypt_blinded(self, msg, r, stream=None):
        """(c*, c_R) device tensors for message `msg` and blinding blocks `r`."""
        import torch

        n = max(self.ct_len, 4)
        cs = torch.empty(n, dtype=torch.uint8, device=msg.device)
        cr = torch.empty(n, dtype=torch.uint8, device=msg.device)
        pmk_encrypt_blinded_plan(self.handle, msg, r, cs, cr, stream, self.ctx.handle)
        return cs, cr

    def decrypt_blinded(self, ct_star, ct_r, msg=None, stream=None):
        import torch

        if msg is None:
            msg = torch.empty(max(self._dec_len(), 4), dtype=torch.uint8, device=ct_star.device)
        pmk_decrypt_blinded_plan(self.handle, ct_star, ct_r, msg, stream, self.ctx.handle)
        return msg

    def encrypt_host(self, msg, ct, slices: int = 0) -> int:
        """Host buffers in and out (pmk_encrypt_host); returns the status."""
        return pmk_encrypt_host(self.handle, msg, ct, slices)

    def decrypt_host(self, ct, msg, slices: int = 0) -> int:
        """Host buffers in and out (pmk_decrypt_host); returns the status."""
        return pmk_decrypt_host(self.handle, ct, msg, slices)

    def check(self, stream=None) -> int:
        return pmk_plan_check(self.handle, stream)

    def profile(self, enable: bool = True) -> None:
        pmk_plan_profile(self.handle, enable)

    def kernel_time(self, kind: int) -> Tuple[float, int]:
        """(total ms, launches) of one kernel kind since profiling was switched on."""
        return pmk_plan_kernel_time(self.handle, kind)

    def close(self):
        if self.handle:
            pmk_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The request server of a context (pmk_server_*).  Keeps each request's
    host buffers alive until its ticket is reported done."""

    def __init__(self, ctx: "Context", staging_bytes: int = 0, round_chunks: int = 0, pipeline_depth: int = 0):
        self.ctx = ctx
        pmk_server_start(ctx.handle, staging_bytes, round_chunks, pipeline_depth)
        self._held = {}
        self.running = True

    def submit(self, op: int, data: np.ndarray, msg_len: int, key_map, out: Optional[np.ndarray] = None):
        """Submit one request; returns (ticket, out array).  Raises PmkError on a
        validation error."""
        data = np.ascontiguousarray(data, dtype=np.uint8)
        if out is None:
            if op == PMK_OP_ENCRYPT:
                bits = [pmk_key_bits(self.ctx.handle, int(k)) for k in np.asarray(key_map)]
                n = int(sum(b // 8 for b in bits))
            else:
                n = int(msg_len)
            out = np.zeros(n, dtype=np.uint8)
        km = _map_array(key_map)
        rc, t = pmk_submit(self.ctx.handle, op, data, out, msg_len, km)
        if rc != PMK_OK:
            raise PmkError(rc, "submit")
        self._held[t] = (data, out, km)
        return t, out

    def poll(self, ticket: int) -> Optional[dict]:
        rc, info = pmk_poll(self.ctx.handle, ticket)
        if rc != PMK_OK:
            raise PmkError(rc, "poll")
        if info["state"] == PMK_REQ_DONE:
            self._held.pop(ticket, None)
            return info
        return None

    def wait(self, ticket: int) -> dict:
        rc, info = pmk_wait(self.ctx.handle, ticket)
        if rc != PMK_OK:
            raise PmkError(rc, "wait")
        self._held.pop(ticket, None)
        return info

    def stats(self) -> dict:
        return pmk_server_stats_get(self.ctx.handle)

    def stop(self) -> None:
        if self.running:
            pmk_server_stop(self.ctx.handle)
            self.running = False
            self._held.clear()


class Context:
    """pmk_create / pmk_keys_load / plans on one GPU."""

    def __init__(self, device: int = 0):
        import weakref

        self.handle = pmk_create(device)
        self.device = device
        self._plans = weakref.WeakSet()

    def load_keys(self, keys: Sequence) -> None:
        pmk_keys_load(self.handle, keys)

    def load_mp_keys(self, keys: Sequence) -> None:
        pmk_mp_keys_load(self.handle, keys)

    def mp_decrypt(self, ct, key_map, msg_len: int, msg=None, stream=None):
        """Multi-prime CRT decryption (pmk_mp_decrypt, synchronous); returns the message tensor."""
        import torch

        if msg is None:
            msg = torch.empty(max(1, msg_len), dtype=torch.uint8, device=ct.device)
        _check(pmk_mp_decrypt(self.handle, ct, ct.numel(), key_map, msg, msg_len, stream), self.handle)
        return msg

    def set_window(self, bits: int, win: int) -> None:
        pmk_set_window(self.handle, bits, win)

    def window(self, bits: int) -> int:
        return pmk_get_window(self.handle, bits)

    def set_lanes(self, bits: int, fill_lanes: int, tail_lanes: Optional[int] = None) -> None:
        """Lanes per number of the CRT halves of a launch under one round and of
        the partial round after full ones (default: the same): 1, 2 or 4 for the
        one-lane classes (fill also 8 at 2048-4096 bits); 4, or 8 for small
        launches, for 6144/8192 bits."""
        pmk_set_lanes(self.handle, bits, fill_lanes, fill_lanes if tail_lanes is None else tail_lanes)

    def lanes(self, bits: int) -> Tuple[int, int]:
        return pmk_get_lanes(self.handle, bits)

    def set_grid_limit(self, waves: int) -> None:
        """At most `waves` resident waves per persistent launch (0: the device's occupancy)."""
        pmk_set_grid_limit(self.handle, waves)

    def autotune(self, cache_path: Optional[str] = None, force: bool = False) -> None:
        """Pick each loaded size class's CRT window width by timing (pmk_autotune)."""
        pmk_autotune(self.handle, cache_path, PMK_AUTOTUNE_FORCE if force else 0)

    def server(self, staging_bytes: int = 0, round_chunks: int = 0, pipeline_depth: int = 0) -> "Server":
        return Server(self, staging_bytes, round_chunks, pipeline_depth)

    def plan(self, key_map, msg_len: int) -> Plan:
        p = Plan(self, key_map, msg_len)
        self._plans.add(p)
        return p

    def close(self):
        for p in list(self._plans):
            p.close()
        if self.handle:
            pmk_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
