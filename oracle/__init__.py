"""CPU oracle for the PMKRSA hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use this package.  It wraps ``oracle.c`` through ctypes: plain C with
schoolbook multiplication, Knuth Algorithm D remainders, x^e mod N (the
operation of Algorithm 2) by left-to-right square-and-multiply, and CRT-RSA
decryption as in Sec. 2.1.  Operands beyond its fixed limb capacity (520
limbs; moduli up to 260 limbs) raise instead of being cut.  It shares no code
with the GPU library.

Pins (tests/test_oracle_*.py) tie it to facts outside itself: Python's own
integer arithmetic (an independent implementation), brute-force repeated
multiplication on tiny moduli, exhaustive bijection over a 12-bit key, the
RSA/PMKRSA correctness identities (Sec. 1.1, Sec. 3.1) and hand-checkable
worked values.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

U32P = C.POINTER(C.c_uint32)


class OracleKey(C.Structure):
    _fields_ = [
        ("bits", C.c_int32),
        ("n", U32P), ("n_len", C.c_int32),
        ("e", U32P), ("e_len", C.c_int32),
        ("d", U32P), ("d_len", C.c_int32),
        ("p", U32P), ("p_len", C.c_int32),
        ("q", U32P), ("q_len", C.c_int32),
        ("dp", U32P), ("dp_len", C.c_int32),
        ("dq", U32P), ("dq_len", C.c_int32),
        ("qinv", U32P), ("qinv_len", C.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + f".{os.getpid()}.tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, SRC_PATH])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        L.oracle_mul.argtypes = [U32P, C.c_int, U32P, C.c_int, U32P, C.c_int]
        L.oracle_divmod.argtypes = [U32P, C.c_int, U32P, C.c_int, U32P, C.c_int, U32P, C.c_int]
        L.oracle_modexp.argtypes = [U32P, C.c_int, U32P, C.c_int, U32P, C.c_int, U32P, C.c_int]
        L.oracle_plan.argtypes = [C.POINTER(OracleKey), C.c_int, U32P, C.c_longlong, C.c_longlong,
                                  C.POINTER(C.c_longlong), C.POINTER(C.c_longlong),
                                  C.POINTER(C.c_longlong)]
        L.oracle_plan.restype = C.c_longlong
        L.oracle_encrypt.argtypes = [C.POINTER(OracleKey), C.c_int, C.c_void_p, C.c_longlong, U32P,
                                     C.c_longlong, C.c_void_p]
        L.oracle_decrypt.argtypes = [C.POINTER(OracleKey), C.c_int, C.c_void_p, C.c_longlong, U32P,
                                     C.c_longlong, C.c_void_p, C.c_int]
        L.oracle_rsa_int.argtypes = [C.POINTER(OracleKey), C.c_int, U32P, C.c_int, U32P, C.c_int]
        L.oracle_blind_int.argtypes = [C.POINTER(OracleKey), C.c_int, U32P, C.c_int, U32P, C.c_int,
                                       U32P, U32P, C.c_int]
        L.oracle_threads.restype = C.c_int
        L.oracle_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


# ---------- integer <-> limb helpers (little-endian base 2^32) ---------------------------

def to_limbs(x: int, n: int = 0) -> np.ndarray:
    if x < 0:
        raise ValueError("negative")
    n = max(n, (x.bit_length() + 31) // 32, 1)
    return np.frombuffer(x.to_bytes(4 * n, "little"), dtype=np.uint32).copy()


def from_limbs(a: np.ndarray) -> int:
    return int.from_bytes(np.ascontiguousarray(a, dtype=np.uint32).tobytes(), "little")


def _p(a: np.ndarray):
    return a.ctypes.data_as(U32P)


def mul(a: int, b: int) -> int:
    A, B = to_limbs(a), to_limbs(b)
    R = np.zeros(len(A) + len(B), dtype=np.uint32)
    rc = lib().oracle_mul(_p(A), len(A), _p(B), len(B), _p(R), len(R))
    if rc != 0:
        raise OverflowError("operands beyond the oracle's limb capacity")
    return from_limbs(R)


def divmod_(u: int, v: int) -> Tuple[int, int]:
    U, V = to_limbs(u), to_limbs(v)
    Q = np.zeros(len(U), dtype=np.uint32)
    R = np.zeros(len(V), dtype=np.uint32)
    rc = lib().oracle_divmod(_p(U), len(U), _p(V), len(V), _p(Q), len(Q), _p(R), len(R))
    if rc == -2:
        raise OverflowError("operands beyond the oracle's limb capacity")
    if rc != 0:
        raise ZeroDivisionError
    return from_limbs(Q), from_limbs(R)


def modexp(x: int, e: int, m: int) -> int:
    X, E, M = to_limbs(x), to_limbs(e), to_limbs(m)
    Y = np.zeros(len(M), dtype=np.uint32)
    rc = lib().oracle_modexp(_p(X), len(X), _p(E), len(E), _p(M), len(M), _p(Y), len(Y))
    if rc == -2:
        raise OverflowError("operands beyond the oracle's limb capacity")
    if rc != 0:
        raise ValueError("modulus 0")
    return from_limbs(Y)


class KeyTable:
    """The oracle's own copy of a key set, as C structs (built from ints)."""

    FIELDS = ("n", "e", "d", "p", "q", "dp", "dq", "qinv")

    def __init__(self, keys: Sequence):
        self._keep: List[np.ndarray] = []
        self.arr = (OracleKey * max(1, len(keys)))()
        self.count = len(keys)
        for i, k in enumerate(keys):
            s = self.arr[i]
            s.bits = int(k.bits)
            for f in self.FIELDS:
                limbs = to_limbs(int(getattr(k, f)))
                self._keep.append(limbs)
                setattr(s, f, _p(limbs))
                setattr(s, f + "_len", len(limbs))
        self.bits = [int(k.bits) for k in keys]

    def ptr(self):
        return self.arr


def plan(table: KeyTable, key_map: np.ndarray, msg_len: int):
    """(msg_off, chunk_len, ct_off, ct_len) of every chunk; ValueError on a bad plan."""
    km = np.ascontiguousarray(key_map, dtype=np.uint32)
    n = len(km)
    off = (C.c_longlong * max(n, 1))()
    ln = (C.c_longlong * max(n, 1))()
    cto = (C.c_longlong * max(n, 1))()
    total = lib().oracle_plan(table.ptr(), table.count, _p(km), n, msg_len, off, ln, cto)
    if total < 0:
        raise ValueError("chunk count does not match the message")
    return (np.array(off[:n], dtype=np.int64), np.array(ln[:n], dtype=np.int64),
            np.array(cto[:n], dtype=np.int64), int(total))


def encrypt(table: KeyTable, msg: np.ndarray, key_map: np.ndarray) -> np.ndarray:
    """Ciphertext blocks (kb bytes each, big-endian) of every chunk, concatenated."""
    msg = np.ascontiguousarray(msg, dtype=np.uint8)
    km = np.ascontiguousarray(key_map, dtype=np.uint32)
    _, _, _, total = plan(table, km, len(msg))
    ct = np.zeros(total, dtype=np.uint8)
    rc = lib().oracle_encrypt(table.ptr(), table.count, msg.ctypes.data, len(msg), _p(km), len(km),
                              ct.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_encrypt: {rc}")
    return ct


def decrypt(table: KeyTable, ct: np.ndarray, msg_len: int, key_map: np.ndarray,
            crt: bool = True) -> Tuple[np.ndarray, int]:
    """(message bytes, status): status 0, or -3 when some block is not below its modulus."""
    ct = np.ascontiguousarray(ct, dtype=np.uint8)
    km = np.ascontiguousarray(key_map, dtype=np.uint32)
    _, _, _, total = plan(table, km, msg_len)
    if len(ct) < total:
        raise ValueError("ciphertext too short")
    out = np.zeros(msg_len, dtype=np.uint8)
    rc = lib().oracle_decrypt(table.ptr(), table.count, ct.ctypes.data, msg_len, _p(km), len(km),
                              out.ctypes.data, 1 if crt else 0)
    if rc not in (0, -3):
        raise ValueError(f"oracle_decrypt: {rc}")
    return out, rc


def rsa_int(table: KeyTable, key_index: int, mode: str, x: int) -> int:
    """Single integer: mode 'enc' (x^e), 'dec' (x^d) or 'crt' (CRT decryption)."""
    X = to_limbs(x)
    nl = (table.bits[key_index] + 31) // 32 + 1
    out = np.zeros(nl, dtype=np.uint32)
    m = {"enc": 0, "dec": 1, "crt": 2}[mode]
    k = C.pointer(table.arr[key_index])
    rc = lib().oracle_rsa_int(k, m, _p(X), len(X), _p(out), nl)
    if rc == -2:
        raise OverflowError("key or input beyond the oracle's limb capacity")
    if rc != 0:
        raise ValueError(f"oracle_rsa_int: {rc}")
    return from_limbs(out)


def blind_int(table: KeyTable, key_index: int, mode: str, x: int, aux: int) -> Tuple[int, int]:
    """PMKRSA blinding (Sec. 3.1): mode 'enc' gives (c*, c_R) from (m, r); mode 'dec'
    gives (m, r') from (c*, c_R)."""
    X, A = to_limbs(x), to_limbs(aux)
    nl = (table.bits[key_index] + 31) // 32 + 1
    o1 = np.zeros(nl, dtype=np.uint32)
    o2 = np.zeros(nl, dtype=np.uint32)
    k = C.pointer(table.arr[key_index])
    rc = lib().oracle_blind_int(k, 0 if mode == "enc" else 1, _p(X), len(X), _p(A), len(A),
                                _p(o1), _p(o2), nl)
    if rc != 0:
        raise ValueError(f"oracle_blind_int: {rc}")
    return from_limbs(o1), from_limbs(o2)


def threads() -> int:
    return lib().oracle_threads()


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


# ---------- primality (key generation) -----------------------------------------------------

def small_odd_primes(limit: int = 4096):
    """Odd primes below `limit`, by a plain sieve of Eratosthenes."""
    comp = [False] * limit
    out = []
    for i in range(3, limit, 2):
        if not comp[i]:
            out.append(i)
            for j in range(i * i, limit, 2 * i):
                comp[j] = True
    return out


def trial_division_pass(m: int, limit: int = 4096) -> bool:
    """True if no odd prime below `limit` divides m."""
    return all(m % p for p in small_odd_primes(limit))


def miller_rabin(m: int, bases) -> bool:
    """The Miller-Rabin test written out (m odd, m > 3): with m - 1 = 2^s d, d
    odd, base a passes if a^d = 1 or a^(2^j d) = m - 1 for some 0 <= j < s
    (Python's built-in pow is the modular exponentiation step).  True if every
    base passes (probable prime), False if one shows m composite."""
    d, s = m - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in bases:
        x = pow(a, d, m)
        if x == 1 or x == m - 1:
            continue
        for _ in range(s - 1):
            x = x * x % m
            if x == m - 1:
                break
        else:
            return False
    return True

