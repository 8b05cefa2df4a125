"""float128 CPU oracle for the Torontonian (Sec. 3.1, Eq. 2).

TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.  It shares
no code with the GPU path.  The arithmetic lives in tor_oracle.c (binary128
per-subset Hermitian Cholesky with Neumaier-compensated sums); this module
only marshals arguments through ctypes and returns values exactly as Python
Fractions (the C side hands back non-overlapping 3-term binary64 expansions
of each binary128 result).

Also here, in plain numpy (binary64): the selector's reference pieces --
feature extraction, the bound-based fallback of Eq. 5-7 and the MLP
forward/backward -- in oracle/selector_ref.py.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tor_oracle.c")
_LIB = os.path.join(_HERE, "libtor_oracle.so")

OK, EINVAL, ENOTPD, ENOMEM = 0, -1, -2, -4
NMAX_FULL = 26


class _Result(ctypes.Structure):
    _fields_ = [
        ("tor", ctypes.c_double * 3),
        ("abs_sum", ctypes.c_double * 3),
        ("min_det", ctypes.c_double * 3),
        ("max_term", ctypes.c_double * 3),
        ("bad_mask", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("threads", ctypes.c_int32),
    ]


def build(force: bool = False) -> str:
    """Compile tor_oracle.c into libtor_oracle.so (gcc, OpenMP, libquadmath)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-Wall",
               "-o", tmp, _SRC, "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.toro_tor.argtypes = [dp, ctypes.c_int, ctypes.c_int64, ctypes.c_int, dp,
                                 ctypes.POINTER(_Result)]
        lib.toro_tor.restype = ctypes.c_int
        lib.toro_terms.argtypes = [dp, ctypes.c_int, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64, ctypes.c_int,
                                   dp, dp, ctypes.POINTER(ctypes.c_int32)]
        lib.toro_terms.restype = ctypes.c_int
        lib.toro_level_sums.argtypes = [dp, ctypes.c_int, ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_int32), ctypes.c_int, ctypes.c_int, dp]
        lib.toro_level_sums.restype = ctypes.c_int
        lib.toro_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _frac3(a) -> Fraction:
    return Fraction(a[0]) + Fraction(a[1]) + Fraction(a[2])


def _as_o(O):
    O = np.ascontiguousarray(np.asarray(O, dtype=np.complex128))
    if O.ndim != 2 or O.shape[0] != O.shape[1] or O.shape[0] % 2:
        raise ValueError("O must be 2n x 2n")
    return O, O.shape[0] // 2


def asymmetry(O) -> dict:
    """How far O is from the conventions every Torontonian code here
    assumes (reported, never repaired): the largest |O - O^H| entry, and
    the largest deviations from the block structure of the sampling matrix
    (Eq. 3: O11 = conj(O00), O10 = conj(O01)).  All zero for inputs built
    by gbs_inputs."""
    O, n = _as_o(O)
    if n == 0:
        return dict(hermitian=0.0, o11=0.0, o10=0.0)
    herm = float(np.max(np.abs(O - O.conj().T)))
    o11 = float(np.max(np.abs(O[n:, n:] - O[:n, :n].conj())))
    o10 = float(np.max(np.abs(O[n:, :n] - O[:n, n:].conj())))
    return dict(hermitian=herm, o11=o11, o10=o10)


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(msg)
        self.code = code


def max_threads() -> int:
    return int(_load().toro_max_threads())


def tor(O, threads: int = 0, level_sums: bool = False) -> dict:
    """Tor(O) over all subsets (n <= 26), exactly as Fractions.

    Returns dict(tor, abs_sum, kappa, min_det, max_term, asymmetry, levels?,
    threads); asymmetry reports (does not repair) O's deviations from
    Hermitian and from the block structure of Eq. 3.
    Raises OracleError(ENOTPD) when I - O_Z is not positive definite for some Z.
    """
    lib = _load()
    O, n = _as_o(O)
    res = _Result()
    lv = np.zeros(3 * (n + 1), dtype=np.float64)
    rc = lib.toro_tor(_dptr(O) if n else None, n, max(2 * n, 1), int(threads),
                      _dptr(lv) if level_sums else None, ctypes.byref(res))
    if rc == ENOTPD:
        raise OracleError(rc, "I - O_Z not positive definite (first mask %d)" % res.bad_mask)
    if rc != OK:
        raise OracleError(rc, "oracle error %d" % rc)
    t = _frac3(res.tor)
    a = _frac3(res.abs_sum)
    out = dict(tor=t, abs_sum=a, min_det=_frac3(res.min_det), max_term=_frac3(res.max_term),
               threads=int(res.threads))
    out["kappa"] = float(a / abs(t)) if t != 0 else float("inf")
    out["asymmetry"] = asymmetry(O)
    if level_sums:
        out["levels"] = [_frac3(lv[3 * m:3 * m + 3]) for m in range(n + 1)]
    return out


def terms(O, masks, threads: int = 0):
    """Per-mask det(I - O_Z) and signed term, any n <= 60, as float64 arrays
    of the leading word plus exact Fractions on request via terms_exact()."""
    d3, t3, st = _terms3(O, masks, threads)
    return d3[:, 0] + d3[:, 1], t3[:, 0] + t3[:, 1], st


def _terms3(O, masks, threads=0):
    lib = _load()
    O, n = _as_o(O)
    masks = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    k = masks.size
    d3 = np.zeros((k, 3), dtype=np.float64)
    t3 = np.zeros((k, 3), dtype=np.float64)
    st = np.zeros(k, dtype=np.int32)
    rc = lib.toro_terms(_dptr(O) if n else None, n, max(2 * n, 1),
                        masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), k, int(threads),
                        _dptr(d3), _dptr(t3), st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc not in (OK, ENOTPD):
        raise OracleError(rc, "oracle error %d" % rc)
    return d3, t3, st


def terms_exact(O, masks, threads: int = 0):
    """Per-mask (det, term) as lists of Fractions, plus status codes."""
    d3, t3, st = _terms3(O, masks, threads)
    return [_frac3(r) for r in d3], [_frac3(r) for r in t3], st


def level_sums(O, levels, threads: int = 0):
    """L_m = sum over |Z| = m of det(I - O_Z)^(-1/2) for the given levels."""
    lib = _load()
    O, n = _as_o(O)
    lv = np.ascontiguousarray(np.asarray(levels, dtype=np.int32))
    out = np.zeros(3 * lv.size, dtype=np.float64)
    rc = lib.toro_level_sums(_dptr(O) if n else None, n, max(2 * n, 1),
                             lv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), lv.size, int(threads),
                             _dptr(out))
    if rc != OK:
        raise OracleError(rc, "oracle error %d" % rc)
    return [_frac3(out[3 * i:3 * i + 3]) for i in range(lv.size)]
