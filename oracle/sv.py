"""ctypes wrapper of the plain-C state-vector oracle (``oracle/sv.c``).

Oracle (test infrastructure).  amp(s) = <s|U|0^N> computed by applying every
gate of the circuit, in time order, to the dense complex128 vector |0...0>.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv.c")
_LIB = os.path.join(_HERE, "_build", "liboracle_sv.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile sv.c with gcc (plain C, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_sv_run.restype = ctypes.c_int
        lib.oracle_sv_run.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int]
        lib.oracle_sv_gather.restype = None
        lib.oracle_sv_gather.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_sv_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return _load().oracle_sv_max_threads()


def _arrays(circ_or_arrays):
    if hasattr(circ_or_arrays, "gate_arrays"):
        n = circ_or_arrays.n
        q0, q1, _, mats = circ_or_arrays.gate_arrays()
    else:
        n, q0, q1, mats = circ_or_arrays
    return (n, np.ascontiguousarray(q0, np.int32), np.ascontiguousarray(q1, np.int32),
            np.ascontiguousarray(mats, np.float64))


def state(circ, n_threads: int = 0) -> np.ndarray:
    """Full output state U|0^N> as complex128 [2^N]."""
    n, q0, q1, mats = _arrays(circ)
    psi = np.empty(1 << n, np.complex128)
    rc = _load().oracle_sv_run(n, psi.ctypes.data, len(q0), q0.ctypes.data, q1.ctypes.data,
                               mats.ctypes.data, int(n_threads))
    if rc != 0:
        raise ValueError("oracle_sv_run rejected the circuit")
    return psi


def amplitudes_from_state(n: int, psi: np.ndarray, bits: np.ndarray) -> np.ndarray:
    bits = np.ascontiguousarray(bits, np.uint8).reshape(-1, n)
    out = np.empty(bits.shape[0], np.complex128)
    _load().oracle_sv_gather(n, psi.ctypes.data, bits.shape[0], bits.ctypes.data,
                             out.ctypes.data)
    return out


def amplitudes(circ, bits: np.ndarray, n_threads: int = 0) -> np.ndarray:
    """amp(s) for each row s of ``bits`` (uint8 [n, N])."""
    n = circ.n if hasattr(circ, "n") else circ[0]
    psi = state(circ, n_threads)
    return amplitudes_from_state(n, psi, bits)


def index_of(bits_row) -> int:
    """Dense index sum_q s_q 2^(N-1-q)."""
    idx = 0
    for b in bits_row:
        idx = (idx << 1) | int(b)
    return idx
