"""Python binding of ``libtns.so`` (include/tns.h): argument marshalling only.

Every step of the amplitude computation runs in the library's HIP kernels.
The binding converts numpy arrays to the C structures, calls the C ABI and
turns error codes into exceptions.  If the shared library is missing it raises
-- there is no fallback path.
"""

import ctypes
import os
import weakref
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtns.so")

TNS_OK = 0
STATUS = {0: "TNS_OK", -1: "TNS_E_INVALID_ARG", -2: "TNS_E_BAD_CIRCUIT", -3: "TNS_E_BAD_PATH",
          -4: "TNS_E_OUT_OF_MEMORY", -5: "TNS_E_ADMISSION", -6: "TNS_E_DEVICE",
          -7: "TNS_E_CANCELLED", -8: "TNS_E_UNSUPPORTED", -9: "TNS_E_NO_DEVICE"}
PRECISION = {"c128": 0, "c64": 1, "c64_bf16x3": 2, "c64_bf16x6": 3}
PATH_MODE = {"greedy": 0, "algorithm1": 1}

EXPORTED = ["tns_init", "tns_set_allocator", "tns_finalize", "tns_plan_opts_default",
            "tns_plan_create", "tns_plan_info_get", "tns_plan_destroy", "tns_amplitudes",
            "tns_amplitudes_sliced", "tns_amplitudes_noalloc", "tns_sample_frugal",
            "tns_serving_configure", "tns_submit", "tns_poll", "tns_wait", "tns_cancel", "tns_request_free",
            "tns_request_latency", "tns_path_search", "tns_last_error", "tns_version"]


class TnsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class _Gate(ctypes.Structure):
    _fields_ = [("q0", ctypes.c_int32), ("q1", ctypes.c_int32), ("cycle", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("m", ctypes.c_double * 32)]


GATE_DTYPE = np.dtype([("q0", np.int32), ("q1", np.int32), ("cycle", np.int32),
                       ("reserved", np.int32), ("m", np.float64, (32,))])


class _CircuitDesc(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("edges", ctypes.c_void_p), ("n_gates", ctypes.c_int32),
                ("gates", ctypes.c_void_p)]


class _PlanOpts(ctypes.Structure):
    _fields_ = [("split_cycle", ctypes.c_int32), ("path", ctypes.c_void_p),
                ("path_mode", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("path_assumptions", ctypes.c_int32), ("n_cuts", ctypes.c_int32),
                ("cut_edges", ctypes.c_void_p), ("max_intermediate_elems", ctypes.c_uint64),
                ("svd_rel_cutoff", ctypes.c_double), ("max_search_states", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("n_open", ctypes.c_int32),
                ("open_qubits", ctypes.c_void_p), ("path_branches", ctypes.c_int32)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("split_cycle", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("path", ctypes.POINTER(ctypes.c_int32)),
                ("step_m", ctypes.POINTER(ctypes.c_int64)),
                ("step_k", ctypes.POINTER(ctypes.c_int64)),
                ("step_n", ctypes.POINTER(ctypes.c_int64)),
                ("step_kernel", ctypes.POINTER(ctypes.c_int32)),
                ("step_permute", ctypes.POINTER(ctypes.c_int32)),
                ("bond_ket", ctypes.POINTER(ctypes.c_int32)),
                ("bond_bra", ctypes.POINTER(ctypes.c_int32)),
                ("bond_overlap", ctypes.POINTER(ctypes.c_int32)),
                ("n_cuts", ctypes.c_int32), ("cut_edges", ctypes.POINTER(ctypes.c_int32)),
                ("n_slices", ctypes.c_int64), ("flops_per_amp", ctypes.c_double),
                ("gemm_bytes_per_amp", ctypes.c_double),
                ("permute_bytes_per_amp", ctypes.c_double), ("path_score", ctypes.c_double),
                ("peak_elems", ctypes.c_int64), ("device_bytes_resident", ctypes.c_int64),
                ("device_bytes_per_unit", ctypes.c_int64), ("n_fused_ket", ctypes.c_int32),
                ("n_fused_bra", ctypes.c_int32), ("search_complete", ctypes.c_int32),
                ("search_states", ctypes.c_int64), ("max_rank_used", ctypes.c_int32),
                ("fidelity", ctypes.c_double), ("n_samples", ctypes.c_double),
                ("precision", ctypes.c_int32), ("n_open", ctypes.c_int32),
                ("open_qubits", ctypes.POINTER(ctypes.c_int32)),
                ("n_branches", ctypes.c_int32),
                ("branch_windows", ctypes.POINTER(ctypes.c_int32)),
                ("step_chain", ctypes.POINTER(ctypes.c_int32)),
                ("linear_score", ctypes.c_double), ("n_prefix_steps", ctypes.c_int32),
                ("prefix_flops_per_amp", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_bra", ctypes.c_double),
                ("ms_merge", ctypes.c_double), ("ms_contract", ctypes.c_double),
                ("flops", ctypes.c_double), ("units", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("peak_device_bytes", ctypes.c_int64),
                ("ms_gemm", ctypes.c_double), ("gemm_launches", ctypes.c_int64),
                ("gemm_flops", ctypes.c_double), ("gemm_bytes", ctypes.c_double),
                ("ms_permute", ctypes.c_double), ("permute_bytes", ctypes.c_double),
                ("ms_small", ctypes.c_double), ("gemm_mfma_flops", ctypes.c_double),
                ("ms_gemm3m", ctypes.c_double), ("gemm3m_launches", ctypes.c_int64),
                ("gemm3m_flops", ctypes.c_double), ("gemm3m_mfma_flops", ctypes.c_double),
                ("gemm3m_bytes", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtns.so; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with python -m paper_2011_02621_amd.build")
    # One HIP runtime per process: torch carries its own copy of the runtime
    # library, and two copies loaded side by side each see the GPU only if
    # the other has not opened it.  With torch imported first, the library's
    # dependency resolves to the copy already loaded.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "tns_init": ([ctypes.c_int, u64, ctypes.POINTER(vp)], i32),
        "tns_set_allocator": ([vp, vp, vp, vp], i32),
        "tns_finalize": ([vp], i32),
        "tns_plan_opts_default": ([ctypes.POINTER(_PlanOpts)], None),
        "tns_plan_create": ([vp, ctypes.POINTER(_CircuitDesc), ctypes.POINTER(_PlanOpts),
                             ctypes.POINTER(vp)], i32),
        "tns_plan_info_get": ([vp, ctypes.POINTER(_PlanInfo)], i32),
        "tns_plan_destroy": ([vp], i32),
        "tns_amplitudes": ([vp, vp, i64, vp, vp, vp, ctypes.POINTER(_Stats)], i32),
        "tns_amplitudes_sliced": ([vp, vp, i64, vp, i64, i64, vp, vp, ctypes.POINTER(_Stats)], i32),
        "tns_amplitudes_noalloc": ([vp, vp, i64, vp, vp, vp], i32),
        "tns_sample_frugal": ([vp, vp, i64, vp, vp, ctypes.c_double, vp, vp, vp, ctypes.POINTER(_Stats)], i32),
        "tns_serving_configure": ([vp, i32, ctypes.c_double], i32),
        "tns_submit": ([vp, vp, i64, vp, vp, ctypes.POINTER(vp)], i32),
        "tns_poll": ([vp, ctypes.POINTER(ctypes.c_int)], i32),
        "tns_wait": ([vp], i32),
        "tns_cancel": ([vp], i32),
        "tns_request_free": ([vp], i32),
        "tns_request_latency": ([vp, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_double)], i32),
        "tns_path_search": ([i32, i32, vp, vp, i32, i32, i32, i64, ctypes.c_double, vp,
                             ctypes.POINTER(ctypes.c_double)], i32),
        "tns_last_error": ([], ctypes.c_char_p),
        "tns_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc):
    if rc != TNS_OK:
        raise TnsError(rc, load_library().tns_last_error().decode())


def version() -> str:
    return load_library().tns_version().decode()


# ---------------------------------------------------------------------------

def _circuit_arrays(circ):
    """Accepts any object with ``n``, ``edge_array()`` and ``gate_arrays()``."""
    edges = np.ascontiguousarray(circ.edge_array(), np.int32).reshape(-1, 2)
    q0, q1, cy, mats = circ.gate_arrays()
    gates = np.zeros(len(q0), GATE_DTYPE)
    gates["q0"], gates["q1"], gates["cycle"], gates["m"] = q0, q1, cy, mats
    return int(circ.n), edges, gates


@dataclass
class PlanInfo:
    n_qubits: int
    split_cycle: int
    path: np.ndarray
    step_m: np.ndarray
    step_k: np.ndarray
    step_n: np.ndarray
    step_kernel: np.ndarray
    step_permute: np.ndarray
    bond_ket: np.ndarray
    bond_bra: np.ndarray
    bond_overlap: np.ndarray
    cut_edges: np.ndarray
    n_slices: int
    flops_per_amp: float
    gemm_bytes_per_amp: float
    permute_bytes_per_amp: float
    path_score: float
    peak_elems: int
    device_bytes_resident: int
    device_bytes_per_unit: int
    n_fused_ket: int
    n_fused_bra: int
    search_complete: bool
    search_states: int
    max_rank_used: int
    fidelity: float
    n_samples: float
    precision: int
    open_qubits: np.ndarray
    branch_windows: np.ndarray   # [n_branches][2]
    step_chain: np.ndarray
    linear_score: float
    n_prefix_steps: int          # leading steps shared by every slice (computed once per bitstring)
    prefix_flops_per_amp: float


def _arr(ptr, n, dtype):
    if n == 0 or not ptr:
        return np.zeros(0, dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype).copy()


class Plan:
    def __init__(self, ctx: "Context", handle, keep):
        self.ctx, self._h, self._keep = ctx, handle, keep
        ctx._plans.add(self)
        inf = self.info()
        self.n_qubits = inf.n_qubits
        self.n_open = len(inf.open_qubits)

    def info(self) -> PlanInfo:
        inf = _PlanInfo()
        _check(load_library().tns_plan_info_get(self._h, ctypes.byref(inf)))
        ns, ne = inf.n_steps, inf.n_edges
        return PlanInfo(
            inf.n_qubits, inf.split_cycle, _arr(inf.path, inf.n_qubits, np.int32),
            _arr(inf.step_m, ns, np.int64), _arr(inf.step_k, ns, np.int64),
            _arr(inf.step_n, ns, np.int64), _arr(inf.step_kernel, ns, np.int32),
            _arr(inf.step_permute, ns, np.int32), _arr(inf.bond_ket, ne, np.int32),
            _arr(inf.bond_bra, ne, np.int32), _arr(inf.bond_overlap, ne, np.int32),
            _arr(inf.cut_edges, inf.n_cuts, np.int32), inf.n_slices, inf.flops_per_amp,
            inf.gemm_bytes_per_amp, inf.permute_bytes_per_amp, inf.path_score, inf.peak_elems,
            inf.device_bytes_resident, inf.device_bytes_per_unit, inf.n_fused_ket,
            inf.n_fused_bra, bool(inf.search_complete), inf.search_states, inf.max_rank_used,
            inf.fidelity, inf.n_samples, inf.precision, _arr(inf.open_qubits, inf.n_open, np.int32),
            _arr(inf.branch_windows, 2 * inf.n_branches, np.int32).reshape(-1, 2),
            _arr(inf.step_chain, ns, np.int32), inf.linear_score, inf.n_prefix_steps,
            inf.prefix_flops_per_amp)

    def close(self):
        if self._h:
            _check(load_library().tns_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Request:
    def __init__(self, handle, bits, amps):
        self._h, self.bits, self.amps = handle, bits, amps

    def done(self) -> bool:
        d = ctypes.c_int(0)
        _check(load_library().tns_poll(self._h, ctypes.byref(d)))
        return bool(d.value)

    def wait(self) -> np.ndarray:
        _check(load_library().tns_wait(self._h))
        return self.amps.view(np.complex128).reshape(-1)

    def cancel(self):
        _check(load_library().tns_cancel(self._h))

    def latency_ms(self):
        t, r = ctypes.c_double(), ctypes.c_double()
        _check(load_library().tns_request_latency(self._h, ctypes.byref(t), ctypes.byref(r)))
        return t.value, r.value

    def close(self):
        if self._h:
            load_library().tns_request_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """device >= 0: a GPU context; device = -1: planning only."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.tns_init(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self.device = device
        self._alloc_cb = None
        self._plans = weakref.WeakSet()   # closed before the context is

    def use_torch_allocator(self):
        """Route device allocations through torch's caching allocator."""
        import torch
        alloc_t = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
        free_t = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
        dev = self.device

        def _alloc(size, stream, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), dev, stream)
            except Exception:
                return None

        def _free(ptr, stream, user):
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc_cb = (alloc_t(_alloc), free_t(_free))
        _check(load_library().tns_set_allocator(
            self._h, ctypes.cast(self._alloc_cb[0], ctypes.c_void_p),
            ctypes.cast(self._alloc_cb[1], ctypes.c_void_p), None))

    def plan(self, circ, split_cycle: int = -1, path: Optional[Sequence[int]] = None,
             path_mode: str = "algorithm1", max_rank: int = 0, path_assumptions: bool = True,
             cuts: Optional[Sequence[int]] = None, max_intermediate_elems: int = 1 << 32,
             precision: str = "c128", max_search_states: int = 0,
             svd_rel_cutoff: float = 1e-12, open_qubits: Optional[Sequence[int]] = None,
             branches: bool = True) -> Plan:
        lib = load_library()
        n, edges, gates = _circuit_arrays(circ)
        desc = _CircuitDesc(n, edges.shape[0], edges.ctypes.data, gates.shape[0], gates.ctypes.data)
        o = _PlanOpts()
        lib.tns_plan_opts_default(ctypes.byref(o))
        o.split_cycle = int(split_cycle)
        keep = [edges, gates]
        if path is not None:
            pa = np.ascontiguousarray(path, np.int32)
            keep.append(pa)
            o.path = pa.ctypes.data
        o.path_mode = PATH_MODE[path_mode]
        o.max_rank = int(max_rank)
        o.path_assumptions = 1 if path_assumptions else 0
        if cuts is None:
            o.n_cuts = -1
        else:
            ca = np.ascontiguousarray(cuts, np.int32)
            keep.append(ca)
            o.n_cuts = len(ca)
            o.cut_edges = ca.ctypes.data if len(ca) else None
        o.max_intermediate_elems = int(max_intermediate_elems)
        o.svd_rel_cutoff = float(svd_rel_cutoff)
        o.max_search_states = int(max_search_states)
        o.precision = PRECISION[precision]
        o.path_branches = 1 if branches else 0
        if open_qubits:
            oq = np.ascontiguousarray(open_qubits, np.int32)
            keep.append(oq)
            o.n_open = len(oq)
            o.open_qubits = oq.ctypes.data
        h = ctypes.c_void_p()
        _check(lib.tns_plan_create(self._h, ctypes.byref(desc), ctypes.byref(o), ctypes.byref(h)))
        return Plan(self, h, [])

    def amplitudes(self, plan: Plan, bits: np.ndarray, stream: Optional[int] = None,
                   stats: bool = False, slices: Optional[tuple] = None):
        """Amplitudes of the rows of ``bits``; with ``slices=(begin, end)`` the
        partial sums over that range of slices."""
        bits = np.ascontiguousarray(bits, np.uint8).reshape(-1, plan.n_qubits)
        per = 1 << plan.n_open
        amps = np.zeros((bits.shape[0] * per, 2), np.float64)
        st = _Stats()
        lib = load_library()
        if slices is None:
            _check(lib.tns_amplitudes(self._h, plan._h, bits.shape[0], bits.ctypes.data,
                                      amps.ctypes.data, stream, ctypes.byref(st)))
        else:
            _check(lib.tns_amplitudes_sliced(self._h, plan._h, bits.shape[0], bits.ctypes.data,
                                             int(slices[0]), int(slices[1]), amps.ctypes.data,
                                             stream, ctypes.byref(st)))
        out = amps.view(np.complex128).reshape(-1)
        if plan.n_open:
            out = out.reshape(bits.shape[0], per)
        if stats:
            return out, {f: getattr(st, f) for f, _ in _Stats._fields_}
        return out

    def amplitudes_noalloc(self, plan: Plan, n: int, bits_dev: int, amps_dev: int,
                           stream: Optional[int] = None):
        """Allocation-free amplitudes: ``bits_dev`` (uint8 [n][N]) and
        ``amps_dev`` (complex128 [n][2^open]) are device addresses owned by
        the caller; the work is only enqueued on ``stream``."""
        _check(load_library().tns_amplitudes_noalloc(self._h, plan._h, int(n), bits_dev, amps_dev,
                                                     stream))

    NOALLOC_SCRATCH_BYTES = 64 << 20

    def sample_frugal(self, plan: Plan, fixed_bits: np.ndarray, uniforms: np.ndarray,
                      m_bound: float = 10.0, stream: Optional[int] = None, stats: bool = False):
        """Frugal rejection over correlated batches: (accepted [n][2^k] bool,
        amplitudes [n][2^k]) for the rows of ``fixed_bits`` and the caller's
        uniform numbers ``uniforms`` [n][2^k]."""
        bits = np.ascontiguousarray(fixed_bits, np.uint8).reshape(-1, plan.n_qubits)
        per = 1 << plan.n_open
        u = np.ascontiguousarray(uniforms, np.float64).reshape(bits.shape[0], per)
        acc = np.zeros((bits.shape[0], per), np.uint8)
        amps = np.zeros((bits.shape[0] * per, 2), np.float64)
        st = _Stats()
        _check(load_library().tns_sample_frugal(self._h, plan._h, bits.shape[0], bits.ctypes.data,
                                                u.ctypes.data, float(m_bound), acc.ctypes.data,
                                                amps.ctypes.data, stream, ctypes.byref(st)))
        out = acc.astype(bool), amps.view(np.complex128).reshape(bits.shape[0], per)
        if stats:
            return out + ({f: getattr(st, f) for f, _ in _Stats._fields_},)
        return out

    def configure_serving(self, n_workers: int = 0, item_flops: float = 0.0):
        """Serving knobs (before the first submit): worker threads and the
        contraction flops per work item."""
        _check(load_library().tns_serving_configure(self._h, int(n_workers), float(item_flops)))

    def submit(self, plan: Plan, bits: np.ndarray) -> Request:
        bits = np.ascontiguousarray(bits, np.uint8).reshape(-1, plan.n_qubits)
        amps = np.zeros((bits.shape[0] << plan.n_open, 2), np.float64)
        h = ctypes.c_void_p()
        _check(load_library().tns_submit(self._h, plan._h, bits.shape[0], bits.ctypes.data,
                                         amps.ctypes.data, ctypes.byref(h)))
        return Request(h, bits, amps)

    def close(self):
        if self._h:
            for p in list(self._plans):
                p.close()
            _check(load_library().tns_finalize(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def path_search(n: int, edges, dims, mode: str = "algorithm1", max_rank: int = 0,
                assumptions: bool = True, max_states: int = 0, max_intermediate: float = 0.0):
    """(order, score) of a linear contraction path over a weighted graph;
    max_intermediate > 0 bounds every intermediate's size (Algorithm 1)."""
    e = np.ascontiguousarray(edges, np.int32).reshape(-1, 2)
    d = np.ascontiguousarray(dims, np.float64)
    out = np.zeros(n, np.int32)
    score = ctypes.c_double()
    _check(load_library().tns_path_search(n, e.shape[0], e.ctypes.data, d.ctypes.data,
                                          PATH_MODE[mode], max_rank, 1 if assumptions else 0,
                                          max_states, float(max_intermediate), out.ctypes.data,
                                          ctypes.byref(score)))
    return out.tolist(), score.value
