"""ctypes binding of libqtn (argument marshalling only).

Every step of the contraction runs in libqtn's HIP kernels; this module only
converts Python/NumPy arguments, hands over device pointers and HIP streams
(PyTorch supplies device memory and streams), and raises on error codes.  If
libqtn.so is missing the import of any entry point raises: there is no other
execution path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int32, c_uint32, c_uint64, c_uint8, c_void_p
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqtn.so")

QTN_OK, QTN_EINVAL, QTN_ERANGE, QTN_ERANK, QTN_ENOMEM, QTN_EHIP, QTN_ESTATE, QTN_ETIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7
QTN_FP64, QTN_FP32, QTN_3XBF16 = 0, 1, 2
PRECISIONS = {"fp64": QTN_FP64, "fp32": QTN_FP32, "3xbf16": QTN_3XBF16}
STEP_REC, TENSOR_REC = 24, 40


class QtnGraph(ctypes.Structure):
    _fields_ = [("n", c_uint32), ("m", c_uint32), ("edges", POINTER(c_uint32))]


class QtnPlanOpts(ctypes.Structure):
    _fields_ = [("k", c_int32), ("max_rank", c_int32), ("k_max", c_int32),
                ("cut_vars", POINTER(c_uint32)), ("seed", c_uint64),
                ("ga_pop", c_int32), ("ga_iters", c_int32), ("precision", c_int32),
                ("fuse_chains", c_int32), ("exec_mode", c_int32),
                ("use_cost_model", c_int32), ("offspring_factor", c_int32),
                ("cost_model", c_void_p), ("density_matrix", c_int32)]


class QtnPartial(ctypes.Structure):
    _fields_ = [("re", c_double), ("im", c_double), ("re_comp", c_double), ("im_comp", c_double)]

    def value(self) -> complex:
        return complex(self.re + self.re_comp, self.im + self.im_comp)


class QtnPlanInfo(ctypes.Structure):
    _fields_ = [("n", c_uint32), ("p", c_uint32), ("n_vars", c_uint32), ("n_bitstrings", c_uint32),
                ("k", c_int32), ("width", c_int32), ("n_steps", c_int32), ("n_tensors", c_int32),
                ("log2_flops", c_double), ("bytes_per_slice", c_double),
                ("flops_hoisted", c_double), ("work", c_double), ("prefactor", c_double),
                ("search_seconds", c_double), ("precision", c_int32),
                ("f64_below_rank", c_int32), ("n_programs_wide", c_int32),
                ("n_launches_wide", c_int32), ("slice_lds_bytes", c_uint32),
                ("slice_scratch_bytes", c_double), ("mf_width", c_int32),
                ("rescaled", c_int32)]


class QtnKernelTiming(ctypes.Structure):
    _fields_ = [("launches", c_uint64), ("total_ms", c_double), ("alg_bytes", c_double),
                ("alg_flops", c_double), ("dropped", c_uint64), ("last_error", c_int32)]


class QtnSearchStats(ctypes.Structure):
    _fields_ = [("seconds", c_double), ("exact_evals", c_uint64), ("model_evals", c_uint64),
                ("width", c_int32), ("log2_cost", c_double)]


class QtnRangeStats(ctypes.Structure):
    _fields_ = [("ranges", c_uint64), ("contracted", c_uint64), ("resumed", c_uint64),
                ("retried", c_uint64)]


class QtnGate(ctypes.Structure):
    _fields_ = [("nq", c_uint32), ("q", c_uint32 * 2), ("re", c_double * 16), ("im", c_double * 16)]


class QtnTuneStats(ctypes.Structure):
    _fields_ = [("steps", c_uint32), ("measured", c_uint32), ("cached", c_uint32),
                ("default_us", c_double), ("tuned_us", c_double),
                ("whole_default_us", c_double), ("whole_tuned_us", c_double), ("kept", c_uint32),
                ("graph_us", c_double), ("direct_us", c_double), ("graphs", c_uint32)]


class QtnError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("qtn error %d: %s" % (code, msg))
        self.code = code


_lib = None

EXPORTS = ["qtn_plan_opts_default", "qtn_plan", "qtn_plan_destroy", "qtn_plan_query",
           "qtn_plan_cut", "qtn_plan_order", "qtn_plan_export", "qtn_plan_kappa",
           "qtn_plan_index_table", "qtn_plan_leaf_values", "qtn_plan_workspace_bytes",
           "qtn_plan_bind_workspace", "qtn_contract", "qtn_partial_combine",
           "qtn_plan_set_timing", "qtn_plan_timing", "qtn_plan_set_graphs", "qtn_last_error",
           "qtn_cost_features", "qtn_cost_exact", "qtn_mlp_create", "qtn_mlp_destroy",
           "qtn_mlp_num_params", "qtn_mlp_get_params", "qtn_mlp_set_params", "qtn_mlp_get_grads",
           "qtn_mlp_set_normalization", "qtn_mlp_forward", "qtn_mlp_train_step", "qtn_cut_search",
           "qtn_plan_step_timing", "qtn_plan_step_kernel", "qtn_plan_step_tune", "qtn_plan_set_step_tune",
           "qtn_plan_range_state",
           "qtn_contract_async",
           "qtn_contract_ranges", "qtn_plan_fingerprint", "qtn_plan_inject_faults",
           "qtn_contract_noalloc", "qtn_batch_contract", "qtn_plan_autotune", "qtn_plan_circuit"]
COST_FEATURES = 32


def lib():
    """Loads libqtn.so (built in-tree by paper_2010_14962_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqtn.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # torch supplies device memory and streams; its HIP runtime is brought up
    # before libqtn's code object registers, the order every caller relies on
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    L.qtn_plan_opts_default.argtypes = [POINTER(QtnPlanOpts)]
    L.qtn_plan_opts_default.restype = None
    L.qtn_plan.argtypes = [POINTER(QtnGraph), c_uint32, POINTER(c_double), POINTER(c_double),
                           POINTER(c_uint8), c_uint32, POINTER(QtnPlanOpts), POINTER(c_void_p)]
    L.qtn_plan_destroy.argtypes = [c_void_p]
    L.qtn_plan_destroy.restype = None
    L.qtn_plan_query.argtypes = [c_void_p, POINTER(QtnPlanInfo)]
    L.qtn_plan_cut.argtypes = [c_void_p, POINTER(c_uint32), c_uint32]
    L.qtn_plan_order.argtypes = [c_void_p, POINTER(c_uint32), c_uint32]
    L.qtn_plan_export.argtypes = [c_void_p, POINTER(c_int32), c_uint32, POINTER(c_int32), c_uint32]
    L.qtn_plan_kappa.argtypes = [c_void_p, c_int32, POINTER(c_int32), c_uint32]
    L.qtn_plan_index_table.argtypes = [c_void_p, c_int32, c_int32, POINTER(c_uint32), c_uint32,
                                       POINTER(c_uint32)]
    L.qtn_plan_leaf_values.argtypes = [c_void_p, c_int32, POINTER(c_double), c_uint64,
                                       POINTER(c_uint64)]
    L.qtn_plan_workspace_bytes.argtypes = [c_void_p, c_uint64, POINTER(c_uint64)]
    L.qtn_plan_bind_workspace.argtypes = [c_void_p, c_void_p, c_uint64, c_uint64]
    L.qtn_contract.argtypes = [c_void_p, c_uint64, c_uint64, c_void_p, POINTER(QtnPartial)]
    L.qtn_contract_async.argtypes = [c_void_p, c_uint64, c_uint64, c_void_p, c_void_p]
    L.qtn_partial_combine.argtypes = [POINTER(QtnPartial), POINTER(QtnPartial), POINTER(QtnPartial)]
    L.qtn_plan_set_timing.argtypes = [c_void_p, c_int32]
    L.qtn_plan_set_graphs.argtypes = [c_void_p, c_int32]
    L.qtn_plan_timing.argtypes = [c_void_p, POINTER(QtnKernelTiming)]
    L.qtn_plan_step_timing.argtypes = [c_void_p, c_int32, POINTER(QtnKernelTiming)]
    L.qtn_plan_step_kernel.argtypes = [c_void_p, c_int32, c_char_p, c_uint32]
    L.qtn_plan_step_tune.argtypes = [c_void_p, c_int32, POINTER(c_uint32), POINTER(c_int32)]
    L.qtn_plan_set_step_tune.argtypes = [c_void_p, c_int32, c_uint32, c_int32]
    L.qtn_plan_range_state.argtypes = [c_void_p, POINTER(c_int32), POINTER(c_uint64)]
    L.qtn_last_error.argtypes = []
    L.qtn_last_error.restype = c_char_p
    pf, pu32 = POINTER(ctypes.c_float), POINTER(c_uint32)
    L.qtn_cost_features.argtypes = [POINTER(QtnGraph), c_uint32, pu32, c_uint32, c_uint32, pf]
    L.qtn_cost_exact.argtypes = [POINTER(QtnGraph), c_uint32, pu32, c_uint32, c_uint32,
                                 POINTER(c_int32), POINTER(c_double), c_int32]
    L.qtn_mlp_create.argtypes = [c_uint32, c_uint32, c_uint32, c_uint32, c_uint32, c_uint64,
                                 POINTER(c_void_p)]
    L.qtn_mlp_destroy.argtypes = [c_void_p]
    L.qtn_mlp_destroy.restype = None
    L.qtn_mlp_num_params.argtypes = [c_void_p, POINTER(c_uint64)]
    L.qtn_mlp_get_params.argtypes = [c_void_p, pf, c_uint64]
    L.qtn_mlp_set_params.argtypes = [c_void_p, pf, c_uint64]
    L.qtn_mlp_get_grads.argtypes = [c_void_p, pf, c_uint64]
    L.qtn_mlp_set_normalization.argtypes = [c_void_p, pf, pf, pf, pf]
    L.qtn_mlp_forward.argtypes = [c_void_p, c_void_p, c_uint32, c_void_p, c_void_p]
    L.qtn_mlp_train_step.argtypes = [c_void_p, c_void_p, c_void_p, c_uint32, ctypes.c_float,
                                     c_void_p, pf]
    L.qtn_cut_search.argtypes = [POINTER(QtnGraph), c_uint32, c_uint32, c_int32, c_int32,
                                 c_uint64, c_void_p, c_int32, pu32, POINTER(QtnSearchStats)]
    L.qtn_contract_ranges.argtypes = [c_void_p, c_uint64, c_int32, c_char_p, c_void_p,
                                      POINTER(QtnPartial), POINTER(QtnRangeStats)]
    L.qtn_plan_fingerprint.argtypes = [c_void_p, POINTER(c_uint64)]
    L.qtn_contract_noalloc.argtypes = [c_void_p, c_uint64, c_uint64, c_uint64, c_void_p, c_void_p]
    L.qtn_plan_circuit.argtypes = [c_uint32, POINTER(QtnGate), c_uint32, POINTER(c_uint8), c_uint32,
                                   POINTER(QtnPlanOpts), POINTER(c_void_p)]
    L.qtn_plan_autotune.argtypes = [c_void_p, c_void_p, c_char_p, POINTER(QtnTuneStats)]
    L.qtn_batch_contract.argtypes = [POINTER(c_void_p), c_uint32, POINTER(c_uint64), POINTER(c_uint64),
                                     c_void_p, POINTER(QtnPartial)]
    L.qtn_plan_inject_faults.argtypes = [c_void_p, c_uint64, c_int32]
    for name in EXPORTS:
        if name not in ("qtn_plan_opts_default", "qtn_plan_destroy", "qtn_last_error",
                        "qtn_mlp_destroy"):
            getattr(L, name).restype = c_int32
    _lib = L
    return L


def _check(rc: int):
    if rc != QTN_OK:
        raise QtnError(rc, lib().qtn_last_error().decode())


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint32))


class Plan:
    """Owns one qtn_plan_t handle (and, once bound, a torch workspace)."""

    def __init__(self, handle: int, n: int, n_bitstrings: int):
        self._h = c_void_p(handle)
        self.n = n
        self.n_bitstrings = n_bitstrings
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def close(self):
        if self._h is not None and self._h.value:
            lib().qtn_plan_destroy(self._h)
        self._h = None

    # queries --------------------------------------------------------------
    def info(self) -> dict:
        inf = QtnPlanInfo()
        _check(lib().qtn_plan_query(self._h, byref(inf)))
        return {f: getattr(inf, f) for f, _ in QtnPlanInfo._fields_}

    def cut(self) -> List[int]:
        k = self.info()["k"]
        buf = (c_uint32 * max(k, 1))()
        _check(lib().qtn_plan_cut(self._h, buf, k))
        return [int(buf[i]) for i in range(k)]

    def order(self) -> List[int]:
        inf = self.info()
        m = inf["n_vars"] - inf["k"]
        buf = (c_uint32 * max(m, 1))()
        _check(lib().qtn_plan_order(self._h, buf, m))
        return [int(buf[i]) for i in range(m)]

    def export(self):
        inf = self.info()
        ns, nt = inf["n_steps"], inf["n_tensors"]
        steps = np.zeros((ns, STEP_REC), dtype=np.int32)
        tens = np.zeros((nt, TENSOR_REC), dtype=np.int32)
        _check(lib().qtn_plan_export(self._h, steps.ctypes.data_as(POINTER(c_int32)), ns,
                                     tens.ctypes.data_as(POINTER(c_int32)), nt))
        return steps, tens

    def kappa(self, step: int) -> List[int]:
        buf = (c_int32 * 64)()
        _check(lib().qtn_plan_kappa(self._h, step, buf, 64))
        steps, _ = self.export()
        return [int(buf[i]) for i in range(int(steps[step, 2]))]

    def index_table(self, step: int, inp: int) -> np.ndarray:
        cnt = c_uint32(0)
        _check(lib().qtn_plan_index_table(self._h, step, inp, None, 0, byref(cnt)))
        out = np.zeros(cnt.value, dtype=np.uint32)
        _check(lib().qtn_plan_index_table(self._h, step, inp, out.ctypes.data_as(POINTER(c_uint32)),
                                          cnt.value, byref(cnt)))
        return out

    def leaf_values(self, tensor: int) -> np.ndarray:
        cnt = c_uint64(0)
        _check(lib().qtn_plan_leaf_values(self._h, tensor, None, 0, byref(cnt)))
        out = np.zeros(2 * cnt.value, dtype=np.float64)
        _check(lib().qtn_plan_leaf_values(self._h, tensor, out.ctypes.data_as(POINTER(c_double)),
                                          cnt.value, byref(cnt)))
        return out[0::2] + 1j * out[1::2]

    def workspace_bytes(self, slices_per_wave: int) -> int:
        b = c_uint64(0)
        _check(lib().qtn_plan_workspace_bytes(self._h, slices_per_wave, byref(b)))
        return int(b.value)

    # device ---------------------------------------------------------------
    def bind_workspace(self, device_ptr: int, nbytes: int, slices_per_wave: int):
        _check(lib().qtn_plan_bind_workspace(self._h, c_void_p(device_ptr), nbytes, slices_per_wave))

    def bind_torch(self, slices_per_wave: int, device=None):
        """Allocates the workspace as a torch uint8 tensor on `device` and binds it."""
        import torch
        nbytes = self.workspace_bytes(slices_per_wave)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=device or "cuda")
        self.bind_workspace(ws.data_ptr(), nbytes, slices_per_wave)
        self._workspace = ws
        return ws

    def set_graphs(self, enable: bool = True):
        _check(lib().qtn_plan_set_graphs(self._h, 1 if enable else 0))

    def set_timing(self, enable: bool = True):
        _check(lib().qtn_plan_set_timing(self._h, 1 if enable else 0))

    def timing(self) -> dict:
        t = QtnKernelTiming()
        _check(lib().qtn_plan_timing(self._h, byref(t)))
        return {f: getattr(t, f) for f, _ in QtnKernelTiming._fields_}

    def step_timing(self, step: int) -> dict:
        t = QtnKernelTiming()
        _check(lib().qtn_plan_step_timing(self._h, step, byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}

    def step_kernel(self, step: int) -> str:
        buf = ctypes.create_string_buffer(128)
        _check(lib().qtn_plan_step_kernel(self._h, step, buf, len(buf)))
        return buf.value.decode()

    def step_tune(self, step: int) -> dict:
        """Launch configuration in use for a grid-wide step (autotuned or default)."""
        blocks, variant = c_uint32(0), c_int32(0)
        _check(lib().qtn_plan_step_tune(self._h, step, byref(blocks), byref(variant)))
        return {"blocks": blocks.value, "direct": variant.value == 1, "pair": variant.value == 2}

    def range_state(self) -> dict:
        """Whether synchronous contractions run without rescaling, and how
        many were repeated with rescaling after leaving the 64-bit range."""
        u, r = c_int32(0), c_uint64(0)
        _check(lib().qtn_plan_range_state(self._h, byref(u), byref(r)))
        return {"unscaled": bool(u.value), "reruns": r.value}

    def set_step_tune(self, step: int, blocks: int = 1024, direct: bool = False, pair: bool = False):
        """Sets a grid-wide step's launch configuration by hand."""
        _check(lib().qtn_plan_set_step_tune(self._h, step, blocks, 2 if pair else 1 if direct else 0))

    def contract_async(self, slice_lo: int, slice_hi: int, out_ptr: int,
                       stream: Optional[int] = None) -> None:
        """Enqueues the contraction and the copy of the partials to the host
        address out_ptr (n_bitstrings x 4 doubles; pinned memory keeps it
        asynchronous); valid after the stream is synchronised."""
        _check(lib().qtn_contract_async(self._h, slice_lo, slice_hi, c_void_p(stream or 0),
                                        c_void_p(out_ptr)))

    def contract(self, slice_lo: int, slice_hi: int, stream: Optional[int] = None) -> List[QtnPartial]:
        out = (QtnPartial * self.n_bitstrings)()
        _check(lib().qtn_contract(self._h, slice_lo, slice_hi, c_void_p(stream or 0), out))
        return [out[i] for i in range(self.n_bitstrings)]

    def contract_ranges(self, range_slices: int, max_retries: int = 0,
                        checkpoint: Optional[str] = None, stream: Optional[int] = None):
        """All slices as ranges of range_slices, re-issuing failed ranges and
        keeping a JSONL checkpoint; returns (partials, stats dict)."""
        out = (QtnPartial * self.n_bitstrings)()
        st = QtnRangeStats()
        _check(lib().qtn_contract_ranges(self._h, range_slices, max_retries,
                                         checkpoint.encode() if checkpoint else None,
                                         c_void_p(stream or 0), out, byref(st)))
        return [out[i] for i in range(self.n_bitstrings)], {
            "ranges": st.ranges, "contracted": st.contracted, "resumed": st.resumed,
            "retried": st.retried}

    def contract_noalloc(self, slice_lo: int, slice_hi: int, slices_per_wave: int, out_dev: int,
                         stream: Optional[int] = None) -> None:
        """Enqueues the contraction using the library's fixed device scratch
        (no allocation); partials go to device address out_dev."""
        _check(lib().qtn_contract_noalloc(self._h, slice_lo, slice_hi, slices_per_wave,
                                          c_void_p(stream or 0), c_void_p(out_dev)))

    def autotune(self, cache: Optional[str] = None, stream: Optional[int] = None) -> dict:
        """Measures and keeps the launch configuration of each streaming step."""
        st = QtnTuneStats()
        _check(lib().qtn_plan_autotune(self._h, c_void_p(stream or 0),
                                       cache.encode() if cache else None, byref(st)))
        return {f: getattr(st, f) for f, _ in QtnTuneStats._fields_}

    def fingerprint(self) -> int:
        v = c_uint64()
        _check(lib().qtn_plan_fingerprint(self._h, byref(v)))
        return v.value

    def inject_faults(self, slice_lo: int, count: int) -> None:
        _check(lib().qtn_plan_inject_faults(self._h, slice_lo, count))


def qtn_plan(n: int, edges: Sequence, p: int, gamma: Sequence[float], beta: Sequence[float],
             bitstrings, k: int = -1, max_rank: int = 0, k_max: int = 24,
             cut_vars: Optional[Sequence[int]] = None, seed: int = 0, ga_pop: int = 11,
             ga_iters: int = 4, precision: str = "fp64", fuse_chains: bool = True,
             exec_mode: str = "auto", cost_model=None, offspring_factor: int = 16,
             use_cost_model: Optional[bool] = None, density_matrix: bool = False) -> Plan:
    """Builds a plan: network, cut set, order and schedule (host only, except
    that a cost model ranks search candidates on its device).  With
    `cost_model` (a CostMLP) the cut search is the model-guided one."""
    L = lib()
    e = _u32(edges).reshape(-1)
    g = QtnGraph(n, len(e) // 2, e.ctypes.data_as(POINTER(c_uint32)))
    bits = np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint8).reshape(-1, n))
    ga = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64))
    be = np.ascontiguousarray(np.asarray(beta, dtype=np.float64))
    opts = QtnPlanOpts()
    L.qtn_plan_opts_default(byref(opts))
    opts.k = k
    opts.max_rank = max_rank
    opts.k_max = k_max
    opts.seed = seed
    opts.ga_pop = ga_pop
    opts.ga_iters = ga_iters
    opts.precision = PRECISIONS[precision]
    opts.fuse_chains = 1 if fuse_chains else 0
    opts.exec_mode = {"auto": -1, "wide": 0, "slice": 1}[exec_mode]
    if use_cost_model is None:
        use_cost_model = cost_model is not None
    opts.use_cost_model = 1 if use_cost_model else 0
    opts.offspring_factor = offspring_factor
    opts.cost_model = cost_model.handle.value if cost_model is not None else None
    opts.density_matrix = 1 if density_matrix else 0
    cv = None
    if cut_vars is not None:
        cv = _u32(cut_vars)
        opts.k = len(cv)
        opts.cut_vars = cv.ctypes.data_as(POINTER(c_uint32))
    h = c_void_p()
    _check(L.qtn_plan(byref(g), p, ga.ctypes.data_as(POINTER(c_double)),
                      be.ctypes.data_as(POINTER(c_double)), bits.ctypes.data_as(POINTER(c_uint8)),
                      bits.shape[0], byref(opts), byref(h)))
    return Plan(h.value, n, bits.shape[0])


def qtn_partial_combine(a: QtnPartial, b: QtnPartial) -> QtnPartial:
    out = QtnPartial()
    _check(lib().qtn_partial_combine(byref(a), byref(b), byref(out)))
    return out


def qtn_plan_circuit(n: int, gates, bitstrings, k: int = -1, max_rank: int = 0, k_max: int = 24,
                     cut_vars: Optional[Sequence[int]] = None, seed: int = 0, ga_pop: int = 11,
                     ga_iters: int = 4, precision: str = "fp64", fuse_chains: bool = True,
                     exec_mode: str = "auto") -> Plan:
    """Plan for a general circuit: gates are (qubits, matrix[out][in]) pairs."""
    L = lib()
    arr = (QtnGate * max(1, len(gates)))()
    for i, (qs, U) in enumerate(gates):
        U = np.asarray(U, dtype=np.complex128).reshape(-1)
        arr[i].nq = len(qs)
        for j, q in enumerate(qs):
            arr[i].q[j] = int(q)
        for j, v in enumerate(U):
            arr[i].re[j] = float(v.real)
            arr[i].im[j] = float(v.imag)
    bits = np.ascontiguousarray(np.asarray(bitstrings, dtype=np.uint8).reshape(-1, n))
    opts = QtnPlanOpts()
    L.qtn_plan_opts_default(byref(opts))
    opts.k, opts.max_rank, opts.k_max, opts.seed = k, max_rank, k_max, seed
    opts.ga_pop, opts.ga_iters = ga_pop, ga_iters
    opts.precision = PRECISIONS[precision]
    opts.fuse_chains = 1 if fuse_chains else 0
    opts.exec_mode = {"auto": -1, "wide": 0, "slice": 1}[exec_mode]
    cv = None
    if cut_vars is not None:
        cv = _u32(cut_vars)
        opts.k = len(cv)
        opts.cut_vars = cv.ctypes.data_as(POINTER(c_uint32))
    h = c_void_p()
    _check(L.qtn_plan_circuit(n, arr, len(gates), bits.ctypes.data_as(POINTER(c_uint8)), bits.shape[0],
                              byref(opts), byref(h)))
    return Plan(h.value, n, bits.shape[0])


def batch_contract(plans: Sequence["Plan"], ranges: Sequence[tuple], stream: Optional[int] = None):
    """Several plans (bound with exec_mode="slice", one wave each) in one
    persistent launch; returns one list of partials per plan."""
    n = len(plans)
    hs = (c_void_p * n)(*[p._h.value for p in plans])
    lo = (c_uint64 * n)(*[int(r[0]) for r in ranges])
    hi = (c_uint64 * n)(*[int(r[1]) for r in ranges])
    out = (QtnPartial * sum(p.n_bitstrings for p in plans))()
    _check(lib().qtn_batch_contract(hs, n, lo, hi, c_void_p(stream or 0), out))
    res, at = [], 0
    for p in plans:
        res.append([out[at + i] for i in range(p.n_bitstrings)])
        at += p.n_bitstrings
    return res


def plan_instance(inst, **kw) -> Plan:
    """qtn_plan for an instances.Instance."""
    return qtn_plan(inst.n, inst.edges, inst.p, inst.gamma, inst.beta, inst.bitstrings, **kw)


def _graph(n: int, edges):
    e = _u32(edges).reshape(-1)
    return QtnGraph(n, len(e) // 2, e.ctypes.data_as(POINTER(c_uint32))), e


def _sets(cut_sets) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(cut_sets, dtype=np.uint32))
    if a.ndim != 2:
        raise ValueError("cut_sets must be a 2-D array (sets x k)")
    return a


def cost_features(n: int, edges, p: int, cut_sets) -> np.ndarray:
    """Model input features of each cut set (rows of cut_sets)."""
    g, _e = _graph(n, edges)
    a = _sets(cut_sets)
    out = np.zeros((a.shape[0], COST_FEATURES), dtype=np.float32)
    _check(lib().qtn_cost_features(byref(g), p, a.ctypes.data_as(POINTER(c_uint32)), a.shape[0],
                                   a.shape[1], out.ctypes.data_as(POINTER(ctypes.c_float))))
    return out


def cost_exact(n: int, edges, p: int, cut_sets, threads: int = 1):
    """Exact (width, log2 cost) of each cut set."""
    g, _e = _graph(n, edges)
    a = _sets(cut_sets)
    w = np.zeros(a.shape[0], dtype=np.int32)
    c = np.zeros(a.shape[0], dtype=np.float64)
    _check(lib().qtn_cost_exact(byref(g), p, a.ctypes.data_as(POINTER(c_uint32)), a.shape[0],
                                a.shape[1], w.ctypes.data_as(POINTER(c_int32)),
                                c.ctypes.data_as(POINTER(c_double)), threads))
    return w, c


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(POINTER(ctypes.c_float))


class CostMLP:
    """Owns one qtn_mlp_t (parameters and activations on the current device)."""

    def __init__(self, in_dim: int = COST_FEATURES, hidden: int = 256, n_hidden: int = 3,
                 out_dim: int = 2, max_batch: int = 4096, seed: int = 0):
        h = c_void_p()
        _check(lib().qtn_mlp_create(in_dim, hidden, n_hidden, out_dim, max_batch, seed, byref(h)))
        self._h = h
        self.dims = [in_dim] + [hidden] * n_hidden + [out_dim]
        self.max_batch = max_batch

    def __del__(self):
        try:
            if self._h is not None and self._h.value:
                lib().qtn_mlp_destroy(self._h)
                self._h = None
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def num_params(self) -> int:
        c = c_uint64()
        _check(lib().qtn_mlp_num_params(self._h, byref(c)))
        return c.value

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params(), dtype=np.float32)
        _check(lib().qtn_mlp_get_params(self._h, _fptr(out), out.size))
        return out

    def get_grads(self) -> np.ndarray:
        out = np.zeros(self.num_params(), dtype=np.float32)
        _check(lib().qtn_mlp_get_grads(self._h, _fptr(out), out.size))
        return out

    def set_params(self, flat):
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32))
        _check(lib().qtn_mlp_set_params(self._h, _fptr(a), a.size))

    def unflatten(self, flat):
        """[(W, b)] per layer from a flat parameter vector."""
        out, o = [], 0
        for din, dout in zip(self.dims[:-1], self.dims[1:]):
            W = np.asarray(flat[o:o + din * dout]).reshape(din, dout)
            o += din * dout
            b = np.asarray(flat[o:o + dout])
            o += dout
            out.append((W, b))
        return out

    def set_normalization(self, x_mean, x_std, y_mean, y_std):
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in
                (x_mean, x_std, y_mean, y_std)]
        _check(lib().qtn_mlp_set_normalization(self._h, *[_fptr(a) for a in arrs]))

    def forward(self, x_ptr: int, batch: int, y_ptr: int, stream: Optional[int] = None):
        _check(lib().qtn_mlp_forward(self._h, c_void_p(x_ptr), batch, c_void_p(y_ptr),
                                     c_void_p(stream or 0)))

    def train_step(self, x_ptr: int, t_ptr: int, batch: int, lr: float,
                   stream: Optional[int] = None) -> float:
        loss = ctypes.c_float()
        _check(lib().qtn_mlp_train_step(self._h, c_void_p(x_ptr), c_void_p(t_ptr), batch, lr,
                                        c_void_p(stream or 0), byref(loss)))
        return loss.value


def cut_search(n: int, edges, p: int, k: int, pop: int = 11, iters: int = 4, seed: int = 0,
               model: Optional[CostMLP] = None, offspring_factor: int = 16):
    """Cut set of size k and the search statistics (model-guided when `model`)."""
    g, _e = _graph(n, edges)
    out = np.zeros(max(k, 1), dtype=np.uint32)
    st = QtnSearchStats()
    _check(lib().qtn_cut_search(byref(g), p, k, pop, iters, seed,
                                model.handle if model is not None else None, offspring_factor,
                                out.ctypes.data_as(POINTER(c_uint32)), byref(st)))
    return [int(v) for v in out[:k]], {"seconds": st.seconds, "exact_evals": st.exact_evals,
                                       "model_evals": st.model_evals, "width": st.width,
                                       "log2_cost": st.log2_cost}
