"""ctypes binding of libqft.so (the C ABI in include/qft.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  PyTorch is used for device memory and streams.  If the shared
library is missing this module raises at import time; there is no fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqft.so")

QFT_NORM_UNITARY = 0
QFT_NORM_NONE = 1
QFT_NORM_INV_N = 2
QFT_C64 = 0x0
QFT_C128 = 0x1
QFT_ORDER_NATURAL = 0x0
QFT_ORDER_BITREV = 0x2
QFT_SCHEDULE_FUSED = 0x0
QFT_SCHEDULE_GATES = 0x4
QFT_PLAN_NO_WORKSPACE = 0x8
QFT_INVERSE = 0x10
QFT_PLAN_TUNED = 0x20
QFT_CUTOFF_EXACT = -1
QFT_MAX_PASSES = 8
QFT_RNG_GAUSSIAN = 0
QFT_RNG_UNIFORM = 1
QFT_BATCH_EAGER = 0x1

QFT_OK = 0
QFT_ERR_INVALID = -1
QFT_ERR_UNSUPPORTED = -2
QFT_ERR_NOMEM = -3
QFT_ERR_HIP = -4
QFT_ERR_POINTER = -5
QFT_ERR_BUSY = -6

NORMS = {"unitary": QFT_NORM_UNITARY, "none": QFT_NORM_NONE, "inv_n": QFT_NORM_INV_N}


class QftError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libqft error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("tile_log2", ctypes.c_int), ("radix_log2", ctypes.c_int),
                ("spec_log2", ctypes.c_int), ("rev_spec_log2", ctypes.c_int),
                ("nontemporal", ctypes.c_int),
                ("pass_bits", ctypes.c_int * QFT_MAX_PASSES),
                ("pass_tile_log2", ctypes.c_int * QFT_MAX_PASSES)]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("cutoff", ctypes.c_int), ("norm", ctypes.c_int),
        ("layout", ctypes.c_int), ("num_passes", ctypes.c_int),
        ("pass_lo", ctypes.c_int * QFT_MAX_PASSES),
        ("pass_bits", ctypes.c_int * QFT_MAX_PASSES),
        ("pass_spec", ctypes.c_int * QFT_MAX_PASSES),
        ("pass_reverse", ctypes.c_int * QFT_MAX_PASSES),
        ("pass_kernel", ctypes.c_int * QFT_MAX_PASSES),
        ("pass_streaming", ctypes.c_int * QFT_MAX_PASSES),
        ("config", Config),
        ("gates_h", ctypes.c_longlong), ("gates_cr", ctypes.c_longlong),
        ("gates_swap", ctypes.c_longlong),
        ("state_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
        ("table_bytes", ctypes.c_size_t), ("hbm_bytes", ctypes.c_size_t),
    ]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if isinstance(v, Config):
                v = {f: getattr(v, f) for f, _ in Config._fields_}
            elif hasattr(v, "__len__"):
                v = list(v)[: self.num_passes]
            d[name] = v
        return d


def _init_torch_device():
    """Let torch bring up the HIP runtime first.  The library links the same
    libamdhip64 soname, so it shares torch's runtime, device view and
    streams."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def _load():
    _init_torch_device()
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2606_18981_amd.build` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I = ctypes.c_int
    sig = {
        "qft_plan": (P, [I, I, I, I]),
        "qft_plan_config": (P, [I, I, I, I, ctypes.POINTER(Config)]),
        "qft_execute": (I, [P, P, P]),
        "qft_execute_ws": (I, [P, P, P, P]),
        "qft_execute_norm": (I, [P, P, P, P, P]),
        "qft_execute_norm_static": (I, [P, P, P, P, P]),
        "qft_destroy": (None, [P]),
        "qft_last_error": (ctypes.c_char_p, []),
        "qft_plan_info": (I, [P, ctypes.POINTER(PlanInfo)]),
        "qft_plan_device_bytes": (ctypes.c_size_t, [P]),
        "qft_plan_describe": (I, [I, I, I, I, ctypes.POINTER(Config), ctypes.POINTER(PlanInfo)]),
        "qft_plan_set_timing": (I, [P, I]),
        "qft_plan_pass_times": (I, [P, ctypes.POINTER(ctypes.c_double), I,
                                    ctypes.POINTER(ctypes.c_longlong)]),
        "qft_execute_batch": (I, [ctypes.POINTER(P), ctypes.POINTER(P), I, P]),
        "qft_execute_batch_ex": (I, [ctypes.POINTER(P), ctypes.POINTER(P), I, I, P]),
        "qft_fill_random": (I, [P, I, I, I, ctypes.c_uint64, ctypes.c_uint64, P]),
        "qft_tune": (I, [I, I, I, I, P, I, ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_double)]),
        "qft_tune_batch": (I, [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), I, I, I,
                               ctypes.POINTER(P), I, ctypes.POINTER(Config),
                               ctypes.POINTER(ctypes.c_double)]),
        "qft_tune_lookup": (I, [I, I, I, ctypes.POINTER(Config)]),
        "qft_tune_insert": (I, [I, I, I, ctypes.POINTER(Config), ctypes.c_double]),
        "qft_tune_clear": (I, []),
        "qft_tune_save": (I, [ctypes.c_char_p]),
        "qft_tune_load": (I, [ctypes.c_char_p]),
        "qft_pad": (I, [P, ctypes.c_size_t, P, I, I, P]),
        "qft_circuit_create": (P, [I, I]),
        "qft_circuit_destroy": (None, [P]),
        "qft_circuit_add_1q": (I, [P, I, ctypes.POINTER(ctypes.c_double)]),
        "qft_circuit_add_controlled": (I, [P, I, I, ctypes.POINTER(ctypes.c_double)]),
        "qft_circuit_add_swap": (I, [P, I, I]),
        "qft_circuit_compile": (I, [P, I]),
        "qft_circuit_info": (I, [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "qft_circuit_describe": (I, [P, I, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int), I]),
        "qft_circuit_execute": (I, [P, P, P]),
        "qft_qubits_for": (I, [ctypes.c_size_t]),
        "qft_compare_workspace_bytes": (ctypes.c_size_t, [I]),
        "qft_compare": (I, [P, P, I, I, P, P, P]),
        "qft_execute_compare_workspace_bytes": (ctypes.c_size_t, [P]),
        "qft_execute_compare": (I, [P, P, P, P, P, P, P]),
        "qft_aqft_expected_error": (ctypes.c_double, [I, I]),
        "qft_select_cutoff": (I, [I, ctypes.c_double]),
        "qft_debug_pass_desc_size": (ctypes.c_size_t, []),
        "qft_debug_pass": (I, [I, I, I, I, ctypes.POINTER(Config), I, P, ctypes.c_size_t,
                               ctypes.POINTER(ctypes.c_int)]),
        "qft_debug_tables": (I, [I, I, I, I, ctypes.POINTER(Config), P, ctypes.c_size_t,
                                 ctypes.POINTER(ctypes.c_size_t)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def last_error() -> str:
    return (lib.qft_last_error() or b"").decode()


def _check(rc: int):
    if rc != QFT_OK:
        raise QftError(rc, last_error())


def layout_flags(dtype="c64", order="natural", schedule="fused", inverse: bool = False) -> int:
    f = QFT_INVERSE if inverse else 0
    if dtype in ("c128", "complex128") or str(dtype) == "torch.complex128":
        f |= QFT_C128
    elif not (dtype in ("c64", "complex64") or str(dtype) == "torch.complex64"):
        raise ValueError(f"unsupported dtype {dtype!r}")
    if order == "bitrev":
        f |= QFT_ORDER_BITREV
    elif order != "natural":
        raise ValueError(f"unknown order {order!r}")
    if schedule == "gates":
        f |= QFT_SCHEDULE_GATES
    elif schedule != "fused":
        raise ValueError(f"unknown schedule {schedule!r}")
    return f


def _norm(norm) -> int:
    return NORMS[norm] if isinstance(norm, str) else int(norm)


def _config(config) -> Optional[Config]:
    if config is None:
        return None
    if isinstance(config, Config):
        return config
    c = Config()
    for k, v in dict(config).items():
        if k in ("pass_bits", "pass_tile_log2"):
            arr = getattr(c, k)
            for i, b in enumerate(list(v)[:QFT_MAX_PASSES]):
                arr[i] = int(b)
        else:
            setattr(c, k, int(v))
    return c


def describe(n: int, cutoff: int = -1, norm="unitary", dtype="c64", order="natural",
             schedule="fused", config=None, inverse: bool = False) -> PlanInfo:
    """Host-only planner description (no device use)."""
    info = PlanInfo()
    c = _config(config)
    _check(lib.qft_plan_describe(n, cutoff, _norm(norm),
                                 layout_flags(dtype, order, schedule, inverse),
                                 ctypes.byref(c) if c is not None else None, ctypes.byref(info)))
    return info


def _stream_handle(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """A planned 2^n-point transform (owns device tables and workspace)."""

    def __init__(self, n: int, cutoff: int = -1, norm="unitary", dtype="c64",
                 order="natural", schedule="fused", config=None, workspace: bool = True,
                 inverse: bool = False, tuned: bool = False):
        """tuned=True (and no config): take the tuning table's entry for this
        shape when there is one (QFT_PLAN_TUNED)."""
        self.n = n
        self.cutoff = cutoff
        self.layout = layout_flags(dtype, order, schedule, inverse)
        if not workspace:
            self.layout |= QFT_PLAN_NO_WORKSPACE
        if tuned:
            self.layout |= QFT_PLAN_TUNED
        self.c128 = bool(self.layout & QFT_C128)
        c = _config(config)
        h = lib.qft_plan_config(n, cutoff, _norm(norm), self.layout,
                                ctypes.byref(c) if c is not None else None)
        if not h:
            raise QftError(QFT_ERR_INVALID, last_error())
        self._h = ctypes.c_void_p(h)
        self.info = PlanInfo()
        _check(lib.qft_plan_info(self._h, ctypes.byref(self.info)))

    @property
    def handle(self):
        return self._h

    @property
    def device_bytes(self) -> int:
        """Device memory the plan holds (tables, workspace, norm partials)."""
        return int(lib.qft_plan_device_bytes(self._h))

    def _check_tensor(self, x):
        import torch
        want = torch.complex128 if self.c128 else torch.complex64
        if not x.is_cuda:
            raise ValueError("tensor must be on the GPU")
        if x.dtype != want:
            raise ValueError(f"tensor dtype {x.dtype} does not match the plan ({want})")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if x.numel() != (1 << self.n):
            raise ValueError(f"tensor has {x.numel()} elements, plan needs {1 << self.n}")

    def execute(self, x, stream=None, workspace=None, norm_out=None, ref=None,
                metrics_out=None, cmp_workspace=None):
        """In-place transform of the CUDA tensor x (complex64/128, 2^n elements).
        With norm_out (a float64 CUDA tensor), ||x||_2 of the input is written
        to norm_out[0] by the same call (the paper's scale_in).  With ref (a
        tensor like x holding a reference output) and metrics_out (a float64
        CUDA tensor of len(METRIC_NAMES)), the accuracy metrics of the output
        against ref are written to metrics_out by the same call, the last
        pass comparing the tiles it stores (qft_execute_compare); see
        metrics_dict().  cmp_workspace: a CUDA tensor of at least
        compare_workspace_bytes() bytes, else one kept by the plan."""
        self._check_tensor(x)
        if workspace is not None and \
                workspace.numel() * workspace.element_size() < self.info.workspace_bytes:
            raise ValueError("workspace too small")
        ws = None if workspace is None else ctypes.c_void_p(workspace.data_ptr())
        if ref is not None:
            if norm_out is not None:
                raise ValueError("norm_out and ref cannot be combined in one call")
            return self._execute_compare(x, ref, metrics_out, ws, cmp_workspace, stream)
        if metrics_out is not None:
            raise ValueError("metrics_out needs ref")
        if norm_out is not None:
            import torch
            if not (norm_out.is_cuda and norm_out.dtype == torch.float64 and norm_out.numel() >= 1):
                raise ValueError("norm_out must be a float64 CUDA tensor")
            rc = lib.qft_execute_norm(self._h, ctypes.c_void_p(x.data_ptr()), ws,
                                      ctypes.c_void_p(norm_out.data_ptr()), _stream_handle(stream))
        elif ws is None:
            rc = lib.qft_execute(self._h, ctypes.c_void_p(x.data_ptr()), _stream_handle(stream))
        else:
            rc = lib.qft_execute_ws(self._h, ctypes.c_void_p(x.data_ptr()), ws,
                                    _stream_handle(stream))
        _check(rc)
        return x

    def compare_workspace_bytes(self) -> int:
        """Device workspace an execute with a reference needs, in bytes."""
        return int(lib.qft_execute_compare_workspace_bytes(self._h))

    def _execute_compare(self, x, ref, metrics_out, ws, cmp_workspace, stream):
        import torch
        self._check_tensor(ref)
        if metrics_out is None or not (metrics_out.is_cuda and metrics_out.dtype == torch.float64
                                       and metrics_out.is_contiguous()
                                       and metrics_out.numel() >= len(METRIC_NAMES)):
            raise ValueError(f"metrics_out must be a contiguous float64 CUDA tensor of "
                             f"{len(METRIC_NAMES)} elements")
        nb = self.compare_workspace_bytes()
        if cmp_workspace is None:
            cw = getattr(self, "_cmp_ws", None)
            if cw is None or cw.numel() * 8 < nb or cw.device != x.device:
                cw = torch.empty(max(1, (nb + 7) // 8), dtype=torch.float64, device=x.device)
                self._cmp_ws = cw
            cmp_workspace = cw
        elif not cmp_workspace.is_cuda or \
                cmp_workspace.numel() * cmp_workspace.element_size() < nb:
            raise ValueError("cmp_workspace too small")
        _check(lib.qft_execute_compare(self._h, ctypes.c_void_p(x.data_ptr()), ws,
                                       ctypes.c_void_p(ref.data_ptr()),
                                       ctypes.c_void_p(cmp_workspace.data_ptr()),
                                       ctypes.c_void_p(metrics_out.data_ptr()),
                                       _stream_handle(stream)))
        return x

    def set_timing(self, enable: bool = True):
        _check(lib.qft_plan_set_timing(self._h, int(bool(enable))))

    def pass_times(self):
        """(mean ms per launch list, number of timed executes); clears them."""
        k = max(1, self.info.num_passes)
        buf = (ctypes.c_double * k)()
        ex = ctypes.c_longlong(0)
        _check(lib.qft_plan_pass_times(self._h, buf, k, ctypes.byref(ex)))
        return list(buf), int(ex.value)

    def close(self):
        self._cmp_ws = None
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.qft_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _batch_arrays(plans, tensors):
    if len(plans) != len(tensors):
        raise ValueError("plans and tensors differ in length")
    for p, t in zip(plans, tensors):
        p._check_tensor(t)
    cnt = len(plans)
    ph = (ctypes.c_void_p * cnt)(*[p.handle.value for p in plans])
    tp = (ctypes.c_void_p * cnt)(*[t.data_ptr() for t in tensors])
    return ph, tp, cnt


def execute_batch(plans: Sequence[Plan], tensors, stream=None, graph: bool = True):
    """Uneven transforms (plans[i] on tensors[i]) launched pass level by pass
    level over all transforms' tiles.

    graph=True replays a captured HIP graph (captured on the first call for
    this set of plans and tensors); graph=False launches directly."""
    ph, tp, cnt = _batch_arrays(plans, tensors)
    flags = 0 if graph else QFT_BATCH_EAGER
    _check(lib.qft_execute_batch_ex(ph, tp, cnt, flags, _stream_handle(stream)))


class Batch:
    """A fixed set of (plan, tensor) pairs run as one batch: the arguments
    are checked and marshalled once, so that each execute() is one call into
    the library (which replays the set's captured graph)."""

    def __init__(self, plans: Sequence[Plan], tensors):
        self._ph, self._tp, self._cnt = _batch_arrays(plans, tensors)
        self._keep = (list(plans), list(tensors))  # keep them alive

    def execute(self, stream=None, graph: bool = True):
        flags = 0 if graph else QFT_BATCH_EAGER
        _check(lib.qft_execute_batch_ex(self._ph, self._tp, self._cnt, flags,
                                        _stream_handle(stream)))


def fill_random(x, dist="gaussian", seed: int = 0, stream_id: int = 0, stream=None):
    """Fill a CUDA complex tensor of 2^n elements from the device Philox generator."""
    import torch
    n = x.numel().bit_length() - 1
    if x.numel() != (1 << n) or not x.is_cuda or not x.is_contiguous():
        raise ValueError("need a contiguous CUDA tensor of 2^n elements")
    if x.dtype == torch.complex128:
        lay = QFT_C128
    elif x.dtype == torch.complex64:
        lay = QFT_C64
    else:
        raise ValueError("need complex64 or complex128")
    d = QFT_RNG_GAUSSIAN if dist == "gaussian" else QFT_RNG_UNIFORM
    _check(lib.qft_fill_random(ctypes.c_void_p(x.data_ptr()), n, lay, d, seed, stream_id,
                               _stream_handle(stream)))
    return x


# ---- autotuner ------------------------------------------------------------

def _cfg_dict(c: Config) -> dict:
    d = {f: getattr(c, f) for f, _ in Config._fields_
         if f not in ("pass_bits", "pass_tile_log2", "nontemporal")}
    if c.nontemporal:
        d["nontemporal"] = c.nontemporal
    pb = [int(x) for x in c.pass_bits if int(x) > 0]
    if pb:
        d["pass_bits"] = pb
    pt = [int(x) for x in c.pass_tile_log2]
    if any(pt):
        d["pass_tile_log2"] = pt[:max(i + 1 for i, x in enumerate(pt) if x)]
    return d


def tune(n: int, cutoff: int = -1, norm="unitary", dtype="c64", order="natural",
         data=None, reps: int = 3):
    """Time the candidate configurations on `data` (a CUDA tensor of 2^n
    elements, overwritten) and record the fastest in the tuning table."""
    lay = layout_flags(dtype, order)
    best = Config()
    ms = ctypes.c_double(0)
    _check(lib.qft_tune(n, cutoff, _norm(norm), lay, ctypes.c_void_p(data.data_ptr()), reps,
                        ctypes.byref(best), ctypes.byref(ms)))
    return _cfg_dict(best), ms.value


def tune_batch(ns, cutoffs, tensors, norm="unitary", dtype="c64", order="natural", reps=3):
    """One configuration for a whole batch (timed through the batched launch)."""
    cnt = len(ns)
    na = (ctypes.c_int * cnt)(*[int(v) for v in ns])
    ka = (ctypes.c_int * cnt)(*[int(v) for v in cutoffs])
    da = (ctypes.c_void_p * cnt)(*[t.data_ptr() for t in tensors])
    best = Config()
    ms = ctypes.c_double(0)
    _check(lib.qft_tune_batch(na, ka, cnt, _norm(norm), layout_flags(dtype, order), da, reps,
                              ctypes.byref(best), ctypes.byref(ms)))
    return _cfg_dict(best), ms.value


def tune_lookup(n, cutoff=-1, dtype="c64", order="natural"):
    c = Config()
    rc = lib.qft_tune_lookup(n, cutoff, layout_flags(dtype, order), ctypes.byref(c))
    return _cfg_dict(c) if rc == QFT_OK else None


def tune_insert(n, cutoff, dtype, order, config, ms=0.0):
    c = _config(config)
    _check(lib.qft_tune_insert(n, cutoff, layout_flags(dtype, order), ctypes.byref(c), ms))


def tune_clear():
    lib.qft_tune_clear()


def tune_save(path):
    _check(lib.qft_tune_save(str(path).encode()))


def tune_load(path) -> int:
    rc = lib.qft_tune_load(str(path).encode())
    if rc < 0:
        raise QftError(rc, last_error())
    return rc


# ---- accuracy metrics (include/qft_metrics.h) ------------------------------

METRIC_NAMES = ("rel_l2", "max_err", "fidelity", "leakage", "norm_y", "norm_ref", "argmax")


def expected_error(n: int, cutoff: int) -> float:
    """Expected rel-L2 error of the range-k AQFT for i.i.d. complex Gaussian
    inputs (closed form, host); negative when too costly to evaluate."""
    return float(lib.qft_aqft_expected_error(n, cutoff))


def select_cutoff(n: int, rel_l2_budget: float) -> int:
    """Smallest cutoff whose expected error meets the budget (host)."""
    k = int(lib.qft_select_cutoff(n, float(rel_l2_budget)))
    if k < 0:
        raise ValueError("invalid n or budget")
    return k


def compare(y, ref, stream=None, workspace=None, out=None, as_dict=True):
    """Accuracy metrics of y against ref (CUDA tensors of one complex dtype and
    2^n elements), computed on the device in FP64.  Returns a dict; `out`
    (a float64 CUDA tensor of 7 elements) receives the raw metrics.  With
    as_dict=False, returns `out` without waiting for the device."""
    import torch
    if y.dtype != ref.dtype or y.numel() != ref.numel():
        raise ValueError("y and ref must have the same dtype and size")
    if not (y.is_cuda and ref.is_cuda and y.is_contiguous() and ref.is_contiguous()):
        raise ValueError("y and ref must be contiguous CUDA tensors")
    N = y.numel()
    n = N.bit_length() - 1
    if N != 1 << n:
        raise ValueError("size must be a power of two")
    lay = layout_flags(y.dtype)
    if workspace is None:
        nb = int(lib.qft_compare_workspace_bytes(n))
        workspace = torch.empty(max(1, nb // 8), dtype=torch.float64, device=y.device)
    if out is None:
        out = torch.empty(len(METRIC_NAMES), dtype=torch.float64, device=y.device)
    _check(lib.qft_compare(ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(ref.data_ptr()), n, lay,
                           ctypes.c_void_p(workspace.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                           _stream_handle(stream)))
    return metrics_dict(out) if as_dict else out


def metrics_dict(out) -> dict:
    """The metrics array of compare() or Plan.execute(ref=...) as a dict
    (synchronises with the device to read it)."""
    vals = out[: len(METRIC_NAMES)].cpu().tolist()
    d = dict(zip(METRIC_NAMES, vals))
    d["argmax"] = int(d["argmax"])
    return d


# ---- lengths that are not powers of two --------------------------------------

def padded(x, stream=None):
    """A new CUDA tensor of 2^ceil(log2 len(x)) elements: x followed by zeros
    (one device pass).  Transforming it gives DFT_{2^n} of the padded input,
    as the method defines for such lengths, not DFT_len(x)."""
    import torch
    if not (x.is_cuda and x.is_contiguous() and x.dim() == 1):
        raise ValueError("x must be a contiguous 1-D CUDA tensor")
    n = int(lib.qft_qubits_for(x.numel()))
    if n < 0:
        raise ValueError("length out of range")
    n = max(n, 1)  # plans take at least one qubit
    out = torch.empty(1 << n, dtype=x.dtype, device=x.device)
    _check(lib.qft_pad(ctypes.c_void_p(x.data_ptr()), x.numel(), ctypes.c_void_p(out.data_ptr()),
                       n, layout_flags(x.dtype), _stream_handle(stream)))
    return out


# ---- general fused circuits (include/qft_circuit.h) ---------------------------

def _mat8(u):
    import numpy as np
    m = np.asarray(u, dtype=np.complex128).reshape(2, 2)
    flat = np.empty(8, dtype=np.float64)
    flat[0::2] = m.real.ravel()
    flat[1::2] = m.imag.ravel()
    return (ctypes.c_double * 8)(*flat.tolist())


class Circuit:
    """A list of one- and two-qubit gates on n qubits, run in fused passes
    (runs of consecutive gates whose qubits fit in one tile share one HBM
    pass)."""

    def __init__(self, n: int, dtype="c64"):
        self.n = n
        self.c128 = bool(layout_flags(dtype) & QFT_C128)
        h = lib.qft_circuit_create(n, layout_flags(dtype))
        if not h:
            raise QftError(QFT_ERR_INVALID, last_error())
        self._h = ctypes.c_void_p(h)

    def add_1q(self, q, u):
        _check(lib.qft_circuit_add_1q(self._h, q, _mat8(u)))
        return self

    def add_controlled(self, control, target, u):
        _check(lib.qft_circuit_add_controlled(self._h, control, target, _mat8(u)))
        return self

    def add_swap(self, a, b):
        _check(lib.qft_circuit_add_swap(self._h, a, b))
        return self

    def compile(self, tile_qubits: int = 0):
        _check(lib.qft_circuit_compile(self._h, tile_qubits))
        return self

    def describe(self, tile_qubits: int = 0, max_passes: int = 4096):
        """Host-only grouping: (first gate of each pass, tile bits of each pass)."""
        gb = (ctypes.c_int * max_passes)()
        tb = (ctypes.c_int * max_passes)()
        rc = lib.qft_circuit_describe(self._h, tile_qubits, gb, tb, max_passes)
        _check(min(rc, 0))
        k = min(rc, max_passes)
        return list(gb)[:k], list(tb)[:k]

    def info(self):
        g, p = ctypes.c_int(0), ctypes.c_int(0)
        _check(lib.qft_circuit_info(self._h, ctypes.byref(g), ctypes.byref(p)))
        return {"gates": g.value, "passes": p.value}

    def execute(self, x, stream=None):
        import torch
        want = torch.complex128 if self.c128 else torch.complex64
        if not (x.is_cuda and x.dtype == want and x.is_contiguous() and x.numel() == 1 << self.n):
            raise ValueError("x must be a contiguous CUDA tensor of 2^n elements of the "
                             "circuit's dtype")
        _check(lib.qft_circuit_execute(self._h, ctypes.c_void_p(x.data_ptr()),
                                       _stream_handle(stream)))
        return x

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.qft_circuit_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
