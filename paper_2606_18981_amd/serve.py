"""ctypes binding of the request server (include/qft_serve.h).

The scheduling loop, admission, device input generation and transforms all
run in libqft.so; this module only builds the request arrays and summarises
the per-request timestamps.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import qft as Q

lib = Q.lib


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("cutoff", ctypes.c_int), ("norm", ctypes.c_int),
                ("layout", ctypes.c_int), ("dist", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("arrival", ctypes.c_double), ("out", ctypes.c_void_p)]


class RequestResult(ctypes.Structure):
    _fields_ = [("arrival", ctypes.c_double), ("admitted", ctypes.c_double),
                ("completed", ctypes.c_double), ("status", ctypes.c_int),
                ("stream", ctypes.c_int), ("bytes", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("peak_reserved_bytes", ctypes.c_size_t), ("peak_inflight", ctypes.c_int),
                ("wall_seconds", ctypes.c_double), ("hbm_bytes", ctypes.c_double),
                ("plan_bytes", ctypes.c_size_t)]


_P = ctypes.c_void_p
lib.qft_server_create.restype = _P
lib.qft_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int]
lib.qft_server_destroy.restype = None
lib.qft_server_destroy.argtypes = [_P]
lib.qft_server_prepare.restype = ctypes.c_int
lib.qft_server_prepare.argtypes = [_P, ctypes.POINTER(Request), ctypes.c_int]
lib.qft_server_run.restype = ctypes.c_int
lib.qft_server_run.argtypes = [_P, ctypes.POINTER(Request), ctypes.c_int,
                               ctypes.POINTER(RequestResult), ctypes.POINTER(ServerStats)]
lib.qft_server_simulate.restype = ctypes.c_int
lib.qft_server_simulate.argtypes = [ctypes.c_size_t, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                                    ctypes.POINTER(RequestResult), ctypes.POINTER(ServerStats)]


def requests_from_trace(trace, norm="unitary", order="natural", dist="gaussian", outs=None):
    """Request array from a trace dict (arrival, n, dtype, cutoff, seed)."""
    m = len(trace["arrival"])
    reqs = (Request * m)()
    d = Q.QFT_RNG_GAUSSIAN if dist == "gaussian" else Q.QFT_RNG_UNIFORM
    for i in range(m):
        r = reqs[i]
        r.n = int(trace["n"][i])
        r.cutoff = int(trace["cutoff"][i])
        r.norm = Q._norm(norm)
        r.layout = Q.layout_flags("c128" if int(trace["dtype"][i]) else "c64", order)
        r.dist = d
        r.seed = int(trace["seed"][i])
        r.arrival = float(trace["arrival"][i])
        r.out = outs[i].data_ptr() if outs is not None and outs[i] is not None else None
    return reqs


def _results(res, m):
    out = {f: np.array([getattr(res[i], f) for i in range(m)]) for f, _ in RequestResult._fields_}
    out["latency"] = out["completed"] - out["arrival"]
    return out


def _stats(st):
    return {f: getattr(st, f) for f, _ in ServerStats._fields_}


class Server:
    def __init__(self, budget_bytes: int, max_inflight: int = 64, num_streams: int = 4):
        h = lib.qft_server_create(int(budget_bytes), int(max_inflight), int(num_streams))
        if not h:
            raise Q.QftError(Q.QFT_ERR_INVALID, Q.last_error())
        self._h = ctypes.c_void_p(h)

    def prepare(self, reqs):
        Q._check(lib.qft_server_prepare(self._h, reqs, len(reqs)))

    def run(self, reqs):
        m = len(reqs)
        res = (RequestResult * m)()
        st = ServerStats()
        rc = lib.qft_server_run(self._h, reqs, m, res, ctypes.byref(st))
        if rc != Q.QFT_OK and rc != Q.QFT_ERR_HIP:
            raise Q.QftError(rc, Q.last_error())
        return _results(res, m), _stats(st)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.qft_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def simulate(budget_bytes, max_inflight, arrival, nbytes, service):
    """Run the scheduler against a simulated device with a virtual clock."""
    m = len(arrival)
    a = (ctypes.c_double * m)(*[float(x) for x in arrival])
    b = (ctypes.c_size_t * m)(*[int(x) for x in nbytes])
    s = (ctypes.c_double * m)(*[float(x) for x in service])
    res = (RequestResult * m)()
    st = ServerStats()
    Q._check(lib.qft_server_simulate(int(budget_bytes), int(max_inflight), a, b, s, m, res,
                                     ctypes.byref(st)))
    return _results(res, m), _stats(st)


def latency_summary(results) -> dict:
    lat = results["latency"][results["status"] == 0]
    if lat.size == 0:
        return {}
    return {
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p90_ms": float(np.percentile(lat, 90) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "p999_ms": float(np.percentile(lat, 99.9) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "max_ms": float(lat.max() * 1e3),
    }
