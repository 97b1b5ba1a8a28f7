"""Thin ctypes binding of libgeraf.so (declared in include/geraf.h).

Argument marshalling only: every step of the build and query path runs in
the native library.  Tensors are passed by pointer: torch CUDA tensors as
device pointers (with torch's current stream), numpy arrays as host
pointers.  The binding raises if the library has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgeraf.so")

GF_OK, GF_EINVAL, GF_ENOMEM, GF_EHIP, GF_EUNSUPPORTED, GF_EINTERNAL = 0, -1, -2, -3, -4, -5
FORM_FP32, FORM_BF16, FORM_FP8 = 0, 1, 2
KEEP_BF16, KEEP_FP8 = 1 << 1, 1 << 2
BUILD_DEVICE = 1 << 8
VARIANT_HOUSEHOLDER = 1 << 0
VARIANT_JITTER, VARIANT_JITTER_EXACT = 1 << 1, 1 << 2
FORMS = {"fp32": FORM_FP32, "bf16": FORM_BF16, "fp8": FORM_FP8}

EXPORTED = ["gf_build_forest", "gf_build_forest_ex", "gf_free_forest", "gf_forest_info", "gf_export_tree", "gf_query",
            "gf_query_multi", "gf_multi_stats", "gf_query_trace", "gf_query_trace_ex",
            "gf_query_noalloc",
            "gf_fp8_tables", "gf_hbm_probe",
            "gf_last_query_timing", "gf_last_error", "gf_version", "gf_device_bytes"]
MULTI_AUTOTUNE, MULTI_EAGER = 1, 2


class Job(ctypes.Structure):
    """gf_job (include/geraf.h)."""
    _fields_ = [("forest", ctypes.c_void_p), ("Q", ctypes.c_void_p), ("nq", ctypes.c_int64),
                ("k", ctypes.c_int32), ("checks", ctypes.c_int32),
                ("checks_per_query", ctypes.c_void_p), ("eps", ctypes.c_double),
                ("form", ctypes.c_int32), ("rerank", ctypes.c_int32), ("ids", ctypes.c_void_p),
                ("dists", ctypes.c_void_p)]

_lib = None


class GerafError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"geraf status {status}: {msg}")
        self.status = status


def load():
    """Load libgeraf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1603_09596_amd.build` (no fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double)
    lib.gf_build_forest.argtypes = [P, i64, i32, i32, i32, i32, u64, u32, P, ctypes.POINTER(P)]
    lib.gf_build_forest_ex.argtypes = [P, i64, i32, i32, i32, i32, u64, u32, u32, P,
                                       ctypes.POINTER(P)]
    lib.gf_free_forest.argtypes = [P]
    lib.gf_forest_info.argtypes = [P, P, P, P, P, P, P]
    lib.gf_export_tree.argtypes = [P, P, P, P, P, P]
    lib.gf_query.argtypes = [P, P, i64, i32, i32, P, f64, i32, i32, P, P, P]
    lib.gf_query_noalloc.argtypes = [P, P, i64, i32, i32, P, f64, i32, i32, P, P, P]
    lib.gf_query_trace.argtypes = [P, P, i64, i32, P, f64, P, P, P, P]
    lib.gf_query_trace_ex.argtypes = [P, P, i64, i32, P, f64, i32, P, P, P, P]
    lib.gf_query_multi.argtypes = [ctypes.POINTER(Job), i32, u32, P]
    lib.gf_multi_stats.argtypes = [P, P, P]
    lib.gf_fp8_tables.argtypes = [P, P, P, i32, P]
    lib.gf_hbm_probe.argtypes = [P, i64, i32, P, P]
    lib.gf_last_query_timing.argtypes = [P, i32, P, P]
    lib.gf_last_error.restype = ctypes.c_char_p
    lib.gf_device_bytes.restype = ctypes.c_int64
    lib.gf_device_bytes.argtypes = []
    lib.gf_version.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("gf_last_error", "gf_version", "gf_device_bytes"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != GF_OK:
        raise GerafError(status, load().gf_last_error().decode(errors="replace"))


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x):
    """Raw pointer of a numpy array or a torch tensor (contiguous)."""
    if x is None:
        return None
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr())
    if not x.flags["C_CONTIGUOUS"]:
        raise ValueError("array must be C-contiguous")
    return x.ctypes.data_as(ctypes.c_void_p)


def _stream_of(*xs):
    for x in xs:
        if _is_torch(x) and x.is_cuda:
            import torch
            return ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    return None


def version() -> str:
    return load().gf_version().decode()


class Forest:
    """A built forest (owns the native handle)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        n, d, m, t, p, H = (ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(),
                            ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32())
        _check(load().gf_forest_info(handle, ctypes.byref(n), ctypes.byref(d), ctypes.byref(m),
                                     ctypes.byref(t), ctypes.byref(p), ctypes.byref(H)))
        self.n, self.d, self.m, self.t, self.leaf, self.H = (n.value, d.value, m.value, t.value,
                                                              p.value, H.value)

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h is not None:
            load().gf_free_forest(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def leaf_words(self) -> int:
        return max(1, (1 << self.H) // 32)

    def export_tree(self) -> dict:
        nint = (1 << self.H) - 1
        D = np.empty(self.t, np.int32)
        sd = np.empty((self.m, max(nint, 1)), np.int32)
        sv = np.empty((self.m, max(nint, 1)), np.float32)
        perm = np.empty((self.m, self.n), np.uint32)
        lo = np.empty((self.m, (1 << self.H) + 1), np.uint32)
        _check(load().gf_export_tree(self._h, _ptr(D), _ptr(sd), _ptr(sv), _ptr(perm), _ptr(lo)))
        return dict(n=self.n, d=self.d, m=self.m, t=self.t, p=self.leaf, H=self.H, D=D,
                    split_dim=sd[:, :nint], split_val=sv[:, :nint], perm=perm, leaf_off=lo)


def build_forest(X, m: int, t: int, leaf: int, seed: int, forms=(), stream=None,
                 householder: bool = False, device_build: bool = False,
                 jitter: Optional[str] = None) -> Forest:
    """gf_build_forest, or gf_build_forest_ex with the Householder isometry
    variant or split-value jitter (jitter="approx" or "exact": the diameter
    used).  X: [n, d] float32 (numpy or torch, host or device).  With
    device_build the trees are built on the GPU (GF_BUILD_DEVICE)."""
    n, d = X.shape
    mask = BUILD_DEVICE if device_build else 0
    for f in forms:
        mask |= {"bf16": KEEP_BF16, "fp8": KEEP_FP8}[f]
    h = ctypes.c_void_p()
    st = stream if stream is not None else _stream_of(X)
    variants = (VARIANT_HOUSEHOLDER if householder else 0) | \
        {None: 0, "approx": VARIANT_JITTER, "exact": VARIANT_JITTER_EXACT}[jitter]
    if variants:
        _check(load().gf_build_forest_ex(_ptr(X), n, d, m, t, leaf, seed & 0xFFFFFFFFFFFFFFFF, mask,
                                         variants, st, ctypes.byref(h)))
    else:
        _check(load().gf_build_forest(_ptr(X), n, d, m, t, leaf, seed & 0xFFFFFFFFFFFFFFFF, mask,
                                      st, ctypes.byref(h)))
    return Forest(h)


def query(F: Forest, Q, k: int, checks: int, ids, dists, checks_per_query=None, eps: float = 0.0,
          form: str = "fp32", rerank: int = 0, stream=None):
    """gf_query: fills ids [nq, k] int32 and dists [nq, k] float32 in place."""
    nq = Q.shape[0]
    st = stream if stream is not None else _stream_of(Q, ids)
    _check(load().gf_query(F.handle, _ptr(Q), nq, k, checks, _ptr(checks_per_query), float(eps),
                           FORMS[form], rerank, _ptr(ids), _ptr(dists), st))


def query_noalloc(F: Forest, Q, k: int, checks: int, ids, dists, checks_per_query=None,
                  eps: float = 0.0, form: str = "fp32", rerank: int = 0, stream=None):
    """gf_query_noalloc: gf_query's row path with no device allocation (the
    library's static scratch array); every tensor on the device."""
    nq = Q.shape[0]
    st = stream if stream is not None else _stream_of(Q, ids)
    _check(load().gf_query_noalloc(F.handle, _ptr(Q), nq, k, checks, _ptr(checks_per_query),
                                   float(eps), FORMS[form], rerank, _ptr(ids), _ptr(dists), st))


def query_multi(jobs, autotune: bool = False, eager: bool = False, stream=None):
    """gf_query_multi.  jobs: sequence of dicts with the keys of gf_query
    (forest, Q, k, checks, ids, dists; optional checks_per_query, eps, form,
    rerank), every tensor on the device; outputs are filled in place."""
    arr = (Job * len(jobs))()
    for i, j in enumerate(jobs):
        Q = j["Q"]
        arr[i] = Job(j["forest"].handle, _ptr(Q), Q.shape[0], j["k"], j.get("checks", 1),
                     _ptr(j.get("checks_per_query")), float(j.get("eps", 0.0)),
                     FORMS[j.get("form", "fp32")], j.get("rerank", 0), _ptr(j["ids"]),
                     _ptr(j["dists"]))
    st = stream if stream is not None else _stream_of(*[j["Q"] for j in jobs])
    flags = (MULTI_AUTOTUNE if autotune else 0) | (MULTI_EAGER if eager else 0)
    _check(load().gf_query_multi(arr, len(jobs), flags, st))


def multi_stats() -> dict:
    """gf_multi_stats counters."""
    b, r, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().gf_multi_stats(ctypes.byref(b), ctypes.byref(r), ctypes.byref(t)))
    return dict(graphs_built=b.value, graphs_reused=r.value, tuned=t.value)


TRACE_PATHS = {"rows": 0, "tile": 1}


def query_trace(F: Forest, Q, checks: int, leaf_bits=None, cand_bits=None, ncand=None,
                checks_per_query=None, eps: float = 0.0, stream=None, path: str = "rows"):
    """gf_query_trace_ex: opened-leaf bits [nq, m, W], candidate bits
    [nq, ceil(n/32)], candidate counts [nq]; any output may be None.  path
    "rows" reports the row scan's visited bitmap, "tile" the tile path's
    per-point candidate words (forest built with bf16)."""
    nq = Q.shape[0]
    st = stream if stream is not None else _stream_of(Q, leaf_bits, cand_bits, ncand)
    _check(load().gf_query_trace_ex(F.handle, _ptr(Q), nq, checks, _ptr(checks_per_query),
                                    float(eps), TRACE_PATHS[path], _ptr(leaf_bits), _ptr(cand_bits),
                                    _ptr(ncand), st))


def last_query_timing() -> dict:
    """Phase times (ms, HIP events on the query stream) of the last query call
    on this thread, the path of its last batch and the number of batches."""
    ph = (ctypes.c_double * 5)()
    path = ctypes.c_int32()
    nb = ctypes.c_int64()
    _check(load().gf_last_query_timing(ph, 5, ctypes.byref(path), ctypes.byref(nb)))
    names = ("prep_ms", "select_ms", "scan_or_expand_ms", "tile_ms", "merge_ms")
    out = {n: ph[i] for i, n in enumerate(names)}
    out["path"] = "tile" if path.value == 1 else "rows"
    out["batches"] = nb.value
    return out


def fp8_tables(enc_in: Optional[np.ndarray] = None):
    """(hardware decode[256], definition decode[256], encode(enc_in))."""
    hw = np.empty(256, np.float32)
    sw = np.empty(256, np.float32)
    if enc_in is None:
        enc_in = np.zeros(0, np.float32)
    enc_in = np.ascontiguousarray(enc_in, np.float32)
    out = np.empty(enc_in.size, np.uint8)
    _check(load().gf_fp8_tables(_ptr(hw), _ptr(sw), _ptr(enc_in) if enc_in.size else None,
                                enc_in.size, _ptr(out) if enc_in.size else None))
    return hw, sw, out


def hbm_probe(buf, reps: int = 5, stream=None) -> float:
    """gf_hbm_probe: streaming read GB/s over the bytes of device tensor `buf`."""
    out = ctypes.c_double(0.0)
    st = stream if stream is not None else _stream_of(buf)
    nbytes = buf.numel() * buf.element_size() if _is_torch(buf) else buf.nbytes
    _check(load().gf_hbm_probe(_ptr(buf), nbytes, reps, ctypes.byref(out), st))
    return out.value
