"""Thin ctypes binding over the C ABI in include/unifrac_mi.h.

Argument marshalling only: every step of the distance computation runs inside
libunifrac_mi.so.  If the library has not been built this module raises at import time;
there is no fallback implementation.

Inputs are numpy arrays (host).  Outputs are numpy arrays (host) or, for the distance
entry point, optionally a device tensor whose data pointer is handed to the library
(torch is used only for that memory and for the current stream).
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libunifrac_mi.so")

try:
    # Load torch's HIP runtime first when torch is present: the library then binds to that
    # same runtime (identical soname), so device tensors and streams are valid in both.
    import torch  # noqa: F401
except ImportError:
    pass

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_2005_05826_amd.build` (or __graft_entry__.build())")

_lib = ctypes.CDLL(LIB_PATH)

c_i32, c_i64, c_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p

UF_OK = 0
STATUS_NAMES = {0: "UF_OK", 1: "UF_E_ARG", 2: "UF_E_TREE", 3: "UF_E_TABLE",
                4: "UF_E_EMPTY_SAMPLE", 5: "UF_E_DEVICE", 6: "UF_E_OOM",
                7: "UF_E_UNSUPPORTED", 8: "UF_E_INTERNAL"}
METHODS = {"unweighted": 0, "weighted_normalized": 1, "weighted_unnormalized": 2}
PRECISIONS = {"fp64": 0, "fp32": 1, "mfma_bf16x2": 2}
DTYPES = {"f64": 0, "f32": 1}

# every entry point declared in include/unifrac_mi.h
EXPORTED = ["uf_status_string", "uf_last_error", "uf_validate", "uf_context_create",
            "uf_context_destroy", "uf_plan_create", "uf_plan_destroy", "uf_plan_query",
            "uf_plan_embedding_counts", "uf_plan_embedding_counts16",
            "uf_plan_embedding_presence", "uf_plan_distance", "uf_plan_distance_stripes", "uf_plan_stripes", "uf_plan_trim", "uf_plan_set_profiling",
            "uf_plan_get_profile", "uf_plan_autotune", "uf_batch_create", "uf_batch_run", "uf_batch_capture",
            "uf_batch_set_profiling", "uf_batch_get_profile", "uf_batch_destroy",
            "uf_distance_batch", "uf_mantel", "uf_distance", "uf_debug_embedding_counts",
            "uf_autotune", "uf_autotune_lookup", "uf_plan_distance_noalloc",
            "uf_plan_set_memory_limit", "uf_plan_distance_block", "uf_merge_block"]


class UfTree(ctypes.Structure):
    _fields_ = [("n_nodes", c_i32), ("parent", c_p), ("length", c_p)]


class UfTable(ctypes.Structure):
    _fields_ = [("n_samples", c_i32), ("n_features", c_i32), ("indptr", c_p),
                ("indices", c_p), ("counts", c_p), ("feature_node", c_p)]


class UfTuning(ctypes.Structure):
    _fields_ = [("emb_batch", c_i32), ("k_chunk", c_i32), ("den_mode", c_i32),
                ("variant", c_i32), ("tile", c_i32), ("count_width", c_i32),
                ("k_split", c_i32)]


class UfKernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", c_i64), ("total_ms", ctypes.c_double)]


class UfJob(ctypes.Structure):
    _fields_ = [("tree", UfTree), ("table", UfTable), ("method", ctypes.c_int),
                ("prec", ctypes.c_int), ("out_dtype", ctypes.c_int), ("out", c_p),
                ("out_on_device", c_i32)]


class UfPlanInfo(ctypes.Structure):
    _fields_ = [("n_samples", c_i32), ("n_nodes", c_i32), ("n_branches", c_i32),
                ("n_leaves", c_i32), ("n_levels", c_i32), ("n_stripes", c_i32),
                ("n_pairs", c_i64), ("nnz", c_i64)]


_lib.uf_status_string.argtypes = [ctypes.c_int]
_lib.uf_status_string.restype = ctypes.c_char_p
_lib.uf_last_error.argtypes = [c_p]
_lib.uf_last_error.restype = ctypes.c_char_p
_lib.uf_validate.argtypes = [ctypes.POINTER(UfTree), ctypes.POINTER(UfTable)]
_lib.uf_context_create.argtypes = [c_i32, ctypes.POINTER(c_p)]
_lib.uf_context_destroy.argtypes = [c_p]
_lib.uf_context_destroy.restype = None
_lib.uf_plan_create.argtypes = [c_p, ctypes.POINTER(UfTree), ctypes.POINTER(UfTable), c_p,
                                ctypes.POINTER(c_p)]
_lib.uf_plan_destroy.argtypes = [c_p]
_lib.uf_plan_destroy.restype = None
_lib.uf_plan_query.argtypes = [c_p, ctypes.POINTER(UfPlanInfo)]
_lib.uf_plan_embedding_counts.argtypes = [c_p, c_p, c_i32, c_p]
_lib.uf_plan_embedding_presence.argtypes = [c_p, c_p, c_i32, c_p]
_lib.uf_plan_embedding_counts16.argtypes = [c_p, c_p, c_i32, c_p]
_lib.uf_plan_distance.argtypes = [c_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(UfTuning),
                                  ctypes.c_int, c_p, c_i32, c_p]
_lib.uf_plan_distance_stripes.argtypes = [c_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(UfTuning),
                                          c_i32, c_i32, ctypes.c_int, c_p, c_i32, c_p]
_lib.uf_plan_stripes.argtypes = [c_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(UfTuning),
                                 c_p, c_p, c_p]
_lib.uf_plan_trim.argtypes = [c_p]
_lib.uf_plan_set_profiling.argtypes = [c_p, c_i32]
_lib.uf_plan_get_profile.argtypes = [c_p, ctypes.POINTER(UfKernelStat), c_i32,
                                     ctypes.POINTER(c_i32)]
_lib.uf_plan_autotune.argtypes = [c_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(UfTuning), c_i32,
                                  ctypes.c_char_p, ctypes.POINTER(UfTuning), ctypes.POINTER(ctypes.c_double)]
_lib.uf_autotune.argtypes = [c_p, ctypes.POINTER(UfJob), c_i32]
_lib.uf_autotune_lookup.argtypes = [c_p, ctypes.c_int, ctypes.c_int, c_i32, c_i32, ctypes.POINTER(UfTuning),
                                    ctypes.POINTER(c_i32)]
_lib.uf_plan_distance_noalloc.argtypes = [c_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(UfTuning),
                                          ctypes.c_int, c_p, c_p]
_lib.uf_plan_set_memory_limit.argtypes = [c_p, c_i64]
_lib.uf_plan_distance_block.argtypes = [c_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(UfTuning),
                                        c_i32, c_i32, ctypes.c_int, c_p, c_i32, c_p]
_lib.uf_merge_block.argtypes = [c_p, c_i32, c_i32, c_i32, ctypes.c_int, c_p, c_i32, c_p, c_p]
_lib.uf_debug_embedding_counts.argtypes = [c_p, ctypes.POINTER(UfTree), ctypes.POINTER(UfTable), c_p]
_lib.uf_batch_create.argtypes = [c_p, ctypes.POINTER(UfJob), c_i32, ctypes.POINTER(UfTuning), c_p,
                                 ctypes.POINTER(c_p)]
_lib.uf_batch_run.argtypes = [c_p, c_p]
_lib.uf_batch_capture.argtypes = [c_p]
_lib.uf_batch_set_profiling.argtypes = [c_p, c_i32]
_lib.uf_batch_get_profile.argtypes = [c_p, ctypes.POINTER(UfKernelStat), c_i32, ctypes.POINTER(c_i32)]
_lib.uf_batch_destroy.argtypes = [c_p]
_lib.uf_batch_destroy.restype = None
_lib.uf_distance_batch.argtypes = [c_p, ctypes.POINTER(UfJob), c_i32, c_p]
_lib.uf_mantel.argtypes = [c_p, c_p, c_p, c_i32, c_p, c_i32, ctypes.POINTER(ctypes.c_double),
                           c_p, ctypes.POINTER(ctypes.c_double), c_p]
_lib.uf_mantel.restype = ctypes.c_int
_lib.uf_distance.argtypes = [c_p, ctypes.POINTER(UfTree), ctypes.POINTER(UfTable), ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, c_p, c_i32, c_p]
for _name in ("uf_validate", "uf_context_create", "uf_plan_create", "uf_plan_query",
              "uf_plan_embedding_counts", "uf_plan_embedding_counts16",
              "uf_plan_embedding_presence", "uf_plan_distance", "uf_plan_distance_stripes", "uf_plan_stripes", "uf_plan_trim", "uf_plan_set_profiling",
              "uf_plan_get_profile", "uf_plan_autotune", "uf_batch_create", "uf_batch_run", "uf_batch_capture",
              "uf_batch_set_profiling", "uf_batch_get_profile", "uf_distance_batch",
              "uf_distance", "uf_debug_embedding_counts", "uf_autotune", "uf_autotune_lookup",
              "uf_plan_set_memory_limit", "uf_plan_distance_block", "uf_merge_block",
              "uf_plan_distance_noalloc"):
    getattr(_lib, _name).restype = ctypes.c_int


class UniFracError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.status_name}: {message}")


def library():
    return _lib


def _ptr(a):
    return None if a is None else c_p(a.ctypes.data)


_PINNED_MAX_BYTES = 2 << 30


def _host_array(n, dtype):
    """A new host array of n elements for results copied back from the device: page-locked
    (torch's pinned-memory allocator, which caches the blocks) when a GPU is in use and the
    array is at most 2 GiB, so the copy runs at full link rate, else ordinary memory.  The
    array keeps its block alive."""
    if int(n) * np.dtype(dtype).itemsize <= _PINNED_MAX_BYTES:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                tdt = torch.float64 if np.dtype(dtype) == np.float64 else torch.float32
                return torch.empty(max(int(n), 1), dtype=tdt, pin_memory=True).numpy()[:n]
        except (ImportError, RuntimeError):
            pass
    return np.empty(n, dtype)


class _Inputs:
    """Contiguous typed copies of the inputs plus the ABI structs pointing at them."""

    def __init__(self, parent, length, indptr, indices, counts, n_features, feature_node=None):
        self.parent = np.ascontiguousarray(parent, np.int32)
        self.length = np.ascontiguousarray(length, np.float64)
        self.indptr = np.ascontiguousarray(indptr, np.int64)
        self.indices = np.ascontiguousarray(indices, np.int32)
        self.counts = np.ascontiguousarray(counts, np.int32)
        self.feature_node = None if feature_node is None else np.ascontiguousarray(feature_node, np.int32)
        self.tree = UfTree(self.parent.shape[0], _ptr(self.parent), _ptr(self.length))
        self.table = UfTable(self.indptr.shape[0] - 1, int(n_features), _ptr(self.indptr),
                             _ptr(self.indices), _ptr(self.counts), _ptr(self.feature_node))


def _problem_args(prob):
    return (prob.parent, prob.length, prob.indptr, prob.indices, prob.counts, prob.n_features,
            prob.feature_node)


def validate(parent, length, indptr, indices, counts, n_features, feature_node=None):
    """Host-only validation.  Returns (status, message)."""
    inp = _Inputs(parent, length, indptr, indices, counts, n_features, feature_node)
    st = _lib.uf_validate(ctypes.byref(inp.tree), ctypes.byref(inp.table))
    return st, _lib.uf_last_error(None).decode()


def validate_problem(prob):
    return validate(*_problem_args(prob))


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return c_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return c_p(stream)
    return c_p(stream.cuda_stream)


def _tuning(t):
    if t is None:
        return None
    if isinstance(t, UfTuning):
        return ctypes.byref(t)
    return ctypes.byref(UfTuning(int(t.get("emb_batch", 0)), int(t.get("k_chunk", 0)),
                                 int(t.get("den_mode", 0)), int(t.get("variant", 0)),
                                 int(t.get("tile", 0)), int(t.get("count_width", 0)),
                                 int(t.get("k_split", 0))))


class Context:
    def __init__(self, device: int = 0):
        h = c_p()
        st = _lib.uf_context_create(int(device), ctypes.byref(h))
        if st != UF_OK:
            raise UniFracError(st, _lib.uf_last_error(None).decode())
        self._h = h
        self.device = device
        # plans and batches made on this context: a context outlives them in the C ABI,
        # so close() releases the ones still open first
        self._children = weakref.WeakSet()

    @property
    def handle(self):
        return self._h

    def _check(self, st):
        if st != UF_OK:
            raise UniFracError(st, _lib.uf_last_error(self._h).decode())

    def autotune(self, jobs):
        """uf_autotune over representative jobs: a list of (problem, method, precision).
        The winners stay in this context for problems of the same kind and size."""
        arr, keep = _job_array([dict(problem=p, method=m, precision=pr, out=None) for p, m, pr in jobs])
        self._check(_lib.uf_autotune(self._h, arr, len(jobs)))
        del keep

    def tuned(self, method, precision, n_samples, n_nodes):
        """The knobs uf_autotune stored for such a problem (dict), or None."""
        t = UfTuning()
        found = c_i32(0)
        self._check(_lib.uf_autotune_lookup(self._h, METHODS[method], PRECISIONS[precision],
                                            int(n_samples), int(n_nodes), ctypes.byref(t),
                                            ctypes.byref(found)))
        return {f: int(getattr(t, f)) for f, _ in UfTuning._fields_} if found.value else None

    def debug_embedding_counts(self, prob) -> np.ndarray:
        """uf_debug_embedding_counts: [n_nodes - 1][n_samples] int32, non-root nodes in
        ascending id order."""
        inp = _Inputs(*_problem_args(prob))
        out = np.empty((max(inp.parent.shape[0] - 1, 0), inp.indptr.shape[0] - 1), np.int32)
        self._check(_lib.uf_debug_embedding_counts(self._h, ctypes.byref(inp.tree),
                                                   ctypes.byref(inp.table), _ptr(out)))
        return out

    def close(self):
        if self._h:
            for child in list(self._children):
                child.close()
            _lib.uf_context_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """Inputs validated, preprocessed and resident on the device."""

    def __init__(self, ctx: Context, parent, length, indptr, indices, counts, n_features,
                 feature_node=None, stream=None):
        self.ctx = ctx
        inp = _Inputs(parent, length, indptr, indices, counts, n_features, feature_node)
        h = c_p()
        ctx._check(_lib.uf_plan_create(ctx.handle, ctypes.byref(inp.tree), ctypes.byref(inp.table),
                                       _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        ctx._children.add(self)
        self.info = self.query()

    @classmethod
    def from_problem(cls, ctx: Context, prob, stream=None):
        return cls(ctx, *_problem_args(prob), stream=stream)

    def query(self) -> UfPlanInfo:
        info = UfPlanInfo()
        self.ctx._check(_lib.uf_plan_query(self._h, ctypes.byref(info)))
        return info

    def embedding_counts(self, stream=None) -> np.ndarray:
        out = np.empty((self.info.n_nodes, self.info.n_samples), np.int32)
        self.ctx._check(_lib.uf_plan_embedding_counts(self._h, _ptr(out), 0, _stream_handle(stream)))
        return out

    def embedding_counts16(self, stream=None) -> np.ndarray:
        out = np.empty((self.info.n_nodes, self.info.n_samples), np.int32)
        self.ctx._check(_lib.uf_plan_embedding_counts16(self._h, _ptr(out), 0, _stream_handle(stream)))
        return out

    def embedding_presence(self, stream=None) -> np.ndarray:
        words = (self.info.n_samples + 31) // 32
        out = np.empty((self.info.n_nodes, words), np.uint32)
        self.ctx._check(_lib.uf_plan_embedding_presence(self._h, _ptr(out), 0, _stream_handle(stream)))
        return out

    def distance(self, method="unweighted", precision="fp64", out=None, out_dtype="f64",
                 tuning=None, stream=None):
        """Condensed distances.  `out` may be None (a host numpy array is returned), a numpy
        array, or a device tensor of n*(n-1)/2 elements (torch; its pointer is passed)."""
        n_pairs = self.info.n_pairs
        if out is None:
            out = _host_array(n_pairs, np.float64 if out_dtype == "f64" else np.float32)
        if isinstance(out, np.ndarray):
            if out.size != n_pairs or not out.flags.c_contiguous:
                raise ValueError("out must be a contiguous array of n*(n-1)/2 elements")
            want = np.float64 if out_dtype == "f64" else np.float32
            if out.dtype != want:
                raise ValueError(f"out dtype must be {want}")
            ptr, on_dev = _ptr(out), 0
        else:  # device tensor
            if out.numel() != n_pairs or not out.is_contiguous():
                raise ValueError("out must be a contiguous tensor of n*(n-1)/2 elements")
            import torch
            want = torch.float64 if out_dtype == "f64" else torch.float32
            if out.dtype != want:
                raise ValueError(f"out dtype must be {want}")
            ptr, on_dev = c_p(out.data_ptr()), 1
        self.ctx._check(_lib.uf_plan_distance(self._h, METHODS[method], PRECISIONS[precision],
                                              _tuning(tuning), DTYPES[out_dtype], ptr, on_dev,
                                              _stream_handle(stream)))
        return out

    def distance_noalloc(self, out, method="unweighted", precision="fp64", out_dtype="f64",
                         tuning=None, stream=None):
        """uf_plan_distance_noalloc into a contiguous device tensor `out` of n*(n-1)/2
        elements; asynchronous on `stream` (torch's current stream by default)."""
        import torch
        want = torch.float64 if out_dtype == "f64" else torch.float32
        if out.numel() != self.info.n_pairs or not out.is_contiguous() or out.dtype != want:
            raise ValueError("out must be a contiguous device tensor of n*(n-1)/2 elements of out_dtype")
        self.ctx._check(_lib.uf_plan_distance_noalloc(self._h, METHODS[method], PRECISIONS[precision],
                                                      _tuning(tuning), DTYPES[out_dtype],
                                                      c_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def distance_stripes(self, s_begin, s_end, out, method="unweighted", precision="fp64",
                         out_dtype="f64", tuning=None, stream=None):
        """Fill the pairs of stripes [s_begin, s_end) into `out` (full condensed array)."""
        if isinstance(out, np.ndarray):
            ptr, on_dev = _ptr(out), 0
        else:
            ptr, on_dev = c_p(out.data_ptr()), 1
        self.ctx._check(_lib.uf_plan_distance_stripes(self._h, METHODS[method], PRECISIONS[precision],
                                                      _tuning(tuning), int(s_begin), int(s_end),
                                                      DTYPES[out_dtype], ptr, on_dev,
                                                      _stream_handle(stream)))
        return out

    def distance_block(self, s_begin, s_end, method="unweighted", precision="fp64", out=None,
                       out_dtype="f64", tuning=None, stream=None):
        """Stripes [s_begin, s_end) as a dense [s_end - s_begin][n] block (numpy array, or
        `out`: a numpy array or device tensor of that many elements)."""
        n = self.info.n_samples
        rows = int(s_end) - int(s_begin)
        if out is None:
            out = np.empty((rows, n), np.float64 if out_dtype == "f64" else np.float32)
        if isinstance(out, np.ndarray):
            if out.size != rows * n or not out.flags.c_contiguous:
                raise ValueError("out must be a contiguous array of (s_end - s_begin) * n elements")
            ptr, on_dev = _ptr(out), 0
        else:
            if out.numel() != rows * n or not out.is_contiguous():
                raise ValueError("out must be a contiguous tensor of (s_end - s_begin) * n elements")
            ptr, on_dev = c_p(out.data_ptr()), 1
        self.ctx._check(_lib.uf_plan_distance_block(self._h, METHODS[method], PRECISIONS[precision],
                                                    _tuning(tuning), int(s_begin), int(s_end),
                                                    DTYPES[out_dtype], ptr, on_dev, _stream_handle(stream)))
        return out

    def stripes(self, method="unweighted", precision="fp64", tuning=None, stream=None):
        S, n = self.info.n_stripes, self.info.n_samples
        num = np.empty((S, n), np.float64)
        den = np.empty((S, n), np.float64)
        self.ctx._check(_lib.uf_plan_stripes(self._h, METHODS[method], PRECISIONS[precision],
                                             _tuning(tuning), _ptr(num), _ptr(den),
                                             _stream_handle(stream)))
        return num, den

    def trim(self):
        self.ctx._check(_lib.uf_plan_trim(self._h))

    def set_memory_limit(self, max_device_bytes: int):
        """Device bytes the plan may hold (0: no limit); beyond it the count rows or
        presence bits are generated batch by batch."""
        self.ctx._check(_lib.uf_plan_set_memory_limit(self._h, int(max_device_bytes)))

    def autotune(self, method="unweighted", precision="fp64", base=None, reps=3, cache_path=None):
        """Fastest eligible knobs for this plan: (dict, milliseconds per call)."""
        best = UfTuning()
        ms = ctypes.c_double(0)
        self.ctx._check(_lib.uf_plan_autotune(self._h, METHODS[method], PRECISIONS[precision],
                                              _tuning(base), int(reps),
                                         None if cache_path is None else str(cache_path).encode(),
                                         ctypes.byref(best), ctypes.byref(ms)))
        return ({f: int(getattr(best, f)) for f, _ in UfTuning._fields_}, float(ms.value))

    def set_profiling(self, enable: bool = True):
        self.ctx._check(_lib.uf_plan_set_profiling(self._h, 1 if enable else 0))

    def profile(self) -> dict:
        """{kernel class: (launches, total_ms)} timed with HIP events on the launch stream."""
        cap = 16
        buf = (UfKernelStat * cap)()
        n = c_i32(0)
        self.ctx._check(_lib.uf_plan_get_profile(self._h, buf, cap, ctypes.byref(n)))
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
                for i in range(n.value)}

    def close(self):
        if getattr(self, "_h", None):
            _lib.uf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def distance(ctx: Context, prob, method="unweighted", precision="fp64", out_dtype="f64"):
    """One-shot uf_distance on a host output array."""
    inp = _Inputs(*_problem_args(prob))
    n = inp.indptr.shape[0] - 1
    out = _host_array(n * (n - 1) // 2, np.float64 if out_dtype == "f64" else np.float32)
    ctx._check(_lib.uf_distance(ctx.handle, ctypes.byref(inp.tree), ctypes.byref(inp.table),
                                METHODS[method], PRECISIONS[precision], DTYPES[out_dtype],
                                _ptr(out), 0, None))
    return out


def distance_batch(ctx: Context, jobs, stream=None):
    """One-shot uf_distance_batch: the jobs (dicts as for Batch; outputs given) computed
    together and the call's scratch released again.  Blocks until the outputs are valid."""
    arr, keep = _job_array(jobs)
    ctx._check(_lib.uf_distance_batch(ctx.handle, arr, len(jobs), _stream_handle(stream)))
    del keep
    return [j.get("out") for j in jobs]


def _job_array(jobs):
    """ABI job array for a list of dicts (problem, method, precision, out, out_dtype); `out`
    is a device tensor, a host numpy array, or None.  Returns the array and the objects that
    must stay alive while the library reads it."""
    arr = (UfJob * max(1, len(jobs)))()
    keep = []
    for i, j in enumerate(jobs):
        inp = _Inputs(*_problem_args(j["problem"]))
        keep.append(inp)
        out = j.get("out")
        if out is None:
            ptr, on_dev = None, 0
        elif isinstance(out, np.ndarray):
            if not out.flags.c_contiguous:
                raise ValueError("host outputs must be contiguous")
            ptr, on_dev = _ptr(out), 0
        else:
            ptr, on_dev = c_p(out.data_ptr()), 1
        arr[i] = UfJob(inp.tree, inp.table, METHODS[j["method"]], PRECISIONS[j["precision"]],
                       DTYPES[j.get("out_dtype", "f64")], ptr, on_dev)
    return arr, keep


class Batch:
    """Many jobs computed together.  `jobs` is a list of dicts with keys problem, method,
    precision, out (a contiguous device tensor or host numpy array of n*(n-1)/2 elements)
    and optionally out_dtype ('f64' or 'f32'); the outputs must outlive the batch.  With
    tuning=None every job takes the context's tuned knobs for its kind (Context.autotune)."""

    def __init__(self, ctx: Context, jobs, tuning=None, stream=None):
        self.ctx = ctx
        self._outs = [j["out"] for j in jobs]
        arr, keep = _job_array(jobs)
        h = c_p()
        ctx._check(_lib.uf_batch_create(ctx.handle, arr, len(jobs), _tuning(tuning),
                                        _stream_handle(stream), ctypes.byref(h)))
        del keep
        self._h = h
        ctx._children.add(self)

    def run(self, stream=None):
        self.ctx._check(_lib.uf_batch_run(self._h, _stream_handle(stream)))

    def capture(self):
        self.ctx._check(_lib.uf_batch_capture(self._h))

    def set_profiling(self, enable: bool = True):
        self.ctx._check(_lib.uf_batch_set_profiling(self._h, 1 if enable else 0))

    def profile(self) -> dict:
        cap = 16
        buf = (UfKernelStat * cap)()
        n = c_i32(0)
        self.ctx._check(_lib.uf_batch_get_profile(self._h, buf, cap, ctypes.byref(n)))
        return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
                for i in range(n.value)}

    def close(self):
        if getattr(self, "_h", None):
            _lib.uf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def merge_block(ctx: Context, n, s_begin, s_end, block, condensed, dtype="f64", stream=None):
    """uf_merge_block: scatter a stripe block (numpy array or device tensor) into the
    condensed device tensor `condensed`."""
    if isinstance(block, np.ndarray):
        bptr, on_dev = _ptr(np.ascontiguousarray(block)), 0
        keep = block
    else:
        bptr, on_dev = c_p(block.data_ptr()), 1
    ctx._check(_lib.uf_merge_block(ctx.handle, int(n), int(s_begin), int(s_end), DTYPES[dtype], bptr, on_dev,
                                   c_p(condensed.data_ptr()), _stream_handle(stream)))
    return condensed


def mantel(ctx: Context, x, y, n: int, perms=None, stream=None):
    """Mantel test of two condensed FP64 device tensors; perms: device int32 tensor
    [n_perm][n] of permutations (or None).  Returns (r, p_value, r_perm numpy array)."""
    n_perm = 0 if perms is None else int(perms.shape[0])
    r = ctypes.c_double(0)
    p = ctypes.c_double(0)
    rp = np.empty(max(n_perm, 1), np.float64)
    ctx._check(_lib.uf_mantel(ctx.handle, c_p(x.data_ptr()), c_p(y.data_ptr()), int(n),
                              None if perms is None else c_p(perms.data_ptr()), n_perm,
                              ctypes.byref(r), _ptr(rp), ctypes.byref(p), _stream_handle(stream)))
    return float(r.value), float(p.value), rp[:n_perm]
