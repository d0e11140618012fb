"""MI355X fast graph Fourier transform (Lu & Ortega, symmetry/bipartition butterflies).

Thin ctypes binding of ``libgft.so`` (C ABI in ``include/gft.h``): argument marshalling
only.  Every step of the transform runs in the library's HIP kernels; PyTorch provides
device memory and the current stream.  There is no fallback: if the library is missing
or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libgft.so")

GFT_FP32, GFT_BF16, GFT_FP16, GFT_SPLIT_BF16 = 0, 1, 2, 3
PRECISIONS = {"fp32": GFT_FP32, "bf16": GFT_BF16, "fp16": GFT_FP16, "split_bf16": GFT_SPLIT_BF16}
ORDER_EIGENVALUE, ORDER_BLOCK = 0, 1
ENGINES = {"auto": 0, "generic": 1, "butterfly": 2, "large": 3, "product": 4}
DTYPES = {"fp32": 0, "bf16": 1}
LAPLACIANS = {"combinatorial": 0, "normalized": 1}

STATUS = {
    0: "GFT_OK", 1: "GFT_ERR_INVALID_ARG", 2: "GFT_ERR_GRAPH", 3: "GFT_ERR_NOT_INVOLUTION",
    4: "GFT_ERR_PAIRING_CROSSES_SUBGRAPH", 5: "GFT_ERR_NOT_SYMMETRIC", 6: "GFT_ERR_EIGENSOLVE",
    7: "GFT_ERR_ORTHOGONALITY", 8: "GFT_ERR_ALIGNMENT", 9: "GFT_ERR_UNSUPPORTED",
    10: "GFT_ERR_OOM", 11: "GFT_ERR_HIP",
}

# Every symbol include/gft.h declares.
EXPORTS = [
    "gft_plan", "gft_plan_batch", "gft_forward", "gft_inverse", "gft_forward_batch",
    "gft_inverse_batch", "gft_plan_prepare", "gft_plan_engine", "gft_plan_tiles", "gft_plan_info", "gft_plan_num_graphs",
    "gft_find_pairing", "gft_plan_product",
    "gft_plan_size", "gft_plan_eigenvalues", "gft_plan_basis", "gft_plan_apply_host",
    "gft_plan_blocks", "gft_plan_destroy", "gft_last_error", "gft_version", "gft_stream_copy",
    "gft_apply_noalloc", "gft_plan_tuning",
]


class GFTError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        super().__init__(f"{self.status_name}: {message}")


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("num_edges", ctypes.c_int32),
                ("src", ctypes.POINTER(ctypes.c_int32)), ("dst", ctypes.POINTER(ctypes.c_int32)),
                ("weight", ctypes.POINTER(ctypes.c_double)),
                ("self_loop", ctypes.POINTER(ctypes.c_double))]


class _Pairing(ctypes.Structure):
    _fields_ = [("num_stages", ctypes.c_int32), ("phi", ctypes.POINTER(ctypes.c_int32))]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("order", ctypes.c_int32),
                ("tile_override", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("sym_tol", ctypes.c_double), ("in_dtype", ctypes.c_int32),
                ("out_dtype", ctypes.c_int32), ("laplacian", ctypes.c_int32),
                ("right_haar", ctypes.c_int32), ("autotune", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("fwd_tile", ctypes.c_int32), ("inv_tile", ctypes.c_int32),
                ("grid_fwd", ctypes.c_int32), ("grid_inv", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("batch_rounds", ctypes.c_int32), ("batch_cost16", ctypes.c_int32),
                ("large_tile_kb", ctypes.c_int32), ("source", ctypes.c_int32), ("tune_ms", ctypes.c_double),
                ("onepass_fwd", ctypes.c_int32), ("onepass_inv", ctypes.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["engine"] = {1: "generic", 2: "butterfly", 3: "large", 4: "product"}.get(d["engine"], d["engine"])
        d["source"] = {0: "builtin", 1: "timed", 2: "cached"}.get(d["source"], d["source"])
        return d


class PlanStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("num_stages", ctypes.c_int32),
                ("num_units", ctypes.c_int32), ("num_blocks", ctypes.c_int32),
                ("max_block", ctypes.c_int32), ("num_z_scalings", ctypes.c_int32),
                ("adds", ctypes.c_int64), ("mults", ctypes.c_int64),
                ("max_residual", ctypes.c_double), ("max_orth_error", ctypes.c_double),
                ("num_right_units", ctypes.c_int32), ("num_right_leaves", ctypes.c_int32),
                ("num_kron_leaves", ctypes.c_int32), ("separable_mults", ctypes.c_int64),
                ("num_closed_form_leaves", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgft.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libgft.so not found at {path}; run paper_1907_07875_amd/build.py "
                          "(or __graft_entry__.build()) first")
    # PyTorch ships its own HIP runtime (same soname as ROCm's).  Loading torch first makes
    # libgft bind to that instance: one HIP runtime per process, shared streams and memory.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "gft_plan": ([ctypes.POINTER(_Graph), ctypes.POINTER(_Pairing), ctypes.POINTER(_Options), pp], i32),
        "gft_plan_batch": ([i32, ctypes.POINTER(_Graph), ctypes.POINTER(_Pairing), ctypes.POINTER(_Options), pp], i32),
        "gft_plan_product": ([ctypes.POINTER(_Graph), ctypes.POINTER(_Pairing), ctypes.POINTER(_Graph),
                              ctypes.POINTER(_Pairing), ctypes.POINTER(_Options), pp], i32),
        "gft_forward": ([P, P, P, i64, P], i32),
        "gft_inverse": ([P, P, P, i64, P], i32),
        "gft_forward_batch": ([P, P, P, P, i64, P], i32),
        "gft_inverse_batch": ([P, P, P, P, i64, P], i32),
        "gft_plan_prepare": ([P], i32),
        "gft_plan_engine": ([P, ctypes.POINTER(i32)], i32),
        "gft_plan_tiles": ([P, ctypes.POINTER(i32), ctypes.POINTER(i32)], i32),
        "gft_find_pairing": ([ctypes.POINTER(_Graph), ctypes.POINTER(_Options), i32, i64, P,
                              ctypes.POINTER(i32)], i32),
        "gft_plan_info": ([P, i32, ctypes.POINTER(PlanStats)], i32),
        "gft_plan_num_graphs": ([P, ctypes.POINTER(i32)], i32),
        "gft_plan_size": ([P, i32, ctypes.POINTER(i32)], i32),
        "gft_plan_eigenvalues": ([P, i32, P], i32),
        "gft_plan_basis": ([P, i32, P], i32),
        "gft_plan_apply_host": ([P, i32, i32, P, P, i64], i32),
        "gft_plan_blocks": ([P, i32, P, P], i32),
        "gft_plan_destroy": ([P], i32),
        "gft_last_error": ([], ctypes.c_char_p),
        "gft_version": ([], ctypes.c_char_p),
        "gft_stream_copy": ([P, P, i64, P], i32),
        "gft_apply_noalloc": ([P, i32, P, P, i64, P], i32),
        "gft_plan_tuning": ([P, ctypes.POINTER(Tuning)], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        msg = load_library().gft_last_error().decode(errors="replace")
        raise GFTError(status, msg)


def version() -> str:
    return load_library().gft_version().decode()


def _graph_struct(n, src, dst, weight, self_loop, keep):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    keep += [src, dst, weight]
    g = _Graph(int(n), int(src.shape[0]),
               src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
               dst.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
               weight.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None)
    if self_loop is not None:
        s = np.ascontiguousarray(self_loop, dtype=np.float64)
        keep.append(s)
        g.self_loop = s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return g


def _pairing_struct(n, stages, keep):
    if stages is None or len(stages) == 0:
        return _Pairing(0, None)
    phi = np.ascontiguousarray(np.stack([np.asarray(p) for p in stages]).astype(np.int32))
    keep.append(phi)
    return _Pairing(int(phi.shape[0]), phi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))


def _options(precision="fp32", order=ORDER_EIGENVALUE, tile=0, sym_tol=0.0, engine="auto",
             in_dtype="fp32", out_dtype="fp32", laplacian="combinatorial", right_haar=True, autotune=True):
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    eng = ENGINES[engine] if isinstance(engine, str) else int(engine)
    lap = LAPLACIANS[laplacian] if isinstance(laplacian, str) else int(laplacian)
    return _Options(prec, int(order), int(tile), eng, float(sym_tol), DTYPES[in_dtype], DTYPES[out_dtype], lap,
                    0 if right_haar else 1, 0 if autotune else 1)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Plan:
    """A fast-GFT plan: ``gft_plan`` (one graph) or ``gft_plan_batch`` (several graphs)."""

    def __init__(self, handle: int, sizes: List[int], batch: bool, precision: str,
                 in_dtype: str = "fp32", out_dtype: str = "fp32"):
        self._h = ctypes.c_void_p(handle)
        self.sizes = sizes
        self.batch = batch
        self.precision = precision
        self.in_dtype = in_dtype      # storage of signals
        self.out_dtype = out_dtype    # storage of coefficients

    # -- construction ---------------------------------------------------------------
    @classmethod
    def from_graph(cls, graph, precision="fp32", order=ORDER_EIGENVALUE, tile=0, sym_tol=0.0,
                   engine="auto", in_dtype="fp32", out_dtype="fp32", laplacian="combinatorial",
                   right_haar=True, autotune=True):
        """Plan one graph (an object with n, src, dst, weight, self_loop, stages)."""
        return gft_plan(graph.n, graph.src, graph.dst, graph.weight, graph.self_loop,
                        graph.stages, precision=precision, order=order, tile=tile, sym_tol=sym_tol,
                        engine=engine, in_dtype=in_dtype, out_dtype=out_dtype, laplacian=laplacian,
                        right_haar=right_haar, autotune=autotune)

    @classmethod
    def from_product(cls, graph_a, graph_b, precision="fp32", order=ORDER_EIGENVALUE, sym_tol=0.0,
                     right_haar=True, autotune=True, in_dtype="fp32", out_dtype="fp32"):
        """Plan the Cartesian product of two graphs (node (i, j) = i * graph_b.n + j)."""
        return gft_plan_product(graph_a, graph_b, order=order, sym_tol=sym_tol, right_haar=right_haar,
                                precision=precision, autotune=autotune, in_dtype=in_dtype, out_dtype=out_dtype)

    @property
    def n(self) -> int:
        return self.sizes[0]

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            load_library().gft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- introspection ---------------------------------------------------------------
    def info(self, index: int = 0) -> dict:
        st = PlanStats()
        _check(load_library().gft_plan_info(self._h, index, ctypes.byref(st)))
        return st.as_dict()

    def eigenvalues(self, index: int = 0) -> np.ndarray:
        lam = np.empty(self.sizes[index], dtype=np.float64)
        _check(load_library().gft_plan_eigenvalues(self._h, index, lam.ctypes.data))
        return lam

    def basis(self, index: int = 0) -> np.ndarray:
        n = self.sizes[index]
        U = np.empty((n, n), dtype=np.float64)
        _check(load_library().gft_plan_basis(self._h, index, U.ctypes.data))
        return U

    def blocks(self, index: int = 0):
        nb = self.info(index)["num_blocks"]
        sizes = np.empty(nb, dtype=np.int32)
        nodes = np.empty(self.sizes[index], dtype=np.int32)
        _check(load_library().gft_plan_blocks(self._h, index, sizes.ctypes.data, nodes.ctypes.data))
        out, p = [], 0
        for s in sizes:
            out.append(nodes[p:p + s].copy())
            p += s
        return out

    def apply_host(self, x: np.ndarray, direction: int = 0, index: int = 0) -> np.ndarray:
        """The plan's factorisation in FP64 on the host (no GPU)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.empty_like(x)
        _check(load_library().gft_plan_apply_host(self._h, index, direction, x.ctypes.data,
                                                  y.ctypes.data, x.shape[0]))
        return y

    def prepare(self):
        _check(load_library().gft_plan_prepare(self._h))

    def engine(self) -> str:
        """Kernel family the plan runs on the current device."""
        e = ctypes.c_int32()
        _check(load_library().gft_plan_engine(self._h, ctypes.byref(e)))
        return {1: "generic", 2: "butterfly", 3: "large", 4: "product"}[e.value]

    def tuning(self) -> dict:
        """Launch choices on the current device and where they came from (C: gft_plan_tuning)."""
        t = Tuning()
        _check(load_library().gft_plan_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    def tiles(self):
        """(forward, inverse) signals per tile on the current device (0 = large engine)."""
        f, i = ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().gft_plan_tiles(self._h, ctypes.byref(f), ctypes.byref(i)))
        return f.value, i.value

    # -- device apply ----------------------------------------------------------------
    def forward(self, x, out=None, stream=None):
        return gft_forward(self, x, out, stream)

    def inverse(self, y, out=None, stream=None):
        return gft_inverse(self, y, out, stream)


def gft_plan(n, src, dst, weight, self_loop=None, stages=None, precision="fp32",
             order=ORDER_EIGENVALUE, tile=0, sym_tol=0.0, engine="auto", in_dtype="fp32",
             out_dtype="fp32", laplacian="combinatorial", right_haar=True, autotune=True) -> Plan:
    """Plan the fast GFT of one graph (C: ``gft_plan``).  ``in_dtype`` / ``out_dtype``
    ("fp32" or "bf16") are the storage types of signals and coefficients."""
    lib = load_library()
    keep = []
    g = _graph_struct(n, src, dst, weight, self_loop, keep)
    p = _pairing_struct(n, stages, keep)
    o = _options(precision, order, tile, sym_tol, engine, in_dtype, out_dtype, laplacian, right_haar, autotune)
    h = ctypes.c_void_p()
    _check(lib.gft_plan(ctypes.byref(g), ctypes.byref(p), ctypes.byref(o), ctypes.byref(h)))
    return Plan(h.value, [int(n)], False, precision, in_dtype, out_dtype)


def gft_plan_product(graph_a, graph_b, order=ORDER_EIGENVALUE, sym_tol=0.0, right_haar=True,
                     precision="fp32", laplacian="combinatorial", engine="auto", autotune=True,
                     in_dtype="fp32", out_dtype="fp32") -> Plan:
    """Plan the GFT of the Cartesian product of two graphs (C: ``gft_plan_product``): each
    argument is an object with n, src, dst, weight, self_loop, stages."""
    lib = load_library()
    keep = []
    ga = _graph_struct(graph_a.n, graph_a.src, graph_a.dst, graph_a.weight, graph_a.self_loop, keep)
    pa = _pairing_struct(graph_a.n, graph_a.stages, keep)
    gb = _graph_struct(graph_b.n, graph_b.src, graph_b.dst, graph_b.weight, graph_b.self_loop, keep)
    pb = _pairing_struct(graph_b.n, graph_b.stages, keep)
    o = _options(precision=precision, order=order, sym_tol=sym_tol, engine=engine,
                 laplacian=laplacian, right_haar=right_haar, autotune=autotune, in_dtype=in_dtype,
                 out_dtype=out_dtype)
    h = ctypes.c_void_p()
    _check(lib.gft_plan_product(ctypes.byref(ga), ctypes.byref(pa), ctypes.byref(gb), ctypes.byref(pb),
                                ctypes.byref(o), ctypes.byref(h)))
    return Plan(h.value, [int(graph_a.n) * int(graph_b.n)], False, precision, in_dtype, out_dtype)


def gft_find_pairing(n, src, dst, weight, self_loop=None, max_stages=16, max_steps=0,
                     laplacian="combinatorial", sym_tol=0.0):
    """Search left Haar pairings stage by stage (C: ``gft_find_pairing``); returns a list of
    int32 arrays, one involution per stage, usable as ``stages`` of :func:`gft_plan`."""
    lib = load_library()
    keep = []
    g = _graph_struct(n, src, dst, weight, self_loop, keep)
    o = _options(laplacian=laplacian, sym_tol=sym_tol)
    phi = np.empty(max(1, max_stages) * int(n), dtype=np.int32)
    k = ctypes.c_int32()
    _check(lib.gft_find_pairing(ctypes.byref(g), ctypes.byref(o), int(max_stages), int(max_steps),
                                phi.ctypes.data, ctypes.byref(k)))
    return [phi[s * n:(s + 1) * n].copy() for s in range(k.value)]


def gft_plan_batch(graphs: Sequence, precision="fp32", order=ORDER_EIGENVALUE, tile=0,
                   sym_tol=0.0, engine="auto", in_dtype="fp32", out_dtype="fp32",
                   laplacian="combinatorial", right_haar=True, autotune=True) -> Plan:
    """Plan several graphs for one persistent launch (C: ``gft_plan_batch``); signals and
    coefficients share one storage type, ``in_dtype`` = ``out_dtype`` ("fp32" or "bf16")."""
    lib = load_library()
    keep = []
    G = (_Graph * len(graphs))()
    Pr = (_Pairing * len(graphs))()
    for i, gr in enumerate(graphs):
        G[i] = _graph_struct(gr.n, gr.src, gr.dst, gr.weight, gr.self_loop, keep)
        Pr[i] = _pairing_struct(gr.n, gr.stages, keep)
    o = _options(precision, order, tile, sym_tol, engine, in_dtype, out_dtype, laplacian, right_haar, autotune)
    h = ctypes.c_void_p()
    _check(lib.gft_plan_batch(len(graphs), G, Pr, ctypes.byref(o), ctypes.byref(h)))
    return Plan(h.value, [int(g.n) for g in graphs], True, precision, in_dtype, out_dtype)


def _torch_dtype(name):
    import torch
    return {"fp32": torch.float32, "bf16": torch.bfloat16}[name]


def _check_tensor(t, n, what, dtype="fp32"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != _torch_dtype(dtype):
        raise TypeError(f"{what} must be {_torch_dtype(dtype)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if t.dim() < 1 or t.shape[-1] != n:
        raise ValueError(f"{what} must have last dimension n = {n}")


def _apply(fn_name, plan: Plan, x, out, stream):
    import torch
    if plan.batch:
        raise ValueError("batch plans use gft_forward_batch / gft_inverse_batch")
    fwd = fn_name == "gft_forward"
    din, dout = (plan.in_dtype, plan.out_dtype) if fwd else (plan.out_dtype, plan.in_dtype)
    _check_tensor(x, plan.n, "input", din)
    if out is None:
        out = torch.empty(x.shape, dtype=_torch_dtype(dout), device=x.device)
    else:
        _check_tensor(out, plan.n, "output", dout)
        if out.shape != x.shape:
            raise ValueError("output shape must equal input shape")
    S = x.numel() // plan.n
    _check(getattr(load_library(), fn_name)(plan.handle, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()), S, _stream_ptr(stream)))
    return out


def gft_forward(plan: Plan, x, out=None, stream=None):
    """Coefficients U^T x of every signal (rows of x, shape [..., n]) (C: ``gft_forward``)."""
    return _apply("gft_forward", plan, x, out, stream)


def gft_inverse(plan: Plan, y, out=None, stream=None):
    """Signals U y from coefficients (C: ``gft_inverse``)."""
    return _apply("gft_inverse", plan, y, out, stream)


def gft_apply_noalloc(plan: Plan, x, out, direction=0, stream=None):
    """Forward (direction 0) or inverse (1) into the caller's ``out`` without any device
    allocation (C: ``gft_apply_noalloc``): the plan must be prepared on x's device, and the
    large-signal engine's workspace is the library's static scratch (64 MiB per GPU)."""
    if plan.batch:
        raise ValueError("batch plans use gft_forward_batch / gft_inverse_batch")
    fwd = direction == 0
    din, dout = (plan.in_dtype, plan.out_dtype) if fwd else (plan.out_dtype, plan.in_dtype)
    _check_tensor(x, plan.n, "input", din)
    _check_tensor(out, plan.n, "output", dout)
    if out.shape != x.shape:
        raise ValueError("output shape must equal input shape")
    _check(load_library().gft_apply_noalloc(plan.handle, int(direction), ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(out.data_ptr()), x.numel() // plan.n,
                                            _stream_ptr(stream)))
    return out


def gft_stream_copy(src, dst, stream=None):
    """Copy the bytes of tensor ``src`` into ``dst`` with the library's streaming copy kernel
    (C: ``gft_stream_copy``), the HBM reference quoted beside the transform's rooflines."""
    import torch
    for t in (src, dst):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
            raise TypeError("src and dst must be contiguous CUDA tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst must have the same size in bytes")
    _check(load_library().gft_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                          nbytes, _stream_ptr(stream)))
    return dst


def _apply_batch(fn_name, plan: Plan, x, signal_offsets, out, stream):
    import torch
    if not plan.batch:
        raise ValueError("single-graph plans use gft_forward / gft_inverse")
    dt = _torch_dtype(plan.in_dtype)
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dt and x.is_contiguous()):
        raise TypeError(f"x must be a contiguous {dt} CUDA tensor")
    if not (isinstance(signal_offsets, torch.Tensor) and signal_offsets.is_cuda
            and signal_offsets.dtype == torch.int64 and signal_offsets.numel() == len(plan.sizes) + 1):
        raise TypeError("signal_offsets must be an int64 CUDA tensor of num_graphs + 1 entries")
    if signal_offsets.device != x.device:
        raise ValueError("signal_offsets must be on the device of x")
    if out is None:
        out = torch.empty_like(x)
    elif not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == dt and out.is_contiguous()):
        raise TypeError(f"out must be a contiguous {dt} CUDA tensor")
    elif out.device != x.device or out.numel() != x.numel():
        raise ValueError("out must be on the device of x and hold as many values as x")
    _check(getattr(load_library(), fn_name)(plan.handle, ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(out.data_ptr()),
                                             ctypes.c_void_p(signal_offsets.data_ptr()),
                                             x.numel(), _stream_ptr(stream)))
    return out


def gft_forward_batch(plan: Plan, x, signal_offsets, out=None, stream=None):
    """Mixed batch forward in one launch (C: ``gft_forward_batch``)."""
    return _apply_batch("gft_forward_batch", plan, x, signal_offsets, out, stream)


def gft_inverse_batch(plan: Plan, y, signal_offsets, out=None, stream=None):
    """Mixed batch inverse in one launch (C: ``gft_inverse_batch``)."""
    return _apply_batch("gft_inverse_batch", plan, y, signal_offsets, out, stream)


def _make_autograd():
    import torch

    class GFTFunction(torch.autograd.Function):
        """y = U^T x with backward grad_x = U grad_y, run by the library's inverse kernel.

        U is orthogonal, so the adjoint of the forward GFT is the inverse GFT (Sec. III).
        """

        @staticmethod
        def forward(ctx, x, plan):
            ctx.plan = plan
            return gft_forward(plan, x.contiguous())

        @staticmethod
        def backward(ctx, gy):
            return gft_inverse(ctx.plan, gy.contiguous()), None

    class IGFTFunction(torch.autograd.Function):
        """x = U y with backward grad_y = U^T grad_x (the forward kernel)."""

        @staticmethod
        def forward(ctx, y, plan):
            ctx.plan = plan
            return gft_inverse(plan, y.contiguous())

        @staticmethod
        def backward(ctx, gx):
            return gft_forward(ctx.plan, gx.contiguous()), None

    return GFTFunction, IGFTFunction


_autograd = None


def gft(x, plan: Plan):
    """Differentiable forward GFT."""
    global _autograd
    if _autograd is None:
        _autograd = _make_autograd()
    return _autograd[0].apply(x, plan)


def igft(y, plan: Plan):
    """Differentiable inverse GFT."""
    global _autograd
    if _autograd is None:
        _autograd = _make_autograd()
    return _autograd[1].apply(y, plan)
