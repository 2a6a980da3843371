"""ctypes binding of libhm.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module converts
arguments, owns handles and raises on error codes.  PyTorch provides device
tensors and the current stream.  There is no CPU fallback: if the library is
missing, or no device is usable, the compute calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhm.so")

HM_OK, HM_EINVAL, HM_ENOMEM, HM_ESINGULAR, HM_ENOCONV, HM_EDEVICE, HM_ERANK = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
LAPLACE3D, LOG2D = 0, 1
DATAFLOW, LEVEL = 0, 1

OP_NAMES = ["nop", "getrf", "trsm_l", "trsm_ut", "trsm_u", "gemm", "lrgemm", "trunc", "zero", "copy", "trunc2",
            "gemmp", "seq", "trtri"]


class HmError(RuntimeError):
    def __init__(self, code: int, msg: str, info: int = 0):
        super().__init__(f"hm error {code}: {msg}")
        self.code = code
        self.info = info


class Opts(C.Structure):
    _fields_ = [("leaf", C.c_int), ("eta", C.c_double), ("eps", C.c_double), ("max_rank", C.c_int),
                ("prec", C.c_int), ("exec", C.c_int), ("lazy", C.c_int), ("coarsen", C.c_int)]


class Tuning(C.Structure):
    """hm_tuning: launch choices of the executors (set by autotune.py)."""
    _fields_ = [("exec_wg_per_cu", C.c_int), ("solve_wg", C.c_int), ("batch_order", C.c_int),
                ("reserved", C.c_int * 5)]


class LuStats(C.Structure):
    _fields_ = [("ntasks", C.c_int64), ("nedges", C.c_int64), ("nlevels", C.c_int64),
                ("tasks_by_op", C.c_int64 * 16), ("bytes_alg", C.c_int64), ("flops_alg", C.c_int64),
                ("exec_ms", C.c_double), ("temp_bytes", C.c_int64), ("rank_overflows", C.c_int64),
                ("op_busy_ms", C.c_double * 16), ("trunc_phase_ms", C.c_double * 12),
                ("trunc_mean_k", C.c_double), ("trunc_mean_mn", C.c_double)]


# numpy view of one traced task record (struct Task in csrc/hm_internal.h)
VIEW_DTYPE = np.dtype([("off", "<i8"), ("rows", "<i4"), ("cols", "<i4"), ("rs", "<i4"), ("cs", "<i4"),
                       ("type", "<i4"), ("dyn", "<i4"), ("rank_id", "<i4"), ("rank_id2", "<i4")])
TASK_DTYPE = np.dtype([("op", "<i4"), ("lr", "<i4"), ("r0", "<i4"), ("c0", "<i4"), ("row0", "<i4"),
                       ("c1", "<i4"), ("piv", "<i8"), ("alpha", "<f8"), ("beta", "<f8"),
                       ("y", VIEW_DTYPE), ("a", VIEW_DTYPE), ("b", VIEW_DTYPE), ("x", VIEW_DTYPE)])

_lib = None


def exported_symbols():
    """Names every build of libhm.so must export (the entry points of include/hm.h)."""
    return ["hm_set_allocator", "build_htree", "hm_tree_sizes", "hm_tree_export", "h_assemble", "h_lu", "h_lu_solve",
            "h_solve", "h_matvec", "hm_footprint", "hm_export_leaf", "hm_lu_stats_get", "hm_dag_sizes",
            "hm_dag_export", "hm_dag_calls", "hm_semiauto_dag", "hm_lu_trace", "hm_tree_free", "hm_matrix_free", "hm_lu_free", "hm_last_error",
            "h_solve_async", "h_solve_noalloc", "h_lu_batched", "hm_batch_dag_export", "hm_get_tuning",
            "hm_set_tuning", "hm_import", "hm_dag_seq_export", "hm_solve_trace"]


def lib():
    """Load libhm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run paper_1911_07531_amd/build.py (or __graft_entry__.build())")
    # torch ships its own libamdhip64.so.7; load it first so that the process
    # holds a single HIP runtime, shared by torch's tensors and this library
    try:
        import torch  # noqa: F401
    except Exception:
        pass
    L = C.CDLL(LIB_PATH)
    vp, i64, dbl, ip = C.c_void_p, C.c_int64, C.c_double, C.c_int
    L.hm_last_error.restype = C.c_char_p
    sig = {
        "build_htree": [C.POINTER(C.c_double), i64, ip, C.POINTER(Opts), C.POINTER(vp)],
        "hm_tree_sizes": [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)],
        "hm_tree_export": [vp, vp, vp, vp, vp],
        "h_assemble": [vp, ip, dbl, C.POINTER(Opts), vp, C.POINTER(vp)],
        "h_lu": [vp, C.POINTER(Opts), vp, C.POINTER(vp), C.POINTER(i64)],
        "h_lu_solve": [vp, C.POINTER(Opts), vp, i64, i64, vp, C.POINTER(vp), C.POINTER(i64)],
        "h_solve": [vp, vp, vp, i64, i64, dbl, ip, vp, vp, vp],
        "h_solve_async": [vp, vp, i64, i64, vp, vp],
        "h_lu_batched": [vp, ip, C.POINTER(Opts), vp, vp, vp],
        "hm_batch_dag_export": [vp, ip, C.POINTER(Opts), vp, vp, vp, vp, vp, vp, vp, vp],
        "hm_get_tuning": [C.POINTER(Tuning)],
        "hm_import": [vp, C.POINTER(Opts), vp, vp, i64, vp, C.POINTER(vp)],
        "hm_set_tuning": [C.POINTER(Tuning)],
        "h_solve_noalloc": [vp, vp, vp, i64, i64, dbl, ip, vp, vp, vp],
        "h_matvec": [vp, dbl, vp, i64, dbl, vp, i64, i64, vp],
        "hm_footprint": [vp, ip, C.POINTER(C.c_size_t)],
        "hm_export_leaf": [vp, ip, i64, vp, C.POINTER(C.c_int32), vp],
        "hm_lu_stats_get": [vp, C.POINTER(LuStats)],
        "hm_dag_sizes": [vp, C.POINTER(Opts), ip, vp],
        "hm_dag_export": [vp, C.POINTER(Opts), ip, vp, vp, vp, vp, vp, vp],
        "hm_dag_seq_export": [vp, C.POINTER(Opts), ip, C.POINTER(i64), vp],
        "hm_lu_trace": [vp, vp, C.POINTER(i64), C.POINTER(i64)],
        "hm_solve_trace": [vp, vp, C.POINTER(i64), C.POINTER(i64)],
        "hm_dag_calls": [vp, C.POINTER(Opts), ip, C.POINTER(i64), vp, vp],
        "hm_semiauto_dag": [vp, ip, ip, C.POINTER(i64), C.POINTER(i64), vp, vp],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    for name in ("hm_tree_free", "hm_matrix_free", "hm_lu_free"):
        getattr(L, name).argtypes = [vp]
        getattr(L, name).restype = None
    L.hm_set_allocator.argtypes = [vp, vp, vp]
    L.hm_set_allocator.restype = C.c_int
    _lib = L
    _install_torch_allocator(L)
    return L


_ALLOC_T = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_T = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_callbacks = []


def _install_torch_allocator(L):
    """Route the library's device allocations through torch's caching allocator."""
    try:
        import torch
        if not torch.cuda.is_available():
            return
    except Exception:
        return

    def alloc(size, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(size), torch.cuda.current_device(), stream or 0)
        except Exception:
            return None

    def free(ptr, size, stream, ctx):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    ca, cf = _ALLOC_T(alloc), _FREE_T(free)
    _callbacks[:] = [ca, cf]
    _check(L.hm_set_allocator(C.cast(ca, C.c_void_p), C.cast(cf, C.c_void_p), None))


def _check(code: int, info: int = 0):
    if code != HM_OK:
        raise HmError(code, lib().hm_last_error().decode(), info)


def make_opts(leaf=32, eta=2.0, eps=1e-6, max_rank=0, prec=FP64, exec_mode=DATAFLOW, lazy=1, coarsen=64) -> Opts:
    """hm_opts; coarsen (rows, 0 = off) stops the substitution's task refinement at diagonal blocks of
    that size: 64 (one leaf with its neighbour's product) measured fastest at n = 131072."""
    return Opts(int(leaf), float(eta), float(eps), int(max_rank), int(prec), int(exec_mode), int(lazy), int(coarsen))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_ptr(t):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError("expected a float64 CUDA (HIP) tensor")
    return C.c_void_p(t.data_ptr())


def _col_major(t):
    """(n, nrhs) float64 tensor -> (ptr, ld) for column-major access; requires Fortran order."""
    if t.dim() == 1:
        return _dev_ptr(t), t.shape[0], 1
    n, k = t.shape
    if (n > 1 and t.stride(0) != 1) or (k > 1 and t.stride(1) < n):
        raise ValueError("expected a column-major (n, nrhs) tensor: use t.t().contiguous().t()")
    return _dev_ptr(t), max(n, t.stride(1)) if k > 1 else n, k


class Tree:
    """Cluster tree and block tree (build_htree; host only)."""

    def __init__(self, points: np.ndarray, opts: Opts):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        n, dim = pts.shape
        h = C.c_void_p()
        _check(lib().build_htree(pts.ctypes.data_as(C.POINTER(C.c_double)), n, dim, C.byref(opts), C.byref(h)))
        self.h = h
        self.opts = opts
        self.n = n

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hm_tree_free(self.h)
            self.h = None

    def tables(self):
        """(perm, clusters (ncl, 5), boxes (ncl, 6), blocks (nbl, 7))."""
        n, ncl, nbl = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().hm_tree_sizes(self.h, C.byref(n), C.byref(ncl), C.byref(nbl)))
        perm = np.zeros(n.value, np.int64)
        cl = np.zeros((ncl.value, 5), np.int64)
        box = np.zeros((ncl.value, 6), np.float64)
        bl = np.zeros((nbl.value, 7), np.int32)
        _check(lib().hm_tree_export(self.h, perm.ctypes.data, cl.ctypes.data, box.ctypes.data, bl.ctypes.data))
        return perm, cl, box, bl

    def dag_sizes(self, opts: Opts, which: int = 0) -> dict:
        """Sizes of a traced DAG (hm_dag_sizes; host only): tasks, edges, levels."""
        sz = np.zeros(9, np.int64)
        _check(lib().hm_dag_sizes(self.h, C.byref(opts), which, sz.ctypes.data))
        return {"tasks": int(sz[0]), "edges": int(sz[1]), "levels": int(sz[2])}

    def calls(self, opts: Opts, which: int = 0):
        """(calls (ncalls, 4) int32, task_call (ntasks,) int32) of a traced DAG (hm_dag_calls)."""
        nc = C.c_int64(0)
        _check(lib().hm_dag_calls(self.h, C.byref(opts), which, C.byref(nc), None, None))
        sz = np.zeros(10, np.int64)
        _check(lib().hm_dag_sizes(self.h, C.byref(opts), which, sz.ctypes.data))
        calls = np.zeros((max(1, nc.value), 4), np.int32)
        tc = np.zeros(max(1, int(sz[0])), np.int32)
        _check(lib().hm_dag_calls(self.h, C.byref(opts), which, C.byref(nc), calls.ctypes.data, tc.ctypes.data))
        return calls[:nc.value], tc[:int(sz[0])]

    def semiauto_dag(self, sparsify: bool = False, max_path: int = 0):
        """The paper's semi-automatic H-LU task graph (hm_semiauto_dag): (tasks (n, 4), edges (m, 2))."""
        nt, ne = C.c_int64(0), C.c_int64(0)
        _check(lib().hm_semiauto_dag(self.h, int(sparsify), max_path, C.byref(nt), C.byref(ne), None, None))
        tasks = np.zeros((max(1, nt.value), 4), np.int32)
        edges = np.zeros((max(1, ne.value), 2), np.int32)
        _check(lib().hm_semiauto_dag(self.h, int(sparsify), max_path, C.byref(nt), C.byref(ne), tasks.ctypes.data,
                                     edges.ctypes.data))
        return tasks[:nt.value], edges[:ne.value]

    def dag(self, opts: Opts, which: int = 0):
        """The traced DAG (host only): dict of numpy arrays and sizes."""
        sz = np.zeros(9, np.int64)
        _check(lib().hm_dag_sizes(self.h, C.byref(opts), which, sz.ctypes.data))
        ntasks, nedges, nlevels, tbytes, n64, n32, npiv, nlr, nranks = (int(x) for x in sz)
        assert tbytes == TASK_DTYPE.itemsize, (tbytes, TASK_DTYPE.itemsize)
        tasks = np.zeros(ntasks, TASK_DTYPE)
        sp = np.zeros(ntasks + 1, np.int32)
        si = np.zeros(max(1, nedges), np.int32)
        lv = np.zeros(max(1, ntasks), np.int32)
        _, _, _, bl = self.tables()
        boff = np.zeros((len(bl), 4), np.int64)
        lr = np.zeros((max(1, nlr), 6), np.int64)
        _check(lib().hm_dag_export(self.h, C.byref(opts), which, tasks.ctypes.data, sp.ctypes.data, si.ctypes.data,
                                   lv.ctypes.data, boff.ctypes.data, lr.ctypes.data))
        nseq = C.c_int64(0)
        _check(lib().hm_dag_seq_export(self.h, C.byref(opts), which, C.byref(nseq), None))
        seq = np.zeros(nseq.value, TASK_DTYPE)
        if nseq.value:
            _check(lib().hm_dag_seq_export(self.h, C.byref(opts), which, C.byref(nseq), seq.ctypes.data))
        return dict(tasks=tasks, succ_ptr=sp, succ_idx=si[:nedges], level=lv[:ntasks], block_off=boff,
                    lr=lr[:nlr], n_f64=n64, n_f32=n32, n_piv=npiv, nranks=nranks, nlevels=nlevels, nedges=nedges,
                    seq=seq)


class Matrix:
    """H-matrix assembled on the device (h_assemble)."""

    def __init__(self, tree: Tree, kernel: int, diag: float, opts: Opts, stream=None, _handle=None):
        if _handle is not None:  # built by import_matrix
            self.h, self.tree, self.opts = _handle, tree, opts
            return
        h = C.c_void_p()
        code = lib().h_assemble(tree.h, kernel, diag, C.byref(opts), _stream_ptr(stream), C.byref(h))
        if code == HM_ERANK and h.value:
            lib().hm_matrix_free(h)
        _check(code)
        self.h = h
        self.tree = tree
        self.opts = opts

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hm_matrix_free(self.h)
            self.h = None

    def matvec(self, x, y=None, alpha=1.0, beta=0.0, stream=None):
        import torch
        if y is None:
            y = torch.zeros_like(x)
            beta = 0.0
        xp, ldx, k = _col_major(x)
        yp, ldy, k2 = _col_major(y)
        assert k == k2
        _check(lib().h_matvec(self.h, alpha, xp, ldx, beta, yp, ldy, k, _stream_ptr(stream)))
        return y

    def leaf(self, block: int):
        return export_leaf(self.h, 0, block, self.tree)

    def footprint(self) -> int:
        b = C.c_size_t()
        _check(lib().hm_footprint(self.h, 0, C.byref(b)))
        return b.value


class LU:
    """H-LU factors (h_lu).  With rhs (an (n, nrhs) column-major float64 device
    tensor) the factorization and the substitution of rhs run as one DAG
    (h_lu_solve) and rhs is overwritten by the solution."""

    def __init__(self, a: Matrix, opts: Opts, stream=None, rhs=None, _handle=None):
        if _handle is not None:  # built by lu_batched
            self.h, self.a, self.tree, self.opts = _handle, a, a.tree, opts
            return
        h = C.c_void_p()
        info = C.c_int64(0)
        if rhs is None:
            code = lib().h_lu(a.h, C.byref(opts), _stream_ptr(stream), C.byref(h), C.byref(info))
        else:
            bp, ldb, k = _col_major(rhs)
            code = lib().h_lu_solve(a.h, C.byref(opts), bp, ldb, k, _stream_ptr(stream), C.byref(h), C.byref(info))
        if code == HM_ERANK and h.value:
            lib().hm_lu_free(h)  # factors exist, but some block needed more than the capacity
        _check(code, info.value)
        self.h = h
        self.a = a
        self.tree = a.tree
        self.opts = opts

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hm_lu_free(self.h)
            self.h = None

    def solve(self, b, refine_with: Matrix | None = None, rtol=1e-10, max_iter=50, stream=None):
        """Solve in place on the (n, nrhs) column-major float64 device tensor b; returns (b, iters, relres)."""
        bp, ldb, k = _col_major(b)
        iters = np.zeros(max(1, (k + 63) // 64), np.int32)
        rel = np.zeros(max(1, k), np.float64)
        code = lib().h_solve(self.h, refine_with.h if refine_with is not None else None, bp, ldb, k, rtol,
                             max_iter, _stream_ptr(stream), iters.ctypes.data, rel.ctypes.data)
        if code == HM_ENOCONV:
            return b, iters, rel
        _check(code)
        return b, iters, rel

    def solve_async(self, b, status, stream=None):
        """Queue the substitution (no refinement) of the (n, nrhs) column-major float64 device
        tensor b on `stream` (h_solve_async); status (an int32 device tensor) receives the
        hm_status when the work completes.  Returns b."""
        import torch
        if not isinstance(status, torch.Tensor) or not status.is_cuda or status.dtype != torch.int32:
            raise TypeError("status must be an int32 device tensor")
        bp, ldb, k = _col_major(b)
        _check(lib().h_solve_async(self.h, bp, ldb, k, _stream_ptr(stream), C.c_void_p(status.data_ptr())))
        return b

    def solve_noalloc(self, b, refine_with: Matrix | None = None, rtol=1e-10, max_iter=50, stream=None):
        """h_solve_noalloc: as solve(), with the refinement vectors in the library's fixed scratch;
        returns (b, max corrections over the chunks, relres)."""
        bp, ldb, k = _col_major(b)
        it = np.zeros(1, np.int32)
        rel = np.zeros(max(1, k), np.float64)
        code = lib().h_solve_noalloc(self.h, refine_with.h if refine_with is not None else None, bp, ldb, k, rtol,
                                     max_iter, _stream_ptr(stream), it.ctypes.data, rel.ctypes.data)
        if code != HM_ENOCONV:
            _check(code)
        return b, int(it[0]), rel

    def stats(self) -> dict:
        s = LuStats()
        _check(lib().hm_lu_stats_get(self.h, C.byref(s)))
        d = {f: getattr(s, f) for f, _ in LuStats._fields_ if f not in ("tasks_by_op", "op_busy_ms", "trunc_phase_ms")}
        ph = ["gram", "cholesky", "core", "svd", "solve", "rebuild"]
        d["trunc_phase_ms"] = dict(zip([f"{x}_small" for x in ph] + [f"{x}_large" for x in ph],
                                       [float(x) for x in s.trunc_phase_ms]))
        d["tasks_by_op"] = {OP_NAMES[i]: int(s.tasks_by_op[i]) for i in range(len(OP_NAMES)) if s.tasks_by_op[i]}
        d["op_busy_ms"] = {OP_NAMES[i]: float(s.op_busy_ms[i]) for i in range(len(OP_NAMES)) if s.tasks_by_op[i]}
        return d

    def leaf(self, block: int):
        return export_leaf(self.h, 1, block, self.tree)

    def timeline(self):
        """(ntasks, 8) uint64 (start, end, info, info2, phases x3, queued) and the tick rate in kHz
        (needs HM_DEBUG_TRACE=1);
        info: workgroup in bits 0-15, for truncations term width / m / n in bits 16-31 / 32-47 / 48-63;
        info2 (truncations): route / SVD rows / SVD columns / sweeps / rank in bits 0-7 / 8-19 / 20-31 /
        32-39 / 40-47; words 4-6: ticks of the six truncation phases, two 32-bit counts per word."""
        n, khz = C.c_int64(), C.c_int64()
        _check(lib().hm_lu_trace(self.h, None, C.byref(n), C.byref(khz)))
        out = np.zeros((n.value, 8), np.uint64)
        _check(lib().hm_lu_trace(self.h, out.ctypes.data, C.byref(n), C.byref(khz)))
        return out, khz.value

    def solve_timeline(self):
        """The last substitution pass's (ntasks, 8) task records as in timeline() and the tick rate
        in kHz (needs HM_DEBUG_TRACE=1 before the factorization)."""
        n, khz = C.c_int64(), C.c_int64()
        _check(lib().hm_solve_trace(self.h, None, C.byref(n), C.byref(khz)))
        out = np.zeros((n.value, 8), np.uint64)
        _check(lib().hm_solve_trace(self.h, out.ctypes.data, C.byref(n), C.byref(khz)))
        return out, khz.value

    def footprint(self, kind=1) -> int:
        b = C.c_size_t()
        _check(lib().hm_footprint(self.h, kind, C.byref(b)))
        return b.value


def import_matrix(tree: Tree, opts: Opts, leaves: dict, stream=None) -> Matrix:
    """hm_import: an H-matrix from host leaves {block index: ('D', array) or ('R', U, V)}
    on tree's block structure (every leaf block must be given)."""
    _, cl, _, bl = tree.tables()
    ranks = np.full(len(bl), -1, np.int32)
    parts = []
    for b in range(len(bl)):
        if bl[b, 2] == 0:
            continue
        leaf = leaves[b]
        if bl[b, 2] == 1:
            parts.append(np.asarray(leaf[1], np.float64).ravel(order="F"))
        else:
            u, v = np.asarray(leaf[1], np.float64), np.asarray(leaf[2], np.float64)
            ranks[b] = u.shape[1]
            parts.append(u.ravel(order="F"))
            parts.append(v.ravel(order="F"))
    data = np.ascontiguousarray(np.concatenate(parts)) if parts else np.zeros(1)
    n = sum(p.size for p in parts)
    h = C.c_void_p()
    _check(lib().hm_import(tree.h, C.byref(opts), ranks.ctypes.data, data.ctypes.data, n, _stream_ptr(stream),
                           C.byref(h)))
    return Matrix(tree, -1, 0.0, opts, _handle=h)


def get_tuning() -> dict:
    t = Tuning()
    _check(lib().hm_get_tuning(C.byref(t)))
    return {"exec_wg_per_cu": t.exec_wg_per_cu, "solve_wg": t.solve_wg, "batch_order": t.batch_order}


def set_tuning(exec_wg_per_cu=None, solve_wg=None, batch_order=None):
    """Change some launch choices (hm_set_tuning); returns the previous ones."""
    old = get_tuning()
    t = Tuning()
    _check(lib().hm_get_tuning(C.byref(t)))
    if exec_wg_per_cu is not None:
        t.exec_wg_per_cu = int(exec_wg_per_cu)
    if solve_wg is not None:
        t.solve_wg = int(solve_wg)
    if batch_order is not None:
        t.batch_order = int(batch_order)
    _check(lib().hm_set_tuning(C.byref(t)))
    return old


def lu_batched(mats, opts: Opts, stream=None):
    """h_lu_batched: the H-LUs of several matrices as one DAG on one launch; returns a list of LU."""
    k = len(mats)
    arr = (C.c_void_p * k)(*[m.h for m in mats])
    outs = (C.c_void_p * k)()
    infos = np.zeros(k, np.int64)
    code = lib().h_lu_batched(arr, k, C.byref(opts), _stream_ptr(stream), outs, infos.ctypes.data)
    hs = [outs[i] for i in range(k)]
    if code != HM_OK:
        for h in hs:
            if h:
                lib().hm_lu_free(C.c_void_p(h))
        bad = int(np.nonzero(infos >= 0)[0][0]) if code == HM_ESINGULAR and np.any(infos >= 0) else -1
        try:
            _check(code, int(infos[bad]) if bad >= 0 else 0)
        except HmError as e:
            e.instance = bad
            raise
    return [LU(m, opts, _handle=C.c_void_p(h)) for m, h in zip(mats, hs)]


def batch_dag(trees, opts: Opts):
    """The combined DAG of h_lu_batched over the trees (host only): dict of numpy arrays."""
    k = len(trees)
    arr = (C.c_void_p * k)(*[t.h for t in trees])
    sz = np.zeros(7, np.int64)
    _check(lib().hm_batch_dag_export(arr, k, C.byref(opts), sz.ctypes.data, None, None, None, None, None, None,
                                     None))
    nt, ne, nl, n64, n32, npv, nrk = (int(x) for x in sz)
    tasks = np.zeros(nt, TASK_DTYPE)
    sp = np.zeros(nt + 1, np.int32)
    si = np.zeros(max(1, ne), np.int32)
    order = np.zeros(max(1, nt), np.int32)
    lp = np.zeros(nl + 1, np.int32)
    lr = np.zeros((max(1, nrk), 6), np.int64)
    bases = np.zeros((k, 8), np.int64)
    _check(lib().hm_batch_dag_export(arr, k, C.byref(opts), sz.ctypes.data, tasks.ctypes.data, sp.ctypes.data,
                                     si.ctypes.data, order.ctypes.data, lp.ctypes.data, lr.ctypes.data,
                                     bases.ctypes.data))
    return dict(tasks=tasks, succ_ptr=sp, succ_idx=si[:ne], order=order[:nt], level_ptr=lp, lr=lr[:nrk],
                bases=bases, n_f64=n64, n_f32=n32, n_piv=npv, nranks=nrk, nedges=ne, nlevels=nl)


def export_leaf(handle, kind, block, tree: Tree):
    """('D', array, piv) or ('R', U, V) for one leaf block, FP64 host copies."""
    _, cl, _, bl = tree.tables() if not hasattr(tree, "_tables") else tree._tables
    tree._tables = (None, cl, None, bl)
    tau, sigma, k = bl[block, 0], bl[block, 1], bl[block, 2]
    m = int(cl[tau, 1] - cl[tau, 0])
    n = int(cl[sigma, 1] - cl[sigma, 0])
    rank = C.c_int32()
    _check(lib().hm_export_leaf(handle, kind, block, None, C.byref(rank), None))
    if k == 1:
        d = np.zeros(m * n, np.float64)
        piv = np.zeros(m, np.int32)
        _check(lib().hm_export_leaf(handle, kind, block, d.ctypes.data, C.byref(rank), piv.ctypes.data))
        return "D", d.reshape(n, m).T.copy(), piv
    r = rank.value
    d = np.zeros(max(1, (m + n) * r), np.float64)
    _check(lib().hm_export_leaf(handle, kind, block, d.ctypes.data, C.byref(rank), None))
    u = d[:m * r].reshape(r, m).T.copy()
    v = d[m * r:(m + n) * r].reshape(r, n).T.copy()
    return "R", u, v


# names of the C-ABI, for callers who prefer the functional form
def build_htree(points, opts: Opts) -> Tree:
    return Tree(points, opts)


def h_assemble(tree: Tree, kernel: int, diag: float, opts: Opts, stream=None) -> Matrix:
    return Matrix(tree, kernel, diag, opts, stream)


def h_lu(a: Matrix, opts: Opts, stream=None) -> LU:
    return LU(a, opts, stream)


def h_solve(f: LU, b, a: Matrix | None = None, rtol=1e-10, max_iter=50, stream=None):
    return f.solve(b, a, rtol, max_iter, stream)


def h_matvec(a: Matrix, x, y=None, alpha=1.0, beta=0.0, stream=None):
    return a.matvec(x, y, alpha, beta, stream)
