"""ctypes binding to ``libcqrrpt.so`` (the C ABI of ``include/cqrrpt.h``).

Argument marshalling only: every function here checks tensor placement and
layout, passes raw device pointers and the current HIP stream to the library,
and returns. There is no CPU fallback; a missing library or a tensor that is
not on the GPU raises.

Matrices are FP64 and column-major. A torch tensor ``A`` of shape (m, n) is
column-major when ``A.stride(0) == 1``; ``colmajor(A)`` returns such a view
(copying if needed), and ``empty_colmajor`` allocates one.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcqrrpt.so")

CQRRPT_FP64 = 0
CQRRPT_MIXED = 1
CQRRPT_MIXED_CHECKED = 2
CQRRPT_MIXED_FP32_CHOLQR2 = 3

STATUS = {
    0: "ok", 1: "non-finite input", 2: "device-memory budget exceeded",
    3: "HIP runtime error", 4: "workspace too small", 5: "grid barrier timed out",
    6: "size beyond the library's limits",
}


class CqrrptInfo(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int64), ("rank_stage1", ctypes.c_int64),
                ("chol_fail_col", ctypes.c_int64), ("status", ctypes.c_int32),
                ("cholqr2_passes", ctypes.c_int32), ("smax", ctypes.c_double),
                ("orth_est", ctypes.c_double)]


INFO_BYTES = ctypes.sizeof(CqrrptInfo)

_lib = None

_i64, _i32, _u64, _dbl, _vp, _sz = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                    ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t)
_SIGS = {
    "cqrrpt_saso_sample": (ctypes.c_int, [_i64, _i64, _i32, _u64, _vp, _vp, _vp]),
    "cqrrpt_sketch_workspace_bytes": (_sz, [_i64, _i64, _i64, _i32]),
    "cqrrpt_sketch": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i32, _u64, _vp, _i64,
                                     _vp, _sz, _vp]),
    "cqrrpt_qrcp_workspace_bytes": (_sz, [_i64, _i64]),
    "cqrrpt_qrcp": (ctypes.c_int, [_vp, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _sz, _vp]),
    "cqrrpt_factor": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i32, _u64, _dbl,
                                     _vp, _i64, _vp, _i64, _vp, ctypes.POINTER(_i64)]),
    "cqrrpt_workspace_bytes": (_sz, [_i64, _i64, _i64, _i32, ctypes.c_int]),
    "cqrrpt_factor_ex": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i32, _u64, _dbl,
                                        _vp, _i64, _vp, _i64, _vp, ctypes.c_int,
                                        _vp, _sz, _vp, _vp]),
    "cqrrpt_factor_implicit_ex": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i32, _u64,
                                                 _dbl, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                                 _vp, _sz, _vp, _vp]),
    "cqrrpt_factor_noalloc": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i32, _u64, _dbl,
                                             _vp, _i64, _vp, _i64, _vp, ctypes.c_int, _vp,
                                             _vp]),
    "cqrrpt_sketched_cholqr_ex": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i32, _u64,
                                                 _vp, _i64, _vp, _i64, _vp, _sz, _vp, _vp]),
    "cqrrpt_dense_workspace_bytes": (_sz, [_i64, _i64, _i64]),
    "cqrrpt_hqrrp_workspace_bytes": (_sz, [_i64, _i64, _i32, _i32]),
    "cqrrpt_hqrrp": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i32, _i32, _u64, _vp, _vp, _i64,
                                    _vp, _sz, _vp, _vp]),
    "cqrrpt_factor_hqrrp_workspace_bytes": (_sz, [_i64, _i64, _i64, _i32, _i32, _i32]),
    "cqrrpt_factor_hqrrp_ex": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i32, _u64, _dbl,
                                              _i32, _i32, _u64, _vp, _i64, _vp, _i64, _vp, _vp,
                                              _sz, _vp, _vp]),
    "cqrrpt_factor_dense_ex": (ctypes.c_int, [_vp, _i64, _i64, _i64, _i64, _i32, _u64, _dbl,
                                              _vp, _i64, _vp, _i64, _vp, _vp, _sz, _vp, _vp]),
    "cqrrpt_probe_copy": (ctypes.c_int, [_vp, _vp, _i64, _vp]),
    "cqrrpt_probe_mfma": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _vp, _i64,
                                         ctypes.POINTER(_i64), _vp]),
    "cqrrpt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "cqrrpt_stage_timing": (ctypes.c_int, [ctypes.c_int]),
    "cqrrpt_stage_times": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
    "cqrrpt_stage_name": (ctypes.c_char_p, [ctypes.c_int]),
    "cqrrpt_server_create": (_vp, [_sz, _i32, ctypes.c_int]),
    "cqrrpt_server_submit": (ctypes.c_int, [_vp, _vp, _i64, _i64, _i64, _i64, _i32, _u64, _dbl,
                                            _vp, _i64, _vp, _i64, _vp, _vp,
                                            ctypes.POINTER(_u64)]),
    "cqrrpt_server_poll": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(_i32)]),
    "cqrrpt_server_ticket_times": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(_dbl)]),
    "cqrrpt_server_release": (ctypes.c_int, [_vp, _u64]),
    "cqrrpt_server_drain": (ctypes.c_int, [_vp]),
    "cqrrpt_server_destroy": (None, [_vp]),
}

STAGES = ("sketch", "qrcp", "rank_stage1", "precondition", "gram", "cholesky", "q_solve",
          "r_product", "cholqr2")


def lib():
    """Load the shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                               "`python paper_2311_08316_amd/build_lib.py`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CqrrptError(RuntimeError):
    pass


def _check(rc, what):
    if rc != 0:
        if rc < 0:
            raise CqrrptError(f"{what}: argument {-rc} is invalid")
        raise CqrrptError(f"{what}: {STATUS.get(rc, rc)}")


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _on_gpu(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise CqrrptError(f"{name} must be a GPU tensor")


def colmajor(A):
    """Column-major FP64 view of a 2-D GPU tensor (copying only if needed)."""
    _on_gpu(A, "A")
    if A.dtype != torch.float64:
        raise CqrrptError("A must be float64")
    if A.dim() != 2:
        raise CqrrptError("A must be 2-D")
    if A.stride(0) == 1 and A.stride(1) >= max(1, A.shape[0]):
        return A
    return A.t().contiguous().t()


def empty_colmajor(m, n, device, dtype=torch.float64):
    return torch.empty((n, m), dtype=dtype, device=device).t()


def padded_ld(m):
    """Leading dimension for an m-row output buffer: m, or m + 16 when 8 m
    is a multiple of 4 KiB. Columns a multiple of 4 KiB apart put the rows
    that a Gram tile reads together on the same cache lines' sets and
    channels; the FP64 mode keeps M_pre in Q, and its Gram ran at 469 ms
    with ld = m against 308 ms with ld = m + 16 at 4194304 x 2048."""
    return m + 16 if m % 512 == 0 else m


def empty_colmajor_ld(m, n, ld, device, dtype=torch.float64):
    """Column-major m x n view with leading dimension ld >= m."""
    return torch.empty((n, ld), dtype=dtype, device=device)[:, :m].t()


def _ld(A):
    return max(1, A.stride(1)) if A.shape[1] > 1 else max(1, A.shape[0])


def saso_sample(m, d, nnz, seed, device="cuda"):
    """Rows (int32[m, nnz]) and signs (int8[m, nnz]) of the sketching operator."""
    rows = torch.empty((m, nnz), dtype=torch.int32, device=device)
    signs = torch.empty((m, nnz), dtype=torch.int8, device=device)
    rc = lib().cqrrpt_saso_sample(m, d, nnz, seed, rows.data_ptr(), signs.data_ptr(),
                                  _stream_handle(rows.device))
    _check(rc, "cqrrpt_saso_sample")
    return rows, signs


def sketch(A, d, nnz, seed):
    """Ahat = S A as a column-major d x n GPU tensor."""
    A = colmajor(A)
    m, n = A.shape
    out = empty_colmajor(d, n, A.device)
    wsb = lib().cqrrpt_sketch_workspace_bytes(m, n, d, nnz)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=A.device)
    rc = lib().cqrrpt_sketch(A.data_ptr(), _ld(A), m, n, d, nnz, seed, out.data_ptr(), d,
                             ws.data_ptr(), wsb, _stream_handle(A.device))
    _check(rc, "cqrrpt_sketch")
    return out


def qrcp(X):
    """Householder QRCP of a d x n GPU matrix (d >= n). Returns (J, R); X is
    copied, not overwritten."""
    src = colmajor(X)
    d, n = src.shape
    X = empty_colmajor(d, n, src.device)
    X.copy_(src)
    J = torch.empty(n, dtype=torch.int64, device=X.device)
    R = empty_colmajor(n, n, X.device)
    wsb = lib().cqrrpt_qrcp_workspace_bytes(d, n)
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=X.device)
    rc = lib().cqrrpt_qrcp(X.data_ptr(), d, d, n, J.data_ptr(), R.data_ptr(), n, ws.data_ptr(),
                           wsb, _stream_handle(X.device))
    _check(rc, "cqrrpt_qrcp")
    return J, R


def stage_timing(slots):
    """Record per-stage HIP events for the next calls (ring of ``slots``)."""
    _check(lib().cqrrpt_stage_timing(slots), "cqrrpt_stage_timing")


def stage_times(slot):
    """Stage durations (ms) of the call that used event set ``slot``."""
    buf = (ctypes.c_double * len(STAGES))()
    _check(lib().cqrrpt_stage_times(slot, buf), "cqrrpt_stage_times")
    return dict(zip(STAGES, list(buf)))


def probe_copy(src, dst):
    """Streaming device copy dst <- src (FP64, same length) on the current
    stream (the library's bandwidth probe)."""
    _on_gpu(src, "src")
    _on_gpu(dst, "dst")
    if src.numel() != dst.numel() or src.dtype != torch.float64 or dst.dtype != torch.float64:
        raise CqrrptError("src and dst must be FP64 of the same length")
    _check(lib().cqrrpt_probe_copy(src.data_ptr(), dst.data_ptr(), src.numel(),
                                   _stream_handle(src.device)), "cqrrpt_probe_copy")


def probe_mfma(out, iters, fp64=True):
    """Matrix-core throughput loop on the current stream; returns its flop
    count. ``out`` is an FP64 device scratch array of at least 32 values
    per compute unit."""
    _on_gpu(out, "out")
    flops = ctypes.c_int64(0)
    _check(lib().cqrrpt_probe_mfma(1 if fp64 else 0, iters, out.data_ptr(), out.numel(),
                                   ctypes.byref(flops), _stream_handle(out.device)),
           "cqrrpt_probe_mfma")
    return flops.value


def workspace_bytes(m, n, d, nnz, mode=CQRRPT_FP64):
    return lib().cqrrpt_workspace_bytes(m, n, d, nnz, mode)


class Factorization:
    """Preallocated outputs and workspace for repeated stream-ordered calls."""

    def __init__(self, m, n, d, nnz, mode=CQRRPT_FP64, device="cuda", implicit=False):
        """With implicit=True (FP64 only) ``run`` calls
        ``cqrrpt_factor_implicit_ex``: Q then holds M_pre[:, :k] and Rpre
        holds R_pre[:k, :k], so that the orthonormal factor is
        Q[:, :k] Rpre[:k, :k]^{-1}."""
        if implicit and mode != CQRRPT_FP64:
            raise CqrrptError("the implicit-Q form is FP64 only")
        self.m, self.n, self.d, self.nnz, self.mode = m, n, d, nnz, mode
        self.implicit = implicit
        self.device = torch.device(device)
        self.Q = empty_colmajor_ld(m, n, padded_ld(m), self.device)
        self.ldq = padded_ld(m)
        self.Rpre = empty_colmajor(n, n, self.device) if implicit else None
        self.R = empty_colmajor(n, n, self.device)
        self.J = torch.empty(n, dtype=torch.int64, device=self.device)
        self.ws_bytes = workspace_bytes(m, n, d, nnz, mode)
        if self.ws_bytes == 0:
            raise CqrrptError("unsupported sizes")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.info_buf = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=self.device)

    def run(self, A, seed, tol, stream=None):
        """Enqueue one factorization of A on the current (or given) stream."""
        A = colmajor(A)
        if tuple(A.shape) != (self.m, self.n):
            raise CqrrptError("A has the wrong shape")
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else \
            _stream_handle(self.device)
        if self.implicit:
            rc = lib().cqrrpt_factor_implicit_ex(
                A.data_ptr(), _ld(A), self.m, self.n, self.d, self.nnz, seed, tol,
                self.Q.data_ptr(), self.ldq, self.Rpre.data_ptr(), self.n, self.R.data_ptr(),
                self.n, self.J.data_ptr(), self.ws.data_ptr(), self.ws_bytes, s,
                self.info_buf.data_ptr())
            _check(rc, "cqrrpt_factor_implicit_ex")
            return
        rc = lib().cqrrpt_factor_ex(A.data_ptr(), _ld(A), self.m, self.n, self.d, self.nnz,
                                    seed, tol, self.Q.data_ptr(), self.ldq, self.R.data_ptr(),
                                    self.n, self.J.data_ptr(), self.mode, self.ws.data_ptr(),
                                    self.ws_bytes, s, self.info_buf.data_ptr())
        _check(rc, "cqrrpt_factor_ex")

    def info(self):
        """Copy the device-side diagnostics to the host (synchronises)."""
        raw = bytes(self.info_buf.cpu().numpy().tobytes())
        return CqrrptInfo.from_buffer_copy(raw)


def factor(A, d, nnz, seed, tol, mode=CQRRPT_FP64):
    """One factorization: returns (Q, R, J, info). Q is m x n, R is n x n
    (both column-major, zero past the rank), J holds 0-based pivots."""
    A = colmajor(A)
    m, n = A.shape
    f = Factorization(m, n, d, nnz, mode, A.device)
    f.run(A, seed, tol)
    info = f.info()
    if info.status != 0:
        _check(info.status, "cqrrpt_factor_ex")
    return f.Q, f.R, f.J, info


def factor_implicit(A, d, nnz, seed, tol):
    """Implicit-Q factorization: returns (M, Rpre, R, J, info) with
    Q[:, :k] = M[:, :k] Rpre[:k, :k]^{-1} (k = info.rank)."""
    A = colmajor(A)
    m, n = A.shape
    f = Factorization(m, n, d, nnz, CQRRPT_FP64, A.device, implicit=True)
    f.run(A, seed, tol)
    info = f.info()
    if info.status != 0:
        _check(info.status, "cqrrpt_factor_implicit_ex")
    return f.Q, f.Rpre, f.R, f.J, info


# Size of the library's static workspace for cqrrpt_factor_noalloc
# (CQRRPT_NOALLOC_SCRATCH_BYTES in include/cqrrpt.h).
NOALLOC_SCRATCH_BYTES = 64 << 20


def factor_noalloc_into(A, d, nnz, seed, tol, Q, R, J, info_buf, mode=CQRRPT_FP64):
    """``cqrrpt_factor_noalloc`` into caller-allocated outputs (Q m x n and
    R n x n column-major FP64, J int64[n], info_buf uint8[sizeof info]) on
    the current stream; the library allocates nothing."""
    A = colmajor(A)
    m, n = A.shape
    for t, name in ((Q, "Q"), (R, "R"), (J, "J"), (info_buf, "info")):
        _on_gpu(t, name)
    if Q.shape != (m, n) or Q.stride(0) != 1 or R.shape != (n, n) or R.stride(0) != 1:
        raise CqrrptError("Q and R must be column-major m x n and n x n")
    if J.dtype != torch.int64 or J.numel() != n or info_buf.numel() < INFO_BYTES:
        raise CqrrptError("J must be int64[n] and info_buf hold a cqrrpt_info_t")
    rc = lib().cqrrpt_factor_noalloc(A.data_ptr(), _ld(A), m, n, d, nnz, seed, tol,
                                     Q.data_ptr(), _ld(Q), R.data_ptr(), _ld(R), J.data_ptr(),
                                     mode, _stream_handle(A.device), info_buf.data_ptr())
    _check(rc, "cqrrpt_factor_noalloc")


def sketched_cholqr(A, d, nnz, seed):
    """The unpivoted precursor of Sec. 1.3 (``cqrrpt_sketched_cholqr_ex``):
    returns (Q, R, info) with A = Q R for full-rank A (no pivoting)."""
    A = colmajor(A)
    m, n = A.shape
    Q = empty_colmajor(m, n, A.device)
    R = empty_colmajor(n, n, A.device)
    wsb = workspace_bytes(m, n, d, nnz, CQRRPT_FP64)
    if wsb == 0:
        raise CqrrptError("unsupported sizes")
    ws = torch.empty(wsb, dtype=torch.uint8, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    rc = lib().cqrrpt_sketched_cholqr_ex(A.data_ptr(), _ld(A), m, n, d, nnz, seed, Q.data_ptr(),
                                         m, R.data_ptr(), n, ws.data_ptr(), wsb,
                                         _stream_handle(A.device), info.data_ptr())
    _check(rc, "cqrrpt_sketched_cholqr_ex")
    inf = CqrrptInfo.from_buffer_copy(bytes(info.cpu().numpy().tobytes()))
    if inf.status != 0:
        _check(inf.status, "cqrrpt_sketched_cholqr_ex")
    return Q, R, inf


SKETCH_GAUSSIAN = 1
SKETCH_SRHT = 2


def factor_dense(A, d, kind, seed, tol):
    """CQRRPT with a dense sketching operator (``cqrrpt_factor_dense_ex``):
    kind SKETCH_GAUSSIAN or SKETCH_SRHT. Returns (Q, R, J, info)."""
    A = colmajor(A)
    m, n = A.shape
    Q = empty_colmajor(m, n, A.device)
    R = empty_colmajor(n, n, A.device)
    J = torch.empty(n, dtype=torch.int64, device=A.device)
    wsb = lib().cqrrpt_dense_workspace_bytes(m, n, d)
    if wsb == 0:
        raise CqrrptError("unsupported sizes")
    ws = torch.empty(wsb, dtype=torch.uint8, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    rc = lib().cqrrpt_factor_dense_ex(A.data_ptr(), _ld(A), m, n, d, kind, seed, tol,
                                      Q.data_ptr(), m, R.data_ptr(), n, J.data_ptr(),
                                      ws.data_ptr(), wsb, _stream_handle(A.device),
                                      info.data_ptr())
    _check(rc, "cqrrpt_factor_dense_ex")
    inf = CqrrptInfo.from_buffer_copy(bytes(info.cpu().numpy().tobytes()))
    if inf.status != 0:
        _check(inf.status, "cqrrpt_factor_dense_ex")
    return Q, R, J, inf


def hqrrp(X, block, oversample, seed):
    """HQRRP of a d x n GPU matrix (``cqrrpt_hqrrp``; X is copied, not
    overwritten). Returns (J, R, info)."""
    src = colmajor(X)
    d, n = src.shape
    X = empty_colmajor(d, n, src.device)
    X.copy_(src)
    J = torch.empty(n, dtype=torch.int64, device=X.device)
    R = empty_colmajor(n, n, X.device)
    wsb = lib().cqrrpt_hqrrp_workspace_bytes(d, n, block, oversample)
    if wsb == 0:
        raise CqrrptError("unsupported sizes")
    ws = torch.empty(wsb, dtype=torch.uint8, device=X.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=X.device)
    rc = lib().cqrrpt_hqrrp(X.data_ptr(), d, d, n, block, oversample, seed, J.data_ptr(),
                            R.data_ptr(), n, ws.data_ptr(), wsb, _stream_handle(X.device),
                            info.data_ptr())
    _check(rc, "cqrrpt_hqrrp")
    inf = CqrrptInfo.from_buffer_copy(bytes(info.cpu().numpy().tobytes()))
    return J, R, inf


def factor_hqrrp(A, d, nnz, seed, tol, block=16, oversample=8, hseed=0):
    """CQRRPT with HQRRP on the sketch (``cqrrpt_factor_hqrrp_ex``).
    Returns (Q, R, J, info)."""
    A = colmajor(A)
    m, n = A.shape
    Q = empty_colmajor_ld(m, n, padded_ld(m), A.device)
    R = empty_colmajor(n, n, A.device)
    J = torch.empty(n, dtype=torch.int64, device=A.device)
    wsb = lib().cqrrpt_factor_hqrrp_workspace_bytes(m, n, d, nnz, block, oversample)
    if wsb == 0:
        raise CqrrptError("unsupported sizes")
    ws = torch.empty(wsb, dtype=torch.uint8, device=A.device)
    info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
    rc = lib().cqrrpt_factor_hqrrp_ex(A.data_ptr(), _ld(A), m, n, d, nnz, seed, tol, block,
                                      oversample, hseed, Q.data_ptr(), _ld(Q), R.data_ptr(), n,
                                      J.data_ptr(), ws.data_ptr(), wsb,
                                      _stream_handle(A.device), info.data_ptr())
    _check(rc, "cqrrpt_factor_hqrrp_ex")
    inf = CqrrptInfo.from_buffer_copy(bytes(info.cpu().numpy().tobytes()))
    if inf.status != 0:
        _check(inf.status, "cqrrpt_factor_hqrrp_ex")
    return Q, R, J, inf


def factor_sync(A, d, nnz, seed, tol):
    """The synchronous C entry point ``cqrrpt_factor`` (allocates internally)."""
    A = colmajor(A)
    m, n = A.shape
    Q = empty_colmajor(m, n, A.device)
    R = empty_colmajor(n, n, A.device)
    J = torch.empty(n, dtype=torch.int64, device=A.device)
    rank = ctypes.c_int64(-1)
    torch.cuda.synchronize(A.device)
    rc = lib().cqrrpt_factor(A.data_ptr(), _ld(A), m, n, d, nnz, seed, tol, Q.data_ptr(), m,
                             R.data_ptr(), n, J.data_ptr(), ctypes.byref(rank))
    _check(rc, "cqrrpt_factor")
    return Q, R, J, rank.value


class Server:
    """Serving form (``cqrrpt_server_*``): requests are submitted as they
    arrive, admitted by the library in arrival order as a slot and device
    memory free up, and run concurrently. ``submit`` allocates the request's
    outputs and returns a ticket; ``result`` returns them once done."""

    def __init__(self, budget_bytes, slots=4, mode=CQRRPT_FP64, device=None):
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.mode = mode
        self._h = lib().cqrrpt_server_create(int(budget_bytes), int(slots), int(mode))
        if not self._h:
            raise CqrrptError("cqrrpt_server_create failed")
        self._out = {}

    def submit(self, A, d, nnz, seed, tol):
        """Queue one factorization of A (the caller's pending writes to A are
        completed first). Returns the ticket."""
        A = colmajor(A)
        m, n = A.shape
        Q = empty_colmajor(m, n, A.device)
        R = empty_colmajor(n, n, A.device)
        J = torch.empty(n, dtype=torch.int64, device=A.device)
        info = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=A.device)
        torch.cuda.current_stream(A.device).synchronize()
        t = ctypes.c_uint64(0)
        rc = lib().cqrrpt_server_submit(self._h, A.data_ptr(), _ld(A), m, n, d, nnz, seed, tol,
                                        Q.data_ptr(), m, R.data_ptr(), n, J.data_ptr(),
                                        info.data_ptr(), ctypes.byref(t))
        _check(rc, "cqrrpt_server_submit")
        self._out[t.value] = (A, Q, R, J, info)
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int32(0)
        rc = lib().cqrrpt_server_poll(self._h, ticket, ctypes.byref(done))
        if done.value:
            _check(rc, "server request")
        elif rc < 0:
            _check(rc, "cqrrpt_server_poll")
        return bool(done.value)

    def times(self, ticket):
        """(submit, admit, done) host times in ms."""
        buf = (ctypes.c_double * 3)()
        _check(lib().cqrrpt_server_ticket_times(self._h, ticket, buf), "ticket_times")
        return tuple(buf)

    def result(self, ticket):
        """(Q, R, J, info) of a finished request; forgets the ticket."""
        if not self.poll(ticket):
            raise CqrrptError("request not finished")
        _, Q, R, J, info = self._out.pop(ticket)
        lib().cqrrpt_server_release(self._h, ticket)
        return Q, R, J, CqrrptInfo.from_buffer_copy(bytes(info.cpu().numpy().tobytes()))

    def drain(self):
        _check(lib().cqrrpt_server_drain(self._h), "cqrrpt_server_drain")

    def close(self):
        if self._h:
            lib().cqrrpt_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
