"""GPU test of the allocation-free entry point ``cqrrpt_factor_noalloc``
(through the C ABI): its factors must be the same bits as
``cqrrpt_factor_ex``'s on the same input (the same kernels run on the
library's static workspace instead of a caller-supplied one), on two calls
in a row, the second with a smaller input, in FP64 and mixed mode; a request
whose workspace exceeds the static array is refused before any launch."""

import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2311_08316_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_2311_08316_amd as pkg
    pkg.lib()
    return pkg


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _noalloc(P, A, d, nnz, seed, tol, mode):
    m, n = A.shape
    Q = P.empty_colmajor(m, n, A.device)
    R = P.empty_colmajor(n, n, A.device)
    Q.fill_(7.0)
    R.fill_(7.0)
    J = torch.full((n,), -5, dtype=torch.int64, device=A.device)
    info = torch.zeros(ctypes.sizeof(P.CqrrptInfo), dtype=torch.uint8, device=A.device)
    P.factor_noalloc_into(A, d, nnz, seed, tol, Q, R, J, info, mode=mode)
    torch.cuda.synchronize()
    return Q, R, J, P.CqrrptInfo.from_buffer_copy(bytes(info.cpu().numpy().tobytes()))


@pytest.mark.parametrize("mode_name", ["fp64", "mixed"])
def test_noalloc_matches_ex(P, mode_name):
    mode = {"fp64": P.CQRRPT_FP64, "mixed": P.CQRRPT_MIXED}[mode_name]
    # Second call smaller than the first: the static array keeps the first
    # call's contents, which the second must not depend on.
    for (m, n, d, nnz, cond, seed) in ((20011, 256, 320, 8, 1e8, 3), (9001, 100, 125, 4, 1e4, 4)):
        say(f"noalloc {mode_name} m={m} n={n} d={d} nnz={nnz}")
        assert P.workspace_bytes(m, n, d, nnz, mode) <= P.NOALLOC_SCRATCH_BYTES
        A = torch.from_numpy(W.spectrum_matrix(m, n, W.logspaced_spectrum(n, cond),
                                               seed=seed)).to("cuda")
        A = P.colmajor(A)
        Qn, Rn, Jn, In = _noalloc(P, A, d, nnz, seed, 1e-14, mode)
        Qe, Re, Je, Ie = P.factor(A, d, nnz, seed, 1e-14, mode=mode)
        torch.cuda.synchronize()
        assert In.status == 0 and In.rank == Ie.rank == n
        assert In.rank_stage1 == Ie.rank_stage1 and In.chol_fail_col == Ie.chol_fail_col
        assert torch.equal(Jn, Je), "pivots differ"
        assert torch.equal(Rn, Re), "R differs"
        assert torch.equal(Qn, Qe), "Q differs"
        Qh = Qn.cpu().numpy()
        orth = np.linalg.norm(Qh.T @ Qh - np.eye(n), 2)
        say(f"  rank {In.rank} orth {orth:.2e}")
        assert orth <= 1e-12


def test_noalloc_refuses_oversize(P):
    # The mixed workspace holds the FP32 M_pre (4 m n bytes = 1 GiB here).
    m, n, d, nnz = 262144, 1024, 1280, 8
    assert P.workspace_bytes(m, n, d, nnz, P.CQRRPT_MIXED) > P.NOALLOC_SCRATCH_BYTES
    A = P.empty_colmajor(m, n, "cuda")
    A.zero_()
    with pytest.raises(P.CqrrptError, match="workspace"):
        _noalloc(P, A, d, nnz, 1, 1e-14, P.CQRRPT_MIXED)
