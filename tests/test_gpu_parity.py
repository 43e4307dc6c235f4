"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Bars:
  * sketching operator positions and signs: bit-exact;
  * sketch: within the componentwise rounding bound of a p-term sum, p the
    largest number of nonzeros in a row of S;
  * pivots J and ranks: identical on inputs whose pivot decisions have a
    margin (well-separated column norms, or the spectra used here);
  * R: ||R - R_oracle||_F / ||R_oracle||_F <= 1e-12;
  * Q: ||Q - Q_oracle||_F / ||Q_oracle||_F <= max(1e-12, 100 u cond(R[:, :k]));
  * reconstruction ||A[:, J] - Q R||_F / ||A||_F and orthogonality
    ||Q^T Q - I||_2 <= 1e-12 in FP64;
  * repeated calls are bit-identical.
"""

import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cqrrpt_oracle as O
from paper_2311_08316_amd import workloads as W

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    import paper_2311_08316_amd as pkg
    pkg.lib()  # raises if the HIP library is not built
    return pkg


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_gpu(A):
    t = torch.from_numpy(np.asfortranarray(A)).to("cuda")
    if t.stride(0) != 1:
        t = t.t().contiguous().t()
    return t


def to_np(t):
    return t.detach().cpu().numpy()


def metrics(A, Q, R, J, k):
    n = A.shape[1]
    recon = np.linalg.norm(A[:, J] - Q @ R) / np.linalg.norm(A)
    Qk = Q[:, :k]
    orth = np.linalg.norm(Qk.T @ Qk - np.eye(k), 2) if k else 0.0
    return recon, orth


def compare_factor(A, gpu, orc, label, q_extra=1.0):
    Qg, Rg, Jg, info = gpu
    Qg, Rg, Jg = to_np(Qg), to_np(Rg), to_np(Jg)
    k = orc["rank"]
    assert info.rank == k, f"{label}: rank {info.rank} vs oracle {k}"
    assert info.rank_stage1 == orc["rank_stage1"], label
    assert np.array_equal(Jg, orc["J"]), f"{label}: pivots differ"
    Ro, Qo = orc["R"], orc["Q"]
    if k == 0:
        assert not Qg.any() and not Rg.any()
        return
    dR = np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro)
    assert dR <= 1e-12, f"{label}: dR {dR:.3e}"
    kap = np.linalg.cond(Ro[:k, :k])
    dQ = np.linalg.norm(Qg - Qo) / np.linalg.norm(Qo)
    assert dQ <= max(1e-12, 100 * U64 * kap) * q_extra, f"{label}: dQ {dQ:.3e} (cond {kap:.2e})"
    recon, orth = metrics(A, Qg, Rg, Jg, k)
    # The reconstruction is exact only when rank(S A) = rank(A) (Theorem on
    # correctness); otherwise the GPU must reach what the oracle reaches.
    recon_o, _ = metrics(A, Qo, Ro, orc["J"], k)
    assert recon <= max(1e-12, recon_o * (1 + 1e-6)), f"{label}: recon {recon:.3e}"
    assert orth <= 1e-12, f"{label}: orth {orth:.3e}"
    assert not Qg[:, k:].any() and not Rg[k:, :].any()
    assert np.array_equal(Rg, np.triu(Rg)) and np.all(np.diag(Rg)[:k] > 0)
    say(f"  {label}: rank {k} dR {dR:.2e} dQ {dQ:.2e} recon {recon:.2e} orth {orth:.2e}")


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,d,nnz,seed", [(1, 1, 1, 0), (1000, 13, 4, 0), (5000, 125, 4, 7),
                                          (777, 640, 8, 2 ** 40 + 3), (300, 32, 32, 5),
                                          (4097, 1280, 8, 123456789)])
def test_saso_bit_exact(P, m, d, nnz, seed):
    say(f"saso m={m} d={d} nnz={nnz} seed={seed}")
    rows, signs = P.saso_sample(m, d, nnz, seed)
    ro, so = O.saso_sample(m, d, nnz, seed)
    assert np.array_equal(to_np(rows).astype(np.int64), ro)
    assert np.array_equal(to_np(signs).astype(np.int64), so.astype(np.int64))


@pytest.mark.parametrize("m,n,d,nnz", [(1000, 7, 13, 4), (5000, 37, 50, 8), (20000, 100, 125, 4),
                                       (3001, 130, 170, 1), (70000, 20, 25, 8),
                                       (2000, 9, 640, 32)])
def test_sketch_parity(P, m, n, d, nnz):
    say(f"sketch m={m} n={n} d={d} nnz={nnz}")
    A = W.gaussian_matrix(m, n, seed=m + n)
    Ag = to_gpu(A)
    seed = 11
    S1 = to_np(P.sketch(Ag, d, nnz, seed))
    S2 = to_np(P.sketch(Ag, d, nnz, seed))
    assert np.array_equal(S1, S2), "sketch is not deterministic"
    rows, signs = O.saso_sample(m, d, nnz, seed)
    So = O.sketch(A, rows, signs, d)
    absS = O.sketch(np.abs(A), rows, np.ones_like(signs), d)
    p = np.bincount(rows.ravel(), minlength=d).max()
    bound = (2 * p + 4) * U64 * absS
    assert np.all(np.abs(S1 - So) <= bound + 1e-300)


# Sketch shapes reaching every kernel variant (with the small shapes above,
# which take 512 threads with one or two target rows per thread and 512- or
# 256-row sub-chunks): 1024 threads with two target rows on 1024-row
# sub-chunks (d = 1800 and 1500, the latter with nnz = 16 and with fewer
# rows than one sub-chunk), with three on 1024-row sub-chunks (d = 2560 and
# 3000) and, past 8 nonzeros per column, on 512-row ones (d = 2600), 512
# threads with eight (d = 4096), and the LDS variant past 4096.
@pytest.mark.parametrize("m,n,d,nnz", [(30000, 40, 1800, 8), (30000, 21, 1500, 16),
                                       (700, 12, 1500, 8), (30000, 37, 2560, 8),
                                       (20000, 33, 3000, 8), (20000, 15, 2600, 12),
                                       (40000, 20, 4096, 8), (30000, 24, 5000, 8),
                                       (25000, 9, 9000, 4)])
def test_sketch_parity_wide(P, m, n, d, nnz):
    test_sketch_parity(P, m, n, d, nnz)


@pytest.mark.parametrize("d,n", [(13, 10), (125, 100), (170, 130), (300, 257), (640, 512),
                                 (1500, 300), (2000, 150), (2600, 40)])
def test_qrcp_parity_separated(P, d, n):
    say(f"qrcp d={d} n={n}")
    X = W.column_scaled_well_separated(d, n, seed=d * 7 + n, ratio=1.05)
    Jg, Rg = P.qrcp(to_gpu(X))
    Jo, Ro = O.qrcp(X)
    Jg, Rg = to_np(Jg), to_np(Rg)
    assert np.array_equal(Jg, Jo)
    assert np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro) <= 1e-13
    assert np.array_equal(Rg, np.triu(Rg))


def test_qrcp_parity_2560x2048_stored(P):
    """The sketch shape of the 4,194,304 x 2,048 workload (d = 2560, the widest
    register-resident QRCP variant) against the oracle's QRCP stored in
    tests/golden/qrcp_2560x2048_sep105.txt (written by make_qrcp_golden.py,
    which calls only the oracle; the oracle takes minutes on this shape):
    pivots identical, diagonal and first superdiagonal of R to 1e-12
    relative to |R[0,0]|, and R^T R = X[:, J]^T X[:, J] on the device."""
    import os
    say("qrcp 2560 x 2048 (stored oracle result)")
    path = os.path.join(os.path.dirname(__file__), "golden", "qrcp_2560x2048_sep105.txt")
    rows = [ln.split() for ln in open(path) if not ln.startswith("#")]
    Jo = np.array([int(r[1]) for r in rows])
    diag_o = np.array([float.fromhex(r[2]) for r in rows])
    sup_o = np.array([float.fromhex(r[3]) for r in rows])
    d, n = 2560, 2048
    X = W.column_scaled_well_separated(d, n, seed=d * 7 + n, ratio=1.05)
    Xg = to_gpu(X)
    Jg, Rg = P.qrcp(Xg)
    assert np.array_equal(to_np(Jg), Jo)
    Rn = to_np(Rg)
    scale = abs(diag_o[0])
    assert np.max(np.abs(np.diag(Rn) - diag_o)) <= 1e-12 * scale
    assert np.max(np.abs(np.append(np.diag(Rn, 1), 0.0) - sup_o)) <= 1e-12 * scale
    XJ = Xg[:, Jg]
    dg = float(torch.linalg.norm(Rg.t() @ Rg - XJ.t() @ XJ) / torch.linalg.norm(Xg) ** 2)
    say(f"  pivots identical, ||R^T R - X_J^T X_J|| / ||X||^2 = {dg:.2e}")
    assert dg <= 1e-13
    assert np.array_equal(Rn, np.triu(Rn))


def test_qrcp_ties_zero_and_identity(P):
    say("qrcp ties")
    Jg, Rg = P.qrcp(to_gpu(np.eye(9, 6)))
    assert to_np(Jg).tolist() == list(range(6))
    assert np.array_equal(to_np(Rg), np.eye(6))
    Jg, Rg = P.qrcp(to_gpu(np.zeros((8, 5))))
    assert to_np(Jg).tolist() == list(range(5)) and not to_np(Rg).any()


CASES = [
    # label, m, n, d, nnz, spectrum kind, cond, tol
    ("c1-like-small", 3000, 60, 75, 4, "log", 1e6, 1e-14),
    ("ragged", 5007, 150, 188, 4, "log", 1e4, 1e-14),
    ("n1", 500, 1, 2, 1, "log", 1.0, 1e-14),
    ("tiles-and-tail", 20003, 200, 250, 8, "log", 1e8, 1e-14),
    ("nnz1-gamma1", 4000, 64, 64, 1, "log", 1e3, 1e-14),
    ("wide-16-blocks", 20000, 1024, 1280, 8, "log", 1e8, 1e-14),
    ("wide-ragged", 12001, 700, 875, 4, "log", 1e6, 1e-14),
    # Edges of the direct-load solve and Q product: a last panel of one
    # column (k = 129), fewer rows than one 128-row workgroup, m just above d.
    ("one-column-panel", 3000, 129, 162, 4, "log", 1e5, 1e-14),
    ("rows-below-tile", 90, 40, 50, 4, "log", 1e3, 1e-14),
    ("m-just-above-d", 170, 128, 160, 4, "log", 1e4, 1e-14),
]


@pytest.mark.parametrize("label,m,n,d,nnz,kind,cond,tol", CASES)
def test_factor_parity(P, label, m, n, d, nnz, kind, cond, tol):
    say(f"factor {label} m={m} n={n} d={d} nnz={nnz}")
    A = W.spectrum_matrix(m, n, W.logspaced_spectrum(n, cond), seed=m % 97)
    orc = O.cqrrpt(A, d, nnz, seed=5, tol=tol)
    gpu = P.factor(to_gpu(A), d, nnz, 5, tol)
    compare_factor(A, gpu, orc, label)


def test_factor_config_10000x100(P):
    """The 10,000 x 100 workload (cond 1e6, d = 125, nnz = 4, tol 1e-14)."""
    say("factor 10000x100")
    A, w = W.make_workload("fp64_10000x100_cond1e6")
    orc = O.cqrrpt(A, w["d"], w["nnz"], seed=0, tol=w["tol"])
    gpu = P.factor(to_gpu(A), w["d"], w["nnz"], 0, w["tol"])
    compare_factor(A, gpu, orc, "10000x100")


def test_factor_planted_rank(P):
    say("factor planted rank")
    m, n, r = 6000, 96, 40
    s = np.zeros(n)
    s[:r] = W.logspaced_spectrum(r, 1e3)
    A = W.spectrum_matrix(m, n, s, seed=3)
    for tol in (1e-11, 1e-6):
        orc = O.cqrrpt(A, 120, 8, seed=9, tol=tol)
        gpu = P.factor(to_gpu(A), 120, 8, 9, tol)
        assert orc["rank"] == r
        Qg, Rg, Jg, info = gpu
        assert info.rank == r
        assert np.array_equal(to_np(Jg)[:r], orc["J"][:r])
        Qn, Rn = to_np(Qg), to_np(Rg)
        recon, orth = metrics(A, Qn, Rn, to_np(Jg), r)
        assert recon <= 1e-12 and orth <= 1e-12
        assert not Qn[:, r:].any() and not Rn[r:, :].any()


def test_factor_cholesky_failure(P):
    """Cholesky stops early and the second rank stage truncates (Sec. 3.3).

    Rows of magnitude 1e10 next to rows of magnitude 1 with a one-nonzero
    sketch (8000 x 128, d = 128): the sketch keeps full rank (k_o = 128) but
    the preconditioned Gram is numerically singular. The oracle's pivots of
    rows 0..81 are positive with margin (row 81: 3.1e15); the pivot of row 82
    is 256 against a diagonal of 2e22, i.e. rounding noise, so the GPU must
    stop at row 82 or later, where exactly depends on summation order. The
    rank of stage 2 is robust (the diagonal ratio jumps from 2.5 to 1.9e8 at
    row 75) and must match, together with the factors on those 75 columns.
    """
    say("factor cholesky failure 8000x128 coherent nnz=1")
    A = W.high_coherence_matrix(8000, 128, 4, boost=1e10)
    orc = O.cqrrpt(A, 128, 1, seed=0, tol=1e-14)
    assert orc["rank_stage1"] == 128 and orc["rank"] == 75 and orc["chol_fail_col"] == 83
    gpu = P.factor(to_gpu(A), 128, 1, 0, 1e-14)
    info = gpu[3]
    say(f"  chol_fail_col gpu {info.chol_fail_col} oracle {orc['chol_fail_col']}")
    assert 82 <= info.chol_fail_col < 128 and info.status == 0
    compare_factor(A, gpu, orc, "cholesky-failure")


def test_factor_degenerate(P):
    say("factor zero / nonfinite")
    Z = np.zeros((400, 12))
    Qg, Rg, Jg, info = P.factor(to_gpu(Z), 15, 4, 1, 1e-14)
    assert info.rank == 0 and info.status == 0
    assert not to_np(Qg).any() and not to_np(Rg).any()
    rng = np.random.Generator(np.random.PCG64(1))
    B = rng.standard_normal((400, 12))
    B[17, 3] = np.nan
    with pytest.raises(P.CqrrptError):
        P.factor(to_gpu(B), 15, 4, 1, 1e-14)
    # argument checks (LAPACK-style negative codes)
    with pytest.raises(P.CqrrptError):
        P.factor(to_gpu(B[:, :5]), 4, 2, 1, 1e-14)   # d < n


def test_factor_deterministic_and_sync_entry(P):
    say("factor determinism")
    A = W.spectrum_matrix(9000, 80, W.logspaced_spectrum(80, 1e5), seed=4)
    Ag = to_gpu(A)
    f = P.Factorization(9000, 80, 100, 4)
    f.run(Ag, 3, 1e-14)
    Q1, R1, J1 = to_np(f.Q).copy(), to_np(f.R).copy(), to_np(f.J).copy()
    f.run(Ag, 3, 1e-14)
    assert np.array_equal(Q1, to_np(f.Q)) and np.array_equal(R1, to_np(f.R))
    assert np.array_equal(J1, to_np(f.J))
    Q2, R2, J2, rank = P.factor_sync(Ag, 100, 4, 3, 1e-14)
    assert rank == 80
    assert np.array_equal(Q1, to_np(Q2)) and np.array_equal(R1, to_np(R2))


IMPLICIT_CASES = [
    # label, m, n, d, nnz, spectrum kind, cond, tol (the planted and failing
    # cases truncate the rank below the first-stage one)
    ("implicit-c1-like", 3000, 60, 75, 4, "log", 1e6, 1e-14),
    ("implicit-tiles-and-tail", 20003, 200, 250, 8, "log", 1e8, 1e-14),
    ("implicit-planted", 6000, 96, 120, 8, "planted", 1e3, 1e-11),
    ("implicit-cholesky-failure", 8000, 128, 128, 1, "coherent", 1e10, 1e-14),
]


@pytest.mark.parametrize("label,m,n,d,nnz,kind,cond,tol", IMPLICIT_CASES)
def test_factor_implicit_q(P, label, m, n, d, nnz, kind, cond, tol):
    """Implicit Q (Sec. 2.1, arithmetic complexity): M = M_pre[:, :k] and
    Rpre = R_pre[:k, :k] against the oracle's, R and J bit-identical to the
    explicit call, and Q = M Rpre^{-1} (formed here on the host) matching
    the explicit Q with the same orthogonality and reconstruction bars.
    M_pre and R_pre are each formed through the solve with R_sk, so each
    carries a forward error of order u cond(R_sk) (a GPU and an oracle
    M_pre differ by rounding amplified that way); only their combination,
    Q = M_pre R_pre^{-1} and R = R_pre R_sk, is accurate to the FP64 bars.
    Both therefore take the bound used for Q."""
    import scipy.linalg
    say(f"factor implicit {label} m={m} n={n} d={d} nnz={nnz}")
    if kind == "planted":
        sv = np.zeros(n)
        sv[:40] = W.logspaced_spectrum(40, cond)
        A = W.spectrum_matrix(m, n, sv, seed=3)
    elif kind == "coherent":
        A = W.high_coherence_matrix(m, n, 4, boost=cond)
    else:
        A = W.spectrum_matrix(m, n, W.logspaced_spectrum(n, cond), seed=m % 97)
    orc = O.cqrrpt(A, d, nnz, seed=5 if kind == "log" else 0, tol=tol)
    seed = 5 if kind == "log" else 0
    Ag = to_gpu(A)
    Mg, Rpg, Rg, Jg, info = P.factor_implicit(Ag, d, nnz, seed, tol)
    Qe, Re, Je, info_e = P.factor(Ag, d, nnz, seed, tol)
    Mg, Rpg, Rg, Jg = to_np(Mg), to_np(Rpg), to_np(Rg), to_np(Jg)
    k = orc["rank"]
    assert info.rank == k == info_e.rank, f"{label}: rank {info.rank} vs {k}"
    # Pivots past the rank pick among noise-level columns (not unique): the
    # leading k must match the oracle, all of them the explicit call's.
    assert np.array_equal(Jg[:k], orc["J"][:k]) and np.array_equal(Jg, to_np(Je))
    assert np.array_equal(np.sort(Jg), np.arange(n))
    assert np.array_equal(Rg, to_np(Re)), f"{label}: R differs from the explicit call"
    assert not Mg[:, k:].any()
    assert not Rpg[k:, :].any() and not Rpg[:, k:].any()
    assert np.array_equal(Rpg, np.triu(Rpg)) and np.all(np.diag(Rpg)[:k] > 0)
    Rpo, Mpo = orc["Rpre"], orc["Mpre"][:, :k]
    kap = np.linalg.cond(orc["R"][:k, :k])
    bound = max(1e-12, 100 * U64 * kap)
    dRp = np.linalg.norm(Rpg[:k, :k] - Rpo) / np.linalg.norm(Rpo)
    assert dRp <= bound, f"{label}: dRpre {dRp:.3e} (cond {kap:.2e})"
    dM = np.linalg.norm(Mg[:, :k] - Mpo) / np.linalg.norm(Mpo)
    assert dM <= bound, f"{label}: dM {dM:.3e} (cond {kap:.2e})"
    Qi = np.zeros_like(Mg)
    Qi[:, :k] = scipy.linalg.solve_triangular(Rpg[:k, :k], Mg[:, :k].T, trans="T",
                                              lower=False).T
    dQ = np.linalg.norm(Qi - to_np(Qe)) / np.linalg.norm(to_np(Qe))
    assert dQ <= bound, f"{label}: implicit vs explicit Q {dQ:.3e}"
    recon, orth = metrics(A, Qi, Rg, Jg, k)
    recon_o, _ = metrics(A, orc["Q"], orc["R"], orc["J"], k)
    assert recon <= max(1e-12, recon_o * (1 + 1e-6)), f"{label}: recon {recon:.3e}"
    assert orth <= 1e-12, f"{label}: orth {orth:.3e}"
    say(f"  {label}: rank {k} dRpre {dRp:.2e} dM {dM:.2e} dQ {dQ:.2e} recon {recon:.2e} "
        f"orth {orth:.2e}")


def test_factor_implicit_degenerate(P):
    """Implicit Q on A = 0 (rank 0: M, R_pre and R all zero) and on an input
    holding a NaN (reported as non-finite, like the explicit entry)."""
    say("factor implicit zero / nonfinite")
    Z = np.zeros((400, 12))
    Mg, Rpg, Rg, Jg, info = P.factor_implicit(to_gpu(Z), 15, 4, 1, 1e-14)
    assert info.rank == 0 and info.status == 0
    assert not to_np(Mg).any() and not to_np(Rpg).any() and not to_np(Rg).any()
    rng = np.random.Generator(np.random.PCG64(2))
    B = rng.standard_normal((400, 12))
    B[5, 7] = np.inf
    with pytest.raises(P.CqrrptError):
        P.factor_implicit(to_gpu(B), 15, 4, 1, 1e-14)


# ---------------------------------------------------------------------------
# Mixed precision (FP32 preconditioning solve, FP64 elsewhere) with the
# adaptive CholeskyQR2 re-pass. Pivots and the first-stage rank come from the
# FP64 sketch QRCP in both modes, so they must equal the oracle's; Q must
# reach the FP64 orthogonality bar (with or without the pass); the
# reconstruction is FP32-level by the stability analysis of the
# preconditioned method and is stated against a loose bound, not matched.
# Which inputs need the pass: after column pivoting R_sk is graded, so the
# FP32 solve leaves one CholeskyQR pass orthogonal to about 1e-13 even at
# cond 1e10 (no pass); rows of magnitude 1e10 next to rows of magnitude 1
# (the coherent workload of Sec. 4.2) lose the small rows to FP32 rounding in
# the solve, and one pass leaves ||Q^T Q - I|| near 1e-10 (one pass).

@pytest.mark.parametrize("kind,cond,expect_pass", [("logspaced", 1e2, 0), ("logspaced", 1e10, 0),
                                                   ("coherent", 1e10, 1)])
def test_mixed_cholqr2(P, kind, cond, expect_pass):
    m, n, d, nnz = 40000, 256, 320, 8
    say(f"mixed m={m} n={n} {kind} {cond:.0e}")
    if kind == "logspaced":
        A = W.spectrum_matrix(m, n, W.logspaced_spectrum(n, cond), seed=11)
    else:
        A = W.high_coherence_matrix(m, n, 5, boost=cond)
    orc = O.cqrrpt(A, d, nnz, seed=2, tol=1e-14)
    Qg, Rg, Jg, info = P.factor(to_gpu(A), d, nnz, 2, 1e-14, mode=P.CQRRPT_MIXED_CHECKED)
    Qn, Rn, Jn = to_np(Qg), to_np(Rg), to_np(Jg)
    k = orc["rank"]
    assert k == n and info.rank == k and info.rank_stage1 == orc["rank_stage1"]
    assert np.array_equal(Jn, orc["J"])
    assert info.cholqr2_passes == expect_pass, (info.cholqr2_passes, info.orth_est)
    recon, orth = metrics(A, Qn, Rn, Jn, k)
    dR = np.linalg.norm(Rn - orc["R"]) / np.linalg.norm(orc["R"])
    say(f"  passes {info.cholqr2_passes} orth_est {info.orth_est:.2e} orth {orth:.2e} "
        f"recon {recon:.2e} dR {dR:.2e}")
    assert orth <= 1e-12
    assert recon <= 1e-5 and dR <= 1e-4
    assert np.array_equal(Rn, np.triu(Rn)) and np.all(np.diag(Rn) > 0)
    if expect_pass == 0:
        # The estimate is of ||Q^T Q - I||_2 for the returned Q.
        assert 0.0 < info.orth_est <= 5e-13 and info.orth_est <= 2 * orth + 1e-13
    else:
        assert info.orth_est > 1e-11


@pytest.mark.parametrize("cond", [1e2, 1e10])
def test_mixed_one_pass(P, cond):
    """CQRRPT_MIXED is the paper's method: FP32 preconditioning, one
    CholeskyQR pass, no estimate. Where the checked mode does not re-pass,
    its factors are the same bits (the same kernels up to the check)."""
    m, n, d, nnz = 40000, 256, 320, 8
    A = W.spectrum_matrix(m, n, W.logspaced_spectrum(n, cond), seed=11)
    Ag = to_gpu(A)
    Q1, R1, J1, i1 = P.factor(Ag, d, nnz, 2, 1e-14, mode=P.CQRRPT_MIXED)
    Q2, R2, J2, i2 = P.factor(Ag, d, nnz, 2, 1e-14, mode=P.CQRRPT_MIXED_CHECKED)
    assert i1.cholqr2_passes == 0 and i1.orth_est == 0.0 and i1.rank == n
    assert i2.cholqr2_passes == 0
    Q1, R1, J1 = to_np(Q1), to_np(R1), to_np(J1)
    assert np.array_equal(Q1, to_np(Q2)) and np.array_equal(R1, to_np(R2))
    assert np.array_equal(J1, to_np(J2))
    recon, orth = metrics(A, Q1, R1, J1, n)
    say(f"  mixed one pass cond {cond:.0e}: orth {orth:.2e} recon {recon:.2e}")
    assert orth <= 1e-12 and recon <= 1e-5


def test_fp64_mode_runs_no_repass(P):
    A = W.spectrum_matrix(5000, 64, W.logspaced_spectrum(64, 1e8), seed=12)
    _, _, _, info = P.factor(to_gpu(A), 80, 4, 3, 1e-14)
    assert info.cholqr2_passes == 0 and info.orth_est == 0.0


@pytest.mark.parametrize("mode_name", ["mixed", "mixed_checked"])
def test_mixed_rank_matches_oracle(P, mode_name):
    """Mixed modes on inputs whose rank is decided by the rank stages: the
    planted-rank input (first stage) and the coherent input whose Gram loses
    positive definiteness (Cholesky failure, then the second stage). Pivots
    and the first stage come from the FP64 sketch QRCP; the final rank must
    equal the FP64 oracle's, and the returned Q must meet the FP64
    orthogonality bar."""
    mode = {"mixed": P.CQRRPT_MIXED, "mixed_checked": P.CQRRPT_MIXED_CHECKED}[mode_name]
    s = np.zeros(96)
    s[:40] = W.logspaced_spectrum(40, 1e3)
    cases = [("planted", W.spectrum_matrix(6000, 96, s, seed=3), 120, 8, 9, 1e-11),
             ("planted-loose", W.spectrum_matrix(6000, 96, s, seed=3), 120, 8, 9, 1e-6),
             ("cholesky-failure", W.high_coherence_matrix(8000, 128, 4, boost=1e10), 128, 1, 0,
              1e-14)]
    for label, A, d, nnz, seed, tol in cases:
        say(f"{mode_name} {label}")
        orc = O.cqrrpt(A, d, nnz, seed=seed, tol=tol)
        Qg, Rg, Jg, info = P.factor(to_gpu(A), d, nnz, seed, tol, mode=mode)
        k = orc["rank"]
        Qn, Rn, Jn = to_np(Qg), to_np(Rg), to_np(Jg)
        say(f"  rank {info.rank} (oracle {k}), stage 1 {info.rank_stage1} "
            f"(oracle {orc['rank_stage1']}), chol fail {info.chol_fail_col} "
            f"(oracle {orc['chol_fail_col']}), passes {info.cholqr2_passes}")
        assert info.status == 0 and info.rank_stage1 == orc["rank_stage1"]
        assert info.rank == k, f"{label}: rank {info.rank} vs oracle {k}"
        assert np.array_equal(Jn[:k], orc["J"][:k])
        recon, orth = metrics(A, Qn, Rn, Jn, k)
        recon_o, _ = metrics(A, orc["Q"], orc["R"], orc["J"], k)
        say(f"  orth {orth:.2e} recon {recon:.2e} (oracle {recon_o:.2e})")
        assert orth <= 1e-12
        assert recon <= max(1e-5, 10 * recon_o)
        assert not Qn[:, k:].any() and not Rn[k:, :].any()


# ---------------------------------------------------------------------------
# The unpivoted precursor of Sec. 1.3 (cqrrpt_sketched_cholqr_ex) against the
# oracle's five steps: no pivots, R to 1e-12, Q to the cond-scaled bound.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,d,nnz,cond", [(3000, 60, 75, 4, 1e6), (20003, 200, 250, 8, 1e8),
                                            (12001, 700, 875, 4, 1e6), (500, 1, 2, 1, 1.0),
                                            (40000, 1024, 1280, 8, 1e10)])
def test_sketched_cholqr_parity(P, m, n, d, nnz, cond):
    say(f"precursor m={m} n={n} d={d} nnz={nnz} cond={cond:.0e}")
    A = W.spectrum_matrix(m, n, W.logspaced_spectrum(n, cond), seed=m % 89)
    orc = O.sketched_cholqr(A, d, nnz, seed=4)
    Qg, Rg, info = P.sketched_cholqr(to_gpu(A), d, nnz, 4)
    Qn, Rn = to_np(Qg), to_np(Rg)
    assert info.rank == orc["rank"] == n and info.rank_stage1 == n
    assert info.chol_fail_col == -1
    dR = np.linalg.norm(Rn - orc["R"]) / np.linalg.norm(orc["R"])
    kap = np.linalg.cond(orc["R"])
    dQ = np.linalg.norm(Qn - orc["Q"]) / np.linalg.norm(orc["Q"])
    recon = np.linalg.norm(A - Qn @ Rn) / np.linalg.norm(A)
    orth = np.linalg.norm(Qn.T @ Qn - np.eye(n), 2)
    say(f"  dR {dR:.2e} dQ {dQ:.2e} (cond {kap:.1e}) recon {recon:.2e} orth {orth:.2e}")
    assert dR <= 1e-12 and dQ <= max(1e-12, 100 * U64 * kap)
    assert recon <= 1e-12 and orth <= 1e-12
    assert np.array_equal(Rn, np.triu(Rn)) and np.all(np.diag(Rn) > 0)


def test_sketched_cholqr_zero_column(P):
    """An exactly zero last column: rank n - 1 from the zero trailing block,
    as in the oracle, with Q and R zero past it."""
    A = W.spectrum_matrix(2000, 20, W.logspaced_spectrum(20, 1e2), seed=8)
    A[:, 19] = 0.0
    orc = O.sketched_cholqr(A, 25, 4, seed=1)
    Qg, Rg, info = P.sketched_cholqr(to_gpu(A), 25, 4, 1)
    Qn, Rn = to_np(Qg), to_np(Rg)
    assert info.rank == orc["rank"] == 19 and info.rank_stage1 == 19
    assert not Qn[:, 19:].any() and not Rn[19:, :].any()
    assert np.linalg.norm(Rn - orc["R"]) / np.linalg.norm(orc["R"]) <= 1e-12


# ---------------------------------------------------------------------------
# FP32 CholeskyQR lines + FP64 CholeskyQR2 (CQRRPT_MIXED_FP32_CHOLQR2): the
# solve, Gram and Q product on FP32 matrix cores with FP32 accumulation, then
# an FP64 pass that always runs. Pivots and ranks must equal the FP64
# oracle's; Q must reach the FP64 orthogonality bar after the pass; the
# reconstruction is FP32-level (stated, not matched).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,cond", [("logspaced", 1e2), ("logspaced", 1e10),
                                       ("coherent", 1e10), ("planted", 1e3),
                                       ("cholesky-failure", 1e10)])
def test_mixed_fp32_lines_cholqr2(P, kind, cond):
    say(f"fp32 lines + cholqr2 {kind} {cond:.0e}")
    if kind == "logspaced":
        A = W.spectrum_matrix(40000, 256, W.logspaced_spectrum(256, cond), seed=11)
        d, nnz, seed, tol = 320, 8, 2, 1e-14
    elif kind == "coherent":
        A = W.high_coherence_matrix(40000, 256, 5, boost=cond)
        d, nnz, seed, tol = 320, 8, 2, 1e-14
    elif kind == "planted":
        s = np.zeros(96)
        s[:40] = W.logspaced_spectrum(40, cond)
        A = W.spectrum_matrix(6000, 96, s, seed=3)
        d, nnz, seed, tol = 120, 8, 9, 1e-11
    else:
        A = W.high_coherence_matrix(8000, 128, 4, boost=cond)
        d, nnz, seed, tol = 128, 1, 0, 1e-14
    orc = O.cqrrpt(A, d, nnz, seed=seed, tol=tol)
    Qg, Rg, Jg, info = P.factor(to_gpu(A), d, nnz, seed, tol, mode=P.CQRRPT_MIXED_FP32_CHOLQR2)
    Qn, Rn, Jn = to_np(Qg), to_np(Rg), to_np(Jg)
    k = orc["rank"]
    say(f"  rank {info.rank} (oracle {k}) stage 1 {info.rank_stage1} passes "
        f"{info.cholqr2_passes} chol fail {info.chol_fail_col}")
    assert info.status == 0 and info.rank_stage1 == orc["rank_stage1"]
    assert info.rank == k
    assert np.array_equal(Jn[:k], orc["J"][:k])
    assert info.cholqr2_passes == 1
    recon, orth = metrics(A, Qn, Rn, Jn, k)
    recon_o, _ = metrics(A, orc["Q"], orc["R"], orc["J"], k)
    say(f"  orth {orth:.2e} recon {recon:.2e} (oracle {recon_o:.2e})")
    assert orth <= 1e-12
    assert recon <= max(1e-5, 10 * recon_o)
    assert not Qn[:, k:].any() and not Rn[k:, :].any()
    assert np.array_equal(Rn, np.triu(Rn)) and np.all(np.diag(Rn)[:k] > 0)


# ---------------------------------------------------------------------------
# Dense sketching operators (Gaussian, SRHT; cqrrpt_factor_dense_ex) against
# the oracle's CQRRPT with the same operator. The Gaussian entries come from
# the same counter-based draws on both sides but through each side's own
# log/cos/sin, so they agree to a few ulps; pivots and ranks must be
# identical on inputs with pivot margins, R to 1e-12, Q to the cond bound.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["gaussian", "srht"])
@pytest.mark.parametrize("m,n,d,spec", [(3000, 60, 75, "log1e6"), (20003, 200, 250, "log1e8"),
                                        (5000, 100, 125, "separated"), (8192, 64, 80, "log1e4")])
def test_dense_sketch_factor_parity(P, kind, m, n, d, spec):
    say(f"dense sketch {kind} m={m} n={n} d={d} {spec}")
    if spec == "separated":
        A = W.column_scaled_well_separated(m, n, seed=41, ratio=1.1)
    else:
        A = W.spectrum_matrix(m, n, W.logspaced_spectrum(n, float(spec[3:])), seed=m % 83)
    orc = O.cqrrpt_dense(A, d, kind, seed=6, tol=1e-14)
    code = P.SKETCH_GAUSSIAN if kind == "gaussian" else P.SKETCH_SRHT
    gpu = P.factor_dense(to_gpu(A), d, code, 6, 1e-14)
    compare_factor(A, gpu, orc, f"{kind} {m}x{n}")


# ---------------------------------------------------------------------------
# HQRRP on the sketch (Sec. 5.2.2; cqrrpt_hqrrp, cqrrpt_factor_hqrrp_ex)
# against the oracle's hqrrp. The sample Omega X is one product on each side
# (sums in different orders), so pivots must be identical wherever the
# sample's norms are not within rounding of each other (random inputs), R to
# 1e-13 relative; the GEQP3 order is not expected.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,n,b,s,spec", [(60, 40, 4, 4, "gauss"), (50, 50, 16, 8, "log1e6"),
                                          (300, 257, 16, 8, "log1e10"), (700, 333, 7, 3, "gauss"),
                                          (1280, 1024, 16, 8, "log1e8")])
def test_hqrrp_parity(P, d, n, b, s, spec):
    say(f"hqrrp d={d} n={n} b={b} s={s} {spec}")
    if spec == "gauss":
        X = W.gaussian_matrix(d, n, seed=d + n)
    else:
        X = W.spectrum_matrix(d, n, W.logspaced_spectrum(n, float(spec[3:])), seed=d % 97)
    Jo, Ro = O.hqrrp(X, b, s, seed=5)
    Jg, Rg, info = P.hqrrp(to_gpu(X), b, s, 5)
    assert info.status == 0
    Jg, Rg = to_np(Jg), to_np(Rg)
    assert np.array_equal(Jg, Jo)
    dR = np.linalg.norm(Rg - Ro) / np.linalg.norm(Ro)
    assert dR <= 1e-13, f"dR {dR:.2e}"
    assert np.array_equal(Rg, np.triu(Rg)) and np.all(np.diag(Rg) >= 0)
    say(f"  dR {dR:.2e}")


def test_hqrrp_zero_columns_and_limits(P):
    # Exactly zero columns are chosen last and leave zero diagonal entries
    # (the zero-diagonal rule of the sample update keeps the rest finite);
    # shapes past the register-resident limits are refused.
    X = W.gaussian_matrix(80, 30, seed=3)
    X[:, [4, 17]] = 0.0
    Jo, Ro = O.hqrrp(X, 8, 4, seed=2)
    Jg, Rg, info = P.hqrrp(to_gpu(X), 8, 4, 2)
    Jg, Rg = to_np(Jg), to_np(Rg)
    assert np.array_equal(Jg, Jo) and set(Jg[-2:].tolist()) == {4, 17}
    assert np.all(np.isfinite(Rg)) and Rg[-1, -1] == 0.0 and Rg[-2, -2] == 0.0
    assert np.linalg.norm(Rg - Ro) <= 1e-13 * np.linalg.norm(Ro)
    for d, n, b, s in ((4000, 100, 16, 8), (2600, 2100, 16, 8), (100, 50, 17, 0),
                       (100, 50, 16, 9)):
        assert P.lib().cqrrpt_hqrrp_workspace_bytes(d, n, b, s) == 0


@pytest.mark.parametrize("m,n,d,nnz,spec", [(20003, 200, 250, 8, "log1e8"),
                                            (8192, 100, 125, 4, "cliff"),
                                            (30000, 512, 640, 8, "log1e12")])
def test_factor_hqrrp_parity(P, m, n, d, nnz, spec):
    say(f"factor hqrrp m={m} n={n} d={d} {spec}")
    if spec == "cliff":
        # A drop of 100x after 60 columns, then a graded tail well above the
        # rounding level (pivot decisions there stay defined).
        s = np.concatenate([np.geomspace(1.0, 1e-6, 60), np.geomspace(1e-8, 1e-10, n - 60)])
        A = W.spectrum_matrix(m, n, s, seed=3)
    else:
        A = W.spectrum_matrix(m, n, W.logspaced_spectrum(n, float(spec[3:])), seed=m % 89)
    orc = O.cqrrpt_hqrrp(A, d, nnz, seed=7, tol=1e-14, b=16, s=8, hseed=11)
    gpu = P.factor_hqrrp(to_gpu(A), d, nnz, 7, 1e-14, block=16, oversample=8, hseed=11)
    compare_factor(A, gpu, orc, f"hqrrp {m}x{n}")
