"""Seeded synthetic inputs shaped like the paper's workloads.

Every matrix here is FP64 and is returned column-major (Fortran order), the
layout the library expects. Nothing in this module performs any step of the
factorization itself; it only synthesises inputs:

* ``spectrum_matrix``: A = U diag(s) V^T (+ iid Gaussian noise) with U, V
  Haar-distributed orthonormal factors. The paper builds its pivot-quality
  test matrices this way (Sec. 4.1: singular vectors from orthogonalised
  Gaussian matrices, prescribed spectra).
* ``gaussian_matrix``: iid N(0,1) entries, optionally with per-column scales;
  the paper's speed benchmarks use iid Gaussian inputs (Sec. 5).
* ``high_coherence_matrix``: the stacked-identity construction of Sec. 4.2.
* named recipes for the five workloads this library is measured on.

Haar factors are drawn as the Q factor of a Gaussian matrix's QR with the
signs fixed so that R has a positive diagonal (Mezzadri, Notices AMS 2007).
"""

import math

import numpy as np


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def haar_orthonormal(rng, m, n):
    """m x n matrix with orthonormal columns, Haar distributed."""
    G = rng.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    sgn = np.where(np.diag(R) < 0.0, -1.0, 1.0)
    return Q * sgn


def logspaced_spectrum(n, cond):
    """s_i = cond^(-i/(n-1)), i = 0..n-1 (1 down to 1/cond, endpoints included)."""
    if n == 1:
        return np.ones(1)
    e = math.log10(cond)
    return 10.0 ** (-e * np.arange(n) / (n - 1))


def planted_spectrum(n, rank, cond):
    """Geometric from 1 down to 1/cond over the first ``rank`` entries, then 0."""
    s = np.zeros(n)
    s[:rank] = logspaced_spectrum(rank, cond)
    return s


def spectrum_matrix(m, n, s, seed, noise_std=0.0):
    """A = U diag(s) V^T + noise_std * N(0,1), column-major FP64."""
    rng = _rng(seed)
    U = haar_orthonormal(rng, m, n)
    V = haar_orthonormal(rng, n, n)
    A = (U * np.asarray(s, dtype=np.float64)) @ V.T
    if noise_std:
        A += noise_std * rng.standard_normal((m, n))
    return np.asfortranarray(A)


def gaussian_matrix(m, n, seed, col_scale_range=None):
    """iid N(0,1) entries; with ``col_scale_range=(lo, hi)`` every column is
    multiplied by exp(U(ln lo, ln hi)) (log-uniform column scales)."""
    rng = _rng(seed)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    if col_scale_range is not None:
        lo, hi = col_scale_range
        c = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))
        A *= c
    return A


def high_coherence_matrix(m, n, seed, boost=1e10):
    """Sec. 4.2: stack floor(m/n) copies of I_n plus the leading rows of one
    more, multiply n randomly chosen rows by ``boost``, then rotate by a
    random n x n orthogonal matrix."""
    rng = _rng(seed)
    reps = m // n
    M = np.vstack([np.eye(n)] * reps + [np.eye(n)[: m - reps * n]])
    rows = rng.choice(m, size=n, replace=False)
    M[rows, :] *= boost
    V = haar_orthonormal(rng, n, n)
    return np.asfortranarray(M @ V)


def column_scaled_well_separated(m, n, seed, ratio=2.0):
    """Gaussian matrix whose column j is scaled by ratio^(-rank_j) for a random
    permutation rank_j: column norms are separated by a factor ``ratio``, so
    max-norm pivot decisions have a wide margin at every step."""
    rng = _rng(seed)
    A = rng.standard_normal((m, n))
    A /= np.linalg.norm(A, axis=0)
    perm = rng.permutation(n)
    A *= ratio ** (-perm.astype(np.float64))
    return np.asfortranarray(A)


# ---------------------------------------------------------------------------
# Named workloads (sizes and parameters of the measured configurations)
# ---------------------------------------------------------------------------

WORKLOADS = {
    # Plain FP64, full rank, cond 1e6 log-spaced spectrum.
    "fp64_10000x100_cond1e6": dict(m=10_000, n=100, d=125, nnz=4, tol=1e-14,
                                   kind="logspaced", cond=1e6, noise=0.0),
    # Planted rank 512 of 1024, geometric 1..1e-10, noise 1e-15.
    "fp64_131072x1024_rank512": dict(m=131_072, n=1_024, d=1_280, nnz=8, tol=1e-14,
                                     kind="planted", rank=512, cond=1e10, noise=1e-15),
    # Full rank, cond 1e10 log-spaced; FP64 and mixed forms.
    "mixed_1048576x512_cond1e10": dict(m=1_048_576, n=512, d=640, nnz=8, tol=1e-14,
                                       kind="logspaced", cond=1e10, noise=0.0),
    # Large: planted rank 1536 of 2048, geometric 1..1e-12, noise 1e-16.
    "fp64_4194304x2048_rank1536": dict(m=4_194_304, n=2_048, d=2_560, nnz=8, tol=1e-14,
                                       kind="planted", rank=1_536, cond=1e12, noise=1e-16),
}


def spectrum_matrix_gpu(m, n, s, seed, noise_std=0.0, device="cuda"):
    """Device-side version of ``spectrum_matrix`` for large inputs: the same
    recipe (Haar U, V from positive-diagonal QR of Gaussians, A = U diag(s) V^T
    plus noise), drawn with torch's seeded device generator. Returns a
    column-major FP64 torch tensor on ``device``."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))

    def haar(rows, cols):
        G = torch.randn((cols, rows), dtype=torch.float64, device=device, generator=gen).t()
        Q, R = torch.linalg.qr(G)
        sgn = torch.where(torch.diagonal(R) < 0, -1.0, 1.0).to(torch.float64)
        return Q * sgn

    U = haar(m, n)
    V = haar(n, n)
    sv = torch.as_tensor(np.asarray(s, dtype=np.float64), device=device)
    A = (U * sv) @ V.t()
    del U
    if noise_std:
        A += noise_std * torch.randn((n, m), dtype=torch.float64, device=device,
                                     generator=gen).t()
    return A.t().contiguous().t()


def spectrum_matrix_gpu_blocked(m, n, s, seed, noise_std=0.0, device="cuda",
                                block_rows=1 << 18):
    """``spectrum_matrix_gpu`` for matrices too large for a device QR next to
    their own copies: the same distribution, built in the output buffer one
    row block at a time. U is the Q factor of a Gaussian G by CholeskyQR2
    (G = U R with R = R2 R1, R1 = chol(G^T G), R2 = chol(U1^T U1),
    U1 = G R1^{-1}); R has a positive diagonal, so U is Haar distributed
    (the positive-diagonal QR of a Gaussian). Then A = U (diag(s) V^T), V Haar
    from the host, plus noise. Every row block draws its Gaussians from its
    own seeded generator; the n x n factorizations run on the host in FP64.
    Peak device memory: the m x n output plus one block."""
    import torch

    A = torch.empty((n, m), dtype=torch.float64, device=device).t()
    blocks = [(r, min(m, r + block_rows)) for r in range(0, m, block_rows)]
    gen = torch.Generator(device=device)
    for b, (r0, r1) in enumerate(blocks):
        gen.manual_seed(int(seed) * 1_000_003 + b)
        A[r0:r1] = torch.randn((n, r1 - r0), dtype=torch.float64, device=device,
                               generator=gen).t()

    def gram():
        G = torch.zeros((n, n), dtype=torch.float64, device=device)
        for r0, r1 in blocks:
            X = A[r0:r1]
            G += X.t() @ X
        return G.cpu().numpy()

    def right_multiply(W):
        Wd = torch.as_tensor(W, device=device)
        for r0, r1 in blocks:
            A[r0:r1] = A[r0:r1] @ Wd

    for _ in range(2):
        G = gram()
        R = np.linalg.cholesky((G + G.T) * 0.5).T  # upper, positive diagonal
        right_multiply(np.linalg.inv(R))
    V = haar_orthonormal(_rng(seed + 7_919), n, n)
    right_multiply(np.asarray(s, dtype=np.float64)[:, None] * V.T)
    if noise_std:
        for b, (r0, r1) in enumerate(blocks):
            gen.manual_seed(int(seed) * 1_000_003 + len(blocks) + b)
            A[r0:r1] += noise_std * torch.randn((n, r1 - r0), dtype=torch.float64,
                                                device=device, generator=gen).t()
    return A


# Above this many elements the device workloads are built block by block.
BLOCKED_ELEMENTS = 1 << 31


def make_workload_gpu(name, seed=0, m=None, device="cuda"):
    """Named workload built on the device (``spectrum_matrix_gpu``, or the
    block-by-block ``spectrum_matrix_gpu_blocked`` for the largest sizes)."""
    w = dict(WORKLOADS[name])
    if m is not None:
        w["m"] = m
    n = w["n"]
    if w["kind"] == "logspaced":
        s = logspaced_spectrum(n, w["cond"])
    else:
        s = planted_spectrum(n, w["rank"], w["cond"])
    if w["m"] * n > BLOCKED_ELEMENTS:
        return spectrum_matrix_gpu_blocked(w["m"], n, s, seed, w["noise"], device), w
    return spectrum_matrix_gpu(w["m"], n, s, seed, w["noise"], device), w


def make_workload(name, seed=0, m=None):
    """Build the input matrix of a named workload (optionally with fewer rows)."""
    w = dict(WORKLOADS[name])
    if m is not None:
        w["m"] = m
    mm, n = w["m"], w["n"]
    if w["kind"] == "logspaced":
        s = logspaced_spectrum(n, w["cond"])
    else:
        s = planted_spectrum(n, w["rank"], w["cond"])
    A = spectrum_matrix(mm, n, s, seed, w["noise"])
    return A, w


# ---------------------------------------------------------------------------
# Serving stream: requests arrive as a Poisson process; each is an iid
# Gaussian matrix with log-uniform column scales, log-uniform height and a
# width drawn from a fixed set; d = ceil(1.25 n), nnz = 4, tol = 1e-14.
# ---------------------------------------------------------------------------
SERVING = dict(rate_per_s=200.0, m_range=(20_000, 500_000), n_set=(64, 128, 256, 512, 1024),
               col_scale_range=(1e-4, 1.0), nnz=4, tol=1e-14)


def serving_stream(count, seed=0, rate_per_s=None, m_range=None, n_set=None):
    """Arrival times (s, cumulative exponential gaps) and shapes of ``count``
    requests: list of dicts with t, m, n, d, nnz, tol and the request's own
    matrix/sketch seed (index + 1)."""
    rate = SERVING["rate_per_s"] if rate_per_s is None else rate_per_s
    lo, hi = SERVING["m_range"] if m_range is None else m_range
    widths = SERVING["n_set"] if n_set is None else n_set
    rng = _rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    ms = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)
    ns = rng.choice(np.asarray(widths, dtype=np.int64), size=count)
    out = []
    for i in range(count):
        n = int(ns[i])
        m = max(int(ms[i]), math.ceil(1.25 * n))
        out.append(dict(t=float(t[i]), m=m, n=n, d=math.ceil(1.25 * n), nnz=SERVING["nnz"],
                        tol=SERVING["tol"], seed=i + 1))
    return out


def serving_matrix_gpu(m, n, seed, device="cuda"):
    """Device-side serving request: iid N(0,1) times log-uniform column
    scales from ``SERVING['col_scale_range']``, column-major FP64."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    lo, hi = SERVING["col_scale_range"]
    A = torch.randn((n, m), dtype=torch.float64, device=device, generator=gen)
    c = torch.exp(torch.empty(n, dtype=torch.float64, device=device).uniform_(
        math.log(lo), math.log(hi), generator=gen))
    A *= c[:, None]
    return A.t()
