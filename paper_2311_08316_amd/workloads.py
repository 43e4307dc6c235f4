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


def make_workload_gpu(name, seed=0, m=None, device="cuda"):
    """Named workload built on the device (see ``spectrum_matrix_gpu``)."""
    w = dict(WORKLOADS[name])
    if m is not None:
        w["m"] = m
    n = w["n"]
    if w["kind"] == "logspaced":
        s = logspaced_spectrum(n, w["cond"])
    else:
        s = planted_spectrum(n, w["rank"], w["cond"])
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
