"""CQRRPT oracle: a plain, slow, FP64 CPU implementation of the method.

THIS MODULE IS TEST INFRASTRUCTURE. Only the test suite, the package's smoke
check and the benchmark's CPU-baseline leg may import or call it. The product
path (the HIP library behind ``include/cqrrpt.h`` and its Python binding) never
imports, links or executes anything here, and nothing here imports the product.

Paper: Melnichenko, Balabanov, Murray, Demmel, Mahoney, Luszczek,
"CholeskyQR with Randomization and Pivoting for Tall Matrices (CQRRPT)",
arXiv:2311.08316.

What is computed, step by step, in the paper's order (Algorithm 2,
``cqrrpt_core``, with the sketching operator drawn as in Algorithm 1):

  S1  sample a SASO S (d x m): every column has exactly ``nnz`` nonzeros at
      distinct rows chosen uniformly, with values +-1/sqrt(nnz)   (Sec. 2.3.1)
  S2  sketch  Ahat = S A                                          (Alg. 2, sketch)
  S3  Householder QR with max-norm column pivoting of Ahat -> J, R_sk
                                                                  (Alg. 2, qrcp;
      Sec. 1 and 5 name LAPACK GEQP3, i.e. Businger-Golub pivoting)
  S4  first-stage rank bound k_o                                  (Sec. 3.3, first stage)
  S5  M_pre = A[:, J[:k_o]] R_sk[:k_o, :k_o]^{-1}                  (Alg. 2, precondition)
  S6  G = M_pre^T M_pre                                           (Alg. 2, Gram)
  S7  R_pre = chol(G), truncating at the first failing pivot      (Alg. 2; Remark in
                                                                   Sec. 3.3 on Cholesky
                                                                   failure)
  S8  second-stage rank k from cond(diag(R_pre[:l, :l])) <= sqrt(eps_tol/u),
      eps_tol = 100 u, so the threshold is 10                     (Sec. 3.3, second stage)
  S9  Q = M_pre[:, :k] R_pre[:k, :k]^{-1}                          (Alg. 2, Q-factor)
  S10 R = R_pre[:k, :k] R_sk[:k, :]                                (Alg. 2, undo preconditioning)

Also here: the unpivoted precursor of Sec. 1.3 (``sketched_cholqr``): sketch,
unpivoted QR of the sketch, precondition, CholeskyQR, for full-rank inputs;
the dense Gaussian and SRHT operators of Sec. 2.3.1 (``cqrrpt_dense``); and
HQRRP, the randomized block-pivoted QR of Sec. 5.2.2, in place of GEQP3 on
the sketch (``hqrrp``, ``cqrrpt_hqrrp``).

Readings where the paper is silent:
  * random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the seed,
    one counter stream per column of S; Floyd's subset sampler (Bentley and
    Floyd, CACM 1987) for the distinct rows; Lemire's multiply-shift with
    rejection (ACM TOMACS 2019) for exact uniform integers.
  * the 1/sqrt(nnz) scale is applied once to the accumulated signed sum.
  * pivot ties go to the smallest original column index; column norms are
    recomputed from scratch at every step (no downdating).
  * Householder reflector in the LAPACK convention beta = -sign(alpha)||x||
    (sign(0) = +1); rows of R_sk with a negative diagonal are negated at the
    end, so diag(R_sk) >= 0 and Q, R are unique.
  * stage 1 uses ``tol`` in place of the unit roundoff u, compares squared
    Frobenius norms, and s is the largest |entry| of R_sk.
  * a Cholesky pivot that is <= 0 or not finite at 0-based column j sets k = j.
  * outputs are full-size: Q is m x n and R is n x n, zero past the rank.

Dense steps use library primitives (matrix product, triangular solve) as the
paper's own implementation does (BLAS TRSM/SYRK, Sec. 1.2 and App. A.1).
"""

import math

import numpy as np
import scipy.linalg
import scipy.sparse

# ---------------------------------------------------------------------------
# S1. Random numbers and the SASO sampler
# ---------------------------------------------------------------------------

_MASK32 = np.uint64(0xFFFFFFFF)
# Philox4x32 multipliers and Weyl key increments, from the published
# definition (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4 "Philox").
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
# Fourth counter word of every SASO draw: ASCII "SAS0". Separates these
# streams from any other use of the same key.
SASO_DOMAIN = 0x53415330


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds, vectorised over numpy arrays of uint32 words.

    One round maps (c0, c1, c2, c3) with key (k0, k1) to
      (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
    the key is bumped by the Weyl constants (W0, W1) between rounds.
    """
    c0, c1, c2, c3, k0, k1 = (np.asarray(x, dtype=np.uint64) & _MASK32
                              for x in (c0, c1, c2, c3, k0, k1))
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
        p0 = np.uint64(PHILOX_M0) * c0
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


class _ColumnWordStream:
    """The stream of 32-bit words that column j of S consumes, for many j at once.

    Word w of column j is word (w mod 4) of Philox4x32-10 applied to the
    counter (lo32(j), hi32(j), w div 4, SASO_DOMAIN) under the key
    (lo32(seed), hi32(seed)).
    """

    def __init__(self, seed, cols):
        self.cols = np.asarray(cols, dtype=np.uint64)
        self.k0 = seed & 0xFFFFFFFF
        self.k1 = (seed >> 32) & 0xFFFFFFFF
        self._cache = {}

    def block(self, b):
        if b not in self._cache:
            lo = self.cols & _MASK32
            hi = self.cols >> np.uint64(32)
            self._cache[b] = philox4x32_10(lo, hi, b, SASO_DOMAIN, self.k0, self.k1)
        return self._cache[b]

    def word(self, w):
        """Word index ``w`` (array, one entry per column) of every column."""
        w = np.asarray(w, dtype=np.int64)
        w = np.broadcast_to(w, self.cols.shape)
        out = np.empty(self.cols.shape, dtype=np.uint32)
        for b in np.unique(w // 4):
            sel = (w // 4) == b
            words = self.block(int(b))
            for lane in range(4):
                s2 = sel & ((w % 4) == lane)
                out[s2] = words[lane][s2]
        return out


def lemire_uniform(stream, pos, s):
    """Exact uniform integers in [0, s) by Lemire's multiply-shift with rejection.

    ``pos`` is the per-column index of the next unused word; it is advanced in
    place. Draw x, form the 64-bit product x*s, and accept the high word unless
    the low word falls below (2^32 - s) mod s, in which case draw again.
    """
    s = np.asarray(s, dtype=np.uint64)
    x = stream.word(pos).astype(np.uint64)
    pos += 1
    prod = x * s
    low = prod & _MASK32
    thresh = (np.uint64(1 << 32) - s) % s
    reject = low < thresh
    while np.any(reject):
        idx = np.flatnonzero(reject)
        x2 = stream.word(pos)[idx].astype(np.uint64)
        pos[idx] += 1
        prod[idx] = x2 * s[idx] if s.ndim else x2 * s
        low[idx] = prod[idx] & _MASK32
        reject = low < thresh
    return (prod >> np.uint64(32)).astype(np.int64)


def floyd_sample(d, nnz, uniform):
    """Floyd's algorithm: ``nnz`` distinct integers from [0, d), in draw order.

    ``uniform(t)`` must return an exact uniform integer in [0, t]
    (vectorised: one value per independent instance). For t = d-nnz, ..., d-1
    a draw r in [0, t] is kept unless it was already taken, in which case t
    itself is taken instead.
    """
    picks = []
    for step in range(nnz):
        t = d - nnz + step
        r = uniform(t)
        taken = np.zeros(r.shape, dtype=bool)
        for prev in picks:
            taken |= prev == r
        picks.append(np.where(taken, t, r))
    return np.stack(picks, axis=-1) if picks else np.zeros((0,), dtype=np.int64)


def saso_sample(m, d, nnz, seed):
    """The SASO of Sec. 2.3.1 as (rows, signs): column j of S holds +-1/sqrt(nnz)
    at rows[j, t] with sign signs[j, t], t < nnz; the rows of a column are
    distinct. Word 0 of column j's stream gives the signs (bit t set means the
    t-th entry is negative); words 1, 2, ... feed Floyd's sampler.
    """
    if not (1 <= nnz <= 32 and nnz <= d):
        raise ValueError("need 1 <= nnz <= min(32, d)")
    cols = np.arange(m, dtype=np.uint64)
    stream = _ColumnWordStream(seed, cols)
    sign_word = stream.word(np.zeros(m, dtype=np.int64)).astype(np.int64)
    signs = np.empty((m, nnz), dtype=np.int8)
    for t in range(nnz):
        signs[:, t] = np.where((sign_word >> t) & 1, -1, 1)
    pos = np.ones(m, dtype=np.int64)
    rows = floyd_sample(d, nnz, lambda t: lemire_uniform(stream, pos, t + 1))
    return rows.astype(np.int64).reshape(m, nnz), signs


def saso_matrix(m, d, nnz, seed):
    """S as a scipy sparse d x m matrix with entries +-1/sqrt(nnz)."""
    rows, signs = saso_sample(m, d, nnz, seed)
    cols = np.repeat(np.arange(m), nnz)
    vals = signs.reshape(-1).astype(np.float64) * (1.0 / math.sqrt(nnz))
    return scipy.sparse.csr_matrix((vals, (rows.reshape(-1), cols)), shape=(d, m))


# ---------------------------------------------------------------------------
# Dense sketching operators (Sec. 2.3.1: Gaussian matrices and SRHTs)
# ---------------------------------------------------------------------------

GAUSS_DOMAIN = 0x47415553       # "GAUS"
HQRRP_DOMAIN = 0x48515250       # "HQRP": the sampling matrix of ``hqrrp``
SRHT_SIGN_DOMAIN = 0x53524844   # "SRHD"
SRHT_ROW_DOMAIN = 0x53524852    # "SRHR"


def _u53(hi_word, lo_word):
    """53-bit integer from the top 27 bits of one word and the top 26 of
    another."""
    return (np.asarray(hi_word, dtype=np.uint64) >> np.uint64(5)) * np.uint64(1 << 26) + \
        (np.asarray(lo_word, dtype=np.uint64) >> np.uint64(6))


def gaussian_sketch_matrix(m, d, seed, domain=GAUSS_DOMAIN):
    """S (d x m) with iid N(0, 1/d) entries (Sec. 2.3.1, Gaussian matrices).
    Entries (2q, j) and (2q + 1, j) come from one Philox4x32-10 block with
    counter (lo32(j), hi32(j), q, "GAUS"): u1 = (U(w0, w1) + 1) 2^-53 in
    (0, 1], u2 = U(w2, w3) 2^-53 in [0, 1), where U takes the top 27 bits of
    its first word and the top 26 of its second; Box-Muller gives
    sqrt(-2 ln u1) cos(2 pi u2) for the even row and the sine for the odd."""
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    j = np.arange(m, dtype=np.uint64)[None, :]
    r = np.arange(d, dtype=np.uint64)[:, None]
    w0, w1, w2, w3 = philox4x32_10(j & _MASK32, j >> np.uint64(32), r >> np.uint64(1),
                                   domain, k0, k1)
    u1 = (_u53(w0, w1) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = _u53(w2, w3).astype(np.float64) * 2.0 ** -53
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * math.pi * u2
    z = np.where((r & np.uint64(1)) == 0, rad * np.cos(ang), rad * np.sin(ang))
    return z * (1.0 / math.sqrt(d))


class _ScalarWordStream:
    """Word w = output word (w mod 4) of Philox4x32-10 at counter
    (lo32(w div 4), hi32(w div 4), 0, domain)."""

    def __init__(self, seed, domain):
        self.k0, self.k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
        self.domain = domain
        self.pos = 0
        self.block = None

    def next(self):
        b, lane = divmod(self.pos, 4)
        if lane == 0 or self.block is None:
            self.block = [int(x) for x in philox4x32_10(b & 0xFFFFFFFF, b >> 32, 0, self.domain,
                                                        self.k0, self.k1)]
        self.pos += 1
        return self.block[lane]

    def uniform(self, s):
        """Exact uniform integer in [0, s), Lemire's multiply-shift with rejection."""
        thresh = ((1 << 32) - s) % s
        while True:
            prod = self.next() * s
            if (prod & 0xFFFFFFFF) >= thresh:
                return prod >> 32


def srht_rows(m, d, seed):
    """The d distinct rows of the Hadamard transform an SRHT keeps (the first
    d of a random permutation of 0..m'-1, m' = 2^ceil(log2 m)): Floyd's
    sampler fed by the "SRHR" word stream, in draw order."""
    mp = 1 << max(0, (m - 1).bit_length())
    if not 1 <= d <= mp:
        raise ValueError("need 1 <= d <= m'")
    st = _ScalarWordStream(seed, SRHT_ROW_DOMAIN)
    picks, taken = [], set()
    for t in range(d):
        top = mp - d + t
        r = st.uniform(top + 1)
        if r in taken:
            r = top
        picks.append(r)
        taken.add(r)
    return np.array(picks, dtype=np.int64), mp


def srht_signs(m, seed):
    """Rademacher diagonal of D: bit 0 of word 0 of the block at counter
    (lo32(j), hi32(j), 0, "SRHD"); set means -1."""
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    j = np.arange(m, dtype=np.uint64)
    w0 = philox4x32_10(j & _MASK32, j >> np.uint64(32), 0, SRHT_SIGN_DOMAIN, k0, k1)[0]
    return np.where((w0 & np.uint32(1)) != 0, -1.0, 1.0)


def srht_sketch_matrix(m, d, seed):
    """S = sqrt(m / d) Pi[:d, :] H D (Sec. 2.3.1, SRHTs) as a dense d x m
    matrix: H the orthonormal Sylvester-Hadamard matrix of order m'
    (entries (-1)^popcount(p & j) / sqrt(m')), D = diag(signs) on the first
    m rows, Pi[:d, :] keeping rows srht_rows(m, d, seed)."""
    p, mp = srht_rows(m, d, seed)
    sg = srht_signs(m, seed)
    j = np.arange(m, dtype=np.int64)
    bits = np.bitwise_and(p[:, None], j[None, :])
    parity = np.zeros(bits.shape, dtype=np.int64)
    x = bits.copy()
    while np.any(x):
        parity ^= x & 1
        x >>= 1
    H = np.where(parity == 1, -1.0, 1.0)
    return H * sg[None, :] * math.sqrt(m / (d * mp))


def cqrrpt_dense(A, d, kind, seed, tol, cond_max=10.0):
    """CQRRPT with a dense sketching operator: kind "gaussian" or "srht"."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= n <= m and n <= d <= m):
        raise ValueError("need 1 <= n <= d <= m")
    S = gaussian_sketch_matrix(m, d, seed) if kind == "gaussian" else srht_sketch_matrix(m, d, seed)
    return cqrrpt_core(A, S, tol, cond_max)


# ---------------------------------------------------------------------------
# S2. The sketch
# ---------------------------------------------------------------------------

def sketch(A, rows, signs, d):
    """Ahat = S A for the SASO given by (rows, signs), in FP64 (Alg. 2, sketch).

    The signed sum sum_j sign * A[j, :] is accumulated first and scaled by
    1/sqrt(nnz) once at the end.
    """
    m, nnz = rows.shape
    cols = np.repeat(np.arange(m), nnz)
    S_pm1 = scipy.sparse.csr_matrix(
        (signs.reshape(-1).astype(np.float64), (rows.reshape(-1), cols)), shape=(d, m))
    return np.asarray(S_pm1 @ np.asarray(A, dtype=np.float64)) * (1.0 / math.sqrt(nnz))


# ---------------------------------------------------------------------------
# S3. QR with column pivoting of the sketch
# ---------------------------------------------------------------------------

def qrcp(X, return_reflectors=False):
    """Householder QR with max-norm (Businger-Golub) column pivoting.

    Returns (J, R): J is the 0-based pivot order (Alg. 2 returns it in full)
    and R is n x n upper triangular with a non-negative diagonal, so that
    X[:, J] = Q R with Q orthonormal (d x n). At step i every remaining
    column's norm ||X[i:, c]|| is recomputed; the largest wins, ties going to
    the smallest original column index.
    """
    X = np.array(X, dtype=np.float64, copy=True)
    d, n = X.shape
    if d < n:
        raise ValueError("qrcp expects at least as many rows as columns")
    J = np.arange(n)
    betas = np.zeros(n)
    refl = []
    for i in range(n):
        nu = np.sqrt(np.sum(X[i:, i:] ** 2, axis=0))
        top = nu.max()
        cand = np.flatnonzero(nu == top)
        p = i + cand[np.argmin(J[i + cand])]
        if p != i:
            X[:, [i, p]] = X[:, [p, i]]
            J[[i, p]] = J[[p, i]]
        x = X[i:, i].copy()
        alpha, normx = x[0], nu[p - i]
        if normx == 0.0:
            tau, beta, v = 0.0, 0.0, np.zeros_like(x)
        else:
            beta = -normx if alpha >= 0.0 else normx
            v = x / (alpha - beta)
            v[0] = 1.0
            tau = (beta - alpha) / beta
            w = v @ X[i:, i + 1:]
            X[i:, i + 1:] -= tau * np.outer(v, w)
        betas[i] = beta
        X[i, i] = beta
        X[i + 1:, i] = 0.0
        refl.append((v, tau))
    R = np.triu(X[:n, :n])
    flip = np.diag(R) < 0.0
    R[flip, :] = -R[flip, :]
    if return_reflectors:
        return J, R, refl, flip
    return J, R


def qrcp_q_factor(refl, flip, d):
    """Explicit d x n Q of ``qrcp`` from its reflectors (for invariant checks)."""
    n = len(refl)
    Q = np.eye(d, n)
    for i in range(n - 1, -1, -1):
        v, tau = refl[i]
        if tau != 0.0:
            Q[i:, :] -= tau * np.outer(v, v @ Q[i:, :])
    Q[:, flip] = -Q[:, flip]
    return Q


def _householder(x):
    """LAPACK-convention reflector of x: (v, tau, beta) with v[0] = 1,
    (I - tau v v^T) x = beta e_1; tau = beta = 0 when ||x|| = 0."""
    normx = math.sqrt(float(np.sum(x * x)))
    if normx == 0.0:
        return np.zeros_like(x), 0.0, 0.0
    alpha = x[0]
    beta = -normx if alpha >= 0.0 else normx
    v = x / (alpha - beta)
    v[0] = 1.0
    return v, (beta - alpha) / beta, beta


def hqrrp(X, b, s, seed, Omega=None):
    """Householder QR with randomized block pivoting (HQRRP) of a d x n
    matrix, as the paper substitutes it for GEQP3 on the sketch (Sec. 5.2.2),
    following the loop of the randomized QRCP methods it outlines in Sec. 1
    (sample Y = Omega X with b + s rows; per block: pivots from Y, QR of the
    chosen columns, update of X and Y) with the sample update
    Y2 <- Y2 - Y1 R11^{-1} R12 of the cited HQRRP work.

    Per block of bb = min(b, n - i) columns starting at position i:
      1. the first bb pivots of max-norm QRCP (exact norms, ties to the
         smallest original column index) of a copy of Y[:, i:]; the chosen
         columns move to positions i.., in pivot order, and the others keep
         their relative order (in X, Y and J);
      2. unpivoted Householder QR of X[i:, i:i+bb], each reflector applied to
         all later columns (LAPACK convention, as ``qrcp``);
      3. Y[:, i+bb:] -= Y[:, i:i+bb] Z with R11 Z = R12, R11 = X[i:i+bb,
         i:i+bb] (upper) and R12 = X[i:i+bb, i+bb:], by back substitution; a
         zero diagonal entry of R11 gives a zero row of Z.
    Omega defaults to the Gaussian (b + s) x d matrix of
    ``gaussian_sketch_matrix`` with the "HQRP" counter domain.
    Returns (J, R) as ``qrcp``: R upper triangular with a non-negative
    diagonal and X[:, J] = Q R."""
    X = np.array(X, dtype=np.float64, copy=True)
    d, n = X.shape
    if d < n:
        raise ValueError("hqrrp expects at least as many rows as columns")
    if b < 1 or s < 0:
        raise ValueError("need b >= 1 and s >= 0")
    if Omega is None:
        Omega = gaussian_sketch_matrix(d, b + s, seed, HQRRP_DOMAIN)
    Y = np.asarray(Omega, dtype=np.float64) @ X
    p = Y.shape[0]
    J = np.arange(n)
    i = 0
    while i < n:
        bb = min(b, n - i)
        # 1. pivots of the block from a reflected copy of Y's remaining columns
        Yc = Y[:, i:].copy()
        alive = list(range(n - i))
        sel = []
        for t in range(bb):
            if t < p:
                nu = np.sqrt(np.sum(Yc[t:, alive] ** 2, axis=0))
            else:
                nu = np.zeros(len(alive))
            top = nu.max()
            cand = [alive[c] for c in np.flatnonzero(nu == top)]
            c = min(cand, key=lambda q: J[i + q])
            sel.append(c)
            alive.remove(c)
            if t < p and alive:
                v, tau, _ = _householder(Yc[t:, c].copy())
                if tau != 0.0:
                    w = v @ Yc[t:, alive]
                    Yc[t:, alive] -= tau * np.outer(v, w)
        perm = np.array(sel + alive, dtype=np.int64)
        X[:, i:] = X[:, i:][:, perm]
        Y[:, i:] = Y[:, i:][:, perm]
        J[i:] = J[i:][perm]
        # 2. unpivoted Householder QR of the chosen columns, applied to the rest
        for j in range(i, i + bb):
            v, tau, beta = _householder(X[j:, j].copy())
            if tau != 0.0 and j + 1 < n:
                w = v @ X[j:, j + 1:]
                X[j:, j + 1:] -= tau * np.outer(v, w)
            X[j, j] = beta
            X[j + 1:, j] = 0.0
        # 3. sample update of the remaining columns
        if i + bb < n:
            R11 = X[i:i + bb, i:i + bb]
            R12 = X[i:i + bb, i + bb:]
            Z = np.zeros_like(R12)
            for r in range(bb - 1, -1, -1):
                if R11[r, r] != 0.0:
                    Z[r] = (R12[r] - R11[r, r + 1:] @ Z[r + 1:]) / R11[r, r]
            Y[:, i + bb:] -= Y[:, i:i + bb] @ Z
        i += bb
    R = np.triu(X[:n, :n])
    flip = np.diag(R) < 0.0
    R[flip, :] = -R[flip, :]
    return J, R


def cqrrpt_hqrrp(A, d, nnz, seed, tol, b, s, hseed, cond_max=10.0):
    """CQRRPT whose QRCP of the sketch is ``hqrrp`` (Sec. 5.2.2)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= n <= m and n <= d <= m):
        raise ValueError("need 1 <= n <= d <= m")
    rows, signs = saso_sample(m, d, nnz, seed)
    Ahat = sketch(A, rows, signs, d)
    return _core_from_sketch(A, Ahat, tol, cond_max,
                             qrcp_fn=lambda X: hqrrp(X, b, s, hseed))


# ---------------------------------------------------------------------------
# S4 / S8. Numerical rank (Sec. 3.3)
# ---------------------------------------------------------------------------

def rank_stage1(R, tol):
    """k_o = min{ l : ||R[l:, l:]||_F <= tol * s }, s = max |R| (first stage).

    Compared in squared form; the trailing block norms are accumulated as
    suffix sums of squared row norms from the last row upward.
    """
    n = R.shape[1]
    Rt = np.triu(R[:n, :n])
    s = np.max(np.abs(Rt)) if Rt.size else 0.0
    if s == 0.0:
        return 0
    rn2 = np.sum(Rt ** 2, axis=1)
    thr = (tol * s) ** 2
    suf = 0.0
    k_o = n
    for l in range(n - 1, -1, -1):
        suf = suf + rn2[l]
        if suf <= thr:
            k_o = l
        else:
            break
    return k_o


def rank_stage2(Rpre, cond_max=10.0):
    """k = max{ l : max|diag R_pre[:l,:l]| / min|diag R_pre[:l,:l]| <= cond_max }.

    cond(diag(.)) is the paper's preferred estimator; it is non-decreasing in
    l, so the scan stops at the first violation.
    """
    dg = np.abs(np.diag(Rpre))
    k = 0
    dmax, dmin = 0.0, math.inf
    for l in range(1, len(dg) + 1):
        dmax = max(dmax, dg[l - 1])
        dmin = min(dmin, dg[l - 1])
        if dmax / dmin <= cond_max:
            k = l
        else:
            break
    return k


# ---------------------------------------------------------------------------
# S7. Cholesky with the failure index
# ---------------------------------------------------------------------------

def cholesky_upper(G):
    """Upper Cholesky R^T R = G, row by row. Returns (R, k): if the pivot of
    0-based row j is <= 0 or not finite, the factor stops there and k = j
    (the leading j x j block is exact: Remark on Cholesky failure, Sec. 3.3).
    """
    n = G.shape[0]
    R = np.zeros((n, n))
    for j in range(n):
        piv = G[j, j] - R[:j, j] @ R[:j, j]
        if not (piv > 0.0) or not math.isfinite(piv):
            return R[:j, :j].copy(), j
        r = math.sqrt(piv)
        R[j, j] = r
        R[j, j + 1:] = (G[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / r
    return R, n


# ---------------------------------------------------------------------------
# The whole path
# ---------------------------------------------------------------------------

STATUS_OK = 0
STATUS_NONFINITE = 1


def cqrrpt_core(A, S, tol, cond_max=10.0):
    """Algorithm 2 with an explicit sketching operator S (dense or sparse d x m).

    Returns dict(Q, R, J, rank, rank_stage1, chol_fail_col, status, Ahat, Rsk).
    Q is m x n and R is n x n, both zero past the rank.
    """
    A = np.asarray(A, dtype=np.float64)
    Ahat = np.asarray(S @ A, dtype=np.float64)
    return _core_from_sketch(A, Ahat, tol, cond_max)


def _core_from_sketch(A, Ahat, tol, cond_max, qrcp_fn=None):
    m, n = A.shape
    out = dict(Q=np.zeros((m, n)), R=np.zeros((n, n)), J=np.arange(n), rank=0,
               rank_stage1=0, chol_fail_col=-1, status=STATUS_OK, Ahat=Ahat, Rsk=None)
    if not np.all(np.isfinite(Ahat)):
        out["status"] = STATUS_NONFINITE
        return out
    J, Rsk = qrcp(Ahat) if qrcp_fn is None else qrcp_fn(Ahat)
    out["J"], out["Rsk"] = J, Rsk
    k_o = rank_stage1(Rsk, tol)
    out["rank_stage1"] = k_o
    if k_o == 0:
        return out
    # S5: M_pre R_sk[:k_o,:k_o] = A[:, J[:k_o]]  (right solve with an upper factor)
    Mpre = scipy.linalg.solve_triangular(Rsk[:k_o, :k_o], A[:, J[:k_o]].T,
                                         trans="T", lower=False).T
    G = Mpre.T @ Mpre                                   # S6
    Rpre, k_chol = cholesky_upper(G)                    # S7
    if k_chol < k_o:
        out["chol_fail_col"] = k_chol
    k = rank_stage2(Rpre, cond_max) if k_chol > 0 else 0   # S8
    out["rank"] = k
    if k == 0:
        return out
    Rp = Rpre[:k, :k]
    Q = scipy.linalg.solve_triangular(Rp, Mpre[:, :k].T, trans="T", lower=False).T  # S9
    out["Q"][:, :k] = Q
    out["R"][:k, :] = Rp @ Rsk[:k, :]                   # S10
    out["Rpre"] = Rp
    out["Mpre"] = Mpre
    return out


def cqrrpt(A, d, nnz, seed, tol, cond_max=10.0):
    """Algorithm 1 with a SASO of ``nnz`` nonzeros per column and d rows."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= n <= m and n <= d <= m):
        raise ValueError("need 1 <= n <= d <= m")
    rows, signs = saso_sample(m, d, nnz, seed)
    Ahat = sketch(A, rows, signs, d)
    return _core_from_sketch(A, Ahat, tol, cond_max)


def factor_given_pivots(A, J, k):
    """The plain definition the path must reach when rank(S A) = rank(A) = k
    (Theorem on correctness, Sec. 2.1): with pivots J fixed, (Q_k, R_k[:, :k])
    is the thin QR of A[:, J[:k]] with a positive diagonal, and
    R_k[:, k:] = Q_k^T A[:, J[k:]]. Computed here through an unpivoted
    Householder QR (a library primitive) for cross-checks.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Ak = A[:, J[:k]]
    Qk, Rk = np.linalg.qr(Ak)
    sgn = np.where(np.diag(Rk) < 0.0, -1.0, 1.0)
    Qk = Qk * sgn
    Rk = Rk * sgn[:, None]
    R = np.zeros((n, n))
    R[:k, :k] = Rk
    R[:k, k:] = Qk.T @ A[:, J[k:]]
    Q = np.zeros((m, n))
    Q[:, :k] = Qk
    return Q, R


# ---------------------------------------------------------------------------
# The unpivoted precursor (Sec. 1.3, "Randomized preconditioning for
# CholeskyQR"): sketch, QR of the sketch, precondition, CholeskyQR.
# ---------------------------------------------------------------------------

def _positive_diag_r(X):
    """Upper-triangular factor of an unpivoted QR of X (d x n, d >= n) with
    a non-negative diagonal: LAPACK's Householder QR (numpy, a library
    primitive) with the rows of negative diagonal negated, which makes it the
    unique R of a full-rank X."""
    R = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="r")
    n = X.shape[1]
    R = np.triu(R[:n, :n])
    flip = np.diag(R) < 0.0
    R[flip, :] = -R[flip, :]
    return R


def sketched_cholqr_core(A, S):
    """The five steps of Sec. 1.3 with an explicit sketching operator S:
    M_sk = S M; [Q_sk, R_sk] = qr(M_sk); M_pre = M R_sk^{-1};
    G = M_pre^T M_pre, R_pre = chol(G); Q = M_pre R_pre^{-1}, R = R_pre R_sk.
    M must have full rank. A Cholesky failure at 0-based column j truncates
    the result to j columns (Q and R zero past them; rank = j); an exactly
    zero trailing block of R_sk (first-stage bound with tolerance 0) is
    dropped before the solve.
    Returns dict(Q, R, rank, rank_stage1, chol_fail_col, Rsk, Rpre, status)."""
    A = np.asarray(A, dtype=np.float64)
    return _sketched_cholqr_from_sketch(A, np.asarray(S @ A, dtype=np.float64))


def _sketched_cholqr_from_sketch(A, Ahat):
    m, n = A.shape
    out = dict(Q=np.zeros((m, n)), R=np.zeros((n, n)), rank=0, rank_stage1=0,
               chol_fail_col=-1, status=STATUS_OK, Rsk=None, Rpre=None)
    if not np.all(np.isfinite(Ahat)):
        out["status"] = STATUS_NONFINITE
        return out
    Rsk = _positive_diag_r(Ahat)
    out["Rsk"] = Rsk
    k_o = rank_stage1(Rsk, 0.0)
    out["rank_stage1"] = k_o
    if k_o == 0:
        return out
    Mpre = scipy.linalg.solve_triangular(Rsk[:k_o, :k_o], A[:, :k_o].T,
                                         trans="T", lower=False).T
    G = Mpre.T @ Mpre
    Rpre, k = cholesky_upper(G)
    if k < k_o:
        out["chol_fail_col"] = k
    out["rank"] = k
    if k == 0:
        return out
    Rp = Rpre[:k, :k]
    out["Q"][:, :k] = scipy.linalg.solve_triangular(Rp, Mpre[:, :k].T, trans="T",
                                                    lower=False).T
    out["R"][:k, :] = Rp @ Rsk[:k, :]
    out["Rpre"] = Rp
    return out


def sketched_cholqr(A, d, nnz, seed):
    """The precursor with the SASO of ``cqrrpt`` (same rows and signs)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= n <= m and n <= d <= m):
        raise ValueError("need 1 <= n <= d <= m")
    rows, signs = saso_sample(m, d, nnz, seed)
    return _sketched_cholqr_from_sketch(A, sketch(A, rows, signs, d))
