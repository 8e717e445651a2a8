"""Seeded synthetic workloads for the five benchmark configurations.

Everything here is input preparation.  The paper treats the structured
approximations and their error bounds as given ("precomputed", Section III-B;
the SuKro approximations of Section V-A are learned elsewhere), so the
nearest-Kronecker-product truncations, the BF16 / FP8 copies and the exact
per-atom bounds eps_j = ||a_j - a~_j||_2 are produced here and handed to both
the oracle and the GPU path.

Conventions
-----------
* A dictionary is an (N, K) float64 matrix of exact values.  For FP32
  configurations the exact dictionary *is* the FP32-rounded matrix, so an FP32
  copy of it carries no approximation error.
* Kronecker layout: atom j = j1*k2 + j2, row i = i1*n2 + i2 and
  (B kron C)[i, j] = B[i1, j1] * C[i2, j2] (numpy.kron order).
* Dense storage arrays are atom-major: ``data[j]`` is atom j (column-major
  N x K with leading dimension N).  Kronecker factors are stored as
  ``B[r, j1, i1]`` (each term column-major n1 x k1) and ``C[r, j2, i2]``.
* BF16 and FP8 storage arrays hold raw bit patterns (uint16 / uint8).
* FAuST stages (products of sparse factors A~ = S_1 S_2 ... S_J, the model cited
  in Section I-D and used for the paper's MEG operator in Section V-G) keep each
  factor in CSR form: (row_ptr int32, col_idx int32, values) with S_l of shape
  (dims[l-1], dims[l]), dims[0] = N and dims[J] = K.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 181206635          # arXiv identifier 1812.06635

_FP8_MAX = 448.0


def rng_for(config_id: int, realization: int, purpose: int) -> np.random.Generator:
    """Independent, reproducible stream per (configuration, realization, purpose)."""
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE, config_id, realization, purpose]))


# ----------------------------------------------------------------------------
# Low-precision encodings (round to nearest, ties to even)
# ----------------------------------------------------------------------------

def bf16_round(v: np.ndarray) -> np.ndarray:
    """Round float32-representable values to bfloat16; returns uint16 bit patterns."""
    f = np.ascontiguousarray(v, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((bits >> 16) & 1)
    out = ((bits + bias) >> 16).astype(np.uint16)
    return out


def bf16_decode(bits: np.ndarray) -> np.ndarray:
    """Exact float64 values of bfloat16 bit patterns."""
    b = (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16)
    return b.view(np.float32).astype(np.float64)


def _fp8_table() -> np.ndarray:
    """Values of the 256 OCP FP8 E4M3FN codes (NaN for 0x7F / 0xFF)."""
    vals = np.empty(256, dtype=np.float64)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = s * m * 2.0 ** -9
        else:
            vals[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return vals


_FP8_VALUES = _fp8_table()
_FP8_POS_CODES = np.arange(0, 0x7F)              # 0 .. 126 (non-negative finite)
_FP8_POS_VALUES = _FP8_VALUES[_FP8_POS_CODES]    # strictly increasing


def fp8_e4m3_decode(codes: np.ndarray) -> np.ndarray:
    return _FP8_VALUES[np.asarray(codes, dtype=np.uint8)]


def fp8_e4m3_round(v: np.ndarray) -> np.ndarray:
    """Round to OCP FP8 E4M3FN (saturating at +-448); returns uint8 codes."""
    v = np.asarray(v, dtype=np.float64)
    a = np.minimum(np.abs(v), _FP8_MAX)
    hi = np.searchsorted(_FP8_POS_VALUES, a, side="left")
    hi = np.clip(hi, 0, len(_FP8_POS_VALUES) - 1)
    lo = np.clip(hi - 1, 0, len(_FP8_POS_VALUES) - 1)
    dlo = a - _FP8_POS_VALUES[lo]
    dhi = _FP8_POS_VALUES[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (_FP8_POS_CODES[hi] % 2 == 0))
    code = np.where(pick_hi, _FP8_POS_CODES[hi], _FP8_POS_CODES[lo]).astype(np.uint8)
    code = code | np.where((v < 0) & (code != 0), 0x80, 0).astype(np.uint8)
    return code


# ----------------------------------------------------------------------------
# Data containers
# ----------------------------------------------------------------------------

@dataclass
class Stage:
    """One dictionary of the sequence A~^0 .. A~^I (the last one is exact)."""
    kind: str                  # "dense" | "kron" | "faust"
    dtype: str                 # storage: "f64" | "f32" | "bf16" | "fp8"
    N: int
    K: int
    data: np.ndarray | None = None     # dense: (K, N) storage array
    scale: np.ndarray | None = None    # dense low precision: (K,) float32 power-of-two scales
    B: np.ndarray | None = None        # kron: (R, k1, n1) storage array
    C: np.ndarray | None = None        # kron: (R, k2, n2) storage array
    dims: tuple | None = None          # kron: (n1, k1, n2, k2); faust: (d_0 = N, d_1, ..., d_J = K)
    factors: list | None = None        # faust: [(row_ptr, col_idx, values)] per factor, CSR
    eps: np.ndarray | None = None      # (K,) exact bound on ||a_j - a~_j||_q
    q: float = 2.0                     # norm of the bounds eps, 1 <= q <= inf
    L: float = 0.0                     # ||A~||_2^2 (FP64)
    rc_theory: float = 1.0             # relative complexity model of the products
    label: str = ""

    @property
    def R(self) -> int:
        return 0 if self.B is None else int(self.B.shape[0])

    def factor_values(self):
        """(B, C) as float64 arrays of shape (R, n1, k1), (R, n2, k2)."""
        dec = _decoder(self.dtype)
        return (dec(self.B).transpose(0, 2, 1), dec(self.C).transpose(0, 2, 1))

    def factor_matrices(self):
        """FAuST factors as dense float64 arrays S_1 .. S_J."""
        out = []
        dec = _decoder(self.dtype)
        for l, (rp, ci, v) in enumerate(self.factors):
            M = np.zeros((self.dims[l], self.dims[l + 1]))
            rows = np.repeat(np.arange(self.dims[l]), np.diff(rp))
            M[rows, ci] = dec(v)
            out.append(M)
        return out

    def values(self) -> np.ndarray:
        """Exact float64 values of the stored dictionary, shape (N, K)."""
        if self.kind == "faust":
            out = None
            for M in self.factor_matrices():
                out = M if out is None else out @ M
            return out
        if self.kind == "dense":
            v = _decoder(self.dtype)(self.data)
            if self.scale is not None:
                v = v * self.scale.astype(np.float64)[:, None]
            return np.ascontiguousarray(v.T)
        B, C = self.factor_values()
        return _kron_sum(B, C)


@dataclass
class Problem:
    name: str
    A: np.ndarray              # (N, K) float64 values of the exact dictionary
    stages: list               # list[Stage]; stages[-1] is the exact dictionary
    Y: np.ndarray              # (batch, N) float64, representable in the working precision
    lam: np.ndarray            # (batch,)
    X0: np.ndarray             # (batch, K) generating sparse codes
    work: str                  # "f64" | "f32"
    atom_norm: np.ndarray      # (K,) ||a_j||_2 of the exact atoms
    lam_max: np.ndarray        # (batch,) ||A^T y||_inf
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.A.shape[0]

    @property
    def K(self):
        return self.A.shape[1]

    @property
    def batch(self):
        return self.Y.shape[0]


def _decoder(dtype):
    if dtype in ("f64", "f32"):
        return lambda a: np.asarray(a, dtype=np.float64)
    if dtype == "bf16":
        return bf16_decode
    if dtype == "fp8":
        return fp8_e4m3_decode
    raise ValueError(dtype)


def _encode(values: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f64":
        return np.ascontiguousarray(values, dtype=np.float64)
    if dtype == "f32":
        return np.ascontiguousarray(values, dtype=np.float32)
    if dtype == "bf16":
        return bf16_round(values.astype(np.float32))
    if dtype == "fp8":
        return fp8_e4m3_round(values)
    raise ValueError(dtype)


def _kron_sum(B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """sum_r kron(B[r], C[r]) for B (R, n1, k1), C (R, n2, k2) -> (n1*n2, k1*k2)."""
    R, n1, k1 = B.shape
    _, n2, k2 = C.shape
    T = np.einsum("rac,rbd->abcd", B, C, optimize=True)   # (n1, n2, k1, k2)
    return T.reshape(n1 * n2, k1 * k2)


def _round_work(M: np.ndarray, work: str) -> np.ndarray:
    return M.astype(np.float32).astype(np.float64) if work == "f32" else M


def _bound(diff_norm: np.ndarray, a_norm: np.ndarray, at_norm: np.ndarray) -> np.ndarray:
    """Exact FP64 column-difference norm, widened by a few FP64 ulps of the operands."""
    return diff_norm + 1e-13 * (a_norm + at_norm)


def _col_norm(M: np.ndarray, q: float) -> np.ndarray:
    return np.linalg.norm(M, ord=q, axis=0) if np.isinf(q) or q in (1.0, 2.0) else \
        np.sum(np.abs(M) ** q, axis=0) ** (1.0 / q)


def with_lq_bounds(problem, q, stages=None):
    """A copy of `problem` whose approximate stages carry l_q error bounds
    eps_j = ||a_j - a~_j||_q (widened like the l2 ones) instead of l2 bounds: the
    zone B_q(a~_j, eps_j) of Lemma 1 (Section III-B).  `stages` selects the stage
    indices that switch (default: every stage but the exact one; selected, the exact
    one takes the norm q and keeps eps = 0); q may be a number or np.inf."""
    import copy
    q = float(q)
    out = copy.copy(problem)
    out.stages = [copy.copy(st) for st in problem.stages]
    last = len(out.stages) - 1
    sel = range(last) if stages is None else stages
    A = problem.A
    for i in sel:
        st = out.stages[i]
        st.q = q
        if i == last:                  # the exact dictionary: no error, eps = 0 in any norm
            continue
        At = st.values()
        st.eps = _bound(_col_norm(A - At, q), _col_norm(A, q), _col_norm(At, q))
    return out


# ----------------------------------------------------------------------------
# Dictionaries and approximations
# ----------------------------------------------------------------------------

def kron_dictionary(rng, n1, k1, n2, k2, R_A, noise, work):
    """A = sum_{r<=R_A} B_r kron C_r + noise*G with unit-norm columns."""
    Bt = rng.standard_normal((R_A, n1, k1))
    Ct = rng.standard_normal((R_A, n2, k2))
    G = rng.standard_normal((n1 * n2, k1 * k2))
    A = _kron_sum(Bt, Ct) + noise * G
    A /= np.linalg.norm(A, axis=0, keepdims=True)
    return _round_work(A, work)


def _rearrange(A, n1, k1, n2, k2):
    """Van Loan-Pitsianis rearrangement: rows (i1, j1), columns (i2, j2)."""
    return A.reshape(n1, n2, k1, k2).transpose(0, 2, 1, 3).reshape(n1 * k1, n2 * k2)


def nkp_factors(A, n1, k1, n2, k2, R, seed=0):
    """Truncated nearest-Kronecker-product SVD: best R-term sum_r B_r kron C_r in
    Frobenius norm (Eckart-Young on the rearranged matrix).  Returns float64
    (B, C, sigma) with B (R, n1, k1), C (R, n2, k2)."""
    M = _rearrange(A, n1, k1, n2, k2)
    m, n = M.shape
    if min(m, n) <= 1024:
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
    else:
        # Seeded subspace iteration for the leading singular triplets.
        p = R + 12
        rs = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 99, seed]))
        Q = np.linalg.qr(M @ rs.standard_normal((n, p)))[0]
        for _ in range(6):
            Q = np.linalg.qr(M.T @ Q)[0]
            Q = np.linalg.qr(M @ Q)[0]
        Ub, s, Vt = np.linalg.svd(Q.T @ M, full_matrices=False)
        U = Q @ Ub
    U, s, Vt = U[:, :R], s[:R], Vt[:R]
    # deterministic sign: largest-magnitude entry of each left vector positive
    sg = np.sign(U[np.argmax(np.abs(U), axis=0), np.arange(R)])
    sg[sg == 0] = 1.0
    U = U * sg
    Vt = Vt * sg[:, None]
    rt = np.sqrt(s)
    B = (U * rt).T.reshape(R, n1, k1)
    C = (Vt.T * rt).T.reshape(R, n2, k2)
    return B, C, s


def _spectral_norm_sq(matvec, rmatvec, shape, seed):
    n_rows, n_cols = shape
    if n_rows * n_cols <= 1024 * 4096:
        return None
    from scipy.sparse.linalg import LinearOperator, svds
    op = LinearOperator(shape, matvec=matvec, rmatvec=rmatvec, dtype=np.float64)
    v0 = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 98, seed])).standard_normal(min(shape))
    s = svds(op, k=1, tol=1e-13, v0=v0, return_singular_vectors=False, solver="arpack")
    return float(s[0]) ** 2


def lipschitz_dense(M, seed=0):
    """||M||_2^2 in FP64 (Lipschitz constant of the least-squares gradient)."""
    N, K = M.shape
    if N * K <= 1024 * 4096:
        small = M @ M.T if N <= K else M.T @ M
        return float(np.linalg.eigvalsh(small)[-1]) * (1 + 1e-12)
    L = _spectral_norm_sq(lambda v: M @ v, lambda v: M.T @ v, M.shape, seed)
    return L * (1 + 1e-10)


def lipschitz_kron(B, C, seed=0):
    R, n1, k1 = B.shape
    _, n2, k2 = C.shape
    N, K = n1 * n2, k1 * k2
    if N * K <= 1024 * 4096:
        return lipschitz_dense(_kron_sum(B, C))

    def mv(v):
        X = v.reshape(k1, k2).T                      # X[j2, j1]
        U = sum(C[r] @ X @ B[r].T for r in range(R))  # (n2, n1)
        return U.T.reshape(-1)

    def rmv(w):
        P = w.reshape(n1, n2).T                      # P[i2, i1]
        G = sum(C[r].T @ P @ B[r] for r in range(R))  # (k2, k1)
        return G.T.reshape(-1)

    return _spectral_norm_sq(mv, rmv, (N, K), seed) * (1 + 1e-10)


def exact_stage(A: np.ndarray, work: str, seed=0) -> Stage:
    N, K = A.shape
    return Stage(kind="dense", dtype=work, N=N, K=K, data=_encode(A.T, work),
                 eps=np.zeros(K), L=lipschitz_dense(A, seed), rc_theory=1.0, label=f"A ({work})")


def kron_rc(R, n1, k2):
    """Relative complexity model of an R-term Kronecker product with n1 x k1 and
    n2 x k2 factors: R (1/n1 + 1/k2), i.e. R (1/sqrt(N) + 1/sqrt(K)) for square
    factor grids (Section V-A, Table IV)."""
    return R * (1.0 / n1 + 1.0 / k2)


def kron_stage(A, B, C, dtype, seed=0) -> Stage:
    """Stage holding the R-term Kronecker approximation with factors rounded to
    ``dtype`` and the exact per-atom error bound against A."""
    R, n1, k1 = B.shape
    _, n2, k2 = C.shape
    if dtype == "fp8":
        # balance each term's two factors by a power of two (B_r 2^e, C_r 2^-e leave the
        # product unchanged) so that both sit in the same part of the FP8 range
        e = np.round(0.5 * np.log2(np.max(np.abs(C), axis=(1, 2)) / np.max(np.abs(B), axis=(1, 2))))
        B = B * np.exp2(e)[:, None, None]
        C = C * np.exp2(-e)[:, None, None]
    Bs = _encode(B.transpose(0, 2, 1), dtype)      # (R, k1, n1)
    Cs = _encode(C.transpose(0, 2, 1), dtype)      # (R, k2, n2)
    st = Stage(kind="kron", dtype=dtype, N=n1 * n2, K=k1 * k2, B=Bs, C=Cs, dims=(n1, k1, n2, k2),
               rc_theory=kron_rc(R, n1, k2), label=f"kron R={R} ({dtype})")
    Bv, Cv = st.factor_values()
    At = _kron_sum(Bv, Cv)
    st.eps = _bound(np.linalg.norm(A - At, axis=0), np.linalg.norm(A, axis=0), np.linalg.norm(At, axis=0))
    st.L = lipschitz_kron(Bv, Cv, seed)
    return st


def quantized_stage(A, dtype, seed=0) -> Stage:
    """Per-column power-of-two scaled BF16 / FP8 copy of A with exact error bounds."""
    N, K = A.shape
    amax = np.max(np.abs(A), axis=0)
    qmax = _FP8_MAX if dtype == "fp8" else 1.0
    e = np.ceil(np.log2(np.maximum(amax, 1e-300) / qmax))
    scale = np.exp2(e).astype(np.float32)
    Q = _encode((A / scale.astype(np.float64)[None, :]).T, dtype)     # (K, N)
    st = Stage(kind="dense", dtype=dtype, N=N, K=K, data=Q, scale=scale,
               rc_theory={"fp8": 0.25, "bf16": 0.5}[dtype], label=f"A ({dtype}, column-scaled)")
    At = st.values()
    st.eps = _bound(np.linalg.norm(A - At, axis=0), np.linalg.norm(A, axis=0), np.linalg.norm(At, axis=0))
    st.L = lipschitz_dense(At, seed)
    return st


def _csr(M: np.ndarray, dtype: str):
    """CSR (row_ptr, col_idx, values) of a dense matrix, values encoded in dtype."""
    rows, cols = np.nonzero(M)
    rp = np.zeros(M.shape[0] + 1, dtype=np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return rp, cols.astype(np.int32), _encode(M[rows, cols], dtype)


def faust_chain(rng, dims, col_nnz):
    """Sparse factors S_l of shape (dims[l-1], dims[l]) with col_nnz[l-1] nonzeros
    per column at distinct uniform rows, N(0,1) values."""
    out = []
    for l in range(1, len(dims)):
        r, c = dims[l - 1], dims[l]
        M = np.zeros((r, c))
        for j in range(c):
            idx = rng.choice(r, size=col_nnz[l - 1], replace=False)
            M[idx, j] = rng.standard_normal(col_nnz[l - 1])
        out.append(M)
    return out


def faust_dictionary(rng, dims, col_nnz, noise, work):
    """A = (S_1 ... S_J + noise G) D with unit-norm columns (D diagonal); returns A
    and the factors with the column scaling folded into the last one."""
    S = faust_chain(rng, dims, col_nnz)
    F = S[0]
    for M in S[1:]:
        F = F @ M
    F = F + noise * rng.standard_normal(F.shape)
    d = 1.0 / np.linalg.norm(F, axis=0)
    S[-1] = S[-1] * d[None, :]
    return _round_work(F * d[None, :], work), S


def faust_stage(A, S, keep, dtype, seed=0) -> Stage:
    """FAuST approximation S_1 ... S_{J-1} S_J' where S_J' keeps the `keep` entries
    of largest magnitude of each column of S_J; factors rounded to dtype; exact
    per-atom bounds against A.  The relative-complexity model is the nonzero count
    of the factors over N K (the cost of the chain of sparse products against a
    dense product)."""
    S = [np.array(M) for M in S]
    last = S[-1]
    order = np.argsort(-np.abs(last), axis=0, kind="stable")
    pruned = np.zeros_like(last)
    cols = np.arange(last.shape[1])
    for q in range(min(keep, last.shape[0])):
        pruned[order[q], cols] = last[order[q], cols]
    S[-1] = pruned
    dims = tuple([S[0].shape[0]] + [M.shape[1] for M in S])
    N, K = dims[0], dims[-1]
    st = Stage(kind="faust", dtype=dtype, N=N, K=K, dims=dims, factors=[_csr(M, dtype) for M in S],
               label=f"faust keep={keep} ({dtype})")
    nnz = sum(len(f[1]) for f in st.factors)
    st.rc_theory = nnz / float(N * K)
    At = st.values()
    st.eps = _bound(np.linalg.norm(A - At, axis=0), np.linalg.norm(A, axis=0), np.linalg.norm(At, axis=0))
    st.L = lipschitz_dense(At, seed)
    return st


# ----------------------------------------------------------------------------
# Signals
# ----------------------------------------------------------------------------

def signals(rng, A, sparsity, sigma, lam_frac, work, normalize=False):
    """y_b = A x0_b + sigma_b * n_b, x0_b with s_b nonzeros at distinct uniform
    positions and N(0,1) values; lambda_b = lam_frac_b * ||A^T y_b||_inf."""
    N, K = A.shape
    sparsity = np.atleast_1d(sparsity)
    batch = len(sparsity)
    sigma = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (batch,))
    lam_frac = np.broadcast_to(np.asarray(lam_frac, dtype=np.float64), (batch,))
    X0 = np.zeros((batch, K))
    Y = np.zeros((batch, N))
    for b in range(batch):
        idx = rng.choice(K, size=int(sparsity[b]), replace=False)
        X0[b, idx] = rng.standard_normal(len(idx))
        y = A @ X0[b] + sigma[b] * rng.standard_normal(N)
        if normalize:
            y = y / np.linalg.norm(y)
        Y[b] = y
    Y = _round_work(Y, work)
    lam_max = np.max(np.abs(Y @ A), axis=1)
    return Y, lam_frac * lam_max, X0, lam_max


# ----------------------------------------------------------------------------
# The five configurations
# ----------------------------------------------------------------------------

def _kron_problem(name, cid, realization, n1, k1, n2, k2, R_A, Rs, factor_dtype, work, seed_sig_stream,
                  sparsity, sigma, lam_frac, noise=0.01):
    A = _kron_dict_cached(cid, realization, n1, k1, n2, k2, R_A, noise, work)
    stages = list(_kron_stages_cached(cid, realization, n1, k1, n2, k2, R_A, noise, work, tuple(Rs), factor_dtype))
    rng = rng_for(cid, realization, seed_sig_stream)
    if callable(sparsity):
        sparsity, sigma, lam_frac = sparsity(rng)
    Y, lam, X0, lmax = signals(rng, A, sparsity, sigma, lam_frac, work)
    return Problem(name=name, A=A, stages=stages, Y=Y, lam=lam, X0=X0, work=work,
                   atom_norm=np.linalg.norm(A, axis=0), lam_max=lmax,
                   meta=dict(n1=n1, k1=k1, n2=n2, k2=k2, R_A=R_A, Rs=tuple(Rs), factor_dtype=factor_dtype))


@functools.lru_cache(maxsize=4)
def _kron_dict_cached(cid, realization, n1, k1, n2, k2, R_A, noise, work):
    A = kron_dictionary(rng_for(cid, realization, 0), n1, k1, n2, k2, R_A, noise, work)
    A.setflags(write=False)
    return A


@functools.lru_cache(maxsize=4)
def _kron_stages_cached(cid, realization, n1, k1, n2, k2, R_A, noise, work, Rs, factor_dtype):
    A = _kron_dict_cached(cid, realization, n1, k1, n2, k2, R_A, noise, work)
    B, C, _ = nkp_factors(A, n1, k1, n2, k2, max(Rs), seed=cid)
    out = [kron_stage(A, B[:R], C[:R], factor_dtype, seed=cid) for R in Rs]
    out.append(exact_stage(A, work, seed=cid))
    return tuple(out)


def config1(realization=0, lam_frac=0.5, n=(16, 32), R_A=4, Rs=(1, 2, 4), s=10, sigma=0.01):
    """Plain method, FP64, one signal: N=256 (16x16), K=1024 (32x32), R_A=4,
    approximations R in {1, 2, 4} from the truncated NKP-SVD, lambda = 0.5 lambda_max."""
    nn, kk = n
    return _kron_problem("C1", 1, realization, nn, kk, nn, kk, R_A, Rs, "f64", "f64", 1,
                         [s], sigma, lam_frac)


def config2(lam_frac=0.5, realization=0, n=(64, 128), R_A=8, Rs=(1, 2, 4, 8), s=40, sigma=0.01,
            batch=1, factor_dtype="f32"):
    """Plain method on GPU, FP32 with FP64 gap and test: N=4096 (64x64),
    K=16384 (128x128), R_A=8, approximations R in {1, 2, 4, 8}, 40-sparse x0."""
    nn, kk = n
    return _kron_problem("C2", 2, realization, nn, kk, nn, kk, R_A, Rs, factor_dtype, "f32", 1 + 10 * batch,
                         [s] * batch, sigma, lam_frac)


@functools.lru_cache(maxsize=2)
def _dense_cached(cid, realization, N, K):
    rng = rng_for(cid, realization, 0)
    A = rng.standard_normal((N, K))
    A /= np.linalg.norm(A, axis=0, keepdims=True)
    A = _round_work(A, "f32")
    A.setflags(write=False)
    stages = (quantized_stage(A, "fp8", cid), quantized_stage(A, "bf16", cid), exact_stage(A, "f32", cid))
    return A, stages


def config3(realization=0, N=2500, K=10000, s=50, lam_frac=0.5, batch=1):
    """Precision: dense i.i.d. Gaussian A (unit columns, FP32), stages FP8-E4M3 and
    BF16 column-scaled copies then A; y = A x0 normalised, noise free."""
    A, stages = _dense_cached(3, realization, N, K)
    rng = rng_for(3, realization, 1 + 10 * batch)
    Y, lam, X0, lmax = signals(rng, A, [s] * batch, 0.0, lam_frac, "f32", normalize=True)
    return Problem(name="C3", A=A, stages=list(stages), Y=Y, lam=lam, X0=X0, work="f32",
                   atom_norm=np.linalg.norm(A, axis=0), lam_max=lmax, meta=dict(N=N, K=K))


def config4(batch=512, realization=0, n=(32, 64), R_A=4, Rs=(1, 2, 4), factor_dtype="bf16",
            s_range=(5, 80), lam_range=(0.2, 0.9), sigma_range=(0.001, 0.05)):
    """Batching: one shared Kronecker dictionary N=1024 (32x32), K=4096 (64x64),
    R_A=4, BF16 factors; per-signal sparsity, lambda/lambda_max and noise drawn
    uniformly from the given ranges."""
    nn, kk = n

    def draw(rng):
        sp = rng.integers(s_range[0], s_range[1] + 1, size=batch)
        lf = rng.uniform(lam_range[0], lam_range[1], size=batch)
        sg = rng.uniform(sigma_range[0], sigma_range[1], size=batch)
        return sp, sg, lf

    return _kron_problem("C4", 4, realization, nn, kk, nn, kk, R_A, Rs, factor_dtype, "f32", 1, draw, None, None)


def config5(batch=64, realization=0, n=(64, 128), R_A=8, Rs=(1, 2, 4, 8), s=40, sigma=0.01, lam_frac=0.5):
    """Differentiation: the C2 dictionary with a batch of 40-sparse signals,
    lambda_b = 0.5 lambda_max,b; the loss target x_t is the generating x0."""
    nn, kk = n
    p = _kron_problem("C5", 2, realization, nn, kk, nn, kk, R_A, Rs, "f32", "f32", 5,
                      [s] * batch, sigma, lam_frac)
    p.name = "C5"
    return p


def kron_near_exact(realization=0, n=(16, 32), noise=1e-3, s=10, sigma=0.01, lam_frac=0.5):
    """A dictionary that is one Kronecker product up to small noise: B (n x k) and
    C (n x k) with N(0,1) entries and unit columns (so B kron C has unit columns),
    A = B kron C + noise G / sqrt(N), unit columns, FP64; stages [B kron C (FP64), A].
    Its structured stage is accurate enough (eps ~ noise) for the stable test to
    screen most atoms while the method stays on it."""
    nn, kk = n
    rng = rng_for(7, realization, 0)
    B = rng.standard_normal((1, nn, kk))
    C = rng.standard_normal((1, nn, kk))
    B /= np.linalg.norm(B, axis=1, keepdims=True)
    C /= np.linalg.norm(C, axis=1, keepdims=True)
    G = rng.standard_normal((nn * nn, kk * kk))
    A = _kron_sum(B, C) + noise * G / nn
    A /= np.linalg.norm(A, axis=0, keepdims=True)
    stages = [kron_stage(A, B, C, "f64", seed=7), exact_stage(A, "f64", seed=7)]
    Y, lam, X0, lmax = signals(rng_for(7, realization, 1), A, [s], sigma, lam_frac, "f64")
    return Problem(name="KN", A=A, stages=stages, Y=Y, lam=lam, X0=X0, work="f64",
                   atom_norm=np.linalg.norm(A, axis=0), lam_max=lmax, meta=dict(n=n, noise=noise))


@functools.lru_cache(maxsize=2)
def _faust_cached(cid, realization, dims, col_nnz, keeps, noise, dtype, work):
    A, S = faust_dictionary(rng_for(cid, realization, 0), dims, col_nnz, noise, work)
    A.setflags(write=False)
    stages = tuple([faust_stage(A, S, k, dtype, seed=cid) for k in keeps] + [exact_stage(A, work, cid)])
    return A, stages


def config6(batch=1, realization=0, N=204, K=8193, depth=4, col_nnz=(32, 32, 32, 64), keeps=(40, 48, 52, 56),
            s=8, lam_frac=0.1, noise=0.01, dtype="f32", work="f32"):
    """FAuST approximations (Section V-G and Table V, MEG shape): A of size 204 x 8193 is a
    product of `depth` sparse factors (N x N, ..., N x K; col_nnz nonzeros per
    column) plus noise, unit columns, FP32; the approximations keep the `keeps`
    largest entries of each column of the last factor (four levels, like the
    paper's four FAuST approximations); 8-sparse x0 with N(0, 1) weights at
    uniform positions, lambda = 0.1 lambda_max.  The MEG gain matrix itself is not
    available: this is a synthetic operator of the same shape.  work="f64" gives
    an FP64 exact stage and signals (with dtype="f64" factors)."""
    dims = tuple([N] * depth + [K])
    A, stages = _faust_cached(6, realization, dims, tuple(col_nnz), tuple(keeps), noise, dtype, work)
    rng = rng_for(6, realization, 1 + 10 * batch)
    Y, lam, X0, lmax = signals(rng, A, [s] * batch, 0.0, lam_frac, work)
    return Problem(name="C6", A=A, stages=list(stages), Y=Y, lam=lam, X0=X0, work=work,
                   atom_norm=np.linalg.norm(A, axis=0), lam_max=lmax,
                   meta=dict(dims=dims, col_nnz=tuple(col_nnz), keeps=tuple(keeps)))
