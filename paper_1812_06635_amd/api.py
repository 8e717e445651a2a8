"""Python binding of the stablel1 C ABI.

Argument marshalling only: tensors are passed by device pointer with the
current torch stream; every step of the solver runs in the HIP library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L

DTYPES = {"f64": L.F64, "f32": L.F32, "bf16": L.BF16, "fp8": L.FP8_E4M3}
_STORAGE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.int16, "fp8": torch.uint8}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _dev(t, dtype=None, what="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t


class Dict:
    """One dictionary stage (handle owned by the library).  A dense stage
    borrows its matrix: the tensor is kept referenced by this object."""

    def __init__(self, handle, keep, N, K, kind, dtype):
        self._h = handle
        self._keep = keep
        self.N, self.K, self.kind, self.dtype = N, K, kind, dtype

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("dictionary handle already freed")
        return self._h

    @classmethod
    def dense(cls, A, eps, dtype, scale=None, q=2.0):
        """A: (K, N) device tensor, atom-major (= column-major N x K), storage
        dtype float64 / float32 / int16 (bf16 bits) / uint8 (fp8 E4M3 codes);
        eps bounds ||a_j - a~_j||_q (q in [1, inf], 2 by default)."""
        _dev(A, _STORAGE[dtype], "A")
        _dev(eps, torch.float64, "eps")
        if scale is not None:
            _dev(scale, torch.float32, "scale")
        K, N = A.shape
        h = L.c_dict()
        L.check(L.load().sl1_dict_dense(ctypes.byref(h), DTYPES[dtype], N, K, _ptr(A), _ptr(scale), _ptr(eps),
                                        float(q), _stream()), "sl1_dict_dense")
        return cls(h, (A, scale), N, K, "dense", dtype)

    @classmethod
    def kron(cls, B, C, eps, dtype, q=2.0):
        """B: (R, k1, n1), C: (R, k2, n2) device tensors (each term column-major);
        eps and q as for dense."""
        _dev(B, _STORAGE[dtype], "B")
        _dev(C, _STORAGE[dtype], "C")
        _dev(eps, torch.float64, "eps")
        R, k1, n1 = B.shape
        R2, k2, n2 = C.shape
        if R2 != R:
            raise ValueError("B and C must have the same number of terms")
        h = L.c_dict()
        L.check(L.load().sl1_dict_kron(ctypes.byref(h), DTYPES[dtype], R, n1, k1, n2, k2, _ptr(B), _ptr(C),
                                       _ptr(eps), float(q), _stream()), "sl1_dict_kron")
        return cls(h, None, n1 * n2, k1 * k2, "kron", dtype)

    @classmethod
    def faust(cls, dims, factors, eps, dtype, q=2.0):
        """A~ = S_1 ... S_J from host CSR factors [(row_ptr int32, col_idx int32,
        values float64/float32)], S_l of dims[l-1] x dims[l]; eps (K,) device FP64
        and q as for dense."""
        if dtype not in ("f64", "f32"):
            raise ValueError("FAuST factors are f64 or f32")
        _dev(eps, torch.float64, "eps")
        J = len(factors)
        if len(dims) != J + 1:
            raise ValueError("dims must hold J + 1 sizes")
        vt = np.float64 if dtype == "f64" else np.float32
        rp = np.ascontiguousarray(np.concatenate([np.asarray(f[0], dtype=np.int32) for f in factors]))
        ci = np.ascontiguousarray(np.concatenate([np.asarray(f[1], dtype=np.int32) for f in factors]))
        va = np.ascontiguousarray(np.concatenate([np.asarray(f[2], dtype=vt) for f in factors]))
        dd = (L.c_i64 * (J + 1))(*[int(v) for v in dims])
        nz = (L.c_i64 * J)(*[len(f[1]) for f in factors])
        h = L.c_dict()
        L.check(L.load().sl1_dict_faust(ctypes.byref(h), DTYPES[dtype], J, dd, nz, rp.ctypes.data, ci.ctypes.data,
                                        va.ctypes.data, _ptr(eps), float(q), _stream()), "sl1_dict_faust")
        return cls(h, None, int(dims[0]), int(dims[-1]), "faust", dtype)

    def set_tile(self, kt2, kt1):
        """Kronecker stage: correlation items of kt2 x kt1 atoms (sl1_dict_kron_tile)."""
        L.check(L.load().sl1_dict_kron_tile(self.handle, int(kt2), int(kt1)), "sl1_dict_kron_tile")

    def info(self):
        N, K = L.c_i64(), L.c_i64()
        em, rc = L.c_d(), L.c_d()
        L.check(L.load().sl1_dict_info(self.handle, ctypes.byref(N), ctypes.byref(K), ctypes.byref(em),
                                       ctypes.byref(rc)), "sl1_dict_info")
        return dict(N=N.value, K=K.value, eps_max=em.value, rc_model=rc.value)

    def free(self):
        if self._h is not None:
            L.load().sl1_dict_free(self._h)
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def upload_stage(stage, device="cuda"):
    """Device copy of a host stage description with attributes kind, dtype,
    data/scale (dense), B/C (kron) or dims/factors (faust), eps (numpy arrays) and
    optionally q, the norm of eps (2 when absent)."""
    eps = torch.from_numpy(np.ascontiguousarray(stage.eps, dtype=np.float64)).to(device)
    q = float(getattr(stage, "q", 2.0))
    if stage.kind == "dense":
        arr = stage.data.view(np.int16) if stage.dtype == "bf16" else stage.data
        A = torch.from_numpy(np.ascontiguousarray(arr)).to(device)
        sc = None if stage.scale is None else torch.from_numpy(np.ascontiguousarray(stage.scale)).to(device)
        return Dict.dense(A, eps, stage.dtype, sc, q=q)
    if stage.kind == "faust":
        return Dict.faust(stage.dims, stage.factors, eps, stage.dtype, q=q)
    conv = (lambda a: a.view(np.int16)) if stage.dtype == "bf16" else (lambda a: a)
    B = torch.from_numpy(np.ascontiguousarray(conv(stage.B))).to(device)
    C = torch.from_numpy(np.ascontiguousarray(conv(stage.C))).to(device)
    return Dict.kron(B, C, eps, stage.dtype, q=q)


_ENGINES = {"auto": 0, "grid": L.FLAG_ENGINE_GRID, "wg": L.FLAG_ENGINE_WG, "hybrid": L.FLAG_ENGINE_HYBRID}


def solve(stages, L_, rc, atom_norm, y, lam, Gamma=0.5, tol=1e-6, max_iter=100000, margin=1e-12, chunk=16,
          trace_cap=0, use_graph=True, profile=False, check=True, engine="auto", tail_gram=True,
          update="fista", rule="gap", batched_gemm=True, screen_every=1, gemm_signals=0, x0=None, noalloc=False,
          kron_first=True, step=None, park_all=False):
    """Algorithm 1 on a batch: y (batch, N) and lam (batch,) device tensors.
    engine: "auto", "grid" (per-iteration launches), "wg" (one workgroup per
    signal for the whole solve) or "hybrid" (grid, then a tail kernel once every
    signal is on the last, dense, stage with a small preserved set); kron_first:
    the hybrid engine runs Kronecker approximations in the whole-solve kernel
    (False: on the grid kernels); park_all: the grid kernels start only once every
    signal has left that phase (by default, for 128 signals or more, they start when at
    most batch / 128 are still on the approximations; those go on beside them on a
    second stream); step: where every live signal can only be on
    dense stages, the grid engine does the update and the next forward in one
    launch with one block per signal (None: for batches of 128 signals or more;
    True: for any batch; False: separate chip-wide launches); tail_gram:
    the tail iterates on G = A_t^T A_t once |A_t| fits (else it streams columns);
    update: "fista" or "ista"; rule: "gap" (stable GAP Safe), "dst" (stable
    Dynamic Safe, Table I) or "dome" (stable GAP Safe intersected with the GAP
    dome of the same dual point; grid engine); batched_gemm: signals with large preserved sets on
    the exact dense stage share one matrix-core correlation product;
    screen_every: atoms are rejected only every screen_every iterations;
    gemm_signals: qualifying signals from which the batched product runs (0: 64);
    x0: optional (batch, K) float64 device tensor, the initial iterate (warm start);
    noalloc: call sl1_solve_noalloc (workspace in the library's fixed device array;
    the outputs below are still allocated here, by torch).
    Returns a dict of device tensors x, gap, gap_cert, screened, iters, stage, the
    status code, and the trace (batch, trace_cap, 13) when requested."""
    if engine not in _ENGINES:
        raise ValueError(f"engine must be one of {sorted(_ENGINES)}")
    if update not in ("fista", "ista") or rule not in ("gap", "dst", "dome"):
        raise ValueError("update must be 'fista' or 'ista', rule 'gap', 'dst' or 'dome'")
    if y.dtype not in (torch.float64, torch.float32):
        raise TypeError("y must be float32 or float64")
    _dev(y, None, "y")
    _dev(lam, torch.float64, "lam")
    _dev(atom_norm, torch.float64, "atom_norm")
    if y.dim() == 1:
        y = y.unsqueeze(0)
    batch, N = y.shape
    K = stages[0].K
    dev = y.device
    n = len(stages)
    arr = (L.c_dict * n)(*[s.handle for s in stages])
    Ls = (L.c_d * n)(*[float(v) for v in L_])
    rcs = (L.c_d * n)(*[float(v) for v in rc])
    opts = L.Opts()
    L.load().sl1_opts_default(ctypes.byref(opts))
    opts.Gamma, opts.tol, opts.margin = Gamma, tol, margin
    opts.max_iter, opts.chunk = max_iter, chunk
    opts.screen_every = int(screen_every)
    opts.gemm_signals = int(gemm_signals)
    if x0 is not None:
        _dev(x0, torch.float64, "x0")
        if x0.dim() == 1:
            x0 = x0.unsqueeze(0)
        if tuple(x0.shape) != (batch, K):
            raise ValueError(f"x0 must have shape ({batch}, {K})")
        x0 = x0.contiguous()
        opts.x0 = x0.data_ptr()
    opts.y_dtype = L.F64 if y.dtype == torch.float64 else L.F32
    opts.flags = (0 if use_graph else L.FLAG_NO_GRAPH) | (L.FLAG_PROFILE if profile else 0) | _ENGINES[engine] | \
        (0 if tail_gram else L.FLAG_TAIL_COLUMNS) | (L.FLAG_ISTA if update == "ista" else 0) | \
        (L.FLAG_RULE_DST if rule == "dst" else 0) | (L.FLAG_RULE_DOME if rule == "dome" else 0) | \
        (0 if batched_gemm else L.FLAG_NO_GEMM) | (0 if kron_first else L.FLAG_HYBRID_GRID_FIRST) | \
        ({None: 0, True: L.FLAG_GRID_STEP, False: L.FLAG_GRID_SPLIT_STEP}[step]) | \
        (L.FLAG_PARK_ALL if park_all else 0)
    trace = None
    if trace_cap > 0:
        trace = torch.zeros((batch, trace_cap, L.TRACE_FIELDS), dtype=torch.float64, device=dev)
        opts.trace = trace.data_ptr()
        opts.trace_cap = trace_cap
    x = torch.empty((batch, K), dtype=torch.float64, device=dev)
    gap = torch.empty(batch, dtype=torch.float64, device=dev)
    gap_cert = torch.empty(batch, dtype=torch.float64, device=dev)
    screened = torch.empty((batch, K), dtype=torch.uint8, device=dev)
    iters = torch.empty(batch, dtype=torch.int32, device=dev)
    stage = torch.empty(batch, dtype=torch.int32, device=dev)
    entry = "sl1_solve_noalloc" if noalloc else "sl1_solve"
    code = getattr(L.load(), entry)(arr, n, Ls, rcs, _ptr(atom_norm), batch, _ptr(y), _ptr(lam), ctypes.byref(opts),
                                    _ptr(x), _ptr(gap), _ptr(gap_cert), _ptr(screened), _ptr(iters), _ptr(stage),
                                    _stream())
    if check:
        L.check(code, entry)
    out = dict(x=x, gap=gap, gap_cert=gap_cert, screened=screened, iters=iters, stage=stage, status=code)
    if trace is not None:
        out["trace"] = trace
    return out


def lambda_max(d, y):
    """Stable lambda'_max of stage d for each signal (Section III-C)."""
    if y.dim() == 1:
        y = y.unsqueeze(0)
    work = L.F64 if y.dtype == torch.float64 else L.F32
    _dev(y, None, "y")
    out = torch.empty(y.shape[0], dtype=torch.float64, device=y.device)
    L.check(L.load().sl1_lambda_max(d.handle, y.shape[0], _ptr(y), work, _ptr(out), _stream()), "sl1_lambda_max")
    return out


def adjoint(d, y):
    """(A~^T z, z) for each signal, with z = y as the solver stores it."""
    if y.dim() == 1:
        y = y.unsqueeze(0)
    work = L.F64 if y.dtype == torch.float64 else L.F32
    _dev(y, None, "y")
    out = torch.empty((y.shape[0], d.K), dtype=torch.float64, device=y.device)
    z = torch.empty(y.shape, dtype=torch.float64, device=y.device)
    L.check(L.load().sl1_dict_adjoint(d.handle, y.shape[0], _ptr(y), work, _ptr(out), _ptr(z), _stream()),
            "sl1_dict_adjoint")
    return out, z


def solve_path(stages, L_, rc, atom_norm, y, lams, warm=True, **kw):
    """Solves along a sequence of regularization parameters: lams is a list of
    (batch,) float64 device tensors (usually decreasing).  With warm=True each solve
    starts from the previous solution (x0), the sequential setting Section I-D
    mentions; the test itself is the same stable screening from the full atom set.
    Returns the list of solve() results."""
    outs = []
    x0 = None
    for lam in lams:
        out = solve(stages, L_, rc, atom_norm, y, lam, x0=x0 if warm else None, **kw)
        outs.append(out)
        x0 = out["x"]
    return outs


def measure_rc(stages, batch=1):
    """Measured relative complexity of each stage's correlation product."""
    n = len(stages)
    arr = (L.c_dict * n)(*[s.handle for s in stages])
    out = (L.c_d * n)()
    L.check(L.load().sl1_measure_rc(arr, n, batch, out, _stream()), "sl1_measure_rc")
    return [out[i] for i in range(n)]


def tune_kron(stages, batch=1):
    """Autotunes the correlation tile shape of every Kronecker stage for this batch size
    (sl1_tune_kron); returns [(kt2, kt1) or None per stage] and the launch times (ms)."""
    n = len(stages)
    arr = (L.c_dict * n)(*[s.handle for s in stages])
    shp = (L.c_i32 * (2 * n))()
    ms = (L.c_d * n)()
    L.check(L.load().sl1_tune_kron(arr, n, batch, shp, ms, _stream()), "sl1_tune_kron")
    return [((shp[2 * i], shp[2 * i + 1]) if shp[2 * i] else None) for i in range(n)], [ms[i] for i in range(n)]


def last_solve_clock(batch, N, K):
    """(start, converged) device clock stamps in seconds of the last solve of this shape."""
    buf = (ctypes.c_longlong * (2 * batch))()
    rate = L.c_d()
    L.check(L.load().sl1_last_solve_clock(batch, N, K, buf, ctypes.byref(rate)), "sl1_last_solve_clock")
    a = np.frombuffer(buf, dtype=np.int64).reshape(batch, 2).astype(np.float64)
    return a / (rate.value * 1e3)


def last_solve_profile(batch, N, K):
    """{kernel: (total ms, launches)} of the grid kernels in the last solve run
    with profile=True."""
    ms = (L.c_d * L.GRID_KERNELS)()
    n = (ctypes.c_longlong * L.GRID_KERNELS)()
    L.check(L.load().sl1_last_solve_profile(batch, N, K, ms, n), "sl1_last_solve_profile")
    names = ("fwd", "adj_dense", "adj_kron", "upd", "adj_gemm", "gemm_fin", "step")
    return {names[k]: (ms[k], n[k]) for k in range(L.GRID_KERNELS)}


def last_solve_phases(batch, N, K):
    """(engine name, {phase: ms}) of the last solve of this shape.  With
    profile=True the whole-solve part fills the phase times (workgroup ms summed
    over signals), "wg_ms" (elapsed ms of its launches) and "wg_launches"; a
    hybrid solve's whole-solve phase on the Kronecker approximations fills
    "kron_wg_ms" (part of "wg_ms"), "kron_wg_phases" (its own four sums) and
    "kron_wg_launches" (their number, a launch beside the grid kernels included);
    "gram_cap" is the Gram capacity of a hybrid tail (0: none), "gemm_min" the
    |A_t| from which signals joined the batched correlation product (0: off)."""
    eng = L.c_i32()
    ph = (L.c_d * 11)()
    n = ctypes.c_longlong()
    gcap = L.c_i32()
    gmin = L.c_i32()
    L.check(L.load().sl1_last_solve_phases(batch, N, K, ctypes.byref(eng), ph, ctypes.byref(n), ctypes.byref(gcap),
                                           ctypes.byref(gmin)), "sl1_last_solve_phases")
    name = {L.ENGINE_GRID: "grid", L.ENGINE_WG: "wg", L.ENGINE_HYBRID: "hybrid"}.get(eng.value, "none")
    keys = ("fwd", "adj_dense", "gram", "upd", "wg_ms") if name == "hybrid" else \
        ("fwd", "adj_dense", "adj_kron", "upd", "wg_ms")
    out = dict(zip(keys, list(ph)[:5]))
    out["kron_wg_ms"] = ph[5]
    out["kron_wg_phases"] = dict(zip(("fwd", "adj_dense", "adj_kron", "upd"), list(ph)[6:10]))
    out["kron_wg_launches"] = int(ph[10])
    out["wg_launches"] = n.value
    out["gram_cap"] = gcap.value
    out["gemm_min"] = gmin.value
    return name, out


def grad(A, x, y, lam, dx):
    """Implicit adjoint on the support of x: returns (dL/dy, dL/dlambda)."""
    if x.dim() == 1:
        x, y, dx = x.unsqueeze(0), y.unsqueeze(0), dx.unsqueeze(0)
    work = L.F64 if y.dtype == torch.float64 else L.F32
    _dev(x, torch.float64, "x")
    _dev(dx, torch.float64, "dx")
    _dev(y, None, "y")
    _dev(lam, torch.float64, "lam")
    dy = torch.empty_like(y)
    dlam = torch.empty(x.shape[0], dtype=torch.float64, device=x.device)
    L.check(L.load().sl1_grad(A.handle, x.shape[0], _ptr(x), _ptr(y), _ptr(lam), _ptr(dx), _ptr(dy), _ptr(dlam),
                              work, _stream()), "sl1_grad", allow_warn=False)
    return dy, dlam


class LassoFunction(torch.autograd.Function):
    """x* = Lasso(y, lambda) through Algorithm 1; backward by the implicit
    adjoint on the final support (the exact dictionary is stages[-1])."""

    @staticmethod
    def forward(ctx, y, lam, stages, L_, rc, atom_norm, opts):
        out = solve(stages, L_, rc, atom_norm, y.detach().contiguous(), lam.detach().contiguous(), **(opts or {}))
        x = out["x"]
        ctx.stages = stages
        ctx.save_for_backward(x, y.detach(), lam.detach())
        return x

    @staticmethod
    def backward(ctx, gx):
        x, y, lam = ctx.saved_tensors
        dy, dlam = grad(ctx.stages[-1], x, y if y.dim() == 2 else y.unsqueeze(0), lam,
                        gx.contiguous().to(torch.float64))
        if y.dim() == 1:
            dy = dy[0]
        return dy, dlam.reshape(lam.shape), None, None, None, None, None


def lasso(y, lam, stages, L_, rc, atom_norm, **opts):
    """Differentiable solution map (see LassoFunction)."""
    return LassoFunction.apply(y, lam, stages, L_, rc, atom_norm, opts)
