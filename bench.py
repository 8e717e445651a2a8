#!/usr/bin/env python3
"""Time-to-gap 1e-6 and FISTA iterations/s of the stable-screening Lasso solver
on one MI355X.

Workload (one "step" = one complete solve of the batch to duality gap 1e-6,
i.e. every row of the hot path, iterated):
  batched low precision: 512 signals on a shared Kronecker dictionary
  N=1024 (32x32), K=4096 (64x64), A = sum_{r<=4} B_r kron C_r + 0.01 G (FP32),
  stages A~_1, A~_2, A~_4 with BF16 factors then A (FP32); per-signal sparsity
  U{5..80}, lambda/lambda_max U[0.2, 0.9], noise U[0.001, 0.05].
Comparator: plain FP32 FISTA + GAP Safe screening on the same batch (the single
stage [A], same kernels).  A second block reports the single-signal FP32
configuration N=4096 (64x64), K=16384 (128x128), R=8, lambda = 0.5 lambda_max.

Prints one JSON line.  Inputs are synthetic and seeded (see synth/).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-single", action="store_true", help="skip the single-signal block")
    ap.add_argument("--no-parity", action="store_true", help="skip the sampled oracle parity check")
    ap.add_argument("--no-variants", action="store_true", help="skip the ISTA / Dynamic Safe variants")
    ap.add_argument("--no-faust", action="store_true", help="skip the FAuST (MEG-shaped) block")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense precision block (N=2500, K=10000)")
    ap.add_argument("--parity-signals", type=int, default=0,
                    help="signals of the batched workload checked against the oracle (0: all)")
    ap.add_argument("--blocks", default="batched,single,faust,dense,grad",
                    help="comma-separated blocks to run (profiling runs of one block; the JSON line's headline "
                         "fields need 'batched')")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (HBM counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def upload(sl1, torch, p):
    st = [sl1.upload_stage(s) for s in p.stages]
    dev = "cuda"
    Y = torch.from_numpy(p.Y).to(torch.float32).to(dev)
    lam = torch.from_numpy(p.lam).to(dev)
    an = torch.from_numpy(p.atom_norm).to(dev)
    return st, Y, lam, an


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    out = None
    for _ in range(steps):
        out = fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / steps, out


UPD_BYTES_PER_ATOM = 76.0   # test/update per preserved atom: index, 7 FP64 gathers, x and index writes


def gemm_plan(S, N, K, batch):
    """Tiles and row splits of one batched-product launch over S signals (the
    rule the product kernel applies): (tiles, splits)."""
    nat = -(-K // 64)
    tiles = nat * -(-S // 64)
    tiles_max = nat * -(-batch // 64)
    grid = min(max(tiles_max, min(tiles_max * 8, 512)), 1024)
    nch = -(-N // 32)
    ks = 1
    if 2 * tiles <= grid:
        ks = max(1, min(8, nch, min(grid, 512) // tiles))
    cps = -(-nch // ks)
    return tiles, -(-nch // cps)


def row_split(p, trace, iters, engine, grid_launches, kron_first):
    """Per signal b, the rows (iterations) of each engine part: rows < s0[b] ran in
    the whole-solve kernel on the Kronecker approximations (hybrid solve that runs
    them there), rows in [s0[b], s1[b]) in the grid kernels, rows >= s1[b] in the
    tail kernel (hybrid) or the whole-solve kernel (whole-solve engine)."""
    import numpy as np
    I = len(p.stages) - 1
    B = trace.shape[0]
    s0 = np.zeros(B, dtype=int)
    s1 = np.zeros(B, dtype=int)
    for b in range(B):
        n = int(iters[b])
        if engine == "wg":
            continue
        if engine == "grid":
            s1[b] = n
            continue
        start = 0
        if kron_first:
            on = np.nonzero(trace[b, :n, 1] == I)[0]
            start = int(on[0]) if len(on) else n
        s0[b] = start
        s1[b] = min(n, start + grid_launches)
    return s0, s1


def product_rows(p, trace, iters, s0, s1, gemm_min, gemm_signals=64, chunk=16, first_by_count=False):
    """(batch, T) mask of the grid rows whose correlations went through the batched
    product: the signal qualifies (exact dense stage, |A_t| >= gemm_min) and the
    product ran in that chunk of grid launches (the first chunk: batch >= gemm_signals,
    or, after the Kronecker whole-solve phase, that many signals qualify at their first
    grid row; a later one: at least gemm_signals signals qualified at the previous
    chunk's last row).  Column u of a signal is its grid row s0 + u."""
    import numpy as np
    B = trace.shape[0]
    T = int(max(1, (s1 - s0).max()))
    I = len(p.stages) - 1
    q = np.zeros((B, T), dtype=bool)
    if gemm_min <= 0 or p.stages[I].kind != "dense":
        return q
    for b in range(B):
        n = int(s1[b] - s0[b])
        r = trace[b, s0[b]:s1[b]]
        q[b, :n] = (r[:, 1] == I) & (r[:, 2] >= gemm_min)
    cnt = q.sum(axis=0)
    for u in range(T):
        c = u // chunk
        if c == 0:
            on = cnt[0] >= gemm_signals if first_by_count else p.batch >= gemm_signals
        else:
            on = cnt[c * chunk - 1] >= gemm_signals
        if not on:
            q[:, u] = False
    return q


def kernel_work(p, trace, iters, s0, s1, step, gram_cap=0, gemm_min=0, kron_first=False):
    """Algorithmic work of each kernel over one solve, from the trace and the row
    split of row_split:
      dense correlations  |A_t| N b bytes (b: bytes per stored element, + 4 B per
                          column scale); Kronecker correlations 2 R k2 n1 (n2 + k1)
                          flops (sum_r C_r^T P B_r);
      forward             per signal: the nonzero list (12 B per nonzero), the gathered
                          columns on dense stages (||x_t||_0 N b), one read of the
                          factors on Kronecker stages (R (n1 k1 + n2 k2) b) or of the
                          factor entries on FAuST stages, the signal read and the FP64
                          residual written (N (b_y + 8)) in the grid kernels;
      update              76 B per preserved atom in the grid kernels (the tail
                          keeps the per-atom state in LDS);
      step                forward and update of the grid rows (one launch does the
                          update of a row and the forward of the next);
      tail, Gram form     rows with |A_t| <= gram_cap: the |A_t| columns read once
                          to form G and A_t^T y, then no HBM traffic per iteration;
      batched product     grid rows that went through it: 2 N |A_t| FP64 flops (the
                          needed entries; the product also forms the discarded ones,
                          2 N K per signal);
      finishing pass      the partial tiles of row-split product launches, read
                          once (64 x 64 doubles per tile and split);
      Kronecker phase     rows before s0 (whole-solve kernel): the Kronecker
                          correlations' matrix-core flops."""
    import numpy as np
    N = p.N
    w = dict(fwd_bytes=[0.0, 0.0], adj_bytes=[0.0, 0.0], adj_flops=[0.0, 0.0], upd_bytes=[0.0, 0.0],
             gram_bytes=0.0, gram_it=0, gemm_flops=0.0, gemm_exec_flops=0.0, gemm_it=0, fin_bytes=0.0,
             dense_it=[0, 0], kron_it=[0, 0], faust_it=[0, 0], kwg_flops=0.0, kwg_it=0, step_bytes=0.0)
    I = len(p.stages) - 1
    prod = product_rows(p, trace, iters, s0, s1, gemm_min, first_by_count=kron_first)
    for S in prod.sum(axis=0):
        if S > 0:
            tiles, ks = gemm_plan(int(S), N, p.K, p.batch)
            if ks > 1:
                w["fin_bytes"] += tiles * ks * 64 * 64 * 8.0
    by = 8 if p.work == "f64" else 4
    for b in range(trace.shape[0]):
        n = int(iters[b])
        rows = trace[b, :n]
        t = np.arange(n)
        kwg = t < s0[b]
        part = np.where(t < s1[b], 0, 1)          # 0: grid kernels, 1: tail / whole-solve kernel
        part[kwg] = 2
        gram = (part == 1) & (rows[:, 2] <= gram_cap) if gram_cap > 0 else np.zeros(n, dtype=bool)
        for s_idx, st in enumerate(p.stages):
            bpe = 0.0
            if st.kind == "dense":
                bpe = {"f64": 8, "f32": 4, "bf16": 2, "fp8": 1}[st.dtype] + (4.0 / N if st.scale is not None else 0)
            on = rows[:, 1] == s_idx
            if st.kind == "kron":
                n1, k1, n2, k2 = st.dims
                m = on & (part == 2)
                w["kwg_flops"] += int(m.sum()) * 2.0 * st.R * k2 * n1 * (n2 + k1)
                w["kwg_it"] += int(m.sum())
            on = on & (part != 2)
            g = on & gram
            if s_idx == I and st.kind == "dense" and gemm_min > 0:
                gm = np.zeros(n, dtype=bool)
                u0, u1 = int(s0[b]), int(min(n, s0[b] + prod.shape[1]))
                gm[u0:u1] = prod[b, :u1 - u0]
                gm &= on
                if gm.any():
                    w["gemm_flops"] += 2.0 * N * float(rows[gm, 2].sum())
                    w["gemm_exec_flops"] += 2.0 * N * p.K * int(gm.sum())
                    w["gemm_it"] += int(gm.sum())
                    w["fwd_bytes"][0] += (N * bpe + 12.0) * float(rows[gm, 12].sum()) + N * (by + 8.0) * int(gm.sum())
                    w["upd_bytes"][0] += UPD_BYTES_PER_ATOM * float(rows[gm, 2].sum())
                on = on & ~gm
            if g.any():
                w["gram_bytes"] += N * bpe * float(rows[np.argmax(g), 2])
                w["gram_it"] += int(g.sum())
            for ph in (0, 1):
                m = on & (part == ph) & ~gram
                cnt = int(m.sum())
                if not cnt:
                    continue
                if ph == 0:
                    w["upd_bytes"][ph] += UPD_BYTES_PER_ATOM * float(rows[m, 2].sum())
                nz = float(rows[m, 12].sum())
                if ph == 0:                   # residual written and signal read by the forward launch
                    w["fwd_bytes"][0] += N * (by + 8.0) * cnt + 12.0 * nz
                if st.kind == "dense":
                    w["adj_bytes"][ph] += N * bpe * float(rows[m, 2].sum())
                    w["fwd_bytes"][ph] += N * bpe * nz
                    w["dense_it"][ph] += cnt
                elif st.kind == "faust":
                    # the adjoint chain: 2 flops per factor entry (FP64), per signal
                    nnz = sum(len(f[1]) for f in st.factors)
                    vb = {"f64": 8, "f32": 4}[st.dtype] + 4.0
                    w["adj_flops"][ph] += cnt * 2.0 * nnz
                    w["fwd_bytes"][ph] += cnt * vb * sum(len(f[1]) for f in st.factors[:-1]) + \
                        vb * nz * len(st.factors[-1][1]) / st.K
                    w["faust_it"][ph] += cnt
                else:
                    n1, k1, n2, k2 = st.dims
                    fb = {"f64": 8, "f32": 4, "bf16": 2, "fp8": 1}[st.dtype]
                    w["adj_flops"][ph] += cnt * 2.0 * st.R * k2 * n1 * (n2 + k1)
                    w["fwd_bytes"][ph] += cnt * st.R * (n1 * k1 + n2 * k2) * fb
                    w["kron_it"][ph] += cnt
    if step:
        w["step_bytes"] = w["fwd_bytes"][0] + w["upd_bytes"][0]
    return w


MFMA_PEAK_TFLOPS = {"bf16": BF16_PEAK_TFLOPS, "f32": FP32_PEAK_TFLOPS, "f64": FP64_PEAK_TFLOPS}


def roofline_entries(prof, phases, work, tail_kernel="k_solve_tail", kron_dtype="bf16"):
    """Roofline of every kernel of the solve: achieved = algorithmic work /
    measured time (HIP events around each launch), against the MI355X peak of
    its bound; the Kronecker products against the matrix-core peak of their
    factors' storage type (BF16, FP32 or FP64 MFMA)."""
    out = []

    def add(name, ms, launches, amount, unit_kind, peak=BF16_PEAK_TFLOPS):
        if ms <= 0 or launches <= 0:
            return
        if unit_kind == "hbm":
            ach = amount / (ms * 1e-3) / 1e9
            out.append(dict(kernel=name, bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                            frac=ach / HBM_PEAK_GBS, traffic=None, launches=launches, total_ms=ms,
                            avg_launch_us=ms * 1e3 / launches))
        else:
            ach = amount / (ms * 1e-3) / 1e12
            out.append(dict(kernel=name, bound=unit_kind, achieved=ach, peak=peak, unit="TFLOP/s",
                            frac=ach / peak, traffic=None, launches=launches, total_ms=ms,
                            avg_launch_us=ms * 1e3 / launches))

    add("k_step", *prof.get("step", (0.0, 0)), work["step_bytes"], "hbm")
    add("k_fwd", *prof["fwd"], work["fwd_bytes"][0], "hbm")
    add("k_adj_dense", *prof["adj_dense"], work["adj_bytes"][0], "hbm")
    if work["faust_it"][0] > work["kron_it"][0]:    # structured launch running FAuST chains (FP64 vector)
        add("k_adj_kron", *prof["adj_kron"], work["adj_flops"][0], "alu", FP64_PEAK_TFLOPS)
    else:
        add("k_adj_kron", *prof["adj_kron"], work["adj_flops"][0], "mfma", MFMA_PEAK_TFLOPS[kron_dtype])
    add("k_upd", *prof["upd"], work["upd_bytes"][0], "hbm")
    if "adj_gemm" in prof:
        add("k_adj_gemm", *prof["adj_gemm"], work["gemm_flops"], "mfma", FP64_PEAK_TFLOPS)
        if out and out[-1]["kernel"] == "k_adj_gemm" and prof["adj_gemm"][0] > 0:
            out[-1]["executed_tflops"] = work["gemm_exec_flops"] / (prof["adj_gemm"][0] * 1e-3) / 1e12
    if "gemm_fin" in prof:
        add("k_gemm_fin", *prof["gemm_fin"], work["fin_bytes"], "hbm")
    kwg_ms = phases.get("kron_wg_ms", 0.0)
    # the Kronecker approximations' whole-solve phase: its launch, and the one beside the
    # grid kernels when late signals went on there (durations summed)
    kwg_n = phases.get("kron_wg_launches", 1) if kwg_ms > 0 else 0
    if kwg_ms > 0:
        add("k_solve_wg", kwg_ms, kwg_n, work["kwg_flops"], "mfma", MFMA_PEAK_TFLOPS[kron_dtype])
    if phases.get("wg_launches", 0) > kwg_n:
        add(tail_kernel, phases["wg_ms"] - kwg_ms, phases["wg_launches"] - kwg_n,
            work["fwd_bytes"][1] + work["adj_bytes"][1] + work["upd_bytes"][1] + work["gram_bytes"], "hbm")
    out.sort(key=lambda e: -e["total_ms"])
    return out


def solve_block(sl1, torch, np, p, tol, steps, warmup, label):
    st, Y, lam, an = upload(sl1, torch, p)
    L = [s.L for s in p.stages]
    tiles = None
    if any(s.kind == "kron" for s in p.stages):
        tiles, _ = sl1.tune_kron(st, batch=p.batch)
        log(f"{label}: Kronecker tile shapes (autotuned) {tiles}")
    log(f"{label}: measuring relative complexities")
    rc_meas = sl1.measure_rc(st, batch=p.batch)
    rc = rc_meas
    log(f"{label}: RC measured {['%.3f' % v for v in rc_meas]} model {['%.3f' % s.rc_theory for s in p.stages]}")

    def method():
        return sl1.solve(st, L, rc, an, Y, lam, tol=tol)

    def plain():
        return sl1.solve([st[-1]], [L[-1]], [1.0], an, Y, lam, tol=tol)

    ms_m, out_m = timed(torch, method, steps, warmup)
    engine = sl1.last_solve_phases(p.batch, p.N, p.K)[0]
    clk = sl1.last_solve_clock(p.batch, p.N, p.K)
    ttg_dev = float(np.max(clk[:, 1] - clk[:, 0])) * 1e3
    ms_p, out_p = timed(torch, plain, steps, warmup)
    engine_p = sl1.last_solve_phases(p.batch, p.N, p.K)[0]
    # the same solve continued to the accuracy gap (untimed), where parity is evaluated
    acc_tol = 1e-10
    out_a = sl1.solve(st, L, rc, an, Y, lam, tol=acc_tol)
    it_m = int(out_m["iters"].sum().item())
    it_p = int(out_p["iters"].sum().item())
    gap_m = out_m["gap"].cpu().numpy()
    gap_p = out_p["gap"].cpu().numpy()
    log(f"{label}: method {ms_m:.3f} ms ({it_m} iters, {engine}), plain {ms_p:.3f} ms ({it_p} iters, {engine_p})")
    # profiled run (not timed): every kernel launched directly between HIP
    # events on the library's stream, and the trace for the algorithmic work
    cap = int(out_m["iters"].max().item()) + 8
    outp = sl1.solve(st, L, rc, an, Y, lam, tol=tol, profile=True, trace_cap=cap)
    prof = sl1.last_solve_profile(p.batch, p.N, p.K)
    _, phases = sl1.last_solve_phases(p.batch, p.N, p.K)
    trace = outp["trace"].cpu().numpy()
    iters = outp["iters"].cpu().numpy()
    step = prof.get("step", (0.0, 0))[1] > 0
    grid_launches = prof["step"][1] if step else prof["fwd"][1]
    kron_first = phases.get("kron_wg_ms", 0.0) > 0
    s0, s1 = row_split(p, trace, iters, engine, grid_launches, kron_first)
    work = kernel_work(p, trace, iters, s0, s1, step, phases.get("gram_cap", 0), phases.get("gemm_min", 0),
                       kron_first)
    t_split = grid_launches
    res = dict(
        ms_method=ms_m, ms_plain=ms_p, iters_method=it_m, iters_plain=it_p, engine=engine, engine_plain=engine_p,
        time_to_gap_ms_device=ttg_dev, max_gap_method=float(gap_m.max()), max_gap_plain=float(gap_p.max()),
        stage_final=sorted(set(out_m["stage"].cpu().numpy().tolist())), rc_measured=rc_meas, kron_tiles=tiles,
        rc_model=[s.rc_theory for s in p.stages], kernel_ms=prof, wg_phases=phases, grid_iterations=t_split,
        roofline_kernels=roofline_entries(prof, phases, work,
                                          "k_solve_tail" if engine == "hybrid" else "k_solve_wg",
                                          next((s.dtype for s in p.stages if s.kind == "kron"), "bf16")),
        gram_iterations=work["gram_it"], gemm_iterations=work["gemm_it"],
        x=out_m["x"].cpu().numpy(), screened=out_m["screened"].cpu().numpy(),
        acc_tol=acc_tol, x_acc=out_a["x"].cpu().numpy(), screened_acc=out_a["screened"].cpu().numpy(),
        max_gap_acc=float(out_a["gap"].max().item()),
        x_plain=out_p["x"].cpu().numpy(), screened_plain=out_p["screened"].cpu().numpy(),
    )
    return res


# sources whose change voids a recorded HBM-traffic figure of a kernel
_GRID_SOURCES = ["paper_1812_06635_amd/csrc/sl1_kernels.hip", "paper_1812_06635_amd/csrc/sl1_device.hpp",
                 "paper_1812_06635_amd/csrc/sl1_internal.hpp", "include/stablel1.h"]
TRAFFIC_SOURCES = {k: _GRID_SOURCES for k in ("k_adj_dense", "k_adj_gemm", "k_gemm_fin", "k_fwd", "k_upd",
                                               "k_adj_kron", "k_step")}
for _k in ("k_solve_tail", "k_solve_wg"):
    TRAFFIC_SOURCES[_k] = ["paper_1812_06635_amd/csrc/sl1_wg.hip", "paper_1812_06635_amd/csrc/sl1_device.hpp",
                           "paper_1812_06635_amd/csrc/sl1_internal.hpp", "include/stablel1.h"]


def sources_sha256(kernel):
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES.get(kernel, []):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(kernel, workload="batched"):
    """HBM bytes per launch of `kernel` on `workload` (a bench block: "batched",
    "single", "dense", ...) from the rocprofv3 FETCH_SIZE/WRITE_SIZE summaries
    under profiles/ (a 'traffic-record:' line; one without a workload key is the
    batched block's), or None when there is none or the kernel's sources changed
    since the counters were taken."""
    if kernel not in TRAFFIC_SOURCES:
        return None
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    want = sources_sha256(kernel)
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if (kv.get("kernel") == kernel and kv.get("workload", "batched") == workload
                        and kv.get("sources_sha256") == want):
                    return float(kv["bytes_per_launch"])
    return None


VARIANTS = (("fista", "dst"), ("ista", "gap"), ("ista", "dst"), ("fista", "dome"))


def apply_tiles(stages, tiles):
    """The autotuned Kronecker tile shapes (one entry per stage, None elsewhere) on new handles."""
    for d, t in zip(stages, tiles or []):
        if t is not None:
            d.set_tile(*t)


def variants_block(sl1, torch, np, p, rc, tol, steps, warmup, plain_ref=None, tiles=None):
    """The other update / test combinations of Table III (FISTA or ISTA, stable GAP
    Safe or stable Dynamic Safe) on the same batch: time-to-gap of the method and
    of plain FP32 (the single stage [A]) with the same update and test; then the
    method with l1 and l_inf error bounds instead of l2 (plain_ref: time and iterations
    of the headline's plain FP32 solve, FISTA + stable GAP Safe, which has no bounds)."""
    import synth
    st, Y, lam, an = upload(sl1, torch, p)
    apply_tiles(st, tiles)
    L = [s.L for s in p.stages]
    out = []
    for update, rule in VARIANTS:
        def method():
            return sl1.solve(st, L, rc, an, Y, lam, tol=tol, update=update, rule=rule)

        def plain():
            return sl1.solve([st[-1]], [L[-1]], [1.0], an, Y, lam, tol=tol, update=update, rule=rule)

        ms_m, o_m = timed(torch, method, steps, warmup)
        ms_p, o_p = timed(torch, plain, steps, warmup)
        it_m, it_p = int(o_m["iters"].sum().item()), int(o_p["iters"].sum().item())
        log(f"variant {update}/{rule}: method {ms_m:.3f} ms ({it_m} iters), plain {ms_p:.3f} ms ({it_p} iters)")
        out.append(dict(update=update, rule=rule, time_to_gap_ms=ms_m, iters=it_m,
                        iters_per_s=it_m / (ms_m * 1e-3), plain_fp32_time_to_gap_ms=ms_p, plain_fp32_iters=it_p,
                        speedup_vs_plain_fp32=ms_p / ms_m, max_gap=float(o_m["gap"].max().item()),
                        _x=o_m["x"].cpu().numpy(), _screened=o_m["screened"].cpu().numpy()))
    # FISTA + stable GAP Safe with the approximations' bounds in l1 and l_inf (Lemma 1 with an
    # l_q zone); the plain comparator has no bounds, so it is the FISTA / GAP one above
    for q, name in ((1.0, "l1"), (float("inf"), "l_inf")):
        pq = synth.with_lq_bounds(p, q)
        stq = [sl1.upload_stage(s) for s in pq.stages]
        apply_tiles(stq, tiles)

        def method_q():
            return sl1.solve(stq, L, rc, an, Y, lam, tol=tol)

        ms_m, o_m = timed(torch, method_q, steps, warmup)
        it_m = int(o_m["iters"].sum().item())
        log(f"variant fista/gap with {name} bounds: method {ms_m:.3f} ms ({it_m} iters)")
        entry = dict(update="fista", rule="gap", bounds=name, time_to_gap_ms=ms_m, iters=it_m,
                     iters_per_s=it_m / (ms_m * 1e-3), max_gap=float(o_m["gap"].max().item()),
                     _x=o_m["x"].cpu().numpy(), _screened=o_m["screened"].cpu().numpy())
        if plain_ref is not None:
            entry.update(plain_fp32_time_to_gap_ms=plain_ref[0], plain_fp32_iters=plain_ref[1],
                         speedup_vs_plain_fp32=plain_ref[0] / ms_m)
        out.append(entry)
        del stq
    # FISTA + stable GAP Safe with the approximations' factors stored in FP8 E4M3 (the same
    # dictionary, signals and lambdas; the factors' own rounding is in their eps)
    p8 = synth.config4(batch=p.batch, factor_dtype="fp8") if p.name == "C4" else None
    if p8 is not None and np.array_equal(p8.Y, p.Y):
        st8 = [sl1.upload_stage(s) for s in p8.stages]
        tiles8, _ = sl1.tune_kron(st8, batch=p8.batch)
        rc8 = sl1.measure_rc(st8, batch=p8.batch)

        def method_8():
            return sl1.solve(st8, [s.L for s in p8.stages], rc8, an, Y, lam, tol=tol)

        ms_m, o_m = timed(torch, method_8, steps, warmup)
        it_m = int(o_m["iters"].sum().item())
        log(f"variant fista/gap with FP8 factors: method {ms_m:.3f} ms ({it_m} iters), tiles {tiles8}")
        entry = dict(update="fista", rule="gap", factors="fp8", time_to_gap_ms=ms_m, iters=it_m,
                     iters_per_s=it_m / (ms_m * 1e-3), max_gap=float(o_m["gap"].max().item()), rc_measured=rc8,
                     kron_tiles_autotuned=tiles8, eps_max=[float(s.eps.max()) for s in p8.stages],
                     _x=o_m["x"].cpu().numpy(), _screened=o_m["screened"].cpu().numpy())
        if plain_ref is not None:
            entry.update(plain_fp32_time_to_gap_ms=plain_ref[0], plain_fp32_iters=plain_ref[1],
                         speedup_vs_plain_fp32=plain_ref[0] / ms_m)
        out.append(entry)
        del st8
    return out


def roofline(res, workload="batched"):
    """The kernel with the largest share of the solve's device time, with its
    recorded HBM traffic per launch on this workload when the counters match the
    current code."""
    r = dict(res["roofline_kernels"][0])
    r["traffic"] = recorded_traffic(r["kernel"], workload)
    return r


def oracle_reference(p, indices=None, label=""):
    """{b: (x*, P*, kkt, margin)} of the FP64 oracle (the Lasso definition, polished
    and certified) for the signals in indices (default: all), in worker processes."""
    import oracle.pool as opool

    def progress(done, total):
        if done % 64 == 0 or done == total:
            log(f"{label}: oracle solved {done} of {total} signals")

    return opool.solve_batch(p.A, p.Y, p.lam, p.stages[-1].L, indices=indices, progress=progress)


def oracle_errors(np, p, x, screened, ref):
    """Error of solutions x (batch, K) against the oracle on the signals of ref: unsafe
    rejections (screened atoms in the support of x*), relative objective error and
    ||x - x*|| / ||x*||, the largest over the signals."""
    import oracle.lasso as ol
    worst_obj, worst_x, unsafe = 0.0, 0.0, 0
    for b, (xs, Ps, _, _) in ref.items():
        xb = np.asarray(x[b], dtype=np.float64)
        P = ol.primal(p.A, p.Y[b], float(p.lam[b]), xb)
        worst_obj = max(worst_obj, (P - Ps) / Ps)
        nx = np.linalg.norm(xs)
        if nx > 0:
            worst_x = max(worst_x, float(np.linalg.norm(xb - xs) / nx))
        unsafe += int(np.sum((screened[b] == 1) & (xs != 0)))
    return dict(signals=len(ref), unsafe_rejections=unsafe, max_rel_obj=float(worst_obj), max_rel_x=worst_x)


def block_parity(np, p, res, ref, tol):
    """Oracle errors of a block: the method at the timed stop (gap < tol) and continued
    to the accuracy gap, and the plain FP32 comparator at the timed stop."""
    return {"signals": len(ref), "timed_stop_gap": tol,
            "method_at_timed_stop": oracle_errors(np, p, res["x"], res["screened"], ref),
            "accuracy_gap": res["acc_tol"],
            "method_at_accuracy_gap": oracle_errors(np, p, res["x_acc"], res["screened_acc"], ref),
            "plain_fp32_at_timed_stop": oracle_errors(np, p, res["x_plain"], res["screened_plain"], ref)}


def blas_info():
    try:
        from threadpoolctl import threadpool_info
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            return info[0].get("internal_api", "?"), max(int(i.get("num_threads", 1)) for i in info)
    except Exception:
        pass
    return "unknown", os.cpu_count()


def cpu_legs(np, p, ref, signals, tol, threads=None):
    """The paper's normalized-time legs (Section V-B), each to gap tol on the same
    signals, timed on the host with the oracle code as it stands: T_N = plain FP64
    FISTA without screening on A (the oracle's solver; its stop test is gap <
    tol max(1, P), given tol / max(1, P*) so that it stops at gap tol), T_A = the
    method reference on [A] alone (FISTA + GAP Safe, the stable test with eps = 0),
    T_A~ = the method reference on the whole stage sequence.  The method reference
    forms every product densely in FP64 (it checks arithmetic, it is not a fast
    implementation), so T_A~ / T_N reflects iteration counts, not the structured
    products' cost.  threads: BLAS threads (None: all)."""
    import contextlib
    import oracle.lasso as ol
    import oracle.screening as osc
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(threads) if threads else contextlib.nullcontext()
    except Exception:
        ctx = contextlib.nullcontext()
    st = [(s.values(), s.eps, s.L) for s in p.stages]
    rc = [s.rc_theory for s in p.stages]
    L = p.stages[-1].L
    t = dict(T_N=0.0, T_A=0.0, T_At=0.0)
    it = dict(T_N=0, T_A=0, T_At=0)
    with ctx:
        for b in signals:
            y, lam = p.Y[b], float(p.lam[b])
            P = ref[b][1]
            t0 = time.perf_counter()
            _, _, n = ol.fista(p.A, y, lam, L, tol=tol / max(1.0, P))
            t["T_N"] += time.perf_counter() - t0
            it["T_N"] += n
            t0 = time.perf_counter()
            r = osc.fast_l1(st[-1:], p.atom_norm, y, lam, [1.0], tol=tol, keep_trace=False)
            t["T_A"] += time.perf_counter() - t0
            it["T_A"] += r.iters
            t0 = time.perf_counter()
            r = osc.fast_l1(st, p.atom_norm, y, lam, rc, tol=tol, keep_trace=False)
            t["T_At"] += time.perf_counter() - t0
            it["T_At"] += r.iters
    n = len(signals)
    return {"signals": list(signals), "threads": threads or blas_info()[1],
            "time_to_gap_s_per_signal": {k: v / n for k, v in t.items()},
            "iterations_per_signal": {k: v / n for k, v in it.items()},
            "T_A_over_T_N": t["T_A"] / t["T_N"], "T_At_over_T_N": t["T_At"] / t["T_N"]}


def cpu_baseline(np, p, ref, tol, signals=(0, 1, 2, 3)):
    """The FP64 oracle (plain FISTA, exact A, no screening) to gap tol on a sample of
    the workload's signals, timed on the host with all BLAS threads and with one, next
    to the method reference's legs T_A and T_A~ (cpu_legs)."""
    vendor, threads = blas_info()
    legs_all = cpu_legs(np, p, ref, signals, tol)
    legs_one = cpu_legs(np, p, ref, signals[:1], tol, threads=1)
    per = legs_all["time_to_gap_s_per_signal"]["T_N"]
    its = legs_all["iterations_per_signal"]["T_N"]
    return dict(value=its / per, unit="iter/s", cores=threads, kind="oracle",
                sample=f"FP64 FISTA without screening, exact A (N={p.N}, K={p.K}), to gap {tol:g}, signals "
                       f"{list(signals)} of the workload: {its:.0f} iterations, {per * 1e3:.1f} ms per signal "
                       f"({vendor} BLAS, {threads} threads)",
                time_to_gap_ms_per_signal=per * 1e3, blas=vendor, legs_all_threads=legs_all,
                legs_one_thread=legs_one)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the solver has no multi-GPU path "
                                   "(a batch would shard by signal, one process per GPU)", "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch
    if args.calibrate_copy:
        # known traffic: each copy reads and writes 2^30 bytes
        src = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": 2 ** 30,
                          "bytes_written_per_copy": 2 ** 30, "copies": 3}))
        return
    import synth
    import paper_1812_06635_amd as sl1
    torch.cuda.set_device(0)
    sl1.load_library()

    blocks = set(args.blocks.split(","))
    args.no_single = args.no_single or "single" not in blocks
    args.no_faust = args.no_faust or "faust" not in blocks
    args.no_dense = args.no_dense or "dense" not in blocks
    line = {"metric": "time-to-gap 1e-6 and FISTA iters/s (batched low-prec vs plain FP32), 1 GPU", "n_gpus": 1,
            "blocks": sorted(blocks)}
    if "batched" not in blocks:
        args.no_cpu = args.no_variants = True
    else:
        log("generating the batched workload (512 signals, N=1024, K=4096)")
        p = synth.config4(batch=512)
        res = solve_block(sl1, torch, np, p, args.tol, args.steps, args.warmup, "batched")
    line = line if "batched" not in blocks else {
        "metric": "time-to-gap 1e-6 and FISTA iters/s (batched low-prec vs plain FP32), 1 GPU",
        "value": res["iters_method"] / (res["ms_method"] * 1e-3),
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_method"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 factors / fp32 A, fp64 vectors",
        "data": "synthetic (seeded)",
        "config": {"workload": "batched low precision: 512 signals, shared Kronecker dictionary N=1024 (32x32), "
                               "K=4096 (64x64), stages A~_1, A~_2, A~_4 (BF16 factors) then A (FP32), tol 1e-6",
                   "global_batch": p.batch, "N": p.N, "K": p.K},
        "time_to_gap_ms": res["ms_method"],
        "time_to_gap_ms_device": res["time_to_gap_ms_device"],
        "plain_fp32": {"time_to_gap_ms": res["ms_plain"], "iters": res["iters_plain"],
                       "iters_per_s": res["iters_plain"] / (res["ms_plain"] * 1e-3)},
        "speedup_vs_plain_fp32": res["ms_plain"] / res["ms_method"],
        "iters": res["iters_method"],
        "max_gap": res["max_gap_method"],
        "rc_measured": res["rc_measured"],
        "rc_model": res["rc_model"],
        "kron_tiles_autotuned": res["kron_tiles"],
        "engine": res["engine"],
        "kernel_ms": res["kernel_ms"],
        "whole_solve_phases_ms": res["wg_phases"],
        "grid_iterations": res["grid_iterations"],
        "tail_gram_signal_iterations": res["gram_iterations"],
        "batched_product_signal_iterations": res["gemm_iterations"],
        "roofline": roofline(res),
        "roofline_kernels": res["roofline_kernels"],
    }
    ref = None
    if "batched" in blocks and (not args.no_parity or not args.no_cpu):
        idx = None if args.parity_signals <= 0 else \
            np.unique(np.linspace(0, p.batch - 1, min(args.parity_signals, p.batch)).astype(int)).tolist()
        if args.no_parity:
            idx = [0, 1, 2, 3]
        log(f"batched: FP64 oracle on {p.batch if idx is None else len(idx)} signals")
        ref = oracle_reference(p, idx, "batched")
    if "batched" in blocks and not args.no_parity:
        line["parity"] = block_parity(np, p, res, ref, args.tol)
    if not args.no_variants:
        log("update / test variants on the batched workload (1 timed solve each)")
        var = variants_block(sl1, torch, np, p, res["rc_measured"], args.tol, 1, 1,
                             plain_ref=(res["ms_plain"], res["iters_plain"]), tiles=res["kron_tiles"])
        for v in var:
            if ref is not None and not args.no_parity:
                v["oracle_error"] = oracle_errors(np, p, v["_x"], v["_screened"], ref)
            del v["_x"], v["_screened"]
        line["variants"] = var
    if not args.no_cpu:
        log("CPU oracle baseline and the method reference's legs")
        line["cpu_baseline"] = cpu_baseline(np, p, ref, args.tol)
    if not args.no_single:
        log("single-signal block (N=4096, K=16384, R=8, FP32)")
        q = synth.config2(lam_frac=0.5)
        r2 = solve_block(sl1, torch, np, q, args.tol, max(1, args.steps), args.warmup, "single")
        line["single_signal"] = {
            "workload": "N=4096 (64x64), K=16384 (128x128), A = sum_{r<=8} B_r kron C_r + 0.01 G (FP32), "
                        "stages A~_1, A~_2, A~_4, A~_8 (FP32 factors) then A, lambda = 0.5 lambda_max, tol 1e-6",
            "time_to_gap_ms": r2["ms_method"], "iters": r2["iters_method"],
            "iters_per_s": r2["iters_method"] / (r2["ms_method"] * 1e-3),
            "plain_fp32_time_to_gap_ms": r2["ms_plain"], "plain_fp32_iters": r2["iters_plain"],
            "speedup_vs_plain_fp32": r2["ms_plain"] / r2["ms_method"],
            "rc_measured": r2["rc_measured"], "kron_tiles_autotuned": r2["kron_tiles"], "engine": r2["engine"],
            "kernel_ms": r2["kernel_ms"],
            "whole_solve_phases_ms": r2["wg_phases"], "roofline": roofline(r2, "single"),
            "roofline_kernels": r2["roofline_kernels"],
            "max_gap": r2["max_gap_method"],
        }
        if not args.no_parity:
            line["single_signal"]["parity"] = block_parity(np, q, r2, oracle_reference(q, None, "single"), args.tol)
    if not args.no_faust:
        log("FAuST block (MEG shape 204 x 8193, 50 signals)")
        q = synth.config6(batch=50)
        r3 = solve_block(sl1, torch, np, q, args.tol, max(1, args.steps), args.warmup, "faust")
        line["faust_meg_shape"] = {
            "workload": "A (204 x 8193, FP32) = product of 4 sparse factors (204 x 204 x3 with 32 nonzeros per "
                        "column, 204 x 8193 with 64) + 0.01 G, unit columns; stages: FAuST approximations keeping "
                        "40, 48, 52, 56 entries per column of the last factor (FP32), then A; 50 signals, 8-sparse "
                        "x0, lambda = 0.1 lambda_max, tol 1e-6 (synthetic stand-in for the MEG operator)",
            "time_to_gap_ms": r3["ms_method"], "iters": r3["iters_method"],
            "plain_fp32_time_to_gap_ms": r3["ms_plain"], "plain_fp32_iters": r3["iters_plain"],
            "speedup_vs_plain_fp32": r3["ms_plain"] / r3["ms_method"],
            "rc_model": r3["rc_model"], "rc_measured": r3["rc_measured"], "engine": r3["engine"],
            "kernel_ms": r3["kernel_ms"], "max_gap": r3["max_gap_method"],
        }
        if not args.no_parity:
            line["faust_meg_shape"]["parity"] = block_parity(np, q, r3, oracle_reference(q, None, "faust"), args.tol)
    if not args.no_dense:
        log("dense precision block (N=2500, K=10000, 25 signals, FP8 -> BF16 -> FP32)")
        q = synth.config3(batch=25)
        r4 = solve_block(sl1, torch, np, q, args.tol, max(1, args.steps), args.warmup, "dense")
        line["dense_precision"] = {
            "workload": "dense A (2500 x 10000, i.i.d. N(0,1), unit columns, FP32 = exact); stages: FP8-E4M3 and "
                        "BF16 copies with per-column power-of-two scales (exact error bounds), then A; 25 signals "
                        "y = A x0 / ||A x0|| with 50-sparse x0, lambda = 0.5 lambda_max, tol 1e-6",
            "time_to_gap_ms": r4["ms_method"], "iters": r4["iters_method"],
            "iters_per_s": r4["iters_method"] / (r4["ms_method"] * 1e-3),
            "plain_fp32_time_to_gap_ms": r4["ms_plain"], "plain_fp32_iters": r4["iters_plain"],
            "speedup_vs_plain_fp32": r4["ms_plain"] / r4["ms_method"],
            "rc_model": r4["rc_model"], "rc_measured": r4["rc_measured"], "engine": r4["engine"],
            "kernel_ms": r4["kernel_ms"], "whole_solve_phases_ms": r4["wg_phases"],
            "roofline": roofline(r4, "dense"), "roofline_kernels": r4["roofline_kernels"], "max_gap": r4["max_gap_method"],
        }
        if not args.no_parity:
            line["dense_precision"]["parity"] = block_parity(np, q, r4, oracle_reference(q, [0, 12, 24], "dense"),
                                                             args.tol)
    if "grad" in blocks:
        log("gradient block (implicit adjoint, N=4096, K=16384, R=8, 64 signals)")
        line["gradient"] = grad_block(sl1, torch, np, args)
    print(json.dumps(line))


def grad_block(sl1, torch, np, args):
    """The implicit adjoint (sl1_grad) after the differentiation workload's solve: 64
    signals, 40-sparse x0, lambda = 0.5 lambda_max, loss ||x - x0||^2 (dL/dx = 2 (x - x0)).
    Work per signal with support s: the Gram matrix N s (s + 1) flops, Cholesky s^3 / 3,
    two substitutions 2 s^2, dL/dy = A_S w 2 N s (FP64, vector units).  Error: against the
    closed form on the FP64 oracle's support for two signals."""
    import synth
    q = synth.config5(batch=64)
    st, Y, lam, an = upload(sl1, torch, q)
    L = [s.L for s in q.stages]
    rc = sl1.measure_rc(st, batch=q.batch)
    out = sl1.solve(st, L, rc, an, Y, lam, tol=1e-10)
    x = out["x"]
    dx = 2.0 * (x - torch.from_numpy(q.X0).to(x.device))
    exact = st[-1]
    steps = max(3, args.steps)
    ms, res = timed(torch, lambda: sl1.grad(exact, x, Y, lam, dx), steps, 1)
    dy, dlam = res
    sup = (x != 0).sum(dim=1).cpu().numpy().astype(np.int64)
    N = q.N
    flops = float(np.sum(N * sup * (sup + 1) + sup ** 3 / 3.0 + 2.0 * sup ** 2 + 2.0 * N * sup))
    ach = flops / (ms * 1e-3) / 1e12
    entry = {"workload": "N=4096 (64x64), K=16384 (128x128), A = sum_{r<=8} B_r kron C_r + 0.01 G (FP32), 64 "
                         "signals, 40-sparse x0, lambda = 0.5 lambda_max; loss ||x - x0||^2 after the solve to gap "
                         "1e-10; sl1_grad on the exact dictionary",
             "ms_per_call": ms, "support": {"min": int(sup.min()), "median": float(np.median(sup)),
                                             "max": int(sup.max())},
             "fp64_flops_per_call": flops,
             "roofline": {"bound": "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": ach / FP64_PEAK_TFLOPS}}
    if not args.no_parity:
        import oracle.lasso as ol
        dyn, dln = dy.cpu().numpy().astype(np.float64), dlam.cpu().numpy()
        worst = 0.0
        for b in (0, 1):
            sol = ol.solve(q.A, q.Y[b], float(q.lam[b]), L=q.stages[-1].L, tol=1e-15)
            S = np.flatnonzero(sol["x"])
            AS = q.A[:, S]
            w = np.linalg.solve(AS.T @ AS, 2.0 * (sol["x"] - q.X0[b])[S])
            g_ref, l_ref = AS @ w, -np.sign(sol["x"][S]) @ w
            worst = max(worst, float(np.linalg.norm(dyn[b] - g_ref) / np.linalg.norm(g_ref)),
                        abs(float(dln[b]) - l_ref) / max(abs(l_ref), 1e-300))
        entry["parity"] = {"signals": [0, 1], "max_rel_error_vs_oracle_closed_form": worst}
    log(f"gradient: {ms:.3f} ms per call, supports {int(sup.min())}-{int(sup.max())}, {ach:.3f} TFLOP/s FP64")
    return entry


if __name__ == "__main__":
    main()
