"""The allocation-free solve entry point (sl1_solve_noalloc) against sl1_solve, through
the C ABI: the same results on two calls in a row, the second with a smaller input
(the fixed device array keeps the previous call's contents), and the size limit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sl1():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1812_06635_amd as m
    m.load_library()
    return m


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _solve(sl1, p, ups, noalloc, **kw):
    import torch
    out = sl1.solve(ups, [s.L for s in p.stages], [s.rc_theory for s in p.stages], _t(p.atom_norm),
                    _t(p.Y, torch.float32), _t(p.lam), tol=1e-9, noalloc=noalloc, **kw)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def _same(a, b):
    assert a["status"] == b["status"] == 0
    for k in ("iters", "stage", "screened"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    scale = max(1.0, float(np.abs(b["x"]).max()))
    np.testing.assert_allclose(a["x"], b["x"], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(a["gap"], b["gap"], rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(a["gap_cert"], b["gap_cert"], rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("engine,rule", [("auto", "gap"), ("grid", "gap"), ("grid", "dst"), ("wg", "gap")])
def test_noalloc_matches_solve_on_two_calls(sl1, engine, rule):
    print(f"[gpu-case] noalloc vs solve engine={engine} rule={rule}", flush=True)
    big = synth.config4(batch=12, n=(16, 32))
    small = synth.config4(batch=12, n=(16, 32))
    small.Y, small.lam = small.Y[:5][::-1].copy(), small.lam[:5][::-1].copy()
    ups = [sl1.upload_stage(s) for s in big.stages]
    for p in (big, small):
        ref = _solve(sl1, p, ups, False, engine=engine, rule=rule)
        got = _solve(sl1, p, ups, True, engine=engine, rule=rule)
        _same(got, ref)


def test_noalloc_rejects_a_workspace_beyond_its_array(sl1):
    print("[gpu-case] noalloc size limit", flush=True)
    from paper_1812_06635_amd._lib import ELIMIT
    p = synth.config4(batch=200)
    ups = [sl1.upload_stage(s) for s in p.stages]
    import torch
    out = sl1.solve(ups, [s.L for s in p.stages], [s.rc_theory for s in p.stages], _t(p.atom_norm),
                    _t(p.Y, torch.float32), _t(p.lam), tol=1e-6, noalloc=True, check=False)
    assert out["status"] == ELIMIT
    # and a request that fits still runs after the refusal
    q = synth.config4(batch=4, n=(16, 32))
    ups = [sl1.upload_stage(s) for s in q.stages]
    _same(_solve(sl1, q, ups, True), _solve(sl1, q, ups, False))
