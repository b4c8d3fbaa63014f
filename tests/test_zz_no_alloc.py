"""bf_pcg_solve_noalloc: the posterior-mean solve (eq. 11) with every temporary
in the library's static per-GPU scratch, for callers that cannot allocate.

It runs the kernels of bf_pcg_solve in the same order on the same data, so its
mean must equal that entry point's bit for bit (and match the FP64 oracle to
1e-6 in FP64, 1e-4 mixed).  The calls run back to back on one context, each
smaller than the one before, so a later call must not depend on what an
earlier one left in the shared scratch.  A system larger than the scratch is
rejected before anything is launched.
"""
import ctypes as C
import dataclasses

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tests import gpu_common as gc  # noqa: E402


def _check_pair(ctx, sys_, ref, wl, prec, tol, x0=None):
    import oracle as O
    import paper_2602_19697_amd as bf
    out = torch.empty(sys_.n, dtype=torch.float64, device=gc.DEV)
    want, rw = ctx.bf_pcg_solve(sys_, tol, precision=prec, x0=x0)
    got, rg = ctx.bf_pcg_solve_noalloc(sys_, tol, precision=prec, x0=x0, out=out)
    mu_ref, _ = O.pcg(ref["nbr"], ref["diag"], wl.lam, ref["rhs"], 1e-12)
    err = gc.rel_l2(got.cpu().numpy(), mu_ref)
    print(f"[{wl.name} prec={prec} x0={x0 is not None}] N={sys_.n} iters {rg['iters']} (allocating {rw['iters']}) "
          f"err vs oracle {err:.2e}", flush=True)
    assert got.data_ptr() == out.data_ptr()
    assert rg["status"] == 0 and rg["iters"] == rw["iters"] and rg["refinements"] == rw["refinements"]
    assert rg["rel_res"] == rw["rel_res"] and rg["used_warm_start"] == rw["used_warm_start"]
    assert torch.equal(got, want)
    assert err <= (1e-6 if prec == bf.L.BF_PREC_FP64 else 1e-4)


def test_noalloc_pcg_matches_allocating_solve():
    import oracle as O
    import paper_2602_19697_amd as bf
    from synth import make_workload
    FP64, MIXED = bf.L.BF_PREC_FP64, bf.L.BF_PREC_MIXED
    ctx = bf.Context(gc.DEV)
    assert ctx.bf_pcg_noalloc_max_n(FP64) > 1_000_000 and ctx.bf_pcg_noalloc_max_n(MIXED) > 2_000_000
    wl = make_workload("union512", device=gc.DEV)
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    n512 = sys_.n
    print(f"[union512] N={n512}; scratch holds FP64 {ctx.bf_pcg_noalloc_max_n(FP64)} / "
          f"mixed {ctx.bf_pcg_noalloc_max_n(MIXED)}", flush=True)
    # too large for the scratch in FP64: rejected with CAPACITY, x untouched
    assert ctx.bf_pcg_noalloc_max_n(FP64) < n512 <= ctx.bf_pcg_noalloc_max_n(MIXED)
    x = torch.full((n512,), 7.0, dtype=torch.float64, device=gc.DEV)
    st = ctx.lib.bf_pcg_solve_noalloc
    o = bf.L.bf_solve_opts()
    o.tol, o.max_iter, o.precision, o.use_x0, o.check_every = 1e-6, 100, FP64, 0, 0
    rep = bf.L.bf_solve_report()
    code = st(ctx.handle, sys_.handle, C.byref(o), None, C.c_void_p(x.data_ptr()), C.byref(rep))
    assert code == bf.L.BF_ERR_CAPACITY
    assert b"static scratch holds" in ctx.lib.bf_last_error(ctx.handle)
    assert bool((x == 7.0).all())
    # 1: union512 in mixed precision (fits); oracle mean of the full band
    ref = O.full_pipeline(wl)
    ref.pop("tsdf_dense")
    ref.pop("w_dense")
    _check_pair(ctx, sys_, ref, wl, MIXED, 1e-6)
    sys_.free()
    band.free()
    # 2: union256 (smaller), FP64 and mixed
    wl = make_workload("union256", device=gc.DEV)
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    ref = O.full_pipeline(wl)
    _check_pair(ctx, sys_, ref, wl, FP64, 1e-8)
    _check_pair(ctx, sys_, ref, wl, MIXED, 1e-6)
    sys_.free()
    band.free()
    # 3: sphere64 (smaller again), FP64, mixed, and from a warm start at a stiffer prior
    wl = gc.workload("sphere64")
    ref = gc.oracle_ref("sphere64")
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    _check_pair(ctx, sys_, ref, wl, FP64, 1e-8)
    _check_pair(ctx, sys_, ref, wl, MIXED, 1e-6)
    sys_.free()
    band.free()
    lam = 1e5
    band, sys_, _, _ = gc.gpu_system(ctx, wl, lam=lam)
    ref = dict(ref)
    ref["diag"] = O.precision_diag(ref["Lambda"], ref["deg"], lam, wl.eps)
    wl_l = dataclasses.replace(wl, lam=lam)
    x0 = torch.from_numpy(ref["rhs"] / ref["diag"]).to(gc.DEV)
    _check_pair(ctx, sys_, ref, wl_l, FP64, 1e-8, x0=x0)
    sys_.free()
    band.free()
    ctx.close()
