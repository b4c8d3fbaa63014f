"""GPU (gfx950) parity of the band, assembly and PCG against the FP64 oracle.

Band keys, TSDF, weights, neighbour table, Lambda, b and diag(Q) are compared
bit for bit; the posterior mean within the relative-L2 tolerances 1e-6 (FP64)
and 1e-4 (mixed precision).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from tests import gpu_common as gc  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    import paper_2602_19697_amd as bf
    c = bf.Context(gc.DEV)
    yield c
    c.close()


@pytest.mark.parametrize("name", ["tiny", "sphere64"])
def test_band_bitexact(ctx, name):
    wl = gc.workload(name)
    ref = gc.oracle_ref(name)
    band, sys_, _, _ = gc.gpu_system(ctx, wl, keep_dense=True)
    a = band.arrays()
    print(f"[{name}] N gpu={band.n} oracle={len(ref['keys'])}", flush=True)
    assert band.n == len(ref["keys"])
    assert np.array_equal(a["keys"].cpu().numpy(), ref["keys"])
    assert np.array_equal(a["tsdf"].cpu().numpy(), ref["tsdf"])
    assert np.array_equal(a["w"].cpu().numpy(), ref["w"])
    assert np.array_equal(a["nbr"].cpu().numpy(), ref["nbr"])
    assert np.array_equal(a["deg"].cpu().numpy(), ref["deg"])
    # dense coarse TSDF over the whole grid, bit for bit
    pos = gc.morton_to_linear(wl.G, a["dense_side"])
    dt = a["dense_tsdf"].cpu().numpy()[pos]
    dw = a["dense_w"].cpu().numpy()[pos]
    assert np.array_equal(dw, ref["w_dense"].ravel())
    assert np.array_equal(dt, ref["tsdf_dense"].ravel())
    sys_.free()
    band.free()


@pytest.mark.parametrize("name,seed", [("tiny", 0), ("sphere64", 0), ("union128", 3)])
def test_band_screening_exact(ctx, name, seed):
    """The screened coarse TSDF (cells that provably hold no band voxel are not
    fused) yields the oracle's band bit for bit, and skips most of the work."""
    wl = gc.workload(name, seed)
    ref = gc.oracle_ref(name, seed)
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    a = band.arrays()
    full = wl.G ** 3 * wl.T
    cell_views = (-(-wl.G // 4)) ** 3 * wl.T
    print(f"[{name}] screened: {a['tsdf_voxel_views']} of {full} voxel-views fused "
          f"({100.0 * a['tsdf_voxel_views'] / full:.1f}%); {a['tsdf_box_tests']} screening tests "
          f"for {cell_views} cell-views", flush=True)
    for key in ("keys", "tsdf", "w", "nbr", "deg"):
        assert np.array_equal(a[key].cpu().numpy(), ref[key]), key
    assert 0 < a["tsdf_voxel_views"] < full
    # the tile-level tests spare most cell tests
    assert 0 < a["tsdf_box_tests"] < cell_views
    assert 0 < a["tsdf_tile_tests"] <= a["tsdf_box_tests"]
    sys_.free()
    band.free()
    # with the dense grid kept, nothing is screened
    band2, sys2, _, _ = gc.gpu_system(ctx, wl, keep_dense=True)
    assert band2.arrays()["tsdf_voxel_views"] == full
    assert band2.arrays()["tsdf_box_tests"] == 0 and band2.arrays()["tsdf_tile_tests"] == 0
    sys2.free()
    band2.free()


@pytest.mark.parametrize("W,H", [(47, 35), (130, 97), (100, 75)])
def test_band_odd_depth_sizes(ctx, W, H):
    """Depth images whose width is not a multiple of 4 (the pyramid's per-pixel
    loads) or is one (its 16-byte row loads), with sides that are not multiples
    of its 32-pixel tiles (partial tiles on the right and bottom edges; at 130 x 97
    levels above the tile are built too): the screened band, TSDF, weights and
    neighbours equal the oracle's bit for bit."""
    import oracle as O
    from synth.configs import union_workload
    wl = union_workload(f"union64_{W}x{H}", 64, 0.016, 12, 2, 2, width=W, height=H, f=525.0 * W / 640.0)
    g, cm = O.grid_of(wl), O.cam(wl.cam)
    td, wd = O.tsdf_dense(g, cm, wl.depth, wl.poses)
    keys, bt, bw = O.band(g, td, wd)
    nbr, deg = O.neighbours(wl.G, keys)
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    a = band.arrays()
    print(f"[{W}x{H}] band {a['keys'].shape[0]} voxels, {a['tsdf_voxel_views']} voxel-views fused", flush=True)
    assert len(keys) > 0
    for key, want in (("keys", keys), ("tsdf", bt), ("w", bw), ("nbr", nbr), ("deg", deg)):
        assert np.array_equal(a[key].cpu().numpy(), want), key
    assert 0 < a["tsdf_voxel_views"] < wl.G ** 3 * wl.T
    sys_.free()
    band.free()


@pytest.mark.parametrize("name", ["tiny", "sphere64"])
def test_assembly_bitexact(ctx, name):
    wl = gc.workload(name)
    ref = gc.oracle_ref(name)
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    s = sys_.arrays()
    assert np.array_equal(s["Lambda"].cpu().numpy(), ref["Lambda"])
    assert np.array_equal(s["b"].cpu().numpy(), ref["b"])
    assert np.array_equal(s["rhs"].cpu().numpy(), ref["rhs"])
    assert np.array_equal(s["diag"].cpu().numpy(), ref["diag"])
    assert np.array_equal(s["acc"].cpu().numpy(), ref["acc"])
    sys_.free()
    band.free()


@pytest.mark.parametrize("name", ["sphere64", "union128"])
def test_assembly_view_masks_exact(ctx, name):
    """The assembly of a screened band skips the views its screen proved give a
    voxel's cell no observation, but only for the depth maps and poses the band
    was built from: the same arrays (masks used) and a copy of them (masks not
    used: other device arrays) give the same bits, equal to the oracle's."""
    import paper_2602_19697_amd as bf
    wl = gc.workload(name)
    ref = gc.oracle_ref(name)
    band, sys_, depth, poses = gc.gpu_system(ctx, wl)
    other = ctx.bf_assemble(band, wl.cam, depth.clone(), poses.clone(), bf.noise_struct(*wl.noise), wl.lam, wl.eps)
    a, b = sys_.arrays(), other.arrays()
    for k in ("Lambda", "b", "rhs", "diag", "acc"):
        assert torch.equal(a[k], b[k]), k
    assert np.array_equal(a["Lambda"].cpu().numpy(), ref["Lambda"])
    assert np.array_equal(a["acc"].cpu().numpy(), ref["acc"])
    # the views gone through: every one without the masks; with them fewer,
    # but at least every view that gave a voxel an observation
    n, T = band.n, wl.T
    masked, plain = sys_.assembly_views(), other.assembly_views()
    observed = int(round(float(a["acc"][:, 0].sum().item())))
    print(f"[{name}] assembly: {masked} of {plain} voxel-views gone through, {observed} observed", flush=True)
    assert plain == n * T
    assert observed <= masked < plain
    other.free()
    sys_.free()
    band.free()


def test_assembly_anchor_bitexact(ctx):
    import oracle as O
    wl = gc.workload("sphere64")
    ref = gc.oracle_ref("sphere64")
    band, sys_, _, _ = gc.gpu_system(ctx, wl, lam_b=250.0)
    s = sys_.arrays()
    diag = O.precision_diag(ref["Lambda"], ref["deg"], wl.lam, wl.eps, 250.0)
    rhs = O.anchor_rhs(ref["b"], ref["deg"], ref["tsdf"], 250.0)
    assert np.array_equal(s["diag"].cpu().numpy(), diag)
    assert np.array_equal(s["rhs"].cpu().numpy(), rhs)
    sys_.free()
    band.free()


def test_apply_Q_matches_oracle(ctx):
    import oracle as O
    wl = gc.workload("sphere64")
    ref = gc.oracle_ref("sphere64")
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    p = np.random.default_rng(0).standard_normal(band.n)
    q = ctx.bf_apply_Q(sys_, torch.from_numpy(p).to(gc.DEV)).cpu().numpy()
    q_ref = O.apply_Q(ref["nbr"], ref["diag"], wl.lam, p)
    assert gc.rel_l2(q, q_ref) <= 1e-15
    sys_.free()
    band.free()


@pytest.mark.parametrize("name,lam,tol", [("tiny", 10.0, 1e-8), ("sphere64", 10.0, 1e-8),
                                          ("sphere64", 1e5, 1e-8), ("sphere64", 1e6, 1e-10)])
def test_pcg_fp64(ctx, name, lam, tol):
    import oracle as O
    import paper_2602_19697_amd as bf
    wl = gc.workload(name)
    ref = gc.oracle_ref(name)
    band, sys_, _, _ = gc.gpu_system(ctx, wl, lam=lam)
    diag = O.precision_diag(ref["Lambda"], ref["deg"], lam, wl.eps)
    mu_ref, rep_ref = O.pcg(ref["nbr"], diag, lam, ref["rhs"], tol)
    mu, rep = ctx.bf_pcg_solve(sys_, tol, precision=bf.L.BF_PREC_FP64)
    err = gc.rel_l2(mu.cpu().numpy(), mu_ref)
    print(f"[{name} lam={lam}] iters gpu={rep['iters']} oracle={rep_ref['iters']} rel_res={rep['rel_res']:.2e} err={err:.2e}")
    assert rep["status"] == 0 and rep["rel_res"] <= tol
    assert err <= 1e-6
    # the same run twice is bitwise identical (deterministic reductions)
    mu2, _ = ctx.bf_pcg_solve(sys_, tol, precision=bf.L.BF_PREC_FP64)
    assert torch.equal(mu, mu2)
    sys_.free()
    band.free()


@pytest.mark.parametrize("name,lam,tol", [("sphere64", 10.0, 1e-6), ("sphere64", 1e5, 1e-6),
                                          ("sphere64", 1e6, 1e-8)])
def test_pcg_mixed(ctx, name, lam, tol):
    import oracle as O
    import paper_2602_19697_amd as bf
    wl = gc.workload(name)
    ref = gc.oracle_ref(name)
    band, sys_, _, _ = gc.gpu_system(ctx, wl, lam=lam)
    diag = O.precision_diag(ref["Lambda"], ref["deg"], lam, wl.eps)
    mu_ref, _ = O.pcg(ref["nbr"], diag, lam, ref["rhs"], 1e-12)
    mu, rep = ctx.bf_pcg_solve(sys_, tol, precision=bf.L.BF_PREC_MIXED)
    err = gc.rel_l2(mu.cpu().numpy(), mu_ref)
    print(f"[mixed {name} lam={lam}] iters={rep['iters']} refinements={rep['refinements']} rel_res={rep['rel_res']:.2e} err={err:.2e}")
    assert rep["status"] == 0 and rep["rel_res"] <= tol
    assert err <= 1e-4
    sys_.free()
    band.free()


def test_pcg_warm_start_and_zero_rhs(ctx):
    import paper_2602_19697_amd as bf
    wl = gc.workload("tiny")
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    mu, rep = ctx.bf_pcg_solve(sys_, 1e-10)
    mu2, rep2 = ctx.bf_pcg_solve(sys_, 1e-8, x0=mu)
    assert rep2["iters"] == 0 and torch.equal(mu, mu2)
    zero = torch.zeros(band.n, dtype=torch.float64, device=gc.DEV)
    x, rep3 = ctx.bf_pcg_solve(sys_, 1e-8, rhs=zero, x0=mu)
    assert rep3["iters"] == 0 and torch.count_nonzero(x).item() == 0
    _, rep4 = ctx.bf_pcg_solve(sys_, 1e-14, max_iter=1, allow_fail=True)
    assert rep4["status"] == bf.L.BF_ERR_NOT_CONVERGED and rep4["iters"] == 1
    sys_.free()
    band.free()


def test_invalid_depth_rejected(ctx):
    import paper_2602_19697_amd as bf
    wl = gc.workload("tiny")
    depth, poses = gc.to_dev(wl)
    depth[0, 3, 3] = float("nan")
    g = bf.grid_struct(wl.G, wl.h, wl.origin, wl.tau, wl.band)
    with pytest.raises(bf.BFError) as e:
        ctx.bf_build_band(g, wl.cam, depth, poses)
    assert e.value.status == bf.L.BF_ERR_INVALID_ARG
    depth[0, 3, 3] = -1.0
    with pytest.raises(bf.BFError):
        ctx.bf_build_band(g, wl.cam, depth, poses)


def test_empty_band(ctx):
    import paper_2602_19697_amd as bf
    wl = gc.workload("tiny")
    depth, poses = gc.to_dev(wl)
    depth.zero_()
    g = bf.grid_struct(wl.G, wl.h, wl.origin, wl.tau, wl.band)
    band = ctx.bf_build_band(g, wl.cam, depth, poses)
    assert band.n == 0
    sys_ = ctx.bf_assemble(band, wl.cam, depth, poses, bf.noise_struct(), wl.lam, wl.eps)
    x, rep = ctx.bf_pcg_solve(sys_, 1e-8)
    assert x.numel() == 0 and rep["iters"] == 0
    sys_.free()
    band.free()


def test_band_many_views_exact(ctx):
    """264 views: the block-tile screen keeps per-view masks for the first 256 views
    only; the views past them are tested cell by cell and always fused.  Band, TSDF,
    weights, neighbours and the assembled Lambda and b match the oracle bit for bit."""
    import oracle as O
    from synth.configs import union_workload
    wl = union_workload("union64_264v", 64, 0.016, 264, 1, 1, width=48, height=36, f=39.375)
    assert wl.T > 256
    g, cm = O.grid_of(wl), O.cam(wl.cam)
    td, wd = O.tsdf_dense(g, cm, wl.depth, wl.poses)
    keys, bt, bw = O.band(g, td, wd)
    nbr, deg = O.neighbours(wl.G, keys)
    Lam, b = O.assemble(g, cm, wl.depth, wl.poses, keys, noise=wl.noise)[:2]
    band, sys_, _, _ = gc.gpu_system(ctx, wl)
    a = band.arrays()
    cells = (-(-wl.G // 4)) ** 3
    print(f"[{wl.T} views] band {a['keys'].shape[0]} voxels, {a['tsdf_voxel_views']} voxel-views fused, "
          f"{a['tsdf_box_tests']} screening tests", flush=True)
    assert len(keys) > 0
    for key, want in (("keys", keys), ("tsdf", bt), ("w", bw), ("nbr", nbr), ("deg", deg)):
        assert np.array_equal(a[key].cpu().numpy(), want), key
    s = sys_.arrays()
    assert np.array_equal(s["Lambda"].cpu().numpy(), Lam)
    assert np.array_equal(s["b"].cpu().numpy(), b)
    # every cell is tested against each view past the masked ones
    assert a["tsdf_box_tests"] >= cells * (wl.T - 256)
    assert 0 < a["tsdf_voxel_views"] < wl.G ** 3 * wl.T
    sys_.free()
    band.free()
