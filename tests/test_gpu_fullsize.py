"""Full-size parity on the GPU, on outputs the FP64 oracle can compute one by one.

* 1 slice of 1024^2, 4096 positions (the whole single-slice scan): every
  intensity, every per-position loss and the whole gradient against the oracle.
* 8 slices of 1024^2, 4096 positions: the autograd.Function gradient (fused
  adjoint kernel) against central finite differences (h = 1e-3) of the FP64
  oracle loss on 64 random voxels, and against the oracle gradient there.
* 16 slices of 2048^2, 16632 positions, 4x4 tiles with a 64 px halo.  The
  launch configuration the benchmark times -- every tile's gradient in one
  persistent launch (AllTilesWalk, ptycho_tiles_grad), then the stitch -- and,
  as a second case, the resident walk with one launch per tile on two lanes
  (ResidentTileWalk, ptycho_tile_grad).  Each is checked against the oracle on
  sampled per-position losses and on a gradient block across the corner of
  four tiles, and against the undecomposed GPU gradient; Parseval holds for
  every pattern and sampled patterns match the oracle.
"""
import numpy as np
import pytest

import oracle
import ptycho_synth as ps
from gpu_helpers import rel_l2, say
from oracle_pool import OraclePool

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def covered_mask(pos, W, M):
    cover = np.zeros((W, W), dtype=bool)
    for y0, x0 in pos:
        cover[y0:y0 + M, x0:x0 + M] = True
    return cover


def test_autograd_gradient_vs_finite_differences_8_slices(torch_cuda):
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.autograd import amplitude_loss
    spec = ps.workload("ms8-1024-m128")
    say("autograd gradient vs FP64 central differences: 8 x 1024^2, 4096 positions, 64 voxels")
    d = ps.build_inputs(spec, workers=8)
    H = oracle.fresnel_propagator(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    pos = d["pos"]
    with OraclePool(d["obj_true"], d["probe"], H) as pool:
        meas = ps.poisson_counts(pool.intensities(pos), d["noise_seed"])
    # 64 voxels, uniform among pixels under at least one window
    rng = np.random.default_rng(d["fd_seed"])
    cover = covered_mask(pos, spec.W, spec.M)
    cy, cx = np.nonzero(cover)
    pick = rng.choice(len(cy), size=64, replace=False)
    voxels = np.stack([rng.integers(0, spec.S, 64), cy[pick], cx[pick]], axis=1)
    covering = [np.nonzero((pos[:, 0] <= y) & (y < pos[:, 0] + spec.M) & (pos[:, 1] <= x) &
                           (x < pos[:, 1] + spec.M))[0] for _, y, x in voxels]
    dev = "cuda:0"
    ctx = pt.Context(spec.M, spec.S, spec.wavelength_A, spec.dz_A, spec.pixel_A, len(pos))
    t = torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev, requires_grad=True)
    probe = torch.tensor(d["probe"], dtype=torch.complex64, device=dev)
    pos_d = torch.tensor(pos, dtype=torch.int32, device=dev)
    meas_d = torch.tensor(meas, dtype=torch.float32, device=dev)
    L = amplitude_loss(ctx, t, probe, pos_d, meas_d)
    L.backward()
    ctx.check()
    G = t.grad.detach().cpu().numpy()
    # the autograd gradient is the fused kernel's gradient; a second call agrees to rounding order
    _, G2 = pt.ptycho_loss_grad(ctx, t.detach(), probe, pos_d, meas_d)
    assert rel_l2(G, G2.cpu().numpy()) <= 1e-6
    # the chain-rule factor reaches the gradient
    t.grad = None
    (3.0 * amplitude_loss(ctx, t, probe, pos_d, meas_d)).backward()
    assert rel_l2(t.grad.detach().cpu().numpy(), 3.0 * G) <= 1e-6
    g_vox = G[voxels[:, 0], voxels[:, 1], voxels[:, 2]]
    need = np.unique(np.concatenate(covering))
    with OraclePool(d["obj_eval"], d["probe"], H, meas=meas) as pool:
        fd = pool.finite_differences(voxels, covering, pos, 1e-3)
        res = pool.loss_grad(need, pos)
    G_or = np.zeros(len(voxels), dtype=np.complex128)
    lookup = {int(i): r for i, r in zip(need, res)}
    for k, ((s, y, x), cov) in enumerate(zip(voxels, covering)):
        for i in cov:
            G_or[k] += lookup[int(i)][1][s, y - pos[i][0], x - pos[i][1]]
    e_fd = rel_l2(g_vox, fd)
    e_or = rel_l2(g_vox, G_or)
    e_pin = rel_l2(G_or, fd)
    say(f"  GPU vs FD {e_fd:.2e}, GPU vs oracle {e_or:.2e}, oracle vs FD {e_pin:.2e}")
    assert e_pin <= 1e-6
    assert e_fd <= 1e-4
    assert e_or <= 1e-4
    L_ref = sum(lookup[int(i)][0] for i in need if True)
    if len(need) == len(pos):
        assert abs(float(L.item()) - L_ref) <= 1e-5 * L_ref


def test_single_slice_1024_full_scan_against_the_oracle(torch_cuda):
    """Single-slice 1024^2 phase object, 128-windows, the whole 64 x 64 scan (4096 positions, step 14) with
    Poisson counts at a dose of 1e5: all intensities (1e-5), all per-position losses and the total loss
    (1e-5) and the whole gradient (1e-4) against the FP64 oracle."""
    import torch
    import paper_2205_06327_amd as pt
    spec = ps.workload("2d-1024-m128")
    say("1 x 1024^2, 4096 positions: oracle intensities, losses and gradient of the whole scan")
    d = ps.build_inputs(spec)
    H = oracle.fresnel_propagator(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    I_true = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    meas = ps.poisson_counts(I_true, d["noise_seed"])
    L_ref, lpp_ref, G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], meas, H)
    dev = "cuda:0"
    n = len(d["pos"])
    ctx = pt.Context(spec.M, spec.S, spec.wavelength_A, spec.dz_A, spec.pixel_A, n)
    probe = torch.tensor(d["probe"], dtype=torch.complex64, device=dev)
    pos = torch.tensor(d["pos"], dtype=torch.int32, device=dev)
    I = pt.ptycho_forward(ctx, torch.tensor(d["obj_true"], dtype=torch.complex64, device=dev), probe, pos)
    lpp = torch.zeros(n, dtype=torch.float64, device=dev)
    loss, grad = pt.ptycho_loss_grad(ctx, torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev), probe, pos,
                                     torch.tensor(meas, dtype=torch.float32, device=dev), loss_per_pos=lpp)
    assert ctx.check() == 0
    torch.cuda.synchronize()
    e_i = rel_l2(I.cpu().numpy(), I_true)
    e_l = abs(float(loss.item()) - L_ref) / L_ref
    e_g = rel_l2(grad.cpu().numpy(), G_ref)
    say(f"  intensities {e_i:.2e}, loss {e_l:.2e}, gradient {e_g:.2e}")
    assert e_i <= 1e-5 and e_l <= 1e-5 and e_g <= 1e-4
    np.testing.assert_allclose(lpp.cpu().numpy(), lpp_ref, rtol=1e-5)


@pytest.fixture(scope="module")
def fullsize(torch_cuda):
    """Inputs of the 16 x 2048^2 workload, oracle values on a sample, and the undecomposed GPU gradient."""
    import torch
    import paper_2205_06327_amd as pt
    spec = ps.workload("ms16-2048-m128-tiles4x4")
    say("16 x 2048^2, 16632 positions, 4x4 tiles: inputs, oracle sample, undecomposed gradient")
    d = ps.build_inputs(spec, workers=8)
    H = oracle.fresnel_propagator(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    pos = d["pos"]
    M, S, W = spec.M, spec.S, spec.W
    # gradient block across the corner of four tiles, all slices
    by, bx, bs = 504, 504, 16
    cov_blk = np.nonzero((pos[:, 0] < by + bs) & (pos[:, 0] + M > by) & (pos[:, 1] < bx + bs) &
                         (pos[:, 1] + M > bx))[0]
    sample = np.linspace(0, len(pos) - 1, 48).round().astype(int)
    exact = np.unique(np.concatenate([cov_blk, sample]))
    # measurements: oracle Poisson counts where the oracle checks; elsewhere Poisson counts of the
    # flat-object closed form D * aperture / N_A (a plain definition, no model evaluation)
    q = np.fft.fftfreq(M) * M
    A = (q[:, None] ** 2 + q[None, :] ** 2) <= spec.R ** 2
    meas = np.zeros((len(pos), M, M), dtype=np.float32)
    meas[:, A] = ps.poisson_counts(np.full((len(pos), int(A.sum())), spec.dose / A.sum()), d["noise_seed"])
    with OraclePool(d["obj_true"], d["probe"], H) as pool:
        I_exact = pool.intensities(pos[exact])
    meas[exact] = ps.poisson_counts(I_exact, np.random.SeedSequence(7))
    dev = "cuda:0"
    ctx = pt.Context(M, S, spec.wavelength_A, spec.dz_A, spec.pixel_A, len(pos))
    probe = torch.tensor(d["probe"], dtype=torch.complex64, device=dev)
    pos_d = torch.tensor(pos, dtype=torch.int32, device=dev)
    # Parseval: every pattern of the pure-phase truth sums to the dose
    obj_t = torch.tensor(d["obj_true"], dtype=torch.complex64, device=dev)
    I_t = pt.ptycho_forward(ctx, obj_t, probe, pos_d)
    sums = I_t.sum(dim=(1, 2), dtype=torch.float64).cpu().numpy()
    assert np.max(np.abs(sums / spec.dose - 1)) <= 2e-5
    del obj_t, I_t
    obj = torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev)
    meas_d = torch.tensor(meas, dtype=torch.float32, device=dev)
    I = pt.ptycho_forward(ctx, obj, probe, pos_d[torch.tensor(sample, device=dev)].contiguous())
    with OraclePool(d["obj_eval"], d["probe"], H, meas=meas) as pool:
        I_ref = pool.intensities(pos[sample])
        res = pool.loss_grad(exact, pos)
    assert rel_l2(I.cpu().numpy(), I_ref) <= 1e-5
    lookup = {int(i): r for i, r in zip(exact, res)}
    blk = np.zeros((S, bs, bs), dtype=np.complex128)
    for i in cov_blk:
        y0, x0 = pos[i]
        patch = lookup[int(i)][1]
        ys, xs = max(by, y0), max(bx, x0)
        ye, xe = min(by + bs, y0 + M), min(bx + bs, x0 + M)
        blk[:, ys - by:ye - by, xs - bx:xe - bx] += patch[:, ys - y0:ye - y0, xs - x0:xe - x0]
    gfull = torch.empty_like(obj)
    lfull, _ = pt.ptycho_loss_grad(ctx, obj, probe, pos_d, meas_d, grad=gfull)
    ctx.check()
    return {"spec": spec, "pos": pos, "ctx": ctx, "obj": obj, "probe": probe, "meas": meas_d, "gfull": gfull,
            "lfull": float(lfull.item()), "sample": sample, "ref_loss": np.array([lookup[int(i)][0] for i in sample]),
            "blk": blk, "block": (by, bx, bs), "cov_blk": cov_blk, "lookup": lookup}


def _check_decomposed(fs, grad, loss_total, lpp_sorted, order, what):
    import torch
    by, bx, bs = fs["block"]
    dec = float(torch.linalg.vector_norm(grad - fs["gfull"]) / torch.linalg.vector_norm(fs["gfull"]))
    say(f"  {what}: decomposed vs undecomposed {dec:.2e}")
    assert dec <= 1e-6
    assert abs(loss_total - fs["lfull"]) <= 1e-9 * fs["lfull"]
    # per-position losses (tile order -> scan order) against the oracle on the sample
    lpp = np.empty(len(order))
    lpp[order] = lpp_sorted.cpu().numpy()
    np.testing.assert_allclose(lpp[fs["sample"]], fs["ref_loss"], rtol=1e-5)
    got = grad[:, by:by + bs, bx:bx + bs].cpu().numpy()
    e = rel_l2(got, fs["blk"])
    say(f"  {what}: gradient block rel L2 {e:.2e} over {len(fs['cov_blk'])} positions")
    assert e <= 1e-4


def test_tiled_16_slices_2048_all_tiles_launch(fullsize):
    """The benchmark's launch configuration: every tile's gradient in one persistent launch
    (ptycho_tiles_grad into per-tile buffers on the extended boxes), then the 16 stitches."""
    import torch
    from paper_2205_06327_amd.tilewalk import AllTilesWalk, TileWalk
    fs = fullsize
    spec, ctx = fs["spec"], fs["ctx"]
    plan = TileWalk(fs["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    walk = AllTilesWalk(ctx, plan)
    order = torch.tensor(plan.order, device="cuda:0")
    meas_sorted = fs["meas"][order].contiguous()
    grad = torch.empty_like(fs["obj"])
    lpp = torch.zeros(plan.n, dtype=torch.float64, device="cuda:0")
    loss = walk.step(fs["obj"], fs["probe"], meas_sorted, grad, loss_per_pos=lpp)
    assert walk.check() == 0
    _check_decomposed(fs, grad, float(loss.item()), lpp, plan.order, "all tiles in one launch")
    # each of the four tiles around the corner holds its own positions' gradient on the block
    by, bx, bs = fs["block"]
    M, S, pos = spec.M, spec.S, fs["pos"]
    owner = oracle.bin_positions(pos, spec.W, spec.W, M, *spec.tiles)
    seen = 0
    for k in sorted({int(owner[i]) for i in fs["cov_blk"]}):
        ref = np.zeros((S, bs, bs), dtype=np.complex128)
        for i in fs["cov_blk"]:
            if owner[i] != k:
                continue
            y0, x0 = pos[i]
            patch = fs["lookup"][int(i)][1]
            ys, xs = max(by, y0), max(bx, x0)
            ye, xe = min(by + bs, y0 + M), min(bx + bs, x0 + M)
            ref[:, ys - by:ye - by, xs - bx:xe - bx] += patch[:, ys - y0:ye - y0, xs - x0:xe - x0]
        ey0, ex0, _, _ = plan.plans[k].box
        got = walk.bufs[k][:, by - ey0:by - ey0 + bs, bx - ex0:bx - ex0 + bs].cpu().numpy()
        e = rel_l2(got, ref)
        say(f"  tile {k} buffer on the corner block: rel L2 {e:.2e}")
        assert e <= 1e-4
        seen += 1
    assert seen == 4


def test_tiled_16_slices_2048_resident_walk(fullsize):
    """The resident walk: one launch per tile (ptycho_tile_grad) on two alternating lanes, each tile's
    gradient stitched into the global gradient in tile order."""
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.tilewalk import ResidentTileWalk, TileWalk
    fs = fullsize
    spec, ctx = fs["spec"], fs["ctx"]
    plan = TileWalk(fs["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    walk = ResidentTileWalk(ctx, plan)
    order = torch.tensor(plan.order, device="cuda:0")
    meas_sorted = fs["meas"][order].contiguous()
    grad = torch.empty_like(fs["obj"])
    tl = walk.step(fs["obj"], fs["probe"], meas_sorted, grad)
    assert walk.check() == 0
    # per-position losses of this walk's kernels: one tile call per tile with loss_per_pos
    lpp = torch.zeros(plan.n, dtype=torch.float64, device="cuda:0")
    scratch = torch.empty((spec.S, *plan.max_box), dtype=torch.complex64, device="cuda:0")
    for p in plan.plans:
        if p.hi == p.lo:
            continue
        ey0, ex0, eh, ew = p.box
        tg = scratch.view(-1)[: spec.S * eh * ew].view(spec.S, eh, ew)
        pt.ptycho_tile_grad(ctx, fs["obj"][:, ey0:ey0 + eh, ex0:ex0 + ew], p.box, p.tile, plan.halo, plan.H, plan.W,
                            fs["probe"], walk.pos[p.lo:p.hi], meas_sorted[p.lo:p.hi], tile_grad=tg,
                            loss_per_pos=lpp[p.lo:p.hi])
    ctx.check()
    _check_decomposed(fs, grad, float(tl.sum().item()), lpp, plan.order, "resident walk, two lanes")
