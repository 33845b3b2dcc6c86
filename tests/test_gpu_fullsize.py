"""Full-size parity on the GPU, on outputs the FP64 oracle can compute one by one.

* 8 slices of 1024^2, 4096 positions: the autograd.Function gradient (fused
  adjoint kernel) against central finite differences (h = 1e-3) of the FP64
  oracle loss on 64 random voxels, and against the oracle gradient there.
* 16 slices of 2048^2, 16632 positions, 4x4 tiles with a 64 px halo, run in
  the launch configuration the benchmark times (resident tile walk): Parseval
  for every pattern, sampled patterns and per-position losses, a gradient
  block across the corner of four tiles, and decomposed vs undecomposed.
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


def test_tiled_16_slices_2048_sampled_parity(torch_cuda):
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.tilewalk import ResidentTileWalk, TileWalk
    spec = ps.workload("ms16-2048-m128-tiles4x4")
    say("16 x 2048^2, 16632 positions, 4x4 tiles: sampled parity in the benchmark's launch configuration")
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
    # tile walk exactly as benchmarked
    plan = TileWalk(pos, W, W, M, spec.tiles, spec.halo)
    walk = ResidentTileWalk(ctx, plan)
    order = torch.tensor(plan.order, device=dev)
    meas_sorted = meas_d[order].contiguous()
    grad = torch.empty_like(obj)
    tl = walk.step(obj, probe, meas_sorted, grad)
    walk.check()
    lpp = torch.zeros(len(pos), dtype=torch.float64, device=dev)
    gfull = torch.empty_like(obj)
    lfull, _ = pt.ptycho_loss_grad(ctx, obj, probe, pos_d, meas_d, grad=gfull, loss_per_pos=lpp)
    ctx.check()
    dec = float(torch.linalg.vector_norm(grad - gfull) / torch.linalg.vector_norm(gfull))
    say(f"  decomposed vs undecomposed {dec:.2e}")
    assert dec <= 1e-6
    assert abs(float(tl.sum()) - float(lfull.item())) <= 1e-9 * float(lfull.item())
    lookup = {int(i): r for i, r in zip(exact, res)}
    lpp_h = lpp.cpu().numpy()
    ref_l = np.array([lookup[int(i)][0] for i in sample])
    np.testing.assert_allclose(lpp_h[sample], ref_l, rtol=1e-5)
    blk = np.zeros((S, bs, bs), dtype=np.complex128)
    for i in cov_blk:
        y0, x0 = pos[i]
        patch = lookup[int(i)][1]
        ys, xs = max(by, y0), max(bx, x0)
        ye, xe = min(by + bs, y0 + M), min(bx + bs, x0 + M)
        blk[:, ys - by:ye - by, xs - bx:xe - bx] += patch[:, ys - y0:ye - y0, xs - x0:xe - x0]
    got = grad[:, by:by + bs, bx:bx + bs].cpu().numpy()
    e = rel_l2(got, blk)
    say(f"  gradient block rel L2 {e:.2e} over {len(cov_blk)} positions")
    assert e <= 1e-4
