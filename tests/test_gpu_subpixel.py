"""Sub-pixel positions on the GPU: the probe translated by the Fourier shift
theorem (ptycho_shift_probes) and the forward / loss / gradient calls with one
probe per position (the stack entry points), against the FP64 oracle's
sub-pixel model (pinned on the CPU by cyclic rolls, a single-mode closed form,
composition and finite differences)."""
import math

import numpy as np
import pytest

import oracle
import ptycho_synth as ps
from gpu_helpers import context, rel_l2, say

pytestmark = pytest.mark.gpu

TOL_I, TOL_G, TOL_L = 1e-5, 1e-4, 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06327_amd as pt
    pt.lib()
    return torch


@pytest.mark.parametrize("base", ["2d-256-m64", "ms8-1024-m128"])
def test_shifted_probes_match_oracle(torch_cuda, base):
    """FP32 forward and inverse transform around a phase ramp: the bound is
    (2 log2(M^2) + 2) * 2^-24 relative L2 (rounding along both transforms and the ramp)."""
    import torch
    import paper_2205_06327_amd as pt
    spec = ps.workload(base)
    M = spec.M
    say(f"shifted probes, M={M}")
    probe = ps.make_probe(M, spec.R, spec.C, spec.dose)
    rng = np.random.default_rng(5)
    shifts = np.concatenate([[[0.0, 0.0], [0.5, 0.5], [0.999, 0.001], [3.0, -2.0], [-0.25, 7.75]],
                             rng.uniform(0.0, 1.0, (11, 2))]).astype(np.float32)
    ctx = context(spec, 16)
    out = pt.ptycho_shift_probes(ctx, torch.tensor(probe, dtype=torch.complex64, device="cuda:0"),
                                 torch.tensor(shifts, device="cuda:0"))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    bound = (2 * math.log2(M * M) + 2) * 2.0 ** -24
    for i, (dy, dx) in enumerate(shifts.astype(np.float64)):
        want = oracle.shift_probe(probe, dy, dx)
        assert rel_l2(got[i], want) <= bound, (i, dy, dx, rel_l2(got[i], want))
    np.testing.assert_allclose(got[3], np.roll(probe, (3, -2), axis=(0, 1)), rtol=0,
                               atol=bound * np.abs(probe).max() * M)


@pytest.mark.parametrize("base,S", [("ms8-1024-m128", 3), ("2d-256-m64", 2)])
def test_subpixel_positions_match_oracle(torch_cuda, base, S):
    import torch
    import paper_2205_06327_amd as pt
    spec = ps.with_overrides(ps.workload(base), W=2 * ps.workload(base).M + 40, S=S, ny=1, nx=1, noise=True)
    M = spec.M
    d = ps.build_inputs(spec)
    rng = np.random.default_rng(17 + S)
    n = 19
    posf = rng.uniform(0.0, spec.W - M - 1e-3, (n, 2))
    posf[0] = (0.0, 0.0)
    posf[1] = (spec.W - M - 0.5, 0.25)
    posf[2] = (10.0, 12.0)  # an integer position in the mix
    say(f"sub-pixel positions, M={M} S={S}, {n} positions")
    Hp = oracle.fresnel_propagator(M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    meas = ps.poisson_counts(oracle.forward_subpixel(d["obj_true"], d["probe"], posf, Hp), d["noise_seed"])
    corner, frac = pt.split_positions(posf)
    dev = "cuda:0"
    obj = torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev)
    probe = torch.tensor(d["probe"], dtype=torch.complex64, device=dev)
    pos_t = torch.tensor(corner, device=dev)
    ctx = context(spec, n)
    stack = pt.ptycho_shift_probes(ctx, probe, torch.tensor(frac, device=dev))
    I = pt.ptycho_forward(ctx, obj, stack, pos_t)
    lpp = torch.zeros(n, dtype=torch.float64, device=dev)
    loss, G = pt.ptycho_loss_grad(ctx, obj, stack, pos_t, torch.tensor(meas, device=dev), loss_per_pos=lpp)
    assert ctx.check() == 0
    torch.cuda.synchronize()
    L_ref, lpp_ref, G_ref = oracle.loss_and_gradient_subpixel(d["obj_eval"], d["probe"], posf, meas, Hp)
    assert rel_l2(I.cpu().numpy(), oracle.forward_subpixel(d["obj_eval"], d["probe"], posf, Hp)) <= TOL_I
    assert abs(float(loss.item()) - L_ref) <= TOL_L * L_ref
    assert rel_l2(G.cpu().numpy(), G_ref) <= TOL_G
    np.testing.assert_allclose(lpp.cpu().numpy(), lpp_ref, rtol=1e-4, atol=1e-6 * np.abs(lpp_ref).max())
    # zero fractions: the stack path equals the shared-probe path up to the shift kernel's rounding
    zero = torch.zeros((n, 2), dtype=torch.float32, device=dev)
    I0 = pt.ptycho_forward(ctx, obj, pt.ptycho_shift_probes(ctx, probe, zero), pos_t)
    I1 = pt.ptycho_forward(ctx, obj, probe, pos_t)
    assert rel_l2(I0.cpu().numpy(), I1.cpu().numpy()) <= 1e-5


def test_probe_stack_validation(torch_cuda):
    import ctypes
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd import _binding as B
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=128, ny=2, nx=2, step=16)
    say("probe stack: no probe gradient, stride checked on the host")
    d = ps.build_inputs(spec)
    dev = "cuda:0"
    ctx = context(spec, 4)
    obj = torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev)
    probe = torch.tensor(d["probe"], dtype=torch.complex64, device=dev)
    pos = torch.tensor(d["pos"], device=dev)
    stack = probe.expand(4, 64, 64).contiguous()
    meas = torch.ones((4, 64, 64), dtype=torch.float32, device=dev)
    with pytest.raises(ValueError):
        pt.ptycho_loss_grad(ctx, obj, stack, pos, meas, probe_grad=torch.zeros_like(probe))
    out = torch.empty((4, 64, 64), dtype=torch.float32, device=dev)
    S, H, W, ss, ld = B._obj_geometry(obj)
    rc = pt.lib().ptycho_forward_stack(ctx.handle, ctypes.c_void_p(obj.data_ptr()), H, W, ss, ld,
                                       ctypes.c_void_p(stack.data_ptr()), 100, ctypes.c_void_p(pos.data_ptr()), 4,
                                       ctypes.c_void_p(out.data_ptr()))
    assert B.ERRORS.get(rc) == "PTYCHO_E_SHAPE"
    I = pt.ptycho_forward(ctx, obj, stack, pos)
    assert rel_l2(I.cpu().numpy(), pt.ptycho_forward(ctx, obj, probe, pos).cpu().numpy()) == 0.0


def test_subpixel_autograd(torch_cuda):
    """amplitude_loss with one probe per position: the forward value from ptycho_loss_stack and the
    object gradient from ptycho_loss_grad_stack, scaled by the upstream factor."""
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.autograd import amplitude_loss
    spec = ps.with_overrides(ps.workload("ms8-1024-m128"), W=300, S=2, ny=1, nx=1, noise=True)
    d = ps.build_inputs(spec)
    rng = np.random.default_rng(23)
    posf = rng.uniform(0.0, spec.W - spec.M - 1e-3, (9, 2))
    say("sub-pixel positions through autograd, 9 positions")
    Hp = oracle.fresnel_propagator(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    meas = ps.poisson_counts(oracle.forward_subpixel(d["obj_true"], d["probe"], posf, Hp), d["noise_seed"])
    corner, frac = pt.split_positions(posf)
    dev = "cuda:0"
    ctx = context(spec, len(posf))
    stack = pt.ptycho_shift_probes(ctx, torch.tensor(d["probe"], dtype=torch.complex64, device=dev),
                                   torch.tensor(frac, device=dev))
    obj = torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev).requires_grad_(True)
    loss = amplitude_loss(ctx, obj, stack, torch.tensor(corner, device=dev), torch.tensor(meas, device=dev))
    (0.25 * loss).backward()
    assert ctx.check() == 0
    L_ref, _, G_ref = oracle.loss_and_gradient_subpixel(d["obj_eval"], d["probe"], posf, meas, Hp)
    assert abs(float(loss.item()) - L_ref) <= TOL_L * L_ref
    assert rel_l2(obj.grad.cpu().numpy(), 0.25 * G_ref) <= TOL_G


def test_subpixel_all_tiles_launch(torch_cuda):
    """The decomposition with sub-pixel positions: tiles binned by the integer window corners, one
    shifted probe per position in tile order, all tiles in one launch (ptycho_tiles_grad_stack),
    stitched, against the oracle's undecomposed sub-pixel gradient."""
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.tilewalk import AllTilesWalk, TileWalk
    spec = ps.with_overrides(ps.workload("ms16-2048-m128-tiles4x4"), W=384, S=3, ny=8, nx=8, step=28,
                             tiles=(2, 2), halo=64)
    d = ps.build_inputs(spec)
    rng = np.random.default_rng(29)
    posf = d["pos"].astype(np.float64) + rng.uniform(0.0, 1.0, d["pos"].shape)
    posf = np.minimum(posf, spec.W - spec.M)  # windows stay inside the object
    say(f"sub-pixel positions through the all-tiles launch, {len(posf)} positions, 2x2 tiles")
    Hp = oracle.fresnel_propagator(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    meas = ps.poisson_counts(oracle.forward_subpixel(d["obj_true"], d["probe"], posf, Hp), d["noise_seed"])
    corner, frac = pt.split_positions(posf)
    plan = TileWalk(corner, spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    dev = "cuda:0"
    ctx = context(spec, len(posf))
    stack = pt.ptycho_shift_probes(ctx, torch.tensor(d["probe"], dtype=torch.complex64, device=dev),
                                   torch.tensor(frac[plan.order], device=dev))
    meas_sorted = torch.tensor(meas[plan.order], device=dev)
    obj = torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev)
    grad = torch.empty_like(obj)
    walk = AllTilesWalk(ctx, plan)
    loss = float(walk.step(obj, stack, meas_sorted, grad).item())
    assert walk.check() == 0
    torch.cuda.synchronize()
    L_ref, _, G_ref = oracle.loss_and_gradient_subpixel(d["obj_eval"], d["probe"], posf, meas, Hp)
    assert abs(loss - L_ref) <= TOL_L * L_ref
    assert rel_l2(grad.cpu().numpy(), G_ref) <= TOL_G
