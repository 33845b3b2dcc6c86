"""Randomised GPU parity: window size, slice count, rectangular object, scattered
positions (edges, repeats, any order), strided object and gradient views, each
case against the FP64 oracle at the standard bounds (intensities 1e-5,
loss 1e-5, gradient 1e-4 relative).  Seeds are fixed; every case prints its
parameters before it runs."""
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


def random_case(seed):
    rng = np.random.default_rng(1000 + seed)
    base = "ms8-1024-m128" if rng.integers(2) else "2d-256-m64"
    spec0 = ps.workload(base)
    M = spec0.M
    S = int(rng.integers(1, 7))
    H = int(rng.integers(M, 2 * M + 41))
    W = int(rng.integers(M, 2 * M + 41))
    n = int(rng.integers(1, 41))
    spec = ps.with_overrides(spec0, W=max(H, W), S=S, ny=1, nx=1, noise=True, strength=0.2)
    d = ps.build_inputs(spec)
    for k in ("obj_true", "obj_eval"):
        d[k] = np.ascontiguousarray(d[k][:, :H, :W])
    pos = np.stack([rng.integers(0, H - M + 1, n), rng.integers(0, W - M + 1, n)], axis=1).astype(np.int32)
    pos[0] = (H - M, W - M)                     # a window in the far corner
    if n > 2:
        pos[1] = (0, 0)
        pos[2] = pos[1]                         # a repeated window
    Hp = oracle.fresnel_propagator(M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    meas = ps.poisson_counts(oracle.forward(d["obj_true"], d["probe"], pos, Hp), d["noise_seed"])
    pad = (int(rng.integers(0, 5)), int(rng.integers(0, 17)))
    strided_grad = bool(rng.integers(2))
    return spec, d, pos, meas, Hp, (S, H, W, n, M), pad, strided_grad


@pytest.mark.parametrize("seed", range(8))
def test_random_configuration(torch_cuda, seed):
    import torch
    import paper_2205_06327_amd as pt
    spec, d, pos, meas, Hp, (S, H, W, n, M), pad, strided_grad = random_case(seed)
    say(f"random case {seed}: M={M} S={S} object {H}x{W} n={n} pad={pad} strided gradient={strided_grad}")
    dev = "cuda:0"
    big = torch.zeros((S, H + pad[0] + 3, W + pad[1] + 5), dtype=torch.complex64, device=dev)
    big[:, pad[0]:pad[0] + H, pad[1]:pad[1] + W] = torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev)
    obj = big[:, pad[0]:pad[0] + H, pad[1]:pad[1] + W]
    probe = torch.tensor(d["probe"], dtype=torch.complex64, device=dev)
    pos_t = torch.tensor(pos, dtype=torch.int32, device=dev)
    meas_t = torch.tensor(meas, dtype=torch.float32, device=dev)
    grad = None
    if strided_grad:
        gbig = torch.full((S, H + 2, W + 9), float("nan"), dtype=torch.complex64, device=dev)
        grad = gbig[:, 1:1 + H, 4:4 + W]
    ctx = context(spec, n)
    I = pt.ptycho_forward(ctx, obj, probe, pos_t)
    loss, G = pt.ptycho_loss_grad(ctx, obj, probe, pos_t, meas_t, grad=grad)
    assert ctx.check() == 0
    torch.cuda.synchronize()
    L_ref, _, G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], pos, meas, Hp)
    assert rel_l2(I.cpu().numpy(), oracle.forward(d["obj_eval"], d["probe"], pos, Hp)) <= TOL_I
    assert abs(float(loss.item()) - L_ref) <= TOL_L * L_ref
    assert rel_l2(G.cpu().numpy(), G_ref) <= TOL_G
    if strided_grad:  # the padding around the gradient view is untouched
        assert torch.isnan(gbig[:, 0]).all() and torch.isnan(gbig[:, :, :4]).all()
