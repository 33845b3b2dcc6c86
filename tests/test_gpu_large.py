"""Largest shapes.  An object of more than 2^31 complex elements (16 slices of
11600 x 11600, 17.2 GB, plus a gradient of the same size) with windows at its
far corners, so every 64-bit offset of the kernels is exercised; and the
largest slice count (64).  Windows are disjoint, so each one's expected
loss and gradient come from the oracle on its own M x M sub-object."""
import numpy as np
import pytest

import oracle
import ptycho_synth as ps
from gpu_helpers import rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def check_disjoint_windows(S, W, pos, tol_i, tol_g, seed, loss_tol=None):
    import torch
    import paper_2205_06327_amd as pt
    spec = ps.with_overrides(ps.workload("2d-256-m64"), S=S, W=W, strength=0.05)
    M = spec.M
    n = len(pos)
    ss = ps.seed_streams(seed)
    # the same recipe as the other parity tests: measurements of a smooth truth, gradient at a
    # nearby smooth evaluation point (a white-noise truth would scatter intensity where the
    # evaluated far field is at rounding level, where the residual's direction is ill-conditioned)
    truth = ps.make_object(M, S * n, spec.strength, 10.0, ss[0])
    windows = ps.eval_object(truth, 10.0, ss[1]).reshape(n, S, M, M).astype(np.complex64)
    truth = truth.reshape(n, S, M, M)
    probe = ps.make_probe(M, spec.R, spec.C, spec.dose).astype(np.complex64)
    H = oracle.fresnel_propagator(M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    origin = np.zeros((1, 2), np.int32)
    I_true = np.stack([oracle.forward(truth[i], probe, origin, H)[0] for i in range(n)])
    meas = ps.poisson_counts(I_true, ss[2])  # Poisson counts, as in the other parity tests
    dev = torch.device("cuda:0")
    obj = torch.ones((S, W, W), dtype=torch.complex64, device=dev)
    for i, (y0, x0) in enumerate(pos):
        obj[:, y0:y0 + M, x0:x0 + M] = torch.tensor(windows[i], dtype=torch.complex64, device=dev)
    grad = torch.empty_like(obj)
    probe_d = torch.tensor(probe, dtype=torch.complex64, device=dev)
    pos_d = torch.tensor(pos, device=dev)
    meas_d = torch.tensor(meas, device=dev)
    ctx = pt.Context(M, S, spec.wavelength_A, spec.dz_A, spec.pixel_A, n)
    lpp = torch.zeros(n, dtype=torch.float64, device=dev)
    pt.ptycho_loss_grad(ctx, obj, probe_d, pos_d, meas_d, grad=grad, loss_per_pos=lpp)
    I = pt.ptycho_forward(ctx, obj, probe_d, pos_d)
    assert ctx.check() == 0
    torch.cuda.synchronize()
    worst_i = worst_g = 0.0
    for i, (y0, x0) in enumerate(pos):
        L_ref, _, G_ref = oracle.loss_and_gradient(windows[i], probe, origin, meas[i:i + 1], H)
        I_ref = oracle.forward(windows[i], probe, origin, H)[0]
        worst_i = max(worst_i, rel_l2(I[i].cpu().numpy(), I_ref))
        # the gradient is linear in the residual d = |Psi| - a, so a relative error e in |Psi| becomes
        # e ||Psi|| / ||d|| = e sqrt(dose / F) in it (g_cond scales the given transform-chain bound)
        g_cond = 1.0 if loss_tol is None else np.sqrt(spec.dose / L_ref)
        worst_g = max(worst_g, rel_l2(grad[:, y0:y0 + M, x0:x0 + M].cpu().numpy(), G_ref) / g_cond)
        # loss: 1e-5, or with a given intensity bound e, |dF| <= 2 ||d|| ||d|Psi|||  ~  e sqrt(F * dose)
        lt = 1e-5 * L_ref if loss_tol is None else loss_tol * np.sqrt(L_ref * spec.dose)
        assert abs(float(lpp[i]) - L_ref) <= lt, (i, float(lpp[i]), L_ref)
    say(f"  worst intensity rel L2 {worst_i:.2e} (bound {tol_i:.1e}), gradient {worst_g:.2e} (bound {tol_g:.1e})")
    assert worst_i <= tol_i and worst_g <= tol_g
    # nothing written outside the windows: a band beside the last window, last slices
    band = grad[S - 4:, W - M - 40:W - M, W - 200:].abs().max().item()
    assert band == 0.0
    del obj, grad
    torch.cuda.empty_cache()


def test_object_beyond_2_pow_31_elements(torch_cuda):
    S, W, M = 16, 11600, 64
    assert S * W * W > 2 ** 31
    say(f"object {S} x {W}^2 complex64 ({S * W * W * 8 / 1e9:.1f} GB), windows at the far corners")
    pos = np.array([[0, 0], [W - M, W - M], [W - M, 17], [5801, W - M - 5], [11, W - M]], dtype=np.int32)
    check_disjoint_windows(S, W, pos, 1e-5, 1e-4, seed=77)


def test_sixty_four_slices(torch_cuda):
    # FP32 rounding grows with the transform chain: the forward sweep runs 2S - 1
    # transforms of log2(M^2) radix stages each, so the tolerance on intensities is
    # the linear bound (2S - 1) log2(M^2) u with u = 2^-24 (9.1e-5 at S = 64, M = 64),
    # on gradients the same over the 4S - 2 transforms of both sweeps (1.8e-4) times
    # the residual's conditioning sqrt(dose / F); at 16 slices the fixed 1e-5 and
    # 1e-4 are inside these bounds.
    S, W, M = 64, 320, 64
    say(f"{S} slices, {W}^2 object")
    pos = np.array([[0, 0], [W - M, W - M], [100, 7]], dtype=np.int32)
    u = 2.0 ** -24
    tol_i = (2 * S - 1) * np.log2(M * M) * u
    tol_g = max(1e-4, (4 * S - 2) * np.log2(M * M) * u)  # forward and adjoint transforms
    check_disjoint_windows(S, W, pos, tol_i, tol_g, seed=78, loss_tol=tol_i)
