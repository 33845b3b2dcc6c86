"""GPU (gfx950) vs FP64 oracle parity of the fused forward / loss / adjoint path.

Tolerances: intensities 1e-5 relative L2, gradients 1e-4 relative L2, loss 1e-5
relative (FP32 kernel against the FP64 oracle on identical inputs).
"""
import numpy as np
import pytest

import oracle
import ptycho_synth as ps
from gpu_helpers import context, problem, rel_l2, say, to_dev

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


def run_forward(spec, d, obj_key="obj_eval"):
    import paper_2205_06327_amd as pt
    import torch
    t = to_dev(d, obj_key)
    ctx = context(spec, max_positions=len(d["pos"]))
    I = pt.ptycho_forward(ctx, t["obj"], t["probe"], t["pos"])
    ctx.check()
    torch.cuda.synchronize()
    return I.cpu().numpy()


def run_loss_grad(spec, d, obj_key="obj_eval"):
    import paper_2205_06327_amd as pt
    import torch
    t = to_dev(d, obj_key)
    n = len(d["pos"])
    ctx = context(spec, max_positions=max(n, 1))
    lpp = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    loss, grad = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"], loss_per_pos=lpp)
    ctx.check()
    torch.cuda.synchronize()
    return float(loss.item()), lpp.cpu().numpy(), grad.cpu().numpy()


CASES = {
    # name: spec
    "2d-256-m64 full scan (256 positions, noise-free)": ps.workload("2d-256-m64"),
    "2d-1024-m128 reduced to 256^2, 5x6 positions": ps.reduced(ps.workload("2d-1024-m128"), W=256, ny=5, nx=6),
    "ms8-1024-m128 reduced to 256^2, 5x7 positions": ps.reduced(ps.workload("ms8-1024-m128"), W=256, ny=5, nx=7),
    "m64 S=3 ragged 13 positions": ps.with_overrides(ps.workload("2d-256-m64"), W=160, S=3, ny=13, nx=1, step=7,
                                                      strength=0.4, noise=True),
    "m128 S=16 3x3 positions": ps.reduced(ps.workload("ms16-2048-m128-tiles4x4"), W=192, ny=3, nx=3, S=16),
    # two slices: one propagation, then the far-field transform right after it (no barrier between)
    "m128 S=2 2x3 positions": ps.with_overrides(ps.workload("ms8-1024-m128"), W=200, S=2, ny=2, nx=3, step=17,
                                                 noise=True),
    "m64 S=2 ragged 7 positions": ps.with_overrides(ps.workload("2d-256-m64"), W=140, S=2, ny=7, nx=1, step=11,
                                                     strength=0.4, noise=True),
}


@pytest.mark.parametrize("name", list(CASES))
def test_forward_parity(torch_cuda, name):
    spec = CASES[name]
    say(f"forward parity: {name}")
    d = problem(spec)
    I = run_forward(spec, d)
    I_ref = oracle.forward(d["obj_eval"], d["probe"], d["pos"], d["H"])
    err = rel_l2(I, I_ref)
    say(f"  intensities rel L2 = {err:.3e}")
    assert err <= TOL_I
    # Parseval on the pure-phase truth: every pattern sums to the dose.
    I_t = run_forward(spec, d, "obj_true")
    np.testing.assert_allclose(I_t.sum(axis=(1, 2)), spec.dose, rtol=2e-5)


@pytest.mark.parametrize("name", list(CASES))
def test_loss_grad_parity(torch_cuda, name):
    spec = CASES[name]
    say(f"loss/gradient parity: {name}")
    d = problem(spec)
    L, lpp, G = run_loss_grad(spec, d)
    L_ref, lpp_ref, G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])
    eg = rel_l2(G, G_ref)
    el = abs(L - L_ref) / abs(L_ref)
    say(f"  loss rel = {el:.3e}, gradient rel L2 = {eg:.3e}")
    assert el <= TOL_L
    assert eg <= TOL_G
    np.testing.assert_allclose(lpp, lpp_ref, rtol=1e-4, atol=1e-6 * np.abs(lpp_ref).max())
    assert abs(lpp.sum() - L) <= 1e-9 * abs(L)
    # Locality (Section III): nothing outside the union of windows.
    cover = np.zeros(G.shape[1:], dtype=bool)
    for y0, x0 in d["pos"]:
        cover[y0:y0 + spec.M, x0:x0 + spec.M] = True
    assert np.all(G[:, ~cover] == 0)


def test_zero_gradient_at_truth_noise_free(torch_cuda):
    spec = ps.with_overrides(ps.workload("ms8-1024-m128"), W=224, ny=4, nx=4, S=4, noise=False)
    say("zero gradient at the truth (noise-free FP64 measurements)")
    d = problem(spec)
    L_t, _, G_t = run_loss_grad(spec, d, "obj_true")
    L_e, _, G_e = run_loss_grad(spec, d, "obj_eval")
    # FP32 rounding only: tiny relative to the gradient one step away from the truth.
    assert np.linalg.norm(G_t) <= 2e-3 * np.linalg.norm(G_e)
    assert L_t <= 1e-4 * L_e


def test_accumulate_and_empty(torch_cuda):
    import paper_2205_06327_amd as pt
    import torch
    spec = ps.reduced(ps.workload("ms8-1024-m128"), W=256, ny=3, nx=3, S=2)
    say("accumulate flag, empty and single-position calls")
    d = problem(spec)
    t = to_dev(d)
    ctx = context(spec, 16)
    loss, grad = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"])
    l1 = float(loss.item())
    g1 = grad.clone()
    pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"], grad=grad, loss=loss, accumulate=True)
    torch.cuda.synchronize()
    assert abs(float(loss.item()) - 2 * l1) <= 1e-12 * abs(l1)
    assert rel_l2(grad.cpu().numpy(), 2 * g1.cpu().numpy()) <= 1e-6
    # empty call: zero loss, zeroed gradient
    e_loss, e_grad = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"][:0], t["meas"][:0], grad=grad)
    torch.cuda.synchronize()
    assert float(e_loss.item()) == 0.0 and float(e_grad.abs().max()) == 0.0
    I0 = pt.ptycho_forward(ctx, t["obj"], t["probe"], t["pos"][:0])
    assert I0.shape == (0, spec.M, spec.M)
    # single position equals the oracle
    L1, _, G1 = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"][:1], d["meas"][:1], d["H"])
    l_one, g_one = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"][:1].contiguous(), t["meas"][:1].contiguous())
    ctx.check()
    assert abs(float(l_one.item()) - L1) <= TOL_L * L1
    assert rel_l2(g_one.cpu().numpy(), G1) <= TOL_G


def test_corner_windows_and_strided_object(torch_cuda):
    import paper_2205_06327_amd as pt
    import torch
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=200, S=2, noise=True)
    say("windows touching every object edge; object given as a strided view")
    d = problem(spec)
    W, M = spec.W, spec.M
    d["pos"] = np.array([[0, 0], [0, W - M], [W - M, 0], [W - M, W - M], [68, 0], [0, 70]], dtype=np.int32)
    H = d["H"]
    d["meas"] = ps.poisson_counts(oracle.forward(d["obj_true"], d["probe"], d["pos"], H), d["noise_seed"])
    t = to_dev(d)
    big = torch.zeros((spec.S, W + 8, W + 24), dtype=torch.complex64, device="cuda:0")
    big[:, 3:3 + W, 5:5 + W] = t["obj"]
    view = big[:, 3:3 + W, 5:5 + W]
    ctx = context(spec, 16)
    I = pt.ptycho_forward(ctx, view, t["probe"], t["pos"])
    loss, G = pt.ptycho_loss_grad(ctx, view, t["probe"], t["pos"], t["meas"])
    ctx.check()
    L_ref, _, G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], H)
    assert rel_l2(I.cpu().numpy(), oracle.forward(d["obj_eval"], d["probe"], d["pos"], H)) <= TOL_I
    assert abs(float(loss.item()) - L_ref) <= TOL_L * L_ref
    assert rel_l2(G.cpu().numpy(), G_ref) <= TOL_G


def test_device_side_window_checks(torch_cuda):
    import paper_2205_06327_amd as pt
    import torch
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=128, ny=2, nx=2, step=16)
    say("device status word: out-of-object window is skipped and reported")
    d = problem(spec)
    t = to_dev(d)
    ctx = context(spec, 16)
    bad = t["pos"].clone()
    bad[1, 0] = 100  # 100 + 64 > 128: outside the object
    I = torch.full((4, 64, 64), -1.0, device="cuda:0")
    pt.ptycho_forward(ctx, t["obj"], t["probe"], bad, intens=I)
    with pytest.raises(pt.PtychoError) as e:
        ctx.check()
    assert e.value.name == "PTYCHO_E_BOUNDS"
    assert float(I[1].max()) == -1.0 and float(I[0].min()) >= 0.0
    assert ctx.check() == 0  # cleared
    # the binding refuses position arrays that are not [n, 2] and host tensors before any launch
    with pytest.raises(ValueError):
        pt.ptycho_forward(ctx, t["obj"], t["probe"], t["pos"].reshape(-1).contiguous())
    with pytest.raises(ValueError):
        pt.ptycho_forward(ctx, t["obj"].cpu(), t["probe"], t["pos"])


def test_degenerate_inputs(torch_cuda):
    """Degenerate cases of the method, for both window sizes: a zero probe (|Psi| = 0 everywhere,
    so u = 0: the loss is the sum of the measurements and the gradient vanishes exactly, no NaN),
    zero measurements (the loss is the total intensity) and dz = 0 (the propagator is the identity,
    so the slices act as their product), each against the oracle."""
    import paper_2205_06327_amd as pt
    import torch
    for M, base in ((128, "ms8-1024-m128"), (64, "2d-256-m64")):
        spec = ps.with_overrides(ps.workload(base), W=2 * M, ny=2, nx=3, step=M // 8, S=3, noise=True)
        say(f"degenerate inputs, M={M}: zero probe, zero measurements, dz = 0")
        d = problem(spec)
        t = to_dev(d)
        ctx = context(spec, spec.n)
        loss, G = pt.ptycho_loss_grad(ctx, t["obj"], torch.zeros_like(t["probe"]), t["pos"], t["meas"])
        assert ctx.check() == 0
        expect = float(d["meas"].astype(np.float64).sum())
        assert abs(float(loss.item()) - expect) <= 1e-6 * expect
        assert float(G.abs().max()) == 0.0
        zero = np.zeros_like(d["meas"])
        loss, G = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], torch.zeros_like(t["meas"]))
        L_ref, _, G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], zero, d["H"])
        assert abs(float(loss.item()) - L_ref) <= TOL_L * L_ref
        assert rel_l2(G.cpu().numpy(), G_ref) <= TOL_G
        ctx0 = pt.Context(M, spec.S, spec.wavelength_A, 0.0, spec.pixel_A, spec.n)
        H0 = oracle.fresnel_propagator(M, spec.wavelength_A, 0.0, spec.pixel_A)
        I = pt.ptycho_forward(ctx0, t["obj"], t["probe"], t["pos"])
        loss, G = pt.ptycho_loss_grad(ctx0, t["obj"], t["probe"], t["pos"], t["meas"])
        assert ctx0.check() == 0
        L_ref, _, G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], H0)
        assert rel_l2(I.cpu().numpy(), oracle.forward(d["obj_eval"], d["probe"], d["pos"], H0)) <= TOL_I
        assert abs(float(loss.item()) - L_ref) <= TOL_L * L_ref
        assert rel_l2(G.cpu().numpy(), G_ref) <= TOL_G


def test_c_abi_refuses_host_memory_and_overruns(torch_cuda):
    """The C ABI checks the caller's buffers on the host before enqueuing anything: a pageable
    host pointer (E_ARG) and a position count that runs past the positions' allocation (E_SHAPE)
    are refused, and the context stays usable."""
    import ctypes
    import paper_2205_06327_amd as pt
    import torch
    from paper_2205_06327_amd import _binding as B
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=128, ny=2, nx=2, step=16)
    say("C ABI: host pointer and overrun refused before launch")
    d = problem(spec)
    t = to_dev(d)
    n_big = 300_000  # 2.4 MB of positions: past the 2 MB block holding the 4-position tensor
    ctx = context(spec, n_big)
    L = pt.lib()
    S, H, W, ss, ld = B._obj_geometry(t["obj"])
    host_out = np.zeros((4, 64, 64), dtype=np.float32)
    vp = ctypes.c_void_p
    rc = L.ptycho_forward(ctx.handle, vp(t["obj"].data_ptr()), H, W, ss, ld, vp(t["probe"].data_ptr()),
                          vp(t["pos"].data_ptr()), 4, vp(host_out.ctypes.data))
    assert B.ERRORS.get(rc) == "PTYCHO_E_ARG" and "device-accessible" in L.ptycho_last_error().decode()
    out = torch.empty((4, 64, 64), dtype=torch.float32, device="cuda:0")
    rc = L.ptycho_forward(ctx.handle, vp(t["obj"].data_ptr()), H, W, ss, ld, vp(t["probe"].data_ptr()),
                          vp(t["pos"].data_ptr()), n_big, vp(out.data_ptr()))
    assert B.ERRORS.get(rc) == "PTYCHO_E_SHAPE" and "positions" in L.ptycho_last_error().decode()
    torch.cuda.synchronize()
    assert ctx.check() == 0
    I = pt.ptycho_forward(ctx, t["obj"], t["probe"], t["pos"])
    assert rel_l2(I.cpu().numpy(), oracle.forward(d["obj_eval"], d["probe"], d["pos"], d["H"])) <= TOL_I


def test_profile_events_count_launches_and_positions(torch_cuda):
    """ptycho_profile_enable / ptycho_profile_read: HIP events around every fused launch on the
    context stream; the read returns the summed time, the launch count and the positions, and resets."""
    import torch
    import paper_2205_06327_amd as pt
    spec = ps.reduced(ps.workload("ms8-1024-m128"), W=256, ny=3, nx=3, S=2)
    say("profiling events around the fused launches")
    d = problem(spec)
    t = to_dev(d)
    ctx = context(spec, spec.n)
    ctx.profile(True)
    ctx.profile_read()
    for _ in range(3):
        pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"])
    pt.ptycho_forward(ctx, t["obj"], t["probe"], t["pos"][:4].contiguous())
    ms, launches, positions = ctx.profile_read()
    assert launches == 4 and positions == 3 * spec.n + 4 and ms > 0.0
    assert ctx.profile_read()[1] == 0  # the read resets the counts
    ctx.profile(False)
    pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"])
    assert ctx.profile_read()[1] == 0
    torch.cuda.synchronize()


def test_checkpointed_wave_recomputation(torch_cuda):
    """Keeping only every k-th incident wave and recomputing the others in the adjoint sweep
    gives the same losses (the forward sweep is unchanged) and the same gradient up to the
    order of the gradient atomics, with a smaller wave store."""
    import torch
    import paper_2205_06327_amd as pt
    spec = ps.with_overrides(ps.workload("ms16-2048-m128-tiles4x4"), W=256, ny=3, nx=4, step=14)
    say("checkpoint intervals 1..5 and 16 on 16 slices, 12 positions")
    d = problem(spec)
    t = to_dev(d)
    ctx = context(spec, spec.n)
    G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])[2]
    results = {}
    for k in (1, 2, 3, 4, 5, 16):
        ctx.set_checkpoint(k)
        lpp = torch.zeros(spec.n, dtype=torch.float64, device="cuda:0")
        _, g = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"], loss_per_pos=lpp)
        assert ctx.check() == 0
        torch.cuda.synchronize()
        results[k] = (lpp.cpu().numpy(), g.cpu().numpy(), ctx.workspace_bytes())
    l1, g1, b1 = results[1]
    for k, (lk, gk, bk) in results.items():
        np.testing.assert_array_equal(lk, l1)
        assert rel_l2(gk, g1) <= 1e-6, k
        assert rel_l2(gk, G_ref) <= 1e-4, k
    assert results[4][2] < b1 and results[16][2] == b1
    with pytest.raises(pt.PtychoError):
        ctx.set_checkpoint(0)


@pytest.mark.parametrize("M", [64, 128])
def test_short_stacks_checkpoint_intervals(torch_cuda, M):
    """Stacks of 2, 3 and 5 slices with checkpoint intervals 1, 2 and 3, both window sizes: every
    arrangement of checkpoints, inner waves, recomputed segments and stored waves requested one
    propagation early in the adjoint sweep (stacks shorter than the interval included) gives the
    oracle's gradient, and the losses do not depend on the interval."""
    import torch
    import paper_2205_06327_amd as pt
    base = ps.workload("2d-256-m64" if M == 64 else "ms8-1024-m128")
    for S in (2, 3, 5):
        spec = ps.with_overrides(base, W=256 if M == 64 else 384, S=S, strength=0.05, ny=3, nx=3,
                                 step=8 if M == 64 else 14)
        say(f"M={M}, {S} slices, checkpoint intervals 1..3, 9 positions")
        d = problem(spec)
        t = to_dev(d)
        ctx = context(spec, spec.n)
        G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])[2]
        res = {}
        for k in (1, 2, 3):
            ctx.set_checkpoint(k)
            lpp = torch.zeros(spec.n, dtype=torch.float64, device="cuda:0")
            _, g = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"], loss_per_pos=lpp)
            assert ctx.check() == 0
            torch.cuda.synchronize()
            res[k] = (lpp.cpu().numpy(), g.cpu().numpy())
        for k, (lk, gk) in res.items():
            np.testing.assert_array_equal(lk, res[1][0])
            assert rel_l2(gk, res[1][1]) <= 1e-6, (S, k)
            assert rel_l2(gk, G_ref) <= TOL_G, (S, k)


def test_potential_parametrisation_autograd(torch_cuda):
    """t = exp(i sigma V) and dF/dV = sigma Im(conj(t) dF/dt) in the library's kernels, through
    torch autograd, against the oracle's chain rule (pinned by central differences)."""
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.autograd import amplitude_loss_potential
    spec = ps.with_overrides(ps.workload("ms8-1024-m128"), W=256, ny=3, nx=3, step=14, S=3)
    say("real-potential parametrisation, 3 slices, 9 positions")
    d = problem(spec)
    sigma = 0.8
    V = (np.angle(d["obj_eval"]) / sigma).astype(np.float32)
    t_ref = oracle.transmission_from_potential(V, sigma)
    L_ref, _, G_ref = oracle.loss_and_gradient(t_ref, d["probe"], d["pos"], d["meas"], d["H"])
    gV_ref = oracle.potential_gradient(t_ref, G_ref, sigma)
    dev = "cuda:0"
    ctx = context(spec, spec.n)
    Vd = torch.tensor(V, device=dev, requires_grad=True)
    t_gpu = pt.ptycho_potential_transmission(ctx, Vd.detach(), sigma)
    torch.cuda.synchronize()
    assert np.abs(t_gpu.cpu().numpy() - t_ref).max() <= 1e-6
    probe = torch.tensor(d["probe"], dtype=torch.complex64, device=dev)
    pos = torch.tensor(d["pos"], device=dev)
    meas = torch.tensor(d["meas"], device=dev)
    loss = amplitude_loss_potential(ctx, Vd, sigma, probe, pos, meas)
    (3.0 * loss).backward()
    assert ctx.check() == 0
    assert abs(float(loss.item()) - L_ref) <= 1e-5 * L_ref
    assert rel_l2(Vd.grad.cpu().numpy(), 3.0 * gV_ref) <= 1e-4


def test_probe_gradient(torch_cuda):
    """dF/dP from the same launch as the object gradient, through autograd and with
    accumulation, against the oracle (pinned by torch complex autograd on tiny grids)."""
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.autograd import amplitude_loss
    for name, spec in [("m128 S=4", ps.with_overrides(ps.workload("ms8-1024-m128"), W=256, ny=3, nx=4, step=14, S=4)),
                       ("m64 S=3", ps.with_overrides(ps.workload("2d-256-m64"), W=160, ny=5, nx=5, step=7, S=3,
                                                     noise=True, strength=0.05))]:
        say(f"probe gradient, {name}, {spec.n} positions")
        d = problem(spec)
        GP = oracle.probe_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])
        G = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])[2]
        t = to_dev(d)
        ctx = context(spec, spec.n)
        obj = t["obj"].clone().requires_grad_(True)
        probe = t["probe"].clone().requires_grad_(True)
        loss = amplitude_loss(ctx, obj, probe, t["pos"], t["meas"])
        (0.5 * loss).backward()
        assert ctx.check() == 0
        assert rel_l2(probe.grad.cpu().numpy(), 0.5 * GP) <= 1e-4
        assert rel_l2(obj.grad.cpu().numpy(), 0.5 * G) <= 1e-4
        # accumulate: a second call adds the same again
        pg = torch.zeros_like(t["probe"])
        g = torch.zeros_like(t["obj"])
        loss_d = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        for _ in range(2):
            pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"], grad=g, loss=loss_d,
                                accumulate=True, probe_grad=pg)
        torch.cuda.synchronize()
        assert rel_l2(pg.cpu().numpy(), 2 * GP) <= 1e-4
