"""Batched persistent launch over uneven reconstructions, the gradient-descent
iteration, its hipGraph replay and the launch-shape autotuner.

Parity: per-reconstruction loss and gradient of the first iteration against
the FP64 oracle, and the loss trajectory of several iterations against the
oracle's own gradient descent (relative 1e-4 per iteration)."""
import numpy as np
import pytest

import oracle
import ptycho_synth as ps
from gpu_helpers import problem, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def small_specs():
    base = ps.workload("ms8-1024-m128")
    m64 = ps.workload("2d-256-m64")
    return [
        ps.with_overrides(m64, name="b0", W=128, S=1, ny=5, nx=4, step=7, noise=True, seed=101, strength=0.05),
        ps.with_overrides(base, name="b1", W=192, S=2, ny=3, nx=4, step=14, seed=102),
        ps.with_overrides(m64, name="b2", W=160, S=3, ny=6, nx=6, step=7, noise=True, seed=103, strength=0.05),
        ps.with_overrides(base, name="b3", W=256, S=1, ny=5, nx=3, step=14, seed=104, dose=1e4),
        ps.with_overrides(base, name="b4", W=224, S=4, ny=4, nx=4, step=14, seed=105, dose=1e6),
        ps.with_overrides(m64, name="b5", W=96, S=2, ny=2, nx=3, step=7, noise=True, seed=106, strength=0.05),
    ]


def build(specs, torch):
    from paper_2205_06327_amd.batch import Recon
    dev = "cuda:0"
    probs, recons = [], []
    for sp in specs:
        d = problem(sp)
        # the step length is a caller input of both sides; the oracle computes it
        alpha = oracle.gd_step_size(d["probe"], d["pos"], sp.W, sp.W, sp.S)
        d["alpha"] = alpha
        probs.append(d)
        recons.append(Recon(torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev),
                            torch.tensor(d["probe"], dtype=torch.complex64, device=dev),
                            torch.tensor(d["pos"], dtype=torch.int32, device=dev),
                            torch.tensor(d["meas"], dtype=torch.float32, device=dev),
                            sp.wavelength_A, sp.dz_A, sp.pixel_A, alpha))
    return probs, recons


def test_batch_first_iteration_matches_oracle(torch_cuda):
    import torch
    from paper_2205_06327_amd.batch import Batch
    specs = small_specs()
    say("batched loss/gradient: 6 uneven reconstructions (M 64/128, S 1-4)")
    probs, recons = build(specs, torch)
    b = Batch(recons, history_rows=4)
    losses = torch.zeros(len(recons), dtype=torch.float64, device="cuda:0")
    b.loss_grad(losses)
    b.sync()
    for sp, d, r, L in zip(specs, probs, recons, losses.cpu().numpy()):
        L_ref, _, G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])
        assert abs(L - L_ref) <= 1e-5 * L_ref, sp.name
        assert rel_l2(r.grad.cpu().numpy(), G_ref) <= 1e-4, sp.name


def test_batch_gradient_descent_trajectory_and_graph_replay(torch_cuda):
    import torch
    from paper_2205_06327_amd.batch import Batch
    specs = small_specs()
    iters = 5
    say(f"batched gradient descent, {iters} iterations: eager vs oracle, then hipGraph replays vs eager")
    probs, recons = build(specs, torch)
    init = [r.obj.clone() for r in recons]
    b = Batch(recons, history_rows=16)
    for _ in range(iters):
        b.step()
    b.sync()
    hist = b.history()
    assert hist.shape == (iters, len(specs))
    eager_obj = [r.obj.clone() for r in recons]
    for k, (sp, d) in enumerate(zip(specs, probs)):
        t = d["obj_eval"].copy()
        traj = []
        for _ in range(iters):
            L, _, G = oracle.loss_and_gradient(t, d["probe"], d["pos"], d["meas"], d["H"])
            traj.append(L)
            t = oracle.gd_step(t, G, d["alpha"])
        traj = np.array(traj)
        np.testing.assert_allclose(hist[:, k], traj, rtol=1e-4, err_msg=sp.name)
        assert np.all(np.diff(traj) < 0), sp.name
        assert np.all(np.diff(hist[:, k]) < 0), sp.name
    # graph: restore the start, capture one iteration, replay with eager work and syncs in between
    torch.cuda.synchronize()
    for r, o in zip(recons, init):
        r.obj.copy_(o)
    torch.cuda.synchronize()
    b.reset_history()
    b.sync()
    b.capture()
    scratch = torch.randn(1 << 20, device="cuda:0")
    for it in range(iters):
        b.replay()
        b.sync()
        scratch.mul_(1.0001).add_(1.0)  # unrelated eager work between replays
        torch.cuda.synchronize()
        h = b.history()
        assert h.shape[0] == it + 1
        np.testing.assert_allclose(h[it], hist[it], rtol=1e-6)
    for r, e in zip(recons, eager_obj):
        assert rel_l2(r.obj.cpu().numpy(), e.cpu().numpy()) <= 1e-6


def test_autotuner_picks_a_valid_shape_and_caches(torch_cuda, tmp_path):
    import torch
    from paper_2205_06327_amd.autotune import tune
    from paper_2205_06327_amd.batch import Batch
    specs = small_specs()
    say("autotuner on the small batch")
    probs, recons = build(specs, torch)
    b = Batch(recons, history_rows=2)
    cache = str(tmp_path / "tune.json")
    first = tune(b, reps=2, cache_path=cache)
    assert not first["cached"] and first["ms"] > 0
    losses = torch.zeros(len(recons), dtype=torch.float64, device="cuda:0")
    b.loss_grad(losses)
    b.sync()
    for d, L in zip(probs, losses.cpu().numpy()):
        L_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])[0]
        assert abs(L - L_ref) <= 1e-5 * L_ref
    b2 = Batch(recons, history_rows=2)
    second = tune(b2, reps=2, cache_path=cache)
    assert second["cached"] and second[64] == first[64] and second[128] == first[128]
    assert b2.grid(64) == min(first[64], sum(r.pos.shape[0] for r in recons if r.probe.shape[0] == 64))


@pytest.mark.parametrize("M", [64, 128])
def test_batch_one_window_size_with_an_empty_reconstruction(torch_cuda, M):
    """A batch with a single window-size class (no side stream) and a reconstruction without
    positions: its loss is 0, its gradient 0 and the update leaves it unchanged; the others match
    the oracle."""
    import torch
    from paper_2205_06327_amd.batch import Batch, Recon
    specs = [sp for sp in small_specs() if sp.M == M][:2]
    say(f"batch of one window size (M={M}) plus an empty reconstruction")
    probs, recons = build(specs, torch)
    sp0, d0 = specs[0], probs[0]
    dev = "cuda:0"
    empty_obj = torch.tensor(d0["obj_eval"], dtype=torch.complex64, device=dev)
    recons.append(Recon(empty_obj.clone(), torch.tensor(d0["probe"], dtype=torch.complex64, device=dev),
                        torch.zeros((0, 2), dtype=torch.int32, device=dev),
                        torch.zeros((0, M, M), dtype=torch.float32, device=dev),
                        sp0.wavelength_A, sp0.dz_A, sp0.pixel_A, 1e-3))
    b = Batch(recons, history_rows=4)
    losses = torch.full((len(recons),), -1.0, dtype=torch.float64, device=dev)
    b.loss_grad(losses)
    b.sync()
    L = losses.cpu().numpy()
    assert L[-1] == 0.0 and float(recons[-1].grad.abs().max()) == 0.0
    for sp, d, r, Lk in zip(specs, probs, recons, L):
        L_ref, _, G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])
        assert abs(Lk - L_ref) <= 1e-5 * L_ref, sp.name
        assert rel_l2(r.grad.cpu().numpy(), G_ref) <= 1e-4, sp.name
    b.update()
    b.sync()
    assert torch.equal(recons[-1].obj, empty_obj)


def test_batch32_uneven_parity_with_autotuner_and_graph_replay(torch_cuda):
    """The 32 uneven reconstructions of the batched workload at their own shapes (objects of 256-1024 px,
    1-8 slices, 64- and 128-windows, Poisson doses 1e4-1e6), launch shapes chosen by the autotuner:
    first-iteration loss (1e-5) and a gradient block on every slice (1e-4) per reconstruction, then
    20 hipGraph-replayed gradient-descent iterations against the oracle's loss trajectory (1e-4 per
    iteration, every reconstruction), descending monotonically.  The oracle's values are stored in
    tests/golden/batch32_gd_trajectory.json (written by make_batch32_trajectory.py from oracle/ only)."""
    import json
    import os

    import torch
    from oracle_pool import batch_problems
    from paper_2205_06327_amd.autotune import tune
    from paper_2205_06327_amd.batch import Batch, Recon
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch32_gd_trajectory.json")) as f:
        golden = json.load(f)
    specs = ps.batch_specs(4)
    assert [g["name"] for g in golden["recons"]] == [sp.name for sp in specs]
    iters, bs = golden["iterations"], golden["block"]
    say(f"32 uneven reconstructions: inputs and oracle measurements ({sum(sp.n for sp in specs)} positions)")
    probs = batch_problems(specs)
    dev = "cuda:0"
    recons = []
    for sp, p, g in zip(specs, probs, golden["recons"]):
        assert (sp.M, sp.S, sp.W, sp.n) == (g["M"], g["S"], g["W"], g["n"])
        assert abs(p["alpha"] - g["alpha"]) <= 1e-12 * g["alpha"], sp.name  # the same inputs as the golden run
        recons.append(Recon(torch.tensor(p["obj"], device=dev), torch.tensor(p["probe"], device=dev),
                            torch.tensor(p["pos"], dtype=torch.int32, device=dev),
                            torch.tensor(p["meas"], dtype=torch.float32, device=dev),
                            sp.wavelength_A, sp.dz_A, sp.pixel_A, p["alpha"]))
    del probs
    b = Batch(recons, history_rows=iters)
    tuned = tune(b, reps=2, rounds=1, cache_path=None)
    say(f"  autotuner: 64-windows {tuned[64]} workgroups, 128-windows {tuned[128]}")
    losses = torch.zeros(len(recons), dtype=torch.float64, device=dev)
    b.loss_grad(losses)
    b.sync()
    L = losses.cpu().numpy()
    worst_l, worst_g = 0.0, 0.0
    for k, (sp, r, g) in enumerate(zip(specs, recons, golden["recons"])):
        el = abs(L[k] - g["loss"][0]) / g["loss"][0]
        by, bx = g["block_origin"]
        ref = np.array(g["grad_block_re"]) + 1j * np.array(g["grad_block_im"])
        eg = rel_l2(r.grad[:, by:by + bs, bx:bx + bs].cpu().numpy(), ref)
        worst_l, worst_g = max(worst_l, el), max(worst_g, eg)
        assert el <= 1e-5, (sp.name, el)
        assert eg <= 1e-4, (sp.name, eg)
    say(f"  first iteration: worst loss rel err {worst_l:.2e}, worst gradient block rel L2 {worst_g:.2e}")
    b.reset_history()
    b.capture()
    for _ in range(iters):
        b.replay()
    b.sync()
    hist = b.history()
    assert hist.shape == (iters, len(specs))
    worst = 0.0
    for k, (sp, g) in enumerate(zip(specs, golden["recons"])):
        ref = np.array(g["loss"])
        assert np.all(np.diff(ref) < 0), sp.name
        assert np.all(np.diff(hist[:, k]) < 0), sp.name
        e = float(np.max(np.abs(hist[:, k] - ref) / ref))
        worst = max(worst, e)
        assert e <= 1e-4, (sp.name, e)
    say(f"  {iters} replayed iterations: worst per-iteration loss rel err {worst:.2e}")
