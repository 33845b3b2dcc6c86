"""ptycho_loss_grad_static (no context, no device allocation) against ptycho_loss_grad.

Both run the same fused kernel; the static entry point takes its tables,
per-position losses and incident-wave store from the library's static device
array instead of a context.  Each test makes two calls in a row, the second on
a smaller input, and compares every output of each call with the context
entry point's on the same inputs (loss, per-position losses, gradient: 1e-6
relative, well inside the 1e-5 / 1e-4 bar against the FP64 oracle).
"""
import numpy as np
import pytest

import ptycho_synth as ps
from gpu_helpers import context, problem, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-6


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06327_amd as pt
    pt.lib()
    return torch


def both(spec, d, accumulate_twice=False):
    """(context result, static result), each as (loss, per-position losses, gradient) on the host."""
    import paper_2205_06327_amd as pt
    import torch
    t = to_dev(d)
    n = len(d["pos"])
    ctx = context(spec, max_positions=max(n, 1))
    lpp_c = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    loss_c, grad_c = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"], loss_per_pos=lpp_c)
    ctx.check()
    lpp_s = torch.full((n,), -1.0, dtype=torch.float64, device="cuda:0")
    grad_s = torch.full_like(t["obj"], complex(7.0, -7.0))  # overwritten (not accumulated) by the call
    loss_s = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    pt.ptycho_loss_grad_static(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A, t["obj"], t["probe"], t["pos"],
                               t["meas"], grad=grad_s, loss=loss_s, loss_per_pos=lpp_s)
    if accumulate_twice:
        pt.ptycho_loss_grad_static(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A, t["obj"], t["probe"],
                                   t["pos"], t["meas"], grad=grad_s, loss=loss_s, accumulate=True)
    torch.cuda.synchronize()
    ctx.close()
    c = (float(loss_c.item()), lpp_c.cpu().numpy(), grad_c.cpu().numpy())
    s = (float(loss_s.item()), lpp_s.cpu().numpy(), grad_s.cpu().numpy())
    return c, s


def check_pair(name, c, s, factor=1.0):
    rl = abs(s[0] - factor * c[0]) / abs(c[0])
    rp = float(np.max(np.abs(s[1] - c[1]) / np.maximum(np.abs(c[1]), 1e-300)))
    rg = rel_l2(s[2], factor * c[2])
    say(f"{name}: loss {rl:.2e}, per-position {rp:.2e}, gradient {rg:.2e}")
    assert rl <= TOL and rp <= TOL and rg <= TOL, (rl, rp, rg)


CALLS = {
    "m128": [
        ("m128 S=8 5x7 positions on 256^2", ps.reduced(ps.workload("ms8-1024-m128"), W=256, ny=5, nx=7)),
        ("m128 S=2 2x3 positions on 200^2", ps.with_overrides(ps.workload("ms8-1024-m128"), W=200, S=2, ny=2, nx=3,
                                                              step=17, noise=True)),
    ],
    "m64": [
        ("m64 S=3 13 positions on 160^2", ps.with_overrides(ps.workload("2d-256-m64"), W=160, S=3, ny=13, nx=1, step=7,
                                                            strength=0.4, noise=True)),
        ("m64 S=2 7 positions on 140^2", ps.with_overrides(ps.workload("2d-256-m64"), W=140, S=2, ny=7, nx=1, step=11,
                                                           strength=0.4, noise=True)),
    ],
    # 16 slices of 128-windows: the static store holds them only with checkpointed incident waves
    "m128-16-slices": [
        ("m128 S=16 3x3 positions on 192^2", ps.reduced(ps.workload("ms16-2048-m128-tiles4x4"), W=192, ny=3, nx=3,
                                                        S=16)),
        ("m128 S=16 2x2 positions on 160^2", ps.reduced(ps.workload("ms16-2048-m128-tiles4x4"), W=160, ny=2, nx=2,
                                                        S=16)),
    ],
}


@pytest.mark.parametrize("group", list(CALLS))
def test_static_entry_point_matches_the_context_entry_point_on_two_calls(torch_cuda, group):
    for name, spec in CALLS[group]:
        say(f"static vs context: {name}")
        c, s = both(spec, problem(spec))
        check_pair(name, c, s)


def test_static_entry_point_accumulates(torch_cuda):
    name, spec = CALLS["m128"][1]
    say(f"static, overwrite then accumulate: {name}")
    c, s = both(spec, problem(spec), accumulate_twice=True)
    check_pair(name + " (twice)", c, s, factor=2.0)


def test_static_entry_point_edge_cases(torch_cuda):
    """No positions: the gradient is zeroed and the loss is 0.  A window outside the object is skipped
    on the device without a memory access (loss 0 for it), as by ptycho_loss_grad, whose context
    reports it in its status word."""
    import torch
    import paper_2205_06327_amd as pt
    name, spec = CALLS["m128"][1]
    d = problem(spec)
    t = to_dev(d)
    say(f"static entry point, no positions: {name}")
    grad = torch.full_like(t["obj"], complex(5.0, 5.0))
    loss = torch.full((1,), 7.0, dtype=torch.float64, device="cuda:0")
    empty_pos = torch.zeros((0, 2), dtype=torch.int32, device="cuda:0")
    empty_meas = torch.zeros((0, spec.M, spec.M), dtype=torch.float32, device="cuda:0")
    pt.ptycho_loss_grad_static(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A, t["obj"], t["probe"], empty_pos,
                               empty_meas, grad=grad, loss=loss)
    torch.cuda.synchronize()
    assert float(loss.item()) == 0.0 and not bool(grad.abs().gt(0).any())
    say(f"static entry point, one window outside the object: {name}")
    pos = t["pos"].clone()
    pos[1, 1] = spec.W - spec.M + 1  # one column past the right edge
    n = pos.shape[0]
    ctx = context(spec, n)
    lpp_c = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    loss_c, grad_c = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], pos, t["meas"], loss_per_pos=lpp_c)
    with pytest.raises(pt.PtychoError) as e:
        ctx.check()
    assert e.value.name == "PTYCHO_E_BOUNDS"
    lpp_s = torch.full((n,), -1.0, dtype=torch.float64, device="cuda:0")
    loss_s, grad_s = pt.ptycho_loss_grad_static(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A, t["obj"],
                                                t["probe"], pos, t["meas"], loss_per_pos=lpp_s)
    torch.cuda.synchronize()
    c = (float(loss_c.item()), lpp_c.cpu().numpy(), grad_c.cpu().numpy())
    s = (float(loss_s.item()), lpp_s.cpu().numpy(), grad_s.cpu().numpy())
    assert s[1][1] == 0.0 and c[1][1] == 0.0
    check_pair(name + " (one window outside)", c, s)
    ctx.close()
