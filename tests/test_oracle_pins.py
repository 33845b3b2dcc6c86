"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test checks the oracle against a closed form, a brute-force definition,
an invariance of the physics, or a derivative identity, chosen so that a
plausible slip (wrong FFT sign or normalisation, swapped window axes, a
missing propagation, a conjugate in the wrong place, a dropped term of the
adjoint) breaks at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import ptycho_synth as ps

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAM, DZ, PIX = 0.0197, 2.0, 0.1


# --- independent brute-force helpers (explicit sums, no FFT library) ---------
def dft_matrix(M):
    q = np.arange(M)
    return np.exp(-2j * np.pi * np.outer(q, q) / M)


def bf_dft2(x):
    D = dft_matrix(x.shape[0])
    return D @ x @ D.T


def bf_idft2(X):
    M = X.shape[0]
    Dc = np.conj(dft_matrix(M))
    return Dc @ X @ Dc.T / (M * M)


def bf_freq(M, pixel):
    q = np.arange(M)
    q = np.where(q < M // 2, q, q - M)   # even M: 0..M/2-1, -M/2..-1
    return q / (M * pixel)


def bf_propagator(M, lam, dz, pixel):
    k = bf_freq(M, pixel)
    return np.exp(-1j * np.pi * lam * dz * (k[:, None] ** 2 + k[None, :] ** 2))


def bf_far_field(obj, probe, y0, x0, lam, dz, pixel):
    """Multislice by explicit DFT sums: transmit, propagate between slices, far field."""
    M = probe.shape[0]
    Hb = bf_propagator(M, lam, dz, pixel)
    psi = probe.astype(np.complex128)
    S = obj.shape[0]
    for s in range(S):
        phi = psi * obj[s, y0:y0 + M, x0:x0 + M]
        if s < S - 1:
            psi = bf_idft2(Hb * bf_dft2(phi))
    return bf_dft2(phi)


def bf_intensity(obj, probe, y0, x0, lam, dz, pixel):
    return np.abs(bf_far_field(obj, probe, y0, x0, lam, dz, pixel)) ** 2


def rand_complex(rng, shape, lo=0.5, hi=1.5):
    return rng.uniform(lo, hi, shape) * np.exp(1j * rng.uniform(-np.pi, np.pi, shape))


def tiny_problem(seed=0, M=8, S=3, W=12, ny=3, nx=3, step=2, phase_only=False):
    rng = np.random.default_rng(seed)
    if phase_only:
        obj = np.exp(1j * rng.uniform(-1, 1, (S, W, W)))
    else:
        obj = rand_complex(rng, (S, W, W))
    probe = rand_complex(rng, (M, M))
    pos = ps.raster_positions(W, M, ny, nx, step)
    return rng, obj, probe, pos


# --- forward model ---------------------------------------------------------
@pytest.mark.parametrize("M,S", [(4, 1), (4, 2), (8, 1), (8, 3), (16, 2)])
def test_forward_matches_bruteforce_dft(M, S):
    rng, obj, probe, pos = tiny_problem(seed=M * 10 + S, M=M, S=S, W=M + 4, ny=2, nx=3, step=2)
    H = oracle.fresnel_propagator(M, LAM, DZ, PIX)
    I = oracle.forward(obj, probe, pos, H)
    for i, (y0, x0) in enumerate(pos):
        ref = bf_intensity(obj, probe, int(y0), int(x0), LAM, DZ, PIX)
        np.testing.assert_allclose(I[i], ref, rtol=1e-11, atol=1e-11 * ref.max())


def test_propagator_is_paraxial_angular_spectrum():
    # Exact free-space transfer exp(2 pi i dz (sqrt(1/lam^2 - k^2) - 1/lam)) differs from the
    # paraxial one by a phase pi lam^3 dz k^4 / 4 + O(lam^5 dz k^6): pins sign and the pi*lam*dz factor.
    for M in (64, 128):
        H = oracle.fresnel_propagator(M, LAM, DZ, PIX)
        k = bf_freq(M, PIX)
        k2 = k[:, None] ** 2 + k[None, :] ** 2
        # sqrt(1/lam^2 - k^2) - 1/lam written without cancellation.
        kz_minus = -k2 / (np.sqrt(1.0 / LAM ** 2 - k2) + 1.0 / LAM)
        exact = np.exp(2j * np.pi * DZ * kz_minus)
        dphase = np.angle(H / exact)
        lead = np.pi * LAM ** 3 * DZ * k2 ** 2 / 4.0
        nxt = np.pi * LAM ** 5 * DZ * k2 ** 3 / 8.0
        assert np.all(np.abs(dphase - lead) <= 1.5 * nxt + 1e-13)
        assert np.abs(dphase).max() > 1e-7  # the check is not vacuous
        assert np.allclose(np.abs(H), 1.0, atol=1e-15)


@pytest.mark.parametrize("S", [1, 3])
def test_parseval_phase_object(S):
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=128, ny=4, nx=4, S=S, strength=0.7)
    d = ps.build_inputs(spec, with_eval=False)
    H = oracle.fresnel_propagator(spec.M, LAM, DZ, PIX)
    I = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    np.testing.assert_allclose(I.sum(axis=(1, 2)), spec.dose, rtol=1e-12)


def _aperture_count(R):
    # Lattice points with a^2 + b^2 <= R^2, summed column by column.
    r = int(math.floor(R))
    return sum(2 * int(math.floor(math.sqrt(R * R - a * a))) + 1 for a in range(-r, r + 1))


def test_aperture_counts_golden():
    with open(os.path.join(GOLDEN, "aperture_counts.json")) as f:
        g = json.load(f)
    for row in g["counts"]:
        assert _aperture_count(row["R"]) == row["N"]


@pytest.mark.parametrize("S,M,R,C", [(1, 64, 12.0, 2.0), (3, 64, 12.0, 2.0), (2, 128, 20.0, 4.0)])
def test_flat_object_closed_form(S, M, R, C):
    # t == 1: |Psi| = |F(P)| (propagators have unit modulus), and |F(P)|^2 = D * A(q) / N_A.
    dose = 1e5
    W = M + 20
    obj = np.ones((S, W, W), dtype=np.complex128)
    probe = ps.make_probe(M, R, C, dose)
    pos = np.array([[0, 0], [3, 17], [20, 5]], dtype=np.int32)
    H = oracle.fresnel_propagator(M, LAM, DZ, PIX)
    I = oracle.forward(obj, probe, pos, H)
    q = np.fft.fftfreq(M) * M
    A = (q[:, None] ** 2 + q[None, :] ** 2) <= R * R
    expect = dose * A / _aperture_count(R)
    for i in range(len(pos)):
        np.testing.assert_allclose(I[i], expect, rtol=1e-9, atol=1e-9 * dose)


def test_localised_absorber_orientation():
    # An absorber at (row 40, col 20) changes only windows that contain that pixel; a window
    # containing the transposed pixel (row 20, col 40) must keep the flat-object pattern.
    M, W, S = 16, 64, 2
    obj = np.ones((S, W, W), dtype=np.complex128)
    yy, xx = np.mgrid[0:W, 0:W]
    obj[1][(yy - 40) ** 2 + (xx - 20) ** 2 <= 2] = 0.3
    probe = ps.make_probe(M, 4.0, 1.0, 1e4)
    pos = np.array([[30, 10], [12, 32], [0, 0]], dtype=np.int32)
    H = oracle.fresnel_propagator(M, LAM, DZ, PIX)
    I = oracle.forward(obj, probe, pos, H)
    flat = oracle.forward(np.ones_like(obj), probe, pos, H)
    assert np.max(np.abs(I[0] - flat[0])) > 1e-3 * flat[0].max()
    np.testing.assert_allclose(I[1], flat[1], rtol=0, atol=1e-9 * flat[1].max())
    np.testing.assert_allclose(I[2], flat[2], rtol=0, atol=1e-9 * flat[2].max())


def test_slice_order_special_cases():
    rng, obj, probe, pos = tiny_problem(seed=7, M=16, S=2, W=24, ny=2, nx=2, step=8)
    H = oracle.fresnel_propagator(16, LAM, DZ, PIX)
    # (a) flat last slice: the wave meets slice 0 directly and the last propagation is invisible.
    o = obj.copy()
    o[1] = 1.0
    I = oracle.forward(o, probe, pos, H)
    for i, (y0, x0) in enumerate(pos):
        ref = np.abs(bf_dft2(probe * obj[0, y0:y0 + 16, x0:x0 + 16])) ** 2
        np.testing.assert_allclose(I[i], ref, rtol=1e-11, atol=1e-11 * ref.max())
    # (b) flat first slice: slice 1 sees the probe propagated by one slice thickness.
    o = obj.copy()
    o[0] = 1.0
    I = oracle.forward(o, probe, pos, H)
    p_dz = bf_idft2(bf_propagator(16, LAM, DZ, PIX) * bf_dft2(probe))
    for i, (y0, x0) in enumerate(pos):
        ref = np.abs(bf_dft2(p_dz * obj[1, y0:y0 + 16, x0:x0 + 16])) ** 2
        np.testing.assert_allclose(I[i], ref, rtol=1e-11, atol=1e-11 * ref.max())
    # (c) zero slice thickness: the slices collapse into one with the product transmission.
    H0 = oracle.fresnel_propagator(16, LAM, 0.0, PIX)
    I = oracle.forward(obj, probe, pos, H0)
    J = oracle.forward(obj.prod(axis=0, keepdims=True), probe, pos, H0)
    np.testing.assert_allclose(I, J, rtol=1e-11, atol=1e-11 * J.max())


def test_translation_covariance():
    rng, obj, probe, pos = tiny_problem(seed=3, M=8, S=3, W=20, ny=2, nx=2, step=3)
    H = oracle.fresnel_propagator(8, LAM, DZ, PIX)
    I = oracle.forward(obj, probe, pos, H)
    shifted = np.roll(obj, (0, 3, 5), axis=(0, 1, 2))
    J = oracle.forward(shifted, probe, pos + np.array([3, 5], dtype=np.int32), H)
    np.testing.assert_allclose(I, J, rtol=1e-12, atol=1e-12 * I.max())


# --- loss and gradient -----------------------------------------------------
def _meas_for(obj, probe, pos, H, rng, jitter=0.3):
    I = oracle.forward(obj, probe, pos, H)
    return I * rng.uniform(1 - jitter, 1 + jitter, I.shape)


def test_global_phase_rotates_only_that_slice_gradient():
    rng, obj, probe, pos = tiny_problem(seed=11, M=8, S=3)
    H = oracle.fresnel_propagator(8, LAM, DZ, PIX)
    meas = _meas_for(obj, probe, pos, H, rng)
    L0, _, G0 = oracle.loss_and_gradient(obj, probe, pos, meas, H)
    th = 0.7
    o = obj.copy()
    o[1] *= np.exp(1j * th)
    L1, _, G1 = oracle.loss_and_gradient(o, probe, pos, meas, H)
    assert abs(L1 - L0) <= 1e-12 * abs(L0)
    sc = np.abs(G0).max()
    np.testing.assert_allclose(G1[1], np.exp(1j * th) * G0[1], atol=1e-11 * sc)
    np.testing.assert_allclose(G1[0], G0[0], atol=1e-11 * sc)
    np.testing.assert_allclose(G1[2], G0[2], atol=1e-11 * sc)


def test_central_finite_differences():
    rng, obj, probe, pos = tiny_problem(seed=5, M=8, S=3)
    H = oracle.fresnel_propagator(8, LAM, DZ, PIX)
    meas = _meas_for(obj, probe, pos, H, rng)
    _, _, G = oracle.loss_and_gradient(obj, probe, pos, meas, H)
    h = 1e-6
    fd = np.zeros_like(G)
    for idx in np.ndindex(obj.shape):
        for part, unit in ((0, 1.0), (1, 1j)):
            op = obj.copy()
            om = obj.copy()
            op[idx] += h * unit
            om[idx] -= h * unit
            d = (oracle.loss_and_gradient(op, probe, pos, meas, H)[0]
                 - oracle.loss_and_gradient(om, probe, pos, meas, H)[0]) / (2 * h)
            fd[idx] += d * unit
    np.testing.assert_allclose(G, fd, rtol=0, atol=2e-6 * np.abs(G).max())


@pytest.mark.parametrize("S", [1, 3])
def test_adjoint_dot_product(S):
    """Eq. 2 as an adjoint identity.  With the other slices fixed, the far field
    of one position is complex-linear in slice s's window (and in the probe), so
    dPsi = J_s dt exactly, with J_s dt the far field of the object whose window
    on slice s is replaced by dt.  Since dF = Re sum conj(g) dPsi with
    g = 2(|Psi| - a) Psi/|Psi|, the gradient G_s must satisfy
    Re<g, J_s dt> = Re<G_s, dt> for every dt.  J_s dt is evaluated by explicit
    DFT sums, so a missing conjugate of H, a wrong M^2, a swapped slice or a
    conjugated incident wave in the oracle's adjoint breaks the identity."""
    rng = np.random.default_rng(31 + S)
    M, W, y0, x0 = 8, 12, 3, 2
    obj = rand_complex(rng, (S, W, W))
    probe = rand_complex(rng, (M, M))
    H = oracle.fresnel_propagator(M, LAM, DZ, PIX)
    far = bf_far_field(obj, probe, y0, x0, LAM, DZ, PIX)
    meas = rng.uniform(0.2, 2.0, (M, M)) * np.abs(far) ** 2
    g = 2.0 * (np.abs(far) - np.sqrt(meas)) * far / np.abs(far)
    _, grads = oracle.position_loss_and_patch_gradients(obj, probe, y0, x0, meas, H)
    for s in range(S):
        dt = rand_complex(rng, (M, M))
        o2 = obj.copy()
        o2[s, y0:y0 + M, x0:x0 + M] = dt
        lhs = np.real(np.vdot(g, bf_far_field(o2, probe, y0, x0, LAM, DZ, PIX)))
        rhs = np.real(np.vdot(grads[s], dt))
        scale = np.linalg.norm(grads[s]) * np.linalg.norm(dt)
        assert abs(lhs - rhs) <= 1e-11 * scale, (s, lhs, rhs)
    dP = rand_complex(rng, (M, M))
    lhs = np.real(np.vdot(g, bf_far_field(obj, dP, y0, x0, LAM, DZ, PIX)))
    GP = oracle.probe_gradient(obj, probe, np.array([[y0, x0]]), meas[None], H)
    rhs = np.real(np.vdot(GP, dP))
    assert abs(lhs - rhs) <= 1e-11 * np.linalg.norm(GP) * np.linalg.norm(dP), (lhs, rhs)


def test_torch_autograd_cross_check():
    torch = pytest.importorskip("torch")
    rng, obj, probe, pos = tiny_problem(seed=9, M=8, S=3)
    H = oracle.fresnel_propagator(8, LAM, DZ, PIX)
    meas = _meas_for(obj, probe, pos, H, rng)
    _, _, G = oracle.loss_and_gradient(obj, probe, pos, meas, H)
    t = torch.tensor(obj, dtype=torch.complex128, requires_grad=True)
    P = torch.tensor(probe, dtype=torch.complex128, requires_grad=True)
    Ht = torch.tensor(H, dtype=torch.complex128)
    loss = 0.0
    for i, (y0, x0) in enumerate(pos):
        psi = P
        for s in range(obj.shape[0]):
            phi = psi * t[s, y0:y0 + 8, x0:x0 + 8]
            if s < obj.shape[0] - 1:
                psi = torch.fft.ifft2(Ht * torch.fft.fft2(phi))
        amp = torch.abs(torch.fft.fft2(phi))
        loss = loss + torch.sum((amp - torch.sqrt(torch.tensor(meas[i]))) ** 2)
    loss.backward()
    np.testing.assert_allclose(t.grad.numpy(), G, rtol=0, atol=1e-12 * np.abs(G).max())
    GP = oracle.probe_gradient(obj, probe, pos, meas, H)
    np.testing.assert_allclose(P.grad.numpy(), GP, rtol=0, atol=1e-12 * np.abs(GP).max())


def test_zero_gradient_at_truth_and_locality():
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=96, ny=3, nx=3, step=12, S=2, M=32, R=6.0)
    d = ps.build_inputs(spec)
    H = oracle.fresnel_propagator(spec.M, LAM, DZ, PIX)
    meas = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    L_t, _, G_t = oracle.loss_and_gradient(d["obj_true"], d["probe"], d["pos"], meas, H)
    L_e, _, G_e = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], meas, H)
    assert L_t <= 1e-20 * spec.dose * len(d["pos"]) + 1e-18
    assert np.abs(G_t).max() <= 1e-9 * np.abs(G_e).max()
    cover = np.zeros((spec.W, spec.W), dtype=bool)
    for y0, x0 in d["pos"]:
        cover[y0:y0 + spec.M, x0:x0 + spec.M] = True
    assert np.all(G_e[:, ~cover] == 0)
    assert np.abs(G_e[:, cover]).max() > 0


# --- decomposition ---------------------------------------------------------
def test_tile_binning_bruteforce_full_scan_geometry():
    spec = ps.workload("ms16-2048-m128-tiles4x4")
    pos = ps.raster_positions(spec.W, spec.M, spec.ny, spec.nx, spec.step)
    owner = oracle.bin_positions(pos, spec.W, spec.W, spec.M, 4, 4)
    counts = np.bincount(owner, minlength=16)
    assert counts.sum() == 16632
    assert counts.min() == 754 and counts.max() == 1369
    T = spec.W // 4
    for i in range(0, len(pos), 7):
        cy, cx = pos[i][0] + 64, pos[i][1] + 64
        hits = [ty * 4 + tx for ty in range(4) for tx in range(4)
                if ty * T <= cy < (ty + 1) * T and tx * T <= cx < (tx + 1) * T]
        assert hits == [owner[i]]
        ty, tx = divmod(int(owner[i]), 4)
        ey0, ey1, ex0, ex1 = oracle.extended_box(spec.W, spec.W, 4, 4, ty, tx, spec.halo)
        assert ey0 <= pos[i][0] and pos[i][0] + 128 <= ey1 and ex0 <= pos[i][1] and pos[i][1] + 128 <= ex1


def test_decomposed_gradient_sums_to_global():
    rng, obj, probe, pos = tiny_problem(seed=13, M=16, S=2, W=96, ny=9, nx=9, step=10)
    H = oracle.fresnel_propagator(16, LAM, DZ, PIX)
    meas = _meas_for(obj, probe, pos, H, rng)
    L, _, G = oracle.loss_and_gradient(obj, probe, pos, meas, H)
    parts = [oracle.tile_gradient(obj, probe, pos, meas, H, (2, 3), 8, ty, tx)
             for ty in range(2) for tx in range(3)]
    assert sorted(np.concatenate([p["positions"] for p in parts]).tolist()) == list(range(len(pos)))
    Gs = oracle.stitch_tile_gradients(obj.shape, parts)
    np.testing.assert_allclose(Gs, G, rtol=0, atol=1e-12 * np.abs(G).max())
    assert abs(sum(p["loss"] for p in parts) - L) <= 1e-12 * L
    with pytest.raises(ValueError):
        oracle.tile_gradient(obj, probe, pos, meas, H, (2, 3), 4, 1, 1)


@pytest.mark.parametrize("S", [2, 8])
def test_gradient_descent_decreases_loss(S):
    # With eight slices the single-slice step (no factor S) oscillates on this
    # problem; the bound over all slices descends monotonically.
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=64, ny=5, nx=5, step=6, S=S, M=32, R=6.0, C=1.0,
                             strength=0.5)
    d = ps.build_inputs(spec)
    H = oracle.fresnel_propagator(spec.M, LAM, DZ, PIX)
    meas = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    alpha = oracle.gd_step_size(d["probe"], d["pos"], spec.W, spec.W, spec.S)
    t = ps.eval_object(d["obj_true"], spec.pitch, np.random.SeedSequence(99), amp=0.3)
    losses = []
    for _ in range(8):
        L, _, G = oracle.loss_and_gradient(t, d["probe"], d["pos"], meas, H)
        losses.append(L)
        t = oracle.gd_step(t, G, alpha)
    assert all(b < a for a, b in zip(losses, losses[1:]))
    assert losses[-1] < 0.8 * losses[0]
    if S == 8:  # the step without the slice factor does not descend here
        t = ps.eval_object(d["obj_true"], spec.pitch, np.random.SeedSequence(99), amp=0.3)
        big = []
        for _ in range(8):
            L, _, G = oracle.loss_and_gradient(t, d["probe"], d["pos"], meas, H)
            big.append(L)
            t = oracle.gd_step(t, G, alpha * S)
        assert not all(b < a for a, b in zip(big, big[1:]))


def _random_tile_buffers(W, S, tiles, halo, seed):
    rng = np.random.default_rng(seed)
    out = []
    for ty in range(tiles[0]):
        for tx in range(tiles[1]):
            box = oracle.extended_box(W, W, tiles[0], tiles[1], ty, tx, halo)
            shape = (S, box[1] - box[0], box[3] - box[2])
            out.append({"box": box, "grad": rng.standard_normal(shape) + 1j * rng.standard_normal(shape)})
    return out


@pytest.mark.parametrize("W,tiles,halo", [
    (192, (3, 3), 16),   # tile 64 >= 2 * halo: only direct neighbours overlap
    (192, (4, 4), 32),   # tile 48 < 2 * halo: tiles two apart overlap too
    (200, (3, 5), 40),   # uneven tiles (66-67 by 40 px), 40 px halo: 2-apart overlaps along x only
])
def test_directional_passes_leave_the_global_sum_on_every_box(W, tiles, halo):
    S = 2
    bufs = _random_tile_buffers(W, S, tiles, halo, seed=W + halo)
    total = oracle.stitch_tile_gradients((S, W, W), bufs)
    acc = oracle.directional_passes(bufs, tiles)
    for b, a in zip(bufs, acc):
        ey0, ey1, ex0, ex1 = b["box"]
        np.testing.assert_allclose(a["grad"], total[:, ey0:ey1, ex0:ex1], rtol=0, atol=1e-12 * np.abs(total).max())
    # the single direct-neighbour exchange of Section III is exact only when no two
    # non-adjacent tiles overlap (tile >= 2 * halo on both axes)
    nb = oracle.neighbour_add(bufs, tiles)
    exact = all(np.allclose(n["grad"], total[:, n["box"][0]:n["box"][1], n["box"][2]:n["box"][3]], rtol=0,
                            atol=1e-12 * np.abs(total).max()) for n in nb)
    t_min = min(W // tiles[0], W // tiles[1])
    assert exact == (t_min >= 2 * halo)


def test_directional_passes_on_physical_tile_gradients():
    # 16-windows, 4 x 4 tiles of 12-13 px with an 8 px halo (= M/2), so tiles two apart overlap;
    # every tile's buffer must end with the undecomposed gradient on its box
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=50, ny=5, nx=5, step=7, S=2, M=16, R=4.0, C=1.0,
                             strength=0.3)
    d = ps.build_inputs(spec, with_eval=True)
    H = oracle.fresnel_propagator(spec.M, LAM, DZ, PIX)
    meas = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    tiles, halo = (4, 4), 8
    parts = [oracle.tile_gradient(d["obj_eval"], d["probe"], d["pos"], meas, H, tiles, halo, ty, tx)
             for ty in range(4) for tx in range(4)]
    assert sum(len(p["positions"]) for p in parts) == len(d["pos"])
    G = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], meas, H)[2]
    acc = oracle.directional_passes(parts, tiles)
    for a in acc:
        ey0, ey1, ex0, ex1 = a["box"]
        np.testing.assert_allclose(a["grad"], G[:, ey0:ey1, ex0:ex1], rtol=0, atol=1e-12 * np.abs(G).max())


def _alg1_problem():
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=56, ny=5, nx=5, step=6, S=2, M=16, R=4.0, C=1.0,
                             strength=0.3)
    d = ps.build_inputs(spec, with_eval=True)
    H = oracle.fresnel_propagator(spec.M, LAM, DZ, PIX)
    meas = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    return spec, d, H, meas


def test_alg1_single_tile_full_batch_is_gradient_descent_with_double_step():
    # one tile holding every position, one batch per iteration: the per-batch step and the
    # step with the (identical) accumulated buffer add up to one gradient step of 2 * step
    spec, d, H, meas = _alg1_problem()
    alpha = oracle.gd_step_size(d["probe"], d["pos"], spec.W, spec.W, spec.S)
    losses, V = oracle.alg1_tiles(d["obj_eval"], d["probe"], d["pos"], meas, H, (1, 1), 8, alpha,
                                  batch=len(d["pos"]), T=1, iterations=3)
    t = d["obj_eval"].astype(np.complex128)
    ref = []
    for _ in range(3):
        L, _, G = oracle.loss_and_gradient(t, d["probe"], d["pos"], meas, H)
        ref.append(L)
        t = oracle.gd_step(t, G, 2 * alpha)
    np.testing.assert_allclose(losses, ref, rtol=1e-12)
    np.testing.assert_allclose(V, t, rtol=0, atol=1e-12)


@pytest.mark.parametrize("batch,T", [(1, 1), (2, 3), (4, 100)])
def test_alg1_tiles_descend(batch, T):
    # 4 x 4 tiles of 14 px with an 8 px halo (tiles two apart overlap): the loss falls every
    # iteration for per-probe updates, delayed accumulation and once-per-iteration passes
    spec, d, H, meas = _alg1_problem()
    alpha = 0.5 * oracle.gd_step_size(d["probe"], d["pos"], spec.W, spec.W, spec.S)
    losses, V = oracle.alg1_tiles(d["obj_eval"], d["probe"], d["pos"], meas, H, (4, 4), 8, alpha,
                                  batch=batch, T=T, iterations=4)
    assert all(b < a for a, b in zip(losses, losses[1:]))
    assert oracle.loss_and_gradient(V, d["probe"], d["pos"], meas, H)[0] < losses[0]


def test_potential_gradient_by_central_differences():
    # F(V) = F(exp(i sigma V)) on a tiny 2-slice problem; the chain rule against central
    # differences on a few voxels of the real potential
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=24, ny=2, nx=2, step=4, S=2, M=16, R=4.0, C=1.0,
                             strength=0.3)
    d = ps.build_inputs(spec)
    H = oracle.fresnel_propagator(spec.M, LAM, DZ, PIX)
    meas = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    sigma = 0.7
    rng = np.random.default_rng(5)
    V = rng.uniform(0.0, 0.5, size=(2, spec.W, spec.W))
    t = oracle.transmission_from_potential(V, sigma)
    G = oracle.loss_and_gradient(t, d["probe"], d["pos"], meas, H)[2]
    gV = oracle.potential_gradient(t, G, sigma)
    h = 1e-6
    for s_, y, x in [(0, 9, 9), (1, 12, 7), (0, 5, 14), (1, 17, 17)]:
        Vp, Vm = V.copy(), V.copy()
        Vp[s_, y, x] += h
        Vm[s_, y, x] -= h
        Fp = oracle.loss_and_gradient(oracle.transmission_from_potential(Vp, sigma), d["probe"], d["pos"], meas, H)[0]
        Fm = oracle.loss_and_gradient(oracle.transmission_from_potential(Vm, sigma), d["probe"], d["pos"], meas, H)[0]
        fd = (Fp - Fm) / (2 * h)
        assert abs(fd - gV[s_, y, x]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7 * np.abs(gV).max()


# --- sub-pixel positions (probe translated by a fraction of a pixel) --------
def test_shift_probe_integer_shift_is_a_cyclic_roll():
    rng = np.random.default_rng(41)
    P = rand_complex(rng, (16, 16))
    for dy, dx in [(2, -3), (0, 5), (-7, 0), (15, 1)]:
        np.testing.assert_allclose(oracle.shift_probe(P, dy, dx), np.roll(P, (dy, dx), axis=(0, 1)),
                                   rtol=0, atol=1e-12)


def test_shift_probe_single_fourier_mode_closed_form():
    """A single Fourier mode exp(2 pi i f.r / M) translated by any real d is exp(2 pi i f.(r - d) / M):
    pins the sign of the ramp and the integer-frequency convention (evaluated by explicit DFT sums
    as well as by the oracle)."""
    M = 16
    r = np.arange(M)
    for fy, fx in [(1, 0), (-3, 2), (7, -7), (0, -1)]:
        P = np.exp(2j * np.pi * (fy * r[:, None] + fx * r[None, :]) / M)
        for dy, dx in [(0.25, 0.0), (0.5, 0.75), (-0.3, 0.9), (1.5, -2.25)]:
            want = np.exp(2j * np.pi * (fy * (r[:, None] - dy) + fx * (r[None, :] - dx)) / M)
            np.testing.assert_allclose(oracle.shift_probe(P, dy, dx), want, rtol=0, atol=1e-12)
            q = np.where(r < M // 2, r, r - M)  # integer frequencies, -M/2 at the Nyquist bin
            ramp = np.exp(-2j * np.pi * (q[:, None] * dy + q[None, :] * dx) / M)
            np.testing.assert_allclose(bf_idft2(bf_dft2(P) * ramp), want, rtol=0, atol=1e-11)


def test_shift_probe_composes_and_is_unitary():
    rng = np.random.default_rng(43)
    P = rand_complex(rng, (32, 32))
    a = oracle.shift_probe(oracle.shift_probe(P, 0.3, -0.45), 0.5, 0.2)
    np.testing.assert_allclose(a, oracle.shift_probe(P, 0.8, -0.25), rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.shift_probe(oracle.shift_probe(P, 0.37, 0.61), -0.37, -0.61), P,
                               rtol=0, atol=1e-12)
    assert abs(np.linalg.norm(oracle.shift_probe(P, 0.37, 0.61)) - np.linalg.norm(P)) <= 1e-12 * np.linalg.norm(P)


def test_subpixel_model_reduces_to_the_integer_model():
    rng, obj, probe, pos = tiny_problem(seed=44, M=8, S=3)
    H = oracle.fresnel_propagator(8, LAM, DZ, PIX)
    meas = _meas_for(obj, probe, pos, H, rng)
    posf = pos.astype(np.float64)
    corner, frac = oracle.split_subpixel(posf + 0.0)
    assert np.array_equal(corner, pos) and not frac.any()
    np.testing.assert_allclose(oracle.forward_subpixel(obj, probe, posf, H), oracle.forward(obj, probe, pos, H),
                               rtol=0, atol=1e-12)
    L0, _, G0 = oracle.loss_and_gradient(obj, probe, pos, meas, H)
    L1, _, G1 = oracle.loss_and_gradient_subpixel(obj, probe, posf, meas, H)
    assert abs(L1 - L0) <= 1e-12 * L0  # the zero shift is the identity up to FFT rounding
    np.testing.assert_allclose(G1, G0, rtol=0, atol=1e-12 * np.abs(G0).max())
    # a fraction goes to the probe, the integer part to the window corner
    corner, frac = oracle.split_subpixel(np.array([[2.25, 3.5], [0.0, 1.75]]))
    assert corner.tolist() == [[2, 3], [0, 1]] and np.allclose(frac, [[0.25, 0.5], [0.0, 0.75]])


def test_subpixel_gradient_by_central_differences():
    rng, obj, probe, pos = tiny_problem(seed=45, M=8, S=2)
    H = oracle.fresnel_propagator(8, LAM, DZ, PIX)
    posf = pos.astype(np.float64) + rng.uniform(0.0, 1.0, pos.shape)
    posf = np.minimum(posf, obj.shape[1] - 8)  # windows stay inside the object
    meas = oracle.forward_subpixel(obj, probe, posf, H) * rng.uniform(0.5, 1.5, (len(pos), 8, 8))
    _, _, G = oracle.loss_and_gradient_subpixel(obj, probe, posf, meas, H)
    h = 1e-6
    fd = np.zeros_like(G)
    for idx in np.ndindex(obj.shape):
        for unit in (1.0, 1j):
            op, om = obj.copy(), obj.copy()
            op[idx] += h * unit
            om[idx] -= h * unit
            d = (oracle.loss_and_gradient_subpixel(op, probe, posf, meas, H)[0]
                 - oracle.loss_and_gradient_subpixel(om, probe, posf, meas, H)[0]) / (2 * h)
            fd[idx] += d * unit
    np.testing.assert_allclose(G, fd, rtol=0, atol=2e-6 * np.abs(G).max())
