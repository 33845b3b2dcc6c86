"""Plain FP64 CPU oracle for gradient-decomposed multislice ptychography.

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct
reference that the GPU path is checked against.  Only the test suite, the
package smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.  It shares no code, table or helper with the HIP
library: it is written directly from the paper's statement of the problem
with numpy's FFT as the only library primitive.

What it computes (per probe location i with window top-left corner (y0, x0)):

* Multislice model G (Section II-B, the paragraph after Eq. 1): the incident
  wave is the probe; at each slice the wave is multiplied by the slice's
  transmission over the window, then propagated to the next slice by a Fourier
  transform, a multiplication by the Fresnel propagator and an inverse Fourier
  transform; the output of one slice feeds the next.  The detector sees the
  Fourier transform of the last exit wave.
* Amplitude cost (Eq. 1): f_i = sum_q (|y_i| - |G(p_i, V)|)^2 with |y_i| the
  square root of the measured intensity (reading of |y_i| as the measured
  amplitude) and the modulus taken per detector pixel.
* Gradient (Eq. 2): dF/dV = sum_i df_i/dV, each term non-zero only inside
  window i (Section III).  The complex gradient is dF/dRe t + i dF/dIm t with
  respect to the complex slice transmissions t_s.
* Decomposition (Section III; the tile/halo construction): positions are
  assigned to tiles, each tile accumulates the gradients of its own positions
  on its halo-extended box, and the global gradient is the sum of the embedded
  tile gradients (the one-device form of the neighbour add and the final
  stitch of Alg. 1).
* Full-batch gradient descent t <- t - alpha * G (Section II-B, last paragraph
  of the formulation; the tile update of Alg. 1).

Conventions: F is the unnormalised forward DFT (numpy ``fft2``); F^-1 carries
1/M^2 (numpy ``ifft2``); frequencies are ``fftfreq(M, d=pixel)``; the
propagator is H = exp(-i pi lambda dz |k|^2); intensities are in unshifted DFT
order (DC at [0, 0]).

Pins (tests/test_oracle_pins.py): brute-force DFT sums on tiny grids,
Parseval, the flat-object closed form, a localised absorber (window
orientation), propagator vs the exact angular-spectrum phase, slice-order
special cases, translation and global-phase covariance, zero gradient at the
truth, central finite differences, the adjoint dot-product identity, torch
autograd on tiny grids, the decomposition sum, tile binning by brute force,
the directional passes and the neighbour add against the summed tile
gradients (exact only with tile >= 2 halo for the neighbour add), monotone
descent, and the Alg. 1 schedule of ``alg1_tiles`` in closed form
(tests/test_oracle_alg1.py: one batch per tile, and two batches with the
passes after each batch or after both, for tiles at least and less than twice
the halo, built from the global gradient, the tile gradients and the passes'
exactness; planted schedule mistakes fail them).  ``gd_step_size`` is a reading (the paper states no step
size): its descent property is tested, its value is not pinned ("parity
unpinned" for the step length itself).
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np

__all__ = [
    "fresnel_propagator",
    "exit_waves",
    "forward",
    "loss_and_gradient",
    "position_loss_and_patch_gradients",
    "probe_gradient",
    "tile_bounds",
    "bin_positions",
    "extended_box",
    "tile_gradient",
    "stitch_tile_gradients",
    "gd_step_size",
    "shift_probe",
    "split_subpixel",
    "forward_subpixel",
    "loss_and_gradient_subpixel",
    "transmission_from_potential",
    "potential_gradient",
    "neighbour_add",
    "directional_passes",
    "alg1_tiles",
    "gd_step",
]


# ---------------------------------------------------------------------------
# Physics: the Fresnel propagator between slices (Section II-B; the propagator
# form exp(-i pi lambda dz |k|^2) is the paraxial free-space transfer function).
# ---------------------------------------------------------------------------
def fresnel_propagator(M: int, wavelength: float, dz: float, pixel: float) -> np.ndarray:
    """H[ky, kx] = exp(-i pi lambda dz (ky^2 + kx^2)), k = fftfreq(M, d=pixel); complex128 [M, M]."""
    k = np.fft.fftfreq(M, d=pixel)
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    return np.exp(-1j * math.pi * wavelength * dz * k2)


def _window(obj_slice: np.ndarray, y0: int, x0: int, M: int) -> np.ndarray:
    if y0 < 0 or x0 < 0 or y0 + M > obj_slice.shape[0] or x0 + M > obj_slice.shape[1]:
        raise ValueError(f"window ({y0},{x0})+{M} outside object {obj_slice.shape}")
    return obj_slice[y0:y0 + M, x0:x0 + M]


# ---------------------------------------------------------------------------
# Multislice forward model G(p_i, V) (Section II-B).
# ---------------------------------------------------------------------------
def exit_waves(obj: np.ndarray, probe: np.ndarray, y0: int, x0: int, H: np.ndarray
               ) -> Tuple[List[np.ndarray], np.ndarray]:
    """Incident waves psi_0..psi_{S-1} at each slice and the far field Psi for one window.

    psi_0 is the probe; phi_s = psi_s * t_s[window]; psi_{s+1} = F^-1(H F(phi_s));
    Psi = F(phi_{S-1}).
    """
    M = probe.shape[0]
    S = obj.shape[0]
    psi = np.asarray(probe, dtype=np.complex128)
    incident = []
    phi = None
    for s in range(S):
        incident.append(psi)
        phi = psi * _window(obj[s], y0, x0, M)
        if s < S - 1:
            psi = np.fft.ifft2(H * np.fft.fft2(phi))
    far_field = np.fft.fft2(phi)
    return incident, far_field


def forward(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray, H: np.ndarray) -> np.ndarray:
    """Simulated intensities |G(p_i, V)|^2 for every position, float64 [n, M, M]."""
    obj = np.asarray(obj, dtype=np.complex128)
    M = probe.shape[0]
    out = np.empty((len(pos), M, M), dtype=np.float64)
    for i, (y0, x0) in enumerate(np.asarray(pos)):
        _, far = exit_waves(obj, probe, int(y0), int(x0), H)
        out[i] = np.abs(far) ** 2
    return out


# ---------------------------------------------------------------------------
# Amplitude cost f_i (Eq. 1) and its gradient (Eq. 2) for one position.
# ---------------------------------------------------------------------------
def position_loss_and_patch_gradients(obj: np.ndarray, probe: np.ndarray, y0: int, x0: int,
                                      meas: np.ndarray, H: np.ndarray) -> Tuple[float, np.ndarray]:
    """f_i and the S window-sized pieces of df_i/dt (complex128 [S, M, M]).

    With u = Psi/|Psi| (u = 0 where |Psi| = 0) and a = sqrt(meas):
      dF/dPsi* direction g = 2 (|Psi| - a) u,
      chi_{S-1} = F^H g = M^2 F^-1 g,
      grad_s = chi_s * conj(psi_s),
      chi_{s-1} = F^-1(conj(H) F(chi_s * conj(t_s)))     (adjoint of the propagation step).
    """
    M = probe.shape[0]
    S = obj.shape[0]
    incident, far = exit_waves(obj, probe, y0, x0, H)
    a = np.sqrt(np.asarray(meas, dtype=np.float64))
    mod = np.abs(far)
    loss = float(np.sum((mod - a) ** 2))
    u = np.zeros_like(far)
    nz = mod > 0
    u[nz] = far[nz] / mod[nz]
    g_far = 2.0 * (mod - a) * u
    chi = (M * M) * np.fft.ifft2(g_far)
    grads = np.empty((S, M, M), dtype=np.complex128)
    for s in range(S - 1, -1, -1):
        grads[s] = chi * np.conj(incident[s])
        if s > 0:
            t_s = _window(obj[s], y0, x0, M)
            chi = np.fft.ifft2(np.conj(H) * np.fft.fft2(chi * np.conj(t_s)))
    return loss, grads


def probe_gradient(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray, meas: np.ndarray,
                   H: np.ndarray) -> np.ndarray:
    """dF/dRe P + i dF/dIm P (complex128 [M, M]).

    phi_0 = P * t_0[window] is symmetric in P and t_0, so each position adds
    chi_0 * conj(t_0[window]), chi_0 being the adjoint wave at the first slice:
    chi_{S-1} = F^H g, chi_{s-1} = F^-1(conj(H) F(chi_s conj(t_s))) down to s = 1."""
    obj = np.asarray(obj, dtype=np.complex128)
    M = probe.shape[0]
    S = obj.shape[0]
    out = np.zeros((M, M), dtype=np.complex128)
    for i, (y0, x0) in enumerate(np.asarray(pos)):
        y0, x0 = int(y0), int(x0)
        _, far = exit_waves(obj, probe, y0, x0, H)
        a = np.sqrt(np.asarray(meas[i], dtype=np.float64))
        mod = np.abs(far)
        u = np.zeros_like(far)
        nz = mod > 0
        u[nz] = far[nz] / mod[nz]
        chi = (M * M) * np.fft.ifft2(2.0 * (mod - a) * u)
        for s in range(S - 1, 0, -1):
            chi = np.fft.ifft2(np.conj(H) * np.fft.fft2(chi * np.conj(_window(obj[s], y0, x0, M))))
        out += chi * np.conj(_window(obj[0], y0, x0, M))
    return out


def loss_and_gradient(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray, meas: np.ndarray,
                      H: np.ndarray) -> Tuple[float, np.ndarray, np.ndarray]:
    """F(V) summed over positions in order, per-position f_i, and dF/dt (complex128 like obj)."""
    obj = np.asarray(obj, dtype=np.complex128)
    M = probe.shape[0]
    grad = np.zeros_like(obj)
    per_pos = np.empty(len(pos), dtype=np.float64)
    total = 0.0
    for i, (y0, x0) in enumerate(np.asarray(pos)):
        y0, x0 = int(y0), int(x0)
        f_i, patches = position_loss_and_patch_gradients(obj, probe, y0, x0, meas[i], H)
        per_pos[i] = f_i
        total += f_i
        grad[:, y0:y0 + M, x0:x0 + M] += patches
    return total, per_pos, grad


# ---------------------------------------------------------------------------
# Gradient decomposition into tiles with halos (Section III).
# Reading: tiles are an even split of the object; a position belongs to the
# tile that contains its window centre; the extended box is the tile grown by
# the halo on every side and clipped to the object.
# ---------------------------------------------------------------------------
def tile_bounds(extent: int, count: int) -> List[int]:
    """Tile edges along one axis: edge_k = floor(k * extent / count), k = 0..count."""
    return [(k * extent) // count for k in range(count + 1)]


def bin_positions(pos: np.ndarray, Hobj: int, Wobj: int, M: int, tiles_y: int, tiles_x: int) -> np.ndarray:
    """Tile index (row-major) of every position, by the tile holding its window centre."""
    ey = tile_bounds(Hobj, tiles_y)
    ex = tile_bounds(Wobj, tiles_x)
    out = np.empty(len(pos), dtype=np.int32)
    for i, (y0, x0) in enumerate(np.asarray(pos)):
        cy = int(y0) + M // 2
        cx = int(x0) + M // 2
        ty = 0
        while ty + 1 < tiles_y and ey[ty + 1] <= cy:
            ty += 1
        tx = 0
        while tx + 1 < tiles_x and ex[tx + 1] <= cx:
            tx += 1
        out[i] = ty * tiles_x + tx
    return out


def extended_box(Hobj: int, Wobj: int, tiles_y: int, tiles_x: int, ty: int, tx: int, halo: int
                 ) -> Tuple[int, int, int, int]:
    """(ey0, ey1, ex0, ex1): tile (ty, tx) grown by the halo, clipped to the object (half-open)."""
    ey = tile_bounds(Hobj, tiles_y)
    ex = tile_bounds(Wobj, tiles_x)
    return (max(ey[ty] - halo, 0), min(ey[ty + 1] + halo, Hobj),
            max(ex[tx] - halo, 0), min(ex[tx + 1] + halo, Wobj))


def tile_gradient(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray, meas: np.ndarray, H: np.ndarray,
                  tiles: Tuple[int, int], halo: int, ty: int, tx: int) -> Dict[str, object]:
    """Loss and gradient of one tile's own positions, held on the tile's extended box."""
    obj = np.asarray(obj, dtype=np.complex128)
    S, Hobj, Wobj = obj.shape
    M = probe.shape[0]
    tiles_y, tiles_x = tiles
    owner = bin_positions(pos, Hobj, Wobj, M, tiles_y, tiles_x)
    ey0, ey1, ex0, ex1 = extended_box(Hobj, Wobj, tiles_y, tiles_x, ty, tx, halo)
    box = np.zeros((S, ey1 - ey0, ex1 - ex0), dtype=np.complex128)
    loss = 0.0
    mine = np.nonzero(owner == ty * tiles_x + tx)[0]
    for i in mine:
        y0, x0 = int(pos[i][0]), int(pos[i][1])
        if y0 < ey0 or x0 < ex0 or y0 + M > ey1 or x0 + M > ex1:
            raise ValueError(f"window of position {i} leaves the extended tile: halo too small")
        f_i, patches = position_loss_and_patch_gradients(obj, probe, y0, x0, meas[i], H)
        loss += f_i
        box[:, y0 - ey0:y0 - ey0 + M, x0 - ex0:x0 - ex0 + M] += patches
    return {"box": (ey0, ey1, ex0, ex1), "grad": box, "loss": loss, "positions": mine}


def stitch_tile_gradients(shape: Sequence[int], tile_results: Sequence[Dict[str, object]]) -> np.ndarray:
    """Sum of the tile gradients embedded at their extended boxes (overlaps add)."""
    out = np.zeros(tuple(shape), dtype=np.complex128)
    for r in tile_results:
        ey0, ey1, ex0, ex1 = r["box"]
        out[:, ey0:ey1, ex0:ex1] += r["grad"]
    return out


# ---------------------------------------------------------------------------
# Real-potential parametrisation (Section II-B: V is the scattering potential;
# each slice enters through its transmission t = exp(i sigma V)).
# ---------------------------------------------------------------------------
def transmission_from_potential(V: np.ndarray, sigma: float) -> np.ndarray:
    return np.exp(1j * sigma * np.asarray(V, dtype=np.float64))


def potential_gradient(t: np.ndarray, G: np.ndarray, sigma: float) -> np.ndarray:
    """dF/dV from G = dF/dRe t + i dF/dIm t: with dRe t/dV = -sigma Im t and
    dIm t/dV = sigma Re t, dF/dV = sigma (Re t Im G - Im t Re G) = sigma Im(conj(t) G)."""
    return sigma * np.imag(np.conj(t) * G)


# ---------------------------------------------------------------------------
# Exchanges between separately held tile buffers (one per device in the
# paper).  A buffer is {"box": (ey0, ey1, ex0, ex1), "grad": [S, eh, ew]}; the
# tiles form a tiles_y x tiles_x grid in row-major order.
# ---------------------------------------------------------------------------
def _overlap(a: Tuple[int, int, int, int], b: Tuple[int, int, int, int]):
    """Intersection of two half-open boxes, or None."""
    y0, y1 = max(a[0], b[0]), min(a[1], b[1])
    x0, x1 = max(a[2], b[2]), min(a[3], b[3])
    if y0 >= y1 or x0 >= x1:
        return None
    return y0, y1, x0, x1


def _view(buf: Dict[str, object], region: Tuple[int, int, int, int]) -> np.ndarray:
    ey0, _, ex0, _ = buf["box"]
    y0, y1, x0, x1 = region
    return buf["grad"][:, y0 - ey0:y1 - ey0, x0 - ex0:x1 - ex0]


def neighbour_add(tile_results: Sequence[Dict[str, object]], tiles: Tuple[int, int]) -> List[Dict[str, object]]:
    """Section III: every tile adds the gradients of its eight direct neighbours on
    their overlaps (a single exchange of the original tile gradients)."""
    ty_n, tx_n = tiles
    out = [{"box": r["box"], "grad": np.array(r["grad"], copy=True)} for r in tile_results]
    for ty in range(ty_n):
        for tx in range(tx_n):
            k = ty * tx_n + tx
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    if (dy, dx) == (0, 0) or not (0 <= ty + dy < ty_n and 0 <= tx + dx < tx_n):
                        continue
                    j = (ty + dy) * tx_n + tx + dx
                    ov = _overlap(out[k]["box"], tile_results[j]["box"])
                    if ov is not None:
                        _view(out[k], ov)[...] += _view(tile_results[j], ov)
    return out


def directional_passes(tile_results: Sequence[Dict[str, object]], tiles: Tuple[int, int]
                       ) -> List[Dict[str, object]]:
    """Section IV: accumulated-gradient buffers start as copies of the tile
    gradients; then, in this order,
      vertical forward   -- down every tile column, the buffer of row r is added
                            into row r+1 on their overlap;
      vertical backward  -- up every column, row r+1's buffer replaces row r's
                            on their overlap;
      horizontal forward -- along every tile row, column c is added into c+1;
      horizontal backward -- column c+1 replaces column c on their overlap.
    Afterwards every buffer holds the summed gradient of all tiles on its box."""
    ty_n, tx_n = tiles
    acc = [{"box": r["box"], "grad": np.array(r["grad"], copy=True)} for r in tile_results]

    def exchange(src: int, dst: int, replace: bool) -> None:
        ov = _overlap(acc[src]["box"], acc[dst]["box"])
        if ov is None:
            return
        if replace:
            _view(acc[dst], ov)[...] = _view(acc[src], ov)
        else:
            _view(acc[dst], ov)[...] += _view(acc[src], ov)

    for tx in range(tx_n):
        for ty in range(ty_n - 1):
            exchange(ty * tx_n + tx, (ty + 1) * tx_n + tx, replace=False)
    for tx in range(tx_n):
        for ty in range(ty_n - 1, 0, -1):
            exchange(ty * tx_n + tx, (ty - 1) * tx_n + tx, replace=True)
    for ty in range(ty_n):
        for tx in range(tx_n - 1):
            exchange(ty * tx_n + tx, ty * tx_n + tx + 1, replace=False)
    for ty in range(ty_n):
        for tx in range(tx_n - 1, 0, -1):
            exchange(ty * tx_n + tx, ty * tx_n + tx - 1, replace=True)
    return acc


def alg1_tiles(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray, meas: np.ndarray, H: np.ndarray,
               tiles: Tuple[int, int], halo: int, step: float, batch: int, T: int, iterations: int
               ) -> Tuple[List[float], np.ndarray]:
    """Alg. 1 with one tile per device, read with mini-batches of positions.

    Every tile holds its own extended copy V_k of the object and an
    accumulation buffer AccBuf_k.  In every iteration each tile walks its own
    positions in scan order, `batch` at a time (batch = 1 is the per-probe loop
    of Alg. 1): the batch's gradient, evaluated at V_k, is added to AccBuf_k and
    V_k takes the step V_k -= step * gradient.  After every T batches (the
    delayed accumulation) and after the last batch of an iteration, the
    directional passes run on the buffers, every tile takes
    V_k -= step * AccBuf_k, and the buffers are cleared.  Returns the loss of
    each iteration (each position's f_i evaluated when it is visited) and the
    tiles' interiors stitched into one object."""
    obj = np.asarray(obj, dtype=np.complex128)
    S, Hobj, Wobj = obj.shape
    M = probe.shape[0]
    ty_n, tx_n = tiles
    owner = bin_positions(pos, Hobj, Wobj, M, ty_n, tx_n)
    mine = [np.nonzero(owner == k)[0] for k in range(ty_n * tx_n)]
    boxes = [extended_box(Hobj, Wobj, ty_n, tx_n, k // tx_n, k % tx_n, halo) for k in range(ty_n * tx_n)]
    V = [obj[:, b[0]:b[1], b[2]:b[3]].copy() for b in boxes]
    acc = [{"box": b, "grad": np.zeros_like(v)} for b, v in zip(boxes, V)]
    steps = max((len(m) + batch - 1) // batch for m in mine)
    losses = []
    for _ in range(iterations):
        total = 0.0
        for j in range(steps):
            for k, b in enumerate(boxes):
                g = np.zeros_like(V[k])
                for i in mine[k][j * batch:(j + 1) * batch]:
                    y0, x0 = int(pos[i][0]) - b[0], int(pos[i][1]) - b[2]
                    f_i, patches = position_loss_and_patch_gradients(V[k], probe, y0, x0, meas[i], H)
                    total += f_i
                    g[:, y0:y0 + M, x0:x0 + M] += patches
                acc[k]["grad"] += g
                V[k] -= step * g
            if (j + 1) % T == 0 or j == steps - 1:
                acc = directional_passes(acc, tiles)
                for k in range(len(V)):
                    V[k] -= step * acc[k]["grad"]
                    acc[k]["grad"][...] = 0.0
        losses.append(total)
    out = np.empty_like(obj)
    ey, ex = tile_bounds(Hobj, ty_n), tile_bounds(Wobj, tx_n)
    for k, b in enumerate(boxes):
        ty, tx = divmod(k, tx_n)
        y0, y1, x0, x1 = ey[ty], ey[ty + 1], ex[tx], ex[tx + 1]
        out[:, y0:y1, x0:x1] = V[k][:, y0 - b[0]:y1 - b[0], x0 - b[2]:x1 - b[2]]
    return losses, out


# ---------------------------------------------------------------------------
# Full-batch gradient descent on the slice transmissions.
# Reading: the paper gives no step length; alpha = 1 / (2 M^2 S max_r sum_i |P(r - r_i)|^2).
# With unit-modulus slices and a unitary propagator, the far field's
# sensitivity to all S slices together is at most sqrt(S) times the largest
# single-slice one (Cauchy-Schwarz over the slices), so the Gauss-Newton
# curvature of the amplitude cost is bounded by S times the largest
# single-slice diagonal 2 M^2 max_r sum_i |P(r - r_i)|^2; the step is the
# inverse of that bound.
# ---------------------------------------------------------------------------
def gd_step_size(probe: np.ndarray, pos: np.ndarray, Hobj: int, Wobj: int, S: int) -> float:
    M = probe.shape[0]
    cover = np.zeros((Hobj, Wobj), dtype=np.float64)
    p2 = np.abs(probe) ** 2
    for y0, x0 in np.asarray(pos):
        cover[int(y0):int(y0) + M, int(x0):int(x0) + M] += p2
    return 1.0 / (2.0 * M * M * int(S) * float(cover.max()))


def gd_step(obj: np.ndarray, grad: np.ndarray, alpha: float) -> np.ndarray:
    return obj - alpha * grad


# ---------------------------------------------------------------------------
# Sub-pixel positions (a variant of the probe function p_i of Section II-B:
# the probe translated to the i-th location, here by a fraction of a pixel).
# Reading: a position (y, x) is split into the integer window corner
# (floor y, floor x) and the fraction d = (y - floor y, x - floor x) in
# [0, 1)^2; the probe at the position is the probe translated by d with the
# Fourier shift theorem on the periodic M x M window grid,
#   P_d(r) = F^-1[ F(P)(q) exp(-2 pi i (q_y d_y + q_x d_x) / M) ](r),
# q = fftfreq(M) * M (integer frequencies, -M/2 at the Nyquist bin).  Everything
# after the probe is the integer-position model with P replaced by P_d.
# ---------------------------------------------------------------------------
def shift_probe(probe: np.ndarray, dy: float, dx: float) -> np.ndarray:
    """The probe translated by (dy, dx) pixels (any real values), complex128 [M, M]."""
    M = probe.shape[0]
    q = np.fft.fftfreq(M) * M
    ramp = np.exp(-2j * np.pi * (q[:, None] * dy + q[None, :] * dx) / M)
    return np.fft.ifft2(np.fft.fft2(np.asarray(probe, dtype=np.complex128)) * ramp)


def split_subpixel(pos: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Real-valued positions [n, 2] -> (integer window corners int32 [n, 2], fractions float64 [n, 2])."""
    pos = np.asarray(pos, dtype=np.float64)
    corner = np.floor(pos)
    return corner.astype(np.int32), pos - corner


def forward_subpixel(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray, H: np.ndarray) -> np.ndarray:
    """Intensities for real-valued positions, float64 [n, M, M]."""
    obj = np.asarray(obj, dtype=np.complex128)
    corner, frac = split_subpixel(pos)
    M = probe.shape[0]
    out = np.empty((len(corner), M, M), dtype=np.float64)
    for i in range(len(corner)):
        _, far = exit_waves(obj, shift_probe(probe, *frac[i]), int(corner[i, 0]), int(corner[i, 1]), H)
        out[i] = np.abs(far) ** 2
    return out


def loss_and_gradient_subpixel(obj: np.ndarray, probe: np.ndarray, pos: np.ndarray, meas: np.ndarray,
                               H: np.ndarray) -> Tuple[float, np.ndarray, np.ndarray]:
    """F(V), per-position f_i and dF/dt for real-valued positions (the shifted probe per position)."""
    obj = np.asarray(obj, dtype=np.complex128)
    corner, frac = split_subpixel(pos)
    M = probe.shape[0]
    grad = np.zeros_like(obj)
    per_pos = np.empty(len(corner), dtype=np.float64)
    total = 0.0
    for i in range(len(corner)):
        y0, x0 = int(corner[i, 0]), int(corner[i, 1])
        f_i, patches = position_loss_and_patch_gradients(obj, shift_probe(probe, *frac[i]), y0, x0, meas[i], H)
        per_pos[i] = f_i
        total += f_i
        grad[:, y0:y0 + M, x0:x0 + M] += patches
    return total, per_pos, grad
