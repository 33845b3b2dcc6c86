"""Seeded generators for objects, probes, scan positions and noise.

Recipe (the paper's PbTiO3 data are not available, so these stand in for them):

* Object slice: ``phi`` = sum of unit-amplitude Gaussian blobs (sigma 1.5 px,
  truncated at 6 sigma along each axis) centred at lattice sites ``pitch/2 + j*pitch`` jittered
  by U(-0.5, 0.5) px on each axis, min-max normalised to [0, 1]; the slice
  transmission is ``exp(i * strength * phi)`` (a pure-phase object).
* Probe: integer detector frequencies ``q = fftfreq(M) * M``; aperture
  ``|q| <= R``; defocus phase ``exp(-i C (|q|/R)^2)``; the real-space probe is
  the centred inverse DFT of that pupil, scaled so that ``M^2 sum |P|^2`` equals
  the dose ``D`` (the total counts of a pattern for a pure-phase object).
* Scan: row-major raster of ``ny x nx`` integer top-left corners with a fixed
  step, centred in the object (offset ``floor((W - (M + (n-1) step)) / 2)``).
* Noise: Poisson counts of the noise-free intensities, stored as float32.

Every random draw comes from ``numpy.random.SeedSequence(seed)`` spawned into
independent streams, so each array is reproducible on its own.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# Electron-optical constants of the multislice workloads: 300 keV electrons,
# 0.1 Angstrom pixels, 2 Angstrom slices.
PHYSICS = {"wavelength_A": 0.0197, "dz_A": 2.0, "pixel_A": 0.1}


@dataclasses.dataclass(frozen=True)
class WorkloadSpec:
    """Shape and physics of one synthetic reconstruction problem."""

    name: str
    W: int                 # object side (square object W x W per slice)
    S: int                 # number of slices
    strength: float        # maximum phase of a slice, radians
    pitch: float           # lattice pitch of the atoms, px
    M: int                 # probe / window side
    R: float               # aperture radius, px in Fourier space
    C: float               # defocus phase at the aperture edge, rad
    ny: int                # raster rows
    nx: int                # raster columns
    step: int              # raster step, px
    dose: float            # counts per pattern
    noise: bool            # Poisson counts (True) or exact intensities
    seed: int
    tiles: Tuple[int, int] = (1, 1)
    halo: int = 0
    wavelength_A: float = PHYSICS["wavelength_A"]
    dz_A: float = PHYSICS["dz_A"]
    pixel_A: float = PHYSICS["pixel_A"]

    @property
    def n(self) -> int:
        return self.ny * self.nx


def seed_streams(seed: int, count: int = 4) -> List[np.random.SeedSequence]:
    """Independent child seeds: [atoms, noise, finite-difference voxels, batch params]."""
    return np.random.SeedSequence(seed).spawn(count)


def atom_phase(W: int, pitch: float, rng: np.random.Generator, sigma: float = 1.5) -> np.ndarray:
    """Gaussian 'atoms' on a jittered square lattice, min-max normalised to [0, 1] (float64 W x W)."""
    nsite = int(math.ceil((W - pitch / 2.0) / pitch))
    nsite = max(nsite, 1)
    centres = pitch / 2.0 + pitch * np.arange(nsite)
    cy = centres[:, None] + rng.uniform(-0.5, 0.5, size=(nsite, nsite))
    cx = centres[None, :] + rng.uniform(-0.5, 0.5, size=(nsite, nsite))
    iy = np.floor(cy).astype(np.int64)
    ix = np.floor(cx).astype(np.int64)
    fy = cy - iy
    fx = cx - ix
    rad = int(math.ceil(6.0 * sigma))
    offs = np.arange(-rad, rad + 1)
    # Separable Gaussian per atom over a (2 rad + 1)^2 footprint.  The atoms of
    # one lattice row share a band of canvas rows; their sum over that band is
    # the product of a (band x atoms) and an (atoms x columns) matrix.
    Wp = W + 2 * rad
    canvas = np.zeros((Wp, Wp), dtype=np.float64)
    cols = np.arange(nsite)[:, None]
    for i in range(nsite):
        gy = np.exp(-0.5 * ((offs[None, :] - fy[i][:, None]) / sigma) ** 2)   # [atoms, offs]
        gx = np.exp(-0.5 * ((offs[None, :] - fx[i][:, None]) / sigma) ** 2)
        base = int(iy[i].min())
        Hb = int(iy[i].max()) - base + 2 * rad + 1
        Gy = np.zeros((nsite, Hb))
        Gy[cols, (iy[i] - base)[:, None] + offs[None, :] + rad] = gy
        Gx = np.zeros((nsite, Wp))
        xi = ix[i][:, None] + offs[None, :] + rad
        ok = (xi >= 0) & (xi < Wp)
        Gx[np.broadcast_to(cols, xi.shape)[ok], xi[ok]] = gx[ok]
        r0 = base - rad + rad  # canvas row of band row 0 (canvas is padded by rad)
        lo_r, hi_r = max(r0, 0), min(r0 + Hb, Wp)
        if hi_r > lo_r:
            canvas[lo_r:hi_r] += (Gy.T @ Gx)[lo_r - r0:hi_r - r0]
    phi = canvas[rad:rad + W, rad:rad + W]
    lo, hi = phi.min(), phi.max()
    return (phi - lo) / (hi - lo) if hi > lo else np.zeros_like(phi)


def _phases(W: int, pitch: float, children, workers: int) -> List[np.ndarray]:
    if workers > 1 and len(children) > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, len(children))) as ex:
            return list(ex.map(_phase_job, [(W, pitch, c) for c in children]))
    return [_phase_job((W, pitch, c)) for c in children]


def _phase_job(args) -> np.ndarray:
    W, pitch, child = args
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        return atom_phase(W, pitch, np.random.default_rng(child))
    with threadpool_limits(1):
        return atom_phase(W, pitch, np.random.default_rng(child))


def make_object(W: int, S: int, strength: float, pitch: float, seed_seq: np.random.SeedSequence,
                workers: int = 1) -> np.ndarray:
    """Stack of S independent pure-phase slices exp(i*strength*phi_s), complex128 [S, W, W]."""
    phis = _phases(W, pitch, seed_seq.spawn(S), workers)
    obj = np.empty((S, W, W), dtype=np.complex128)
    for s in range(S):
        obj[s] = np.exp(1j * strength * phis[s])
    return obj


def make_probe(M: int, R: float, C: float, dose: float) -> np.ndarray:
    """Defocused aperture probe, complex128 [M, M], with M^2 * sum|P|^2 == dose."""
    q = np.fft.fftfreq(M) * M
    qq = np.sqrt(q[:, None] ** 2 + q[None, :] ** 2)
    pupil = np.where(qq <= R, np.exp(-1j * C * (qq / R) ** 2), 0.0)
    probe = np.fft.fftshift(np.fft.ifft2(pupil))
    norm = np.sum(np.abs(probe) ** 2)
    return probe * math.sqrt(dose / (M * M) / norm)


def raster_offset(W: int, M: int, count: int, step: int) -> int:
    return (W - (M + (count - 1) * step)) // 2


def raster_positions(W: int, M: int, ny: int, nx: int, step: int) -> np.ndarray:
    """Row-major (time-ordered) raster of (y0, x0) top-left corners, int32 [ny*nx, 2]."""
    oy = raster_offset(W, M, ny, step)
    ox = raster_offset(W, M, nx, step)
    if oy < 0 or ox < 0:
        raise ValueError("raster does not fit inside the object")
    yy, xx = np.meshgrid(oy + step * np.arange(ny), ox + step * np.arange(nx), indexing="ij")
    return np.stack([yy.ravel(), xx.ravel()], axis=1).astype(np.int32)


def poisson_counts(intensity: np.ndarray, seed_seq: np.random.SeedSequence) -> np.ndarray:
    """Poisson counts of non-negative intensities, float32 of the same shape."""
    rng = np.random.default_rng(seed_seq)
    lam = np.clip(np.asarray(intensity, dtype=np.float64), 0.0, None)
    return rng.poisson(lam).astype(np.float32)


def eval_object(obj_true: np.ndarray, pitch: float, seed_seq: np.random.SeedSequence, amp: float = 0.01,
                workers: int = 1) -> np.ndarray:
    """A nearby evaluation point t_true * exp(i*amp*phi'), with phi' a fresh lattice draw per slice."""
    S, W, _ = obj_true.shape
    phis = _phases(W, pitch, seed_seq.spawn(S), workers)
    out = np.empty_like(obj_true)
    for s in range(S):
        out[s] = obj_true[s] * np.exp(1j * amp * phis[s])
    return out


WORKLOAD_NAMES = ("2d-256-m64", "2d-1024-m128", "ms8-1024-m128", "ms16-2048-m128-tiles4x4")


def workload(name: str) -> WorkloadSpec:
    """The single-reconstruction workloads by name (object side, slices, probe side)."""
    if name == "2d-256-m64":       # single slice, 256^2 object, 64^2 probe, noise-free
        return WorkloadSpec(name, W=256, S=1, strength=0.3, pitch=8.0, M=64, R=12.0, C=2.0,
                            ny=16, nx=16, step=8, dose=1e5, noise=False, seed=0)
    if name == "2d-1024-m128":     # single slice, 1024^2 object, 128^2 probe, 4096 positions
        return WorkloadSpec(name, W=1024, S=1, strength=0.3, pitch=10.0, M=128, R=20.0, C=4.0,
                            ny=64, nx=64, step=14, dose=1e5, noise=True, seed=1)
    if name == "ms8-1024-m128":    # 8 slices of 1024^2, 4096 positions
        return WorkloadSpec(name, W=1024, S=8, strength=0.05, pitch=10.0, M=128, R=20.0, C=4.0,
                            ny=64, nx=64, step=14, dose=1e5, noise=True, seed=2)
    if name == "ms16-2048-m128-tiles4x4":  # 16 slices of 2048^2, 16632 positions, 4x4 tiles, 64 px halo
        return WorkloadSpec(name, W=2048, S=16, strength=0.05, pitch=10.0, M=128, R=20.0,
                            C=4.0, ny=126, nx=132, step=14, dose=1e5, noise=True, seed=3, tiles=(4, 4), halo=64)
    raise ValueError(f"unknown workload {name!r}; known: {WORKLOAD_NAMES}")


def build_inputs(spec: WorkloadSpec, with_eval: bool = True, workers: int = 1) -> dict:
    """Object (truth and a nearby evaluation point), probe and positions for a spec."""
    s_atoms, s_noise, s_fd, _ = seed_streams(spec.seed)
    s_true, s_eval = s_atoms.spawn(2)
    obj = make_object(spec.W, spec.S, spec.strength, spec.pitch, s_true, workers)
    out = {
        "spec": spec,
        "obj_true": obj,
        "probe": make_probe(spec.M, spec.R, spec.C, spec.dose),
        "pos": raster_positions(spec.W, spec.M, spec.ny, spec.nx, spec.step),
        "noise_seed": s_noise,
        "fd_seed": s_fd,
    }
    if with_eval:
        out["obj_eval"] = eval_object(obj, spec.pitch, s_eval, workers=workers)
    return out


def batch_specs(seed: int = 4, count: int = 32) -> List[WorkloadSpec]:
    """Uneven independent reconstructions for the batched launch.

    Object side in {256, 512, 768, 1024}, slices in {1, 2, 4, 8}, probe 64 or
    128, raster sides uniform in [8, 48] clamped to what fits, step round(M/9),
    dose log-uniform in [1e4, 1e6].
    """
    _, _, _, s_params = seed_streams(seed)
    rng = np.random.default_rng(s_params)
    specs = []
    for r in range(count):
        W = int(rng.choice([256, 512, 768, 1024]))
        S = int(rng.choice([1, 2, 4, 8]))
        M = int(rng.choice([64, 128]))
        step = int(round(M / 9))
        nmax = (W - M) // step + 1
        ny = min(int(rng.integers(8, 49)), nmax)
        nx = min(int(rng.integers(8, 49)), nmax)
        dose = float(10.0 ** rng.uniform(4.0, 6.0))
        R, C = (12.0, 2.0) if M == 64 else (20.0, 4.0)
        specs.append(WorkloadSpec(f"batch{r}", W=W, S=S, strength=0.05, pitch=10.0, M=M, R=R, C=C,
                                  ny=ny, nx=nx, step=step, dose=dose, noise=True,
                                  seed=int(rng.integers(0, 2**31 - 1))))
    return specs


def with_overrides(spec: WorkloadSpec, **kw) -> WorkloadSpec:
    return dataclasses.replace(spec, **kw)


def reduced(spec: WorkloadSpec, W: Optional[int] = None, ny: Optional[int] = None, nx: Optional[int] = None,
            S: Optional[int] = None) -> WorkloadSpec:
    """Same recipe on a smaller object/scan (keeps M, step and physics)."""
    W = W or spec.W
    ny = ny or spec.ny
    nx = nx or spec.nx
    S = S or spec.S
    return dataclasses.replace(spec, W=W, ny=ny, nx=nx, S=S, name=spec.name + f"-reduced{W}x{ny}x{nx}x{S}")
