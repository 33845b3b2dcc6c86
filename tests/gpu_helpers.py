"""Shared helpers of the GPU parity tests: seeded problems, the oracle's
expected values, and relative errors.  Inputs come from ptycho_synth, expected
values from the FP64 oracle only."""
import sys

import numpy as np

import oracle
import ptycho_synth as ps


def say(msg: str) -> None:
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def problem(spec, noise=None):
    """Inputs plus oracle measurements (Poisson of the FP64 truth intensities unless noise-free)."""
    d = ps.build_inputs(spec)
    H = oracle.fresnel_propagator(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    I_true = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    use_noise = spec.noise if noise is None else noise
    d["meas"] = ps.poisson_counts(I_true, d["noise_seed"]) if use_noise else I_true.astype(np.float32)
    d["H"] = H
    return d


def to_dev(d, obj_key="obj_eval"):
    import torch
    dev = torch.device("cuda:0")
    return {
        "obj": torch.tensor(d[obj_key], dtype=torch.complex64, device=dev),
        "probe": torch.tensor(d["probe"], dtype=torch.complex64, device=dev),
        "pos": torch.tensor(np.ascontiguousarray(d["pos"]), dtype=torch.int32, device=dev),
        "meas": torch.tensor(d["meas"], dtype=torch.float32, device=dev),
    }


def context(spec, max_positions=0):
    import paper_2205_06327_amd as pt
    return pt.Context(spec.M, spec.S, spec.wavelength_A, spec.dz_A, spec.pixel_A, max_positions)
