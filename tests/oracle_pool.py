"""Runs the FP64 oracle over many positions in freshly spawned worker
processes (no inherited GPU state); the object is shared through
multiprocessing.shared_memory so tasks only carry indices.

Test infrastructure: used by the full-size GPU parity tests to produce the
oracle's expected values (measurements, per-position losses, sampled gradient
voxels and central finite differences) in seconds instead of minutes.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from multiprocessing import shared_memory

import numpy as np

_W = {}


def _attach(shm_name, shape, dtype, probe, H, meas_name=None, meas_shape=None):
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    shm = shared_memory.SharedMemory(name=shm_name)
    _W["shm"] = shm
    _W["obj"] = np.ndarray(shape, dtype=dtype, buffer=shm.buf)
    _W["probe"] = probe
    _W["H"] = H
    if meas_name is not None:
        m = shared_memory.SharedMemory(name=meas_name)
        _W["mshm"] = m
        _W["meas"] = np.ndarray(meas_shape, dtype=np.float32, buffer=m.buf)


def _windows(y0, x0):
    M = _W["probe"].shape[0]
    return np.ascontiguousarray(_W["obj"][:, y0:y0 + M, x0:x0 + M])


def _intensity(args):
    import oracle
    y0, x0 = args
    _, far = oracle.exit_waves(_windows(y0, x0), _W["probe"], 0, 0, _W["H"])
    return np.abs(far) ** 2


def _loss_grad(args):
    import oracle
    i, y0, x0 = args
    return oracle.position_loss_and_patch_gradients(_windows(y0, x0), _W["probe"], 0, 0, _W["meas"][i], _W["H"])


def _fd_pairs(args):
    """Central differences of f_i at one voxel (real and imaginary part) for a list of positions."""
    import oracle
    s, y, x, h, plist = args
    M = _W["probe"].shape[0]
    out = 0.0 + 0.0j
    for i, y0, x0 in plist:
        base = _windows(y0, x0)
        a = np.sqrt(_W["meas"][i].astype(np.float64))
        for unit in (1.0, 1j):
            vals = []
            for sign in (1.0, -1.0):
                w = base.copy()
                w[s, y - y0, x - x0] += sign * h * unit
                _, far = oracle.exit_waves(w, _W["probe"], 0, 0, _W["H"])
                vals.append(float(np.sum((np.abs(far) - a) ** 2)))
            out += unit * (vals[0] - vals[1]) / (2 * h)
    return out


class OraclePool:
    def __init__(self, obj: np.ndarray, probe: np.ndarray, H: np.ndarray, meas: np.ndarray = None, workers=None,
                 timeout: float = 600.0):
        self.timeout = timeout
        obj = np.ascontiguousarray(obj, dtype=np.complex128)
        self._shm = shared_memory.SharedMemory(create=True, size=obj.nbytes)
        np.ndarray(obj.shape, dtype=obj.dtype, buffer=self._shm.buf)[...] = obj
        self._mshm = None
        margs = (None, None)
        if meas is not None:
            meas = np.ascontiguousarray(meas, dtype=np.float32)
            self._mshm = shared_memory.SharedMemory(create=True, size=meas.nbytes)
            np.ndarray(meas.shape, dtype=np.float32, buffer=self._mshm.buf)[...] = meas
            margs = (self._mshm.name, meas.shape)
        n = workers or max(1, min(16, len(os.sched_getaffinity(0))))
        self.workers = n
        ctx = mp.get_context("spawn")
        self._pool = ctx.Pool(n, initializer=_attach,
                              initargs=(self._shm.name, obj.shape, obj.dtype, probe, H, *margs))

    def _map(self, fn, tasks, chunksize):
        # a bounded wait: a worker that cannot start makes the pool respawn forever
        return self._pool.map_async(fn, tasks, chunksize=chunksize).get(timeout=self.timeout)

    def intensities(self, pos) -> np.ndarray:
        return np.stack(self._map(_intensity, [(int(y), int(x)) for y, x in pos], 8))

    def loss_grad(self, idx, pos):
        return self._map(_loss_grad, [(int(i), int(pos[i][0]), int(pos[i][1])) for i in idx], 4)

    def finite_differences(self, voxels, covering, pos, h):
        """Central-difference dF/dRe t + i dF/dIm t at each voxel, from the positions covering it."""
        tasks = [(int(s), int(y), int(x), h, [(int(i), int(pos[i][0]), int(pos[i][1])) for i in cov])
                 for (s, y, x), cov in zip(voxels, covering)]
        return np.array(self._map(_fd_pairs, tasks, 1))

    def close(self):
        self._pool.terminate()
        self._pool.join()
        self._shm.close()
        self._shm.unlink()
        if self._mshm is not None:
            self._mshm.close()
            self._mshm.unlink()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# the batched workload: seeded inputs of many independent reconstructions
# ---------------------------------------------------------------------------
def batch_problem(spec):
    """Seeded inputs of one reconstruction: complex64-rounded object and probe (held as complex128),
    positions, Poisson measurements of the oracle's intensities at the truth, the oracle's step length
    and propagator."""
    import oracle
    import ptycho_synth as ps
    d = ps.build_inputs(spec)
    H = oracle.fresnel_propagator(spec.M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    probe = d["probe"].astype(np.complex64).astype(np.complex128)
    obj_true = d["obj_true"].astype(np.complex64).astype(np.complex128)
    meas = ps.poisson_counts(oracle.forward(obj_true, probe, d["pos"], H), d["noise_seed"])
    alpha = oracle.gd_step_size(probe, d["pos"], spec.W, spec.W, spec.S)
    return {"obj": d["obj_eval"].astype(np.complex64).astype(np.complex128), "probe": probe, "pos": d["pos"],
            "meas": meas, "alpha": alpha, "H": H}


def _batch_problem_c64(spec):
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        p = batch_problem(spec)
    return {"obj": p["obj"].astype(np.complex64), "probe": p["probe"].astype(np.complex64), "pos": p["pos"],
            "meas": p["meas"], "alpha": p["alpha"]}


def batch_problems(specs, workers=None, timeout: float = 600.0):
    """batch_problem for every spec over spawned worker processes (complex64 object and probe)."""
    n = workers or max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(n, len(specs))) as pool:
        return pool.map_async(_batch_problem_c64, list(specs), chunksize=1).get(timeout=timeout)
