"""CPU checks of the C ABI: the library loads, exports what the header declares,
and its host-side validation, binning and tile geometry agree with the oracle."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import ptycho_synth as ps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptycho.h")

pt = pytest.importorskip("paper_2205_06327_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ptycho_[a-z_]+)\s*\(", text)))


def test_header_declares_the_calls():
    names = declared_functions()
    for required in ("ptycho_forward", "ptycho_loss_grad", "ptycho_tile_grad", "ptycho_create", "ptycho_check"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = pt.lib()
    names = declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", pt._binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT\s+(ptycho_[a-z_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert isinstance(getattr(lib, n), ctypes._CFuncPtr)
    assert set(pt._binding.EXPORTED) == set(names)


def test_create_rejects_unsupported_shapes_before_touching_the_device():
    lib = pt.lib()
    h = ctypes.c_void_p()
    assert lib.ptycho_create(ctypes.byref(h), 96, 4, 0.0197, 2.0, 0.1, 0, None) == -6
    assert "window size" in lib.ptycho_last_error().decode()
    assert lib.ptycho_create(ctypes.byref(h), 128, 0, 0.0197, 2.0, 0.1, 0, None) == -6
    assert lib.ptycho_create(ctypes.byref(h), 128, 65, 0.0197, 2.0, 0.1, 0, None) == -6
    assert lib.ptycho_create(ctypes.byref(h), 128, 4, 0.0197, 2.0, 0.0, 0, None) == -1
    assert lib.ptycho_create(None, 128, 4, 0.0197, 2.0, 0.1, 0, None) == -1
    assert not h.value


def test_null_context_calls_fail_cleanly():
    lib = pt.lib()
    assert lib.ptycho_forward(None, None, 256, 256, 0, 256, None, None, 0, None) == -1
    assert lib.ptycho_loss_grad(None, None, 256, 256, 0, 256, None, None, 0, None, None, None, None, 0, 256, 0, None) == -1
    assert lib.ptycho_loss(None, None, 256, 256, 0, 256, None, None, 0, None, None, None, 0) == -1
    assert lib.ptycho_check(None, None) == -1
    assert lib.ptycho_destroy(None) == 0


def test_validate_positions():
    pt.validate_positions([[0, 0], [192, 192]], 256, 256, 64)
    with pytest.raises(pt.PtychoError) as e:
        pt.validate_positions([[0, 0], [193, 0]], 256, 256, 64)
    assert e.value.name == "PTYCHO_E_BOUNDS"
    with pytest.raises(pt.PtychoError):
        pt.validate_positions([[-1, 0]], 256, 256, 64)
    pt.validate_positions(np.zeros((0, 2), np.int32), 256, 256, 64)


@pytest.mark.parametrize("W,M,tiles,step,n_side", [(2048, 128, (4, 4), 14, (126, 132)), (1000, 64, (3, 5), 9, (40, 31)),
                                                   (256, 64, (2, 2), 8, (16, 16))])
def test_binning_matches_oracle(W, M, tiles, step, n_side):
    pos = ps.raster_positions(W, M, n_side[0], n_side[1], step)
    got = pt.bin_positions(pos, W, W, M, *tiles)
    ref = oracle.bin_positions(pos, W, W, M, *tiles)
    np.testing.assert_array_equal(got, ref)


def test_binning_random_positions_matches_oracle():
    rng = np.random.default_rng(0)
    pos = np.stack([rng.integers(0, 700 - 64, 500), rng.integers(0, 611 - 64, 500)], axis=1).astype(np.int32)
    np.testing.assert_array_equal(pt.bin_positions(pos, 700, 611, 64, 3, 7), oracle.bin_positions(pos, 700, 611, 64, 3, 7))


def test_tile_box_matches_oracle():
    for (H, W, ty_n, tx_n, halo) in [(2048, 2048, 4, 4, 64), (700, 611, 3, 7, 40), (256, 256, 1, 1, 10)]:
        for ty in range(ty_n):
            for tx in range(tx_n):
                (t0, t1, u0, u1), box = pt.tile_box(H, W, ty_n, tx_n, ty, tx, halo)
                assert box == oracle.extended_box(H, W, ty_n, tx_n, ty, tx, halo)
                ey = oracle.tile_bounds(H, ty_n)
                ex = oracle.tile_bounds(W, tx_n)
                assert (t0, t1, u0, u1) == (ey[ty], ey[ty + 1], ex[tx], ex[tx + 1])


def test_batch_descriptor_layout_and_host_validation():
    from paper_2205_06327_amd.batch import ReconDesc, _lib
    assert ctypes.sizeof(ReconDesc) == 112  # 6 int32, 2 int64, 5 pointers, 4 doubles
    L = _lib()
    h = ctypes.c_void_p()
    d = ReconDesc()
    d.M, d.S, d.H, d.W, d.n = 96, 2, 256, 256, 4
    d.slice_stride, d.ld = 256 * 256, 256
    d.obj, d.grad, d.probe, d.pos, d.meas = 16, 32, 48, 64, 80
    d.wavelength_A, d.dz_A, d.pixel_A, d.alpha = 0.0197, 2.0, 0.1, 1e-3
    arr = (ReconDesc * 1)(d)
    assert L.ptycho_batch_create(ctypes.byref(h), arr, 1, 4) == -6
    arr[0].M = 128
    arr[0].ld = 100
    assert L.ptycho_batch_create(ctypes.byref(h), arr, 1, 4) == -2
    arr[0].ld = 256
    arr[0].grad = arr[0].obj
    assert L.ptycho_batch_create(ctypes.byref(h), arr, 1, 4) == -1
    arr[0].grad = 32
    arr[0].reserved = 1
    assert L.ptycho_batch_create(ctypes.byref(h), arr, 1, 4) == -1
    assert L.ptycho_batch_create(ctypes.byref(h), arr, -1, 4) == -1
    assert not h.value
    assert L.ptycho_batch_step(None) == -1 and L.ptycho_batch_destroy(None) == 0


def test_box_exchange_rejects_a_null_context():
    import ctypes
    from paper_2205_06327_amd import _binding as B
    rc = B.lib().ptycho_box_exchange(None, 1, ctypes.c_void_p(8), 0, 0, 1, 1, 1, 1, ctypes.c_void_p(16), 0, 0, 1, 1,
                                     1, 1, 0)
    assert rc == -1 and b"null context" in B.lib().ptycho_last_error()


def test_new_entry_points_reject_a_null_context():
    import ctypes
    from paper_2205_06327_amd import _binding as B
    L = B.lib()
    assert L.ptycho_set_checkpoint(None, 4) == -1
    assert L.ptycho_box_axpy(None, 1, ctypes.c_float(1.0), ctypes.c_void_p(8), 0, 0, 1, 1, 1, 1,
                             ctypes.c_void_p(16), 0, 0, 1, 1, 1, 1) == -1
    assert b"null context" in L.ptycho_last_error()


def test_binding_rejects_host_tensors_and_bad_position_shapes():
    """Host-side argument checks of the binding, before any library call: a host tensor or a
    position array that is not [n, 2] would reach the kernels as invalid device memory."""
    torch = pytest.importorskip("torch")
    from paper_2205_06327_amd import _binding as B
    with pytest.raises(ValueError, match="CUDA tensor"):
        B._obj_geometry(torch.zeros((2, 8, 8), dtype=torch.complex64))
    with pytest.raises(ValueError, match="CUDA tensor"):
        B._need(torch.zeros(4, dtype=torch.float32), torch.float32, None, "meas")
    with pytest.raises(ValueError, match="CUDA tensor"):
        B._need_pos(torch.zeros((3, 2), dtype=torch.int32))
    with pytest.raises(ValueError, match="CUDA tensor"):
        B._on_device(np.zeros(3), "x")


@pytest.mark.parametrize("name,S", [("2d-256-m64", 1), ("ms8-1024-m128", 8)])
def test_gd_step_size_matches_the_oracle(name, S):
    """The library's step length (host helper) and the oracle's, on the same complex64 probe values."""
    spec = ps.reduced(ps.workload(name), W=320, ny=9, nx=7, S=S)
    probe = ps.make_probe(spec.M, spec.R, spec.C, spec.dose).astype(np.complex64)
    pos = ps.raster_positions(spec.W, spec.M, spec.ny, spec.nx, spec.step)
    pos[3] = (0, 0)  # a corner window as well
    want = oracle.gd_step_size(probe.astype(np.complex128), pos, spec.W, spec.W, S)
    got = pt.gd_step_size(probe, pos, spec.W, spec.W, S)
    assert abs(got - want) <= 1e-12 * want


def test_gd_step_size_errors():
    lib = pt.lib()
    probe = np.ones((8, 8), dtype=np.complex64)
    pos = np.array([[0, 0], [4, 4]], dtype=np.int32)
    out = ctypes.c_double(-1.0)
    P = ctypes.POINTER(ctypes.c_int32)
    assert lib.ptycho_gd_step_size(probe.ctypes.data_as(ctypes.c_void_p), 8, pos.ctypes.data_as(P), 2, 12, 12, 2,
                                   ctypes.byref(out)) == 0
    assert abs(out.value - 1.0 / (2 * 64 * 2 * 2.0)) <= 1e-15  # the centre pixels are covered twice
    bad = np.array([[5, 5]], dtype=np.int32)  # leaves the 12 x 12 object
    assert lib.ptycho_gd_step_size(probe.ctypes.data_as(ctypes.c_void_p), 8, bad.ctypes.data_as(P), 1, 12, 12, 2,
                                   ctypes.byref(out)) == -3
    zero = np.zeros((8, 8), dtype=np.complex64)
    out.value = -1.0
    assert lib.ptycho_gd_step_size(zero.ctypes.data_as(ctypes.c_void_p), 8, pos.ctypes.data_as(P), 2, 12, 12, 2,
                                   ctypes.byref(out)) == -1
    assert lib.ptycho_gd_step_size(probe.ctypes.data_as(ctypes.c_void_p), 8, pos.ctypes.data_as(P), 0, 12, 12, 2,
                                   ctypes.byref(out)) == -1
    assert out.value == -1.0  # nothing written on failure
    assert lib.ptycho_gd_step_size(None, 8, pos.ctypes.data_as(P), 2, 12, 12, 2, ctypes.byref(out)) == -1


def test_static_entry_point_rejects_before_touching_the_device():
    """ptycho_loss_grad_static: unsupported shapes and more positions than its static workspace holds are
    rejected by host validation, before any HIP call."""
    lib = pt.lib()
    f = lib.ptycho_loss_grad_static
    args = (0.0197, 2.0, 0.1, None, None, 256, 256, 256 * 256, 256, None, None)
    assert f(96, 4, *args, 0, None, None, None, None, 0, 256, 0, None) == -6
    assert "window size" in lib.ptycho_last_error().decode()
    assert f(128, 0, *args, 0, None, None, None, None, 0, 256, 0, None) == -6
    assert f(128, 4, *args, (1 << 20) + 1, None, None, None, None, 0, 256, 0, None) == -9
    assert "static workspace" in lib.ptycho_last_error().decode()
    assert f(128, 4, *args, -1, None, None, None, None, 0, 256, 0, None) == -1
    assert f(128, 4, 0.0197, 2.0, 0.0, *args[3:], 0, None, None, None, None, 0, 256, 0, None) == -1
