"""Exact pins of the oracle's Alg. 1 schedule (per-tile updates, delayed
accumulation every T batches, directional passes of Section IV, AccBuf update
and clear, final stitch of the tile interiors).

The expected objects are composed by hand from functions that are pinned on
their own elsewhere: the global loss and gradient (finite differences, torch
autograd, brute-force DFT sums), the tile gradients (their embedded sum is the
global gradient) and the passes (they leave the summed gradient of all tiles
on every box, for tiles both at least and less than twice the halo).  Each
schedule is written out straight-line for its case instead of as a loop with
a modular flush condition.

The last test plants plausible mistakes in a scratch copy of
``alg1_tiles`` (an AccBuf that is never cleared, or cleared before the
update, passes left out, the per-batch step left out, the window offsets taken
from the wrong box corner) and requires every mutant to fail at least one of
the closed forms.
"""
import inspect
import textwrap

import numpy as np
import pytest

import oracle
import oracle.ptycho_oracle as oracle_module
import ptycho_synth as ps

LAM, DZ, PIX = 0.0197, 2.0, 0.1


def _problem():
    # 16-windows on a 56 px object, 5 x 5 raster with step 6 (25 positions)
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=56, ny=5, nx=5, step=6, S=2, M=16, R=4.0, C=1.0,
                             strength=0.3)
    d = ps.build_inputs(spec, with_eval=True)
    H = oracle.fresnel_propagator(spec.M, LAM, DZ, PIX)
    meas = oracle.forward(d["obj_true"], d["probe"], d["pos"], H)
    alpha = 0.5 * oracle.gd_step_size(d["probe"], d["pos"], spec.W, spec.W, spec.S)
    return spec, d, H, meas, alpha


def _tiles(spec, tiles, halo, pos):
    """Boxes, interiors and each tile's positions (scan order), by window centre."""
    W, M = spec.W, spec.M
    owner = oracle.bin_positions(pos, W, W, M, *tiles)
    ey, ex = oracle.tile_bounds(W, tiles[0]), oracle.tile_bounds(W, tiles[1])
    out = []
    for ty in range(tiles[0]):
        for tx in range(tiles[1]):
            k = ty * tiles[1] + tx
            out.append({"box": oracle.extended_box(W, W, tiles[0], tiles[1], ty, tx, halo),
                        "inner": (ey[ty], ey[ty + 1], ex[tx], ex[tx + 1]),
                        "mine": np.nonzero(owner == k)[0]})
    return out


def _embed(V_box, box, full):
    """A full-size object equal to V_box on the box and to `full` elsewhere."""
    out = np.array(full, dtype=np.complex128, copy=True)
    out[:, box[0]:box[1], box[2]:box[3]] = V_box
    return out


def _grad_on(V_full, probe, pos, meas, H, idx):
    """(loss, full-size gradient) of the positions idx at V_full (the global functions)."""
    if len(idx) == 0:
        return 0.0, np.zeros_like(V_full)
    L, _, G = oracle.loss_and_gradient(V_full, probe, pos[idx], meas[idx], H)
    return L, G


def _box(a, box):
    return a[:, box[0]:box[1], box[2]:box[3]]


def _stitch(spec, tl, Vs):
    out = np.zeros((spec.S, spec.W, spec.W), dtype=np.complex128)
    for t, V in zip(tl, Vs):
        y0, y1, x0, x1 = t["inner"]
        b = t["box"]
        out[:, y0:y1, x0:x1] = V[:, y0 - b[0]:y1 - b[0], x0 - b[2]:x1 - b[2]]
    return out


def _one_batch_per_tile_expected(spec, d, H, meas, alpha, tiles, halo):
    """Every tile's positions in one batch, T = 1, one iteration, common start V:
    V_k = V - alpha g_k - alpha G on its box, so the stitched interior of tile k is
    V - alpha (g_k + G) there (g_k: tile k's own gradient, G: the global gradient)."""
    V = d["obj_eval"].astype(np.complex128)
    L, _, G = oracle.loss_and_gradient(V, d["probe"], d["pos"], meas, H)
    tl = _tiles(spec, tiles, halo, d["pos"])
    Vs = []
    for ty in range(tiles[0]):
        for tx in range(tiles[1]):
            k = ty * tiles[1] + tx
            g = oracle.tile_gradient(V, d["probe"], d["pos"], meas, H, tiles, halo, ty, tx)
            assert g["box"] == tl[k]["box"]
            Vs.append(_box(V, g["box"]) - alpha * g["grad"] - alpha * _box(G, g["box"]))
    return [L], _stitch(spec, tl, Vs)


def _two_batches_expected(spec, d, H, meas, alpha, tiles, halo, batch, T):
    """Two batches per tile (T = 1: passes after each batch; T = 2: after the second), one iteration."""
    probe, pos = d["probe"], d["pos"]
    V = d["obj_eval"].astype(np.complex128)
    tl = _tiles(spec, tiles, halo, pos)
    assert max(len(t["mine"]) for t in tl) <= 2 * batch
    assert max(len(t["mine"]) for t in tl) > batch  # some tile really has a second batch
    Vk = [_box(V, t["box"]).copy() for t in tl]
    loss = 0.0

    def batch_gradients(j):
        nonlocal loss
        gs = []
        for t, vk in zip(tl, Vk):
            idx = t["mine"][j * batch:(j + 1) * batch]
            L, G = _grad_on(_embed(vk, t["box"], V), probe, pos, meas, H, idx)
            loss += L
            gs.append(G)  # full size; zero outside the windows of idx, which lie in the box
        return gs

    def passes(gsum):
        return [_box(gsum, t["box"]) for t in tl]  # the summed gradient of all tiles on every box

    g1 = batch_gradients(0)
    Vk = [vk - alpha * _box(g, t["box"]) for vk, g, t in zip(Vk, g1, tl)]
    if T == 1:
        acc = passes(sum(g1))
        Vk = [vk - alpha * a for vk, a in zip(Vk, acc)]
        g2 = batch_gradients(1)
        Vk = [vk - alpha * _box(g, t["box"]) for vk, g, t in zip(Vk, g2, tl)]
        acc = passes(sum(g2))  # the buffers were cleared after the first flush
        Vk = [vk - alpha * a for vk, a in zip(Vk, acc)]
    else:
        g2 = batch_gradients(1)
        Vk = [vk - alpha * _box(g, t["box"]) for vk, g, t in zip(Vk, g2, tl)]
        acc = passes(sum(g1) + sum(g2))
        Vk = [vk - alpha * a for vk, a in zip(Vk, acc)]
    return [loss], _stitch(spec, tl, Vk)


CASES = [
    # (tiles, halo): 2 x 2 tiles of 28 px >= 2 * 8; 4 x 4 tiles of 14 px < 2 * 8 (tiles two apart overlap)
    ((2, 2), 8),
    ((4, 4), 8),
]


def _check(got, want):
    L_got, V_got = got
    L_want, V_want = want
    np.testing.assert_allclose(L_got, L_want, rtol=1e-12)
    np.testing.assert_allclose(V_got, V_want, rtol=0, atol=1e-12 * np.abs(V_want).max())


@pytest.mark.parametrize("tiles,halo", CASES)
def test_alg1_one_batch_per_tile_closed_form(tiles, halo):
    spec, d, H, meas, alpha = _problem()
    got = oracle.alg1_tiles(d["obj_eval"], d["probe"], d["pos"], meas, H, tiles, halo, alpha,
                            batch=len(d["pos"]), T=1, iterations=1)
    _check(got, _one_batch_per_tile_expected(spec, d, H, meas, alpha, tiles, halo))


@pytest.mark.parametrize("tiles,halo,batch", [((2, 2), 8, 5), ((4, 4), 8, 5)])
@pytest.mark.parametrize("T", [1, 2])
def test_alg1_two_batches_delayed_accumulation(tiles, halo, batch, T):
    spec, d, H, meas, alpha = _problem()
    got = oracle.alg1_tiles(d["obj_eval"], d["probe"], d["pos"], meas, H, tiles, halo, alpha,
                            batch=batch, T=T, iterations=1)
    _check(got, _two_batches_expected(spec, d, H, meas, alpha, tiles, halo, batch, T))


def _mutant(find: str, replace: str):
    src = textwrap.dedent(inspect.getsource(oracle_module.alg1_tiles))
    assert src.count(find) == 1, find
    ns = dict(vars(oracle_module))
    exec(compile(src.replace(find, replace), "<alg1 mutant>", "exec"), ns)
    return ns["alg1_tiles"]


MUTATIONS = {
    "AccBuf never cleared": ('acc[k]["grad"][...] = 0.0', "pass"),
    "passes left out": ("acc = directional_passes(acc, tiles)", "pass"),
    "per-batch step left out": ("V[k] -= step * g", "pass"),
    "window offsets from the wrong box corner": (
        "y0, x0 = int(pos[i][0]) - b[0], int(pos[i][1]) - b[2]",
        "y0, x0 = int(pos[i][0]) - b[2], int(pos[i][1]) - b[0]"),
    "AccBuf cleared before the update": (
        "V[k] -= step * acc[k][\"grad\"]\n                    acc[k][\"grad\"][...] = 0.0",
        "acc[k][\"grad\"][...] = 0.0\n                    V[k] -= step * acc[k][\"grad\"]"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_alg1_pins_catch_planted_mistakes(name):
    """Every planted mistake breaks at least one of the closed forms above."""
    spec, d, H, meas, alpha = _problem()
    bad = _mutant(*MUTATIONS[name])
    runs = [((tiles, halo), dict(batch=len(d["pos"]), T=1),
             _one_batch_per_tile_expected(spec, d, H, meas, alpha, tiles, halo)) for tiles, halo in CASES]
    runs += [(((tiles), halo), dict(batch=b, T=T),
              _two_batches_expected(spec, d, H, meas, alpha, tiles, halo, b, T))
             for tiles, halo, b in [((2, 2), 8, 5), ((4, 4), 8, 5)] for T in (1, 2)]
    caught = 0
    for (tiles, halo), kw, want in runs:
        try:
            got = bad(d["obj_eval"], d["probe"], d["pos"], meas, H, tiles, halo, alpha, iterations=1, **kw)
            _check(got, want)
        except (AssertionError, ValueError, IndexError):
            caught += 1
    assert caught > 0, f"no closed form caught the mistake: {name}"
