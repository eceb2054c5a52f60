"""Two sweeps per HBM pass (pm_params.tblock = 2): the two-step kernel applies
the single-step kernel's arithmetic twice, so every iterate, residual history
and k must be bitwise those of tblock = 1 and of the two-pass reference kernel,
for every output tile and z-chunk, on ragged, thin and wrapped grids (a halo,
window or race error would break the equality)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_19868_amd as ps
import synth

pytestmark = pytest.mark.gpu

TILES2 = [(64, 10), (64, 8), (64, 6), (32, 24), (32, 12), (32, 8)]

MASKS = {
    "spheres_70x13x11": lambda: synth.spheres(70, 13, 11, 2.0, 3.0, 0.55, 8),
    "ragged_33x17x6": lambda: synth.spheres(33, 17, 6, 1.5, 2.5, 0.55, 11),
    "thin_3x2x5": lambda: synth.spheres(3, 2, 5, 0.8, 0.8, 0.7, 9),
    "one_cell_x": lambda: np.ascontiguousarray(synth.spheres(1, 9, 8, 1.5, 1.5, 0.6, 10)),
    "extruded_16x16x1": lambda: synth.test_grid(101),
    "spheres_130x45x40": lambda: synth.spheres(130, 45, 40, 2.0, 4.0, 0.5, 12),
}


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = ps.Context(0)
    yield c
    c.close()


def random_state(mask, seed, scale=1e-2):
    rng = np.random.default_rng(seed)
    fs = oracle.face_solid(mask)
    st = [rng.standard_normal(mask.shape) * scale for _ in range(4)]
    for k in range(3):
        st[k][fs[k] == 1] = 0
    return st


def gpu_iterate(ctx, mask, axis, st, count, prec=ps.FP64, **kw):
    dtype = torch.float64 if prec == ps.FP64 else torch.float32
    f = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype) for a in st]
    ctx.iterate(ps.to_device(mask), axis, f, count, ps.params(precision=prec, **kw))
    torch.cuda.synchronize()
    return [t.cpu() for t in f], ctx.last_stats()


@pytest.mark.parametrize("name", sorted(MASKS))
@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32])
def test_two_step_iterate_bitwise(ctx, name, prec):
    mask = MASKS[name]()
    st = random_state(mask, 41)
    for count in (3, 8):
        ref, _ = gpu_iterate(ctx, mask, count % 3, st, count, prec, kernel=ps.KERNEL_SIMPLE)
        for ox, oy in TILES2:
            for zc in (0, 1, 3, 64):
                got, stats = gpu_iterate(ctx, mask, count % 3, st, count, prec, kernel=ps.KERNEL_FUSED, tblock=2,
                                         tile2_x=ox, tile2_y=oy, zchunk2=zc)
                assert stats["tblock"] == 2 and stats["t2_launches"] == (count - 1) // 2
                for g, r in zip(got, ref):
                    assert torch.equal(g, r), (name, count, ox, oy, zc)


def test_two_step_tiles_and_chunks_bitwise(ctx):
    """Each two-step output tile and z-chunk (through the tuning cache path:
    autotune, then a fixed choice per run) against the single-step iterate."""
    mask = MASKS["spheres_130x45x40"]()
    st = random_state(mask, 42)
    m = ps.to_device(mask)
    for prec in (ps.FP64, ps.FP32):
        dtype = torch.float64 if prec == ps.FP64 else torch.float32
        ref, _ = gpu_iterate(ctx, mask, 2, st, 9, prec, tblock=1)
        with ps.Context(0) as c:
            best = c.autotune(m, prec)
            assert best[3] in (1, 2)
            f = [torch.from_numpy(a).to("cuda", dtype) for a in st]
            c.iterate(m, 2, f, 9, ps.params(precision=prec, tblock=2))
            torch.cuda.synchronize()
            assert c.last_stats()["t2_launches"] == 4
            for g, r in zip(f, ref):
                assert torch.equal(g.cpu(), r)


@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32, ps.FP32_DC])
def test_two_step_solve_bitwise(ctx, prec):
    mask = synth.spheres(40, 36, 30, 2.0, 3.5, 0.5, 43)
    m = ps.to_device(mask)
    a = ctx.solve(m, 1, ps.params(precision=prec, tblock=1))
    b = ctx.solve(m, 1, ps.params(precision=prec, tblock=2))
    st = ctx.last_stats()
    assert st["t2_launches"] > 0
    # the plain FP32 form stops at its rounding floor (NOT_CONVERGED)
    assert a.status == b.status == ("NOT_CONVERGED" if prec == ps.FP32 else "OK") and a.sweeps == b.sweeps
    assert np.array_equal(a.kcol, b.kcol) and np.array_equal(a.hist_r, b.hist_r)
    for fa, fb in zip(a.fields, b.fields):
        assert torch.equal(fa, fb)
    c = ctx.solve(m, 1, ps.params(precision=prec, tblock=2, graphs=0))
    assert np.array_equal(c.kcol, b.kcol) and np.array_equal(c.hist_r, b.hist_r)
    if prec == ps.FP64:
        o = oracle.solve(mask, 1, oracle.params())
        assert o.sweeps == b.sweeps
        assert np.abs(b.kcol - o.kcol).max() / np.abs(o.kcol).max() <= 1e-10


def test_two_step_odd_check_interval_bitwise(ctx):
    """Blocks of 7 and 2 sweeps (check_every 7, max_sweeps ending mid-block):
    the plan's single steps fill the remainder."""
    mask = synth.spheres(30, 28, 26, 2.0, 3.0, 0.5, 44)
    m = ps.to_device(mask)
    for ce, ms in ((7, 100), (2, 31), (3, 50)):
        a = ctx.solve(m, 0, ps.params(check_every=ce, max_sweeps=ms, tblock=1))
        b = ctx.solve(m, 0, ps.params(check_every=ce, max_sweeps=ms, tblock=2))
        assert a.status == b.status and a.sweeps == b.sweeps == ms
        assert np.array_equal(a.kcol, b.kcol) and np.array_equal(a.hist_r, b.hist_r)
        for fa, fb in zip(a.fields, b.fields):
            assert torch.equal(fa, fb)


def test_two_step_batch_uneven_bitwise(ctx):
    """Uneven instances in one batch (each its own two-step decomposition)
    against their single-step single solves."""
    masks = [synth.spheres(40, 36, 30, 2.0, 3.5, 0.5, 45), synth.spheres(33, 17, 21, 1.5, 2.5, 0.55, 46),
             synth.spheres(64, 20, 12, 2.0, 3.0, 0.5, 47)]
    probs = [(ps.to_device(mk), a) for mk in masks for a in (0, 2)]
    prm = ps.params(precision=ps.FP32_DC, tblock=2)
    st, res = ctx.solve_batch(probs, prm)
    for (mk, a), r in zip(probs, res):
        g = ctx.solve(mk, a, ps.params(precision=ps.FP32_DC, tblock=1))
        assert r["status"] == g.status == "OK" and r["sweeps"] == g.sweeps
        assert np.array_equal(r["kcol"], g.kcol)


@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32])
def test_two_step_rotated_order_bitwise(ctx, prec):
    """1040 x 180 planes hold 17 x 18 = 306 two-step tiles of 64 x 10: the
    rotated XCD order (ragged in x and y, uneven over the XCDs)."""
    mask = synth.spheres(1040, 180, 4, 2.0, 4.0, 0.5, 48)
    st = random_state(mask, 49)
    ref, _ = gpu_iterate(ctx, mask, 1, st, 5, prec, kernel=ps.KERNEL_SIMPLE)
    got, stats = gpu_iterate(ctx, mask, 1, st, 5, prec, tblock=2, tile2_x=64, tile2_y=10, zchunk2=1)
    assert stats["t2_launches"] == 2
    for g, r in zip(got, ref):
        assert torch.equal(g, r)
