"""Persistent sweeps of small instances (pm_params.persistent = 1): each block
of check_every - 1 sweeps of an instance whose fields and codes fit one XCD's
L2 runs as one cooperative launch on one XCD, with a barrier in that XCD's L2
between sweeps.  Every field, residual history and k must be bitwise those of
one launch per sweep (persistent = 0, the default): for single solves in every
precision form, tensors (three instances, three XCDs), batches of more
instances than XCDs mixed with instances too large for the path, odd check
intervals, ragged, thin and one-plane grids, and the fixed-pressure reading.
A stale read after a barrier, a missed barrier or a wrong sweep parity would
break the equality.  The 32^3 solve is also held to the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_19868_amd as ps
import synth

pytestmark = pytest.mark.gpu

MASKS = {
    "spheres_32": synth.single_spheres_32,
    "spheres_40x36x30": lambda: synth.spheres(40, 36, 30, 2.0, 3.5, 0.5, 43),
    "ragged_33x17x6": lambda: synth.spheres(33, 17, 6, 1.5, 2.5, 0.55, 11),
    "thin_3x2x5": lambda: synth.spheres(3, 2, 5, 0.8, 0.8, 0.7, 9),
    "one_cell_x": lambda: np.ascontiguousarray(synth.spheres(1, 9, 8, 1.5, 1.5, 0.6, 10)),
    "extruded_16x16x1": lambda: synth.test_grid(101),
}


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = ps.Context(0)
    yield c
    c.close()


def assert_same(a, b):
    assert a.status == b.status and a.sweeps == b.sweeps
    assert np.array_equal(a.kcol, b.kcol)
    assert np.array_equal(a.hist_sweep, b.hist_sweep) and np.array_equal(a.hist_r, b.hist_r)
    for fa, fb in zip(a.fields, b.fields):
        assert torch.equal(fa, fb)


@pytest.mark.parametrize("name", sorted(MASKS))
@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32, ps.FP32_DC])
def test_persistent_solve_bitwise(ctx, name, prec):
    mask = MASKS[name]()
    m = ps.to_device(mask)
    axis = len(name) % 3
    ref = ctx.solve(m, axis, ps.params(precision=prec, persistent=0, max_sweeps=3000))
    assert ctx.last_stats()["pers_launches"] == 0
    got = ctx.solve(m, axis, ps.params(precision=prec, max_sweeps=3000, persistent=1))
    st = ctx.last_stats()
    if ref.status != "NO_FLOW":
        assert st["pers_launches"] > 0 and st["pers_sweeps"] > 0
    assert_same(got, ref)


def test_persistent_c1_against_oracle(ctx):
    """The 32^3 single solve (FP64, r < 1e-8) through the persistent path: the
    oracle's sweep count and k within 1e-10."""
    mask = synth.single_spheres_32()
    got = ctx.solve(ps.to_device(mask), 0, ps.params(persistent=1))
    st = ctx.last_stats()
    assert st["pers_launches"] > 0
    o = oracle.solve(mask, 0, oracle.params())
    assert got.status == "OK" and got.sweeps == o.sweeps
    assert np.abs(got.kcol - o.kcol).max() / np.abs(o.kcol).max() <= 1e-10
    # 1400 sweeps in blocks of 100: 14 persistent launches of 99 sweeps each
    assert st["pers_launches"] == got.sweeps // 100 and st["pers_sweeps"] == 99 * st["pers_launches"]


@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32_DC])
def test_persistent_tensor_bitwise(ctx, prec):
    m = ps.to_device(synth.spheres(28, 30, 26, 2.0, 3.0, 0.5, 51))
    a = ctx.tensor(m, ps.params(precision=prec, persistent=0))
    b = ctx.tensor(m, ps.params(precision=prec, persistent=1))
    assert ctx.last_stats()["pers_launches"] > 0
    assert a.status == b.status == "OK"
    assert np.array_equal(a.sweeps, b.sweeps) and np.array_equal(a.k, b.k)


def test_persistent_batch_mixed_bitwise(ctx):
    """Eleven small instances (more than the eight XCDs: two persistent
    launches per block) of uneven sizes and axes, plus one too large for the
    path, against the same batch with one launch per sweep."""
    masks = [synth.spheres(20 + 3 * i, 24 - i, 14 + 2 * i, 1.5, 3.0, 0.5, 60 + i) for i in range(11)]
    masks.append(synth.spheres(96, 96, 64, 2.0, 4.0, 0.45, 72))  # 4.7 MB per set in FP64
    probs = [(ps.to_device(mk), i % 3) for i, mk in enumerate(masks)]
    for prec in (ps.FP64, ps.FP32):
        st_a, ra = ctx.solve_batch(probs, ps.params(precision=prec, persistent=0, max_sweeps=1500))
        st_b, rb = ctx.solve_batch(probs, ps.params(precision=prec, max_sweeps=1500, persistent=1))
        stats = ctx.last_stats()
        assert stats["pers_launches"] >= 2
        assert st_a == st_b
        for x, y in zip(ra, rb):
            assert x["status"] == y["status"] and x["sweeps"] == y["sweeps"]
            assert np.array_equal(x["kcol"], y["kcol"])


def test_persistent_odd_check_intervals_bitwise(ctx):
    """Blocks of 7, 2 and 3 sweeps (persistent launches of 6, 1 and 2 sweeps)
    and a budget ending mid-block."""
    m = ps.to_device(synth.spheres(30, 28, 26, 2.0, 3.0, 0.5, 44))
    for ce, ms in ((7, 100), (2, 31), (3, 50)):
        a = ctx.solve(m, 0, ps.params(check_every=ce, max_sweeps=ms, persistent=0))
        b = ctx.solve(m, 0, ps.params(check_every=ce, max_sweeps=ms, persistent=1))
        assert ctx.last_stats()["pers_launches"] > 0
        assert_same(a, b)


def test_persistent_fixed_pressure_bitwise(ctx):
    m = ps.to_device(synth.spheres(24, 20, 18, 1.5, 3.0, 0.5, 52))
    for axis in range(3):
        a = ctx.solve(m, axis, ps.params(fixed_pressure=1, persistent=0, max_sweeps=2000))
        b = ctx.solve(m, axis, ps.params(fixed_pressure=1, max_sweeps=2000, persistent=1))
        assert ctx.last_stats()["pers_launches"] > 0
        assert_same(a, b)


def test_persistent_rejects_bad_flag(ctx):
    m = ps.to_device(synth.single_spheres_32())
    with pytest.raises(ps.PorestokesError) as e:
        ctx.solve(m, 0, ps.params(persistent=2))
    assert e.value.status == ps.PM_ERR_ARG
