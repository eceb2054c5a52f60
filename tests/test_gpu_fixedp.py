"""Fixed pressure in the main flow direction (pm_params.fixed_pressure, §4 and
Fig. 2: p~ held on the cell layer x_axis = 0, flux periodic) on the GPU
against the oracle's same reading: iterates after N sweeps within 1e-12,
every kernel variant bitwise equal to the two-pass kernel (the held layer is
met by the own cell, the -x / -y neighbour pressures and, along z, by whole
planes, prologue planes of z-chunks included), converged k within 1e-10 at the
same sweep count, residual sums, and the plane-Poiseuille closed form."""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_19868_amd as ps
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = ps.Context(0)
    yield c
    c.close()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def normwise(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


MASKS = {
    "spheres_24x20x18": lambda: synth.spheres(24, 20, 18, 2.0, 3.0, 0.5, 51),
    "ragged_33x17x6": lambda: synth.spheres(33, 17, 6, 1.5, 2.5, 0.55, 52),
    "thin_3x2x5": lambda: synth.spheres(3, 2, 5, 0.8, 0.8, 0.7, 53),
    "one_cell_x": lambda: np.ascontiguousarray(synth.spheres(1, 9, 8, 1.5, 1.5, 0.6, 54)),
}


def held_state(mask, axis, seed, scale=1e-2):
    """Random state with solid faces zero and the held layer's p~ zero."""
    rng = np.random.default_rng(seed)
    fs = oracle.face_solid(mask)
    st = oracle.State(*(rng.standard_normal(mask.shape) * scale for _ in range(4)))
    st.u[fs[0] == 1] = 0
    st.v[fs[1] == 1] = 0
    st.w[fs[2] == 1] = 0
    sl = [slice(None)] * 3
    sl[2 - axis] = 0
    st.p[tuple(sl)] = 0.0
    return st


def gpu_iterate(ctx, mask, axis, st, count, prec=ps.FP64, **kw):
    dtype = torch.float64 if prec == ps.FP64 else torch.float32
    f = [torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype) for a in st.arrays()]
    ctx.iterate(ps.to_device(mask), axis, f, count, ps.params(precision=prec, fixed_pressure=1, **kw))
    torch.cuda.synchronize()
    return [host(t) for t in f]


@pytest.mark.parametrize("name", sorted(MASKS))
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fixed_pressure_iterate_against_oracle(ctx, name, axis):
    mask = MASKS[name]()
    st = held_state(mask, axis, 61 + axis)
    prm = oracle.params(fixed_pressure=1)
    want = st
    for _ in range(7):
        want = oracle.sweep(mask, axis, want, prm)
    got = gpu_iterate(ctx, mask, axis, st, 7)
    for g, w in zip(got, want.arrays()):
        assert np.abs(g - w).max() / max(np.abs(w).max(), 1e-300) <= 1e-12


@pytest.mark.parametrize("name", sorted(MASKS))
@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32])
def test_fixed_pressure_kernel_variants_bitwise(ctx, name, prec):
    mask = MASKS[name]()
    for axis in range(3):
        st = held_state(mask, axis, 71 + axis)
        ref = gpu_iterate(ctx, mask, axis, st, 9, prec, kernel=ps.KERNEL_SIMPLE)
        variants = [dict(tile_x=64, tile_y=8, zchunk=1), dict(tile_x=32, tile_y=16, zchunk=3),
                    dict(tile_x=128, tile_y=8, zchunk=0), dict(tblock=2, tile2_x=64, tile2_y=8, zchunk2=1),
                    dict(tblock=2, tile2_x=32, tile2_y=12, zchunk2=4)]
        for kw in variants:
            got = gpu_iterate(ctx, mask, axis, st, 9, prec, kernel=ps.KERNEL_FUSED, **kw)
            for g, r in zip(got, ref):
                assert np.array_equal(g, r), (name, axis, kw)


@pytest.mark.parametrize("seed, axis", [(100, 0), (101, 1), (102, 2), (104, 2)])
def test_fixed_pressure_solve_matches_oracle(ctx, seed, axis):
    mask = synth.test_grid(seed)
    print(f"[fixed pressure] seed {seed} axis {axis}", flush=True)
    g = ctx.solve(ps.to_device(mask), axis, ps.params(fixed_pressure=1))
    o = oracle.solve(mask, axis, oracle.params(fixed_pressure=1))
    assert g.status == o.status == "OK"
    assert g.sweeps == o.sweeps
    assert normwise(g.kcol, o.kcol) <= 1e-10
    # r is a root of sums of momentum residuals that cancel O(1) terms: its
    # rounding is absolute (~1e-16 per face), as in the periodic parity test
    assert np.allclose(g.hist_r, o.hist_r, rtol=1e-9, atol=1e-13)
    for gf, of in zip(g.fields, o.state.arrays()):
        assert np.abs(host(gf) - of).max() / max(np.abs(of).max(), 1e-300) < 1e-8
    # the held layer keeps p~ = 0 exactly
    sl = [slice(None)] * 3
    sl[2 - axis] = 0
    assert not host(g.fields[3])[tuple(sl)].any()
    # FP32 fields with the FP64 defect correction: k within 1e-5; two sweeps per pass: bitwise
    d = ctx.solve(ps.to_device(mask), axis, ps.params(fixed_pressure=1, precision=ps.FP32_DC))
    assert d.status == "OK" and normwise(d.kcol, o.kcol) <= 1e-5
    t = ctx.solve(ps.to_device(mask), axis, ps.params(fixed_pressure=1, tblock=2))
    assert t.sweeps == g.sweeps and np.array_equal(t.kcol, g.kcol)


def test_fixed_pressure_residual_sums(ctx):
    mask = MASKS["spheres_24x20x18"]()
    for axis in range(3):
        st = held_state(mask, axis, 81)
        want = oracle.state_sums(mask, axis, st, oracle.params(fixed_pressure=1))
        f = [torch.from_numpy(a).to("cuda", torch.float64) for a in st.arrays()]
        got = ctx.residual(ps.to_device(mask), axis, f, ps.params(fixed_pressure=1))
        assert np.allclose(got, want, rtol=1e-12, atol=1e-14 * np.abs(want).max())
        free = oracle.state_sums(mask, axis, st, oracle.params())
        assert got[1] < free[1]  # the held layer's divergences are left out


def test_fixed_pressure_channel_closed_form(ctx):
    n, s = 5, 3
    m = np.zeros((4, n + s, 6), dtype=np.uint8)  # walls normal to y; flow along x
    m[:, n:, :] = 1
    g = ctx.solve(ps.to_device(m), 0, ps.params(fixed_pressure=1, tol=1e-11))
    assert g.status == "OK"
    assert g.kcol[0] == pytest.approx((n * n / 12.0 + 1.0 / 24.0) * n / (n + s), rel=1e-9)
