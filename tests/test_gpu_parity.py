"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars (from the method's arithmetic):
  * face flags and stencil codes: bit-exact;
  * kernel variants (tiles, z-chunks, batched, two-pass): bitwise identical iterates;
  * FP64 iterate after N sweeps: <= 1e-12 relative (max-norm over each field);
  * FP64 converged k: <= 1e-10 relative, normwise |dk_ij| / max|k|, same sweep count;
  * FP32 (+ FP64 defect correction) converged k: <= 1e-5 relative, normwise.
"""
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


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def random_state(mask, seed, scale=1e-2):
    rng = np.random.default_rng(seed)
    fs = oracle.face_solid(mask)
    st = oracle.State(*(rng.standard_normal(mask.shape) * scale for _ in range(4)))
    st.u[fs[0] == 1] = 0
    st.v[fs[1] == 1] = 0
    st.w[fs[2] == 1] = 0
    return st


MASKS = {
    "spheres_12x10x9": lambda: synth.spheres(12, 10, 9, 2.0, 2.5, 0.5, 7),
    "spheres_70x13x11": lambda: synth.spheres(70, 13, 11, 2.0, 3.0, 0.55, 8),
    "extruded_16x16x1": lambda: synth.test_grid(101),
    "thin_3x2x5": lambda: synth.spheres(3, 2, 5, 0.8, 0.8, 0.7, 9),
    "one_cell_x": lambda: np.ascontiguousarray(synth.spheres(1, 9, 8, 1.5, 1.5, 0.6, 10)),
    "ragged_33x17x6": lambda: synth.spheres(33, 17, 6, 1.5, 2.5, 0.55, 11),
}


# ------------------------------------------------------------ preprocessing

@pytest.mark.parametrize("name", sorted(MASKS))
def test_face_bits_bit_exact(ctx, name):
    mask = MASKS[name]()
    bits = ctx.preprocess(ps.to_device(mask))
    want = oracle.pack_bits(oracle.face_solid(mask))
    got = bits.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("name", sorted(MASKS))
def test_face_codes_match_oracle_classifier(ctx, name):
    mask = MASKS[name]()
    codes = ctx.face_codes(ps.to_device(mask)).cpu().numpy().view(np.uint32)
    fs = oracle.face_solid(mask)
    nz, ny, nx = mask.shape
    perp = {0: (1, 2), 1: (0, 2), 2: (0, 1)}
    # case number of a 3-bit code L | R<<1 | F<<2
    code_case = {0: 6, 1: 4, 2: 5, 3: 1, 5: 2, 6: 3}
    for k in range(3):
        c = (codes >> np.uint32(8 * k)) & np.uint32(0x7F)
        assert np.array_equal((c >> np.uint32(6)) & np.uint32(1), fs[k].astype(np.uint32))
        for slot, i in enumerate(perp[k]):
            code = (c >> np.uint32(3 * slot)) & np.uint32(7)
            ax = 2 - i
            s = [np.roll(fs[k], -d, axis=ax) for d in (-2, -1, 1, 2)]
            for z in range(nz):
                for y in range(ny):
                    for x in range(nx):
                        want = oracle.case(s[0][z, y, x], s[1][z, y, x], s[2][z, y, x], s[3][z, y, x])
                        got = code_case.get(int(code[z, y, x]), -1)
                        assert got == want, (k, i, x, y, z, int(code[z, y, x]))


# ------------------------------------------------------------ sweeps

def gpu_iterate(ctx, mask, axis, st, count, prec=ps.FP64, **kw):
    dtype = torch.float64 if prec == ps.FP64 else torch.float32
    f = [dev(a, dtype) for a in st.arrays()]
    ctx.iterate(ps.to_device(mask), axis, f, count, ps.params(precision=prec, **kw))
    torch.cuda.synchronize()
    return [host(t) for t in f]


@pytest.mark.parametrize("name", sorted(MASKS))
@pytest.mark.parametrize("count", [1, 2, 7])
def test_iterate_fp64_against_oracle(ctx, name, count):
    mask = MASKS[name]()
    axis = count % 3
    st = random_state(mask, 17 + count)
    prm = oracle.params()
    want = st
    for _ in range(count):
        want = oracle.sweep(mask, axis, want, prm)
    got = gpu_iterate(ctx, mask, axis, st, count)
    for g, w in zip(got, want.arrays()):
        scale = max(np.abs(w).max(), 1e-300)
        assert np.abs(g - w).max() / scale <= 1e-12


TILES = [(64, 8, 0), (64, 8, 3), (32, 16, 1), (32, 8, 5), (32, 16, 2), (64, 8, 64), (64, 16, 1), (64, 16, 0),
         (128, 8, 0), (128, 8, 2)]
TILES_F32 = []


@pytest.mark.parametrize("name", ["spheres_70x13x11", "ragged_33x17x6", "thin_3x2x5", "extruded_16x16x1"])
@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32])
def test_kernel_variants_bitwise(ctx, name, prec):
    """Every tile / z-chunk of the fused kernel and the two-pass kernel give
    bitwise identical iterates (a race or halo error would break this)."""
    mask = MASKS[name]()
    st = random_state(mask, 5)
    ref = gpu_iterate(ctx, mask, 1, st, 9, prec, kernel=ps.KERNEL_SIMPLE)
    for tx, ty, zc in TILES + (TILES_F32 if prec == ps.FP32 else []):
        got = gpu_iterate(ctx, mask, 1, st, 9, prec, kernel=ps.KERNEL_FUSED, tile_x=tx, tile_y=ty,
                          zchunk=zc)
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), (tx, ty, zc)


@pytest.mark.parametrize("shape", [(512, 128, 6), (520, 130, 5)])
@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32])
def test_rotated_block_order_bitwise(ctx, shape, prec):
    """Planes of at least 256 tiles (32x8 tiles here: 256 and 289 per plane,
    the second with ragged edges and an uneven split over the XCDs) take the
    rotated block order; the iterates stay bitwise equal to the two-pass
    kernel's, and to a decomposition without rotation (64 tiles per plane)."""
    nx, ny, nz = shape
    mask = synth.spheres(nx, ny, nz, 2.0, 4.0, 0.5, 31)
    st = random_state(mask, 6)
    ref = gpu_iterate(ctx, mask, 0, st, 5, prec, kernel=ps.KERNEL_SIMPLE)
    for tx, ty, zc in [(32, 8, 2), (32, 8, 0), (64, 16, 0)]:
        got = gpu_iterate(ctx, mask, 0, st, 5, prec, kernel=ps.KERNEL_FUSED, tile_x=tx, tile_y=ty, zchunk=zc)
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), (tx, ty, zc)


@pytest.mark.parametrize("shape", [(512, 128, 6), (520, 130, 5)])
def test_round_major_order_bitwise(ctx, shape):
    """FP64 workgroups of 1024 threads take the round-major order: one-plane
    z-chunks give 384 and 425 workgroups (a full round of 256 and a partial
    one, split unevenly over the XCDs).  Iterates and residual sums stay
    bitwise equal to the two-pass kernel's."""
    nx, ny, nz = shape
    mask = synth.spheres(nx, ny, nz, 2.0, 4.0, 0.5, 32)
    st = random_state(mask, 7)
    ref = gpu_iterate(ctx, mask, 1, st, 5, kernel=ps.KERNEL_SIMPLE)
    for tx, ty, zc in [(64, 16, 1), (128, 8, 1), (128, 8, 0)]:
        got = gpu_iterate(ctx, mask, 1, st, 5, kernel=ps.KERNEL_FUSED, tile_x=tx, tile_y=ty, zchunk=zc)
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), (tx, ty, zc)
    m = ps.to_device(mask)
    a = ctx.solve(m, 1, ps.params(max_sweeps=300, tile_x=128, tile_y=8, zchunk=1))
    b = ctx.solve(m, 1, ps.params(max_sweeps=300, tile_x=64, tile_y=8, zchunk=1))
    assert a.sweeps == b.sweeps == 300
    assert normwise(a.kcol, b.kcol) <= 1e-13


def test_one_workgroup_per_cu_bitwise(ctx):
    """FP32 1024-thread tiles on planes of 1024 tiles (1024 x 1024) launch with
    the LDS reservation that leaves one workgroup per CU; the iterates stay
    bitwise equal to the two-pass kernel's."""
    mask = synth.spheres(1024, 1024, 3, 3.0, 6.0, 0.5, 33)
    st = random_state(mask, 8)
    ref = gpu_iterate(ctx, mask, 2, st, 3, ps.FP32, kernel=ps.KERNEL_SIMPLE)
    for tx, ty in [(128, 8), (64, 16)]:
        got = gpu_iterate(ctx, mask, 2, st, 3, ps.FP32, kernel=ps.KERNEL_FUSED, tile_x=tx, tile_y=ty)
        for g, r in zip(got, ref):
            assert np.array_equal(g, r), (tx, ty)


def test_iterate_fp32_against_oracle(ctx):
    mask = MASKS["spheres_70x13x11"]()
    st = random_state(mask, 3)
    want = st
    for _ in range(5):
        want = oracle.sweep(mask, 0, want, oracle.params())
    got = gpu_iterate(ctx, mask, 0, st, 5, ps.FP32)
    for g, w in zip(got, want.arrays()):
        assert np.abs(g - w).max() / np.abs(w).max() < 1e-5


@pytest.mark.parametrize("name", sorted(MASKS))
def test_residual_sums_against_oracle(ctx, name):
    mask = MASKS[name]()
    st = random_state(mask, 23)
    axis = len(name) % 3
    got = ctx.residual(ps.to_device(mask), axis, [dev(a) for a in st.arrays()])
    want = oracle.state_sums(mask, axis, st)
    assert got[0] == pytest.approx(want[0], rel=1e-12)
    assert got[1] == pytest.approx(want[1], rel=1e-12)
    scale = max(abs(want[2:]).max(), 1e-300)
    assert np.abs(got[2:] - want[2:]).max() / scale < 1e-12


# ------------------------------------------------------------ solves

def normwise(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("seed", range(100, 110))
def test_solve_fp64_test_grids(ctx, seed):
    mask = synth.test_grid(seed)
    axis = seed % 3
    g = ctx.solve(ps.to_device(mask), axis, ps.params())
    o = oracle.solve(mask, axis, oracle.params())
    assert g.status == o.status == "OK"
    assert g.sweeps == o.sweeps
    assert normwise(g.kcol, o.kcol) <= 1e-10
    assert np.array_equal(g.hist_sweep, o.hist_sweep)
    # r is scaled so that r = 1 at rest; near convergence it differs by rounding
    # of the iterate (absolute, relative to that scale)
    assert np.allclose(g.hist_r, o.hist_r, rtol=1e-9, atol=1e-13)
    # fields of the returned state
    for gf, of in zip(g.fields, o.state.arrays()):
        assert np.abs(host(gf) - of).max() / max(np.abs(of).max(), 1e-300) < 1e-8


def test_solve_fp64_single_spheres_32(ctx):
    """32^3 packing, radius 4, porosity 0.40, seed 1, load along x, tol 1e-8."""
    mask = synth.single_spheres_32()
    g = ctx.solve(ps.to_device(mask), 0, ps.params())
    o = oracle.solve(mask, 0, oracle.params())
    assert g.status == o.status == "OK"
    assert g.sweeps == o.sweeps
    assert normwise(g.kcol, o.kcol) <= 1e-10


@pytest.mark.parametrize("seed", [100, 101, 102])
def test_solve_fp32_dc_against_fp64_oracle(ctx, seed):
    mask = synth.test_grid(seed)
    axis = seed % 3
    g = ctx.solve(ps.to_device(mask), axis, ps.params(precision=ps.FP32_DC))
    o = oracle.solve(mask, axis, oracle.params())
    assert g.status == "OK"
    assert normwise(g.kcol, o.kcol) <= 1e-5
    assert g.hist_r[-1] < 1e-8


def test_tensor_against_oracle(ctx):
    mask = synth.spheres(16, 14, 12, 2.0, 3.0, 0.5, 55)
    g = ctx.tensor(ps.to_device(mask), ps.params())
    k, ksym, _ = oracle.tensor(mask, oracle.params())
    assert g.status == "OK"
    assert normwise(g.k, k) <= 1e-10
    assert np.allclose(g.k_sym, 0.5 * (g.k + g.k.T), rtol=0, atol=0)


def test_batch_equals_single_solves(ctx):
    masks = [synth.spheres(20, 18, 16, 2.0, 3.0, 0.5, 60 + i) for i in range(3)]
    masks.append(synth.spheres(33, 9, 14, 1.5, 2.5, 0.55, 64))
    probs = [(ps.to_device(m), i % 3) for i, m in enumerate(masks)]
    st, res = ctx.solve_batch(probs, ps.params())
    assert st == "OK"
    for (m, axis), r in zip(probs, res):
        single = ctx.solve(m, axis, ps.params())
        assert r["status"] == single.status == "OK"
        assert r["sweeps"] == single.sweeps
        assert np.array_equal(r["kcol"], single.kcol)


# ------------------------------------------------------------ stop rules and errors

def test_not_converged_history(ctx):
    mask = synth.spheres(10, 10, 10, 2.5, 2.5, 0.5, 81)
    g = ctx.solve(ps.to_device(mask), 0, ps.params(max_sweeps=250))
    o = oracle.solve(mask, 0, oracle.params(max_sweeps=250))
    assert g.status == o.status == "NOT_CONVERGED"
    assert g.sweeps == 250
    assert list(g.hist_sweep) == [0, 100, 200, 250]
    assert normwise(g.kcol, o.kcol) <= 1e-10


def test_diverged(ctx):
    mask = synth.spheres(10, 10, 10, 2.5, 2.5, 0.5, 81)
    g = ctx.solve(ps.to_device(mask), 0, ps.params(dt=2.0 ** -10, check_every=20, max_sweeps=20000))
    assert g.status == "DIVERGED"


def test_no_flow(ctx):
    solid = np.ones((4, 4, 4), dtype=np.uint8)
    assert ctx.solve(ps.to_device(solid), 0).status == "NO_FLOW"
    fluid = np.zeros((4, 4, 4), dtype=np.uint8)
    assert ctx.solve(ps.to_device(fluid), 0).status == "NO_FLOW"
    striped = np.zeros((4, 4, 4), dtype=np.uint8)
    striped[:, :, ::2] = 1
    assert ctx.solve(ps.to_device(striped), 0).status == "NO_FLOW"


def test_argument_errors(ctx):
    m = ps.to_device(synth.spheres(8, 8, 8, 2.0, 2.0, 0.5, 1))
    with pytest.raises(ps.PorestokesError, match="ERR_ARG"):
        ctx.solve(m, 3)
    with pytest.raises(ps.PorestokesError, match="ERR_ARG"):
        ctx.solve(m, 0, ps.params(tile_x=48, tile_y=8))
    with pytest.raises(ps.PorestokesError, match="ERR_ARG"):
        ctx.solve(m, 0, ps.params(dt=-1.0))


def test_memory_cap(ctx):
    m = ps.to_device(synth.spheres(16, 16, 16, 2.0, 2.0, 0.5, 1))
    with ps.Context(0, mem_cap=4096) as small:
        with pytest.raises(ps.PorestokesError, match="ERR_OOM"):
            small.solve(m, 0)


def test_kept_blocks_are_reused_and_trimmed():
    """Blocks released by one call serve the next call of the same size (held
    memory does not grow, results are identical); pm_trim returns them."""
    m = ps.to_device(synth.spheres(24, 20, 18, 2.0, 3.0, 0.5, 3))
    with ps.Context(0) as c:
        assert c.mem_used() == 0
        a = c.solve(m, 0)
        held = c.mem_used()
        assert held >= c.last_stats()["peak_bytes"] > 0
        b = c.solve(m, 0)
        assert c.mem_used() == held
        assert a.sweeps == b.sweeps and np.array_equal(a.kcol, b.kcol)
        c.trim()
        assert c.mem_used() == 0
        d = c.solve(m, 0)
        assert np.array_equal(a.kcol, d.kcol)


def test_kept_blocks_yield_to_the_cap():
    """Under a cap that fits either of two problems but not both, the blocks kept
    from the first are returned when the second needs room."""
    ma = ps.to_device(synth.spheres(32, 32, 32, 2.0, 3.0, 0.5, 4))
    mb = ps.to_device(synth.spheres(40, 36, 28, 2.0, 3.0, 0.5, 5))
    with ps.Context(0) as c:
        ra = c.solve(ma, 0, ps.params(max_sweeps=200))
        pa = c.last_stats()["peak_bytes"]
        rb = c.solve(mb, 0, ps.params(max_sweeps=200))
        pb = c.last_stats()["peak_bytes"]
    cap = max(pa, pb) + 4096
    assert cap < pa + pb
    with ps.Context(0, mem_cap=cap) as c:
        for m, want in ((ma, ra), (mb, rb), (ma, ra)):
            got = c.solve(m, 0, ps.params(max_sweeps=200))
            assert np.array_equal(got.kcol, want.kcol)
            assert c.mem_used() <= cap


# ------------------------------------------------------------ graphs, tuning, precision forms

def test_graph_replay_equals_direct_launches(ctx):
    mask = synth.spheres(20, 18, 16, 2.0, 3.0, 0.5, 71)
    m = ps.to_device(mask)
    a = ctx.solve(m, 1, ps.params(graphs=1))
    b = ctx.solve(m, 1, ps.params(graphs=0))
    assert a.status == b.status == "OK"
    assert a.sweeps == b.sweeps
    assert np.array_equal(a.kcol, b.kcol)
    assert np.array_equal(a.hist_r, b.hist_r)
    for fa, fb in zip(a.fields, b.fields):
        assert torch.equal(fa, fb)


@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32])
def test_autotune_choice_is_supported_and_exact(prec):
    mask = synth.spheres(40, 36, 30, 2.0, 3.5, 0.5, 72)
    m = ps.to_device(mask)
    with ps.Context(0) as c:
        ref = c.solve(m, 0, ps.params(precision=prec, max_sweeps=300))
        best = c.autotune(m, prec)
        assert tuple(best[:2]) in {(128, 8), (64, 8), (64, 16), (32, 8), (32, 16)} and 1 <= best[2] <= 30
        assert best[3] in (1, 2) and (best[4], best[5]) in {(64, 10), (64, 8), (64, 6), (32, 24), (32, 12), (32, 8)}
        assert 1 <= best[6] <= 30
        tuned = c.solve(m, 0, ps.params(precision=prec, max_sweeps=300))
        st = c.last_stats()
        assert st["tile_x"] == best[0] and st["zchunk"] == best[2] and st["tblock"] == best[3]
        # the iterate is bitwise identical; sums over another block decomposition
        # differ by rounding of the summation order only
        for fa, fb in zip(ref.fields, tuned.fields):
            assert torch.equal(fa, fb)
        assert np.allclose(ref.kcol, tuned.kcol, rtol=1e-13, atol=0)
        assert np.allclose(ref.hist_r, tuned.hist_r, rtol=1e-12, atol=0)


def test_solve_with_autotune_flag(ctx):
    mask = synth.spheres(24, 20, 18, 2.0, 3.0, 0.5, 73)
    m = ps.to_device(mask)
    g = ctx.solve(m, 2, ps.params(autotune=1))
    o = oracle.solve(mask, 2, oracle.params())
    assert g.status == o.status == "OK" and g.sweeps == o.sweeps
    assert normwise(g.kcol, o.kcol) <= 1e-10


def test_fp32_dc_hands_over_to_fp64(ctx):
    """dc_form 1: the FP32 phase stops at its rounding floor (or at tol) and the
    FP64 phase restarts from the promoted state: its first record repeats the
    sweep count."""
    mask = synth.test_grid(102)
    g = ctx.solve(ps.to_device(mask), 1, ps.params(precision=ps.FP32_DC, tol=1e-10, dc_form=1))
    assert g.status == "OK"
    dup = np.nonzero(np.diff(g.hist_sweep) == 0)[0]
    assert dup.size == 1  # one hand-over: FP32 record, then FP64 record at the same sweep
    assert g.hist_r[-1] < 1e-10
    assert ctx.last_stats()["precision"] == ps.FP64
    o = oracle.solve(mask, 1, oracle.params(tol=1e-10))
    assert normwise(g.kcol, o.kcol) <= 1e-7


@pytest.mark.parametrize("seed", [100, 101, 102])
def test_fp32_dc_correction_form_converges_in_fp32(ctx, seed):
    """dc_form 0: after the FP32 phase the correction e (FP32 sweeps with the
    FP64-formed defect of s0 as source) takes s0 + e to tol; the last sweeps
    are FP32 and k matches the FP64 oracle at the same tol."""
    mask = synth.test_grid(seed)
    axis = (seed + 1) % 3
    g = ctx.solve(ps.to_device(mask), axis, ps.params(precision=ps.FP32_DC, tol=1e-10))
    assert g.status == "OK"
    assert g.hist_r[-1] < 1e-10
    dup = np.nonzero(np.diff(g.hist_sweep) == 0)[0]
    assert dup.size == 1  # FP32 phase -> correction form, no promotion to FP64
    assert ctx.last_stats()["precision"] == ps.FP32
    # the record at the hand-over is the residual of s0 (from its FP64 defect):
    # no larger than the FP32 phase's last, which carries FP32 rounding
    assert g.hist_r[dup[0] + 1] <= 10 * g.hist_r[dup[0]]
    o = oracle.solve(mask, axis, oracle.params(tol=1e-10))
    assert normwise(g.kcol, o.kcol) <= 1e-7
    f64 = ctx.solve(ps.to_device(mask), axis, ps.params(tol=1e-10))
    for a, b in zip(g.fields, f64.fields):
        assert a.dtype == torch.float64
        assert float((a - b).abs().max()) <= 1e-6 * float(b.abs().max())


def test_fp32_dc_correction_form_eps_rule(ctx):
    """stop_rule 1 (relative change of |q| between checks) with FP32-DC: the FP32
    iterate's stagnation at its floor and the repeated state at a hand-over
    (eps_q = 0 in both) do not stop the solve; it ends with the FP64 solve's k."""
    mask = synth.test_grid(100)
    prm = dict(stop_rule=1, tol=1e-11)
    g = ctx.solve(ps.to_device(mask), 2, ps.params(precision=ps.FP32_DC, **prm))
    f = ctx.solve(ps.to_device(mask), 2, ps.params(**prm))
    assert g.status == f.status == "OK"
    assert g.sweeps >= f.sweeps - 300
    assert normwise(g.kcol, f.kcol) <= 1e-8


def test_fp32_dc_eps_rule_hands_over_while_r_falls(ctx):
    """eps_q < tol reached by the FP32 phase within three decades of its rounding
    floor, while r still makes a new minimum at every check, hands over to FP64,
    which confirms the rule: the solve ends where the FP64 solve does (96^3
    packing, eps_q < 1e-6: FP64 4300 sweeps; a hand-over that waited for the
    FP32 floor ran 7400 sweeps)."""
    mask = synth.spheres(96, 96, 96, 4.0, 8.0, 0.25, 9)
    m = ps.to_device(mask)
    prm = dict(stop_rule=1, tol=1e-6)
    f = ctx.solve(m, 0, ps.params(**prm))
    g = ctx.solve(m, 0, ps.params(precision=ps.FP32_DC, **prm))
    assert f.status == g.status == "OK"
    hs = np.asarray(g.hist_sweep)
    hand = hs[1:][np.diff(hs) == 0]
    assert len(hand) == 1 and hand[0] <= f.sweeps + 100  # one hand-over, FP32 stopped on eps_q
    assert g.sweeps <= f.sweeps + 300
    assert g.hist_eps[-1] < 1e-6
    # both stop on the same rule a few checks apart: k agrees to the size of the
    # flux change that the rule still allows over those checks
    assert normwise(g.kcol, f.kcol) <= 1e-5


def test_fp32_eps_rule_does_not_stop_on_stagnation(ctx):
    """At its rounding floor an FP32 iterate stops changing and eps_q reads 0:
    that is not convergence (the FP32 form ends NOT_CONVERGED at the floor)."""
    mask = synth.test_grid(100)
    g = ctx.solve(ps.to_device(mask), 2, ps.params(precision=ps.FP32, stop_rule=1, tol=1e-11))
    assert g.status == "NOT_CONVERGED"
    assert g.hist_r[-1] > 1e-8


def test_fp32_dc_correction_form_stops_at_max_sweeps(ctx):
    """A budget that ends inside the correction form returns NOT_CONVERGED with
    s0 + e in the fields and k of the last check."""
    mask = synth.test_grid(102)
    m = ps.to_device(mask)
    full = ctx.solve(m, 1, ps.params(precision=ps.FP32_DC, tol=1e-10))
    hand = full.hist_sweep[np.nonzero(np.diff(full.hist_sweep) == 0)[0][0]]
    assert full.sweeps > hand + 300
    g = ctx.solve(m, 1, ps.params(precision=ps.FP32_DC, tol=1e-10, max_sweeps=int(hand) + 300))
    assert g.status == "NOT_CONVERGED" and g.sweeps == hand + 300
    assert ctx.last_stats()["precision"] == ps.FP32
    # identical history up to the budget: the same sweeps in the same order
    n = len(g.hist_r)
    assert np.array_equal(g.hist_r, full.hist_r[:n])
    assert normwise(g.kcol, full.hist_q[n - 1] / 0.01) <= 1e-12  # k = q / (Re G)
    assert normwise(g.kcol, full.kcol) <= 1e-4
    for t in g.fields:
        assert bool(torch.isfinite(t).all())


def test_fp32_dc_correction_form_batch_equals_single(ctx):
    masks = [synth.test_grid(100), synth.spheres(20, 18, 16, 2.0, 3.0, 0.5, 9)]
    probs = [(ps.to_device(m), a) for m in masks for a in (0, 2)]
    prm = ps.params(precision=ps.FP32_DC)
    st, res = ctx.solve_batch(probs, prm)
    for (m, a), r in zip(probs, res):
        g = ctx.solve(m, a, prm)
        assert r["status"] == g.status == "OK" and r["sweeps"] == g.sweeps
        assert np.array_equal(r["kcol"], g.kcol)


def test_fp32_dc_correction_form_yields_to_the_cap():
    """Without room for the defect field the FP32 iterate is promoted instead:
    the same result as dc_form 1."""
    mask = synth.test_grid(100)  # 35,840 voxels: the defect field needs 573 KB
    m = ps.to_device(mask)
    with ps.Context(0) as c:
        want = c.solve(m, 0, ps.params(precision=ps.FP32_DC, dc_form=1))
        peak = c.last_stats()["peak_bytes"]
    with ps.Context(0, mem_cap=peak + 4096) as c:
        got = c.solve(m, 0, ps.params(precision=ps.FP32_DC))
        assert c.last_stats()["precision"] == ps.FP64
        assert c.last_stats()["dc_promoted_for_memory"] == 1
    assert got.status == want.status == "OK" and got.sweeps == want.sweeps
    assert np.array_equal(got.kcol, want.kcol)


def test_fp32_form_reaches_floor_with_k_within_1e5(ctx):
    mask = synth.test_grid(100)
    g = ctx.solve(ps.to_device(mask), 0, ps.params(precision=ps.FP32))
    o = oracle.solve(mask, 0, oracle.params())
    assert g.status in ("OK", "NOT_CONVERGED")
    assert normwise(g.kcol, o.kcol) <= 1e-5
    assert g.fields[0].dtype == torch.float32


def test_batch_clogged_instance_only_changes_its_status(ctx):
    open_ = synth.spheres(20, 16, 12, 2.0, 2.5, 0.5, 74)
    clogged = open_.copy()
    clogged[:, :, 7] = 1  # a solid wall normal to x blocks flow along x
    probs = [(ps.to_device(open_), 0), (ps.to_device(clogged), 0), (ps.to_device(open_), 1)]
    st, res = ctx.solve_batch(probs, ps.params())
    assert [r["status"] for r in res][0] == "OK" and res[2]["status"] == "OK"
    assert res[1]["status"] == "OK"
    # The solid plane x = 7 carries exactly zero flux, and by the slice-flux
    # identity every x-slice flux differs from it by a sum of cell divergences:
    # |Q_x(s)| <= sqrt(N) |d|_2 with |nu d|_2 <= r G sqrt(N_f) (definition of r).
    # Averaged over the nx slices, k_x = q_x / (Re G) <= nx sqrt(N_f / N) r <= nx r,
    # with r the residual of the reported state (< tol = 1e-8).
    nx = clogged.shape[2]
    r_last = res[1]["r"][-1]
    assert r_last < 1e-8
    assert abs(res[1]["kcol"][0]) <= nx * r_last * (1 + 1e-9)
    single = ctx.solve(probs[0][0], 0)
    assert np.array_equal(res[0]["kcol"], single.kcol)


def test_fp32_dc_stays_fp32_far_above_its_floor(ctx):
    """A very open foam (k ~ 55 voxel^2) converges slowly from r = 1; its FP32
    floor lies near 2^-24 |q| / (dt G) ~ 1e-4.  After 1500 sweeps r is still
    ~0.7: the FP32 phase must go on (the slowly decelerating residual once
    passed for a plateau and handed over to FP64 sweeps at r ~ 0.7)."""
    m = synth.foam_series()[7]
    r = ctx.solve(ps.to_device(m), 2, ps.params(precision=ps.FP32_DC, max_sweeps=1500, tol=1e-12))
    assert r.status == "NOT_CONVERGED"
    assert r.hist_r[-1] > 1e-2
    assert ctx.last_stats()["precision"] == ps.FP32


@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32_DC])
def test_tensor_runs_cases_one_after_another_when_they_do_not_fit(prec):
    """Under a cap that holds one load case but not three, pm_tensor solves the
    axes one after another: the same tensor, sweeps and histories as the batch."""
    mask = synth.test_grid(100)
    m = ps.to_device(mask)
    prm = ps.params(precision=prec)
    with ps.Context(0) as c:
        want = c.tensor(m, prm)
        assert c.last_stats()["tensor_cases_at_once"] == 3
    with ps.Context(0, mem_cap=120 * mask.size) as c:
        got = c.tensor(m, prm)
        st = c.last_stats()
        assert st["tensor_cases_at_once"] == 1
        assert st["dc_promoted_for_memory"] == 0
        assert st["sweep_launches"] > 0
    assert got.status == want.status == "OK"
    assert np.array_equal(got.k, want.k) and np.array_equal(got.sweeps, want.sweeps)
    for a, b in zip(got.hists, want.hists):
        assert np.array_equal(a["r"], b["r"])
