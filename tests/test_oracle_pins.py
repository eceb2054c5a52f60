"""Pins of the oracle's iteration and its fixed point.

* one sweep equals the affine map written with independently assembled sparse
  operators (momentum, divergence);
* the first sweep from rest has a closed form;
* the converged k equals the direct sparse solve of the discrete steady system;
* plane Poiseuille flow: the discrete closed form k = (n^2/12 + 1/24) n/(n+s);
* rectangular duct: exact discrete Sylvester solve, and White's series as the
  continuum limit (§6.2);
* Hagen-Poiseuille tube (§6.1) and Kozeny-Carman (§6.3), loose;
* invariants: slice-flux identity, pressure mean per pore, permutation,
  reflection, translation, drive scaling, independence of dt and c^2,
  extrusion;
* stop rules and argument errors.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import oracle.direct as direct
import synth


def random_state(mask, seed):
    rng = np.random.default_rng(seed)
    fs = oracle.face_solid(mask)
    st = oracle.State(*(rng.standard_normal(mask.shape) * 1e-2 for _ in range(4)))
    st.u[fs[0] == 1] = 0
    st.v[fs[1] == 1] = 0
    st.w[fs[2] == 1] = 0
    return st


def small_masks():
    out = [synth.spheres(6, 6, 6, 1.6, 1.6, 0.55, 11),
           synth.spheres(7, 5, 4, 1.3, 1.8, 0.6, 12),
           np.ascontiguousarray(synth.ellipses2d(8, 6, 1.2, 2.0, 0.6, 13)[None])]
    m = np.zeros((5, 6, 7), dtype=np.uint8)
    m[:, 2, :] = 1
    m[1, :, 3] = 1
    out.append(m)
    return out


# ------------------------------------------------------------ one sweep

@pytest.mark.parametrize("mi", range(4))
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sweep_equals_assembled_affine_map(mi, axis):
    mask = small_masks()[mi]
    prm = oracle.params()
    st = random_state(mask, 100 + mi)
    got = oracle.sweep(mask, axis, st, prm)
    sysm = direct.System(mask, axis, re=prm.re, drive=prm.drive)
    want = sysm.sweep(st.u, st.v, st.w, st.p, prm.dt, prm.c2)
    for g, w in zip(got.arrays(), want):
        scale = max(np.abs(w).max(), 1e-300)
        assert np.abs(g - w).max() / scale < 1e-13


def test_first_sweep_closed_form():
    mask = synth.spheres(9, 8, 7, 2.0, 2.0, 0.6, 21)
    prm = oracle.params()
    fs = oracle.face_solid(mask)
    for axis in range(3):
        st = oracle.sweep(mask, axis, oracle.State.zeros(mask.shape), prm)
        # at rest F = G on every fluid face normal to the load axis, zero elsewhere
        vel = [st.u, st.v, st.w]
        for k in range(3):
            want = np.where(fs[k] == 0, prm.dt * prm.drive if k == axis else 0.0, 0.0)
            assert np.array_equal(vel[k], want)
        # the pressure update sees the new velocity: p = -c2 dt div(v')
        f = np.where(fs[axis] == 0, prm.dt * prm.drive, 0.0)
        div = np.roll(f, -1, axis=2 - axis) - f
        assert np.allclose(st.p, -prm.c2 * prm.dt * div, rtol=1e-15, atol=1e-15)


# ------------------------------------------------------------ fixed point

@pytest.mark.parametrize("mi", range(4))
def test_converged_k_equals_direct_solve(mi):
    mask = small_masks()[mi]
    prm = oracle.params(tol=1e-12)
    sols = [direct.solve_steady(mask, axis) for axis in range(3)]
    # normwise: a blocked direction has k ~ 0, measured against the largest entry
    kscale = max(np.abs(s[0]).max() for s in sols)
    for axis in range(3):
        kd, ud, vd, wd, pd, lam = sols[axis]
        r = oracle.solve(mask, axis, prm)
        assert r.status == "OK"
        assert np.abs(r.kcol - kd).max() / kscale < 1e-9, (axis, r.kcol, kd)
        # fields too (pressure has zero mean per pore in both)
        vscale = max(np.abs(f).max() for sol in sols for f in sol[1:4])
        for g, w in zip(r.state.arrays()[:3], (ud, vd, wd)):
            assert np.abs(g - w).max() / vscale < 1e-7
        assert np.abs(r.state.p - pd).max() / max(np.abs(pd).max(), vscale) < 1e-7
        assert np.abs(lam).max() < 1e-9


@pytest.mark.parametrize("n,s", [(1, 1), (2, 1), (3, 2), (4, 1), (5, 3), (8, 2)])
def test_plane_poiseuille_discrete_closed_form(n, s):
    """Channel of n fluid layers between s solid layers, flow along the walls.
    The App. B stencils reproduce the parabola exactly, so
    k = (n^2/12 + 1/24) n / (n + s) in voxel^2 units and no transverse flux."""
    L = n + s
    want = (n * n / 12.0 + 1.0 / 24.0) * n / L
    prm = oracle.params(tol=1e-11)
    for wall_axis, flow_axis in [(1, 0), (2, 1), (0, 2)]:
        shape = [3, 3, 3]
        shape[2 - wall_axis] = L
        m = np.zeros(shape, dtype=np.uint8)
        sl = [slice(None)] * 3
        sl[2 - wall_axis] = slice(n, L)
        m[tuple(sl)] = 1
        r = oracle.solve(m, flow_axis, prm)
        assert r.status == "OK"
        assert r.kcol[flow_axis] == pytest.approx(want, rel=1e-9)
        others = [k for k in range(3) if k != flow_axis]
        assert np.abs(r.kcol[others]).max() < 1e-12 * want


def _channel_matrix(n):
    """1-D matrix of the perpendicular second derivative over n fluid faces
    bounded by solid faces, from the derived stencils."""
    A = np.zeros((n, n))
    for i in range(n):
        def solid(j):
            return int(j < 0 or j >= n)
        pat = (solid(i - 2), solid(i - 1), solid(i + 1), solid(i + 2))
        for off, c in direct.perpendicular_stencil(*pat).items():
            A[i, i + off] += float(c)
    return A


@pytest.mark.parametrize("H,W", [(1, 1), (2, 3), (3, 3), (4, 7), (6, 5)])
def test_rectangular_duct_discrete_sylvester(H, W):
    """Duct of H x W fluid voxels, one solid layer around it, flow along x.
    The discrete equations separate: nu (A_H U + U A_W^T) = -G."""
    prm = oracle.params(tol=1e-11)
    nu = 1.0 / prm.re
    AH, AW = _channel_matrix(H), _channel_matrix(W)
    U = scipy.linalg.solve_sylvester(nu * AH, nu * AW.T, -np.ones((H, W)) * prm.drive)
    N_cross = (H + 1) * (W + 1)
    want = U.sum() / N_cross / (prm.re * prm.drive)
    m = np.ones((W + 1, H + 1, 2), dtype=np.uint8)  # (z, y, x): y spans H, z spans W
    m[:W, :H, :] = 0
    r = oracle.solve(m, 0, prm)
    assert r.status == "OK"
    assert r.kcol[0] == pytest.approx(want, rel=1e-9)


def white_series_mean_velocity_coeff(aspect):
    """Mean velocity of laminar flow in an h x b rectangle (b = aspect * h), in
    units of G h^2 / mu: (1/12) [1 - (192 h / (pi^5 b)) sum_{m odd} tanh(m pi b / (2h)) / m^5]."""
    s = sum(math.tanh(m * math.pi * aspect / 2.0) / m ** 5 for m in range(1, 400, 2))
    return (1.0 - 192.0 / (math.pi ** 5 * aspect) * s) / 12.0


def test_duct_converges_to_white_series():
    """§6.2: channel of height h and width b = 2h against the White (2006)
    series; the discrete mean velocity approaches it as h grows."""
    nu = 100.0
    errs = []
    for h in (4, 8, 16, 32):
        b = 2 * h
        A, B = _channel_matrix(h), _channel_matrix(b)
        U = scipy.linalg.solve_sylvester(nu * A, nu * B.T, -np.ones((h, b)))
        mean = U.mean() * nu / h ** 2  # in units of G h^2 / mu
        errs.append(abs(mean / white_series_mean_velocity_coeff(2.0) - 1.0))
    assert errs[-1] < 5e-3
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    # the square duct value quoted for h = b
    assert white_series_mean_velocity_coeff(1.0) == pytest.approx(0.0351443, rel=2e-5)


def test_hagen_poiseuille_tube_loose():
    """§6.1: voxelised tube, flow along its axis; the mean velocity over the
    tube cross-section approaches the Hagen-Poiseuille value R^2/8 (G/mu)."""
    R = 7.0
    n = 2 * int(R) + 2
    y, z = np.meshgrid(np.arange(n) + 0.5 - n / 2, np.arange(n) + 0.5 - n / 2, indexing="xy")
    solid2d = (y * y + z * z > R * R).astype(np.uint8)  # indexed [z, y]
    m = np.ascontiguousarray(np.repeat(solid2d[:, :, None], 2, axis=2))
    r = oracle.solve(m, 0, oracle.params(tol=1e-9))
    assert r.status == "OK"
    fluid_area = (solid2d == 0).sum()
    k_tube = r.kcol[0] * n * n / fluid_area  # permeability per unit tube area
    r_eff = math.sqrt(fluid_area / math.pi)
    assert k_tube == pytest.approx(r_eff ** 2 / 8.0, rel=0.08)


def test_kozeny_carman_band_simple_cubic():
    """§6.3: simple cubic sphere packing against Kozeny-Carman with c = 180,
    within a factor 2 (a semi-empirical relation)."""
    L, Rs = 20, 7.0
    c = np.arange(L) + 0.5 - L / 2
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    m = ((xx ** 2 + yy ** 2 + zz ** 2) <= Rs ** 2).astype(np.uint8)
    phi = 1.0 - m.mean()
    r = oracle.solve(m, 0, oracle.params(tol=1e-8))
    assert r.status == "OK"
    D = 2 * Rs
    kkc = D ** 2 / 180.0 * phi ** 3 / (1 - phi) ** 2
    assert 0.5 < r.kcol[0] / kkc < 2.0


# ------------------------------------------------------------ invariants

def test_slice_flux_identity_every_sweep():
    """Q_k(s+1) - Q_k(s) = sum of div over layer s (telescoping), for the state
    after any sweep; div is read off the pressure update p' = p - c2 dt div."""
    mask = synth.spheres(10, 9, 8, 2.0, 2.0, 0.55, 31)
    prm = oracle.params()
    st = random_state(mask, 5)
    for _ in range(3):
        new = oracle.sweep(mask, 1, st, prm)
        div = (st.p - new.p) / (prm.c2 * prm.dt)
        qs = oracle.slice_flux(mask, new)
        nz, ny, nx = mask.shape
        for k, n in enumerate((nx, ny, nz)):
            layer = div.sum(axis=tuple(a for a in range(3) if a != 2 - k))
            lhs = np.roll(qs[k, :n], -1) - qs[k, :n]
            assert np.allclose(lhs, layer, rtol=1e-9, atol=1e-13)
        st = new


def test_pressure_mean_zero_per_pore():
    mask = synth.spheres(10, 10, 10, 2.5, 2.5, 0.5, 41)
    st = oracle.run_sweeps(mask, 0, 300)
    from oracle.direct import _components
    fluid = mask == 0
    _, lab = _components(fluid)
    lab = lab.reshape(mask.shape)
    for c in np.unique(lab[fluid]):
        sel = fluid & (lab == c)
        assert abs(st.p[sel].sum()) < 1e-9 * max(1.0, np.abs(st.p).max() * sel.sum())


@pytest.fixture(scope="module")
def aniso_mask():
    return synth.spheres(10, 9, 8, 1.5, 3.0, 0.55, 51)


@pytest.fixture(scope="module")
def aniso_tensor(aniso_mask):
    k, ksym, res = oracle.tensor(aniso_mask, oracle.params(tol=1e-11))
    assert all(r.status == "OK" for r in res)
    return k


def test_tensor_permutation(aniso_mask, aniso_tensor):
    """Permuting the mask axes permutes k."""
    k = aniso_tensor
    # swap x and y: mask[z, y, x] -> mask2[z, x, y]
    m2 = np.ascontiguousarray(aniso_mask.transpose(0, 2, 1))
    k2, _, _ = oracle.tensor(m2, oracle.params(tol=1e-11))
    P = [1, 0, 2]
    assert np.allclose(k2, k[np.ix_(P, P)], rtol=1e-8, atol=1e-9 * np.abs(k).max())


def test_tensor_reflection(aniso_mask, aniso_tensor):
    """Reflecting axis x flips the sign of k_xy, k_xz (and k_yx, k_zx)."""
    k = aniso_tensor
    m2 = np.ascontiguousarray(aniso_mask[:, :, ::-1])
    k2, _, _ = oracle.tensor(m2, oracle.params(tol=1e-11))
    S = np.diag([-1.0, 1.0, 1.0])
    assert np.allclose(k2, S @ k @ S, rtol=1e-8, atol=1e-9 * np.abs(k).max())


def test_tensor_translation(aniso_mask, aniso_tensor):
    m2 = np.ascontiguousarray(np.roll(aniso_mask, (3, -2, 5), axis=(0, 1, 2)))
    k2, _, _ = oracle.tensor(m2, oracle.params(tol=1e-11))
    assert np.allclose(k2, aniso_tensor, rtol=1e-8, atol=1e-9 * np.abs(aniso_tensor).max())


def test_tensor_positive_and_sym_spd(aniso_tensor):
    k = aniso_tensor
    assert (np.diag(k) > 0).all()
    ksym = 0.5 * (k + k.T)
    assert (np.linalg.eigvalsh(ksym) > 0).all()


def test_drive_scaling_leaves_k(aniso_mask):
    r1 = oracle.solve(aniso_mask, 2, oracle.params(tol=1e-11))
    r2 = oracle.solve(aniso_mask, 2, oracle.params(tol=1e-11, drive=3.0))
    assert np.allclose(r1.kcol, r2.kcol, rtol=1e-8, atol=1e-12)
    assert np.allclose(r2.state.w, 3.0 * r1.state.w, rtol=1e-6, atol=1e-12)


def test_fixed_point_independent_of_dt_and_c2(aniso_mask):
    base = oracle.solve(aniso_mask, 0, oracle.params(tol=1e-11))
    for kw in ({"dt": 2.0 ** -13}, {"c2": 0.5e6}, {"re": 0.02}, {"check_every": 37}):
        r = oracle.solve(aniso_mask, 0, oracle.params(tol=1e-11, **kw))
        assert r.status == "OK"
        assert np.allclose(r.kcol, base.kcol, rtol=1e-8, atol=1e-10 * abs(base.kcol[0])), kw


def test_extrusion_invariance():
    """A z-invariant mask gives the same k for nz = 1 and nz = 5."""
    img = synth.ellipses2d(12, 10, 1.5, 2.5, 0.6, 61)
    m1 = np.ascontiguousarray(img[None])
    m5 = np.ascontiguousarray(np.repeat(img[None], 5, axis=0))
    for axis in (0, 1, 2):
        a = oracle.solve(m1, axis, oracle.params(tol=1e-11))
        b = oracle.solve(m5, axis, oracle.params(tol=1e-11))
        assert a.status == b.status == "OK"
        assert np.allclose(a.kcol, b.kcol, rtol=1e-9, atol=1e-13)


def test_divergence_vanishes_at_convergence():
    mask = synth.spheres(12, 12, 12, 2.5, 2.5, 0.5, 71)
    prm = oracle.params(tol=1e-10)
    r = oracle.solve(mask, 1, prm)
    s = oracle.state_sums(mask, 1, r.state, prm)
    nf = int((oracle.face_solid(mask)[1] == 0).sum())
    assert math.sqrt(s[1]) / math.sqrt(nf) < 1e-10
    assert r.hist_r[0] == pytest.approx(1.0, rel=1e-15)
    assert r.hist_sweep[0] == 0


# ------------------------------------------------------------ stop rules / errors

def test_not_converged_and_history():
    mask = synth.spheres(10, 10, 10, 2.5, 2.5, 0.5, 81)
    r = oracle.solve(mask, 0, oracle.params(max_sweeps=250, check_every=100))
    assert r.status == "NOT_CONVERGED"
    assert r.sweeps == 250
    assert list(r.hist_sweep) == [0, 100, 200, 250]
    assert np.isinf(r.hist_eps[0])


def test_diverged_with_unstable_dt():
    mask = synth.spheres(10, 10, 10, 2.5, 2.5, 0.5, 81)
    r = oracle.solve(mask, 0, oracle.params(dt=2.0 ** -10, check_every=20, max_sweeps=20000))
    assert r.status == "DIVERGED"


def test_no_flow_cases():
    solid = np.ones((4, 4, 4), dtype=np.uint8)
    assert oracle.solve(solid, 0).status == "NO_FLOW"
    fluid = np.zeros((4, 4, 4), dtype=np.uint8)
    assert oracle.solve(fluid, 0).status == "NO_FLOW"
    striped = np.zeros((4, 4, 4), dtype=np.uint8)
    striped[:, :, ::2] = 1  # every x-face touches a solid voxel
    assert oracle.solve(striped, 0).status == "NO_FLOW"
    assert oracle.solve(striped, 1).status in ("OK", "NOT_CONVERGED")


def test_bad_arguments():
    m = np.zeros((4, 4, 4), dtype=np.uint8)
    m[0] = 1
    assert oracle.solve(m, 3).status == "ERR_ARG"
    assert oracle.solve(m, 0, oracle.params(dt=0.0)).status == "ERR_ARG"
    assert oracle.solve(m, 0, oracle.params(tol=-1.0)).status == "ERR_ARG"


def test_eps_q_stop_rule():
    mask = synth.spheres(10, 10, 10, 2.5, 2.5, 0.5, 81)
    r = oracle.solve(mask, 0, oracle.params(stop_rule=1, tol=1e-6))
    assert r.status == "OK"
    assert r.hist_eps[-1] < 1e-6


@pytest.mark.parametrize("mi", range(4))
def test_state_sums_against_assembled_operators(mi):
    """S_F, S_D and the face-velocity sums written with the assembled operators."""
    mask = small_masks()[mi]
    prm = oracle.params()
    st = random_state(mask, 200 + mi)
    axis = mi % 3
    sysm = direct.System(mask, axis, re=prm.re, drive=prm.drive)
    x = sysm.pack(st.u, st.v, st.w, st.p)
    F = sysm.Mom @ x + sysm.b
    d = (1.0 / prm.re) * (sysm.Div @ x[:sysm.nF])
    # solid cells have zero divergence (all faces solid), so fluid rows suffice
    got = oracle.state_sums(mask, axis, st, prm)
    assert got[0] == pytest.approx(float(F @ F), rel=1e-12)
    assert got[1] == pytest.approx(float(d @ d), rel=1e-12)
    for k, f in enumerate((st.u, st.v, st.w)):
        assert got[2 + k] == pytest.approx(f.sum(), rel=1e-12, abs=1e-15)


def test_sweep_points_against_assembled_operators():
    mask = synth.spheres(9, 7, 8, 1.8, 2.4, 0.55, 91)
    prm = oracle.params()
    st = random_state(mask, 300)
    sysm = direct.System(mask, 2, re=prm.re, drive=prm.drive)
    want = sysm.sweep(st.u, st.v, st.w, st.p, prm.dt, prm.c2)
    cells = np.random.default_rng(1).choice(mask.size, 60, replace=False)
    got = oracle.sweep_points(mask, 2, st, cells, prm)
    for f in range(4):
        w = want[f].reshape(-1)[cells]
        scale = np.abs(want[f]).max()
        assert np.abs(got[:, f] - w).max() / scale < 1e-13


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_outer_walls_channel_closed_form(n):
    """Outer walls on one axis around n fluid layers, flow along the walls:
    the plane Poiseuille value with no solid layer inside the sample,
    k = n^2/12 + 1/24 exactly, and NO_FLOW for a load across the walls."""
    want = n * n / 12.0 + 1.0 / 24.0
    prm = oracle.params(tol=1e-11)
    for wall_axis, flow_axis in [(1, 0), (2, 1), (0, 2)]:
        shape = [3, 3, 3]
        shape[2 - wall_axis] = n
        m = np.zeros(shape, dtype=np.uint8)
        r = oracle.solve_walls(m, flow_axis, 1 << wall_axis, prm)
        assert r.status == "OK"
        assert r.kcol[flow_axis] == pytest.approx(want, rel=1e-9)
        assert oracle.solve_walls(m, wall_axis, 1 << wall_axis, prm).status == "NO_FLOW"


@pytest.mark.parametrize("H, W", [(3, 4), (6, 5)])
def test_outer_walls_duct_sylvester(H, W):
    """A duct of H x W fluid voxels whose four sides are outer walls: the
    discrete equations separate as for the duct with one solid layer around it,
    now averaged over the H x W cross-section of the sample."""
    prm = oracle.params(tol=1e-11)
    nu = 1.0 / prm.re
    U = scipy.linalg.solve_sylvester(nu * _channel_matrix(H), nu * _channel_matrix(W).T,
                                     -np.ones((H, W)) * prm.drive)
    want = U.sum() / (H * W) / (prm.re * prm.drive)
    m = np.zeros((W, H, 2), dtype=np.uint8)
    r = oracle.solve_walls(m, 0, 0b110, prm)
    assert r.status == "OK"
    assert r.kcol[0] == pytest.approx(want, rel=1e-9)
    assert r.state.u.shape == m.shape


# ------------------------------------------------------------ fixed pressure (§4)
#
# Reading of §4's fixed pressure along the main flow direction, with a flux
# that stays periodic: p~ is held on the cell layer x_axis = 0
# (p = p_in there, p_out = p_in - G n one period later) and that layer's mass
# balance is not imposed.

@pytest.mark.parametrize("mi", range(4))
def test_fixed_pressure_sweep_equals_assembled_affine_map(mi):
    mask = small_masks()[mi]
    prm = oracle.params(fixed_pressure=1)
    for axis in range(3):
        st = random_state(mask, 200 + mi)
        sl = [slice(None)] * 3
        sl[2 - axis] = 0
        st.p[tuple(sl)] = 0.0  # the held value (0 from rest); the assembled map has p = 0 there
        got = oracle.sweep(mask, axis, st, prm)
        sysm = direct.System(mask, axis, re=prm.re, drive=prm.drive, fixed_pressure=True)
        want = sysm.sweep(st.u, st.v, st.w, st.p, prm.dt, prm.c2)
        for g, w in zip(got.arrays(), want):
            assert np.abs(g - w).max() / max(np.abs(w).max(), 1e-300) < 1e-13
        # the held layer keeps its pressure exactly
        assert np.array_equal(got.p[tuple(sl)], st.p[tuple(sl)])


@pytest.mark.parametrize("mi", range(4))
def test_fixed_pressure_converged_k_equals_direct_solve(mi):
    mask = small_masks()[mi]
    prm = oracle.params(tol=1e-12, fixed_pressure=1)
    sols = [direct.solve_steady(mask, axis, fixed_pressure=True) for axis in range(3)]
    kscale = max(np.abs(s[0]).max() for s in sols)
    for axis in range(3):
        kd, ud, vd, wd, pd, lam = sols[axis]
        r = oracle.solve(mask, axis, prm)
        assert r.status == "OK"
        assert np.abs(r.kcol - kd).max() / kscale < 1e-9, (axis, r.kcol, kd)
        vscale = max(np.abs(f).max() for sol in sols for f in sol[1:4])
        for g, w in zip(r.state.arrays(), (ud, vd, wd, pd)):
            assert np.abs(g - w).max() / max(np.abs(w).max(), vscale) < 1e-7


@pytest.mark.parametrize("n,s", [(1, 1), (3, 2), (5, 3)])
def test_fixed_pressure_plane_poiseuille_closed_form(n, s):
    """A channel along the drive has a uniform pressure in every cross-section,
    so holding it on one layer changes nothing: the same discrete closed form."""
    L = n + s
    want = (n * n / 12.0 + 1.0 / 24.0) * n / L
    prm = oracle.params(tol=1e-11, fixed_pressure=1)
    for wall_axis, flow_axis in [(1, 0), (2, 1), (0, 2)]:
        shape = [4, 4, 4]
        shape[2 - wall_axis] = L
        m = np.zeros(shape, dtype=np.uint8)
        sl = [slice(None)] * 3
        sl[2 - wall_axis] = slice(n, L)
        m[tuple(sl)] = 1
        r = oracle.solve(m, flow_axis, prm)
        assert r.status == "OK"
        assert r.kcol[flow_axis] == pytest.approx(want, rel=1e-9)
        others = [k for k in range(3) if k != flow_axis]
        assert np.abs(r.kcol[others]).max() < 1e-12 * want


def test_fixed_pressure_flux_constant_across_slices():
    """Every layer but the held one balances its mass; with a periodic flux the
    held layer's net source is then zero as well, so at the fixed point every
    slice normal to the drive carries the same flux (the held layer only
    redistributes it across the section)."""
    mask = synth.spheres(9, 8, 10, 1.8, 2.4, 0.55, 33)
    for axis in range(3):
        r = oracle.solve(mask, axis, oracle.params(tol=1e-12, fixed_pressure=1))
        assert r.status == "OK"
        qs = oracle.slice_flux(mask, r.state)
        n = mask.shape[2 - axis]
        q = qs[axis, :n]
        assert np.abs(q - q.mean()).max() < 1e-8 * np.abs(q).max()
        assert q.mean() / (mask.size / n) == pytest.approx(r.hist_q[-1][axis], rel=1e-9)


def test_fixed_pressure_reflection_and_difference_from_periodic():
    """Reflecting a transverse axis flips the sign of the coupling (the held
    layer maps to itself); the held layer does change k on a mask whose
    sections are not uniform."""
    mask = synth.spheres(9, 8, 7, 1.8, 2.4, 0.55, 34)
    prm = oracle.params(tol=1e-11, fixed_pressure=1)
    a = oracle.solve(mask, 2, prm)
    b = oracle.solve(np.ascontiguousarray(mask[:, ::-1, :]), 2, prm)
    assert b.kcol[2] == pytest.approx(a.kcol[2], rel=1e-8)
    assert b.kcol[1] == pytest.approx(-a.kcol[1], rel=1e-6, abs=1e-12)
    per = oracle.solve(mask, 2, oracle.params(tol=1e-11))
    assert abs(per.kcol[2] - a.kcol[2]) > 1e-4 * abs(a.kcol[2])
