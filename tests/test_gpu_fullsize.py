"""GPU parity at the full sizes of the named workloads.

The oracle cannot iterate these grids to convergence, so the checks are:
  * sweeps from a seeded random state, compared with the oracle's sweep at
    sampled cells (full host arrays up to 256^3, local windows beyond);
  * k columns after a few sweeps of the batched launch the benchmark times
    (three load axes per launch), against the oracle's state sums.
Bars: FP64 1e-12 relative (iterate), 1e-10 (k); FP32 fields against the FP64
oracle 1e-5 relative, normwise.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_19868_amd as ps
import synth

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = ps.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def spheres256():
    log("[fullsize] generating the 256^3 packing")
    return synth.spheres_256()


def random_state(shape, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal(shape) * 1e-2).astype(dtype) for _ in range(4)]


def normwise_fields(got, want):
    return max(np.abs(g - w).max() / np.abs(w).max() for g, w in zip(got, want))


@pytest.mark.parametrize("prec,count", [(ps.FP64, 1), (ps.FP64, 3), (ps.FP32, 2)])
def test_spheres256_sweeps_sampled(ctx, spheres256, prec, count):
    """256^3 packing, default (benchmark) decomposition, oracle sweeps on the host."""
    mask = spheres256
    dt = np.float64 if prec == ps.FP64 else np.float32
    st = random_state(mask.shape, 1000 + count, dt)
    f = [torch.from_numpy(a).cuda() for a in st]
    log(f"[fullsize] 256^3 {'fp64' if prec == ps.FP64 else 'fp32'}: {count} GPU sweeps")
    ctx.iterate(ps.to_device(mask), 1, f, count, ps.params(precision=prec))
    torch.cuda.synchronize()
    want = oracle.State(*(a.astype(np.float64) for a in st))
    # the library zeroes faces touching solid before sweeping; so does the oracle's sweep
    for _ in range(count):
        want = oracle.sweep(mask, 1, want)
    rng = np.random.default_rng(7)
    cells = rng.choice(mask.size, 4096, replace=False)
    got = [t.cpu().numpy().reshape(-1)[cells].astype(np.float64) for t in f]
    ref = [a.reshape(-1)[cells] for a in want.arrays()]
    err = normwise_fields(got, ref)
    log(f"[fullsize] 256^3 sampled rel error {err:.2e}")
    assert err <= (1e-12 if prec == ps.FP64 else 1e-5)


@pytest.mark.timeout(600)
def test_spheres256_tensor_launch_k_after_sweeps(ctx, spheres256):
    """The benchmark's launch (3 load axes in one batched sweep), 5 sweeps:
    k columns of that state against the oracle's."""
    mask = spheres256
    r = ctx.tensor(ps.to_device(mask), ps.params(max_sweeps=5))
    assert r.status == "NOT_CONVERGED" and list(r.sweeps) == [5, 5, 5]
    prm = oracle.params()
    for axis in range(3):
        st = oracle.run_sweeps(mask, axis, 5, prm)
        s = oracle.state_sums(mask, axis, st, prm)
        k = s[2:] / (mask.size * prm.re * prm.drive)
        err = np.abs(r.k[:, axis] - k).max() / np.abs(k).max()
        log(f"[fullsize] tensor column {axis}: rel error {err:.2e}")
        assert err <= 1e-10


def windows(mask, fields_gpu, cells, half=4):
    """Periodic (2 half + 1)^3 windows around cells: mask (host) and fields (GPU gather)."""
    nz, ny, nx = mask.shape
    d = np.arange(-half, half + 1)
    out = []
    for c in cells:
        z, y, x = c // (nx * ny), (c // nx) % ny, c % nx
        zi = (z + d) % nz
        yi = (y + d) % ny
        xi = (x + d) % nx
        mw = np.ascontiguousarray(mask[np.ix_(zi, yi, xi)])
        idx = torch.from_numpy(((zi[:, None, None] * ny + yi[None, :, None]) * nx
                                + xi[None, None, :]).reshape(-1)).cuda()
        fw = [t.reshape(-1).index_select(0, idx).reshape(mw.shape).double().cpu().numpy()
              for t in fields_gpu]
        out.append((mw, fw))
    return out


def check_sampled_one_sweep(ctx, mask, axis, prec, seed, nsamp=48, prm_kw=None):
    """One GPU sweep from a seeded random state; the oracle recomputes the new
    values of sampled cells from local windows of the old state."""
    nz, ny, nx = mask.shape
    dtype = torch.float64 if prec == ps.FP64 else torch.float32
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    f = [(torch.randn(mask.shape, generator=g, device="cuda", dtype=torch.float32) * 1e-2).to(dtype)
         for _ in range(4)]
    rng = np.random.default_rng(seed)
    cells = rng.choice(mask.size, nsamp, replace=False)
    before = windows(mask, f, cells)
    m = ps.to_device(mask)
    ctx.iterate(m, axis, f, 1, ps.params(precision=prec, **(prm_kw or {})))
    torch.cuda.synchronize()
    del m
    flat = [t.reshape(-1) for t in f]
    idx = torch.from_numpy(cells).cuda()
    got = np.stack([t.index_select(0, idx).double().cpu().numpy() for t in flat], axis=1)
    ref = np.zeros_like(got)
    center = 4 * 81 + 4 * 9 + 4
    for j, (mw, fw) in enumerate(before):
        st = oracle.State(*fw)
        ref[j] = oracle.sweep_points(mw, axis, st, [center])[0]
    err = max(np.abs(got[:, k] - ref[:, k]).max() / np.abs(ref[:, k]).max() for k in range(4))
    return err


@pytest.mark.timeout(600)
def test_spheres256_fp32_dc_tensor_equals_fp64(ctx, spheres256):
    """The converged tensor of the 256^3 packing: FP32-DC (FP32 phase, then the
    correction form) against FP64 sweeps throughout, both to r < 1e-8.  The
    two iterates stop at different states within tol; their k agree far
    below it."""
    m = ps.to_device(spheres256)
    log("[fullsize] 256^3 tensor, FP64")
    a = ctx.tensor(m, ps.params())
    log("[fullsize] 256^3 tensor, FP32-DC")
    b = ctx.tensor(m, ps.params(precision=ps.FP32_DC))
    assert a.status == b.status == "OK"
    assert ctx.last_stats()["precision"] == ps.FP32  # the tail ran in the correction form
    assert np.abs(b.k - a.k).max() <= 1e-9 * np.abs(a.k).max()


def test_precipitation_batch_sampled_and_k(ctx):
    """1024x512x18 clogging series (16 states x 2 in-plane load axes = 32
    instances in one batched launch), FP32: the per-instance k after 3 sweeps
    against the oracle for three sampled instances, and one-sweep sampled
    parity on the largest-porosity state."""
    log("[fullsize] generating the precipitation series")
    states = synth.precipitation_series()
    probs = [(ps.to_device(m), axis) for m in states for axis in (0, 1)]
    st, res = ctx.solve_batch(probs, ps.params(precision=ps.FP32, max_sweeps=3))
    assert all(r["sweeps"] == 3 for r in res), [r["sweeps"] for r in res]
    prm = oracle.params()
    for i in (0, 17, 31):
        mask = states[i // 2]
        axis = i % 2
        o = oracle.run_sweeps(mask, axis, 3, prm)
        s = oracle.state_sums(mask, axis, o, prm)
        k = s[2:] / (mask.size * prm.re * prm.drive)
        err = np.abs(res[i]["kcol"] - k).max() / np.abs(k).max()
        log(f"[fullsize] precipitation instance {i}: k rel error {err:.2e}")
        assert err <= 1e-5
    del probs
    err = check_sampled_one_sweep(ctx, states[0], 0, ps.FP64, 11)
    log(f"[fullsize] precipitation state 0 one-sweep sampled error {err:.2e}")
    assert err <= 1e-12


@pytest.mark.timeout(600)
def test_foam_uneven_batch(ctx):
    """Compressed-foam series (512^2 x {512..384}, 8 strain states x 3 load
    axes = 24 instances of uneven size in one batched launch, FP32): every
    instance advances; k of the smallest and largest states after 2 sweeps
    against the oracle."""
    log("[fullsize] generating the foam series")
    states = synth.foam_series()
    probs = [(ps.to_device(m), axis) for m in states for axis in range(3)]
    st, res = ctx.solve_batch(probs, ps.params(precision=ps.FP32, max_sweeps=2))
    assert all(r["sweeps"] == 2 for r in res)
    prm = oracle.params()
    for i in (0, 23):
        mask = states[i // 3]
        axis = i % 3
        o = oracle.run_sweeps(mask, axis, 2, prm)
        s = oracle.state_sums(mask, axis, o, prm)
        k = s[2:] / (mask.size * prm.re * prm.drive)
        err = np.abs(res[i]["kcol"] - k).max() / np.abs(k).max()
        log(f"[fullsize] foam instance {i} ({mask.shape}): k rel error {err:.2e}")
        assert err <= 1e-5


@pytest.mark.timeout(900)
def test_spheres1536_one_sweep_sampled(ctx):
    """1536^3 packing (3.6e9 voxels) in FP32: one sweep, sampled cells against
    the oracle on local windows."""
    log("[fullsize] generating the 1536^3 packing")
    mask = synth.spheres_1536()
    log(f"[fullsize] porosity {1.0 - mask.mean():.4f}; sweeping on the GPU")
    err = check_sampled_one_sweep(ctx, mask, 2, ps.FP32, 15)
    log(f"[fullsize] 1536^3 one-sweep sampled error {err:.2e}")
    assert err <= 1e-5
