"""Pore connectivity on the GPU (pm_pores, pm_params.pore_cleanup) against the
oracle (oracle/pores.py).

Bars: labels, flow bits and counts bit-exact (integer work); solves on the
cleaned mask equal the oracle's solve of the same cleaned mask (same sweeps, k
within 1e-10 normwise); cleanup leaves the converged k of the original mask
unchanged (the removed components carry no flow); an axis along which nothing
winds is NO_FLOW without a sweep.  At the full size of the clogging series,
where the oracle is too slow, the labelling is checked through properties
that hold at any size.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2407_19868_amd as ps
import synth
from oracle import pores as op

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = ps.Context(0)
    yield c
    c.close()


def solid(nx, ny, nz):
    return np.ones((nz, ny, nx), dtype=np.uint8)


def staircase():
    m = solid(7, 7, 3)
    for i in range(7):
        m[1, i, i] = 0
        m[1, i, (i + 1) % 7] = 0
    return m


def ring():
    m = solid(8, 8, 2)
    for x in (6, 7, 0, 1):
        m[0, 2, x] = m[0, 4, x] = 0
    for y in (2, 3, 4):
        m[0, y, 6] = m[0, y, 1] = 0
    return m


def tube_z():
    m = solid(6, 7, 8)
    m[:, 2, 3] = 0
    return m


def random_sites(shape, pore, seed):
    rng = np.random.default_rng(seed)
    return (rng.random(shape) >= pore).astype(np.uint8)


MASKS = {
    "staircase": staircase,
    "ring": ring,
    "tube_z": lambda: tube_z(),
    "all_pore": lambda: np.zeros((5, 6, 7), np.uint8),
    "all_solid": lambda: solid(7, 6, 5),
    "sites_0.25": lambda: random_sites((16, 18, 20), 0.25, 1),
    "sites_0.31": lambda: random_sites((16, 18, 20), 0.31, 2),
    "sites_0.40": lambda: random_sites((20, 20, 20), 0.40, 3),
    "sites_0.31_flat": lambda: random_sites((3, 40, 37), 0.31, 4),
    "test_grid_100": lambda: synth.test_grid(100),
    "test_grid_101": lambda: synth.test_grid(101),
    "test_grid_102": lambda: synth.test_grid(102),
}


@pytest.mark.parametrize("name", sorted(MASKS))
def test_labels_flow_and_counts_bit_exact(ctx, name):
    mask = MASKS[name]()
    print(f"[pores] {name} {mask.shape}", flush=True)
    got = ctx.pores(ps.to_device(mask))
    ref = op.components(mask)
    assert np.array_equal(got["labels"].cpu().numpy(), ref.labels)
    assert np.array_equal(got["flow"].cpu().numpy(), ref.flow)
    assert got["n_components"] == ref.n_components
    assert got["n_pore"] == int((mask == 0).sum())
    assert got["percolates"] == ref.percolates
    for j in range(3):
        assert got["n_flowing"][j] == int(((ref.flow >> j) & 1).sum())
        winding = {l for l, ws in ref.windings.items() if any(w[j] for w in ws)}
        assert got["n_flowing_components"][j] == len(winding)


CLEAN = [("sites_0.40", 0), ("sites_0.40", 1), ("sites_0.40", 2), ("pockets", 0), ("pockets", 2)]


def pockets():
    """A packing with isolated cavities: spheres plus sealed bubbles."""
    m = synth.spheres(14, 13, 12, 2.0, 3.0, 0.45, 21)
    m[6:8, 3:5, 2:4] = 1
    m[6, 3, 2] = 0               # one-voxel cavity walled in...
    m[5, 3, 2] = m[7, 3, 2] = m[6, 2, 2] = m[6, 4, 2] = m[6, 3, 1] = m[6, 3, 3] = 1
    return m


@pytest.mark.parametrize("name, axis", CLEAN)
def test_cleanup_solve_matches_oracle_on_cleaned_mask(ctx, name, axis):
    mask = pockets() if name == "pockets" else MASKS[name]()
    cleaned = op.cleaned_mask(mask, axis)
    ref = op.components(mask)
    if not ref.percolates[axis]:
        pytest.skip("axis does not percolate")
    g = ctx.solve(ps.to_device(mask), axis, ps.params(pore_cleanup=1))
    o = oracle.solve(cleaned, axis, oracle.params())
    assert g.status == o.status == "OK"
    assert g.sweeps == o.sweeps
    assert np.abs(g.kcol - o.kcol).max() <= 1e-10 * np.abs(o.kcol).max()
    # the same fixed point as without cleanup
    tight = dict(tol=1e-11)
    g0 = ctx.solve(ps.to_device(mask), axis, ps.params(**tight))
    g1 = ctx.solve(ps.to_device(mask), axis, ps.params(pore_cleanup=1, **tight))
    assert g0.status == g1.status == "OK"
    assert np.abs(g0.kcol - g1.kcol).max() <= 1e-8 * np.abs(g0.kcol).max()


def test_cleanup_no_flow_axis_without_sweeps(ctx):
    m = solid(8, 9, 10)
    m[:, 4, 5] = 0                     # a tube along z only, plus a cavity
    m[2, 1:3, 1:3] = 0
    r = ctx.tensor(ps.to_device(m), ps.params(pore_cleanup=1))
    assert r.status == "NO_FLOW"
    assert list(r.sweeps[:2]) == [0, 0] and r.sweeps[2] > 0
    assert np.all(r.k[:, :2] == 0)
    # the tube's k_zz is the same with and without cleanup
    r0 = ctx.tensor(ps.to_device(m), ps.params())
    assert r0.k[2, 2] == pytest.approx(r.k[2, 2], rel=1e-8)


def test_batch_with_cleanup_equals_single_solves(ctx):
    masks = [pockets(), MASKS["sites_0.40"]()]
    probs = [(ps.to_device(m), a) for m in masks for a in (0, 2)]
    st, res = ctx.solve_batch(probs, ps.params(pore_cleanup=1))
    for (m, a), r in zip(probs, res):
        g = ctx.solve(m, a, ps.params(pore_cleanup=1))
        assert r["status"] == g.status and r["sweeps"] == g.sweeps
        assert np.array_equal(r["kcol"], g.kcol)


def test_clogging_series_labelling_properties(ctx):
    """Full size (1024 x 512 x 18, 16 states): labels agree across every pair of
    face-adjacent pore voxels (periodic), every label is a pore voxel carrying
    its own index and the smallest index of its class, flow bits are constant
    per component, and clogging (solid only grows) never turns percolation on."""
    states = synth.precipitation_series()
    prev = (True, True, True)
    for s, m in enumerate(states):
        print(f"[pores] clogging state {s}", flush=True)
        md = ps.to_device(m)
        got = ctx.pores(md)
        lab, flow = got["labels"], got["flow"]
        pore = md == 0
        assert torch.equal(lab >= 0, pore)
        for dim in range(3):
            nb = torch.roll(lab, 1, dims=dim)
            both = (lab >= 0) & (nb >= 0)
            assert torch.equal(lab[both], nb[both])
            nbf = torch.roll(flow, 1, dims=dim)
            assert torch.equal(flow[both], nbf[both])
        flat = lab.reshape(-1)
        roots = torch.nonzero(flat == torch.arange(flat.numel(), device=flat.device)).reshape(-1)
        assert roots.numel() == got["n_components"]
        used = torch.unique(flat[flat >= 0])
        assert torch.equal(used, roots)
        # smallest index: no voxel carries a label larger than its own index
        idx = torch.arange(flat.numel(), device=flat.device)
        assert bool(torch.all(flat[flat >= 0] <= idx[flat >= 0]))
        # the walls at z = 0 and z = 17 are solid: nothing winds along z
        assert got["percolates"][2] is False
        for j in range(3):
            assert not (got["percolates"][j] and not prev[j])
        prev = got["percolates"]
