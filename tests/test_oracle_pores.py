"""Pins of the pore-connectivity oracle (oracle/pores.py):

* hand-built geometries with known components and windings, among them a
  staircase that winds along x and y with no straight channel, and a ring that
  crosses the periodic boundary twice with zero net winding;
* with a solid shell on the low faces (no connection across the boundaries)
  the partition equals scipy.ndimage.label with 6-connectivity;
* the flow itself: a component winds along j exactly when the direct solve of
  the discrete steady Stokes equations (oracle/direct.py) gives k_jj > 0, and
  making the non-winding components solid leaves that k column unchanged;
* labels are constant across every pair of face-adjacent pore voxels and
  each equals the smallest index of its class.
"""
import numpy as np
import pytest
from scipy import ndimage

import synth
from oracle import direct
from oracle import pores as op


def solid(nx, ny, nz):
    return np.ones((nz, ny, nx), dtype=np.uint8)


def check_label_invariants(mask, ref):
    nz, ny, nx = mask.shape
    lab = ref.labels
    assert np.all((lab < 0) == (mask != 0))
    for ax in range(3):
        nb = np.roll(lab, 1, axis=2 - ax)
        both = (lab >= 0) & (nb >= 0)
        assert np.array_equal(lab[both], nb[both])
    flat = lab.reshape(-1)
    for l in np.unique(flat[flat >= 0]):
        idx = np.nonzero(flat == l)[0]
        assert idx.min() == l
    assert ref.n_components == len(np.unique(flat[flat >= 0]))


def test_isolated_cavity():
    m = solid(8, 8, 8)
    m[3:5, 2:4, 5:7] = 0
    ref = op.components(m)
    assert ref.n_components == 1 and ref.percolates == (False, False, False)
    assert ref.labels[3, 2, 5] == (3 * 8 + 2) * 8 + 5
    assert not ref.flow.any()
    check_label_invariants(m, ref)


def test_straight_tube_and_slab():
    m = solid(6, 7, 8)
    m[:, 2, 3] = 0                      # tube along z
    ref = op.components(m)
    assert ref.percolates == (False, False, True)
    assert np.array_equal(ref.flow[:, 2, 3], np.full(8, 4, np.uint8))
    m = solid(6, 7, 8)
    m[5, :, :] = 0                      # slab at z = 5
    ref = op.components(m)
    assert ref.percolates == (True, True, False) and ref.n_components == 1
    assert np.all(ref.flow[5] == 3)


def test_diagonal_staircase_winds_along_x_and_y():
    n = 7
    m = solid(n, n, 3)
    for i in range(n):
        m[1, i, i] = 0
        m[1, i, (i + 1) % n] = 0        # staircase: (i, i) -> (i+1, i) -> (i+1, i+1)
    ref = op.components(m)
    # no straight row or column is open, yet the path winds once along x and once along y
    assert not (m[1] == 0).all(axis=0).any() and not (m[1] == 0).all(axis=1).any()
    assert ref.percolates == (True, True, False)
    assert (1, 1, 0) in ref.windings[ref.labels[1, 0, 0]] or (-1, -1, 0) in ref.windings[ref.labels[1, 0, 0]]


def test_ring_across_boundary_does_not_percolate():
    m = solid(8, 8, 1)
    # rectangle ring spanning unwrapped x = 6..9 (wrapped 6, 7, 0, 1), y = 2..4
    for x in (6, 7, 0, 1):
        m[0, 2, x] = 0
        m[0, 4, x] = 0
    for y in (2, 3, 4):
        m[0, y, 6] = 0
        m[0, y, 1] = 0
    ref = op.components(m)
    assert ref.n_components == 1
    # touches both x faces of the box, but winds around nothing
    assert ref.percolates[0] is False and ref.percolates[1] is False
    # with nz = 1 the z direction is a self-loop of every voxel: any pore voxel winds along z
    assert ref.percolates[2] is True


@pytest.mark.parametrize("seed", range(6))
def test_partition_equals_scipy_when_boundary_sealed(seed):
    rng = np.random.default_rng(seed)
    m = (rng.random((9, 10, 11)) < 0.45).astype(np.uint8)
    m[0, :, :] = 1
    m[:, 0, :] = 1
    m[:, :, 0] = 1
    ref = op.components(m)
    lab_sp, n_sp = ndimage.label(m == 0, structure=ndimage.generate_binary_structure(3, 1))
    assert ref.n_components == n_sp
    assert ref.percolates == (False, False, False)
    # same partition: a bijection between the two labellings
    pore = m == 0
    pairs = set(zip(ref.labels[pore].tolist(), lab_sp[pore].tolist()))
    assert len(pairs) == n_sp
    check_label_invariants(m, ref)


@pytest.mark.parametrize("seed", range(12))
def test_winding_iff_flow_and_cleanup_keeps_k(seed):
    rng = np.random.default_rng(1000 + seed)
    n = 5
    porosity = [0.3, 0.4, 0.5][seed % 3]
    m = (rng.random((n, n, n)) >= porosity).astype(np.uint8)
    if m.all() or not m.any():
        pytest.skip("degenerate draw")
    ref = op.components(m)
    check_label_invariants(m, ref)
    for axis in range(3):
        kcol = direct.solve_steady(m, axis)[0]
        assert (kcol[axis] > 1e-9) == ref.percolates[axis], (axis, kcol)
        if ref.percolates[axis]:
            mc = op.cleaned_mask(m, axis)
            assert np.all(mc >= m)
            kc = direct.solve_steady(mc, axis)[0]
            assert np.abs(kc - kcol).max() <= 1e-9 * max(np.abs(kcol).max(), 1e-30)


def test_test_grids_invariants():
    for seed in (100, 101, 102):
        m = synth.test_grid(seed)
        check_label_invariants(m, op.components(m))
