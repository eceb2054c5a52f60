"""Sizes at and beyond the library's limits, through the C ABI: empty grids
(a dimension of 0), planes of more than 2^28 voxels (a field plane must stay
below 2^31 bytes, the range of one buffer descriptor) and batches of no
instance are refused with PM_ERR_ARG before any device work, so the small
buffers passed with the oversized dimensions are never read or written; grids
of one voxel, one row or one column are answered without error."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2407_19868_amd as ps
import synth

pytestmark = pytest.mark.gpu

BAD_DIMS = [(0, 4, 4), (4, 0, 4), (4, 4, 0), (-1, 4, 4), ((1 << 14) + 1, 1 << 14, 1), (1 << 31, 1, 1)]


@pytest.fixture(scope="module")
def ctx():
    torch.cuda.set_device(0)
    c = ps.Context(0)
    yield c
    c.close()


def _stream():
    return torch.cuda.current_stream().cuda_stream


@pytest.mark.parametrize("dims", BAD_DIMS)
def test_bad_dims_refused_before_device_work(ctx, dims):
    nx, ny, nz = dims
    mask = torch.zeros(64, dtype=torch.uint8, device="cuda")
    f = [torch.full((64,), 7.0, dtype=torch.float64, device="cuda") for _ in range(4)]
    prm = ps.params()
    k = np.zeros(3)
    sw = ctypes.c_int64(-5)
    lib = ps.load_library()
    st = lib.pm_solve(ctx._h, _stream(), mask.data_ptr(), nx, ny, nz, 1.0, 1.0, 0, ctypes.byref(prm),
                      *[t.data_ptr() for t in f], None, k.ctypes.data, ctypes.byref(sw))
    assert st == ps.PM_ERR_ARG and "dims" in ctx.last_error()
    st = lib.pm_iterate(ctx._h, _stream(), mask.data_ptr(), nx, ny, nz, 0, ctypes.byref(prm),
                        *[t.data_ptr() for t in f], 3)
    assert st == ps.PM_ERR_ARG
    k9, ks9, sw3 = np.zeros(9), np.zeros(9), np.zeros(3, dtype=np.int64)
    st = lib.pm_tensor(ctx._h, _stream(), mask.data_ptr(), nx, ny, nz, 1.0, 1.0, ctypes.byref(prm),
                       k9.ctypes.data, ks9.ctypes.data, None, sw3.ctypes.data)
    assert st == ps.PM_ERR_ARG
    torch.cuda.synchronize()
    for t in f:
        assert bool((t == 7.0).all())  # nothing written
    assert not bool(mask.any())


def test_empty_batch_refused(ctx):
    lib = ps.load_library()
    prm = ps.params()
    st = lib.pm_solve_batch(ctx._h, _stream(), None, 0, ctypes.byref(prm))
    assert st == ps.PM_ERR_ARG


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 7), (5, 1, 1)])
def test_degenerate_grids_solve(ctx, shape):
    """One voxel, one column, one row: an open cell carries the periodic drive
    with nothing to hold it (DIVERGED or NOT_CONVERGED at the budget are the
    outcomes the discrete equations allow), or NO_FLOW; never an error."""
    mask = np.zeros(shape, dtype=np.uint8)
    r = ctx.solve(ps.to_device(mask), 0, ps.params(max_sweeps=300))
    assert r.status in ("NO_FLOW", "DIVERGED", "NOT_CONVERGED", "OK")
    solid = np.ones(shape, dtype=np.uint8)
    assert ctx.solve(ps.to_device(solid), 0, ps.params(max_sweeps=300)).status == "NO_FLOW"
