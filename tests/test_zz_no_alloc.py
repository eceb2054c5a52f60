"""pm_iterate_static (no device allocation, static scratch per GPU) against
pm_iterate through the C ABI: the same kernels on the same inputs, so the
iterates must be bitwise equal.  Two calls in a row, the second on a smaller
grid, so that the first call's leftovers in the shared scratch cannot leak
into the second's result."""
import numpy as np
import pytest
import torch

import paper_2407_19868_amd as ps
import synth

pytestmark = pytest.mark.gpu


def _state(mask, seed, dtype):
    g = torch.Generator().manual_seed(seed)
    return [(torch.randn(mask.shape, generator=g, dtype=torch.float64) * 1e-2).to("cuda", dtype)
            for _ in range(4)]


@pytest.mark.parametrize("prec", [ps.FP64, ps.FP32])
@pytest.mark.parametrize("kernel,tblock", [(ps.KERNEL_AUTO, 1), (ps.KERNEL_AUTO, 2), (ps.KERNEL_SIMPLE, 1)])
def test_static_iterate_equals_iterate(prec, kernel, tblock):
    torch.cuda.set_device(0)
    dtype = torch.float64 if prec == ps.FP64 else torch.float32
    masks = [synth.spheres(40, 36, 30, 2.0, 3.5, 0.45, 21),   # 43,200 voxels
             synth.spheres(19, 14, 11, 1.5, 2.5, 0.5, 22)]    # smaller, ragged
    prm = ps.params(precision=prec, kernel=kernel, tblock=tblock)
    with ps.Context(0) as c:
        for i, mask in enumerate(masks):
            m = ps.to_device(mask)
            want = c.iterate(m, i, _state(mask, 5 + i, dtype), 7, prm)
            got = c.iterate_static(m, i, _state(mask, 5 + i, dtype), 7, prm)
            torch.cuda.synchronize()
            for a, b in zip(want, got):
                assert torch.equal(a, b)
            assert bool(torch.isfinite(got[3]).all())


def test_static_iterate_rejects_grids_beyond_its_scratch():
    torch.cuda.set_device(0)
    mask = np.zeros((128, 128, 128), dtype=np.uint8)  # 2.10 M voxels: over the FP64 limit (1.97 M)
    mask[:, :, 0] = 1
    m = ps.to_device(mask)
    f = [torch.zeros(mask.shape, dtype=torch.float64, device="cuda") for _ in range(4)]
    with ps.Context(0) as c:
        with pytest.raises(ps.PorestokesError, match="static scratch") as e:
            c.iterate_static(m, 0, f, 3, ps.params())
        assert e.value.status == ps.PM_ERR_ARG
    for t in f:
        assert not bool(t.any())  # nothing written
