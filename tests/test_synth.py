"""Seeded input generators: reproducibility, porosity targets, RNG reference values."""
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_reference_values():
    want = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    s = 0
    for w in want:
        out, s = synth.splitmix64(s)
        assert out == w


def test_spheres_deterministic_and_porosity():
    a = synth.spheres(40, 36, 32, 3.0, 5.0, 0.4, 9)
    b = synth.spheres(40, 36, 32, 3.0, 5.0, 0.4, 9)
    c = synth.spheres(40, 36, 32, 3.0, 5.0, 0.4, 10)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    phi = 1.0 - a.mean()
    assert phi <= 0.4
    assert phi > 0.4 - 0.02  # the last sphere added is small relative to the box


def test_spheres_first_crossing_is_sequential_definition():
    """The parallel stamping equals adding spheres one at a time: removing the
    last sphere (one fewer) must leave porosity above the target."""
    m = synth.spheres(24, 24, 24, 3.0, 3.0, 0.5, 3)
    assert 1.0 - m.mean() <= 0.5
    # a packing with a slightly looser target must be a subset (fewer spheres)
    m2 = synth.spheres(24, 24, 24, 3.0, 3.0, 0.55, 3)
    assert np.all(m2 <= m)


def test_named_small_workloads():
    m = synth.single_spheres_32()
    assert m.shape == (32, 32, 32)
    assert 0.38 < 1.0 - m.mean() <= 0.40
    for s in range(100, 110):
        g = synth.test_grid(s)
        assert g.ndim == 3 and g.any() and not g.all()


def test_precipitation_series_small():
    states = synth.precipitation_series(nx=128, ny=64, depth=4, nstates=5, seed=3)
    assert len(states) == 5
    por = [1.0 - s[1:-1].mean() for s in states]
    assert all(p2 <= p1 for p1, p2 in zip(por, por[1:]))
    for s in states:
        assert s.shape == (6, 64, 128)
        assert s[0].all() and s[-1].all()
    for a, b in zip(states, states[1:]):
        assert np.all(a <= b)  # clogging only adds solid


def test_foam_series_small():
    states = synth.foam_series(n=64, nseeds=12, radius=2.0, nstates=3, seed=4)
    assert [s.shape[0] for s in states] == synth.foam_strain_dims(64, 3)
    assert 0.5 < 1.0 - states[0].mean() < 0.99


@pytest.mark.parametrize("n, axes", [(100, (35.0, 10.0, 35.0)), (50, (17.5, 5.0, 17.5))])
@pytest.mark.parametrize("alpha", [0.0, 20.0, 40.0])
def test_ellipsoid_volume_and_lattice_symmetries(n, axes, alpha):
    """The turned ellipsoid: solid fraction near the analytic volume; turning
    by a further 90 degrees equals rotating the voxel array; -alpha equals the
    mirror image in y; at 45 degrees the body is symmetric under y <-> z.  These
    are exact symmetries of the periodic cell that the flow tests rely on."""
    a, b, c = axes
    m = synth.ellipsoid(n, n, n, a, b, c, alpha)
    assert m.mean() == pytest.approx(4.0 / 3.0 * np.pi * a * b * c / n ** 3, rel=0.02)
    assert np.array_equal(synth.ellipsoid(n, n, n, a, b, c, alpha + 90.0), np.rot90(m, k=1, axes=(0, 1)))
    assert np.array_equal(synth.ellipsoid(n, n, n, a, b, c, -alpha), m[:, ::-1, :])
    m45 = synth.ellipsoid(n, n, n, a, b, c, 45.0)
    assert np.array_equal(m45, m45.transpose(1, 0, 2))
    assert np.array_equal(synth.ellipsoid_100(alpha), synth.ellipsoid(100, 100, 100, 35.0, 10.0, 35.0, alpha))
