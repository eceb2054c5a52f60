"""Pins of the tensor post-processing oracle (oracle/principal.py) to the paper
and to closed forms:

* Table 1 of §6.4: the eigenvalues and the angle computed from the printed
  (k22, k33, k23) of every rotation reproduce the printed k_II, k_III and phi,
  within the rounding of the printed inputs (evaluated over the box of +-0.005
  around them) and of the printed outputs (rounded or truncated);
* the worked example of §6.4 (raw off-diagonals 1.76 / 1.96, 0.364 rad);
* the garbled k23 = 4.57 at alpha = 0 does not reproduce its column, 0.457 does;
* rotated diagonal tensors in a plane and in 3-D return their angle, values
  and axes; classes of designed spectra; trace and determinant invariants.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import principal as ot

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ellipsoid_principal.txt")


def golden_rows():
    rows, example = [], None
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "example":
            example = tuple(map(float, f[1:]))
        else:
            rows.append(tuple(map(float, f)))
    return rows, example


def block(k22, k33, k23, k32=None):
    k = np.eye(3)
    k[1, 1], k[2, 2] = k22, k33
    k[1, 2] = k23
    k[2, 1] = k23 if k32 is None else k32
    return k


def box_range(fn, center, half=0.005):
    """min and max of fn over the corners and centre of the input box."""
    vals = [fn(*center)]
    for signs in itertools.product((-1, 1), repeat=len(center)):
        vals.append(fn(*[c + s * half for c, s in zip(center, signs)]))
    return min(vals), max(vals)


def printed_interval(v, half_unit):
    # a printed value is the exact one rounded (+-half a unit) or truncated (+ one unit)
    return v - half_unit, v + 2 * half_unit


def overlaps(lo, hi, plo, phi_):
    return lo <= phi_ and plo <= hi


ROWS, EXAMPLE = golden_rows()


@pytest.mark.parametrize("row", ROWS, ids=[f"alpha{int(r[0])}" for r in ROWS])
def test_table1_eigenvalues_and_angle(row):
    alpha, k33, k22, k23, k3, k2, phi_deg = row
    lo2 = box_range(lambda a, b, c: ot.plane_angle(block(a, b, c), 1, 2)[1][0], (k22, k33, k23))
    hi2 = box_range(lambda a, b, c: ot.plane_angle(block(a, b, c), 1, 2)[1][1], (k22, k33, k23))
    ang = box_range(lambda a, b, c: math.degrees(ot.plane_angle(block(a, b, c), 1, 2)[0]), (k22, k33, k23))
    assert overlaps(*lo2, *printed_interval(k2, 0.005)), (alpha, lo2, k2)
    assert overlaps(*hi2, *printed_interval(k3, 0.005)), (alpha, hi2, k3)
    assert overlaps(*ang, *printed_interval(phi_deg, 0.05)), (alpha, ang, phi_deg)
    # the larger principal value belongs to the axis near e3, turned by about alpha
    assert abs(math.degrees(ot.plane_angle(block(k22, k33, k23), 1, 2)[0]) - alpha) < 5.0


def test_table1_alpha0_reading():
    alpha, k33, k22, k23, k3, k2, phi_deg = ROWS[0]
    assert alpha == 0 and k23 == 0.457
    phi, lam = ot.plane_angle(block(k22, k33, 4.57), 1, 2)
    assert abs(lam[0] - k2) > 1.0 and abs(lam[1] - k3) > 1.0 and abs(math.degrees(phi) - phi_deg) > 10.0


def test_worked_example():
    k22, k23, k32, k33, k2, k3, phi_rad = EXAMPLE
    k = block(k22, k33, k23, k32)
    ks = ot.symmetric_part(k)
    assert ks[1, 2] == pytest.approx(1.86, abs=1e-12)  # App. C / §6.4: (1.76 + 1.96) / 2
    phi, lam = ot.plane_angle(k, 1, 2)
    assert abs(phi - phi_rad) <= 0.0005 + 0.0007      # printed to 3 decimals; inputs to 2
    assert abs(lam[0] - k2) <= 0.015 and abs(lam[1] - k3) <= 0.015
    # the reading with the sum in the denominator would give 7.8 degrees instead
    assert abs(0.5 * math.atan(2 * 1.86 / (8.71 + 4.54)) - phi_rad) > 0.2


@pytest.mark.parametrize("theta", [-1.4, -0.7, -0.2, 0.0, 0.3, 0.785, 1.2, math.pi / 2])
@pytest.mark.parametrize("ab", [(1, 2), (0, 1), (2, 0)])
def test_plane_angle_of_rotated_block(theta, ab):
    a, b = ab
    lo, hi = 2.5, 7.0
    v_hi = np.zeros(3)
    v_lo = np.zeros(3)
    v_hi[a], v_hi[b] = math.sin(theta), math.cos(theta)
    v_lo[a], v_lo[b] = math.cos(theta), -math.sin(theta)
    c = 3 - a - b
    k = hi * np.outer(v_hi, v_hi) + lo * np.outer(v_lo, v_lo)
    k[c, c] = 1.0
    phi, lam = ot.plane_angle(k, a, b)
    assert lam == pytest.approx([lo, hi], rel=1e-12)
    assert phi == pytest.approx(theta, abs=1e-12)


def random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


@pytest.mark.parametrize("seed", range(6))
def test_principal_of_rotated_diagonal(seed):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(0.1, 10.0, 3))
    q = random_rotation(rng)
    k = q @ np.diag(lam) @ q.T
    skew = rng.normal(size=(3, 3)) * 0.3
    k_raw = k + (skew - skew.T)          # the antisymmetric part is averaged away (App. C)
    p = ot.principal(k_raw, 1e-3)
    assert p.lam == pytest.approx(lam, rel=1e-12)
    for i in range(3):
        assert abs(abs(p.axes[:, i] @ q[:, i]) - 1.0) < 1e-10
    ks = ot.symmetric_part(k_raw)
    assert np.trace(ks) == pytest.approx(lam.sum(), rel=1e-12)
    assert np.linalg.det(ks) == pytest.approx(np.prod(lam), rel=1e-10)


@pytest.mark.parametrize("spectrum, tol, cls, distinct", [
    ((2.0, 2.0, 2.0), 0.05, "isotropic", -1),
    ((2.0, 2.04, 2.08), 0.03, "transverse", 0),   # both neighbouring pairs equal: the closer one counts
    ((2.0, 2.06, 2.08), 0.01, "transverse", 0),
    ((1.0, 2.0, 2.05), 0.05, "transverse", 0),
    ((1.0, 1.02, 2.0), 0.05, "transverse", 2),
    ((1.0, 2.0, 3.0), 0.05, "orthotropic", -1),
    ((1.0, 2.0, 3.0), 0.7, "isotropic", -1),
])
def test_classes(spectrum, tol, cls, distinct):
    q = random_rotation(np.random.default_rng(7))
    k = q @ np.diag(spectrum) @ q.T
    p = ot.principal(k, tol)
    assert (p.cls, p.distinct) == (cls, distinct)
