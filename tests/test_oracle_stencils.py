"""Pins of the oracle's face flags, neighbourhood classifier and App. B stencils.

* the stencil table equals the coefficients printed in App. B (golden file);
* each stencil differentiates exactly every polynomial of its degree that
  vanishes at its walls (the Taylor systems of App. B);
* the classifier agrees, on all 16 neighbour patterns, with stencils derived
  independently by exact polynomial fitting through the implied walls;
* face flags and their bit packing follow the no-penetration definition.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import oracle.direct as direct

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "appendix_b_stencils.txt")


def load_golden():
    rows = {}
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        rows[int(parts[0])] = [Fraction(x) for x in parts[1:]]
    return rows


def oracle_coeffs(cse):
    """Coefficients of the oracle's stencil, read off by unit impulses."""
    out = []
    for j in range(5):
        e = [0.0] * 5
        e[j] = 1.0
        out.append(oracle.d2(cse, *e))
    return out


def test_stencils_match_printed_appendix_b():
    gold = load_golden()
    assert sorted(gold) == list(range(1, 9))
    for cse, coefs in gold.items():
        got = oracle_coeffs(cse)
        for g, c in zip(got, coefs):
            assert g == pytest.approx(float(c), rel=1e-15, abs=0.0), (cse, got, coefs)


# Walls (value 0) and sample offsets of each case; degree of exactness.
CASE_GEOMETRY = {
    1: ([-0.5, 0.5], 3),
    2: ([-0.5, 1.5], 3),
    3: ([-1.5, 0.5], 3),
    4: ([-0.5], 3),
    5: ([0.5], 3),
    6: ([], 3),
    7: ([-0.5], 2),
    8: ([0.5], 2),
}


@pytest.mark.parametrize("cse", range(1, 9))
def test_stencil_exact_for_polynomials_vanishing_at_walls(cse):
    walls, deg = CASE_GEOMETRY[cse]
    rng = np.random.default_rng(cse)
    for trial in range(6):
        # polynomial = prod (x - wall) * free part, total degree <= deg
        free_deg = deg - len(walls)
        coef = [Fraction(int(c)) for c in rng.integers(-9, 10, size=free_deg + 1)]

        def f(x, coef=coef):
            val = sum(c * Fraction(x) ** m for m, c in enumerate(coef))
            for wpos in walls:
                val *= Fraction(x) - Fraction(wpos)
            return val

        # exact f''(0) by finite expansion: f(x) = sum a_m x^m; get a_2 from samples
        xs = [Fraction(i) for i in range(-3, 4)]
        # solve for monomial coefficients up to degree deg+? using 7 samples (deg <= 6)
        A = [[x ** m for m in range(7)] for x in xs]
        inv = direct._solve_exact(A, None)
        a2 = sum(inv[2][j] * f(xs[j]) for j in range(7))
        exact = float(2 * a2)
        vals = [float(f(x)) for x in (-2, -1, 0, 1, 2)]
        got = oracle.d2(cse, *vals)
        assert got == pytest.approx(exact, rel=1e-13, abs=1e-12), (cse, trial, got, exact)


def test_classifier_all_patterns_against_derived_stencils():
    """For every (s-2, s-1, s+1, s+2) pattern the oracle's case stencil equals the
    stencil obtained by fitting a polynomial through the walls the pattern implies."""
    for pat in itertools.product((0, 1), repeat=4):
        cse = oracle.case(*pat)
        derived = direct.perpendicular_stencil(*pat)
        got = oracle_coeffs(cse)
        s_m2, s_m1, s_p1, s_p2 = pat
        solid_at = {-2: s_m2, -1: s_m1, 1: s_p1, 2: s_p2, 0: 0}
        for j, off in enumerate((-2, -1, 0, 1, 2)):
            want = float(derived.get(off, 0))
            if solid_at[off]:
                # a solid face holds an exact zero, its coefficient never matters;
                # the derived stencil never uses it
                assert want == 0.0
                continue
            assert got[j] == pytest.approx(want, rel=1e-15, abs=0.0), (pat, cse, off, got, derived)


def test_classifier_case_numbers():
    # the geometry of each printed case, in flag form
    assert oracle.case(0, 1, 1, 0) == 1
    assert oracle.case(1, 1, 1, 1) == 1
    assert oracle.case(0, 1, 0, 1) == 2
    assert oracle.case(1, 0, 1, 0) == 3
    assert oracle.case(0, 1, 0, 0) == 4
    assert oracle.case(0, 0, 1, 0) == 5
    assert oracle.case(0, 0, 0, 0) == 6
    assert oracle.case(1, 0, 0, 1) == 6


def test_face_solid_definition_small():
    # single solid voxel at (x,y,z) = (1,2,3) in a 4x5x6 box
    m = np.zeros((6, 5, 4), dtype=np.uint8)
    m[3, 2, 1] = 1
    fs = oracle.face_solid(m)
    # the six faces of that voxel: own faces and the faces of the +1 neighbours
    expect = np.zeros_like(fs)
    expect[0, 3, 2, 1] = expect[0, 3, 2, 2] = 1
    expect[1, 3, 2, 1] = expect[1, 3, 3, 1] = 1
    expect[2, 3, 2, 1] = expect[2, 4, 2, 1] = 1
    assert np.array_equal(fs, expect)


def test_face_solid_periodic_wrap():
    m = np.zeros((3, 3, 3), dtype=np.uint8)
    m[0, 0, 2] = 1  # x = 2, last column
    fs = oracle.face_solid(m)
    assert fs[0, 0, 0, 0] == 1  # x-face of cell x=0 touches x=2 through the wrap
    assert fs[0, 0, 0, 2] == 1
    assert fs[0].sum() == 2


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (5, 3, 33), (3, 2, 64), (2, 2, 97)])
def test_pack_bits_layout(shape):
    rng = np.random.default_rng(sum(shape))
    m = (rng.random(shape) < 0.3).astype(np.uint8)
    fs = oracle.face_solid(m)
    bits = oracle.pack_bits(fs)
    nz, ny, nx = shape
    W = (nx + 31) // 32
    assert bits.shape == (3, nz, ny, W)
    for k in range(3):
        for x in range(nx):
            got = (bits[k, :, :, x // 32] >> np.uint32(x % 32)) & np.uint32(1)
            assert np.array_equal(got.astype(np.uint8), fs[k, :, :, x])
    # padding bits beyond nx are zero
    if nx % 32:
        pad = bits[:, :, :, -1] >> np.uint32(nx % 32)
        assert not pad.any()
