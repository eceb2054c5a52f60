"""Oracle for the post-processing of a permeability tensor.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from §2 (the
spectral form eq. 3dK_eigen and the three material classes listed after it),
App. C (averaging the off-diagonal pairs) and §6.4 (the reduced evaluation in
one plane, its angle formula read with k_bb - k_aa in the denominator).  The
eigen-decomposition is numpy's symmetric solver; the angle is taken from the
eigenvector of the larger eigenvalue of the 2x2 block, not from the closed
form, so that the two routes check each other.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def symmetric_part(k) -> np.ndarray:
    """App. C: the off-diagonal pairs averaged, k_sym = (k + k^T) / 2."""
    k = np.asarray(k, dtype=np.float64).reshape(3, 3)
    return 0.5 * (k + k.T)


@dataclass
class PrincipalRef:
    lam: np.ndarray   # principal permeabilities, ascending (k_I, k_II, k_III)
    axes: np.ndarray  # column i: unit principal axis of lam[i] (sign arbitrary)
    cls: str          # "isotropic" | "transverse" | "orthotropic"
    distinct: int     # transverse: index of the value that differs, else -1


def _equal(a: float, b: float, tol: float) -> bool:
    return abs(a - b) <= tol * max(abs(a), abs(b))


def _gap(a: float, b: float) -> float:
    m = max(abs(a), abs(b))
    return abs(a - b) / m if m > 0 else 0.0


def principal(k, rel_tol: float = 0.05) -> PrincipalRef:
    """§2: eigenvalues and eigenvectors of the symmetric tensor, and its class.

    Isotropy: all three principal values equal; transverse anisotropy: exactly
    two equal; orthotropy: all distinct.  Numerically, "equal" means a
    relative difference of at most rel_tol; isotropy is decided on the extreme
    pair, and when both neighbouring pairs are equal the closer pair counts.
    """
    lam, vec = np.linalg.eigh(symmetric_part(k))
    if _equal(lam[0], lam[2], rel_tol):
        return PrincipalRef(lam, vec, "isotropic", -1)
    e01, e12 = _equal(lam[0], lam[1], rel_tol), _equal(lam[1], lam[2], rel_tol)
    if e01 or e12:
        low = e01 and (not e12 or _gap(lam[0], lam[1]) <= _gap(lam[1], lam[2]))
        return PrincipalRef(lam, vec, "transverse", 2 if low else 0)
    return PrincipalRef(lam, vec, "orthotropic", -1)


def plane_angle(k, a: int, b: int) -> tuple[float, np.ndarray]:
    """§6.4: principal directions within the plane of axes a and b.

    Returns (phi, lam): lam the ascending eigenvalues of the block
    [[k_aa, s], [s, k_bb]] with s the averaged off-diagonal pair, and phi the
    angle (in (-pi/2, pi/2]) between e_b and the principal axis of the larger
    value, measured towards e_a: that axis is sin(phi) e_a + cos(phi) e_b.
    """
    k = np.asarray(k, dtype=np.float64).reshape(3, 3)
    s = 0.5 * (k[a, b] + k[b, a])
    block = np.array([[k[a, a], s], [s, k[b, b]]])
    lam, vec = np.linalg.eigh(block)
    va, vb = vec[0, 1], vec[1, 1]  # axis of lam[1] in (e_a, e_b) components
    phi = np.arctan2(va, vb)
    # an axis is a line: fold the angle into (-pi/2, pi/2]
    if phi > np.pi / 2:
        phi -= np.pi
    elif phi <= -np.pi / 2:
        phi += np.pi
    return float(phi), lam
