"""Direct solve of the discrete steady Stokes system (test infrastructure only).

The pseudo-time iteration converges to the steady solution of the discrete
equations (§3: the artificial time derivative vanishes at steady state).  This
module builds those equations explicitly and solves them with a sparse LU, so
the iteration's fixed point can be checked without iterating:

* unknowns: velocity on every fluid face, pressure in every fluid cell, and
  one Lagrange multiplier per connected pore (pressure gauge);
* momentum at each fluid k-face: nu * lap(v_k) - (p(c) - p(c - e_k)) = -G [k = axis];
* mass at each fluid cell: sum_k v_k(c + e_k) - v_k(c) + lambda_pore = 0;
* gauge per pore: sum of p over its cells = 0.

The perpendicular second-derivative stencils are *derived* here, as the paper
derives them (§4 and App. B): a polynomial in the perpendicular coordinate is
fitted, in exact rational arithmetic, through the face value, the wall
positions implied by the neighbouring solid faces (value 0 half a voxel
beyond the last fluid face) and the fluid neighbours the case uses; its
second derivative at the face is the stencil.  Nothing is taken from the
oracle's stencil table, so agreement of the two pins both.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla


def _solve_exact(A, b_cols):
    """Gauss-Jordan over Fractions: returns A^{-1} (square, nonsingular)."""
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [x / pv for x in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [row[n:] for row in M]


def fit_second_derivative(points):
    """points: list of (position, key); key None marks a wall (value 0).
    Fits the polynomial of degree len(points)-1 (<= 3) through the points and
    returns {key: coefficient of that value in f''(0)}."""
    deg = len(points) - 1
    assert 1 <= deg <= 3
    A = [[Fraction(x) ** m for m in range(deg + 1)] for x, _ in points]
    Ainv = _solve_exact(A, None)
    coef = {}
    for j, (_, key) in enumerate(points):
        if key is None:
            continue
        coef[key] = coef.get(key, Fraction(0)) + 2 * Ainv[2][j]
    return coef


@lru_cache(maxsize=None)
def perpendicular_stencil(s_m2: int, s_m1: int, s_p1: int, s_p2: int):
    """Stencil {offset: coefficient} for a fluid face given the solid flags of
    the same-component faces at offsets -2, -1, +1, +2 along a perpendicular axis.

    Geometry (§4, App. B): a solid face at +-1 means a wall at +-1/2; with the
    +-1 face fluid, a solid face at +-2 means a wall at +-3/2.
      walls on both sides              -> points {-1/2 wall, 0, +1/2 wall}
      one wall at -1/2 (other side fluid): {-1/2 wall, 0, +1} plus either the
        wall at +3/2 (face +2 solid) or the fluid face at +2
      mirrored for a wall at +1/2
      no adjacent wall                 -> {-1, 0, +1} (the +-2 faces are not used)
    """
    h = Fraction(1, 2)
    if s_m1 and s_p1:
        pts = [(-h, None), (0, 0), (h, None)]
    elif s_m1:
        pts = [(-h, None), (0, 0), (1, 1), (Fraction(3, 2), None) if s_p2 else (2, 2)]
    elif s_p1:
        pts = [(-2, -2) if not s_m2 else (Fraction(-3, 2), None), (-1, -1), (0, 0), (h, None)]
    else:
        pts = [(-1, -1), (0, 0), (1, 1)]
    return fit_second_derivative(pts)


def _components(fluid: np.ndarray):
    """Connected pores: fluid cells joined through shared (fluid) faces, periodic."""
    nz, ny, nx = fluid.shape
    N = fluid.size
    ids = np.arange(N).reshape(fluid.shape)
    rows, cols = [], []
    for ax in range(3):
        nb = np.roll(ids, -1, axis=2 - ax)
        nbf = np.roll(fluid, -1, axis=2 - ax)
        sel = fluid & nbf
        rows.append(ids[sel])
        cols.append(nb[sel])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    g = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(N, N))
    ncomp, labels = csgraph.connected_components(g, directed=False)
    return ncomp, labels


class System:
    """Assembled discrete steady equations for one mask and load axis."""

    def __init__(self, mask, axis: int, re: float = 0.01, drive: float = 1.0, fixed_pressure: bool = False):
        S = np.ascontiguousarray(mask, dtype=bool)
        self.mask = S
        nz, ny, nx = S.shape
        N = S.size
        nu = 1.0 / re
        self.re, self.drive, self.axis = re, drive, axis
        self.fixed_pressure = fixed_pressure

        def lin(x, y, z):
            return ((z % nz) * ny + (y % ny)) * nx + (x % nx)

        # face solid: touches a solid voxel on either side
        fsolid = []
        for k in range(3):
            back = np.roll(S, 1, axis=2 - k)
            fsolid.append((S | back).reshape(-1))
        self.fsolid = fsolid

        face_index = []
        nF = 0
        for k in range(3):
            idx = -np.ones(N, dtype=np.int64)
            fl = np.nonzero(~fsolid[k])[0]
            idx[fl] = nF + np.arange(fl.size)
            nF += fl.size
            face_index.append(idx)
        fluid = ~S
        cell_index = -np.ones(N, dtype=np.int64)
        # pressure unknowns: every fluid cell, except (fixed pressure, §4) the
        # cells of the layer x_axis = 0, whose p is held at 0 and whose mass
        # balance is not imposed
        unknown = fluid.copy()
        if fixed_pressure:
            layer = [slice(None)] * 3
            layer[2 - axis] = 0
            unknown[tuple(layer)] = False
        fc = np.nonzero(unknown.reshape(-1))[0]
        cell_index[fc] = nF + np.arange(fc.size)
        nC = fc.size
        _, labels = _components(fluid)
        # a pore that reaches the fixed layer has its gauge fixed there; the
        # others keep one multiplier and one gauge row each
        held = np.zeros(labels.max() + 1 if labels.size else 0, dtype=bool)
        if fixed_pressure:
            held[np.unique(labels[(fluid & ~unknown).reshape(-1)])] = True
        fluid_comps = np.array([c for c in np.unique(labels[fc]) if not held[c]], dtype=np.int64)
        comp_index = {c: nF + nC + i for i, c in enumerate(fluid_comps)}
        nL = len(fluid_comps)
        self.face_index, self.cell_index, self.fc = face_index, cell_index, fc
        self.nF, self.nC, self.nL = nF, nC, nL
        self.labels, self.fluid_comps = labels, fluid_comps

        # momentum rows: nu * lap(v_k) - (p(c) - p(c - e_k)); rhs -G [k = axis]
        mr, mc, mv = [], [], []
        self.b = np.zeros(nF)
        row = 0
        for k in range(3):
            for cid in np.nonzero(~fsolid[k])[0]:
                z, y, x = cid // (nx * ny), (cid // nx) % ny, cid % nx
                c = [x, y, z]
                for i in range(3):
                    def off(d, i=i):
                        q = list(c)
                        q[i] += d
                        return lin(*q)
                    if i == k:
                        stencil = {-1: Fraction(1), 0: Fraction(-2), 1: Fraction(1)}
                    else:
                        s = [int(bool(fsolid[k][off(d)])) for d in (-2, -1, 1, 2)]
                        stencil = perpendicular_stencil(*s)
                    for d, coef in stencil.items():
                        fid = off(d)
                        if fsolid[k][fid]:
                            continue  # solid face: exact zero, not an unknown
                        mr.append(row); mc.append(face_index[k][fid]); mv.append(nu * float(coef))
                q = list(c)
                q[k] -= 1
                for cell, sign in ((cid, -1.0), (lin(*q), 1.0)):
                    if cell_index[cell] >= 0:  # a held pressure is 0
                        mr.append(row); mc.append(cell_index[cell]); mv.append(sign)
                self.b[row] = drive if k == axis else 0.0
                row += 1
        # momentum operator over [faces, cells]: F = Mom @ [v; p] + b
        self.Mom = sp.csr_matrix((mv, (mr, mc)), shape=(nF, nF + nC))
        # divergence rows over faces: div(c) = sum_k v_k(c + e_k) - v_k(c)
        dr, dc, dv = [], [], []
        for r, cid in enumerate(fc):
            z, y, x = cid // (nx * ny), (cid // nx) % ny, cid % nx
            c = [x, y, z]
            for k in range(3):
                q = list(c)
                q[k] += 1
                up = lin(*q)
                if not fsolid[k][up]:
                    dr.append(r); dc.append(face_index[k][up]); dv.append(1.0)
                if not fsolid[k][cid]:
                    dr.append(r); dc.append(face_index[k][cid]); dv.append(-1.0)
        self.Div = sp.csr_matrix((dv, (dr, dc)), shape=(nC, nF))

    # -------------------------------------------------------------- helpers
    def pack(self, u, v, w, p):
        """Fields (nz, ny, nx) -> vector [fluid-face velocities; fluid-cell pressures]."""
        x = np.zeros(self.nF + self.nC)
        for k, f in enumerate((u, v, w)):
            f = np.asarray(f).reshape(-1)
            sel = self.face_index[k] >= 0
            x[self.face_index[k][sel]] = f[sel]
        x[self.nF:] = np.asarray(p).reshape(-1)[self.fc]
        return x

    def unpack(self, x, p_full=None):
        N = self.mask.size
        out = []
        for k in range(3):
            f = np.zeros(N)
            sel = self.face_index[k] >= 0
            f[sel] = x[self.face_index[k][sel]]
            out.append(f.reshape(self.mask.shape))
        p = np.zeros(N) if p_full is None else np.asarray(p_full, dtype=np.float64).reshape(-1).copy()
        p[self.fc] = x[self.nF:self.nF + self.nC]
        out.append(p.reshape(self.mask.shape))
        return out

    def sweep(self, u, v, w, p, dt: float, c2: float):
        """The affine pseudo-time map written with the assembled operators:
        v' = v + dt (Mom [v; p] + b) on fluid faces, p' = p - c2 dt Div v'."""
        x = self.pack(u, v, w, p)
        vel = x[:self.nF] + dt * (self.Mom @ x + self.b)
        pres = x[self.nF:] - c2 * dt * (self.Div @ vel)
        return self.unpack(np.concatenate([vel, pres]), p_full=p)

    def solve(self):
        nF, nC, nL = self.nF, self.nC, self.nL
        n = nF + nC + nL
        Mom = self.Mom.tocoo()
        Div = self.Div.tocoo()
        rows = [Mom.row, nF + Div.row]
        cols = [Mom.col, Div.col]
        vals = [Mom.data, Div.data]
        # Lagrange multiplier of each pore in its mass rows, gauge rows sum p = 0
        comp_col = {c: nF + nC + i for i, c in enumerate(self.fluid_comps)}
        lab = self.labels[self.fc]
        gauged = np.array([c in comp_col for c in lab], dtype=bool)
        rows.append(nF + np.arange(nC)[gauged])
        cols.append(np.array([comp_col[c] for c in lab[gauged]], dtype=np.int64))
        vals.append(np.ones(int(gauged.sum())))
        for i, c in enumerate(self.fluid_comps):
            members = np.nonzero(lab == c)[0]
            rows.append(np.full(members.size, nF + nC + i))
            cols.append(nF + members)
            vals.append(np.ones(members.size))
        A = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n, n))
        rhs = np.zeros(n)
        rhs[:nF] = -self.b
        sol = spla.spsolve(A, rhs)
        return sol[:nF + nC], sol[nF + nC:]


def solve_steady(mask, axis: int, re: float = 0.01, drive: float = 1.0, fixed_pressure: bool = False):
    """Discrete steady state for load axis `axis`: returns (kcol, u, v, w, p, lambda).
    kcol[i] = q_i / (Re G), q_i the mean of v_i over all i-faces (App. C).
    fixed_pressure: p held at 0 on the layer x_axis = 0 (§4), no mass rows there."""
    sysm = System(mask, axis, re, drive, fixed_pressure)
    x, lam = sysm.solve()
    u, v, w, p = sysm.unpack(x)
    N = sysm.mask.size
    kcol = np.array([f.sum() / N / (re * drive) for f in (u, v, w)])
    return kcol, u, v, w, p, lam
