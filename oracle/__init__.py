"""CPU oracle for the pseudo-unsteady Stokes permeability method.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the solver library.  The
iteration is plain FP64 C (``oracle.c``) loaded with ctypes; ``direct.py``
holds an independent direct solve of the discrete steady equations that pins
the iteration's fixed point.

Every function states the passage of the paper it follows; the shared
conventions (grid, face flags, cases, drive, Darcy scaling) are listed at the
top of ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 4: "NOT_CONVERGED", 5: "DIVERGED", 6: "NO_FLOW"}


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("re", ctypes.c_double),
        ("c2", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("drive", ctypes.c_double),
        ("voxel_size", ctypes.c_double),
        ("max_sweeps", ctypes.c_int64),
        ("check_every", ctypes.c_int32),
        ("warm_start", ctypes.c_int32),
        ("stop_rule", ctypes.c_int32),
        ("fixed_pressure", ctypes.c_int32),
    ]


def params(**kw) -> OrcParams:
    """Defaults: Re = 0.01 and c*^2 = 1.5e6 (§4 "Simulation parametrization"),
    drive G = 1 per voxel, dt = 2^-12, tol = 1e-8, residual check every 100 sweeps,
    periodic p~ along the load axis (fixed_pressure=1: held on the layer x_axis = 0)."""
    p = OrcParams(re=0.01, c2=1.5e6, dt=2.0**-12, tol=1e-8, drive=1.0, voxel_size=1.0,
                  max_sweeps=10_000_000, check_every=100, warm_start=0, stop_rule=0, fixed_pressure=0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def build(verbose: bool = False) -> str:
    """gcc -O2, OpenMP, no FMA contraction, no fast-math."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    vp = ctypes.c_void_p
    pp = ctypes.POINTER(OrcParams)
    lib.orc_face_solid.argtypes = [vp, i64, i64, i64, vp]
    lib.orc_face_solid.restype = None
    lib.orc_pack_bits.argtypes = [vp, i64, i64, i64, vp]
    lib.orc_pack_bits.restype = None
    lib.orc_case.argtypes = [i32, i32, i32, i32]
    lib.orc_case.restype = i32
    lib.orc_d2.argtypes = [i32, f64, f64, f64, f64, f64]
    lib.orc_d2.restype = f64
    lib.orc_sweep.argtypes = [pp, vp, i64, i64, i64, i32] + [vp] * 8
    lib.orc_sweep.restype = None
    lib.orc_sweep_points.argtypes = [pp, vp, i64, i64, i64, i32] + [vp] * 4 + [vp, i64, vp]
    lib.orc_sweep_points.restype = None
    lib.orc_state_sums.argtypes = [pp, vp, i64, i64, i64, i32] + [vp] * 5
    lib.orc_state_sums.restype = None
    lib.orc_slice_flux.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp]
    lib.orc_slice_flux.restype = None
    lib.orc_solve.argtypes = ([pp, vp, i64, i64, i64, i32] + [vp] * 4 +
                              [i64, vp, vp, vp, vp, vp, vp, vp])
    lib.orc_solve.restype = i32
    lib.orc_run_sweeps.argtypes = [pp, vp, i64, i64, i64, i32, i64] + [vp] * 4
    lib.orc_run_sweeps.restype = i32
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = i32
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_set_threads.restype = None
    _lib = lib
    return lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data


def _mask(mask) -> np.ndarray:
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    assert m.ndim == 3
    return m


def max_threads() -> int:
    return int(_load().orc_max_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (n >= 1)."""
    _load().orc_set_threads(int(n))


# ------------------------------------------------------------------ flags

def face_solid(mask) -> np.ndarray:
    """FS_k(c) = S(c) or S(c - e_k): a face is solid when it touches a solid voxel
    (no penetration at voxel faces, §4 "Boundary ...").  Returns (3, nz, ny, nx) uint8."""
    m = _mask(mask)
    nz, ny, nx = m.shape
    fs = np.empty((3, nz, ny, nx), dtype=np.uint8)
    _load().orc_face_solid(_p(m), nx, ny, nz, _p(fs))
    return fs


def pack_bits(fs: np.ndarray) -> np.ndarray:
    """Face flags packed 32 x-faces per uint32: (3, nz, ny, ceil(nx/32))."""
    fs = np.ascontiguousarray(fs, dtype=np.uint8)
    _, nz, ny, nx = fs.shape
    W = (nx + 31) // 32
    bits = np.empty((3, nz, ny, W), dtype=np.uint32)
    _load().orc_pack_bits(_p(fs), nx, ny, nz, _p(bits))
    return bits


def case(s_m2: int, s_m1: int, s_p1: int, s_p2: int) -> int:
    """Neighbourhood case 1..6 of App. B from the solid flags at offsets -2..+2."""
    return int(_load().orc_case(int(s_m2), int(s_m1), int(s_p1), int(s_p2)))


def d2(cse: int, vm2: float, vm1: float, v0: float, vp1: float, vp2: float) -> float:
    """App. B second-derivative stencil of case `cse` (1..8)."""
    return float(_load().orc_d2(int(cse), vm2, vm1, v0, vp1, vp2))


# ------------------------------------------------------------------ sweeps

@dataclass
class State:
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    p: np.ndarray

    @staticmethod
    def zeros(shape) -> "State":
        return State(*(np.zeros(shape, dtype=np.float64) for _ in range(4)))

    def copy(self) -> "State":
        return State(self.u.copy(), self.v.copy(), self.w.copy(), self.p.copy())

    def arrays(self):
        return (self.u, self.v, self.w, self.p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def sweep(mask, axis: int, st: State, prm: OrcParams | None = None, fs=None) -> State:
    """One pseudo-time sweep (Algorithm 1: velocity, then pressure)."""
    m = _mask(mask)
    nz, ny, nx = m.shape
    prm = prm or params()
    fs = face_solid(m) if fs is None else np.ascontiguousarray(fs, dtype=np.uint8)
    ins = [_f64(a) for a in st.arrays()]
    out = State.zeros(m.shape)
    _load().orc_sweep(ctypes.byref(prm), _p(fs), nx, ny, nz, axis, *[_p(a) for a in ins],
                      *[_p(a) for a in out.arrays()])
    return out


def sweep_points(mask, axis: int, st: State, cells, prm: OrcParams | None = None) -> np.ndarray:
    """New (u, v, w, p) after one sweep at the listed linear cell indices -> (n, 4)."""
    m = _mask(mask)
    nz, ny, nx = m.shape
    prm = prm or params()
    fs = face_solid(m)
    ins = [_f64(a) for a in st.arrays()]
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((cells.size, 4), dtype=np.float64)
    _load().orc_sweep_points(ctypes.byref(prm), _p(fs), nx, ny, nz, axis, *[_p(a) for a in ins],
                             _p(cells), cells.size, _p(out))
    return out


def state_sums(mask, axis: int, st: State, prm: OrcParams | None = None) -> np.ndarray:
    """[S_F, S_D, Q_x, Q_y, Q_z] of a state: squared momentum residual over fluid
    faces, squared (nu div v) over cells, and the summed face velocities."""
    m = _mask(mask)
    nz, ny, nx = m.shape
    prm = prm or params()
    fs = face_solid(m)
    ins = [_f64(a) for a in st.arrays()]
    out = np.empty(5, dtype=np.float64)
    _load().orc_state_sums(ctypes.byref(prm), _p(fs), nx, ny, nz, axis, *[_p(a) for a in ins],
                           _p(out))
    return out


def residual(mask, axis: int, st: State, prm: OrcParams | None = None) -> float:
    """r = sqrt(S_F + S_D) / (G sqrt(N_f)), N_f = fluid faces normal to the load axis."""
    prm = prm or params()
    s = state_sums(mask, axis, st, prm)
    nf = int((face_solid(mask)[axis] == 0).sum())
    return float(np.sqrt(s[0] + s[1]) / (prm.drive * np.sqrt(nf)))


def slice_flux(mask, st: State) -> np.ndarray:
    """qs[k, s] = sum of v_k over the k-faces at coordinate s along axis k."""
    m = _mask(mask)
    nz, ny, nx = m.shape
    L = max(nx, ny, nz)
    fs = face_solid(m)
    qs = np.zeros((3, L), dtype=np.float64)
    _load().orc_slice_flux(_p(fs), nx, ny, nz, *[_p(_f64(a)) for a in st.arrays()[:3]], _p(qs))
    return qs


def run_sweeps(mask, axis: int, count: int, prm: OrcParams | None = None,
               start: State | None = None) -> State:
    m = _mask(mask)
    nz, ny, nx = m.shape
    prm = prm or params()
    st = State.zeros(m.shape) if start is None else State(*(_f64(a).copy() for a in start.arrays()))
    if start is not None:
        prm = params(**{f: getattr(prm, f) for f, _ in OrcParams._fields_})
        prm.warm_start = 1
    _load().orc_run_sweeps(ctypes.byref(prm), _p(m), nx, ny, nz, axis, count,
                           *[_p(a) for a in st.arrays()])
    return st


@dataclass
class Result:
    status: str
    kcol: np.ndarray
    sweeps: int
    state: State
    hist_sweep: np.ndarray
    hist_r: np.ndarray
    hist_eps: np.ndarray
    hist_q: np.ndarray = field(default=None)


def solve(mask, axis: int, prm: OrcParams | None = None, start: State | None = None,
          hist_cap: int = 100000) -> Result:
    """Iterate to the stop rule (Algorithm 1 loop) and return k_{i,axis} (App. C)."""
    m = _mask(mask)
    nz, ny, nx = m.shape
    prm = prm or params()
    st = State.zeros(m.shape) if start is None else State(*(_f64(a).copy() for a in start.arrays()))
    hs = np.zeros(hist_cap, dtype=np.int64)
    hr = np.zeros(hist_cap)
    he = np.zeros(hist_cap)
    hq = np.zeros(3 * hist_cap)
    hn = ctypes.c_int64(0)
    k = np.zeros(3)
    sw = ctypes.c_int64(0)
    rc = _load().orc_solve(ctypes.byref(prm), _p(m), nx, ny, nz, axis,
                           *[_p(a) for a in st.arrays()], hist_cap, _p(hs), _p(hr), _p(he),
                           _p(hq), ctypes.addressof(hn), _p(k), ctypes.addressof(sw))
    n = hn.value
    return Result(STATUS.get(rc, str(rc)), k, sw.value, st, hs[:n], hr[:n], he[:n],
                  hq[:3 * n].reshape(n, 3))


def tensor(mask, prm: OrcParams | None = None):
    """Three load cases a) b) c) (eq. cases_pressure) -> k[i, j] (column j from load
    axis j) and the symmetrised tensor with averaged off-diagonals (App. C)."""
    cols, res = [], []
    for j in range(3):
        r = solve(mask, j, prm)
        cols.append(r.kcol)
        res.append(r)
    k = np.stack(cols, axis=1)
    return k, 0.5 * (k + k.T), res


def solve_walls(mask, axis: int, walls: int, prm: OrcParams | None = None) -> Result:
    """§4: no-slip, no-penetration outer walls at both ends of every axis i with
    bit i of `walls` set.  Written out as the same iteration on the mask with
    one solid layer appended along each wall axis (the wall half a voxel beyond
    the last layer; its periodic image half a voxel before the first), then the
    fields cut back to the original grid and the fluxes averaged over the
    original voxels.  A load axis with walls has no through-flow: NO_FLOW."""
    m = _mask(mask)
    if (walls >> axis) & 1:
        z = State.zeros(m.shape)
        return Result("NO_FLOW", np.zeros(3), 0, z, np.zeros(0, np.int64), np.zeros(0), np.zeros(0),
                      np.zeros((0, 3)))
    pad = [(0, (walls >> 2) & 1), (0, (walls >> 1) & 1), (0, walls & 1)]  # (z, y, x)
    mp = np.pad(m, pad, mode="constant", constant_values=1)
    r = solve(mp, axis, prm)
    nz, ny, nx = m.shape
    scale = mp.size / m.size
    st = State(*(a[:nz, :ny, :nx].copy() for a in r.state.arrays()))
    return Result(r.status, r.kcol * scale, r.sweeps, st, r.hist_sweep, r.hist_r, r.hist_eps,
                  r.hist_q * scale)
