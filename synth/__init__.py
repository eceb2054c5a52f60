"""Seeded synthetic masks (test and benchmark inputs only).

The generators live in ``synth.c`` (plain C, OpenMP) and are loaded with
ctypes.  They hold none of the flow method's arithmetic: the solver library
and the oracle both take their masks from here.  Every mask is a
``numpy.uint8`` array of shape ``(nz, ny, nx)`` (x fastest), 1 = solid.

The named workloads mirror the paper's application classes with synthetic
stand-ins (the paper's XRCT and microfluidic images are not available):

* ``spheres``   - overlapping-sphere packing (sphere-packing benchmarks, §6.3;
  large mirrored packings, §7.1);
* ``precipitation_series`` - extruded 2-D ellipse packing with stochastic
  clogging states (calcite precipitation in a microfluidic cell, §7.3);
* ``foam_series`` - Voronoi-strut open-cell foam under uniaxial compression
  (§7.2).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
SRC_PATH = os.path.join(_HERE, "synth.c")

_lib = None


def build(verbose: bool = False) -> str:
    """Compile libsynth.so with gcc (-O2, OpenMP)."""
    import subprocess

    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64, f64, u64 = ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    lib.synth_spheres.argtypes = [u8p, i64, i64, i64, f64, f64, f64, u64]
    lib.synth_spheres.restype = i64
    lib.synth_ellipses2d.argtypes = [u8p, i64, i64, f64, f64, f64, u64]
    lib.synth_ellipses2d.restype = i64
    lib.synth_clog2d.argtypes = [u8p, i64, i64, ctypes.c_int, u64]
    lib.synth_clog2d.restype = None
    lib.synth_extrude.argtypes = [u8p, i64, i64, i64, u8p]
    lib.synth_extrude.restype = None
    lib.synth_foam.argtypes = [u8p, i64, i64, i64, ctypes.c_int, f64, u64]
    lib.synth_foam.restype = None
    lib.synth_rescale_z.argtypes = [u8p, i64, i64, i64, i64, u8p]
    lib.synth_rescale_z.restype = None
    lib.synth_ellipsoid.argtypes = [u8p, i64, i64, i64, f64, f64, f64, f64]
    lib.synth_ellipsoid.restype = None
    lib.synth_splitmix64.argtypes = [u64, ctypes.POINTER(u64)]
    lib.synth_splitmix64.restype = u64
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.uint8 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def splitmix64(state: int) -> tuple[int, int]:
    """One SplitMix64 step: returns (output, next_state)."""
    nxt = ctypes.c_uint64(0)
    out = _load().synth_splitmix64(ctypes.c_uint64(state & (2**64 - 1)), ctypes.byref(nxt))
    return int(out), int(nxt.value)


def spheres(nx: int, ny: int, nz: int, rmin: float, rmax: float, porosity: float,
            seed: int) -> np.ndarray:
    """Overlapping spheres, radius ~ U[rmin, rmax], added until porosity <= target."""
    m = np.empty((nz, ny, nx), dtype=np.uint8)
    n = _load().synth_spheres(_ptr(m), nx, ny, nz, float(rmin), float(rmax), float(porosity),
                              seed)
    if n < 0:
        raise RuntimeError(f"synth_spheres failed ({n})")
    return m


def ellipses2d(nx: int, ny: int, amin: float, amax: float, porosity: float,
               seed: int) -> np.ndarray:
    img = np.empty((ny, nx), dtype=np.uint8)
    n = _load().synth_ellipses2d(_ptr(img), nx, ny, float(amin), float(amax), float(porosity),
                                 seed)
    if n < 0:
        raise RuntimeError(f"synth_ellipses2d failed ({n})")
    return img


def clog2d(img: np.ndarray, passes: int, seed: int) -> np.ndarray:
    out = np.ascontiguousarray(img, dtype=np.uint8).copy()
    ny, nx = out.shape
    _load().synth_clog2d(_ptr(out), nx, ny, int(passes), seed)
    return out


def extrude(img: np.ndarray, depth: int) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    ny, nx = img.shape
    out = np.empty((depth + 2, ny, nx), dtype=np.uint8)
    _load().synth_extrude(_ptr(img), nx, ny, depth, _ptr(out))
    return out


def foam(nx: int, ny: int, nz: int, nseeds: int, radius: float, seed: int) -> np.ndarray:
    m = np.empty((nz, ny, nx), dtype=np.uint8)
    _load().synth_foam(_ptr(m), nx, ny, nz, int(nseeds), float(radius), seed)
    return m


def rescale_z(mask: np.ndarray, nz_dst: int) -> np.ndarray:
    mask = np.ascontiguousarray(mask, dtype=np.uint8)
    nz, ny, nx = mask.shape
    out = np.empty((nz_dst, ny, nx), dtype=np.uint8)
    _load().synth_rescale_z(_ptr(mask), nx, ny, nz, nz_dst, _ptr(out))
    return out


# ------------------------------------------------------------ named workloads

def ellipsoid(nx: int, ny: int, nz: int, a: float, b: float, c: float, alpha_deg: float) -> np.ndarray:
    """One ellipsoid (semi-axes a, b, c along e1, e2, e3) centred in the box, turned about e1."""
    m = np.empty((nz, ny, nx), dtype=np.uint8)
    _load().synth_ellipsoid(_ptr(m), nx, ny, nz, float(a), float(b), float(c), np.radians(alpha_deg))
    return m


def ellipsoid_100(alpha_deg: float) -> np.ndarray:
    """The principal-direction benchmark: 100^3 box, semi-axes 35, 10, 35, turned by alpha about e1."""
    return ellipsoid(100, 100, 100, 35.0, 10.0, 35.0, alpha_deg)


def single_spheres_32() -> np.ndarray:
    """32^3 packing, radius 4, porosity 0.40, seed 1 (plain FP64 single solve)."""
    return spheres(32, 32, 32, 4.0, 4.0, 0.40, 1)


def spheres_256() -> np.ndarray:
    """256^3 packing, radius U[6,10], porosity 0.35, seed 2 (full tensor, throughput)."""
    return spheres(256, 256, 256, 6.0, 10.0, 0.35, 2)


def spheres_1536() -> np.ndarray:
    """1536^3 packing, radius U[5,12], porosity 0.20, seed 5 (large single domain)."""
    return spheres(1536, 1536, 1536, 5.0, 12.0, 0.20, 5)


def precipitation_series(nx: int = 1024, ny: int = 512, depth: int = 16, nstates: int = 16,
                         seed: int = 3) -> list[np.ndarray]:
    """Extruded ellipse packing (porosity 0.55) with clogging states 0..nstates-1.

    State s applies s stochastic dilation passes to the 2-D image; each state
    is extruded to depth+2 planes with solid walls at the bottom and top.
    """
    base = ellipses2d(nx, ny, 8.0, 20.0, 0.55, seed)
    out = []
    img = base.copy()
    for s in range(nstates):
        if s > 0:
            img = clog2d(img, 1, seed * 1000003 + s)
        out.append(extrude(img, depth))
    return out


def foam_strain_dims(n: int = 512, nstates: int = 8) -> list[int]:
    return [int(round(n * (1.0 - s / 28.0))) for s in range(nstates)]


def foam_series(n: int = 512, nseeds: int = 200, radius: float = 3.0, nstates: int = 8,
                seed: int = 4) -> list[np.ndarray]:
    """Voronoi-strut foam compressed along z: nz_s = round(n (1 - s/28))."""
    base = foam(n, n, n, nseeds, radius, seed)
    return [base if nz == n else rescale_z(base, nz) for nz in foam_strain_dims(n, nstates)]


def test_grid(seed: int) -> np.ndarray:
    """Small parity grids for seeds 100..109: cubic, non-cubic and extruded."""
    kind = seed % 3
    if kind == 0:
        return spheres(24, 24, 24, 3.0, 3.0, 0.45, seed)
    if kind == 1:
        return spheres(40, 32, 28, 2.5, 4.0, 0.45, seed)
    img = ellipses2d(16, 16, 2.0, 3.5, 0.55, seed)
    return np.ascontiguousarray(img[None, :, :])
