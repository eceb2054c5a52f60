"""porestokes: MI355X-native pseudo-unsteady Stokes permeability solver.

Thin Python binding of ``libporestokes.so`` (C ABI in ``include/porestokes.h``).
It only marshals arguments: masks and fields are torch CUDA tensors whose
device pointers and the current HIP stream are handed to the library; every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback -- importing the binding without the built library raises.

Method: Krach, Ruf, Steeb, "POREMAPS" (arXiv 2407.19868): §3-§4 and App. A-C.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libporestokes.so")

PM_OK, PM_ERR_ARG, PM_ERR_OOM, PM_ERR_DEVICE, PM_NOT_CONVERGED, PM_DIVERGED, PM_ERR_NO_FLOW = range(7)
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 3: "ERR_DEVICE", 4: "NOT_CONVERGED",
                5: "DIVERGED", 6: "NO_FLOW"}
FP64, FP32, FP32_DC = 0, 1, 2
KERNEL_AUTO, KERNEL_FUSED, KERNEL_SIMPLE = 0, 1, 2

# Every symbol declared in include/porestokes.h.
EXPORTS = ("pm_params_default", "pm_status_string", "pm_create", "pm_destroy", "pm_last_error",
           "pm_mem_used", "pm_preprocess", "pm_face_codes", "pm_iterate", "pm_residual", "pm_solve",
           "pm_tensor", "pm_solve_batch", "pm_last_stats", "pm_autotune", "pm_principal_axes",
           "pm_plane_angle", "pm_pores", "pm_mirror", "pm_trim", "pm_iterate_static")
ISOTROPIC, TRANSVERSE, ORTHOTROPIC = 0, 1, 2
CLASS_NAMES = {ISOTROPIC: "isotropic", TRANSVERSE: "transverse", ORTHOTROPIC: "orthotropic"}


class PmParams(ctypes.Structure):
    _fields_ = [
        ("re", ctypes.c_double),
        ("c2", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("drive", ctypes.c_double),
        ("max_sweeps", ctypes.c_int64),
        ("check_every", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("stop_rule", ctypes.c_int32),
        ("warm_start", ctypes.c_int32),
        ("kernel", ctypes.c_int32),
        ("tile_x", ctypes.c_int32),
        ("tile_y", ctypes.c_int32),
        ("zchunk", ctypes.c_int32),
        ("graphs", ctypes.c_int32),
        ("autotune", ctypes.c_int32),
        ("progress", ctypes.c_int32),
        ("pore_cleanup", ctypes.c_int32),
        ("outer_walls", ctypes.c_int32),
        ("dc_form", ctypes.c_int32),
        ("tblock", ctypes.c_int32),
        ("tile2_x", ctypes.c_int32),
        ("tile2_y", ctypes.c_int32),
        ("zchunk2", ctypes.c_int32),
        ("fixed_pressure", ctypes.c_int32),
        ("persistent", ctypes.c_int32),
    ]


class PmHistory(ctypes.Structure):
    _fields_ = [
        ("cap", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("sweep", ctypes.c_void_p),
        ("resid", ctypes.c_void_p),
        ("eps_q", ctypes.c_void_p),
        ("q", ctypes.c_void_p),
    ]


class PmInstance(ctypes.Structure):
    _fields_ = [
        ("mask", ctypes.c_void_p),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nz", ctypes.c_int64),
        ("voxel_size", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("axis", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("u", ctypes.c_void_p),
        ("v", ctypes.c_void_p),
        ("w", ctypes.c_void_p),
        ("p", ctypes.c_void_p),
        ("hist", ctypes.c_void_p),
        ("k_col", ctypes.c_double * 3),
        ("sweeps", ctypes.c_int64),
        ("status", ctypes.c_int32),
        ("pad2", ctypes.c_int32),
    ]


class PmStats(ctypes.Structure):
    _fields_ = [
        ("sweep_launches", ctypes.c_int64),
        ("voxel_updates", ctypes.c_int64),
        ("sweep_ms", ctypes.c_double),
        ("total_ms", ctypes.c_double),
        ("tile_x", ctypes.c_int32),
        ("tile_y", ctypes.c_int32),
        ("zchunk", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("peak_bytes", ctypes.c_int64),
        ("tblock", ctypes.c_int32),
        ("tensor_cases_at_once", ctypes.c_int32),
        ("dc_promoted_for_memory", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("t2_launches", ctypes.c_int64),
        ("t2_voxels", ctypes.c_int64),
        ("t2_ms", ctypes.c_double),
        ("pers_launches", ctypes.c_int64),
        ("pers_sweeps", ctypes.c_int64),
    ]


class PmPoreInfo(ctypes.Structure):
    _fields_ = [
        ("n_pore", ctypes.c_int64),
        ("n_components", ctypes.c_int64),
        ("percolates", ctypes.c_int32 * 3),
        ("reserved", ctypes.c_int32),
        ("n_flowing", ctypes.c_int64 * 3),
        ("n_flowing_components", ctypes.c_int64 * 3),
    ]


class PmPrincipal(ctypes.Structure):
    _fields_ = [
        ("k_sym", ctypes.c_double * 9),
        ("lam", ctypes.c_double * 3),
        ("R", ctypes.c_double * 9),
        ("cls", ctypes.c_int32),
        ("distinct", ctypes.c_int32),
        ("ratio", ctypes.c_double),
    ]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libporestokes.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2407_19868_amd._build.build() "
                           "(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    pp = ctypes.POINTER(PmParams)
    lib.pm_params_default.argtypes = [pp]
    lib.pm_params_default.restype = None
    lib.pm_status_string.argtypes = [i32]
    lib.pm_status_string.restype = ctypes.c_char_p
    lib.pm_create.argtypes = [i32, ctypes.c_size_t, ctypes.POINTER(vp)]
    lib.pm_create.restype = i32
    lib.pm_destroy.argtypes = [vp]
    lib.pm_destroy.restype = None
    lib.pm_last_error.argtypes = [vp]
    lib.pm_last_error.restype = ctypes.c_char_p
    lib.pm_mem_used.argtypes = [vp]
    lib.pm_mem_used.restype = ctypes.c_size_t
    lib.pm_trim.argtypes = [vp]
    lib.pm_trim.restype = i32
    lib.pm_preprocess.argtypes = [vp, vp, vp, i64, i64, i64, vp]
    lib.pm_preprocess.restype = i32
    lib.pm_face_codes.argtypes = [vp, vp, vp, i64, i64, i64, vp]
    lib.pm_face_codes.restype = i32
    lib.pm_iterate.argtypes = [vp, vp, vp, i64, i64, i64, i32, pp, vp, vp, vp, vp, i64]
    lib.pm_iterate.restype = i32
    lib.pm_iterate_static.argtypes = [vp, vp, vp, i64, i64, i64, i32, pp, vp, vp, vp, vp, i64]
    lib.pm_iterate_static.restype = i32
    lib.pm_residual.argtypes = [vp, vp, vp, i64, i64, i64, i32, pp, vp, vp, vp, vp, vp]
    lib.pm_residual.restype = i32
    lib.pm_solve.argtypes = [vp, vp, vp, i64, i64, i64, ctypes.c_double, ctypes.c_double, i32, pp,
                             vp, vp, vp, vp, ctypes.POINTER(PmHistory), vp, ctypes.POINTER(i64)]
    lib.pm_solve.restype = i32
    lib.pm_tensor.argtypes = [vp, vp, vp, i64, i64, i64, ctypes.c_double, ctypes.c_double, pp, vp, vp,
                              ctypes.POINTER(PmHistory), vp]
    lib.pm_tensor.restype = i32
    lib.pm_solve_batch.argtypes = [vp, vp, ctypes.POINTER(PmInstance), ctypes.c_int32, pp]
    lib.pm_solve_batch.restype = i32
    lib.pm_last_stats.argtypes = [vp, ctypes.POINTER(PmStats)]
    lib.pm_last_stats.restype = i32
    lib.pm_autotune.argtypes = [vp, vp, vp, i64, i64, i64, i32, vp]
    lib.pm_autotune.restype = i32
    lib.pm_mirror.argtypes = [vp, vp, vp, i64, i64, i64, i32, vp]
    lib.pm_mirror.restype = i32
    lib.pm_pores.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp, ctypes.POINTER(PmPoreInfo)]
    lib.pm_pores.restype = i32
    d9 = ctypes.c_double * 9
    lib.pm_principal_axes.argtypes = [ctypes.POINTER(d9), ctypes.c_double, ctypes.POINTER(PmPrincipal)]
    lib.pm_principal_axes.restype = i32
    lib.pm_plane_angle.argtypes = [ctypes.POINTER(d9), i32, i32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double * 2)]
    lib.pm_plane_angle.restype = i32
    _lib = lib
    return lib


def params(**kw) -> PmParams:
    """pm_params with the library defaults (§4: Re 0.01, c*^2 1.5e6), overridden by kw."""
    p = PmParams()
    load_library().pm_params_default(ctypes.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


class PorestokesError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev_tensor(t: torch.Tensor, dtype=None, name="tensor") -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _mask3(mask: torch.Tensor) -> tuple[torch.Tensor, int, int, int]:
    m = _dev_tensor(mask, torch.uint8, "mask")
    if m.dim() != 3:
        raise ValueError("mask must be (nz, ny, nx)")
    nz, ny, nx = m.shape
    return m, nx, ny, nz


def _hist(cap: int):
    sw = np.zeros(cap, dtype=np.int64)
    r = np.zeros(cap)
    e = np.zeros(cap)
    q = np.zeros(3 * cap)
    h = PmHistory(cap, 0, sw.ctypes.data, r.ctypes.data, e.ctypes.data, q.ctypes.data)
    return h, (sw, r, e, q)


@dataclass
class SolveResult:
    status: str
    kcol: np.ndarray
    sweeps: int
    fields: tuple
    hist_sweep: np.ndarray
    hist_r: np.ndarray
    hist_eps: np.ndarray
    hist_q: np.ndarray


@dataclass
class TensorResult:
    status: str
    k: np.ndarray
    k_sym: np.ndarray
    sweeps: np.ndarray
    hists: list


def field_set(shape, dtype=torch.float64, device="cuda") -> tuple:
    """Zeroed u, v, w, p of one grid as four views of one block, N elements apart.

    The sweep reads the four fields at the same offsets: with their starts
    N elements apart it ran fastest (256^3, FP64: 228 us per sweep; the same
    fields shifted against each other by 32 KiB or 1-8 MiB took 235-245 us).
    Separately allocated tensors land wherever the allocator puts them.
    """
    block = torch.zeros((4, *shape), dtype=dtype, device=device)
    return tuple(block.unbind(0))


class Context:
    """One library context on a HIP device (default: torch's current device)."""

    def __init__(self, device: int | None = None, mem_cap: int = 0):
        self._lib = load_library()
        if device is None:
            device = torch.cuda.current_device()
        self.device = device
        h = ctypes.c_void_p()
        st = self._lib.pm_create(device, mem_cap, ctypes.byref(h))
        if st != PM_OK:
            raise PorestokesError(st, "pm_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def last_error(self) -> str:
        return self._lib.pm_last_error(self._h).decode()

    def mem_used(self) -> int:
        """Device bytes the context holds, blocks kept for reuse included."""
        return int(self._lib.pm_mem_used(self._h))

    def trim(self) -> None:
        """Return the device blocks kept for reuse between calls."""
        self._check(self._lib.pm_trim(self._h))

    def autotune(self, mask, precision: int = FP64) -> tuple:
        """Time the fused-kernel decompositions on this mask; returns (tile_x, tile_y, zchunk,
        tblock, tile2_x, tile2_y, zchunk2)."""
        m, nx, ny, nz = _mask3(mask)
        best = np.zeros(7, dtype=np.int32)
        self._check(self._lib.pm_autotune(self._h, _stream(), m.data_ptr(), nx, ny, nz, precision,
                                          best.ctypes.data))
        return tuple(int(v) for v in best)

    def last_stats(self) -> dict:
        """Sweep-kernel timing of the last call (HIP events on the call's stream)."""
        st = PmStats()
        self._check(self._lib.pm_last_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in PmStats._fields_}

    def _check(self, st: int, allow=(PM_OK,)):
        if st not in allow:
            raise PorestokesError(st, self.last_error())
        return st

    # ---------------------------------------------------------------- calls
    def preprocess(self, mask: torch.Tensor) -> torch.Tensor:
        """Face-solid bit planes (3, nz, ny, ceil(nx/32)) as int32 (bit pattern of uint32)."""
        m, nx, ny, nz = _mask3(mask)
        bits = torch.empty((3, nz, ny, (nx + 31) // 32), dtype=torch.int32, device=m.device)
        self._check(self._lib.pm_preprocess(self._h, _stream(), m.data_ptr(), nx, ny, nz,
                                            bits.data_ptr()))
        return bits

    def face_codes(self, mask: torch.Tensor) -> torch.Tensor:
        m, nx, ny, nz = _mask3(mask)
        codes = torch.empty((nz, ny, nx), dtype=torch.int32, device=m.device)
        self._check(self._lib.pm_face_codes(self._h, _stream(), m.data_ptr(), nx, ny, nz,
                                            codes.data_ptr()))
        return codes

    def iterate(self, mask, axis: int, fields, count: int, prm: PmParams | None = None):
        """Run `count` sweeps on fields (u, v, w, p) in place (float64 or float32)."""
        m, nx, ny, nz = _mask3(mask)
        prm = prm or params()
        f = [_dev_tensor(t, None, "field") for t in fields]
        self._check(self._lib.pm_iterate(self._h, _stream(), m.data_ptr(), nx, ny, nz, axis,
                                         ctypes.byref(prm), *[t.data_ptr() for t in f], count))
        return fields

    def iterate_static(self, mask, axis: int, fields, count: int, prm: PmParams | None = None):
        """pm_iterate_static: as iterate, on the library's static device scratch (no allocation)."""
        m, nx, ny, nz = _mask3(mask)
        prm = prm or params()
        f = [_dev_tensor(t, None, "field") for t in fields]
        self._check(self._lib.pm_iterate_static(self._h, _stream(), m.data_ptr(), nx, ny, nz, axis,
                                                ctypes.byref(prm), *[t.data_ptr() for t in f], count))
        return fields

    def residual(self, mask, axis: int, fields, prm: PmParams | None = None) -> np.ndarray:
        """[S_F, S_D, Q_x, Q_y, Q_z] of a state, FP64 sums on the GPU."""
        m, nx, ny, nz = _mask3(mask)
        prm = prm or params()
        out = np.zeros(5)
        f = [_dev_tensor(t, None, "field") for t in fields]
        self._check(self._lib.pm_residual(self._h, _stream(), m.data_ptr(), nx, ny, nz, axis,
                                          ctypes.byref(prm), *[t.data_ptr() for t in f],
                                          out.ctypes.data))
        return out

    def solve(self, mask, axis: int, prm: PmParams | None = None, fields=None,
              voxel_size: float = 1.0, mu: float = 1.0, hist_cap: int = 100000,
              raise_on=(PM_ERR_ARG, PM_ERR_OOM, PM_ERR_DEVICE)) -> SolveResult:
        m, nx, ny, nz = _mask3(mask)
        prm = prm or params()
        dtype = torch.float32 if prm.precision == FP32 else torch.float64
        if fields is None:
            fields = field_set((nz, ny, nx), dtype, m.device)
        f = [_dev_tensor(t, dtype, "field") for t in fields]
        h, arrs = _hist(hist_cap)
        k = np.zeros(3)
        sw = ctypes.c_int64(0)
        st = self._lib.pm_solve(self._h, _stream(), m.data_ptr(), nx, ny, nz, voxel_size, mu, axis,
                                ctypes.byref(prm), *[t.data_ptr() for t in f], ctypes.byref(h),
                                k.ctypes.data, ctypes.byref(sw))
        if st in raise_on:
            raise PorestokesError(st, self.last_error())
        n = h.n
        return SolveResult(STATUS_NAMES[st], k, sw.value, tuple(fields), arrs[0][:n].copy(),
                           arrs[1][:n].copy(), arrs[2][:n].copy(), arrs[3][:3 * n].reshape(n, 3).copy())

    def tensor(self, mask, prm: PmParams | None = None, voxel_size: float = 1.0, mu: float = 1.0,
               hist_cap: int = 100000) -> TensorResult:
        m, nx, ny, nz = _mask3(mask)
        prm = prm or params()
        hs = (PmHistory * 3)()
        keep = []
        for j in range(3):
            h, arrs = _hist(hist_cap)
            hs[j] = h
            keep.append(arrs)
        k = np.zeros(9)
        ks = np.zeros(9)
        sw = np.zeros(3, dtype=np.int64)
        st = self._lib.pm_tensor(self._h, _stream(), m.data_ptr(), nx, ny, nz, voxel_size, mu,
                                 ctypes.byref(prm), k.ctypes.data, ks.ctypes.data, hs, sw.ctypes.data)
        if st in (PM_ERR_ARG, PM_ERR_OOM, PM_ERR_DEVICE):
            raise PorestokesError(st, self.last_error())
        hists = []
        for j in range(3):
            n = hs[j].n
            sw_, r_, e_, q_ = keep[j]
            hists.append({"sweep": sw_[:n].copy(), "r": r_[:n].copy(), "eps": e_[:n].copy(),
                          "q": q_[:3 * n].reshape(n, 3).copy()})
        return TensorResult(STATUS_NAMES[st], k.reshape(3, 3), ks.reshape(3, 3), sw, hists)

    def mirror(self, mask, axes: int) -> torch.Tensor:
        """The sample followed by its mirror image along every axis in the bit mask (pm_mirror)."""
        m, nx, ny, nz = _mask3(mask)
        shape = (nz * (2 if axes & 4 else 1), ny * (2 if axes & 2 else 1), nx * (2 if axes & 1 else 1))
        out = torch.empty(shape, dtype=torch.uint8, device=m.device)
        self._check(self._lib.pm_mirror(self._h, _stream(), m.data_ptr(), nx, ny, nz, int(axes), out.data_ptr()))
        return out

    def pores(self, mask, labels: bool = True, flow: bool = True) -> dict:
        """Pore components and percolation (pm_pores): counts, per-axis flags, and
        optionally the label (int64) and flow-bit (uint8) volumes as device tensors."""
        m, nx, ny, nz = _mask3(mask)
        lab = torch.empty(m.shape, dtype=torch.int64, device=m.device) if labels else None
        fl = torch.empty(m.shape, dtype=torch.uint8, device=m.device) if flow else None
        info = PmPoreInfo()
        st = self._lib.pm_pores(self._h, _stream(), m.data_ptr(), nx, ny, nz,
                                lab.data_ptr() if lab is not None else None,
                                fl.data_ptr() if fl is not None else None, ctypes.byref(info))
        self._check(st)
        return {"n_pore": info.n_pore, "n_components": info.n_components,
                "percolates": tuple(bool(x) for x in info.percolates),
                "n_flowing": tuple(info.n_flowing), "n_flowing_components": tuple(info.n_flowing_components),
                "labels": lab, "flow": fl}

    def solve_batch(self, problems, prm: PmParams | None = None, hist_cap: int = 100000,
                    fields=None):
        """problems: list of (mask, axis[, voxel_size]).  Returns (status, list of per-instance dicts)."""
        prm = prm or params()
        n = len(problems)
        arr = (PmInstance * n)()
        keep = []
        hs = (PmHistory * n)()
        for i, pr in enumerate(problems):
            mask, axis = pr[0], pr[1]
            dx = pr[2] if len(pr) > 2 else 1.0
            m, nx, ny, nz = _mask3(mask)
            h, arrs = _hist(hist_cap)
            hs[i] = h
            keep.append((m, arrs))
            inst = arr[i]
            inst.mask = m.data_ptr()
            inst.nx, inst.ny, inst.nz = nx, ny, nz
            inst.voxel_size = dx
            inst.mu = 1.0
            inst.axis = axis
            if fields is not None and fields[i] is not None:
                inst.u, inst.v, inst.w, inst.p = [t.data_ptr() for t in fields[i]]
            inst.hist = ctypes.addressof(hs[i])
        st = self._lib.pm_solve_batch(self._h, _stream(), arr, n, ctypes.byref(prm))
        if st in (PM_ERR_ARG, PM_ERR_OOM, PM_ERR_DEVICE):
            raise PorestokesError(st, self.last_error())
        out = []
        for i in range(n):
            hn = hs[i].n
            sw_, r_, e_, q_ = keep[i][1]
            out.append({"status": STATUS_NAMES[arr[i].status], "kcol": np.array(arr[i].k_col[:]),
                        "sweeps": int(arr[i].sweeps), "sweep": sw_[:hn].copy(), "r": r_[:hn].copy(),
                        "eps": e_[:hn].copy()})
        return STATUS_NAMES[st], out


@dataclass
class Principal:
    k_sym: np.ndarray     # (k + k^T) / 2
    lam: np.ndarray       # k_I <= k_II <= k_III
    R: np.ndarray         # column i: principal axis of lam[i]
    cls: str              # "isotropic" | "transverse" | "orthotropic"
    distinct: int         # transverse: index of the differing value, else -1
    ratio: float          # k_III / k_I


def _k9(k) -> "ctypes.Array":
    a = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(3, 3))
    return (ctypes.c_double * 9)(*a.ravel().tolist())


def principal_axes(k, rel_tol: float = 0.05) -> Principal:
    """Principal permeabilities, axes and material class of a 3x3 tensor (pm_principal_axes)."""
    out = PmPrincipal()
    st = load_library().pm_principal_axes(ctypes.byref(_k9(k)), float(rel_tol), ctypes.byref(out))
    if st != PM_OK:
        raise PorestokesError(st, "pm_principal_axes: bad tensor or tolerance")
    return Principal(np.array(out.k_sym[:]).reshape(3, 3), np.array(out.lam[:]), np.array(out.R[:]).reshape(3, 3),
                     CLASS_NAMES[out.cls], int(out.distinct), float(out.ratio))


def plane_angle(k, a: int, b: int) -> tuple[float, np.ndarray]:
    """Principal angle (radians) and eigenvalues of the (a, b) block of a tensor (pm_plane_angle)."""
    phi = ctypes.c_double()
    lam = (ctypes.c_double * 2)()
    st = load_library().pm_plane_angle(ctypes.byref(_k9(k)), int(a), int(b), ctypes.byref(phi), ctypes.byref(lam))
    if st != PM_OK:
        raise PorestokesError(st, "pm_plane_angle: bad tensor or axes")
    return float(phi.value), np.array(lam[:])


def to_device(mask: np.ndarray, device: int | str = "cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(device)
