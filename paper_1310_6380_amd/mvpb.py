"""Thin ctypes binding of the mvpb C-ABI (argument marshalling only).

Every step of the band-structure path runs in the HIP library
``libmvpb.so`` built next to this file; this module only converts Python
arguments to pointers and status codes to exceptions.  It fails loudly when
the library is missing.

Device buffers for device-pointer outputs are allocated through the same HIP
runtime the library is linked against (``DeviceBuffer``).  The torch wheel of
this image carries its own, older HIP/HSA runtime; a second HSA runtime cannot
open the GPU in a process where the first one already has, so torch tensors
are not used as buffers here.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmvpb.so")

OK = 0
E_INVALID = -1
E_NOT_PD = -2
E_NOMEM = -3
E_DEVICE = -4
E_UNSUPPORTED = -5
E_ACCURACY = -6

PROP_ISO_E_NU_RHO = 0
PROP_VOIGT_D_RHO = 1

PREC_FP64 = 0
PREC_SF_FP32 = 1
PREC_SF_BF16 = 2
PREC_SF_BF16X3 = 3
PREC_EIG_FP32_RR64 = 4
PREC_SF_PLAIN64 = 8
PREC_GENERAL = 16

F_DEVICE_PTRS = 1
F_ASYNC = 2

EXPORTS = [
    "mvpb_last_error", "mvpb_version", "mvpb_ctx_create", "mvpb_ctx_destroy",
    "mvpb_cell_create_pixels", "mvpb_cell_destroy", "mvpb_plan_create", "mvpb_plan_dofs",
    "mvpb_plan_destroy", "mvpb_solve", "mvpb_solve_batch", "mvpb_structure_factors",
    "mvpb_kpath_square", "mvpb_ctx_profile", "mvpb_ctx_profile_read", "mvpb_plan_create_batch",
    "mvpb_sur_create", "mvpb_sur_destroy", "mvpb_sur_n_params", "mvpb_sur_get_params", "mvpb_sur_set_params",
    "mvpb_sur_infer", "mvpb_sur_gradients", "mvpb_sur_train_step", "mvpb_copy_device",
    "mvpb_ctx_profile_mask", "mvpb_cell_create_polygons", "mvpb_stress_modes", "mvpb_kpath",
    "mvpb_sur_save", "mvpb_sur_load", "mvpb_structure_factors_noalloc", "mvpb_ctx_set_accuracy",
    "mvpb_ctx_last_accuracy", "mvpb_cell_create_voxels", "mvpb_plan_create3", "mvpb_structure_factors_general",
    "mvpb_band_sensitivities", "mvpb_autotune", "mvpb_ctx_load_tuning", "mvpb_ctx_set_wait_limit",
    "mvpb_ctx_set_launch_shape", "mvpb_ctx_get_launch_shape", "mvpb_solve_cells",
]
N_KERNELS = 15


class MvpbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mvpb error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libmvpb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with paper_1310_6380_amd/build.py")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.POINTER(ctypes.c_double)
    lib.mvpb_last_error.restype = ctypes.c_char_p
    lib.mvpb_version.restype = ctypes.c_char_p
    lib.mvpb_ctx_create.argtypes = [I, P, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.mvpb_ctx_destroy.argtypes = [P]
    lib.mvpb_cell_create_pixels.argtypes = [P, D, I, I, ctypes.POINTER(ctypes.c_int32), I, I, D, ctypes.POINTER(P)]
    lib.mvpb_cell_create_polygons.argtypes = [P, D, I, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                              D, I, I, D, ctypes.POINTER(P)]
    lib.mvpb_cell_destroy.argtypes = [P]
    lib.mvpb_cell_create_voxels.argtypes = [P, D, I, I, I, ctypes.POINTER(ctypes.c_int32), I, I, D,
                                            ctypes.POINTER(P)]
    lib.mvpb_plan_create3.argtypes = [P, I, I, I, I, ctypes.POINTER(P)]
    lib.mvpb_structure_factors_general.argtypes = [P, I, I, I, D]
    lib.mvpb_band_sensitivities.argtypes = [P, I, D, I, P, P, P, ctypes.c_uint]
    lib.mvpb_autotune.argtypes = [P, I, D, I, ctypes.c_char_p, D]
    lib.mvpb_ctx_load_tuning.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(I)]
    lib.mvpb_ctx_set_wait_limit.argtypes = [P, ctypes.c_longlong]
    lib.mvpb_ctx_set_launch_shape.argtypes = [P, I, I, I, I]
    lib.mvpb_ctx_get_launch_shape.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.mvpb_stress_modes.argtypes = [P, I, D, I, D, D, ctypes.c_uint]
    lib.mvpb_plan_create.argtypes = [P, I, I, I, ctypes.POINTER(P)]
    lib.mvpb_plan_dofs.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.mvpb_plan_destroy.argtypes = [P]
    lib.mvpb_solve.argtypes = [P, I, D, I, P, P, ctypes.c_uint]
    lib.mvpb_solve_batch.argtypes = [P, I, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(D), I,
                                     ctypes.POINTER(P), ctypes.c_uint]
    lib.mvpb_solve_cells.argtypes = [P, I, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(I), I, ctypes.POINTER(I),
                                     ctypes.POINTER(D), I, ctypes.POINTER(P), ctypes.c_uint]
    lib.mvpb_structure_factors.argtypes = [P, I, I, I, D]
    lib.mvpb_structure_factors_noalloc.argtypes = [P, I, I, I, P, ctypes.c_uint]
    lib.mvpb_kpath_square.argtypes = [I, D]
    lib.mvpb_kpath.argtypes = [D, ctypes.c_char_p, I, D]
    lib.mvpb_plan_create_batch.argtypes = [P, I, ctypes.POINTER(P), ctypes.POINTER(I), ctypes.POINTER(I), I,
                                           ctypes.POINTER(P)]
    F = ctypes.POINTER(ctypes.c_float)
    lib.mvpb_sur_create.argtypes = [P, I, I, ctypes.c_uint64, ctypes.POINTER(P)]
    lib.mvpb_sur_destroy.argtypes = [P]
    lib.mvpb_sur_n_params.argtypes = [P, ctypes.POINTER(I)]
    lib.mvpb_sur_get_params.argtypes = [P, F]
    lib.mvpb_sur_set_params.argtypes = [P, F]
    lib.mvpb_sur_infer.argtypes = [P, I, P, P, ctypes.c_uint]
    lib.mvpb_sur_gradients.argtypes = [P, I, P, P, F, P, ctypes.c_uint]
    lib.mvpb_sur_train_step.argtypes = [P, I, P, P, ctypes.c_float, F, ctypes.c_uint]
    lib.mvpb_sur_save.argtypes = [P, ctypes.c_char_p]
    lib.mvpb_sur_load.argtypes = [P, ctypes.c_char_p, I, ctypes.POINTER(P)]
    lib.mvpb_copy_device.argtypes = [P, P, P, ctypes.c_size_t]
    lib.mvpb_ctx_profile.argtypes = [P, I]
    lib.mvpb_ctx_set_accuracy.argtypes = [P, ctypes.c_double]
    lib.mvpb_ctx_last_accuracy.argtypes = [P, D]
    lib.mvpb_ctx_profile_mask.argtypes = [P, ctypes.c_ulonglong]
    lib.mvpb_ctx_profile_read.argtypes = [P, I, D, ctypes.POINTER(ctypes.c_longlong),
                                          ctypes.POINTER(ctypes.c_char_p)]
    for name in EXPORTS:
        fn = getattr(lib, name)
        if name not in ("mvpb_last_error", "mvpb_version"):
            fn.restype = ctypes.c_int
    _lib = lib
    return lib


_hip = None


def _hiprt():
    """The HIP runtime libmvpb.so is linked against (already loaded with it)."""
    global _hip
    if _hip is None:
        load()
        _hip = ctypes.CDLL("libamdhip64.so.7")
        _hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        _hip.hipFree.argtypes = [ctypes.c_void_p]
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipDeviceSynchronize.argtypes = []
        for f in (_hip.hipMalloc, _hip.hipFree, _hip.hipMemcpy, _hip.hipDeviceSynchronize):
            f.restype = ctypes.c_int
    return _hip


class DeviceBuffer:
    """Raw device allocation (hipMalloc) of the library's HIP runtime."""

    def __init__(self, nbytes: int):
        self.ptr = ctypes.c_void_p()
        self.nbytes = int(nbytes)
        rc = _hiprt().hipMalloc(ctypes.byref(self.ptr), max(self.nbytes, 1))
        if rc != 0:
            raise MvpbError(E_DEVICE, f"hipMalloc({nbytes}) failed with {rc}")

    @property
    def value(self) -> int:
        return int(self.ptr.value)

    def upload(self, arr):
        a = np.ascontiguousarray(arr)
        assert a.nbytes <= self.nbytes
        rc = _hiprt().hipMemcpy(self.ptr, a.ctypes.data, a.nbytes, 1)  # host to device
        if rc != 0:
            raise MvpbError(E_DEVICE, f"hipMemcpy failed with {rc}")
        return self

    def to_numpy(self, dtype, shape) -> np.ndarray:
        out = np.empty(shape, dtype=dtype)
        assert out.nbytes <= self.nbytes
        rc = _hiprt().hipMemcpy(out.ctypes.data, self.ptr, out.nbytes, 2)  # device to host
        if rc != 0:
            raise MvpbError(E_DEVICE, f"hipMemcpy failed with {rc}")
        return out

    def free(self):
        if self.ptr:
            _hiprt().hipFree(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def device_synchronize():
    rc = _hiprt().hipDeviceSynchronize()
    if rc != 0:
        raise MvpbError(E_DEVICE, f"hipDeviceSynchronize failed with {rc}")


def _check(rc):
    if rc != OK:
        raise MvpbError(rc, load().mvpb_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def version() -> str:
    return load().mvpb_version().decode()


def kpath_square(n_k: int) -> np.ndarray:
    Q = np.zeros((n_k, 2), dtype=np.float64)
    _check(load().mvpb_kpath_square(n_k, _dptr(Q)))
    return Q


def kpath(lattice, path: str, n_k: int) -> np.ndarray:
    """Bloch vectors (fractional Q) equally spaced in Cartesian arc length along
    the symmetry points of ``path`` (letters G, X, Y, M, J)."""
    lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(4))
    Q = np.zeros((n_k, 2), dtype=np.float64)
    _check(load().mvpb_kpath(_dptr(lat), path.encode(), n_k, _dptr(Q)))
    return Q


class Context:
    """A device context (HIP device + stream + workspace)."""

    def __init__(self, device: int = 0, stream=None, workspace_cap: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        s = ctypes.c_void_p(int(stream)) if stream is not None else None
        _check(lib.mvpb_ctx_create(device, s, workspace_cap, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            load().mvpb_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, enable: bool = True):
        _check(load().mvpb_ctx_profile(self.h, 1 if enable else 0))

    def set_accuracy(self, tol: float):
        """Bar on the estimated relative frequency error of solves with the
        FP32 reduction (0 turns the check off)."""
        _check(load().mvpb_ctx_set_accuracy(self.h, float(tol)))

    def load_tuning(self, path: str) -> int:
        """Apply the launch shapes a tuning cache holds for this device; returns how many."""
        n = ctypes.c_int()
        _check(load().mvpb_ctx_load_tuning(self.h, os.fsencode(path), ctypes.byref(n)))
        return n.value

    def set_launch_shape(self, n: int, parts: int, group: int = 0, wg_max: int = 0):
        """Launch shape of the eigensolve for operators of order n's size class."""
        _check(load().mvpb_ctx_set_launch_shape(self.h, n, parts, group, wg_max))

    def launch_shape(self, n: int):
        """(parts, group, wg_max) used for operators of order n."""
        v = [ctypes.c_int() for _ in range(3)]
        _check(load().mvpb_ctx_get_launch_shape(self.h, n, *[ctypes.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def set_wait_limit(self, spins: int):
        """Polls of a bulge-chasing hand-over wait before a point gives up (0: default)."""
        _check(load().mvpb_ctx_set_wait_limit(self.h, int(spins)))

    def last_accuracy(self) -> float:
        """Largest error estimate of the refined bands of the last synchronous solve."""
        v = ctypes.c_double()
        _check(load().mvpb_ctx_last_accuracy(self.h, ctypes.byref(v)))
        return v.value

    def profile_only(self, names):
        """Time only the named kernel families (empty: stop timing)."""
        ids = [self.kernel_names().index(n) for n in names]
        _check(load().mvpb_ctx_profile_mask(self.h, sum(1 << i for i in ids)))

    def kernel_names(self) -> list:
        out = []
        for k in range(N_KERNELS):
            nm = ctypes.c_char_p()
            _check(load().mvpb_ctx_profile_read(self.h, k, None, None, ctypes.byref(nm)))
            out.append(nm.value.decode())
        return out

    def profile_read(self) -> dict:
        """{kernel name: (total_ms, launches)} of the timed launches."""
        out = {}
        for k in range(N_KERNELS):
            ms = ctypes.c_double()
            n = ctypes.c_longlong()
            nm = ctypes.c_char_p()
            _check(load().mvpb_ctx_profile_read(self.h, k, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(nm)))
            out[nm.value.decode()] = (ms.value, n.value)
        return out

    def copy_device(self, dst: int, src: int, nbytes: int):
        """Plain device-to-device copy by the library's copy16 kernel (waits for it)."""
        _check(load().mvpb_copy_device(self.h, ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes))

    def cell(self, phase, props, lattice=None):
        return Cell(self, phase, props, lattice)

    def cell_voxels(self, phase, props, lattice=None):
        """A voxel cell (three-dimensional); phase [nx, ny, nz]."""
        return Cell.from_voxels(self, phase, props, lattice)

    def cell_polygons(self, polygons, poly_phase, props, lattice):
        """A polygon cell: ``polygons`` a list of [n_i, 2] vertex arrays
        (Cartesian; counter-clockwise adds, clockwise subtracts)."""
        return Cell.from_polygons(self, polygons, poly_phase, props, lattice)

    def plans(self, cells, Ms, precision: int = PREC_FP64) -> list:
        """Plans for many cells at once (batched per-cell assembly)."""
        n = len(cells)
        ch = (ctypes.c_void_p * n)(*[c.h for c in cells])
        m1 = (ctypes.c_int * n)(*[int(M if np.isscalar(M) else M[0]) for M in Ms])
        m2 = (ctypes.c_int * n)(*[int(M if np.isscalar(M) else M[1]) for M in Ms])
        out = (ctypes.c_void_p * n)()
        _check(load().mvpb_plan_create_batch(self.h, n, ch, m1, m2, precision, out))
        res = []
        for i in range(n):
            p = Plan.__new__(Plan)
            p.ctx = self
            p.qdim = 2
            p.h = ctypes.c_void_p(out[i])
            nu, ns = ctypes.c_int(), ctypes.c_int()
            _check(load().mvpb_plan_dofs(p.h, ctypes.byref(nu), ctypes.byref(ns)))
            p.n_u, p.n_s = nu.value, ns.value
            res.append(p)
        return res

    def solve_cells(self, cells, Ms, Qs, n_bands: int, precision: int = PREC_FP64) -> list:
        """Bands of many pixel cells, plan build and eigensolve in one captured
        graph (replayed by later calls of the same shape)."""
        lib = load()
        n = len(cells)
        Qs = [np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1, 2)) for q in Qs]
        outs = [np.zeros((q.shape[0], n_bands)) for q in Qs]
        ch = (ctypes.c_void_p * n)(*[c.h for c in cells])
        m1 = (ctypes.c_int * n)(*[int(M if np.isscalar(M) else M[0]) for M in Ms])
        m2 = (ctypes.c_int * n)(*[int(M if np.isscalar(M) else M[1]) for M in Ms])
        nk = (ctypes.c_int * n)(*[q.shape[0] for q in Qs])
        qp = (ctypes.POINTER(ctypes.c_double) * n)(*[_dptr(q) for q in Qs])
        op = (ctypes.c_void_p * n)(*[o.ctypes.data for o in outs])
        _check(lib.mvpb_solve_cells(self.h, n, ch, m1, m2, precision, nk, qp, n_bands, op, 0))
        return outs

    def solve_batch(self, plans, Qs, n_bands: int) -> list:
        lib = load()
        n = len(plans)
        Qs = [np.ascontiguousarray(np.asarray(q, dtype=np.float64).reshape(-1, getattr(p, "qdim", 2)))
              for q, p in zip(Qs, plans)]
        outs = [np.zeros((q.shape[0], n_bands)) for q in Qs]
        ph = (ctypes.c_void_p * n)(*[p.h for p in plans])
        nk = (ctypes.c_int * n)(*[q.shape[0] for q in Qs])
        qp = (ctypes.POINTER(ctypes.c_double) * n)(*[_dptr(q) for q in Qs])
        op = (ctypes.c_void_p * n)(*[o.ctypes.data for o in outs])
        _check(lib.mvpb_solve_batch(self.h, n, ph, nk, qp, n_bands, op, 0))
        return outs


def _prop_kind(props, dim: int):
    """Rows of (E, nu, rho) -> ISO; rows of the engineering-Voigt compliance
    upper triangle plus rho (7 planar, 22 spatial values) -> VOIGT_D_RHO."""
    pr = np.asarray(props, dtype=np.float64)
    width = pr.shape[-1] if pr.ndim == 2 else 3
    voigt = 7 if dim == 2 else 22
    if width == 3:
        return PROP_ISO_E_NU_RHO, np.ascontiguousarray(pr.reshape(-1, 3))
    if width == voigt:
        return PROP_VOIGT_D_RHO, np.ascontiguousarray(pr.reshape(-1, voigt))
    raise ValueError(f"property rows must have 3 (E, nu, rho) or {voigt} (Voigt compliance, rho) values")


class Cell:
    """A pixel unit cell: phase map [nx, ny] (i along h1) and per-phase rows of
    (E, nu, rho) or of the engineering-Voigt compliance (d11, d12, d13, d22,
    d23, d33) and rho."""

    def __init__(self, ctx: Context, phase, props, lattice=None):
        lib = load()
        self.ctx = ctx
        self.dim = 2
        ph = np.ascontiguousarray(np.asarray(phase, dtype=np.int32))
        kind, pr = _prop_kind(props, 2)
        lat = np.ascontiguousarray(np.asarray(lattice if lattice is not None else np.eye(2), dtype=np.float64).reshape(4))
        h = ctypes.c_void_p()
        _check(lib.mvpb_cell_create_pixels(ctx.h, _dptr(lat), ph.shape[0], ph.shape[1],
                                           ph.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), pr.shape[0],
                                           kind, _dptr(pr), ctypes.byref(h)))
        self.h = h

    @classmethod
    def from_voxels(cls, ctx: Context, phase, props, lattice=None):
        """A voxel cell: phase map [nx, ny, nz] (i along h1, k along h3), rows
        of (E, nu, rho) or of the 21 Voigt compliances and rho."""
        lib = load()
        self = cls.__new__(cls)
        self.ctx = ctx
        self.h = None
        self.dim = 3
        ph = np.ascontiguousarray(np.asarray(phase, dtype=np.int32))
        kind, pr = _prop_kind(props, 3)
        lat = np.ascontiguousarray(np.asarray(lattice if lattice is not None else np.eye(3), dtype=np.float64).reshape(9))
        h = ctypes.c_void_p()
        _check(lib.mvpb_cell_create_voxels(ctx.h, _dptr(lat), ph.shape[0], ph.shape[1], ph.shape[2],
                                           ph.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), pr.shape[0], kind,
                                           _dptr(pr), ctypes.byref(h)))
        self.h = h
        return self

    @classmethod
    def from_polygons(cls, ctx: Context, polygons, poly_phase, props, lattice):
        lib = load()
        self = cls.__new__(cls)
        self.ctx = ctx
        self.h = None
        self.dim = 2
        verts = [np.asarray(v, dtype=np.float64).reshape(-1, 2) for v in polygons]
        off = np.zeros(len(verts) + 1, dtype=np.int32)
        off[1:] = np.cumsum([v.shape[0] for v in verts])
        xy = np.ascontiguousarray(np.concatenate(verts, axis=0).reshape(-1))
        ph = np.ascontiguousarray(np.asarray(poly_phase, dtype=np.int32))
        pr = np.ascontiguousarray(np.asarray(props, dtype=np.float64).reshape(-1, 3))
        lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(4))
        h = ctypes.c_void_p()
        I32 = ctypes.POINTER(ctypes.c_int32)
        _check(lib.mvpb_cell_create_polygons(ctx.h, _dptr(lat), len(verts), ph.ctypes.data_as(I32),
                                             off.ctypes.data_as(I32), _dptr(xy), pr.shape[0],
                                             PROP_ISO_E_NU_RHO, _dptr(pr), ctypes.byref(h)))
        self.h = h
        return self

    def close(self):
        if self.h:
            load().mvpb_cell_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def structure_factors(self, M1: int, M2: int, precision: int = PREC_FP64) -> np.ndarray:
        F = np.zeros((4, 4 * M1 + 1, 4 * M2 + 1), dtype=np.complex128)
        _check(load().mvpb_structure_factors(self.h, M1, M2, precision,
                                             F.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return F

    def structure_factors_noalloc(self, M1: int, M2: int, out: "DeviceBuffer", precision: int = PREC_FP64,
                                  flags: int = 0):
        """mvpb_structure_factors_noalloc into the caller's device buffer ``out``
        (4*(4M1+1)*(4M2+1) complex doubles); the library allocates nothing."""
        need = 16 * 4 * (4 * M1 + 1) * (4 * M2 + 1)
        if out.nbytes < need:
            raise ValueError(f"output buffer holds {out.nbytes} bytes, {need} needed")
        _check(load().mvpb_structure_factors_noalloc(self.h, M1, M2, precision, out.ptr, flags))
        return out

    def structure_factors_general(self, M1: int, M2: int, M3: int = 0) -> np.ndarray:
        """Weight fields of the general layout [nf, 4M1+1, 4M2+1, 4M3+1] (Voigt
        compliance upper triangle, then rho)."""
        nf = 7 if self.dim == 2 else 22
        F = np.zeros((nf, 4 * M1 + 1, 4 * M2 + 1, 4 * M3 + 1), dtype=np.complex128)
        _check(load().mvpb_structure_factors_general(self.h, M1, M2, M3,
                                                     F.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return F

    def plan(self, M1: int, M2: int = None, precision: int = PREC_FP64, M3: int = None):
        """Plan at cutoff (M1, M2[, M3]); a voxel cell takes M3 (default: M1)."""
        M2 = M1 if M2 is None else M2
        if self.dim == 3:
            return Plan(self, M1, M2, precision, M1 if M3 is None else M3)
        return Plan(self, M1, M2, precision)


class Plan:
    """k-independent part of the method for one cell and cutoff."""

    def __init__(self, cell: Cell, M1: int, M2: int, precision: int = PREC_FP64, M3: int = None):
        lib = load()
        self.ctx = cell.ctx
        h = ctypes.c_void_p()
        if M3 is None:
            _check(lib.mvpb_plan_create(cell.h, M1, M2, precision, ctypes.byref(h)))
        else:
            _check(lib.mvpb_plan_create3(cell.h, M1, M2, M3, precision, ctypes.byref(h)))
        self.h = h
        self.qdim = getattr(cell, "dim", 2)
        nu, ns = ctypes.c_int(), ctypes.c_int()
        _check(lib.mvpb_plan_dofs(h, ctypes.byref(nu), ctypes.byref(ns)))
        self.n_u, self.n_s = nu.value, ns.value

    def close(self):
        if self.h:
            load().mvpb_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, Q, n_bands: int, vectors: bool = False):
        """Frequencies [n_k, n_bands] (rad/s) and optionally U [n_k, n_bands, n_u]."""
        lib = load()
        Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(-1, self.qdim))
        om = np.zeros((Q.shape[0], n_bands))
        U = np.zeros((Q.shape[0], n_bands, self.n_u), dtype=np.complex128) if vectors else None
        _check(lib.mvpb_solve(self.h, Q.shape[0], _dptr(Q), n_bands, ctypes.c_void_p(om.ctypes.data),
                              ctypes.c_void_p(U.ctypes.data) if vectors else None, 0))
        return (om, U) if vectors else om

    def stress(self, Q, U):
        """Stress modes S = -Phi^-1 H* U [n_k, n_bands, n_s] of displacement modes
        U [n_k, n_bands, n_u] (as returned by solve(..., vectors=True))."""
        lib = load()
        Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(-1, self.qdim))
        U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
        nk, nb = U.shape[0], U.shape[1]
        if U.shape[2] != self.n_u or nk != Q.shape[0]:
            raise ValueError("U must be [n_k, n_bands, n_u] for the Q list")
        S = np.zeros((nk, nb, self.n_s), dtype=np.complex128)
        _check(lib.mvpb_stress_modes(self.h, nk, _dptr(Q), nb, U.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0))
        return S

    def autotune(self, Q, n_bands: int, cache_path: str = None) -> float:
        """Pick the fastest launch shape for this plan's operator size (kept by
        the context, merged into cache_path if given); returns its time in ms."""
        Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(-1, self.qdim))
        ms = ctypes.c_double()
        _check(load().mvpb_autotune(self.h, Q.shape[0], _dptr(Q), n_bands,
                                    os.fsencode(cache_path) if cache_path else None, ctypes.byref(ms)))
        return ms.value

    def sensitivities(self, Q, omega, U, grid_shape):
        """d lambda / d w_f of every pixel / voxel: [n_k, n_bands, nf, *grid_shape]
        from the (omega, U) that solve(..., vectors=True) returned."""
        lib = load()
        Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(-1, self.qdim))
        om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        U = np.ascontiguousarray(np.asarray(U, dtype=np.complex128))
        nk, nb = om.shape
        if U.shape != (nk, nb, self.n_u) or Q.shape[0] != nk:
            raise ValueError("omega [n_k, n_bands] and U [n_k, n_bands, n_u] must match the Q list")
        nf = 7 if self.qdim == 2 else 22
        G = np.zeros((nk, nb, nf) + tuple(grid_shape))
        _check(lib.mvpb_band_sensitivities(self.h, nk, _dptr(Q), nb, ctypes.c_void_p(om.ctypes.data),
                                           ctypes.c_void_p(U.ctypes.data), ctypes.c_void_p(G.ctypes.data), 0))
        return G

    def solve_device(self, Q, n_bands: int, omega_ptr: int, flags: int = F_DEVICE_PTRS):
        """Write frequencies to device memory at omega_ptr (e.g. DeviceBuffer.value)."""
        lib = load()
        Q = np.ascontiguousarray(np.asarray(Q, dtype=np.float64).reshape(-1, self.qdim))
        _check(lib.mvpb_solve(self.h, Q.shape[0], _dptr(Q), n_bands, ctypes.c_void_p(omega_ptr), None,
                              flags | F_DEVICE_PTRS))


class Surrogate:
    """Band-structure screening network trained and run by the library's kernels.

    precision 0: FP32 products; 1: BF16 matrix-core products with FP32
    accumulation.  cells: uint8 [B, 32, 32]; targets / outputs float32 [B, 400].
    """
    N_OUT = 400

    def __init__(self, ctx: Context, max_batch: int = 256, precision: int = 1, seed: int = 0):
        lib = load()
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib.mvpb_sur_create(ctx.h, max_batch, precision, seed, ctypes.byref(h)))
        self.h = h
        n = ctypes.c_int()
        _check(lib.mvpb_sur_n_params(h, ctypes.byref(n)))
        self.n_params = n.value

    def close(self):
        if self.h:
            load().mvpb_sur_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def save(self, path: str):
        """Checkpoint (parameters, Adam moments and step) to ``path``."""
        _check(load().mvpb_sur_save(self.h, os.fsencode(path)))

    @classmethod
    def load(cls, ctx: Context, path: str, max_batch: int = 256):
        """A network restored from a checkpoint written by ``save``."""
        lib = load()
        self = cls.__new__(cls)
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib.mvpb_sur_load(ctx.h, os.fsencode(path), max_batch, ctypes.byref(h)))
        self.h = h
        n = ctypes.c_int()
        _check(lib.mvpb_sur_n_params(h, ctypes.byref(n)))
        self.n_params = n.value
        return self

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        _check(load().mvpb_sur_get_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        _check(load().mvpb_sur_set_params(self.h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    @staticmethod
    def _cells(cells):
        return np.ascontiguousarray(np.asarray(cells, dtype=np.uint8).reshape(-1, 32 * 32))

    def infer(self, cells) -> np.ndarray:
        c = self._cells(cells)
        out = np.zeros((c.shape[0], self.N_OUT), dtype=np.float32)
        _check(load().mvpb_sur_infer(self.h, c.shape[0], ctypes.c_void_p(c.ctypes.data),
                                     ctypes.c_void_p(out.ctypes.data), 0))
        return out

    def infer_device(self, batch: int, cells_ptr: int, out_ptr: int):
        _check(load().mvpb_sur_infer(self.h, batch, ctypes.c_void_p(cells_ptr), ctypes.c_void_p(out_ptr),
                                     F_DEVICE_PTRS))

    def gradients(self, cells, target):
        c = self._cells(cells)
        t = np.ascontiguousarray(np.asarray(target, dtype=np.float32).reshape(c.shape[0], self.N_OUT))
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_float()
        _check(load().mvpb_sur_gradients(self.h, c.shape[0], ctypes.c_void_p(c.ctypes.data),
                                         ctypes.c_void_p(t.ctypes.data), ctypes.byref(loss),
                                         ctypes.c_void_p(g.ctypes.data), 0))
        return float(loss.value), g

    def train_step(self, cells, target, lr: float = 1e-3) -> float:
        c = self._cells(cells)
        t = np.ascontiguousarray(np.asarray(target, dtype=np.float32).reshape(c.shape[0], self.N_OUT))
        loss = ctypes.c_float()
        _check(load().mvpb_sur_train_step(self.h, c.shape[0], ctypes.c_void_p(c.ctypes.data),
                                          ctypes.c_void_p(t.ctypes.data), lr, ctypes.byref(loss), 0))
        return float(loss.value)

    def train_step_device(self, batch: int, cells_ptr: int, target_ptr: int, lr: float = 1e-3) -> float:
        loss = ctypes.c_float()
        _check(load().mvpb_sur_train_step(self.h, batch, ctypes.c_void_p(cells_ptr), ctypes.c_void_p(target_ptr),
                                          lr, ctypes.byref(loss), F_DEVICE_PTRS))
        return float(loss.value)
