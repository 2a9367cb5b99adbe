"""Python binding of libsparsect: sparse Radon operators, normal operator, CG and
split Bregman on AMD MI355X (gfx950).

Every call marshals arguments into the C ABI declared in include/sparsect.h;
all arithmetic runs in the library's HIP kernels.  PyTorch supplies device
memory (tensors) and the current stream.  There is no CPU fallback: without
the built library or a GPU the calls raise.

Method: Barnard & Archibald, "Accelerating optimization-based computed
tomography via sparse matrix approximations" -- the Radon transform is
precomputed as a sparse matrix for a fixed geometry (Section 3) and applied
inside CG solves of eq:KKT / eq:PD_resolve / eq:SB_solve (Section 2) and
anisotropic-TV split Bregman (Section 4).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsparsect.so")

F32, F64, F32_F64 = 0, 1, 2
WS_FWD, WS_NORMAL, WS_CG, WS_SB, WS_PD, WS_TUNE, WS_ADJ = 0, 1, 2, 3, 4, 5, 6
WS_PIXEL_LAYOUT = 0x100
LAYOUT_IMAGE, LAYOUT_PIXEL = 0, 1
SB_WARM, SB_RESUME = 1, 2

_vp = ctypes.c_void_p


class SparsectError(RuntimeError):
    """A libsparsect call returned a negative status."""


class _Geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("measured", ctypes.POINTER(ctypes.c_uint8)),
                ("fwd_bundle", ctypes.c_int32), ("fwd_angles", ctypes.c_int32),
                ("fwd_compact", ctypes.c_int32), ("fwd_symmetric", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n_pixels", ctypes.c_int64), ("n_meas_angles", ctypes.c_int64),
                ("n_meas_rays", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("fwd_slots", ctypes.c_int64), ("adj_slots", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("n", ctypes.c_int32), ("n_angles", ctypes.c_int32), ("n_bins", ctypes.c_int32),
                ("needs_transpose", ctypes.c_int32), ("fwd_bundle", ctypes.c_int32),
                ("fwd_angles", ctypes.c_int32), ("fwd_compact", ctypes.c_int32),
                ("fwd_symmetric", ctypes.c_int32), ("adj_symmetric", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RadonSizes(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in (
        "n_meas_rays", "nnz", "fwd_slots", "adj_slots", "row_ptr_bytes", "col_bytes", "val_bytes",
        "layout_bytes", "ws_bytes")]


class RadonBuffers(ctypes.Structure):
    _fields_ = [("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("layout", ctypes.c_void_p), ("ws", ctypes.c_void_p),
                ("row_ptr_bytes", ctypes.c_int64), ("col_bytes", ctypes.c_int64),
                ("val_bytes", ctypes.c_int64), ("layout_bytes", ctypes.c_int64),
                ("ws_bytes", ctypes.c_int64)]


class CgInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("breakdown", ctypes.c_int32),
                ("rho0", ctypes.c_double), ("rho", ctypes.c_double)]


class SbParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("lambda_", ctypes.c_double), ("tol", ctypes.c_double),
                ("n_outer", ctypes.c_int32), ("n_cg", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class PdParams(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("tau", ctypes.c_double), ("sigma", ctypes.c_double),
                ("n_outer", ctypes.c_int32), ("n_cg", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class FourierInfo(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("grid", ctypes.c_int32), ("m_sp", ctypes.c_int32),
                ("tau", ctypes.c_double), ("fused_tiles", ctypes.c_int64), ("fused_bytes", ctypes.c_int64),
                ("spread_nnz", ctypes.c_int64), ("device_bytes", ctypes.c_int64)]


FOURIER_FUSED, FOURIER_NUFFT = 0, 1
FWS_TRANSFORM, FWS_SB = 0, 1


class Tuning(ctypes.Structure):
    _fields_ = [("fwd_waves", ctypes.c_int32), ("adj_waves", ctypes.c_int32),
                ("fwd_rhs", ctypes.c_int32), ("adj_rhs", ctypes.c_int32),
                ("fwd_layout", ctypes.c_int32), ("fwd_lines", ctypes.c_int32),
                ("adj_layout", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class SbInfo(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int32), ("breakdowns", ctypes.c_int32),
                ("upd_b_first", ctypes.c_double), ("upd_b", ctypes.c_double),
                ("upd_u", ctypes.c_double)]


# exported symbols and their signatures (kept in step with include/sparsect.h)
SIGNATURES = {
    "build_radon_csr": (ctypes.c_int, [ctypes.POINTER(_Geom), _vp, ctypes.POINTER(_vp)]),
    "radon_csr_sizes": (ctypes.c_int, [ctypes.POINTER(_Geom), _vp, ctypes.c_int64, _vp,
                                       ctypes.POINTER(RadonSizes)]),
    "build_radon_csr_into": (ctypes.c_int, [ctypes.POINTER(_Geom), ctypes.POINTER(RadonBuffers), _vp,
                                            ctypes.POINTER(_vp)]),
    "radon_op_info": (ctypes.c_int, [_vp, ctypes.POINTER(_Info)]),
    "radon_op_destroy": (None, [_vp]),
    "radon_last_error": (ctypes.c_char_p, []),
    "radon_workspace_bytes": (ctypes.c_int64, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "radon_fwd": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64,
                                 _vp]),
    "radon_adj": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64,
                                 _vp]),
    "radon_fwd_xt": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_int32, _vp]),
    "normal_apply": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp, _vp,
                                    _vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64, _vp]),
    "normal_apply_noalloc": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                            _vp, _vp, _vp, ctypes.c_int32, _vp]),
    "cg_solve": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp, _vp,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_double, _vp, ctypes.c_int64, _vp, _vp]),
    "split_bregman_tv": (ctypes.c_int, [_vp, ctypes.POINTER(SbParams), _vp, _vp, ctypes.c_int32,
                                        ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp]),
    "radon_set_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(Tuning)]),
    "radon_get_tuning": (ctypes.c_int, [_vp, ctypes.POINTER(Tuning)]),
    "radon_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, ctypes.c_int64, ctypes.c_char_p,
                                      ctypes.c_int32, _vp, ctypes.POINTER(ctypes.c_int32)]),
    "radon_export_csr": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "radon_bandwidth_probe": (ctypes.c_int, [ctypes.c_int32, _vp, _vp, ctypes.c_int64, _vp]),
    "radon_export_adj": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "radon_unrolled_sizes": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64),
                                            ctypes.POINTER(ctypes.c_int64)]),
    "cg_unrolled": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp, _vp,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int64,
                                   _vp, ctypes.c_int64, _vp]),
    "radon_multi_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, _vp, _vp, _vp,
                                          ctypes.POINTER(_vp)]),
    "radon_multi_table_bytes": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32,
                                               ctypes.POINTER(ctypes.c_int64)]),
    "radon_multi_create_into": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, _vp, _vp, _vp, _vp,
                                               ctypes.c_int64, ctypes.POINTER(_vp)]),
    "radon_multi_destroy": (None, [_vp]),
    "radon_multi_info": (ctypes.c_int, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "radon_multi_apply": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int64, _vp]),
    "radon_multi_cg": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_double, _vp,
                                      ctypes.c_int64, _vp, _vp]),
    "radon_multi_cg_graph": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_double, _vp,
                                            ctypes.c_int64, _vp, ctypes.POINTER(_vp)]),
    "radon_graph_launch": (ctypes.c_int, [_vp, _vp]),
    "split_bregman_tv_graph": (ctypes.c_int, [_vp, ctypes.POINTER(SbParams), _vp, _vp, ctypes.c_int32,
                                              _vp, ctypes.c_int64, _vp, ctypes.POINTER(_vp)]),
    "radon_graph_destroy": (None, [_vp]),
    "chambolle_pock_tv": (ctypes.c_int, [_vp, ctypes.POINTER(PdParams), _vp, _vp, ctypes.c_int32,
                                          _vp, ctypes.c_int64, _vp]),
    "radon_surrogate_create": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, ctypes.POINTER(_vp)]),
    "radon_surrogate_destroy": (None, [_vp]),
    "radon_surrogate_weights": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32), _vp]),
    "surrogate_apply": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp,
                                       _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64, _vp]),
    "split_bregman_tv_surrogate": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(SbParams), _vp, _vp,
                                                  ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp]),
    "radon_fourier_create": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _vp,
                                            ctypes.POINTER(_vp)]),
    "radon_fourier_destroy": (None, [_vp]),
    "radon_fourier_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(FourierInfo)]),
    "radon_fourier_workspace_bytes": (ctypes.c_int64, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "fourier_fwd": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64, _vp]),
    "fourier_adj": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32, _vp, ctypes.c_int64,
                                   _vp]),
    "fourier_normal": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, _vp, _vp, _vp, ctypes.c_int32, _vp, ctypes.c_int64,
                                      _vp]),
    "split_bregman_tv_fourier": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(SbParams), _vp, _vp,
                                                ctypes.c_int32, _vp, ctypes.c_int64, _vp, _vp]),
    "cg_unrolled_vjp": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp,
                                       ctypes.c_int64, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, _vp, ctypes.c_int64, _vp]),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libsparsect.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SparsectError(f"{LIB_PATH} is missing: run paper_1705_07497_amd.build_lib.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> None:
    if rc != 0:
        msg = lib().radon_last_error()
        raise SparsectError(f"status {rc}: {msg.decode() if msg else ''}")


def _torch():
    import torch
    return torch


@dataclass
class OpInfo:
    n_pixels: int
    n_meas_angles: int
    n_meas_rays: int
    nnz: int
    fwd_slots: int
    adj_slots: int
    device_bytes: int


class RadonOp:
    """MR and (MR)^T for one geometry, built on the GPU (see build_radon_csr).

    dtype is the type the matrix values are stored in, vec_dtype the type of
    every vector the calls take and return (default: dtype).  float32 values
    with float64 vectors selects the mixed operator: FP32 matrix stream, FP64
    vectors and multiply-adds.

    storage="library" lets build_radon_csr allocate the matrix storage (owned
    by the handle); storage="torch" sizes it with radon_csr_sizes, allocates
    every array as a torch tensor (kept on the object: .csr() returns the CSR
    tensors) and fills them with build_radon_csr_into.

    bundle is the forward layout's rays per bundle (16, 32 or 64) and
    bundle_angles the consecutive measured angles those rays come from (1, 2
    or 4, at least 16 bins of each); bundle 0 takes both from the cached
    choice for this geometry with tuning="cache", else 16 rays of one angle.
    compact=True builds the compact forward layout: one stored length per
    (ray, line), the second derived from the ray's chord (within about one
    rounding of the matrix type of the stored value; the CSR and the adjoint
    keep the stored values).  symmetric=True stores only the measured angles
    in [0, pi/4] in the forward layout and serves their mirror and transpose
    partners from them (the measured set must be closed under theta ->
    pi - theta and theta -> pi/2 - theta); with n a multiple of 8 the adjoint
    layout is stored the same way (.adj_symmetric).
    tuning: "cache" applies cached launch settings for tune_batch images,
    "tune" chooses the bundle layout and times the launch settings now (and
    caches both), "default" leaves the library defaults."""

    def __init__(self, n: int, n_angles: int, n_bins: int, measured=None, dtype=None, device=None,
                 vec_dtype=None, tuning: str = "cache", storage: str = "library", bundle: int = 0,
                 tune_batch: int = 1, bundle_angles: int = 0, compact: bool = False,
                 symmetric: bool = False):
        torch = _torch()
        if not torch.cuda.is_available():
            raise SparsectError("no GPU visible: libsparsect runs on AMD Instinct GPUs only")
        dtype = torch.float32 if dtype is None else dtype
        vec_dtype = dtype if vec_dtype is None else vec_dtype
        kinds = {(torch.float32, torch.float32): F32, (torch.float64, torch.float64): F64,
                 (torch.float32, torch.float64): F32_F64}
        if (dtype, vec_dtype) not in kinds:
            raise SparsectError("(dtype, vec_dtype) must be (f32, f32), (f64, f64) or (f32, f64)")
        self.kind = kinds[(dtype, vec_dtype)]
        self.device = torch.device("cuda" if device is None else device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.mat_dtype = dtype
        self.dtype = vec_dtype
        self.n, self.n_angles, self.n_bins = int(n), int(n_angles), int(n_bins)
        if measured is None:
            self.measured = np.ones(self.n_angles, dtype=np.uint8)
        else:
            self.measured = np.ascontiguousarray(np.asarray(measured, dtype=np.uint8))
            if self.measured.shape != (self.n_angles,):
                raise SparsectError("measured must have one flag per angle")
        self.n_meas = int(np.count_nonzero(self.measured))
        if tuning not in ("cache", "tune", "default"):
            raise SparsectError("tuning must be 'cache', 'tune' or 'default'")
        if bundle == 0 and tuning != "default":
            from . import autotune
            if tuning == "tune":
                ch = autotune.choose_bundle(self.n, self.n_angles, self.n_bins, self.measured,
                                            dtype, vec_dtype, self.device, batch=tune_batch,
                                            compact=compact, symmetric=symmetric)
                bundle, bundle_angles = ch["bundle"], ch["angles"]
            else:
                bundle, bundle_angles = autotune.cached_bundle(self.n, self.n_angles, self.n_bins,
                                                               self.measured, self.kind,
                                                               self.device, compact=compact,
                                                               symmetric=symmetric) or (0, 0)
        g = _Geom(self.n, self.n_angles, self.n_bins, self.kind,
                  self.measured.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), int(bundle),
                  int(bundle_angles), 1 if compact else 0, 1 if symmetric else 0)
        h = _vp()
        self._storage = None
        with torch.cuda.device(self.device):
            if storage == "library":
                _check(lib().build_radon_csr(ctypes.byref(g), self._stream(), ctypes.byref(h)))
            elif storage == "torch":
                self._storage = self._build_into(g, h)
            else:
                raise SparsectError("storage must be 'library' or 'torch'")
        self._h = h
        inf = _Info()
        _check(lib().radon_op_info(self._h, ctypes.byref(inf)))
        self.info = OpInfo(inf.n_pixels, inf.n_meas_angles, inf.n_meas_rays, inf.nnz, inf.fwd_slots,
                           inf.adj_slots, inf.device_bytes)
        self.rows = inf.n_meas_rays
        self.needs_transpose = bool(inf.needs_transpose)
        self.nn = inf.n_pixels
        self.bundle = int(inf.fwd_bundle)
        self.bundle_angles = int(inf.fwd_angles)
        self.compact = bool(inf.fwd_compact)
        self.symmetric = bool(inf.fwd_symmetric)
        self.adj_symmetric = bool(inf.adj_symmetric)
        self._ws = {}
        if tuning == "cache":
            from . import autotune
            autotune.apply_cached(self, batch=tune_batch)
        elif tuning == "tune":
            from . import autotune
            autotune.autotune(self, batch=tune_batch)

    def _build_into(self, g, h):
        """radon_csr_sizes, torch allocations, build_radon_csr_into."""
        torch = _torch()
        sz = RadonSizes()
        _check(lib().radon_csr_sizes(ctypes.byref(g), None, 0, self._stream(), ctypes.byref(sz)))
        ws = torch.empty(max(int(sz.ws_bytes), 1), dtype=torch.uint8, device=self.device)
        _check(lib().radon_csr_sizes(ctypes.byref(g), _vp(ws.data_ptr()), ws.numel(), self._stream(),
                                     ctypes.byref(sz)))
        rp = torch.empty(sz.n_meas_rays + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(sz.nnz, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(sz.nnz, 1), dtype=self.mat_dtype, device=self.device)
        lay = torch.empty(max(int(sz.layout_bytes), 1), dtype=torch.uint8, device=self.device)
        b = RadonBuffers(rp.data_ptr(), col.data_ptr(), val.data_ptr(), lay.data_ptr(), ws.data_ptr(),
                         rp.numel() * 8, col.numel() * 4, val.numel() * val.element_size(),
                         lay.numel(), ws.numel())
        _check(lib().build_radon_csr_into(ctypes.byref(g), ctypes.byref(b), self._stream(),
                                          ctypes.byref(h)))
        self.sizes = {f: int(getattr(sz, f)) for f, _ in RadonSizes._fields_}
        return rp, col[:sz.nnz], val[:sz.nnz], lay

    def csr(self):
        """(row_ptr int64, col int32, val) device tensors of MR when storage="torch"."""
        if self._storage is None:
            raise SparsectError("the CSR tensors exist only for storage='torch' (use export_csr)")
        return self._storage[:3]

    @property
    def tuning(self) -> dict:
        t = Tuning()
        _check(lib().radon_get_tuning(self._h, ctypes.byref(t)))
        return t.as_dict()

    @tuning.setter
    def tuning(self, d: dict) -> None:
        t = Tuning()
        _check(lib().radon_get_tuning(self._h, ctypes.byref(t)))
        names = [f for f, _ in Tuning._fields_]
        for k, v in d.items():
            if k not in names:
                raise SparsectError(f"unknown tuning key {k!r} (known: {', '.join(names)})")
            setattr(t, k, int(v))
        _torch().cuda.synchronize(self.device)
        _check(lib().radon_set_tuning(self._h, ctypes.byref(t)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _torch().cuda.synchronize(self.device)
            except Exception:
                pass
            _lib.radon_op_destroy(h)
            self._h = None

    # -- helpers --------------------------------------------------------------
    def _stream(self):
        torch = _torch()
        return _vp(torch.cuda.current_stream(self.device).cuda_stream)

    def workspace(self, which: int, batch: int, key=None):
        """Cached device workspace of the size the library asks for."""
        torch = _torch()
        nbytes = lib().radon_workspace_bytes(self._h, which, batch)
        if nbytes < 0:
            _check(int(nbytes))
        k = (which, batch) if key is None else key
        buf = self._ws.get(k)
        if buf is None or buf.numel() < nbytes:
            grown = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=self.device)
            if buf is not None:
                # keep what a solver left there (split Bregman's state for a resumed call)
                grown[:buf.numel()].copy_(buf)
            buf = grown
            self._ws[k] = buf
        return buf, int(nbytes)

    def _img(self, x, name="x"):
        torch = _torch()
        if not isinstance(x, torch.Tensor) or x.device != self.device or x.dtype != self.dtype:
            raise SparsectError(f"{name} must be a {self.dtype} tensor on {self.device}")
        if not x.is_contiguous():
            raise SparsectError(f"{name} must be contiguous")
        if x.numel() % self.nn:
            raise SparsectError(f"{name} has {x.numel()} elements, not a multiple of n*n = {self.nn}")
        return x.numel() // self.nn

    def _sino(self, y, name="y"):
        torch = _torch()
        if not isinstance(y, torch.Tensor) or y.device != self.device or y.dtype != self.dtype:
            raise SparsectError(f"{name} must be a {self.dtype} tensor on {self.device}")
        if not y.is_contiguous():
            raise SparsectError(f"{name} must be contiguous")
        if y.numel() % self.rows:
            raise SparsectError(f"{name} has {y.numel()} elements, not a multiple of {self.rows}")
        return y.numel() // self.rows

    def _img_n(self, x, b, name):
        """_img, and the image count must be b (a caller's output buffer)."""
        got = self._img(x, name)
        if got != b:
            raise SparsectError(f"{name} holds {got} images, the call needs {b}")

    def _sino_n(self, y, b, name):
        """_sino, and the sinogram count must be b."""
        got = self._sino(y, name)
        if got != b:
            raise SparsectError(f"{name} holds {got} sinograms, the call needs {b}")

    @staticmethod
    def _p(t):
        return _vp(t.data_ptr()) if t is not None else None

    # -- products -------------------------------------------------------------
    @staticmethod
    def _ws_kind(which: int, layout: int) -> int:
        if layout not in (LAYOUT_IMAGE, LAYOUT_PIXEL):
            raise SparsectError("layout must be LAYOUT_IMAGE (0) or LAYOUT_PIXEL (1)")
        return which | (WS_PIXEL_LAYOUT if layout == LAYOUT_PIXEL else 0)

    @staticmethod
    def _check_shape(t, count: int, layout: int, name: str) -> None:
        """A 2-D tensor of several vectors must be [batch, count] image-major and
        [count, batch] pixel-major (the memory alone cannot tell them apart)."""
        if t is None or t.dim() != 2 or t.numel() == count:
            return
        want = 0 if layout == LAYOUT_PIXEL else 1
        if t.shape[want] != count:
            lay = "pixel-major [count, batch]" if layout == LAYOUT_PIXEL else "image-major [batch, count]"
            raise SparsectError(f"{name} has shape {tuple(t.shape)}, not {lay} with count {count}")

    def _new(self, b: int, count: int, layout: int):
        """An output of b vectors of count elements in the given layout."""
        shape = (count, b) if layout == LAYOUT_PIXEL else (b, count)
        return _torch().empty(shape, dtype=self.dtype, device=self.device)

    def fwd(self, x, out=None, layout: int = LAYOUT_IMAGE):
        """y = M R x; x [..., n*n] (or [..., n, n]) -> y [batch, rows].  With
        layout=LAYOUT_PIXEL, x is [n*n, batch] and y [rows, batch]."""
        b = self._img(x)
        y = self._new(b, self.rows, layout) if out is None else out
        self._sino_n(y, b, "out")
        self._check_shape(x, self.nn, layout, "x")
        self._check_shape(y, self.rows, layout, "out")
        ws, nb = self.workspace(self._ws_kind(WS_FWD, layout), b)
        _check(lib().radon_fwd(self._h, self._p(x), self._p(y), b, layout, self._p(ws), nb,
                               self._stream()))
        return y

    def fwd_xt(self, x, xT, out=None):
        """y = M R x from x and its transposed copy xT (the forward kernel alone)."""
        torch = _torch()
        b = self._img(x)
        if xT is not None and self._img(xT, "xT") != b:
            raise SparsectError("xT must hold as many images as x")
        y = torch.empty((b, self.rows), dtype=self.dtype, device=self.device) if out is None else out
        self._sino_n(y, b, "out")
        _check(lib().radon_fwd_xt(self._h, self._p(x), self._p(xT), self._p(y), b, self._stream()))
        return y

    def adj(self, y, out=None, layout: int = LAYOUT_IMAGE):
        """x = R^T M^T y; y [..., rows] -> x [batch, n*n] (layout as for fwd)."""
        b = self._sino(y)
        x = self._new(b, self.nn, layout) if out is None else out
        self._img_n(x, b, "out")
        self._check_shape(y, self.rows, layout, "y")
        self._check_shape(x, self.nn, layout, "out")
        ws, nb = self.workspace(self._ws_kind(WS_ADJ, layout), b)
        _check(lib().radon_adj(self._h, self._p(y), self._p(x), b, layout, self._p(ws) if nb else None,
                               nb, self._stream()))
        return x

    def normal(self, x, alpha: float, lam: float, sigma: float = 0.0, out=None, dot: bool = False,
               layout: int = LAYOUT_IMAGE):
        """alpha R^T M^T M R x + lam K^T K x + sigma x (and <x, out> per image if dot)."""
        torch = _torch()
        b = self._img(x)
        o = self._new(b, self.nn, layout) if out is None else out
        self._img_n(o, b, "out")
        d = torch.empty(b, dtype=torch.float64, device=self.device) if dot else None
        self._check_shape(x, self.nn, layout, "x")
        self._check_shape(o, self.nn, layout, "out")
        ws, nb = self.workspace(self._ws_kind(WS_NORMAL, layout), b)
        _check(lib().normal_apply(self._h, float(alpha), float(lam), float(sigma), self._p(x),
                                  self._p(o), self._p(d), b, layout, self._p(ws), nb, self._stream()))
        return (o, d) if dot else o

    def normal_noalloc(self, x, alpha: float, lam: float, sigma: float = 0.0, out=None,
                       dot: bool = False):
        """normal() through normal_apply_noalloc: no workspace, the library's fixed
        per-GPU scratch array instead (calls that overlap on one GPU race)."""
        torch = _torch()
        b = self._img(x)
        o = torch.empty((b, self.nn), dtype=self.dtype, device=self.device) if out is None else out
        self._img_n(o, b, "out")
        d = torch.empty(b, dtype=torch.float64, device=self.device) if dot else None
        with torch.cuda.device(self.device):
            _check(lib().normal_apply_noalloc(self._h, float(alpha), float(lam), float(sigma),
                                              self._p(x), self._p(o), self._p(d), b, self._stream()))
        return (o, d) if dot else o

    def cg(self, rhs, alpha: float, lam: float, sigma: float = 0.0, x0=None, n_iter: int = 10,
           rtol: float = 0.0, out=None, layout: int = LAYOUT_IMAGE):
        """CG on A(alpha, lam, sigma) x = rhs; returns (x, info tensor of CgInfo bytes)."""
        torch = _torch()
        b = self._img(rhs, "rhs")
        if out is not None:
            self._img_n(out, b, "out")
        if x0 is not None:
            self._img_n(x0, b, "x0")
            x = x0.clone() if out is None else out.copy_(x0)
        else:
            x = self._new(b, self.nn, layout) if out is None else out
        info = torch.zeros(b * ctypes.sizeof(CgInfo), dtype=torch.uint8, device=self.device)
        self._check_shape(rhs, self.nn, layout, "rhs")
        self._check_shape(x, self.nn, layout, "x")
        ws, nb = self.workspace(self._ws_kind(WS_CG, layout), b)
        _check(lib().cg_solve(self._h, float(alpha), float(lam), float(sigma), self._p(rhs),
                              self._p(x), int(x0 is not None), b, layout, int(n_iter), float(rtol),
                              self._p(ws), nb, self._p(info), self._stream()))
        return x, info

    def sb(self, f, alpha: float, lam: float, n_outer: int, n_cg: int, tol: float = 0.0,
           mu0=None, resume: bool = False, out=None, ws_key="sb", surrogate=None,
           layout: int = LAYOUT_IMAGE):
        """Split Bregman TV; returns (mu, info tensor of SbInfo bytes).  The state
        (d, b, carried residual) stays in a cached workspace so resume=True continues.
        With surrogate (a RadonSurrogate of this operator) every inner solve uses
        alpha T + lam K^T K (eq:surr_SBupd)."""
        torch = _torch()
        b = self._sino(f, "f")
        if out is not None:
            self._img_n(out, b, "out")
        if mu0 is not None:
            self._img_n(mu0, b, "mu0")
        flags = 0
        if resume:
            flags |= SB_RESUME
            if out is None:
                raise SparsectError("resume needs out= (the image of the previous call)")
            mu = out
        elif mu0 is not None:
            flags |= SB_WARM
            mu = mu0.clone() if out is None else out.copy_(mu0)
        else:
            mu = self._new(b, self.nn, layout) if out is None else out
        self._img_n(mu, b, "mu")
        P = SbParams(float(alpha), float(lam), float(tol), int(n_outer), int(n_cg), flags, 0)
        info = torch.zeros(b * ctypes.sizeof(SbInfo), dtype=torch.uint8, device=self.device)
        if surrogate is None:
            self._check_shape(f, self.rows, layout, "f")
            self._check_shape(mu, self.nn, layout, "mu")
            ws, nb = self.workspace(self._ws_kind(WS_SB, layout), b, key=(ws_key, b))
            _check(lib().split_bregman_tv(self._h, ctypes.byref(P), self._p(f), self._p(mu), b, layout,
                                          self._p(ws), nb, self._p(info), self._stream()))
        else:
            if layout != LAYOUT_IMAGE:
                raise SparsectError("the surrogate solver takes image-major vectors only")
            ws, nb = self.workspace(WS_SB, b, key=(ws_key, b))
            _check(lib().split_bregman_tv_surrogate(self._h, surrogate._h, ctypes.byref(P),
                                                    self._p(f), self._p(mu), b, self._p(ws), nb,
                                                    self._p(info), self._stream()))
        return mu, info

    def sb_graph(self, f, alpha: float, lam: float, n_outer: int, n_cg: int, tol: float = 0.0):
        """split_bregman_tv captured as one HIP graph (SbGraph): write the data
        into .f, call launch(), read .mu and .info."""
        return SbGraph(self, f, alpha, lam, n_outer, n_cg, tol)

    def unrolled_sizes(self, n_iter: int, ckpt: int, batch: int) -> tuple[int, int, int]:
        """(tape, forward workspace, reverse workspace) bytes of an unrolled CG."""
        t, wf, wv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().radon_unrolled_sizes(self._h, int(n_iter), int(ckpt), int(batch), ctypes.byref(t),
                                          ctypes.byref(wf), ctypes.byref(wv)))
        return int(t.value), int(wf.value), int(wv.value)

    def cg_unrolled(self, rhs, alpha: float, lam: float, sigma: float, n_iter: int, ckpt: int):
        """x = CG_n(rhs) from 0 with a checkpoint tape; returns (x, tape)."""
        torch = _torch()
        b = self._img(rhs, "rhs")
        tb, wf, _ = self.unrolled_sizes(n_iter, ckpt, b)
        tape = torch.empty(max(tb, 1), dtype=torch.uint8, device=self.device)
        x = torch.empty((b, self.nn), dtype=self.dtype, device=self.device)
        ws, nb = self.workspace(WS_CG, b)
        assert nb >= wf
        _check(lib().cg_unrolled(self._h, float(alpha), float(lam), float(sigma), self._p(rhs),
                                 self._p(x), b, int(n_iter), int(ckpt), self._p(tape), tb,
                                 self._p(ws), nb, self._stream()))
        return x, tape

    def cg_unrolled_vjp(self, tape, gx, alpha: float, lam: float, sigma: float, n_iter: int,
                        ckpt: int):
        """(d x_n / d rhs)^T gx for the solve recorded in tape."""
        torch = _torch()
        b = self._img(gx, "gx")
        tb, _, wv = self.unrolled_sizes(n_iter, ckpt, b)
        if tape.numel() < tb:
            raise SparsectError("tape is smaller than this solve needs")
        g = torch.empty((b, self.nn), dtype=self.dtype, device=self.device)
        ws = self._ws.get(("vjp", b))
        if ws is None or ws.numel() < wv:
            ws = torch.empty(max(wv, 1), dtype=torch.uint8, device=self.device)
            self._ws[("vjp", b)] = ws
        _check(lib().cg_unrolled_vjp(self._h, float(alpha), float(lam), float(sigma), self._p(tape),
                                     tape.numel(), self._p(gx), self._p(g), b, int(n_iter), int(ckpt),
                                     self._p(ws), ws.numel(), self._stream()))
        return g

    def pd(self, f, alpha: float, n_outer: int, n_cg: int, tau: float | None = None,
           sigma: float | None = None, mu0=None, out=None):
        """Chambolle-Pock TV (primal step eq:PD_resolve); tau = sigma = 0.99/sqrt(8)
        by default.  Returns mu."""
        torch = _torch()
        b = self._sino(f, "f")
        step = 0.99 / np.sqrt(8.0)
        tau = step if tau is None else tau
        sigma = step if sigma is None else sigma
        if out is not None:
            self._img_n(out, b, "out")
        if mu0 is not None:
            self._img_n(mu0, b, "mu0")
        flags = 0
        if mu0 is not None:
            flags |= SB_WARM
            mu = mu0.clone() if out is None else out.copy_(mu0)
        else:
            mu = torch.empty((b, self.nn), dtype=self.dtype, device=self.device) if out is None else out
        self._img_n(mu, b, "mu")
        P = PdParams(float(alpha), float(tau), float(sigma), int(n_outer), int(n_cg), flags, 0)
        ws, nb = self.workspace(WS_PD, b)
        _check(lib().chambolle_pock_tv(self._h, ctypes.byref(P), self._p(f), self._p(mu), b,
                                       self._p(ws), nb, self._stream()))
        return mu

    # -- host copies ------------------------------------------------------------
    def export_csr(self):
        rp = np.empty(self.rows + 1, dtype=np.int64)
        col = np.empty(self.info.nnz, dtype=np.int32)
        val = np.empty(self.info.nnz, dtype=np.float64)
        _check(lib().radon_export_csr(self._h, rp.ctypes.data_as(_vp), col.ctypes.data_as(_vp),
                                      val.ctypes.data_as(_vp)))
        return rp, col, val

    def export_adj(self):
        m = self.nn * self.n_meas
        b = np.empty(m, dtype=np.int32)
        v0 = np.empty(m, dtype=np.float64)
        v1 = np.empty(m, dtype=np.float64)
        _check(lib().radon_export_adj(self._h, b.ctypes.data_as(_vp), v0.ctypes.data_as(_vp),
                                      v1.ctypes.data_as(_vp)))
        return b, v0, v1


class RadonSurrogate:
    """The surrogate T of Section 3.2 built from a RadonOp's own products: the
    centre pixel's point-spread function cut to radius r and applied as a
    translated stencil (symmetric part, no wrap-around at the edges)."""

    def __init__(self, op: RadonOp, radius: int):
        torch = _torch()
        self.op, self.radius = op, int(radius)
        self.n, self.nn, self.dtype, self.device = op.n, op.nn, op.dtype, op.device
        h = _vp()
        with torch.cuda.device(op.device):
            _check(lib().radon_surrogate_create(op._h, self.radius, op._stream(), ctypes.byref(h)))
        self._h = h
        k = 2 * self.radius + 1
        w = np.zeros(k * k)
        _check(lib().radon_surrogate_weights(self._h, None, w.ctypes.data_as(_vp)))
        self.weights = w.reshape(k, k)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.radon_surrogate_destroy(h)
            self._h = None

    def apply(self, x, alpha: float = 1.0, lam: float = 0.0, sigma: float = 0.0, out=None,
              dot: bool = False):
        """alpha T x + lam K^T K x + sigma x (and <x, out> per image if dot)."""
        torch = _torch()
        b = self.op._img(x)
        o = torch.empty((b, self.nn), dtype=self.dtype, device=self.device) if out is None else out
        self.op._img_n(o, b, "out")
        d = torch.empty(b, dtype=torch.float64, device=self.device) if dot else None
        t = (self.n + 31) // 32
        nbytes = 8 * t * t * b if dot else 0
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
        _check(lib().surrogate_apply(self._h, float(alpha), float(lam), float(sigma),
                                     _vp(x.data_ptr()), _vp(o.data_ptr()),
                                     _vp(d.data_ptr()) if dot else None, b, _vp(ws.data_ptr()),
                                     nbytes, self.op._stream()))
        return (o, d) if dot else o


class RadonFourier:
    """The Fourier-domain operator of a RadonOp's geometry (Sections 2 and
    3.1): the gridded transforms F^* (image -> polar Fourier samples, one per
    measured angle and radial DFT frequency) and F, and the normal operator
    H = Re(F F^*) of eq:SBFFT, either through the precomputed B B^* of
    eq:fusedop (path "fused") or through the two transforms ("nufft").
    Fourier samples are real tensors [batch, P, 2] (re, im) of the operator's
    vector dtype."""

    PATHS = {"fused": FOURIER_FUSED, "nufft": FOURIER_NUFFT}

    def __init__(self, op: RadonOp, m_sp: int = 6, tau: float = 0.0, grid: int = 0):
        torch = _torch()
        self.op = op   # borrowed by the handle: keep it alive
        self.n, self.nn, self.dtype, self.device = op.n, op.nn, op.dtype, op.device
        h = _vp()
        with torch.cuda.device(op.device):
            _check(lib().radon_fourier_create(op._h, int(m_sp), float(tau), int(grid), op._stream(),
                                              ctypes.byref(h)))
        self._h = h
        info = FourierInfo()
        _check(lib().radon_fourier_get_info(self._h, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in FourierInfo._fields_}
        self.P, self.grid, self.m_sp, self.tau = info.n_points, info.grid, info.m_sp, info.tau
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.radon_fourier_destroy(h)
            self._h = None

    def _stream(self):
        return self.op._stream()

    def workspace(self, which: int, batch: int):
        torch = _torch()
        nbytes = lib().radon_fourier_workspace_bytes(self._h, which, batch)
        if nbytes < 0:
            _check(int(nbytes))
        buf = self._ws.get((which, batch))
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=self.device)
            self._ws[(which, batch)] = buf
        return buf, int(nbytes)

    def _samples(self, f, name="fhat"):
        torch = _torch()
        if not isinstance(f, torch.Tensor) or f.device != self.device or f.dtype != self.dtype:
            raise SparsectError(f"{name} must be a {self.dtype} tensor on {self.device}")
        if not f.is_contiguous() or f.numel() % (2 * self.P):
            raise SparsectError(f"{name} must be contiguous with a multiple of 2 P = {2 * self.P} elements")
        return f.numel() // (2 * self.P)

    def fwd(self, mu, out=None):
        """fhat = F^* mu (gridded), [batch, P, 2]."""
        torch = _torch()
        b = self.op._img(mu, "mu")
        o = torch.empty((b, self.P, 2), dtype=self.dtype, device=self.device) if out is None else out
        if self._samples(o, "out") != b:
            raise SparsectError(f"out holds {self._samples(o, 'out')} sample sets, the call needs {b}")
        ws, nb = self.workspace(FWS_TRANSFORM, b)
        _check(lib().fourier_fwd(self._h, _vp(mu.data_ptr()), _vp(o.data_ptr()), b, _vp(ws.data_ptr()),
                                 nb, self._stream()))
        return o

    def adj(self, fhat, alpha: float = 1.0, out=None):
        """x = alpha Re(F fhat) (gridded), [batch, n*n]."""
        torch = _torch()
        b = self._samples(fhat)
        o = torch.empty((b, self.nn), dtype=self.dtype, device=self.device) if out is None else out
        self.op._img_n(o, b, "out")
        ws, nb = self.workspace(FWS_TRANSFORM, b)
        _check(lib().fourier_adj(self._h, _vp(fhat.data_ptr()), _vp(o.data_ptr()), float(alpha), b,
                                 _vp(ws.data_ptr()), nb, self._stream()))
        return o

    def normal(self, x, alpha: float = 1.0, lam: float = 0.0, sigma: float = 0.0, path: str = "fused",
               out=None, dot: bool = False):
        """alpha H x + lam K^T K x + sigma x (and <x, out> per image if dot)."""
        torch = _torch()
        b = self.op._img(x)
        o = torch.empty((b, self.nn), dtype=self.dtype, device=self.device) if out is None else out
        self.op._img_n(o, b, "out")
        d = torch.empty(b, dtype=torch.float64, device=self.device) if dot else None
        ws, nb = self.workspace(FWS_TRANSFORM, b)
        _check(lib().fourier_normal(self._h, self.PATHS[path], float(alpha), float(lam), float(sigma),
                                    _vp(x.data_ptr()), _vp(o.data_ptr()),
                                    _vp(d.data_ptr()) if dot else None, b, _vp(ws.data_ptr()), nb,
                                    self._stream()))
        return (o, d) if dot else o

    def sb(self, fhat, alpha: float, lam: float, n_outer: int, n_cg: int, tol: float = 0.0,
           path: str = "fused", mu0=None, resume: bool = False, out=None):
        """Split Bregman TV on eq:SBFFT; returns (mu, info tensor of SbInfo bytes)."""
        torch = _torch()
        b = self._samples(fhat)
        if out is not None:
            self.op._img_n(out, b, "out")
        if mu0 is not None:
            self.op._img_n(mu0, b, "mu0")
        flags = 0
        if resume:
            flags |= SB_RESUME
            if out is None:
                raise SparsectError("resume needs out= (the image of the previous call)")
            mu = out
        elif mu0 is not None:
            flags |= SB_WARM
            mu = mu0.clone() if out is None else out.copy_(mu0)
        else:
            mu = torch.empty((b, self.nn), dtype=self.dtype, device=self.device) if out is None else out
        self.op._img_n(mu, b, "mu")
        P = SbParams(float(alpha), float(lam), float(tol), int(n_outer), int(n_cg), flags, 0)
        info = torch.zeros(b * ctypes.sizeof(SbInfo), dtype=torch.uint8, device=self.device)
        ws, nb = self.workspace(FWS_SB, b)
        _check(lib().split_bregman_tv_fourier(self._h, self.PATHS[path], ctypes.byref(P),
                                              _vp(fhat.data_ptr()), _vp(mu.data_ptr()), b,
                                              _vp(ws.data_ptr()), nb, _vp(info.data_ptr()), self._stream()))
        return mu, info


class RadonMulti:
    """A mixed batch: several RadonOps of different geometry (and one dtype
    kind) whose products and CG solves run as one launch per phase.  Weights
    alpha, lam, sigma (scalars or one per instance) fix each instance's normal
    operator.  Vectors are packed: instance i's image is
    packed[img_off[i] : img_off[i] + n_i**2].  storage="torch" keeps the
    group's device tables in a torch tensor (radon_multi_create_into), so the
    library allocates nothing for it."""

    def __init__(self, ops, alpha=1.0, lam=0.0, sigma=0.0, storage: str = "library"):
        torch = _torch()
        self.ops = list(ops)   # keeps the operators alive as long as the group
        k = len(self.ops)
        if k < 1:
            raise SparsectError("a group needs at least one operator")
        self.dtype, self.device = self.ops[0].dtype, self.ops[0].device

        def arr(v):
            a = np.broadcast_to(np.asarray(v, dtype=np.float64), (k,)).copy()
            return a

        if storage not in ("library", "torch"):
            raise SparsectError("storage must be 'library' or 'torch'")
        self.alpha, self.lam, self.sigma = arr(alpha), arr(lam), arr(sigma)
        handles = (_vp * k)(*[o._h for o in self.ops])
        h = _vp()
        self._tables = None
        with torch.cuda.device(self.device):
            if storage == "library":
                _check(lib().radon_multi_create(handles, k, self.alpha.ctypes.data_as(_vp),
                                                self.lam.ctypes.data_as(_vp),
                                                self.sigma.ctypes.data_as(_vp), ctypes.byref(h)))
            else:
                nb = ctypes.c_int64()
                _check(lib().radon_multi_table_bytes(handles, k, ctypes.byref(nb)))
                # 256-byte aligned: torch's caching allocator hands out 512-byte aligned blocks
                self._tables = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=self.device)
                _check(lib().radon_multi_create_into(handles, k, self.alpha.ctypes.data_as(_vp),
                                                     self.lam.ctypes.data_as(_vp),
                                                     self.sigma.ctypes.data_as(_vp),
                                                     _vp(self._tables.data_ptr()), int(nb.value),
                                                     ctypes.byref(h)))
        self._h = h
        self.img_off = np.zeros(k + 1, dtype=np.int64)
        self.sino_off = np.zeros(k + 1, dtype=np.int64)
        wp, wc, fw, aw = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().radon_multi_info(self._h, self.img_off.ctypes.data_as(_vp),
                                      self.sino_off.ctypes.data_as(_vp), ctypes.byref(wp),
                                      ctypes.byref(wc), ctypes.byref(fw), ctypes.byref(aw)))
        self.ws_products, self.ws_cg = int(wp.value), int(wc.value)
        self.fwd_waves, self.adj_waves = int(fw.value), int(aw.value)
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _torch().cuda.synchronize(self.device)
            except Exception:
                pass
            _lib.radon_multi_destroy(h)
            self._h = None

    def _stream(self):
        return _vp(_torch().cuda.current_stream(self.device).cuda_stream)

    def _buf(self, key, nbytes):
        torch = _torch()
        b = self._ws.get(key)
        if b is None or b.numel() < nbytes:
            b = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=self.device)
            self._ws[key] = b
        return b

    def empty_images(self):
        return _torch().zeros(int(self.img_off[-1]), dtype=self.dtype, device=self.device)

    def empty_sinograms(self):
        return _torch().zeros(int(self.sino_off[-1]), dtype=self.dtype, device=self.device)

    def pack_images(self, imgs):
        out = self.empty_images()
        for i, (o, x) in enumerate(zip(self.ops, imgs)):
            out[self.img_off[i]:self.img_off[i] + o.nn] = x.reshape(-1)
        return out

    def pack_sinograms(self, sinos):
        out = self.empty_sinograms()
        for i, (o, y) in enumerate(zip(self.ops, sinos)):
            out[self.sino_off[i]:self.sino_off[i] + o.rows] = y.reshape(-1)
        return out

    def image(self, packed, i):
        return packed[self.img_off[i]:self.img_off[i] + self.ops[i].nn]

    def sinogram(self, packed, i):
        return packed[self.sino_off[i]:self.sino_off[i] + self.ops[i].rows]

    def _check_vec(self, t, n, name):
        torch = _torch()
        if (not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != self.dtype
                or not t.is_contiguous() or t.numel() != n):
            raise SparsectError(f"{name} must be a contiguous {self.dtype} tensor of {n} elements "
                                f"on {self.device}")

    def apply(self, which: int, x, out=None):
        """0: packed images -> sinograms (M R); 1: sinograms -> images (R^T M^T);
        2: images -> images (A_i)."""
        ni, ns = int(self.img_off[-1]), int(self.sino_off[-1])
        self._check_vec(x, ns if which == 1 else ni, "input")
        if out is None:
            out = self.empty_sinograms() if which == 0 else self.empty_images()
        self._check_vec(out, ns if which == 0 else ni, "out")
        ws = self._buf("products", self.ws_products)
        _check(lib().radon_multi_apply(self._h, int(which), _vp(x.data_ptr()), _vp(out.data_ptr()),
                                       _vp(ws.data_ptr()), ws.numel(), self._stream()))
        return out

    def cg(self, rhs, n_iter: int = 10, rtol: float = 0.0, out=None):
        """CG on every instance from 0; returns (x, info tensor of CgInfo bytes)."""
        torch = _torch()
        ni = int(self.img_off[-1])
        self._check_vec(rhs, ni, "rhs")
        x = self.empty_images() if out is None else out
        self._check_vec(x, ni, "out")
        info = torch.zeros(len(self.ops) * ctypes.sizeof(CgInfo), dtype=torch.uint8, device=self.device)
        ws = self._buf("cg", self.ws_cg)
        _check(lib().radon_multi_cg(self._h, _vp(rhs.data_ptr()), _vp(x.data_ptr()), int(n_iter),
                                    float(rtol), _vp(ws.data_ptr()), ws.numel(), _vp(info.data_ptr()),
                                    self._stream()))
        return x, info

    def cg_graph(self, n_iter: int = 10, rtol: float = 0.0) -> "MultiCgGraph":
        """Capture a CG solve into a HIP graph over buffers it owns (see MultiCgGraph)."""
        return MultiCgGraph(self, n_iter, rtol)


class SbGraph:
    """A captured split_bregman_tv of one operator: each launch() runs the
    whole n_outer x n_cg solve from 0 on the data in .f into .mu and .info.
    The graph owns (keeps alive) its buffers."""

    def __init__(self, op: RadonOp, f, alpha: float, lam: float, n_outer: int, n_cg: int,
                 tol: float = 0.0):
        torch = _torch()
        self.op = op
        b = op._sino(f, "f")
        self.f = f.clone()
        self.mu = torch.empty((b, op.nn), dtype=op.dtype, device=op.device)
        self.info = torch.zeros(b * ctypes.sizeof(SbInfo), dtype=torch.uint8, device=op.device)
        nbytes = lib().radon_workspace_bytes(op._h, WS_SB, b)
        if nbytes < 0:
            _check(int(nbytes))
        self.ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=op.device)
        P = SbParams(float(alpha), float(lam), float(tol), int(n_outer), int(n_cg), 0, 0)
        torch.cuda.synchronize(op.device)
        h = _vp()
        with torch.cuda.device(op.device):
            _check(lib().split_bregman_tv_graph(op._h, ctypes.byref(P), _vp(self.f.data_ptr()),
                                                _vp(self.mu.data_ptr()), b, _vp(self.ws.data_ptr()),
                                                int(nbytes), _vp(self.info.data_ptr()), ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().radon_graph_launch(self._h, self.op._stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _torch().cuda.synchronize(self.op.device)
            except Exception:
                pass
            _lib.radon_graph_destroy(h)
            self._h = None


class MultiCgGraph:
    """A captured radon_multi_cg: write the packed right-hand sides into
    .rhs, call launch(), read .x and .info.  The graph keeps its buffers."""

    def __init__(self, group: RadonMulti, n_iter: int, rtol: float):
        torch = _torch()
        self.group = group
        self.rhs = group.empty_images()
        self.x = group.empty_images()
        self.info = torch.zeros(len(group.ops) * ctypes.sizeof(CgInfo), dtype=torch.uint8,
                                device=group.device)
        self.ws = torch.empty(max(group.ws_cg, 1), dtype=torch.uint8, device=group.device)
        torch.cuda.synchronize(group.device)
        h = _vp()
        with torch.cuda.device(group.device):
            _check(lib().radon_multi_cg_graph(group._h, _vp(self.rhs.data_ptr()),
                                              _vp(self.x.data_ptr()), int(n_iter), float(rtol),
                                              _vp(self.ws.data_ptr()), self.ws.numel(),
                                              _vp(self.info.data_ptr()), ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().radon_graph_launch(self._h, self.group._stream()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _torch().cuda.synchronize(self.group.device)
            except Exception:
                pass
            _lib.radon_graph_destroy(h)
            self._h = None


PROBE_COPY, PROBE_READ = 0, 1


def bandwidth_probe(mode: int, src, dst, nbytes: int | None = None) -> None:
    """radon_bandwidth_probe on the current stream: PROBE_COPY copies src into
    dst, PROBE_READ streams src once (dst: >= 4096 uint32 of results)."""
    torch = _torch()
    n = src.numel() * src.element_size() if nbytes is None else int(nbytes)
    _check(lib().radon_bandwidth_probe(int(mode), _vp(src.data_ptr()), _vp(dst.data_ptr()), n,
                                       _vp(torch.cuda.current_stream(src.device).cuda_stream)))


def decode_cg_info(info) -> list[dict]:
    raw = info.cpu().numpy().tobytes()
    n = len(raw) // ctypes.sizeof(CgInfo)
    arr = (CgInfo * n).from_buffer_copy(raw)
    return [dict(iterations=a.iterations, breakdown=a.breakdown, rho0=a.rho0, rho=a.rho) for a in arr]


def decode_sb_info(info) -> list[dict]:
    raw = info.cpu().numpy().tobytes()
    n = len(raw) // ctypes.sizeof(SbInfo)
    arr = (SbInfo * n).from_buffer_copy(raw)
    return [dict(outer=a.outer, breakdowns=a.breakdowns, upd_b_first=a.upd_b_first, upd_b=a.upd_b,
                 upd_u=a.upd_u) for a in arr]
