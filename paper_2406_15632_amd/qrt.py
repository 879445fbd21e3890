"""Python binding of libqrt (include/qrt.h): argument marshalling only.

Every function of the C ABI is exposed under its own name (qrt_create,
qrt_run, ...) on the loaded library; the Context class below wraps a context
with numpy / torch conveniences.  All transport work runs in the HIP kernels of
libqrt.so: this module never computes any part of the method, and it raises
if the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libqrt.so")

QRT_OK, QRT_INVALID_ARG, QRT_BAD_STATE, QRT_HIP_ERROR = 0, -1, -2, -3
QRT_OUT_OF_MEMORY, QRT_UNSUPPORTED, QRT_NOT_TRAINED = -4, -5, -6
SOBOL, HALTON, NIEDERREITER2, HAMMERSLEY, PHILOX, FAURE, SOBOL_OWEN = 0, 1, 2, 3, 4, 5, 6
GRID_HOST_COPY, GRID_DEVICE_COPY, GRID_DEVICE_BORROW = 0, 1, 2
FP32, FP64 = 0, 1
PEEL_EXACT, PEEL_SURROGATE = 0, 1
EMIT_DIRECT, EMIT_INVERSE = 0, 1
MAX_DIMS, MAX_OBSERVERS = 128, 16
MLP_PARAMS = 12929
BATCH_MAX_OBSERVERS, BATCH_MAX_SCENES = 4, 1024
SOURCE_POINT, SOURCE_SPHERE = 0, 1


class qrt_counters(C.Structure):
    _fields_ = [(f, C.c_int64) for f in ("packets", "visits", "peels", "peel_rays", "escapes", "tau_cuts",
                                         "scatterings", "occluded", "surrogate", "fallbacks", "visits_first")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


TIMING_CLASSES = ("sort", "first", "scatter", "walk", "peel_mlp", "other")


class qrt_timing(C.Structure):
    _fields_ = [("ms", C.c_double * len(TIMING_CLASSES)), ("launches", C.c_int64 * len(TIMING_CLASSES))]


class qrt_train_cfg(C.Structure):
    _fields_ = [("steps", C.c_int64), ("batch", C.c_int32), ("init", C.c_int32),
                ("lr", C.c_float), ("lr_final", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("tau_cap", C.c_float), ("weight_floor", C.c_float), ("seed", C.c_uint64)]


class qrt_train_report(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_final", C.c_double), ("steps", C.c_int64)]


class qrt_mask_report(C.Structure):
    _fields_ = [("cells", C.c_int64), ("valid_cells", C.c_int64), ("samples", C.c_int64),
                ("samples_valid", C.c_int64), ("max_err_valid", C.c_double)]


class qrt_batch_scene(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("kappa_rho", C.c_void_p),
                ("source", C.c_int), ("emit_order", C.c_int), ("src", C.c_double * 3), ("radius", C.c_double),
                ("albedo", C.c_double), ("g", C.c_double), ("p_lin", C.c_double),
                ("n_obs", C.c_int), ("theta", C.c_double * BATCH_MAX_OBSERVERS),
                ("phi", C.c_double * BATCH_MAX_OBSERVERS), ("npix", C.c_int), ("half_width", C.c_double),
                ("max_orders", C.c_int), ("tau_min", C.c_double),
                ("first", C.c_uint64), ("count", C.c_uint64), ("n_total", C.c_uint64)]


def _as_dict(st):
    return {f: getattr(st, f) for f, _ in st._fields_}


_P = C.c_void_p
_D3 = C.POINTER(C.c_double)
# exported symbol -> (restype, argtypes); the C-ABI surface checked by the tests
SIGNATURES = {
    "qrt_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, _P]),
    "qrt_destroy": (None, [_P]),
    "qrt_last_error": (C.c_char_p, [_P]),
    "qrt_set_stream": (C.c_int, [_P, _P]),
    "qrt_set_grid": (C.c_int, [_P, C.c_int, C.c_int, C.c_int, _D3, _D3, _P, C.c_int]),
    "qrt_set_point_source": (C.c_int, [_P, C.c_double, C.c_double, C.c_double]),
    "qrt_set_sphere_source": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int]),
    "qrt_set_dust": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_double]),
    "qrt_set_observers": (C.c_int, [_P, C.c_int, _D3, _D3, C.c_int, C.c_double]),
    "qrt_set_sequence": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_uint64]),
    "qrt_set_transport": (C.c_int, [_P, C.c_int, C.c_double, C.c_int, C.c_int]),
    "qrt_run": (C.c_int, [_P, C.c_uint64, C.c_uint64]),
    "qrt_run_static": (C.c_int, [_P, C.c_uint64, C.c_uint64]),
    "qrt_set_overlap": (C.c_int, [_P, C.c_int]),
    "qrt_set_tail": (C.c_int, [_P, C.c_int, C.c_uint64]),
    "qrt_join": (C.c_int, [_P]),
    "qrt_read_images": (C.c_int, [_P, C.c_int, _P, _P, _P, C.c_int]),
    "qrt_image_device_ptr": (C.c_int, [_P, C.POINTER(C.c_void_p)]),
    "qrt_reset_images": (C.c_int, [_P]),
    "qrt_set_order_images": (C.c_int, [_P, C.c_int]),
    "qrt_read_order_images": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, C.c_int]),
    "qrt_get_counters": (C.c_int, [_P, C.POINTER(qrt_counters)]),
    "qrt_set_timing": (C.c_int, [_P, C.c_int]),
    "qrt_get_timing": (C.c_int, [_P, C.POINTER(qrt_timing), C.c_int]),
    "qrt_generate_points": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_int,
                                      _P, C.c_int]),
    "qrt_trace_tau": (C.c_int, [_P, C.c_int64, _P, _P, _P, _P]),
    "qrt_mlp_set_params": (C.c_int, [_P, _P, C.c_int64]),
    "qrt_mlp_get_params": (C.c_int, [_P, _P, C.c_int64]),
    "qrt_mlp_init": (C.c_int, [_P, C.c_uint64]),
    "qrt_mlp_forward": (C.c_int, [_P, C.c_int64, _P, _P]),
    "qrt_mlp_backward": (C.c_int, [_P, C.c_int64, _P, _P, _P]),
    "qrt_surrogate_set_domain": (C.c_int, [_P, _D3, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                           C.c_int, C.c_int]),
    "qrt_surrogate_set_mask": (C.c_int, [_P, _P]),
    "qrt_surrogate_get_mask": (C.c_int, [_P, _P]),
    "qrt_surrogate_inputs": (C.c_int, [_P, C.c_int64, _P, _P]),
    "qrt_surrogate_sample": (C.c_int, [_P, C.c_int64, C.c_uint64, _P, _P, C.POINTER(C.c_int64)]),
    "qrt_surrogate_train": (C.c_int, [_P, C.c_int64, _P, _P, C.POINTER(qrt_train_cfg),
                                      C.POINTER(qrt_train_report)]),
    "qrt_surrogate_validate": (C.c_int, [_P, C.c_int64, _P, _P, C.c_double, C.c_double, C.c_int64,
                                         C.POINTER(qrt_mask_report)]),
    "qrt_surrogate_get_state": (C.c_int, [_P, _P, C.POINTER(C.c_size_t)]),
    "qrt_surrogate_set_state": (C.c_int, [_P, _P, C.c_size_t]),
    "qrt_batch_set": (C.c_int, [_P, C.c_int, C.POINTER(qrt_batch_scene)]),
    "qrt_batch_run": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_int]),
    "qrt_batch_read_images": (C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, C.c_int]),
    "qrt_batch_reset": (C.c_int, [_P]),
}

_lib: Optional[C.CDLL] = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libqrt.so; raises if it is missing (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with `python -m paper_2406_15632_amd.build`")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7);
    # loading torch first makes libqrt bind to that one, so one process never
    # holds two HIP runtimes and device pointers/streams from torch are valid here
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class QRTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libqrt error {code}: {msg}")
        self.code = code


def _d3(v: Sequence[float]):
    return (C.c_double * 3)(*[float(x) for x in v])


def _current_stream_handle() -> int:
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


class Context:
    """One library context on one device and stream."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self.lib = load()
        if stream is None:
            stream = _current_stream_handle()
        h = C.c_void_p()
        rc = self.lib.qrt_create(C.byref(h), device, C.c_void_p(stream))
        if rc != QRT_OK:
            raise QRTError(rc, "qrt_create failed")
        self.h = h

    def _ck(self, rc: int):
        if rc != QRT_OK:
            raise QRTError(rc, self.lib.qrt_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.qrt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -------- configuration
    def set_stream(self, stream: int):
        self._ck(self.lib.qrt_set_stream(self.h, C.c_void_p(stream)))

    def set_grid(self, kappa_rho, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0)):
        """kappa_rho: float32 [nz][ny][nx], a numpy array or a CUDA torch tensor (copied into the library's order)."""
        nz, ny, nx = kappa_rho.shape
        if isinstance(kappa_rho, np.ndarray):
            a = np.ascontiguousarray(kappa_rho, dtype=np.float32)
            self._ck(self.lib.qrt_set_grid(self.h, nx, ny, nz, _d3(lo), _d3(hi), a.ctypes.data, GRID_HOST_COPY))
        else:
            import torch
            t = kappa_rho
            if t.dtype != torch.float32 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("device grid must be a contiguous float32 CUDA tensor")
            self._ck(self.lib.qrt_set_grid(self.h, nx, ny, nz, _d3(lo), _d3(hi), C.c_void_p(t.data_ptr()),
                                           GRID_DEVICE_COPY))

    def set_point_source(self, x=0.0, y=0.0, z=0.0):
        self._ck(self.lib.qrt_set_point_source(self.h, x, y, z))

    def set_sphere_source(self, x, y, z, radius, order=EMIT_DIRECT):
        self._ck(self.lib.qrt_set_sphere_source(self.h, x, y, z, radius, order))

    def set_dust(self, albedo, g, p_lin, p_circ=0.0):
        self._ck(self.lib.qrt_set_dust(self.h, albedo, g, p_lin, p_circ))

    def set_observers(self, observers: Sequence[Tuple[float, float]], npix: int, half_width: float):
        th = (C.c_double * len(observers))(*[o[0] for o in observers])
        ph = (C.c_double * len(observers))(*[o[1] for o in observers])
        self._ck(self.lib.qrt_set_observers(self.h, len(observers), th, ph, npix, half_width))
        self.n_obs, self.npix = len(observers), npix

    def set_sequence(self, kind: int, seed: int = 0, n_total: int = 0):
        self._ck(self.lib.qrt_set_sequence(self.h, kind, seed, n_total))

    def set_transport(self, max_orders: int, tau_min: float = 1e-8, precision: int = FP32,
                      peel_mode: int = PEEL_EXACT):
        self._ck(self.lib.qrt_set_transport(self.h, max_orders, tau_min, precision, peel_mode))

    def set_scene(self, sc, kind: int = SOBOL, seed: int = 0, n_total: Optional[int] = None, grid=None,
                  precision: Optional[int] = None):
        """Configure everything from a synth.Scene (grid may be a device tensor holding its mesh)."""
        self.set_grid(sc.kappa_rho if grid is None else grid, sc.lo, sc.hi)
        if sc.source_kind == 1:
            self.set_sphere_source(*sc.source, sc.r_star, getattr(sc, "emit_order", EMIT_DIRECT))
        else:
            self.set_point_source(*sc.source)
        self.set_dust(sc.albedo, sc.g, sc.p_lin)
        self.set_observers(sc.observers, sc.npix, sc.half_width)
        self.set_sequence(kind, seed, sc.n_packets if n_total is None else n_total)
        prec = (FP64 if sc.fp64 else FP32) if precision is None else precision
        self.set_transport(sc.max_orders, sc.tau_min, prec)

    # -------- work
    def run(self, first: int, count: int):
        self._ck(self.lib.qrt_run(self.h, first, count))

    def set_overlap(self, enable: bool):
        """Overlapped runs on three internal streams (see qrt_set_overlap)."""
        self._ck(self.lib.qrt_set_overlap(self.h, int(enable)))

    def set_tail(self, first_order: int, max_deferred: int = 0):
        """Late orders in one launch from first_order on (0: off; see qrt_set_tail)."""
        self._ck(self.lib.qrt_set_tail(self.h, int(first_order), int(max_deferred)))

    def join(self):
        """The context stream waits for the overlapped runs still pending."""
        self._ck(self.lib.qrt_join(self.h))

    def run_static(self, first: int, count: int):
        """qrt_run on the device's static scratch (no allocation)."""
        self._ck(self.lib.qrt_run_static(self.h, first, count))

    def reset_images(self):
        self._ck(self.lib.qrt_reset_images(self.h))

    def read_images(self, normalized: bool = True) -> np.ndarray:
        """[n_obs][3][npix][npix] float64 (I, Q, U)."""
        out = np.zeros((self.n_obs, 3, self.npix, self.npix), dtype=np.float64)
        for o in range(self.n_obs):
            self._ck(self.lib.qrt_read_images(self.h, o, out[o, 0].ctypes.data, out[o, 1].ctypes.data,
                                              out[o, 2].ctypes.data, int(normalized)))
        return out

    def set_order_images(self, enable: bool):
        self._ck(self.lib.qrt_set_order_images(self.h, int(enable)))

    def read_order_images(self, order: int, normalized: bool = True) -> np.ndarray:
        """[n_obs][3][npix][npix] float64 of one scattering order (1-based)."""
        out = np.zeros((self.n_obs, 3, self.npix, self.npix), dtype=np.float64)
        for o in range(self.n_obs):
            self._ck(self.lib.qrt_read_order_images(self.h, o, order, out[o, 0].ctypes.data, out[o, 1].ctypes.data,
                                                    out[o, 2].ctypes.data, int(normalized)))
        return out

    def image_device_ptr(self) -> int:
        p = C.c_void_p()
        self._ck(self.lib.qrt_image_device_ptr(self.h, C.byref(p)))
        return int(p.value or 0)

    def counters(self) -> dict:
        c = qrt_counters()
        self._ck(self.lib.qrt_get_counters(self.h, C.byref(c)))
        return c.as_dict()

    def set_timing(self, enable: bool):
        self._ck(self.lib.qrt_set_timing(self.h, int(enable)))

    def timing(self, reset: bool = True) -> dict:
        """{class: (summed ms, launches)} of the kernels timed since the last reset."""
        t = qrt_timing()
        self._ck(self.lib.qrt_get_timing(self.h, C.byref(t), int(reset)))
        return {k: (float(t.ms[i]), int(t.launches[i])) for i, k in enumerate(TIMING_CLASSES)}

    def generate_points(self, kind: int, first: int, count: int, dims: int, seed: int = 0,
                        n_total: int = 0) -> np.ndarray:
        out = np.zeros((count, dims), dtype=np.uint32)
        self._ck(self.lib.qrt_generate_points(self.h, kind, seed, n_total, first, count, dims,
                                              out.ctypes.data, 0))
        return out

    def generate_points_device(self, kind: int, first: int, count: int, dims: int, out_tensor, seed: int = 0,
                               n_total: int = 0):
        self._ck(self.lib.qrt_generate_points(self.h, kind, seed, n_total, first, count, dims,
                                              C.c_void_p(out_tensor.data_ptr()), 1))

    def trace_tau(self, p_dev, k_dev, tau_dev, visits_dev=None):
        n = p_dev.shape[0]
        self._ck(self.lib.qrt_trace_tau(self.h, n, C.c_void_p(p_dev.data_ptr()), C.c_void_p(k_dev.data_ptr()),
                                        C.c_void_p(tau_dev.data_ptr()),
                                        C.c_void_p(visits_dev.data_ptr()) if visits_dev is not None else None))

    # -------- surrogate peel-off (network inputs, samples and outputs are CUDA tensors)
    def mlp_set_params(self, params: np.ndarray):
        a = np.ascontiguousarray(params, dtype=np.float32)
        self._ck(self.lib.qrt_mlp_set_params(self.h, a.ctypes.data, a.size))

    def mlp_get_params(self) -> np.ndarray:
        a = np.zeros(MLP_PARAMS, dtype=np.float32)
        self._ck(self.lib.qrt_mlp_get_params(self.h, a.ctypes.data, a.size))
        return a

    def mlp_init(self, seed: int):
        self._ck(self.lib.qrt_mlp_init(self.h, seed))

    def mlp_forward(self, X, y):
        self._ck(self.lib.qrt_mlp_forward(self.h, X.shape[0], C.c_void_p(X.data_ptr()), C.c_void_p(y.data_ptr())))

    def mlp_backward(self, X, dy, grad):
        self._ck(self.lib.qrt_mlp_backward(self.h, X.shape[0], C.c_void_p(X.data_ptr()), C.c_void_p(dy.data_ptr()),
                                           C.c_void_p(grad.data_ptr())))

    def surrogate_set_domain(self, center, r_in, r_out, h0, beta, zmax_over_h, n_r, n_z):
        self.dom_shape = (n_r, n_z)
        self._ck(self.lib.qrt_surrogate_set_domain(self.h, _d3(center), r_in, r_out, h0, beta, zmax_over_h,
                                                   n_r, n_z))

    def surrogate_set_mask(self, mask: np.ndarray):
        a = np.ascontiguousarray(mask, dtype=np.uint8)
        self._ck(self.lib.qrt_surrogate_set_mask(self.h, a.ctypes.data))

    def surrogate_get_mask(self) -> np.ndarray:
        a = np.zeros((self.n_obs,) + tuple(self.dom_shape), dtype=np.uint8)
        self._ck(self.lib.qrt_surrogate_get_mask(self.h, a.ctypes.data))
        return a

    def surrogate_inputs(self, pos_obs, X):
        self._ck(self.lib.qrt_surrogate_inputs(self.h, pos_obs.shape[0], C.c_void_p(pos_obs.data_ptr()),
                                               C.c_void_p(X.data_ptr())))

    def surrogate_sample(self, pos_obs, tau, seed: int) -> int:
        n = C.c_int64(0)
        self._ck(self.lib.qrt_surrogate_sample(self.h, pos_obs.shape[0], seed, C.c_void_p(pos_obs.data_ptr()),
                                               C.c_void_p(tau.data_ptr()), C.byref(n)))
        return int(n.value)

    def surrogate_train(self, pos_obs, tau, steps: int, batch: int = 8192, lr: float = 2e-3,
                        lr_final: float = 5e-5, init: bool = True, seed: int = 1, tau_cap: float = 12.0,
                        weight_floor: float = 0.02, beta1: float = 0.9, beta2: float = 0.999,
                        eps: float = 1e-8) -> dict:
        cfg = qrt_train_cfg(steps=steps, batch=batch, init=int(init), lr=lr, lr_final=lr_final, beta1=beta1,
                            beta2=beta2, eps=eps, tau_cap=tau_cap, weight_floor=weight_floor, seed=seed)
        rep = qrt_train_report()
        self._ck(self.lib.qrt_surrogate_train(self.h, pos_obs.shape[0], C.c_void_p(pos_obs.data_ptr()),
                                              C.c_void_p(tau.data_ptr()), C.byref(cfg), C.byref(rep)))
        return _as_dict(rep)

    def surrogate_validate(self, pos_obs, tau, max_err: float = 0.02, floor_frac: float = 0.0,
                           min_count: int = 16) -> dict:
        rep = qrt_mask_report()
        self._ck(self.lib.qrt_surrogate_validate(self.h, pos_obs.shape[0], C.c_void_p(pos_obs.data_ptr()),
                                                 C.c_void_p(tau.data_ptr()), max_err, floor_frac, min_count,
                                                 C.byref(rep)))
        return _as_dict(rep)

    def surrogate_get_state(self) -> bytes:
        n = C.c_size_t(0)
        self._ck(self.lib.qrt_surrogate_get_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._ck(self.lib.qrt_surrogate_get_state(self.h, buf, C.byref(n)))
        return buf.raw[: n.value]

    def surrogate_set_state(self, blob: bytes):
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self._ck(self.lib.qrt_surrogate_set_state(self.h, buf, len(blob)))
        self.dom_shape = tuple(np.frombuffer(bytes(blob)[16:24], dtype=np.int32))   # header: n_r, n_z

    # -------- batches of scenes
    def batch_set(self, scenes, firsts: Optional[Sequence[int]] = None, counts: Optional[Sequence[int]] = None,
                  n_totals: Optional[Sequence[int]] = None):
        """Set a batch from synth.Scene objects: scene i runs point indices
        firsts[i] .. firsts[i]+counts[i]-1 (defaults: 1 and its n_packets);
        Hammersley's N is n_totals[i] (default: its n_packets)."""
        n = len(scenes)
        arr = (qrt_batch_scene * n)()
        keep = []
        for i, sc in enumerate(scenes):
            kr = np.ascontiguousarray(sc.kappa_rho, dtype=np.float32)
            keep.append(kr)
            d = arr[i]
            d.nx, d.ny, d.nz = sc.n
            d.lo = (C.c_double * 3)(*sc.lo)
            d.hi = (C.c_double * 3)(*sc.hi)
            d.kappa_rho = kr.ctypes.data
            d.source = SOURCE_SPHERE if sc.source_kind == 1 else SOURCE_POINT
            d.emit_order = getattr(sc, "emit_order", EMIT_DIRECT)
            d.src = (C.c_double * 3)(*sc.source)
            d.radius = sc.r_star
            d.albedo, d.g, d.p_lin = sc.albedo, sc.g, sc.p_lin
            d.n_obs = len(sc.observers)
            if d.n_obs > BATCH_MAX_OBSERVERS:
                raise ValueError(f"scene {i}: at most {BATCH_MAX_OBSERVERS} observers in a batch")
            for o, (th, ph) in enumerate(sc.observers):
                d.theta[o], d.phi[o] = th, ph
            d.npix, d.half_width = sc.npix, sc.half_width
            d.max_orders, d.tau_min = sc.max_orders, sc.tau_min
            d.first = 1 if firsts is None else int(firsts[i])
            d.count = sc.n_packets if counts is None else int(counts[i])
            d.n_total = sc.n_packets if n_totals is None else int(n_totals[i])
        self._ck(self.lib.qrt_batch_set(self.h, n, arr))
        self.batch_shapes = [(len(sc.observers), sc.npix) for sc in scenes]

    def batch_run(self, kind: int = SOBOL, seed: int = 0, precision: int = FP32):
        self._ck(self.lib.qrt_batch_run(self.h, kind, seed, precision))

    def batch_read_images(self, scene: int, normalized: bool = True) -> np.ndarray:
        """[n_obs][3][npix][npix] float64 (I, Q, U) of one scene of the batch."""
        if not 0 <= scene < len(getattr(self, "batch_shapes", [])):
            self._ck(self.lib.qrt_batch_read_images(self.h, scene, 0, None, None, None, 0))   # the library refuses
        n_obs, npix = self.batch_shapes[scene]
        out = np.zeros((n_obs, 3, npix, npix), dtype=np.float64)
        for o in range(n_obs):
            self._ck(self.lib.qrt_batch_read_images(self.h, scene, o, out[o, 0].ctypes.data, out[o, 1].ctypes.data,
                                                    out[o, 2].ctypes.data, int(normalized)))
        return out

    def batch_reset(self):
        self._ck(self.lib.qrt_batch_reset(self.h))
