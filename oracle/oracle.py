"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg use this
module.  It builds qrt_oracle.c with gcc (no fast-math, no FMA contraction) and
marshals scenes from the synth package into the oracle's own structures.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from . import tables

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "qrt_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle.so")

SOBOL, HALTON, NIEDERREITER2, HAMMERSLEY, PHILOX, FAURE, SOBOL_OWEN = 0, 1, 2, 3, 4, 5, 6


# Sanitizer builds of the same source (the checker checked): "asan" adds
# AddressSanitizer and UndefinedBehaviorSanitizer (every UB report aborts), "tsan"
# ThreadSanitizer for the OpenMP packet loop.  The TSan build uses LLVM's clang
# and OpenMP runtime, whose Archer tool tells TSan about OpenMP's barriers (GCC's
# libgomp is not instrumented, so TSan would report its joins as races).
# QRT_ORACLE_VARIANT selects which build lib() loads; the process must then
# preload the matching sanitizer runtime.
LLVM_BIN = "/opt/rocm/llvm/bin"
VARIANT_FLAGS = {
    "": ["gcc", "-O2"],
    "asan": ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"],
    "tsan": [os.path.join(LLVM_BIN, "clang"), "-O1", "-g", "-fsanitize=thread"],
}


def lib_path(variant: str = "") -> str:
    return LIB if not variant else os.path.join(HERE, "_build", f"liboracle_{variant}.so")


def build(force: bool = True, variant: str = "") -> str:
    path = lib_path(variant)
    os.makedirs(os.path.dirname(path), exist_ok=True)
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
        tmp = path + ".tmp"
        cmd = [*VARIANT_FLAGS[variant], "-std=gnu11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, path)
    return path


class _Scene(C.Structure):
    _fields_ = [
        ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
        ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("kr", C.POINTER(C.c_float)),
        ("src_kind", C.c_int64), ("src", C.c_double * 3), ("r_star", C.c_double),
        ("albedo", C.c_double), ("g", C.c_double), ("p_lin", C.c_double),
        ("n_obs", C.c_int64), ("npix", C.c_int64),
        ("obs_theta", C.POINTER(C.c_double)), ("obs_phi", C.POINTER(C.c_double)),
        ("half_width", C.c_double),
        ("seq_kind", C.c_int64), ("dims", C.c_int64),
        ("mat", C.POINTER(C.c_uint32)), ("bases", C.POINTER(C.c_uint32)),
        ("seed", C.c_uint64), ("n_total", C.c_uint64),
        ("max_orders", C.c_int64), ("tau_min", C.c_double),
        ("peel_mode", C.c_int64), ("mlp", C.POINTER(C.c_float)),
        ("dom_center", C.c_double * 3),
        ("dom_r_in", C.c_double), ("dom_r_out", C.c_double), ("dom_h0", C.c_double),
        ("dom_beta", C.c_double), ("dom_zmax", C.c_double),
        ("dom_nr", C.c_int64), ("dom_nz", C.c_int64),
        ("dom_valid", C.POINTER(C.c_uint8)),
        ("emit_order", C.c_int64),
        ("order_images", C.c_int64),
    ]


class Counters(C.Structure):
    _fields_ = [(f, C.c_int64) for f in ("packets", "visits", "peels", "peel_rays", "escapes",
                                         "tau_cuts", "scatterings", "occluded")] + \
               [(f, C.c_double) for f in ("e_direct", "e_absorbed", "e_escaped", "e_remaining")] + \
               [(f, C.c_int64) for f in ("surrogate", "fallbacks", "visits_first")]

    def as_dict(self) -> Dict[str, float]:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        path = build(force=False, variant=os.environ.get("QRT_ORACLE_VARIANT", ""))
        L = C.CDLL(path)
        L.oracle_points.argtypes = [C.c_int64, C.c_int64, C.c_void_p, C.c_void_p, C.c_uint64,
                                    C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p]
        L.oracle_tau_ray.argtypes = [C.POINTER(_Scene), C.c_void_p, C.c_void_p, C.POINTER(C.c_int64)]
        L.oracle_tau_ray.restype = C.c_double
        L.oracle_move.argtypes = [C.POINTER(_Scene), C.c_void_p, C.c_void_p, C.c_double, C.c_void_p,
                                  C.POINTER(C.c_int64)]
        L.oracle_hg_cos.argtypes = [C.c_double, C.c_double]
        L.oracle_hg_cos.restype = C.c_double
        L.oracle_run.argtypes = [C.POINTER(_Scene), C.c_uint64, C.c_uint64, C.c_void_p,
                                 C.POINTER(Counters), C.c_int64, C.c_void_p, C.c_int64,
                                 C.POINTER(C.c_int64)]
        L.oracle_max_threads.restype = C.c_int
        L.oracle_emit.argtypes = [C.POINTER(_Scene), C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p]
        L.oracle_quad_flux.argtypes = [C.POINTER(_Scene), C.c_int64, C.c_int64, C.c_int64, C.c_int64]
        L.oracle_quad_flux.restype = C.c_double
        L.oracle_quad_pixels.argtypes = [C.POINTER(_Scene), C.c_int64, C.c_int64, C.c_int64, C.c_void_p]
        L.oracle_mlp_batch.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.oracle_mlp_tau.argtypes = [C.POINTER(_Scene), C.c_void_p, C.c_int64]
        L.oracle_mlp_tau.restype = C.c_double
        L.oracle_dom_cells.argtypes = [C.POINTER(_Scene), C.c_int64, C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def seq_tables(kind: int, dims: int) -> Tuple[np.ndarray, np.ndarray]:
    """(matrix columns [dims][32], bases [dims]) for a sequence kind."""
    mat = np.zeros((max(dims, 1), 32), dtype=np.uint32)
    bases = np.zeros(max(dims, 1), dtype=np.uint32)
    if kind in (SOBOL, SOBOL_OWEN):
        mat = tables.sobol_columns(dims)
    elif kind == NIEDERREITER2:
        mat = tables.niederreiter_columns(dims)
    elif kind in (HALTON, HAMMERSLEY):
        bases = tables.primes(dims)
    elif kind == FAURE:
        b, m, C = tables.faure_matrices(max(dims, 1))
        mat = C.reshape(-1)
        bases = np.array([b, m], dtype=np.uint32)
    return np.ascontiguousarray(mat), np.ascontiguousarray(bases)


def points(kind: int, dims: int, first: int, count: int, seed: int = 0, n_total: int = 0) -> np.ndarray:
    """uint32 [count][dims]: 0.32 fixed-point coordinates of points first..first+count-1."""
    if kind == HAMMERSLEY and n_total < first + count - 1:
        raise ValueError("Hammersley needs n_total >= last index")
    mat, bases = seq_tables(kind, dims)
    out = np.zeros((count, dims), dtype=np.uint32)
    rc = lib().oracle_points(kind, dims, mat.ctypes.data, bases.ctypes.data, seed, n_total,
                             first, count, out.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_points failed")
    return out


class Surrogate:
    """Surrogate peel-off set-up: FP32 network parameters (layout of
    oracle/mlp.py), the cylindrical domain and its validity mask
    [n_obs][n_r][n_z] (1 = network allowed)."""

    def __init__(self, params, center, r_in, r_out, h0, beta, zmax_over_h, valid):
        self.params = np.ascontiguousarray(params, dtype=np.float32)
        self.center = tuple(float(c) for c in center)
        self.r_in, self.r_out, self.h0, self.beta, self.zmax = map(float, (r_in, r_out, h0, beta, zmax_over_h))
        self.valid = np.ascontiguousarray(valid, dtype=np.uint8)
        assert self.valid.ndim == 3


class OracleScene:
    """Keeps the numpy buffers alive behind a _Scene structure."""

    def __init__(self, sc, kind: int = SOBOL, seed: int = 0, n_total: Optional[int] = None,
                 surrogate: Optional[Surrogate] = None):
        self.sc = sc
        self.kr = np.ascontiguousarray(sc.kappa_rho, dtype=np.float32)
        th = np.array([o[0] for o in sc.observers] or [0.0], dtype=np.float64)
        ph = np.array([o[1] for o in sc.observers] or [0.0], dtype=np.float64)
        self.th, self.ph = th, ph
        self.mat, self.bases = seq_tables(kind, sc.dims)
        s = _Scene()
        s.nx, s.ny, s.nz = sc.n
        s.lo = (C.c_double * 3)(*sc.lo)
        s.hi = (C.c_double * 3)(*sc.hi)
        s.kr = self.kr.ctypes.data_as(C.POINTER(C.c_float))
        s.src_kind = sc.source_kind
        s.src = (C.c_double * 3)(*sc.source)
        s.r_star = sc.r_star
        s.albedo, s.g, s.p_lin = sc.albedo, sc.g, sc.p_lin
        s.n_obs = len(sc.observers)
        s.npix = sc.npix
        s.obs_theta = th.ctypes.data_as(C.POINTER(C.c_double))
        s.obs_phi = ph.ctypes.data_as(C.POINTER(C.c_double))
        s.half_width = sc.half_width
        s.seq_kind = kind
        s.dims = sc.dims
        s.mat = self.mat.ctypes.data_as(C.POINTER(C.c_uint32))
        s.bases = self.bases.ctypes.data_as(C.POINTER(C.c_uint32))
        s.seed = seed
        s.n_total = n_total if n_total is not None else sc.n_packets
        s.max_orders = sc.max_orders
        s.tau_min = sc.tau_min
        s.emit_order = getattr(sc, "emit_order", 0)
        self.surrogate = surrogate
        if surrogate is not None:
            sg = surrogate
            s.peel_mode = 1
            s.mlp = sg.params.ctypes.data_as(C.POINTER(C.c_float))
            s.dom_center = (C.c_double * 3)(*sg.center)
            s.dom_r_in, s.dom_r_out, s.dom_h0, s.dom_beta, s.dom_zmax = \
                sg.r_in, sg.r_out, sg.h0, sg.beta, sg.zmax
            s.dom_nr, s.dom_nz = sg.valid.shape[1], sg.valid.shape[2]
            s.dom_valid = sg.valid.ctypes.data_as(C.POINTER(C.c_uint8))
        self.s = s


def tau_ray(osc: OracleScene, p: Sequence[float], k: Sequence[float]) -> Tuple[float, int]:
    pa = np.ascontiguousarray(p, dtype=np.float64)
    ka = np.ascontiguousarray(k, dtype=np.float64)
    v = C.c_int64(0)
    t = lib().oracle_tau_ray(C.byref(osc.s), pa.ctypes.data, ka.ctypes.data, C.byref(v))
    return t, v.value


def move(osc: OracleScene, p, k, target: float):
    pa = np.ascontiguousarray(p, dtype=np.float64)
    ka = np.ascontiguousarray(k, dtype=np.float64)
    out = np.zeros(3)
    v = C.c_int64(0)
    st = lib().oracle_move(C.byref(osc.s), pa.ctypes.data, ka.ctypes.data, float(target),
                           out.ctypes.data, C.byref(v))
    return out, bool(st), v.value


def hg_cos(g: float, v: float) -> float:
    return lib().oracle_hg_cos(g, v)


EVENT_FIELDS = ("px", "py", "pz", "X", "Y", "I", "Q", "U", "cos_obs", "order", "obs")


def run(sc, kind: int = SOBOL, first: int = 1, count: Optional[int] = None, seed: int = 0,
        n_total: Optional[int] = None, nthreads: int = 1, max_events: int = 0,
        normalize: bool = True, surrogate: Optional[Surrogate] = None, per_order: bool = False):
    """Run packets first..first+count-1 of a scene.  Returns (images [n_obs][3][npix][npix],
    counters dict, events array or None).  Images are divided by count when normalize.
    With `surrogate`, peel-off optical depths inside valid cells come from the network.
    With `per_order`, the images are [max_orders][n_obs][3][npix][npix], one set per
    scattering order."""
    count = sc.n_packets if count is None else count
    osc = OracleScene(sc, kind, seed, n_total, surrogate)
    shape = (len(sc.observers), 3, sc.npix, sc.npix)
    if per_order:
        osc.s.order_images = sc.max_orders
        shape = (sc.max_orders,) + shape
    img = np.zeros(shape, dtype=np.float64)
    cnt = Counters()
    ev = np.zeros((max_events, len(EVENT_FIELDS)), dtype=np.float64) if max_events else None
    nev = C.c_int64(0)
    rc = lib().oracle_run(C.byref(osc.s), first, count, img.ctypes.data, C.byref(cnt), nthreads,
                          ev.ctypes.data if ev is not None else None, max_events, C.byref(nev))
    if rc != 0:
        raise ValueError("oracle_run failed")
    if normalize and count > 0:
        img /= count
    if ev is not None:
        ev = ev[: nev.value]
    return img, cnt.as_dict(), ev


def mlp_batch(params, X) -> np.ndarray:
    """Raw outputs of the C network (bfloat16 emulation) for inputs X[n][5]."""
    th = np.ascontiguousarray(params, dtype=np.float32)
    Xa = np.ascontiguousarray(X, dtype=np.float64)
    y = np.zeros(len(Xa))
    lib().oracle_mlp_batch(th.ctypes.data, len(Xa), Xa.ctypes.data, y.ctypes.data)
    return y


def mlp_tau(sc, surrogate: Surrogate, p, obs: int) -> float:
    """Clamped network optical depth from position p toward observer obs."""
    osc = OracleScene(sc, surrogate=surrogate)
    pa = np.ascontiguousarray(p, dtype=np.float64)
    return lib().oracle_mlp_tau(C.byref(osc.s), pa.ctypes.data, obs)


def dom_cells(sc, surrogate: Surrogate, p) -> np.ndarray:
    """Domain cell index ir * n_z + iz (or -1) of positions p[n][3]."""
    osc = OracleScene(sc, surrogate=surrogate)
    pa = np.ascontiguousarray(p, dtype=np.float64)
    out = np.zeros(len(pa), dtype=np.int64)
    lib().oracle_dom_cells(C.byref(osc.s), len(pa), pa.ctypes.data, out.ctypes.data)
    return out


def max_threads() -> int:
    return lib().oracle_max_threads()


def emit(sc, kind: int, first: int, count: int, seed: int = 0, n_total: Optional[int] = None):
    """Emission positions and directions ([count][3] each) of packets first..first+count-1."""
    osc = OracleScene(sc, kind, seed, n_total)
    p = np.zeros((count, 3))
    k = np.zeros((count, 3))
    if lib().oracle_emit(C.byref(osc.s), first, count, p.ctypes.data, k.ctypes.data) != 0:
        raise ValueError("oracle_emit failed")
    return p, k


def quad_flux(sc, obs: int = 0, n_mu: int = 256, n_phi: int = 512, n_seg: int = 4) -> float:
    """First-order scattered flux toward observer obs by direct quadrature (point source)."""
    osc = OracleScene(sc)
    return lib().oracle_quad_flux(C.byref(osc.s), obs, n_mu, n_phi, n_seg)


def quad_pixels(sc, obs: int = 0, n_sub: int = 4, n_seg: int = 4) -> np.ndarray:
    """First-order intensity image [npix][npix] toward observer obs by volume quadrature."""
    osc = OracleScene(sc)
    out = np.zeros((sc.npix, sc.npix))
    lib().oracle_quad_pixels(C.byref(osc.s), obs, n_sub, n_seg, out.ctypes.data)
    return out
