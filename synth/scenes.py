"""Seeded synthetic scenes: the input data every run of the transport consumes.

This module builds density grids, source and dust parameters and observer
lists.  It holds none of the transport arithmetic (no point generation, no
traversal, no scattering): it only samples analytic density laws at cell
centres and scales them to a requested optical depth.  Both the CPU oracle
and the GPU library take its output as plain arrays.

Geometry and dust follow the paper's test problems (Sec. 5 flared disk,
Eq. of the flared disk; Sec. 5 dust envelope; Sec. 7 sphere source), re-scaled
to a unit box because the paper's au-scale parameters and grid resolutions are
not reproducible here.  Readings:

* density is sampled at cell centres (the paper only says densities are
  precomputed on the mesh, Sec. 3.4);
* the extinction scale is fixed by requiring that the grid optical depth
  along the +x ray from the source equals the target.  With an even cell
  count that ray runs along the y=z=0 cell faces, and the floor rule used by
  the traversal puts it in the row j=k=n/2, so the normalisation sums that row.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# sequence kinds (shared numbering of the C-ABI and of the oracle front end)
SOBOL, HALTON, NIEDERREITER2, HAMMERSLEY, PHILOX, FAURE, SOBOL_OWEN = 0, 1, 2, 3, 4, 5, 6
KIND_NAMES = {SOBOL: "sobol", HALTON: "halton", NIEDERREITER2: "niederreiter2",
              HAMMERSLEY: "hammersley", PHILOX: "philox", FAURE: "faure", SOBOL_OWEN: "sobol_owen"}
KIND_BY_NAME = {v: k for k, v in KIND_NAMES.items()}

POINT_SOURCE, SPHERE_SOURCE = 0, 1


@dataclasses.dataclass
class Scene:
    name: str
    n: Tuple[int, int, int]            # (nx, ny, nz)
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    kappa_rho: np.ndarray              # float32 [nz][ny][nx], x fastest
    source: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    source_kind: int = POINT_SOURCE
    r_star: float = 0.0
    emit_order: int = 0          # sphere star: 0 direct, 1 inverse order of the point coordinates
    albedo: float = 0.6
    g: float = 0.5
    p_lin: float = 0.5
    observers: List[Tuple[float, float]] = dataclasses.field(default_factory=list)  # (theta, phi) rad
    npix: int = 64
    half_width: float = 1.0
    max_orders: int = 1
    tau_min: float = 1e-8
    fp64: bool = True
    n_packets: int = 1 << 16

    @property
    def dims(self) -> int:
        """Point dimension: 3 per flight, 2 more for a sphere-star emission point (Sec. 3.7)."""
        base = 5 if self.source_kind == SPHERE_SOURCE else 3
        return base + 3 * (self.max_orders - 1)

    def replace(self, **kw) -> "Scene":
        return dataclasses.replace(self, **kw)


def cell_centres(n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    h = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * h


def _mesh(n: int):
    c = cell_centres(n)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    return x, y, z


def _scale_to_x_ray(rho: np.ndarray, target_tau: float) -> np.ndarray:
    """Scale rho so that the sum of rho*h over row j=k=n/2, i>=n/2 equals target_tau."""
    n = rho.shape[0]
    h = 2.0 / n
    row = rho[n // 2, n // 2, n // 2:]
    s = float(np.sum(row.astype(np.float64)) * h)
    if s <= 0.0:
        raise ValueError("density is zero along the normalisation ray")
    return rho * (target_tau / s)


def envelope32(n_packets: int = 1 << 16) -> Scene:
    """Spherical envelope rho ~ r^-2 on 0.05<r<1, 32^3 grid, radial tau 1, one observer at 45 deg."""
    n = 32
    x, y, z = _mesh(n)
    r = np.sqrt(x * x + y * y + z * z)
    rho = np.where((r > 0.05) & (r < 1.0), 1.0 / np.maximum(r, 1e-30) ** 2, 0.0)
    kr = _scale_to_x_ray(rho, 1.0).astype(np.float32)
    return Scene(name="envelope32", n=(n, n, n), lo=(-1.0,) * 3, hi=(1.0,) * 3, kappa_rho=kr,
                 albedo=0.6, g=0.5, p_lin=0.5, observers=[(math.radians(45.0), 0.0)],
                 npix=64, half_width=1.0, max_orders=1, fp64=True, n_packets=n_packets)


def disk_density(n: int, h0: float = 0.1) -> np.ndarray:
    """Flared disk rho ~ (R/R0)^-2.25 exp(-z^2/2h^2), h = h0 R^1.125 (h0 = 0.1), R0 = 1, 0.05<=R<=1."""
    x, y, z = _mesh(n)
    R = np.sqrt(x * x + y * y)
    Rs = np.maximum(R, 1e-30)
    hR = h0 * Rs ** 1.125
    rho = Rs ** -2.25 * np.exp(-0.5 * (z / hR) ** 2)
    return np.where((R >= 0.05) & (R <= 1.0), rho, 0.0)


def disk128(n_packets: int = 1 << 22, n: int = 128, tau_mid: float = 10.0, h0: float = 0.1) -> Scene:
    """Flared disk, midplane tau 10 (or tau_mid), scale height h0 R^1.125 (h0 = 0.1), 20 orders, three
    inclinations, 256^2 images, FP32 transport."""
    kr = _scale_to_x_ray(disk_density(n, h0), tau_mid).astype(np.float32)
    obs = [(math.radians(t), 0.0) for t in (0.0, 45.0, 90.0)]
    name = f"disk{n}" if (tau_mid == 10.0 and h0 == 0.1) else f"disk{n}_tau{tau_mid:g}_h{h0:g}"
    return Scene(name=name, n=(n, n, n), lo=(-1.0,) * 3, hi=(1.0,) * 3, kappa_rho=kr,
                 albedo=0.5, g=0.6, p_lin=0.5, observers=obs, npix=256, half_width=1.0,
                 max_orders=20, fp64=False, n_packets=n_packets)


def lognormal_field(n: int, sigma: float, corr_voxels: float, seed: int) -> np.ndarray:
    """exp(sigma*G - sigma^2/2) of a periodic Gaussian random field G (zero mean, unit variance)
    whose correlation is exp(-r^2 / (2 corr^2)) in voxel units."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    d = np.minimum(np.arange(n), n - np.arange(n)).astype(np.float64)
    d2 = d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2
    kern = np.exp(-d2 / (2.0 * corr_voxels ** 2))
    P = np.fft.rfftn(kern).real
    np.maximum(P, 0.0, out=P)
    G = np.fft.irfftn(np.sqrt(P) * np.fft.rfftn(w), s=(n, n, n))
    G -= G.mean()
    G /= G.std()
    return np.exp(sigma * G - 0.5 * sigma * sigma)


def clumpy256(n_packets: int = 1 << 24, n: int = 256, seed: int = 1556) -> Scene:
    """Clumpy envelope rho ~ r^-1.5 * lognormal(sigma=1, 8-voxel correlation), sphere star r*=0.02."""
    x, y, z = _mesh(n)
    r = np.sqrt(x * x + y * y + z * z)
    base = np.where((r >= 0.05) & (r <= 1.0), np.maximum(r, 1e-30) ** -1.5, 0.0)
    del x, y, z, r
    rho = base * lognormal_field(n, 1.0, 8.0 * n / 256.0, seed)
    kr = _scale_to_x_ray(rho, 3.0).astype(np.float32)
    return Scene(name=f"clumpy{n}", n=(n, n, n), lo=(-1.0,) * 3, hi=(1.0,) * 3, kappa_rho=kr,
                 source_kind=SPHERE_SOURCE, r_star=0.02, albedo=0.6, g=0.4, p_lin=0.5,
                 observers=[(math.radians(60.0), 0.0)], npix=512, half_width=1.0,
                 max_orders=1, fp64=False, n_packets=n_packets)


def thin_sphere(n: int = 64, R: float = 0.9, tau_R: float = 0.01, npix: int = 64) -> Scene:
    """Homogeneous sphere of radius R (cells whose centre lies inside), radial tau tau_R."""
    x, y, z = _mesh(n)
    r = np.sqrt(x * x + y * y + z * z)
    rho = np.where(r <= R, 1.0, 0.0)
    kr = _scale_to_x_ray(rho, tau_R).astype(np.float32)
    return Scene(name=f"thin_sphere{n}", n=(n, n, n), lo=(-1.0,) * 3, hi=(1.0,) * 3, kappa_rho=kr,
                 albedo=0.6, g=0.5, p_lin=0.5, observers=[(math.radians(45.0), 0.0)],
                 npix=npix, half_width=1.0, max_orders=1, fp64=True)


def uniform_cube(n: int, value: float) -> np.ndarray:
    return np.full((n, n, n), value, dtype=np.float32)


def random_grid(shape: Tuple[int, int, int], seed: int, zero_frac: float = 0.2) -> np.ndarray:
    """Random positive cells with a share of empty ones; shape is (nz, ny, nx)."""
    rng = np.random.default_rng(seed)
    g = rng.uniform(0.1, 3.0, size=shape)
    g[rng.uniform(size=shape) < zero_frac] = 0.0
    return g.astype(np.float32)


def envelope_density(n: int, power: float = 2.0) -> np.ndarray:
    """Spherical envelope rho ~ r^-power on 0.05 < r < 1."""
    x, y, z = _mesh(n)
    r = np.sqrt(x * x + y * y + z * z)
    return np.where((r > 0.05) & (r < 1.0), 1.0 / np.maximum(r, 1e-30) ** power, 0.0)


def uneven_batch(seed: int, n_scenes: int = 64, sizes: Tuple[int, int, int] = (32, 192, 16),
                 log2_packets: Tuple[float, float] = (16.0, 24.0), npix: int = 128,
                 orders: Tuple[int, int] = (1, 20), tau: Tuple[float, float] = (0.1, 20.0)) -> List[Scene]:
    """A batch of uneven scenes drawn from `seed`, each independently:
      grid n^3 with n uniform over sizes[0] .. sizes[1] in steps of sizes[2] (even n);
      packets 2^u, u uniform in log2_packets;
      geometry: spherical envelope (rho ~ r^-2) or flared disk (as disk128), 1:1;
      optical depth along +x from the centre log-uniform in `tau`;
      g uniform in [0, 0.8], albedo uniform in [0.3, 0.9], p_lin 0.5;
      source: point source at the centre, or for an envelope with probability
      1/2 a sphere star of radius 0.02 emitting in the direct or inverse order;
      1 to 4 observers, inclination uniform in [0, 90] deg, azimuth uniform;
      max_orders uniform over orders[0] .. orders[1]; npix^2 images over the box;
      FP32 transport."""
    rng = np.random.default_rng(seed)
    cache = {}
    out = []
    lo_n, hi_n, step = sizes
    choices = list(range(lo_n, hi_n + 1, step))
    for i in range(n_scenes):
        n = int(rng.choice(choices))
        n_packets = int(2.0 ** rng.uniform(*log2_packets))
        disk = bool(rng.integers(2))
        t = float(math.exp(rng.uniform(math.log(tau[0]), math.log(tau[1]))))
        g = float(rng.uniform(0.0, 0.8))
        albedo = float(rng.uniform(0.3, 0.9))
        star = (not disk) and bool(rng.integers(2))
        emit_order = int(rng.integers(2)) if star else 0
        n_obs = int(rng.integers(1, 5))
        observers = [(float(math.radians(rng.uniform(0.0, 90.0))), float(rng.uniform(0.0, 2.0 * math.pi)))
                     for _ in range(n_obs)]
        max_orders = int(rng.integers(orders[0], orders[1] + 1))
        key = (disk, n)
        if key not in cache:
            rho = disk_density(n) if disk else envelope_density(n)
            cache[key] = (rho, _scale_to_x_ray(rho, 1.0))
        kr = (cache[key][1] * t).astype(np.float32)
        out.append(Scene(name=f"batch{seed}_{i}", n=(n, n, n), lo=(-1.0,) * 3, hi=(1.0,) * 3, kappa_rho=kr,
                         source_kind=SPHERE_SOURCE if star else POINT_SOURCE, r_star=0.02 if star else 0.0,
                         emit_order=emit_order, albedo=albedo, g=g, p_lin=0.5, observers=observers,
                         npix=npix, half_width=1.0, max_orders=max_orders, fp64=False, n_packets=n_packets))
    return out


def scene_by_name(name: str, n_packets: Optional[int] = None) -> Scene:
    table = {"envelope32": envelope32, "disk128": disk128, "clumpy256": clumpy256}
    sc = table[name]()
    if n_packets is not None:
        sc = sc.replace(n_packets=n_packets)
    return sc
