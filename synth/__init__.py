"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *generates inputs*: velocity/slowness-squared models, source
signatures, acquisition geometry and probe matrices.  It holds none of the
method's arithmetic (no propagation, damping, probing or imaging) so that the
CPU oracle and the HIP library, which both consume these arrays, stay
independent of each other.

The paper's own workloads (a 2D SEAM slice with salt and sparse ocean-bottom
nodes, a 2D BP TTI subset; Section "Synthetic case studies") are not available;
the recipes below are synthetic stand-ins with the same structure: layered
sediments, a high-velocity salt body, a near-surface source and a dense receiver
spread.  Every generator is deterministic given its seed (numpy default_rng).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "rademacher", "sylvester_hadamard", "ricker", "source_signature",
    "smooth", "pad_edge", "two_layer_2d", "layered_3d", "salt_ellipsoid",
    "plane_receivers", "line_receivers", "Workload", "workload_c1",
    "workload_c2", "workload_small_3d", "workload_small_2d", "workload_batched",
    "tti_parameters", "workload_tti", "model_salt_300",
]


# ----------------------------------------------------------------------------
# probes (Section "Randomized trace estimation": Z is a Rademacher matrix of +-1)
# ----------------------------------------------------------------------------
def rademacher(nt: int, r: int, seed: int) -> np.ndarray:
    """Z[nt][r] with independent +-1 entries, int8, row n is the probe row z_n."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 2, size=(nt, r), dtype=np.int8) * 2 - 1).astype(np.int8)


def sylvester_hadamard(n: int) -> np.ndarray:
    """n x n Sylvester Hadamard matrix (n a power of two), int8 +-1, H H^T = n I."""
    if n < 1 or n & (n - 1):
        raise ValueError("Sylvester construction needs a power of two")
    h = np.ones((1, 1), dtype=np.int8)
    while h.shape[0] < n:
        h = np.block([[h, h], [h, -h]]).astype(np.int8)
    return h


# ----------------------------------------------------------------------------
# source signature
# ----------------------------------------------------------------------------
def ricker(nt: int, dt: float, f0: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet w(n dt), n = 0..nt-1, peak frequency f0, delay t0 (default 1/f0)."""
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def source_signature(nt: int, dt: float, f0: float, h: float, ndim: int,
                     nsrc: int = 1) -> np.ndarray:
    """q[nt][nsrc]: a Ricker wavelet divided by the cell volume h^ndim.

    Injected as is, this makes a unit point source of the continuous equation.
    """
    w = ricker(nt, dt, f0) / h ** ndim
    return np.repeat(w[:, None], nsrc, axis=1)


# ----------------------------------------------------------------------------
# models
# ----------------------------------------------------------------------------
def smooth(v: np.ndarray, sigma: float) -> np.ndarray:
    """Gaussian smoothing with edge replication, radius 4 sigma."""
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(v, sigma=sigma, mode="nearest", truncate=4.0)


def pad_edge(v: np.ndarray, nb: int) -> np.ndarray:
    return np.pad(v, nb, mode="edge")


def two_layer_2d(nz: int = 201, nx: int = 201, iface: int = 50,
                 v1: float = 1500.0, v2: float = 2500.0) -> np.ndarray:
    v = np.full((nz, nx), v1, dtype=np.float64)
    v[iface:, :] = v2
    return v


def layered_3d(nz: int, ny: int, nx: int, nlayers: int, vmin: float, vmax: float,
               pert: float = 0.0, seed: int | None = None,
               dtype=np.float32) -> np.ndarray:
    """Flat layers of equal thickness in z, velocity linear from vmin to vmax,
    optionally multiplied cell by cell by (1 + pert * U[-1, 1))."""
    edges = np.linspace(0, nz, nlayers + 1).round().astype(int)
    v = np.empty((nz, ny, nx), dtype=dtype)
    for l in range(nlayers):
        vl = vmin + (vmax - vmin) * (l / max(nlayers - 1, 1))
        v[edges[l]:edges[l + 1]] = vl
    if pert:
        rng = np.random.default_rng(seed)
        for iz in range(nz):  # plane by plane keeps peak host memory low
            v[iz] *= (1.0 + pert * rng.uniform(-1.0, 1.0, size=(ny, nx))).astype(dtype)
    return v


def salt_ellipsoid(v: np.ndarray, centre, semi, vsalt: float = 4500.0) -> np.ndarray:
    """Overwrite an ellipsoid (grid-cell centre and semi-axes, z,y,x) with vsalt."""
    nz, ny, nx = v.shape
    z, y, x = np.ogrid[:nz, :ny, :nx]
    inside = (((z - centre[0]) / semi[0]) ** 2 + ((y - centre[1]) / semi[1]) ** 2
              + ((x - centre[2]) / semi[2]) ** 2) <= 1.0
    out = v.copy()
    out[inside] = vsalt
    return out


# ----------------------------------------------------------------------------
# geometry (positions in grid units, order z, y, x)
# ----------------------------------------------------------------------------
def plane_receivers(iz: float, ny: int, nx: int) -> np.ndarray:
    yy, xx = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                         indexing="ij")
    pos = np.empty((ny * nx, 3), dtype=np.float64)
    pos[:, 0] = iz
    pos[:, 1] = yy.ravel()
    pos[:, 2] = xx.ravel()
    return pos


def line_receivers(iz: float, ix: np.ndarray, iy: float = 0.0) -> np.ndarray:
    ix = np.asarray(ix, dtype=np.float64)
    pos = np.zeros((ix.size, 3), dtype=np.float64)
    pos[:, 0] = iz
    pos[:, 1] = iy
    pos[:, 2] = ix
    return pos


# ----------------------------------------------------------------------------
# complete workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    """Everything one gradient evaluation needs.  Arrays are host numpy."""
    name: str
    ndim: int
    shape: tuple            # (nz, ny, nx); ny == 1 in 2D
    h: float
    dt: float
    nt: int
    nb: int
    c_ref: float
    R: float
    m: np.ndarray            # slowness squared [N], model the gradient is taken at
    m_true: np.ndarray | None
    src_pos: np.ndarray      # [ns][3]
    q: np.ndarray            # [nt][ns]
    rec_pos: np.ndarray      # [nr][3]
    Z: np.ndarray            # [nt][r] int8
    k_block: int = 32

    @property
    def N(self) -> int:
        return int(np.prod(self.shape))

    @property
    def r(self) -> int:
        return int(self.Z.shape[1])


def workload_c1(dtype=np.float64) -> Workload:
    """2D two-layer acoustic case: 201x201 physical cells, h = 10 m, padded by
    10 damping cells per side, nt = 1000, dt = 1 ms, 15 Hz Ricker at
    (x, z) = (1000 m, 20 m), 101 receivers at z = 20 m every 20 m, r = 32.
    The interface lies at 500 m depth so that its reflection returns within
    the 1 s record (from 1000 m it would arrive at ~1.33 s and the residual
    of the smoothed background would be round-off only)."""
    nb, h, dt, nt = 10, 10.0, 1e-3, 1000
    v_true = two_layer_2d()
    v0 = smooth(v_true, 5.0)
    vt = pad_edge(v_true, nb)
    vb = pad_edge(v0, nb)
    nz, nx = vt.shape
    m_true = (1.0 / vt ** 2).astype(dtype).ravel()
    m0 = (1.0 / vb ** 2).astype(dtype).ravel()
    src = np.array([[nb + 2.0, 0.0, nb + 100.0]])
    rec = line_receivers(nb + 2.0, nb + 2.0 * np.arange(101))
    q = source_signature(nt, dt, 15.0, h, 2).astype(dtype)
    return Workload("2d-two-layer-221x221-nt1000-r32", 2, (nz, 1, nx), h, dt, nt, nb,
                    2500.0, 1e-3, m0, m_true, src, q, rec, rademacher(nt, 32, 0), 32)


def workload_c2(nt: int = 3000, r: int = 128, k_block: int = 32,
                shape=(384, 512, 512)) -> Workload:
    """3D layered acoustic case: 384 x 512 x 512 cells (z, y, x) including 10
    damping cells per face, h = 12.5 m, 12 layers 1.5-4.5 km/s with +-5 %
    cell-wise perturbation (seed 1), 10 Hz Ricker at (12, 256, 256), a full
    receiver plane at iz = 12, dt = 1 ms, r = 128 probes (seed 2)."""
    nz, ny, nx = shape
    h, dt, nb = 12.5, 1e-3, 10
    v = layered_3d(nz, ny, nx, 12, 1500.0, 4500.0, pert=0.05, seed=1)
    m = (1.0 / v.astype(np.float64) ** 2).astype(np.float32).ravel()
    del v
    src = np.array([[12.0, ny // 2, nx // 2]], dtype=np.float64)
    rec = plane_receivers(12.0, ny, nx)
    q = source_signature(nt, dt, 10.0, h, 3).astype(np.float32)
    return Workload(f"3d-layered-{nz}x{ny}x{nx}-nt{nt}-r{r}-k{k_block}", 3, shape, h, dt,
                    nt, nb, 4725.0, 1e-3, m, None, src, q, rec, rademacher(nt, r, 2),
                    k_block)


def workload_small_3d(shape=(40, 36, 70), nt: int = 120, r: int = 16, seed: int = 11,
                      h: float = 12.5, dt: float = 1e-3, nb: int = 6,
                      f0: float = 12.0, dtype=np.float32) -> Workload:
    """Reduced 3D layered case for parity tests: ragged sizes, a few layers with
    a 5 % perturbation, an off-centre source and a sparse receiver plane."""
    nz, ny, nx = shape
    v = layered_3d(nz, ny, nx, 4, 1500.0, 3500.0, pert=0.05, seed=seed)
    m = (1.0 / v.astype(np.float64) ** 2).astype(dtype).ravel()
    src = np.array([[nb + 2.0, ny // 2 - 1, nx // 2 + 3]], dtype=np.float64)
    rec = plane_receivers(nb + 3.0, ny, nx)[::3]
    q = source_signature(nt, dt, f0, h, 3).astype(dtype)
    return Workload(f"3d-small-{nz}x{ny}x{nx}-nt{nt}", 3, shape, h, dt, nt, nb,
                    float(v.max()), 1e-3, m, None, src, q, rec,
                    rademacher(nt, r, seed + 1), 16)


def workload_small_2d(shape=(60, 75), nt: int = 200, r: int = 8, seed: int = 5,
                      h: float = 10.0, dt: float = 1e-3, nb: int = 8,
                      dtype=np.float64) -> Workload:
    nz, nx = shape
    rng = np.random.default_rng(seed)
    v = np.where(np.arange(nz)[:, None] < nz // 2, 1500.0, 2500.0) * np.ones((1, nx))
    v = v * (1.0 + 0.03 * rng.uniform(-1, 1, size=v.shape))
    m = (1.0 / v ** 2).astype(dtype).ravel()
    src = np.array([[nb + 2.0, 0.0, nx // 2 + 0.0]])
    rec = line_receivers(nb + 2.0, np.arange(nb, nx - nb, 2))
    q = source_signature(nt, dt, 15.0, h, 2).astype(dtype)
    return Workload(f"2d-small-{nz}x{nx}-nt{nt}", 2, (nz, 1, nx), h, dt, nt, nb,
                    float(v.max()), 1e-3, m, None, src, q, rec,
                    rademacher(nt, r, seed + 1), 16)


def batched_window_shapes(nshots: int = 16, lo=(128, 128, 128), hi=(256, 320, 320)):
    """Uneven sub-domain windows (z, y, x) growing linearly from lo to hi."""
    shapes = []
    for s in range(nshots):
        f = s / max(nshots - 1, 1)
        shapes.append(tuple(int(round(a + (b - a) * f)) for a, b in zip(lo, hi)))
    return shapes


def workload_batched(nt: int = 2000, r: int = 64, k_block: int = 32, nshots: int = 16,
                     shapes=None) -> list:
    """16 shots on uneven windows 128^3 ... 256 x 320 x 320 (z, y, x), each the
    layered recipe of the 384 x 512 x 512 case (12 layers 1.5-4.5 km/s, +-5 %,
    seed 100 + s), a 10 Hz source at the window's top centre, a full receiver
    plane at iz = 12, nt = 2000, dt = 1 ms, r = 64 probes (seed 200 + s)."""
    shapes = shapes or batched_window_shapes(nshots)
    h, dt, nb = 12.5, 1e-3, 10
    out = []
    for s, (nz, ny, nx) in enumerate(shapes):
        v = layered_3d(nz, ny, nx, 12, 1500.0, 4500.0, pert=0.05, seed=100 + s)
        m = (1.0 / v.astype(np.float64) ** 2).astype(np.float32).ravel()
        del v
        src = np.array([[12.0, ny // 2, nx // 2]], dtype=np.float64)
        rec = plane_receivers(12.0, ny, nx)
        q = source_signature(nt, dt, 10.0, h, 3).astype(np.float32)
        out.append(Workload(f"batched-{s}-{nz}x{ny}x{nx}", 3, (nz, ny, nx), h, dt, nt, nb,
                            4725.0, 1e-3, m, None, src, q, rec, rademacher(nt, r, 200 + s),
                            k_block))
    return out


def tti_parameters(shape, seeds=(3, 4, 5, 6), sigma: float = 10.0, salt=None,
                   dtype=np.float64) -> np.ndarray:
    """[4][N] = (eps, delta, theta, phi): smoothed white noise mapped to
    eps in [0, 0.3], delta in [0, 0.15] (then delta <= eps), tilt theta in
    [0, 30 deg] and azimuth phi in [0, 360 deg) (radians); zero anisotropy
    inside an optional salt mask."""
    from concurrent.futures import ThreadPoolExecutor

    def field(args):
        seed, lo, hi = args
        w = smooth(np.random.default_rng(seed).standard_normal(shape), sigma)
        w = (w - w.min()) / max(w.max() - w.min(), 1e-30)
        return lo + (hi - lo) * w
    # the four fields are independent; the filter releases the GIL
    with ThreadPoolExecutor(4) as ex:
        eps, dl, th, ph = ex.map(field, [(seeds[0], 0.0, 0.3), (seeds[1], 0.0, 0.15),
                                         (seeds[2], 0.0, 30.0), (seeds[3], 0.0, 359.999)])
    dl = np.minimum(dl, eps)
    th = np.deg2rad(th)
    ph = np.deg2rad(ph)
    if salt is not None:
        eps[salt] = 0.0
        dl[salt] = 0.0
    out = np.empty((4, eps.size), dtype=dtype)
    for i, f in enumerate((eps, dl, th, ph)):
        out[i] = f.ravel()
    return out


def workload_tti(shape=(300, 400, 400), nt: int = 2500, r: int = 64, sigma: float = 10.0,
                 salt_centre=None, salt_semi=None, nb: int = 10, f0: float = 10.0,
                 rec_stride: int = 1, dtype=np.float32):
    """Layered TTI model: 10 layers 1.5-3.5 km/s, a 4.5 km/s salt ellipsoid
    (centre (150, 200, 200), semi-axes (60, 120, 120) cells at full size,
    scaled with the grid) with eps = delta = 0 inside, smooth eps / delta /
    tilt / azimuth fields, source at the top centre, receiver plane at iz = 12,
    r probes (seed 7).  Returns (Workload, aniso [4][N])."""
    nz, ny, nx = shape
    h, dt = 12.5, 1e-3
    v = layered_3d(nz, ny, nx, 10, 1500.0, 3500.0, dtype=np.float64)
    centre = salt_centre or (nz * 0.5, ny * 0.5, nx * 0.5)
    semi = salt_semi or (nz * 0.2, ny * 0.3, nx * 0.3)
    z, y, x = np.ogrid[:nz, :ny, :nx]
    inside = (((z - centre[0]) / semi[0]) ** 2 + ((y - centre[1]) / semi[1]) ** 2
              + ((x - centre[2]) / semi[2]) ** 2) <= 1.0
    v[inside] = 4500.0
    aniso = tti_parameters(shape, sigma=sigma, salt=inside, dtype=dtype)
    m = (1.0 / v ** 2).astype(dtype).ravel()
    vh_max = float(np.max(v.ravel() * np.sqrt(1.0 + 2.0 * aniso[0].astype(np.float64))))
    src = np.array([[min(12.0, nz - 1.0), ny // 2, nx // 2]], dtype=np.float64)
    rec = plane_receivers(min(12.0, nz - 1.0), ny, nx)[::rec_stride]
    q = source_signature(nt, dt, f0, h, 3).astype(dtype)
    wl = Workload(f"3d-tti-{nz}x{ny}x{nx}-nt{nt}-r{r}", 3, shape, h, dt, nt, nb, vh_max, 1e-3,
                  m, None, src, q, rec, rademacher(nt, r, 7), 32)
    return wl, aniso


def model_salt_300(n: int = 300, sigma: float = 5.0):
    """300^3 salt case (h = 12.5 m): 10 layers 1.5-3.5 km/s and a 4.5 km/s salt
    ellipsoid at (170, 150, 150) with semi-axes (40, 80, 80) cells (scaled for
    other n).  Returns (m_true, m0) as float32 [N], m0 from the velocity
    smoothed with sigma = 5 cells."""
    f = n / 300.0
    v = layered_3d(n, n, n, 10, 1500.0, 3500.0, dtype=np.float64)
    v = salt_ellipsoid(v, (170 * f, 150 * f, 150 * f), (40 * f, 80 * f, 80 * f), 4500.0)
    m_true = (1.0 / v ** 2).astype(np.float32).ravel()
    m0 = (1.0 / smooth(v, sigma) ** 2).astype(np.float32).ravel()
    return m_true, m0


def shots_salt_300(n: int = 300):
    """Four sources at (12, {75, 225}, {75, 225}) (scaled for other n) and the
    full receiver plane at iz = 12."""
    f = n / 300.0
    src = [np.array([[12.0, y * f, x * f]]) for y in (75, 225) for x in (75, 225)]
    return src, plane_receivers(12.0, n, n)
