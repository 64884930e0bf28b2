"""Seeded synthetic inputs for the traveltime-Jacobian workloads.

This module only *draws* inputs: transducer rings, source-receiver pair
lists, voxel grids and region-of-interest masks, sampled calibration pulses,
velocity phantoms, noise and voxel picks.  It holds none of the method's
arithmetic (no spectra, no kernels, no Jacobian), so that the CPU oracle and
the HIP path can both be fed from it without sharing any computation.

The stand-ins follow the scales of the paper's lab experiment (Sec. III):
a ring of transducers of about 10 cm radius in water, MHz pulses with a
fractional bandwidth given at -6 dB, a millimetre voxel grid and a circular
region of interest covering roughly 70/95 of the ring radius.  The paper's
own data (the SPIE USCT 2017 lab data set) is not available; these seeded
synthetic arrays stand in for it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# Pulse: Gaussian-windowed sine carrier, sampled.
# ----------------------------------------------------------------------------
def gaussian_sigma(fc: float, bw: float) -> float:
    """Std-dev (s) of the Gaussian window whose amplitude spectrum has a
    full width at half maximum (-6 dB) of ``bw * fc`` Hz around ``fc``.

    The amplitude spectrum of exp(-t^2/2s^2) sin(2 pi fc t) near fc is
    proportional to exp(-s^2 (w - wc)^2 / 2); it halves at
    |w - wc| = sqrt(2 ln 2)/s, so the full width in Hz is sqrt(2 ln 2)/(pi s).
    """
    return math.sqrt(2.0 * math.log(2.0)) / (math.pi * fc * bw)


@dataclass(frozen=True)
class Pulse:
    fc: float          # carrier frequency (Hz)
    bw: float          # -6 dB fractional bandwidth
    samples: np.ndarray  # f(t_n), float64
    dt: float          # sample spacing (s)

    @property
    def sigma(self) -> float:
        return gaussian_sigma(self.fc, self.bw)


def sampled_pulse(fc: float, bw: float, *, per_period: int = 64,
                  half_width_sigmas: float = 8.0) -> Pulse:
    """Gaussian-windowed sine sampled symmetrically about t = 0."""
    sigma = gaussian_sigma(fc, bw)
    dt = 1.0 / (per_period * fc)
    half = int(math.ceil(half_width_sigmas * sigma / dt))
    t = (np.arange(2 * half + 1) - half) * dt
    f = np.exp(-0.5 * (t / sigma) ** 2) * np.sin(2.0 * math.pi * fc * t)
    return Pulse(fc=fc, bw=bw, samples=f.astype(np.float64), dt=dt)


# ----------------------------------------------------------------------------
# Geometry
# ----------------------------------------------------------------------------
def ring(n: int, radius: float, z: float = 0.0, phase: float = 0.0) -> np.ndarray:
    """n transducers equally spaced on a circle in the plane z, [n][3] metres."""
    th = phase + 2.0 * math.pi * np.arange(n) / n
    return np.stack([radius * np.cos(th), radius * np.sin(th),
                     np.full(n, z)], axis=1).astype(np.float64)


def all_ordered_pairs(n: int, offset: int = 0) -> np.ndarray:
    """Every ordered (source, receiver) pair with source != receiver."""
    s, r = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = s != r
    return (np.stack([s[keep], r[keep]], axis=1) + offset).astype(np.int32)


@dataclass(frozen=True)
class Grid:
    dims: tuple            # (nx, ny, nz)
    spacing: tuple         # (hx, hy, hz) metres
    origin: tuple          # centre of voxel (0,0,0), metres

    @property
    def n(self) -> int:
        return int(self.dims[0] * self.dims[1] * self.dims[2])

    def centres(self) -> np.ndarray:
        """[N][3] voxel centres, x fastest."""
        nx, ny, nz = self.dims
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                              indexing="ij")
        x = self.origin[0] + i.ravel() * self.spacing[0]
        y = self.origin[1] + j.ravel() * self.spacing[1]
        z = self.origin[2] + k.ravel() * self.spacing[2]
        return np.stack([x, y, z], axis=1)


def centred_grid(dims, spacing) -> Grid:
    if np.isscalar(spacing):
        spacing = (spacing,) * 3
    origin = tuple(-(d - 1) / 2.0 * h for d, h in zip(dims, spacing))
    return Grid(tuple(int(d) for d in dims), tuple(float(h) for h in spacing),
                tuple(float(o) for o in origin))


def cylinder_mask(grid: Grid, radius: float | None) -> np.ndarray:
    """uint8 [N]: 1 where the voxel centre lies within ``radius`` of the z axis."""
    if radius is None:
        return np.ones(grid.n, dtype=np.uint8)
    c = grid.centres()
    return (np.hypot(c[:, 0], c[:, 1]) <= radius).astype(np.uint8)


# ----------------------------------------------------------------------------
# Phantoms and noise
# ----------------------------------------------------------------------------
def cylinder_phantom(grid: Grid, radius: float, value: float) -> np.ndarray:
    c = grid.centres()
    return np.where(np.hypot(c[:, 0], c[:, 1]) <= radius, value, 0.0)


def nested_cylinders(grid: Grid, radii, values) -> np.ndarray:
    """Concentric cylinders: values[0] inside radii[0], values[1] in the
    shell radii[0] < r <= radii[1], and so on."""
    c = grid.centres()
    r = np.hypot(c[:, 0], c[:, 1])
    out = np.zeros(grid.n)
    lo = -1.0
    for rad, v in zip(radii, values):
        out[(r > lo) & (r <= rad)] = v
        lo = rad
    return out


def gaussian_blobs(grid: Grid, n_blobs: int, roi_radius: float, z_half: float,
                   sig_range=(3e-3, 10e-3), amp_range=(-40.0, 40.0),
                   seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    rr = roi_radius * np.sqrt(rng.uniform(0.0, 1.0, n_blobs))
    th = rng.uniform(0.0, 2.0 * math.pi, n_blobs)
    cz = rng.uniform(-z_half, z_half, n_blobs)
    sig = rng.uniform(*sig_range, n_blobs)
    amp = rng.uniform(*amp_range, n_blobs)
    c = grid.centres()
    out = np.zeros(grid.n)
    for k in range(n_blobs):
        d2 = ((c[:, 0] - rr[k] * math.cos(th[k])) ** 2
              + (c[:, 1] - rr[k] * math.sin(th[k])) ** 2
              + (c[:, 2] - cz[k]) ** 2)
        out += amp[k] * np.exp(-0.5 * d2 / sig[k] ** 2)
    return out


def noise(m: int, sigma: float, seed: int) -> np.ndarray:
    return sigma * np.random.default_rng(seed).standard_normal(m)


def pick_voxels(mask: np.ndarray, n: int, seed: int) -> np.ndarray:
    """n distinct active voxel indices, drawn uniformly."""
    act = np.flatnonzero(mask)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(act, size=n, replace=False)).astype(np.int64)


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    c0: float
    tx: np.ndarray           # [n_tx][3]
    pairs: np.ndarray        # [M][2] int32
    grid: Grid
    mask: np.ndarray         # [N] uint8
    pulses: list             # one Pulse per band
    r_max: list              # truncation radius of the detour, per band (m)
    n_table: int = 4096
    model: np.ndarray | None = None   # velocity perturbation (m/s), [N]
    noise_sigma: float = 0.0          # traveltime noise std-dev (s)
    noise_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.pairs.shape[0])

    @property
    def n(self) -> int:
        return self.grid.n

    @property
    def n_bands(self) -> int:
        return len(self.pulses)


# Truncation radii: the smallest detour beyond which |h| stays below 1e-7 of
# its maximum for each pulse family, rounded up to 10 micrometres.
R_MAX_HALF_MHZ_BW50 = 18.21e-3
R_MAX = {0.5e6: 9.53e-3, 1.0e6: 4.77e-3, 1.5e6: 3.18e-3, 2.0e6: 2.39e-3}


# Tikhonov weights (prior covariance I, noise 5 ns).  On the small ring the
# discrepancy principle (misfit ~ number of data) gives 5e-3, i.e. 5.35e-3 of
# the largest eigenvalue of J^T J / sigma^2 (0.934 there); the lab-like ring
# uses the same fraction of its own largest eigenvalue (4.91, power iteration).
ALPHA_SMALL = 5e-3
ALPHA_RING2D = 2.63e-2


def small_fp64() -> Workload:
    """32-element ring (r = 10 cm), 24x24x12 grid at 2 mm, 0.5 MHz, 50 % BW."""
    g = centred_grid((24, 24, 12), 2e-3)
    return Workload(
        name="ring32_grid24x24x12_0.5MHz", c0=1500.0, tx=ring(32, 0.10),
        pairs=all_ordered_pairs(32), grid=g, mask=cylinder_mask(g, None),
        pulses=[sampled_pulse(0.5e6, 0.5)], r_max=[R_MAX_HALF_MHZ_BW50],
        n_table=4096, model=cylinder_phantom(g, 0.02, 30.0),
        noise_sigma=5e-9, noise_seed=0,
        extra=dict(cg_iters=20, alpha=ALPHA_SMALL))


def ring2d(dims=(256, 256, 64)) -> Workload:
    """128-element ring (r = 11 cm), 256x256x64 grid at 0.8 mm, 1 MHz, 0.5-1.5 MHz."""
    g = centred_grid(dims, 0.8e-3)
    R = 0.11
    return Workload(
        name="ring128_grid%dx%dx%d_1MHz" % tuple(dims), c0=1500.0, tx=ring(128, R),
        pairs=all_ordered_pairs(128), grid=g, mask=cylinder_mask(g, 0.75 * R),
        pulses=[sampled_pulse(1.0e6, 1.0)], r_max=[R_MAX[1.0e6]], n_table=4096,
        model=nested_cylinders(g, (0.02, 0.045, 0.07), (15.0, -25.0, 40.0)),
        noise_sigma=5e-9, noise_seed=3, extra=dict(alpha=ALPHA_RING2D))


def slices3d(dims=(256, 256, 160), n_per_ring=256, n_rings=16) -> Workload:
    """256-element ring translated to 16 heights 4 mm apart; pairs within a ring."""
    g = centred_grid(dims, 0.8e-3)
    R = 0.11
    zs = [(k - (n_rings - 1) / 2.0) * 4e-3 for k in range(n_rings)]
    tx = np.concatenate([ring(n_per_ring, R, z) for z in zs])
    pairs = np.concatenate([all_ordered_pairs(n_per_ring, k * n_per_ring)
                            for k in range(n_rings)])
    return Workload(
        name="ring256x16_grid%dx%dx%d_1MHz" % tuple(dims), c0=1500.0, tx=tx,
        pairs=pairs, grid=g, mask=cylinder_mask(g, 0.75 * R),
        pulses=[sampled_pulse(1.0e6, 1.0)], r_max=[R_MAX[1.0e6]], n_table=4096,
        model=gaussian_blobs(g, 32, 0.75 * R, (dims[2] - 1) / 2.0 * 0.8e-3, seed=1),
        extra=dict(lsqr_iters=50))


def multiband(dims=(256, 256, 64)) -> Workload:
    w = ring2d(dims)
    fcs = (0.5e6, 1.0e6, 1.5e6, 2.0e6)
    w.name = "ring128_grid%dx%dx%d_4bands" % tuple(dims)
    w.pulses = [sampled_pulse(f, 1.0) for f in fcs]
    w.r_max = [R_MAX[f] for f in fcs]
    w.noise_seed = 3
    return w


def psf512(dims=(256, 256, 64), n_psf=512) -> Workload:
    w = ring2d(dims)
    w.name = "ring128_grid%dx%dx%d_psf%d" % (tuple(dims) + (n_psf,))
    w.extra["psf_voxels"] = pick_voxels(w.mask, n_psf, seed=2)
    return w


@dataclass
class Workload2D:
    """The 2D approximation: an in-plane grid (``grid`` with one layer at
    z = 0 describes the pixels), the model constant along z over [z0, z1],
    and nz layers for the z integral."""
    name: str
    c0: float
    tx: np.ndarray
    pairs: np.ndarray
    grid: Grid               # in-plane pixels (dims (nx, ny, 1))
    z0: float
    z1: float
    nz: int
    mask: np.ndarray         # [nx * ny] uint8
    pulses: list
    r_max: list
    n_table: int = 4096
    model: np.ndarray | None = None   # [nx * ny] m/s
    noise_sigma: float = 0.0
    noise_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.pairs.shape[0])

    @property
    def n(self) -> int:
        return self.grid.n

    @property
    def n_bands(self) -> int:
        return len(self.pulses)


def small_plane(nz=44) -> Workload2D:
    """2D approximation of the small ring: 24x24 pixels at 2 mm, z over
    +-44 mm (the detour of the longest pair stays below R_max = 18.2 mm
    within |z| < 43.6 mm), 0.5 MHz / 50 % pulse, cylinder phantom."""
    g = centred_grid((24, 24, 1), 2e-3)
    return Workload2D(
        name="ring32_plane24x24_z%d_0.5MHz" % nz, c0=1500.0, tx=ring(32, 0.10),
        pairs=all_ordered_pairs(32), grid=g, z0=-0.044, z1=0.044, nz=nz,
        mask=cylinder_mask(g, None), pulses=[sampled_pulse(0.5e6, 0.5)],
        r_max=[R_MAX_HALF_MHZ_BW50], n_table=4096, model=cylinder_phantom(g, 0.02, 30.0),
        noise_sigma=5e-9, noise_seed=0, extra=dict(alpha=ALPHA_SMALL))


def plane128(nz=60) -> Workload2D:
    """2D approximation of the lab-like ring: 256x256 pixels at 0.8 mm, z
    over +-24 mm (the longest chord's detour reaches R_max = 4.77 mm at
    |z| = 23 mm), 0.8 mm layers, 1 MHz pulse, nested cylinders."""
    g = centred_grid((256, 256, 1), 0.8e-3)
    R = 0.11
    return Workload2D(
        name="ring128_plane256x256_z%d_1MHz" % nz, c0=1500.0, tx=ring(128, R),
        pairs=all_ordered_pairs(128), grid=g, z0=-0.024, z1=0.024, nz=nz,
        mask=cylinder_mask(g, 0.75 * R), pulses=[sampled_pulse(1.0e6, 1.0)],
        r_max=[R_MAX[1.0e6]], n_table=4096,
        model=nested_cylinders(g, (0.02, 0.045, 0.07), (15.0, -25.0, 40.0)),
        noise_sigma=5e-9, noise_seed=3, extra=dict(alpha=ALPHA_RING2D))


WORKLOADS = {
    "small_fp64": small_fp64,
    "ring2d": ring2d,
    "slices3d": slices3d,
    "multiband": multiband,
    "psf512": psf512,
    "small_plane": small_plane,
    "plane128": plane128,
}
