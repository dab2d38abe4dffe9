"""Seeded synthetic workloads.

The only module shared by the GPU path's callers and the oracle's tests: it
draws camera and scene parameters and random ray sets, and holds none of the
method's arithmetic.  Every length is in units of the hole mass M unless a
field says otherwise; the sky sphere sits at 1000 M with 10-degree checker
cells (a procedural stand-in for the paper's NASA/ESA background images,
which are not available).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

R_SKY_IN_M = 1000.0
CHECKER_DEG = 10.0
DISK_POWER = -3.0


@dataclass(frozen=True)
class Scene:
    M: float = 1.0
    r_sky: float = R_SKY_IN_M          # absolute units
    disk: tuple | None = None          # (r_in, r_out), absolute units
    disk_power: float = DISK_POWER
    checker_deg: float = CHECKER_DEG
    sky_tex: object = field(default=None, compare=False)  # (h, w, 4) float32 sky image, or None


@dataclass(frozen=True)
class Camera:
    r: float                           # absolute units
    incl_deg: float
    azim_deg: float
    fov_deg: float
    width: int
    height: int

    @property
    def pixels(self) -> int:
        return self.width * self.height


@dataclass(frozen=True)
class Frame:
    camera: Camera
    scene: Scene
    name: str = ""


def scene_in_m(M: float, disk_in_m=None) -> Scene:
    """Scene whose sky radius and disk radii are given in units of M."""
    disk = None if disk_in_m is None else (disk_in_m[0] * M, disk_in_m[1] * M)
    return Scene(M=M, r_sky=R_SKY_IN_M * M, disk=disk)


# -- the five workloads -------------------------------------------------------

def plain_64() -> Frame:
    """64x64, M = 1, camera at 30 M in the equatorial plane, FOV 60 deg, no
    disk (deterministic)."""
    return Frame(Camera(30.0, 90.0, 0.0, 60.0, 64, 64), scene_in_m(1.0), "plain_64")


def disk_1024(size: int = 1024) -> Frame:
    """1024x1024, M = 1, camera at 50 M, inclination 80 deg, FOV 30 deg, disk
    6-20 M with emissivity r^-3."""
    return Frame(Camera(50.0, 80.0, 0.0, 30.0, size, size), scene_in_m(1.0, (6.0, 20.0)),
                 f"disk_{size}")


def orbit_4k(frames: int = 16, width: int = 3840, height: int = 2160, seed: int = 3) -> list[Frame]:
    """Camera orbit at 4K: per frame M ~ U[0.5, 2], distance ~ U[20, 100] M,
    inclination ~ U[0, 90] deg, azimuth stepping by 360/frames deg; disk 6-30 M;
    FOV 60 deg."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(frames):
        M = float(rng.uniform(0.5, 2.0))
        rho = float(rng.uniform(20.0, 100.0))
        inc = float(rng.uniform(0.0, 90.0))
        az = 360.0 * k / frames
        out.append(Frame(Camera(rho * M, inc, az, 60.0, width, height),
                         scene_in_m(M, (6.0, 30.0)), f"orbit4k_{k}"))
    return out


BATCH_SIZES = (128, 256, 512, 1024, 2048)


def serving_batch(n: int = 512, seed: int = 5, sizes=BATCH_SIZES) -> list[Frame]:
    """Mixed-size render requests: square resolution drawn uniformly from
    ``sizes``, M ~ U[0.5, 2], distance ~ U[15, 200] M, inclination ~ U[0, 90]
    deg, azimuth ~ U[0, 360) deg, disk 6-20 M with probability 1/2, FOV 60."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        s = int(sizes[int(rng.integers(0, len(sizes)))])
        M = float(rng.uniform(0.5, 2.0))
        rho = float(rng.uniform(15.0, 200.0))
        inc = float(rng.uniform(0.0, 90.0))
        az = float(rng.uniform(0.0, 360.0))
        disk = (6.0, 20.0) if rng.uniform() < 0.5 else None
        out.append(Frame(Camera(rho * M, inc, az, 60.0, s, s), scene_in_m(M, disk), f"req{k}"))
    return out


def shrink(frame: Frame, width: int, height: int) -> Frame:
    """Same camera and scene at another resolution (for oracle-sized checks)."""
    return replace(frame, camera=replace(frame.camera, width=width, height=height))


# -- sky images -----------------------------------------------------------------

def sky_texture(width: int = 1024, height: int = 512, seed: int = 7, terms: int = 12,
                stars: int = 400) -> np.ndarray:
    """A seeded procedural equirectangular sky image (float32, (height, width,
    4), alpha 1): a smooth field of low-order waves, periodic in varphi, plus
    small soft spots; a stand-in for the photographs the paper renders behind
    the hole.  Texel (i, j) sits at varphi = 2 pi (i + 1/2) / width,
    theta = pi (j + 1/2) / height."""
    rng = np.random.default_rng(seed)
    ph = 2 * np.pi * (np.arange(width) + 0.5) / width
    th = np.pi * (np.arange(height) + 0.5) / height
    P, T = np.meshgrid(ph, th)
    img = np.zeros((height, width, 4))
    for _ in range(terms):
        m = int(rng.integers(1, 6))          # integer waves in varphi: periodic
        n = float(rng.uniform(0.5, 4.0))
        amp = rng.uniform(0.05, 0.15, 3)
        wave = np.cos(m * P + rng.uniform(0, 2 * np.pi)) * np.sin(n * T + rng.uniform(0, 2 * np.pi))
        img[..., :3] += amp * wave[..., None]
    # soft spots ("stars"), a few texels wide
    for _ in range(stars):
        i, j = int(rng.integers(0, width)), int(rng.integers(0, height))
        rad = rng.uniform(1.5, 3.0)
        c = rng.uniform(0.2, 0.6, 3)
        i0, i1 = max(j - 8, 0), min(j + 9, height)
        di = (np.arange(width) - i + width // 2) % width - width // 2
        dj = np.arange(i0, i1) - j
        g = np.exp(-(dj[:, None] ** 2 + di[None, :] ** 2) / (2 * rad * rad))
        img[i0:i1, :, :3] += g[..., None] * c
    img[..., :3] = np.clip(0.35 + img[..., :3], 0.0, 1.0)
    img[..., 3] = 1.0
    return img.astype(np.float32)


# -- random ray sets -----------------------------------------------------------

def random_rays(n: int, seed: int, r_min: float, r_max: float, aim_scale: float | None = None):
    """Origins uniform in direction with radius ~ U[r_min, r_max]; directions
    uniform on the sphere, or (aim_scale given) pointing at a Gaussian target
    of that scale around the origin of coordinates, so that many rays pass
    near the hole.  Returns (origin, direction) as float64 (n, 3) arrays."""
    rng = np.random.default_rng(seed)
    o = rng.normal(size=(n, 3))
    o *= (rng.uniform(r_min, r_max, n) / np.linalg.norm(o, axis=1))[:, None]
    if aim_scale is None:
        d = rng.normal(size=(n, 3))
    else:
        d = rng.normal(scale=aim_scale, size=(n, 3)) - o
    d /= np.linalg.norm(d, axis=1)[:, None]
    return np.ascontiguousarray(o), np.ascontiguousarray(d)


def surrogate_samples(n: int, seed: int, b_lo: float, b_hi: float, r0_lo: float = 10.0,
                      r0_hi: float = 200.0, max_b_over_r0: float | None = 0.85):
    """(b/M, r0/M) pairs: b log-uniform in [b_lo, b_hi], r0 uniform in
    [r0_lo, r0_hi], keeping b <= max_b_over_r0 * r0 (a camera with a 60-degree
    vertical field of view at 16:9 sees rays up to b = 0.76 r0; nearer b = r0
    the ray starts at its periapsis).  Returns at most n pairs."""
    rng = np.random.default_rng(seed)
    b = np.exp(rng.uniform(np.log(b_lo), np.log(b_hi), n))
    r0 = rng.uniform(r0_lo, r0_hi, n)
    if max_b_over_r0 is not None:
        keep = b <= max_b_over_r0 * r0
        b, r0 = b[keep], r0[keep]
    return b, r0


def capture_samples(n: int, seed: int, b_hi: float, r0_lo: float = 10.0, r0_hi: float = 200.0):
    """(b/M, r0/M) pairs on the capture side: b uniform in [0, b_hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, b_hi, n), rng.uniform(r0_lo, r0_hi, n)
