"""Seeded synthetic inputs shaped like the paper's fluorescence workloads.

Both the HIP path and the FP64 oracle consume the arrays built here; this module
holds no arithmetic of the segmentation method itself (no energies, kernels or
particle rules), only image synthesis: shapes painted into a grid plus noise.

The paper's own images (Figs. 3-10) are not available; these stand in for them:

* ``disk2d``   : 128x128 fp32 two-phase piecewise-constant disk with Gaussian
                 noise, initial contour an offset smaller circle.
* ``ellipses2d``: 1024x1024 fp32 piecewise-smooth scene of ramped ellipses with
                 Poisson (shot) noise, the noise model of the paper's PS
                 experiments (Figs. 6-8).
* ``ellipsoids3d``: 256^3 uint16 piecewise-constant volume of rotated ellipsoids
                 with Gaussian noise, shaped like the 3D confocal stack (Fig. 8).
* ``batch2d``  : 64 independent fp32 images of 128-1024 px sides with 5-30
                 noisy disks/ellipses each (the batched workload).
* ``serve_stream``: Poisson arrivals of 2D (256^2-2048^2 fp32) and 3D
                 (64^3-192^3 uint16) piecewise-constant requests (serving).
* small random multi-label cases and straight/curved contours for the tests.

Pixel (x, y[, z]) has its centre at integer coordinates; arrays are indexed
``[z][y][x]`` (x fastest), 2D arrays ``[y][x]``.

Parameters follow the paper's notation: ``E`` is the Sobolev length scale
(interaction radius E/2), ``eps`` the smoothness hyper-parameter (always 1/24
in the paper so the kernel is local), ``lam`` the prior weight lambda.
"""
from __future__ import annotations

import dataclasses
import numpy as np

PC = 0  # piecewise-constant image-generating function
PS = 1  # piecewise-smooth image-generating function (local means)
GAUSS = 0    # Gaussian pixel noise (squared residuals)
POISSON = 1  # Poisson pixel noise (J - I log J)

MODE_SOBOLEV = 0
MODE_L2 = 1


@dataclasses.dataclass
class Workload:
    """One segmentation job: image, initial labels and method parameters."""
    name: str
    image: np.ndarray          # float32 or uint16, shape (ny, nx) or (nz, ny, nx)
    labels: np.ndarray         # int32, same shape; 0 = background
    E: float
    lam: float
    model: int = PC
    ps_radius: int = 0
    eps: float = 1.0 / 24.0
    iterations: int = 100
    max_labels: int = 2
    noise: int = GAUSS
    topo: int = 0              # 1: ranked acceptance with topological control
    psf_sigma: float = 0.0     # > 0: deconvolving model, Gaussian PSF of this width (pixels)
    tile: int = 0              # cell shape: 0 default, 1 wide (sobrc.TILE_*)

    @property
    def ndim(self) -> int:
        return self.image.ndim

    @property
    def dims_xyz(self):
        """(nx, ny, nz) with nz = 1 for 2D."""
        s = self.image.shape
        if len(s) == 2:
            return s[1], s[0], 1
        return s[2], s[1], s[0]


def _grid2d(ny, nx):
    y, x = np.mgrid[0:ny, 0:nx]
    return x.astype(np.float64), y.astype(np.float64)


def disk2d(seed: int = 0, n: int = 128, r_true: float = 30.0, r_init: float = 20.0,
           offset: float = 8.0, sigma: float = 0.3, E: float = 8.0, lam: float = 0.18,
           iterations: int = 100) -> Workload:
    """128x128 fp32: disk of radius 30 px, intensity 1.0 on background 0.0,
    Gaussian noise sigma 0.3; initial contour a radius-20 circle offset by 8 px
    in +x.  Piecewise-constant model, kernel cutoff 4 px (E = 8)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = _grid2d(n, n)
    c = (n // 2, n // 2)
    truth = (x - c[0]) ** 2 + (y - c[1]) ** 2 <= r_true ** 2
    img = truth.astype(np.float64) + rng.normal(0.0, sigma, size=(n, n))
    lab = ((x - c[0] - offset) ** 2 + (y - c[1]) ** 2 <= r_init ** 2).astype(np.int32)
    return Workload("disk2d_128", img.astype(np.float32), lab, E=E, lam=lam,
                    model=PC, iterations=iterations)


def _ellipse_masks(rng, n, count, axes_lo, axes_hi, margin):
    """Yield (center, semi-axes, angle) for random ellipses inside the frame."""
    shapes = []
    for _ in range(count):
        a, b = rng.uniform(axes_lo, axes_hi, size=2)
        phi = rng.uniform(0.0, np.pi)
        cx, cy = rng.uniform(margin, n - margin, size=2)
        shapes.append((cx, cy, a, b, phi))
    return shapes


def _inside_ellipse(x, y, cx, cy, a, b, phi, shrink=0.0):
    c, s = np.cos(phi), np.sin(phi)
    u = (x - cx) * c + (y - cy) * s
    v = -(x - cx) * s + (y - cy) * c
    aa, bb = max(a - shrink, 0.5), max(b - shrink, 0.5)
    return (u / aa) ** 2 + (v / bb) ** 2 <= 1.0


def ellipses2d(seed: int = 1, n: int = 1024, count: int = 40, photons: float = 20.0,
               E: float = 12.0, ps_radius: int = 8, lam: float = 0.1,
               iterations: int = 200) -> Workload:
    """1024x1024 fp32 piecewise-smooth scene: 40 ellipses (semi-axes 20-80 px,
    random angle, painter's order), each with a linear intensity ramp 0.5 -> 2.0
    along a random direction across the ellipse, background 0.2, Poisson noise at
    mean photon count 20.  Initial labels: the ellipses shrunk by 2 px."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = _grid2d(n, n)
    J = np.full((n, n), 0.2)
    lab = np.zeros((n, n), dtype=np.int32)
    for (cx, cy, a, b, phi) in _ellipse_masks(rng, n, count, 20.0, 80.0, 80.0):
        theta = rng.uniform(0.0, 2 * np.pi)
        d = np.array([np.cos(theta), np.sin(theta)])
        # half-width of the ellipse along d (support function)
        du = d[0] * np.cos(phi) + d[1] * np.sin(phi)
        dv = -d[0] * np.sin(phi) + d[1] * np.cos(phi)
        h = np.sqrt((a * du) ** 2 + (b * dv) ** 2)
        x0, x1 = int(max(cx - 82, 0)), int(min(cx + 83, n))
        y0, y1 = int(max(cy - 82, 0)), int(min(cy + 83, n))
        xs, ys = x[y0:y1, x0:x1], y[y0:y1, x0:x1]
        m = _inside_ellipse(xs, ys, cx, cy, a, b, phi)
        proj = (xs - cx) * d[0] + (ys - cy) * d[1]
        ramp = 0.5 + 1.5 * np.clip((proj + h) / (2 * h), 0.0, 1.0)
        J[y0:y1, x0:x1][m] = ramp[m]
        mi = _inside_ellipse(xs, ys, cx, cy, a, b, phi, shrink=2.0)
        lab[y0:y1, x0:x1][mi] = 1
    img = rng.poisson(photons * J).astype(np.float64) / photons
    return Workload("ellipses2d_1024", img.astype(np.float32), lab, E=E, lam=lam,
                    model=PS, ps_radius=ps_radius, iterations=iterations)


def _random_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoids3d(seed: int = 2, n: int = 256, count: int = 25, fg: float = 800.0,
                 bg: float = 200.0, sigma: float = 120.0, E: float = 6.0,
                 lam: float = 28800.0, iterations: int = 150,
                 axes=(10.0, 40.0), margin: float = 40.0) -> Workload:
    """256^3 uint16 piecewise-constant volume: 25 ellipsoids (semi-axes 10-40
    voxels, uniform random rotations) at intensity 800 on background 200, Gaussian
    noise sigma 120, rounded and clipped to uint16.  Initial labels: the
    ellipsoids shrunk by 2 voxels.  Kernel cutoff 3 voxels (E = 6)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    J = np.full((n, n, n), bg, dtype=np.float32)
    lab = np.zeros((n, n, n), dtype=np.int32)
    amax = axes[1]
    for _ in range(count):
        semi = rng.uniform(axes[0], axes[1], size=3)
        R = _random_rotation(rng)
        c = rng.uniform(margin, n - margin, size=3)  # (x, y, z)
        lo = np.maximum(np.floor(c - amax - 1).astype(int), 0)
        hi = np.minimum(np.ceil(c + amax + 2).astype(int), n)
        zz, yy, xx = np.mgrid[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        p = np.stack([xx - c[0], yy - c[1], zz - c[2]], axis=-1).astype(np.float64)
        q = p @ R  # body-frame coordinates
        r2 = ((q / semi) ** 2).sum(-1)
        inside = r2 <= 1.0
        sub = J[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub[inside] = fg
        s2 = np.maximum(semi - 2.0, 0.5)
        inside2 = ((q / s2) ** 2).sum(-1) <= 1.0
        sl = lab[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sl[inside2] = 1
    noise = rng.normal(0.0, sigma, size=J.shape).astype(np.float32)
    img = np.clip(np.rint(J + noise), 0, 65535).astype(np.uint16)
    return Workload(f"ellipsoids3d_{n}", img, lab, E=E, lam=lam, model=PC,
                    iterations=iterations)


def random_multilabel(seed: int, shape, n_labels: int = 3, dtype=np.float32,
                      blobs: bool = True, E: float = 6.0, lam: float = 0.5,
                      model: int = PC, ps_radius: int = 2, noise: int = GAUSS) -> Workload:
    """Small random image with several labels, for brute-force checks.

    With ``blobs`` the labels are a few random boxes (contours with both straight
    and corner pieces); without, every pixel gets an independent random label
    (the worst case for several particles per pixel).  With Poisson noise the
    image holds photon counts with mean 4 + 6 * label (zero counts occur)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if blobs:
        lab = np.zeros(shape, dtype=np.int32)
        for l in range(1, n_labels):
            for _ in range(2):
                lo = [rng.integers(0, s) for s in shape]
                hi = [min(s, a + rng.integers(1, max(2, s // 2 + 1))) for a, s in zip(lo, shape)]
                lab[tuple(slice(a, b) for a, b in zip(lo, hi))] = l
    else:
        lab = rng.integers(0, n_labels, size=shape).astype(np.int32)
    if noise == POISSON:
        img = rng.poisson(4.0 + 6.0 * lab.astype(np.float64)).astype(dtype)
    elif dtype == np.uint16:
        img = rng.integers(0, 1000, size=shape).astype(np.uint16)
    else:
        img = (lab.astype(np.float64) * 0.7 + rng.normal(0.0, 0.4, size=shape)).astype(np.float32)
    return Workload(f"random_{'x'.join(map(str, shape))}_{seed}", img, lab, E=E, lam=lam,
                    model=model, ps_radius=ps_radius, max_labels=n_labels, noise=noise)


def half_plane(shape, cut: int, axis: int = 0, dtype=np.float32, E: float = 6.0) -> Workload:
    """Straight two-sided contour: label 1 where the coordinate along ``axis``
    (0 = slowest array axis) is below ``cut``."""
    lab = np.zeros(shape, dtype=np.int32)
    sl = [slice(None)] * len(shape)
    sl[axis] = slice(0, cut)
    lab[tuple(sl)] = 1
    img = lab.astype(dtype) if dtype != np.uint16 else (lab * 100).astype(np.uint16)
    return Workload(f"half_plane_{'x'.join(map(str, shape))}", img, lab, E=E, lam=0.0)


def digital_disk(n: int, radius: float, E: float, center=None) -> Workload:
    """Digital disk of the given radius in an n x n frame (label 1 inside)."""
    x, y = _grid2d(n, n)
    c = (n / 2.0, n / 2.0) if center is None else center
    lab = ((x - c[0]) ** 2 + (y - c[1]) ** 2 <= radius ** 2).astype(np.int32)
    return Workload(f"disk_{n}_{radius}", lab.astype(np.float32), lab, E=E, lam=0.0)

def blobs2d(seed: int = 100, side_lo: int = 128, side_hi: int = 1024, E: float = 8.0,
            lam: float = 0.18, iterations: int = 200, square: bool = False) -> Workload:
    """One image of the batched workload: fp32, nx and ny uniform in
    [side_lo, side_hi] (one side for both if square), 5-30 disks or ellipses
    (semi-axes from 6 px up to 6 + 8% of the short side, painter's order) of
    intensity 1.0 on background 0.0, Gaussian noise sigma uniform in
    [0.2, 0.5].  Initial labels: the shapes shrunk by 2 px.
    Piecewise-constant model, E = 8."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if square:
        nx = ny = int(rng.integers(side_lo, side_hi + 1))
    else:
        nx, ny = (int(v) for v in rng.integers(side_lo, side_hi + 1, size=2))
    count = int(rng.integers(5, 31))
    sigma = float(rng.uniform(0.2, 0.5))
    truth = np.zeros((ny, nx), bool)
    lab = np.zeros((ny, nx), dtype=np.int32)
    amax = 6.0 + 0.08 * min(nx, ny)
    for _ in range(count):
        a = rng.uniform(6.0, amax)
        b = a if rng.random() < 0.5 else rng.uniform(6.0, amax)  # disk or ellipse
        phi = rng.uniform(0.0, np.pi)
        cx, cy = rng.uniform(amax, nx - amax), rng.uniform(amax, ny - amax)
        r = int(np.ceil(max(a, b))) + 1
        x0, x1 = max(int(cx) - r, 0), min(int(cx) + r + 2, nx)
        y0, y1 = max(int(cy) - r, 0), min(int(cy) + r + 2, ny)
        xs, ys = _grid2d(y1 - y0, x1 - x0)
        xs, ys = xs + x0, ys + y0
        truth[y0:y1, x0:x1] |= _inside_ellipse(xs, ys, cx, cy, a, b, phi)
        lab[y0:y1, x0:x1][_inside_ellipse(xs, ys, cx, cy, a, b, phi, shrink=2.0)] = 1
    img = truth.astype(np.float32) + rng.normal(0.0, sigma, size=(ny, nx)).astype(np.float32)
    return Workload(f"blobs2d_{seed}", img.astype(np.float32), lab, E=E, lam=lam, model=PC,
                    iterations=iterations)


def deconv2d(seed: int = 11, n: int = 512, psf_sigma: float = 15.0, count: int = 6,
             noise: float = 0.05, E: float = 8.0, lam: float = 1e-3, iterations: int = 100) -> Workload:
    """Blurred 2D scene for the deconvolving model (after the paper's
    deconvolution example): n x n fp32, `count` disks or ellipses (semi-axes
    25-70 px, painter's order) of intensity 1.0 on background 0.2, blurred by
    a Gaussian PSF of width psf_sigma (zero outside the image, truncated at
    3 sigma), Gaussian noise of the given sigma.  Initial labels: the shapes
    shrunk by 6 px.  Piecewise-constant deconvolving model, E = 8."""
    from scipy import ndimage
    rng = np.random.Generator(np.random.PCG64(seed))
    truth = np.zeros((n, n), bool)
    lab = np.zeros((n, n), dtype=np.int32)
    for _ in range(count):
        a = rng.uniform(25.0, 70.0)
        b = a if rng.random() < 0.5 else rng.uniform(25.0, 70.0)
        phi = rng.uniform(0.0, np.pi)
        cx, cy = rng.uniform(80.0, n - 80.0), rng.uniform(80.0, n - 80.0)
        xs, ys = _grid2d(n, n)
        truth |= _inside_ellipse(xs, ys, cx, cy, a, b, phi)
        lab[_inside_ellipse(xs, ys, cx, cy, a, b, phi, shrink=6.0)] = 1
    scene = 0.2 + 0.8 * truth.astype(np.float64)
    blurred = ndimage.gaussian_filter(scene, psf_sigma, mode="constant", cval=0.0, truncate=3.0)
    img = (blurred + rng.normal(0.0, noise, size=(n, n))).astype(np.float32)
    return Workload(f"deconv2d_{n}", img, lab, E=E, lam=lam, model=PC, iterations=iterations,
                    psf_sigma=psf_sigma)


def batch2d(n_images: int = 64, seed0: int = 100) -> list:
    """The batched workload: n_images independent blobs2d images, seeds
    seed0 .. seed0 + n_images - 1."""
    return [blobs2d(seed0 + k) for k in range(n_images)]


def serve_stream(n_requests: int = 120, rate: float = 50.0, seed: int = 7):
    """The serving workload: a Poisson arrival stream (exponential gaps of mean
    1/rate seconds) of independent segmentation requests, 80% 2D fp32 square
    images of side 256-2048 (blobs2d) and 20% 3D uint16 cubes of side 64-192
    (ellipsoids3d: 3-12 ellipsoids, semi-axes 6 up to 6 + 12% of the side,
    800 on 200, Gaussian noise 120).  Returns [(arrival seconds, Workload)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        sub = int(rng.integers(0, 2 ** 31))
        if rng.random() < 0.8:
            w = blobs2d(sub, side_lo=256, side_hi=2048, square=True)
        else:
            n = int(rng.integers(64, 193))
            amax = 6.0 + 0.12 * n
            w = ellipsoids3d(sub, n=n, count=int(rng.integers(3, 13)), axes=(6.0, amax),
                             margin=amax + 2.0)
        w.name = f"req{k}_{w.name}"
        out.append((t, w))
    return out


CONFIGS = {
    "disk2d_128": disk2d,
    "ellipses2d_1024": ellipses2d,
    "ellipsoids3d_256": ellipsoids3d,
    "deconv2d_512": deconv2d,
}


def make(name: str, seed: int | None = None) -> Workload:
    """Build a named workload with its default seed (or the given one)."""
    fn = CONFIGS[name]
    return fn() if seed is None else fn(seed=seed)
