"""Seeded synthetic image-deblurring problems.

This module only *draws* test problems: a true image, a point-spread
function (PSF), a noise vector and the blurred noisy data.  It holds none of
the solver's arithmetic.  The forward blur used to synthesise the data is
``scipy.signal.fftconvolve`` on the zero-padded image, a library routine that
neither the CPU oracle nor the HIP library uses.

The paper (Section 5) draws its problems from the IR Tools MATLAB package:
128x128 images, Gaussian / defocus / speckle / shake / motion blurs, and
noise measured as ||eps|| / ||b_true|| (the noise-level definition at the
start of Section 5).  IR Tools and its images are not available here, so
these generators stand in for them with the shapes, sizes and value
distributions of the workloads this library is measured on.

Conventions shared by every consumer:
  * an image X is an n x n array, row index i vertical, column index j
    horizontal, stored row-major;
  * a PSF is a K x K array with K odd, centre (h, h), h = (K - 1) / 2, row
    offset first;
  * the blur is a true convolution with zero boundary conditions:
        (A X)[i, j] = sum_{u,v} P[h+u, h+v] X[i-u, j-v].

All floating point outputs that a GPU consumes (PSF, data b) are rounded to
float32 so that the CPU oracle and the GPU solve exactly the same problem.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.signal


@dataclasses.dataclass
class Problem:
    """One deblurring test problem b = A x_true + eps (eq. (1) of the paper)."""

    n: int
    psf: np.ndarray          # K x K float64 holding float32-representable values
    x_true: np.ndarray       # n x n float64
    b: np.ndarray            # n x n float32 (blurred + noise)
    noise_norm: float        # ||eps||_2 as realised in float32 b
    noise_level: float       # requested ||eps|| / ||b_true||
    lam: float | None        # fixed regularisation parameter, if the workload fixes one
    seed: int
    kind: str

    @property
    def k(self) -> int:
        return int(self.psf.shape[0])


# --------------------------------------------------------------------------
# true images
# --------------------------------------------------------------------------

def true_image(rng: np.random.Generator, n: int) -> np.ndarray:
    """Sum of 8 axis-aligned rectangles and 4 Gaussian bumps, clipped to [0,1].

    Rectangles: top-left corner uniform over pixels, height and width uniform
    integers in [ceil(n/16), ceil(n/3)], clipped to the image, additive value
    U[0,1].  Bumps: centre uniform in [0,n)^2, width sigma ~ U[2,6] pixels,
    amplitude U[0,1].
    """
    x = np.zeros((n, n), dtype=np.float64)
    lo, hi = max(1, math.ceil(n / 16)), max(1, math.ceil(n / 3))
    for _ in range(8):
        i0, j0 = rng.integers(0, n, size=2)
        hh, ww = rng.integers(lo, hi + 1, size=2)
        val = rng.uniform(0.0, 1.0)
        x[i0:i0 + hh, j0:j0 + ww] += val
    ii, jj = np.meshgrid(np.arange(n, dtype=np.float64),
                         np.arange(n, dtype=np.float64), indexing="ij")
    for _ in range(4):
        ci, cj = rng.uniform(0.0, n, size=2)
        s = rng.uniform(2.0, 6.0)
        a = rng.uniform(0.0, 1.0)
        x += a * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2.0 * s * s))
    return np.clip(x, 0.0, 1.0)


# --------------------------------------------------------------------------
# point-spread functions
# --------------------------------------------------------------------------

def _offsets(k: int):
    h = (k - 1) // 2
    y, x = np.meshgrid(np.arange(-h, h + 1, dtype=np.float64),
                       np.arange(-h, h + 1, dtype=np.float64), indexing="ij")
    return y, x  # y = row offset, x = column offset


def _finish(p: np.ndarray) -> np.ndarray:
    """Normalise to unit sum, then round to float32-representable values."""
    p = p / p.sum()
    return p.astype(np.float32).astype(np.float64)


def psf_gaussian(k: int, sx: float, sy: float, theta: float = 0.0) -> np.ndarray:
    """(Rotated, anisotropic) Gaussian on a k x k support, unit sum.

    Rotated coordinates x' = x cos t + y sin t, y' = -x sin t + y cos t;
    value exp(-x'^2/(2 sx^2) - y'^2/(2 sy^2)).
    """
    if k % 2 != 1:
        raise ValueError("PSF support must be odd")
    y, x = _offsets(k)
    c, s = math.cos(theta), math.sin(theta)
    xr = x * c + y * s
    yr = -x * s + y * c
    return _finish(np.exp(-xr * xr / (2 * sx * sx) - yr * yr / (2 * sy * sy)))


def _motion_line(length: float, angle: float, size: int) -> np.ndarray:
    """Unit-sum anti-aliased line segment centred in a size x size grid."""
    h = (size - 1) // 2
    img = np.zeros((size, size), dtype=np.float64)
    m = max(2, int(math.ceil(length * 16)))
    t = (np.arange(m, dtype=np.float64) + 0.5) / m - 0.5
    t = np.concatenate([t, -t])  # symmetric sample set keeps the segment centred
    px = h + t * length * math.cos(angle)
    py = h - t * length * math.sin(angle)
    x0 = np.floor(px).astype(int)
    y0 = np.floor(py).astype(int)
    fx = px - x0
    fy = py - y0
    for dy, wy in ((0, 1 - fy), (1, fy)):
        for dx, wx in ((0, 1 - fx), (1, fx)):
            np.add.at(img, (y0 + dy, x0 + dx), wy * wx)
    return img / img.sum()


def psf_moffat(k: int, alpha: float, beta: float) -> np.ndarray:
    """Radial Moffat turbulence profile (1 + r^2/alpha^2)^(-beta) on a k x k
    support, unit sum; symmetric in both axes."""
    if k % 2 != 1:
        raise ValueError("PSF support must be odd")
    y, x = _offsets(k)
    return _finish((1.0 + (x * x + y * y) / (alpha * alpha)) ** (-beta))


def psf_moffat_motion(k: int, alpha: float, beta: float, length: float,
                      angle: float) -> np.ndarray:
    """Moffat turbulence profile (1 + r^2/alpha^2)^(-beta) convolved with a
    short anti-aliased motion segment, cropped to k x k, unit sum."""
    if k % 2 != 1:
        raise ValueError("PSF support must be odd")
    y, x = _offsets(k)
    moff = (1.0 + (x * x + y * y) / (alpha * alpha)) ** (-beta)
    line = _motion_line(length, angle, 2 * int(math.ceil(length / 2)) + 3)
    p = scipy.signal.convolve2d(moff, line, mode="same", boundary="fill")
    return _finish(np.maximum(p, 0.0))


def psf_defocus(k: int, radius: float) -> np.ndarray:
    """Out-of-focus blur: a uniform disk of the given radius (pixels) centred
    on the k x k support, each pixel weighted by the fraction of its area
    inside the disk (8 x 8 sub-samples), unit sum."""
    if k % 2 != 1:
        raise ValueError("PSF support must be odd")
    y, x = _offsets(k)
    sub = (np.arange(8) + 0.5) / 8 - 0.5
    cover = np.zeros((k, k))
    for dy in sub:
        for dx in sub:
            cover += ((x + dx) ** 2 + (y + dy) ** 2 <= radius * radius)
    return _finish(cover / 64.0)


# --------------------------------------------------------------------------
# data
# --------------------------------------------------------------------------

def _blur_for_data(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    # 'same' keeps the central n x n block of the full linear convolution,
    # i.e. a zero-boundary convolution centred at (h, h).
    return scipy.signal.fftconvolve(x, psf, mode="same")


def _blur_for_data_periodic(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    # the image extended periodically by h on every side, then the 'valid'
    # part of the linear convolution: the periodic convolution centred at
    # (h, h)
    h = (psf.shape[0] - 1) // 2
    return scipy.signal.fftconvolve(np.pad(x, h, mode="wrap"), psf, mode="valid")


def _blur_for_data_reflexive(psf: np.ndarray, x: np.ndarray) -> np.ndarray:
    # the image extended by h on every side by half-sample reflection
    # (numpy's 'symmetric' padding repeats the edge sample), then the 'valid'
    # part of the linear convolution
    h = (psf.shape[0] - 1) // 2
    return scipy.signal.fftconvolve(np.pad(x, h, mode="symmetric"), psf, mode="valid")


def make_problem(n: int, psf: np.ndarray, rng: np.random.Generator,
                 noise_level: float, lam: float | None, seed: int, kind: str,
                 x_true: np.ndarray | None = None, periodic: bool = False,
                 reflexive: bool = False) -> Problem:
    if x_true is None:
        x_true = true_image(rng, n)
    blur = (_blur_for_data_periodic if periodic else
            _blur_for_data_reflexive if reflexive else _blur_for_data)
    b_true = blur(psf, x_true)
    g = rng.standard_normal((n, n))
    eps = noise_level * np.linalg.norm(b_true) * g / np.linalg.norm(g)
    b32 = (b_true + eps).astype(np.float32)
    noise_norm = float(np.linalg.norm(b32.astype(np.float64) - b_true))
    return Problem(n=n, psf=psf, x_true=x_true, b=b32, noise_norm=noise_norm,
                   noise_level=noise_level, lam=lam, seed=seed, kind=kind)


def small_gaussian(seed: int = 0, n: int = 64) -> Problem:
    """64 x 64, separable Gaussian sigma = 2 on a 15 x 15 support, 1% noise,
    lambda = 0.02."""
    rng = np.random.default_rng(seed)
    x = true_image(rng, n)
    psf = psf_gaussian(15, 2.0, 2.0, 0.0)
    return make_problem(n, psf, rng, 0.01, 0.02, seed, "gauss15", x_true=x)


def mid_anisotropic(seed: int = 0, n: int = 256) -> Problem:
    """256 x 256, anisotropic Gaussian (sigma_x = 4, sigma_y = 2, rotated by
    30 degrees) on a 31 x 31 support, 1% noise, lambda = 0.01."""
    rng = np.random.default_rng(seed)
    x = true_image(rng, n)
    psf = psf_gaussian(31, 4.0, 2.0, math.radians(30.0))
    return make_problem(n, psf, rng, 0.01, 0.01, seed, "aniso31", x_true=x)


def large_moffat(seed: int = 0, n: int = 1024, k: int = 63) -> Problem:
    """1024 x 1024, Moffat turbulence (beta = 2.5, alpha ~ U[3,8]) convolved
    with a motion segment (length ~ U[3,9] px, angle ~ U[0,pi)) on a 63 x 63
    support, 2% noise; lambda is chosen by GCV, so none is fixed here."""
    rng = np.random.default_rng(seed)
    x = true_image(rng, n)
    alpha = rng.uniform(3.0, 8.0)
    length = rng.uniform(3.0, 9.0)
    angle = rng.uniform(0.0, math.pi)
    psf = psf_moffat_motion(k, alpha, 2.5, length, angle)
    return make_problem(n, psf, rng, 0.02, None, seed, "moffat63", x_true=x)


def large_moffat_periodic(seed: int = 0, n: int = 1024, k: int = 63) -> Problem:
    """The large Moffat + motion workload of large_moffat (same seed, image
    and PSF draws) with periodic data: b = A x_true + e where A extends the
    image periodically (K <= n)."""
    rng = np.random.default_rng(seed)
    x = true_image(rng, n)
    alpha = rng.uniform(3.0, 8.0)
    length = rng.uniform(3.0, 9.0)
    angle = rng.uniform(0.0, math.pi)
    psf = psf_moffat_motion(k, alpha, 2.5, length, angle)
    return make_problem(n, psf, rng, 0.02, None, seed, "moffat63-periodic", x_true=x,
                        periodic=True)


def large_moffat_reflexive(seed: int = 0, n: int = 1024, k: int = 63) -> Problem:
    """1024 x 1024, radial Moffat turbulence (beta = 2.5, alpha ~ U[3,8],
    the draw of large_moffat without its motion segment, so the PSF is
    symmetric in both axes) on a 63 x 63 support, reflexive data (the image
    extended by half-sample reflection, K <= n), 2% noise."""
    rng = np.random.default_rng(seed)
    x = true_image(rng, n)
    alpha = rng.uniform(3.0, 8.0)
    rng.uniform(3.0, 9.0)          # the motion draws of large_moffat, unused
    rng.uniform(0.0, math.pi)
    psf = psf_moffat(k, alpha, 2.5)
    return make_problem(n, psf, rng, 0.02, None, seed, "moffat63-reflexive", x_true=x,
                        reflexive=True)


def large_moffat_motion_reflexive(seed: int = 0, n: int = 1024, k: int = 63) -> Problem:
    """The large Moffat + motion workload of large_moffat (same seed, image
    and PSF draws; the PSF is not symmetric) with reflexive data: the image
    extended by half-sample reflection (K <= n), 2% noise."""
    rng = np.random.default_rng(seed)
    x = true_image(rng, n)
    alpha = rng.uniform(3.0, 8.0)
    length = rng.uniform(3.0, 9.0)
    angle = rng.uniform(0.0, math.pi)
    psf = psf_moffat_motion(k, alpha, 2.5, length, angle)
    return make_problem(n, psf, rng, 0.02, None, seed, "moffat63-motion-reflexive", x_true=x,
                        reflexive=True)


BATCH_SIZES = (128, 256, 384, 512, 768, 1024)


def mixed_psf(rng: np.random.Generator, n: int, kmax: int = 63):
    """A PSF from the uneven batch's mix: support odd uniform in [15, kmax]
    (at most 2n-1), then by a fair coin a rotated anisotropic Gaussian
    (sigma ~ U[1.5,5], theta ~ U[0,pi)) or the Moffat + motion blur
    (alpha ~ U[3,8], beta 2.5, length ~ U[3,9], angle ~ U[0,pi))."""
    k = int(rng.choice(np.arange(15, kmax + 1, 2)))
    k = min(k, 2 * n - 1)
    if rng.uniform() < 0.5:
        sx, sy = rng.uniform(1.5, 5.0, size=2)
        return psf_gaussian(k, sx, sy, rng.uniform(0.0, math.pi)), f"gauss{k}"
    psf = psf_moffat_motion(k, rng.uniform(3.0, 8.0), 2.5,
                            rng.uniform(3.0, 9.0), rng.uniform(0.0, math.pi))
    return psf, f"moffat{k}"


def batch_problem(index: int, batch_seed: int = 0, sizes=BATCH_SIZES,
                  kmax: int = 63) -> Problem:
    """Problem `index` of the uneven batch: size uniform over `sizes`, PSF from
    `mixed_psf`, noise U[0.5%, 3%]."""
    seed = 10000 * (batch_seed + 1) + index
    rng = np.random.default_rng(seed)
    n = int(rng.choice(np.asarray(sizes)))
    psf, kind = mixed_psf(rng, n, kmax)
    nu = rng.uniform(0.005, 0.03)
    return make_problem(n, psf, rng, nu, None, seed, kind)


TRAIN_SEED0 = 100000      # training groups of the learned-lambda workload
VAL_SEED0 = 120000        # its validation groups


def training_group(group: int, per_psf: int = 8, n: int = 256, seed0: int = TRAIN_SEED0,
                   kmax: int = 63) -> list:
    """Problems of the learned-lambda workload: group `group` draws one PSF
    from the uneven batch's mix (seed seed0 + group) and `per_psf` images
    with their own noise level U[0.5%, 3%]; all n x n."""
    seed = seed0 + group
    rng = np.random.default_rng(seed)
    psf, kind = mixed_psf(rng, n, kmax)
    out = []
    for _ in range(per_psf):
        nu = rng.uniform(0.005, 0.03)
        out.append(make_problem(n, psf, rng, nu, None, seed, kind))
    return out


STUDY_SEED0 = 130000       # problems of the parameter-choice study


def study_problem(kind: str, n: int, noise_level: float, index: int,
                  seed0: int = STUDY_SEED0) -> Problem:
    """A problem of the parameter-choice study: the paper's blur families at
    its noise levels (Section 5: 1% and 10%), drawn like the other workloads.
    kind: "gauss" (rotated anisotropic Gaussian, sigma ~ U[1.5, 4]),
    "defocus" (disk radius ~ U[3, 6]), "motion" (Moffat alpha = 1.5 with a
    motion segment of length ~ U[6, 14]) or "moffat" (the large workload's
    Moffat + motion mix); support 31 for n <= 256, else 63."""
    key = {"gauss": 0, "defocus": 1, "motion": 2, "moffat": 3}[kind]
    seed = seed0 + 1000 * key + 10 * index + (0 if noise_level < 0.05 else 5)
    rng = np.random.default_rng(seed)
    k = 31 if n <= 256 else 63
    if kind == "gauss":
        sx, sy = rng.uniform(1.5, 4.0, size=2)
        psf = psf_gaussian(k, sx, sy, rng.uniform(0.0, math.pi))
    elif kind == "defocus":
        psf = psf_defocus(k, rng.uniform(3.0, 6.0))
    elif kind == "motion":
        psf = psf_moffat_motion(k, 1.5, 2.5, rng.uniform(6.0, 14.0), rng.uniform(0.0, math.pi))
    else:
        psf = psf_moffat_motion(k, rng.uniform(3.0, 8.0), 2.5, rng.uniform(3.0, 9.0),
                                rng.uniform(0.0, math.pi))
    return make_problem(n, psf, rng, noise_level, None, seed, f"{kind}{k}")


def lambda_grid(count: int = 32, lo: float = 1e-4, hi: float = 1.0) -> np.ndarray:
    """Log-spaced grid lo .. hi with `count` points (32 points on [1e-4, 1]
    for the large workload)."""
    return np.logspace(math.log10(lo), math.log10(hi), count)


def random_image(rng: np.random.Generator, n: int, dtype=np.float32) -> np.ndarray:
    """Plain Gaussian random image, for operator-level parity tests."""
    return rng.standard_normal((n, n)).astype(dtype)
