"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This module only draws and shapes input data (noise, blur, gradient orientation,
pasted patterns). It contains none of the extended-correlation arithmetic, so the
oracle and the HIP path can both consume its arrays without sharing any method code.

All arrays are produced in float64 and returned as float32 (the dtype the library
consumes); the oracle upcasts the same float32 values to float64, so both sides
see bit-identical inputs.

Recipes (the paper has no datasets for this path; these stand in for its images):
  * steering in 3D: a volume of U[0,1] noise blurred at sigma 2, a random S^3 filter
            (N(0,1) entries times a Gaussian window) and the rotation field that turns +z
            onto the local gradient of an independent noise volume blurred at sigma 6
            (alpha = its azimuth, beta = its polar angle) with a smooth third Euler angle
            gamma in [-pi, pi) (the orientation field of a volumetric feature detector)
  * joint rotation and scale smoothing: the block image, an anisotropic Gaussian, the vortex
            angle field and a smooth scale field in [1, 2]
  * line-integral convolution: white U[0,1] noise, a long narrow anisotropic Gaussian
            (elongated along x), and the angle of a vortex vector field plus a smooth
            seeded perturbation (stands in for the paper's vector-field figure)
  * image:  U[0,1] noise blurred by a Gaussian (sigma 2, reflect, truncate 4)
  * filter: N(0,1) entries times a Gaussian window
  * theta:  orientation atan2(d/drow, d/dcol) of an independent noise field
            blurred at sigma 8, taken mod 2*pi (the gradient-angle field of the
            pattern-detection application, Sec. 5.1, eq. (theta))
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = [
    "blurred_noise", "random_filter", "theta_field", "scale_field", "block_image",
    "rotation_config", "matching_scene", "scale_config", "batch_shapes",
    "batch_instance", "adjoint_config", "anisotropic_gaussian", "vortex_field", "lic_config",
    "joint_config", "random_filter3", "orientation_rotation_field", "steer3d_config",
]


def blurred_noise(shape, seed, sigma=2.0):
    rng = np.random.default_rng(seed)
    n = rng.random(shape)
    return ndimage.gaussian_filter(n, sigma, mode="reflect", truncate=4.0).astype(np.float32)


def random_filter(S, seed, window_sigma):
    rng = np.random.default_rng(seed)
    R = (S - 1) // 2
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    w = np.exp(-(xx * xx + yy * yy) / (2.0 * window_sigma ** 2))
    return (rng.standard_normal((S, S)) * w).astype(np.float32)


def theta_field(shape, seed, sigma=8.0):
    rng = np.random.default_rng(seed)
    n = ndimage.gaussian_filter(rng.random(shape), sigma, mode="reflect", truncate=4.0)
    gy, gx = np.gradient(n)  # axis 0 = rows (y, downwards), axis 1 = columns (x)
    th = np.mod(np.arctan2(gy, gx), 2.0 * np.pi)
    return th.astype(np.float32)


def scale_field(shape, seed, s_min=1.0, s_max=8.0, sigma=16.0):
    """Per-pixel scale, log-uniform in [s_min, s_max], spatially smooth."""
    rng = np.random.default_rng(seed)
    u = ndimage.gaussian_filter(rng.random(shape), sigma, mode="reflect", truncate=4.0)
    u = (u - u.min()) / max(u.max() - u.min(), 1e-300)
    s = s_min * (s_max / s_min) ** u
    return s.astype(np.float32)


def block_image(shape, seed_noise, seed_blocks, n_blocks=32, side_range=(64, 512)):
    """Blurred noise plus random axis-aligned piecewise-constant blocks."""
    img = blurred_noise(shape, seed_noise).astype(np.float64)
    rng = np.random.default_rng(seed_blocks)
    ny, nx = shape
    for _ in range(n_blocks):
        h = int(rng.integers(side_range[0], side_range[1] + 1))
        w = int(rng.integers(side_range[0], side_range[1] + 1))
        y0 = int(rng.integers(0, max(ny - h, 0) + 1))
        x0 = int(rng.integers(0, max(nx - w, 0) + 1))
        img[y0:y0 + h, x0:x0 + w] += rng.uniform(-0.5, 0.5)
    return img.astype(np.float32)


def rotation_config(n, S, K, seeds=(0, 1, 2)):
    """Image, filter and angle field for a plain rotation run (n x n image, S x S filter).

    The filter window width scales with S like the 15x15 / sigma-4 base case.
    """
    img = blurred_noise((n, n), seeds[0])
    filt = random_filter(S, seeds[1], 4.0 * S / 15.0)
    theta = theta_field((n, n), seeds[2])
    return img, filt, theta, K


def _bilinear_sample(arr, rows, cols):
    return ndimage.map_coordinates(arr, [rows, cols], order=1, mode="constant", cval=0.0)


def matching_scene(n=1024, S=63, n_paste=3, seeds=(10, 13, 14, 15)):
    """Blurred-noise background with a disk pattern pasted at random positions/angles.

    Returns (image, pattern, truth) where truth is a list of (row, col, angle).
    The pattern is rotated by bilinear resampling; a pattern rotated by angle a
    has values P(R_{-a} x), x = (col offset, row offset).
    """
    R = (S - 1) // 2
    bg = blurred_noise((n, n), seeds[0]).astype(np.float64)
    rng = np.random.default_rng(seeds[1])
    pat = ndimage.gaussian_filter(rng.standard_normal((S, S)), 1.5, mode="reflect", truncate=4.0)
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    disk = (xx * xx + yy * yy) <= R * R
    pat = pat - pat[disk].mean()
    pat[~disk] = 0.0
    rng = np.random.default_rng(seeds[2])
    truth = []
    tries = 0
    while len(truth) < n_paste and tries < 10000:
        tries += 1
        r = int(rng.integers(32 + R, n - 32 - R))
        c = int(rng.integers(32 + R, n - 32 - R))
        if all((r - a) ** 2 + (c - b) ** 2 >= 64 ** 2 for a, b, _ in truth):
            truth.append((r, c, float(rng.uniform(0.0, 2.0 * np.pi))))
    for r, c, a in truth:
        ca, sa = np.cos(a), np.sin(a)
        # value at offset x is P(R_{-a} x)
        src_x = ca * xx + sa * yy
        src_y = -sa * xx + ca * yy
        vals = _bilinear_sample(pat, src_y + R, src_x + R)
        win = bg[r - R:r + R + 1, c - R:c + R + 1]
        win[disk] = vals[disk]
    noise = np.random.default_rng(seeds[3]).normal(0.0, 0.05, size=(n, n))
    img = (bg + noise).astype(np.float32)
    return img, pat.astype(np.float32), truth


def scale_config(n=2048, seeds=(20, 21, 22)):
    img = block_image((n, n), seeds[0], seeds[1])
    s = scale_field((n, n), seeds[2])
    return img, s


def batch_shapes(n_inst=256, seed=42, side=(64, 1024), fside=(7, 63), krange=(4, 24)):
    """Uneven instance shapes: square with probability 1/2, sides uniform integers."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_inst):
        if rng.random() < 0.5:
            ny = nx = int(rng.integers(side[0], side[1] + 1))
        else:
            ny = int(rng.integers(side[0], side[1] + 1))
            nx = int(rng.integers(side[0], side[1] + 1))
        smax = min(fside[1], ny, nx)
        smax -= 1 - smax % 2
        S = int(rng.choice(np.arange(fside[0], smax + 1, 2)))
        K = int(rng.integers(krange[0], krange[1] + 1))
        out.append((ny, nx, S, K))
    return out


def batch_instance(i, ny, nx, S):
    img = blurred_noise((ny, nx), 1000 + i)
    filt = random_filter(S, 2000 + i, 4.0 * S / 15.0)
    theta = theta_field((ny, nx), 3000 + i)
    return img, filt, theta


def adjoint_config(batch=16, n=512, S=21, seed_theta=40, seed_filter=41, seed_grad=43):
    imgs = np.stack([blurred_noise((n, n), 400 + i) for i in range(batch)])
    thetas = np.stack([theta_field((n, n), seed_theta + i) for i in range(batch)])
    filt = random_filter(S, seed_filter, 4.0 * S / 15.0)
    g = np.random.default_rng(seed_grad).standard_normal((batch, n, n)).astype(np.float32)
    return imgs, thetas, filt, g


def anisotropic_gaussian(S, sigma_along, sigma_across):
    """exp(-(x^2 / 2 sa^2 + y^2 / 2 sc^2)) on the S x S grid, x = column offset (the long
    axis), y = row offset; peak 1 at the centre."""
    R = (S - 1) // 2
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1].astype(np.float64)
    g = np.exp(-(xx * xx) / (2.0 * sigma_along ** 2) - (yy * yy) / (2.0 * sigma_across ** 2))
    return g.astype(np.float32)


def vortex_field(shape, seed, wobble=0.6, sigma=24.0):
    """Angle (radians, mod 2 pi) of a circular flow around the image centre, perturbed by
    `wobble` times blurred zero-mean noise (unit standard deviation before scaling)."""
    ny, nx = shape
    yy, xx = np.mgrid[0:ny, 0:nx].astype(np.float64)
    base = np.arctan2(yy - (ny - 1) / 2.0, xx - (nx - 1) / 2.0) + np.pi / 2.0
    n = ndimage.gaussian_filter(np.random.default_rng(seed).standard_normal(shape), sigma,
                                mode="reflect", truncate=4.0)
    n = n / max(float(np.std(n)), 1e-300)
    return np.mod(base + wobble * n, 2.0 * np.pi).astype(np.float32)


def lic_config(n=1024, S=31, seeds=(50, 51), sigma_along=8.0, sigma_across=1.5):
    """White noise image, anisotropic Gaussian filter and vortex angle field."""
    img = np.random.default_rng(seeds[0]).random((n, n)).astype(np.float32)
    return img, anisotropic_gaussian(S, sigma_along, sigma_across), vortex_field((n, n), seeds[1])


def joint_config(n=1024, S=31, seeds=(60, 61, 62, 63), sigma_along=1.8, sigma_across=0.7, s_max=2.0):
    """Image (blurred noise plus blocks), anisotropic Gaussian filter, angle field and scale
    field in [1, s_max] (log-uniform, spatially smooth)."""
    img = block_image((n, n), seeds[0], seeds[1])
    filt = anisotropic_gaussian(S, sigma_along, sigma_across)
    theta = vortex_field((n, n), seeds[2])
    s = scale_field((n, n), seeds[3], 1.0, s_max)
    return img, filt, theta, s


def random_filter3(S, seed, window_sigma):
    """S x S x S filter [z][y][x]: N(0,1) entries times a Gaussian window."""
    rng = np.random.default_rng(seed)
    R = (S - 1) // 2
    zz, yy, xx = np.mgrid[-R:R + 1, -R:R + 1, -R:R + 1]
    w = np.exp(-(xx * xx + yy * yy + zz * zz) / (2.0 * window_sigma ** 2))
    return (rng.standard_normal((S, S, S)) * w).astype(np.float32)


def orientation_rotation_field(shape, seed, sigma=6.0):
    """ZYZ Euler angles (alpha, beta, gamma) of the rotation that takes +z to the gradient
    direction of a blurred noise volume, with a smooth third angle gamma."""
    rng = np.random.default_rng(seed)
    n = ndimage.gaussian_filter(rng.random(shape), sigma, mode="reflect", truncate=4.0)
    gz, gy, gx = (np.gradient(n, axis=i) if n.shape[i] > 1 else np.zeros_like(n) for i in range(3))
    alpha = np.arctan2(gy, gx)
    beta = np.arctan2(np.hypot(gx, gy), gz)
    u = ndimage.gaussian_filter(rng.random(shape), sigma, mode="reflect", truncate=4.0)
    u = (u - u.min()) / max(u.max() - u.min(), 1e-300)
    gamma = 2.0 * np.pi * u - np.pi
    return alpha.astype(np.float32), beta.astype(np.float32), gamma.astype(np.float32)


def steer3d_config(n=128, S=15, seeds=(70, 71, 72)):
    """Volume (nz = ny = nx = n or a shape tuple), filter and rotation field."""
    shape = (n, n, n) if np.isscalar(n) else tuple(n)
    vol = ndimage.gaussian_filter(np.random.default_rng(seeds[0]).random(shape), 2.0, mode="reflect",
                                  truncate=4.0).astype(np.float32)
    filt = random_filter3(S, seeds[1], S / 4.0)
    return (vol, filt) + orientation_rotation_field(shape, seeds[2])
