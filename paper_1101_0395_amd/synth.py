"""Seeded synthetic RGB images standing in for the paper's natural test images.

The paper evaluates on eight photographs (Section 3.1) that are not available
here.  These generators produce uint8 H x W x 3 images with the same sizes and a
comparable fraction of unique colours (29-58 % for the 512 x 512 photographs).
They hold none of the quantizer's arithmetic: they only draw pixels, so both the
CPU oracle and the GPU path can consume the same bytes.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "blobs_on_gradient",
    "smooth_field_blobs",
    "batch_shapes",
    "batch_image",
    "batch_images",
    "C1_SEEDS",
    "C2_SEEDS",
]

# Seed sets used by the tests and the benchmark.
C1_SEEDS = range(100)
C2_SEEDS = range(1, 9)


def _grid(H: int, W: int):
    yy, xx = np.mgrid[0:H, 0:W]
    return yy.astype(np.float64), xx.astype(np.float64)


def blobs_on_gradient(H: int, W: int, seed: int, n_blobs: int = 8) -> np.ndarray:
    """Small test image: linear gradient background with isotropic RGB blobs.

    Background: a linear ramp between two random colours along a random angle.
    Each of ``n_blobs`` blobs is a spatial disc (radius 8-20 % of the short side)
    whose pixels are drawn from an isotropic Gaussian in RGB with mean uniform in
    [0,255]^3 and standard deviation uniform in [10,30].  Later discs overwrite
    earlier ones.  Values are rounded and clipped to [0,255].
    """
    rng = np.random.default_rng(seed)
    yy, xx = _grid(H, W)
    c0 = rng.uniform(0, 255, 3)
    c1 = rng.uniform(0, 255, 3)
    theta = rng.uniform(0, 2 * math.pi)
    t = (xx / max(W - 1, 1) - 0.5) * math.cos(theta) + (yy / max(H - 1, 1) - 0.5) * math.sin(theta)
    t = (t - t.min()) / max(t.max() - t.min(), 1e-12)
    img = c0[None, None, :] + t[..., None] * (c1 - c0)[None, None, :]
    short = min(H, W)
    for _ in range(n_blobs):
        mu = rng.uniform(0, 255, 3)
        sigma = rng.uniform(10, 30)
        r = rng.uniform(0.08, 0.2) * short
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        inside = (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
        cnt = int(inside.sum())
        img[inside] = mu[None, :] + sigma * rng.standard_normal((cnt, 3))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def smooth_field_blobs(H: int, W: int, seed: int, n_blobs: int = 48, rho: float = 0.5,
                       noise: int = 4) -> np.ndarray:
    """Natural-image stand-in: smooth field + Gaussian colour blobs + uniform noise.

    Per channel the background is
    127.5 + A sin(2 pi (fx x/W + fy y/H) + phi) + B ((x/W - 1/2) cos psi + (y/H - 1/2) sin psi)
    with A ~ U[15,35], B ~ U[20,50], fx, fy ~ U[0.25,1.5], phi, psi ~ U[0, 2 pi)
    (amplitudes and frequencies chosen so that a 512 x 512 image holds 1e5-2e5
    unique colours, like the photographs of Section 3.1).
    ``n_blobs`` colour blobs (mean ~ U[0,255]^3, colour standard deviation
    ~ U[5,40]) with Dirichlet(1) mixture weights pi_b cover a fraction ``rho`` of
    the area: blob b is a disc of area pi_b * rho * H * W at a uniform position,
    painted largest first.  Every channel then receives integer noise uniform in
    {-noise..noise}; values are rounded and clipped to [0,255].
    """
    rng = np.random.default_rng(seed)
    yy, xx = _grid(H, W)
    img = np.empty((H, W, 3), dtype=np.float64)
    for c in range(3):
        A = rng.uniform(15, 35)
        B = rng.uniform(20, 50)
        fx, fy = rng.uniform(0.25, 1.5, 2)
        phi, psi = rng.uniform(0, 2 * math.pi, 2)
        img[..., c] = (127.5 + A * np.sin(2 * math.pi * (fx * xx / W + fy * yy / H) + phi)
                       + B * ((xx / W - 0.5) * math.cos(psi) + (yy / H - 0.5) * math.sin(psi)))
    mus = rng.uniform(0, 255, (n_blobs, 3))
    sigmas = rng.uniform(5, 40, n_blobs)
    weights = rng.dirichlet(np.ones(n_blobs))
    order = np.argsort(-weights, kind="stable")
    for b in order:
        area = weights[b] * rho * H * W
        r = math.sqrt(area / math.pi)
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        y0, y1 = max(int(cy - r) - 1, 0), min(int(cy + r) + 2, H)
        x0, x1 = max(int(cx - r) - 1, 0), min(int(cx + r) + 2, W)
        if y0 >= y1 or x0 >= x1:
            continue
        sub_y, sub_x = yy[y0:y1, x0:x1], xx[y0:y1, x0:x1]
        inside = (sub_y - cy) ** 2 + (sub_x - cx) ** 2 <= r * r
        cnt = int(inside.sum())
        if cnt == 0:
            continue
        view = img[y0:y1, x0:x1]
        view[inside] = mus[b][None, :] + sigmas[b] * rng.standard_normal((cnt, 3))
    if noise > 0:
        img += rng.integers(-noise, noise + 1, size=img.shape)
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def batch_shapes(n: int, base_seed: int = 1_000_000, k_choices=(16, 32, 64, 128, 256)):
    """Shapes and palette sizes of a mixed batch of ``n`` images.

    Image i uses seed ``base_seed + i``: long side L = round(exp(U[ln 64, ln 2048])),
    aspect a ~ U[1,2], short side round(L / a), orientation by a fair coin, and K
    uniform over ``k_choices``.  Returns a list of (H, W, K, seed).
    """
    out = []
    for i in range(n):
        seed = base_seed + i
        rng = np.random.default_rng(seed)
        L = int(round(math.exp(rng.uniform(math.log(64), math.log(2048)))))
        a = rng.uniform(1.0, 2.0)
        s = max(int(round(L / a)), 1)
        if rng.integers(0, 2) == 1:
            H, W = L, s
        else:
            H, W = s, L
        K = int(k_choices[int(rng.integers(0, len(k_choices)))])
        out.append((H, W, K, seed))
    return out


def batch_image(H: int, W: int, seed: int) -> np.ndarray:
    """Image of a mixed batch: the natural-image stand-in with its own seed."""
    return smooth_field_blobs(H, W, seed + 7_919)


def _batch_image_args(args):
    H, W, seed = args
    return batch_image(H, W, seed)


def batch_images(shapes, workers: int = 1, threads: bool = False):
    """The images of ``batch_shapes`` output (H, W, K, seed), in order,
    generated by ``workers`` processes (started fresh, so that a caller that
    already uses the GPU passes nothing of it to them), or by ``workers``
    threads of this process if ``threads`` (slower: numpy holds the
    interpreter lock for part of the work)."""
    args = [(H, W, seed) for H, W, _, seed in shapes]
    if workers <= 1 or len(args) <= 1:
        return [_batch_image_args(a) for a in args]
    if threads:
        from concurrent.futures import ThreadPoolExecutor

        with ThreadPoolExecutor(max_workers=workers) as pool:
            return list(pool.map(_batch_image_args, args))
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor

    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as pool:
        return list(pool.map(_batch_image_args, args, chunksize=4))
