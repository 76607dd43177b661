"""Seeded synthetic inputs for the EDGE pipeline.

This module holds no part of the method's arithmetic: it only draws images
and image sizes.  Both the HIP path's tests and the oracle's tests feed it
the same seeds, so both sides see identical inputs.

The paper (Evaluation) runs EDGE on inputs it does not describe; these
synthetic images stand in for them.  Recipe, per image:

* ``rng = numpy.random.default_rng(SeedSequence([config_seed, index]))``
* noise ``rng.uniform(0, 0.2, (H, W))`` in float64;
* ``n_rect`` rectangles, each drawn in this order: width
  ``integers(max(1, W//16), max(1, W//4) + 1)``, height the same rule on H,
  x0 ``integers(0, W - w + 1)``, y0 ``integers(0, H - h + 1)``, value
  ``uniform(0.5, 1.0)``; painted in draw order (later ones overwrite);
* finally cast to float32.

Image sizes for uneven batches and serving draw each side independently as
``round(exp(uniform(ln lo, ln hi)))`` from ``default_rng(config_seed)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Seeds of the five benchmark workloads.
SEED_SINGLE_256 = 1
SEED_BATCH_1080P = 2
SEED_LARGE_8192 = 3
SEED_UNEVEN_512 = 4
SEED_SERVING = 5


def image(H: int, W: int, config_seed: int, index: int = 0,
          n_rect: int = 8) -> np.ndarray:
    """One synthetic HxW float32 image (noise plus painted rectangles)."""
    rng = np.random.default_rng(np.random.SeedSequence([config_seed, index]))
    img = rng.uniform(0.0, 0.2, (H, W))
    for _ in range(n_rect):
        w = int(rng.integers(max(1, W // 16), max(1, W // 4) + 1))
        h = int(rng.integers(max(1, H // 16), max(1, H // 4) + 1))
        x0 = int(rng.integers(0, W - w + 1))
        y0 = int(rng.integers(0, H - h + 1))
        v = rng.uniform(0.5, 1.0)
        img[y0:y0 + h, x0:x0 + w] = v
    return img.astype(np.float32)


def log_uniform_sizes(n: int, lo: int, hi: int, config_seed: int):
    """n (H, W) pairs, each side log-uniform in [lo, hi], drawn in order."""
    rng = np.random.default_rng(config_seed)
    out = []
    for _ in range(n):
        w = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        h = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append((max(lo, min(hi, h)), max(lo, min(hi, w))))
    return out


@dataclass(frozen=True)
class Workload:
    """A named benchmark workload: image sizes plus pipeline constants."""
    name: str
    sizes: tuple
    seed: int
    n_rect: int
    ksize: int
    sigma: float
    theta: float = 0.1

    @property
    def pixels(self) -> int:
        return sum(h * w for h, w in self.sizes)

    def image(self, i: int) -> np.ndarray:
        h, w = self.sizes[i]
        return image(h, w, self.seed, i, self.n_rect)


def single_256() -> Workload:
    """One 256x256 image, 8 rectangles, 5x5 Gaussian sigma 1.0."""
    return Workload("single-256x256-k5", ((256, 256),), SEED_SINGLE_256, 8,
                    5, 1.0)


def batch_1080p(n: int = 64) -> Workload:
    """n images of 1920x1080 (H=1080, W=1920), 8 rectangles, k5 sigma 1.0."""
    return Workload(f"batch-{n}x1920x1080-k5", ((1080, 1920),) * n,
                    SEED_BATCH_1080P, 8, 5, 1.0)


def large_8192() -> Workload:
    """One 8192x8192 image, 64 rectangles, 7x7 Gaussian sigma 1.5."""
    return Workload("single-8192x8192-k7", ((8192, 8192),), SEED_LARGE_8192,
                    64, 7, 1.5)


@dataclass(frozen=True)
class BandWorkload(Workload):
    """Rows [row0, row0 + H) of one larger image of size src_size: one
    GPU's row band of it, halo rows included."""
    src_size: tuple = (0, 0)
    row0: int = 0

    def image(self, i: int) -> np.ndarray:
        h, w = self.sizes[i]
        full = image(self.src_size[0], self.src_size[1], self.seed, 0, self.n_rect)
        return np.ascontiguousarray(full[self.row0:self.row0 + h, :w])


def band_8192(gpus: int = 8) -> Workload:
    """One GPU's share of the 8192x8192 k7 image split into row bands over
    `gpus` GPUs: the fourth band of 8192/gpus rows with the 5 halo rows
    (blur radius 3 + 2) it needs above and below."""
    rows, halo = 8192 // gpus, 5
    return BandWorkload(f"band-{rows}x8192-of-8192x8192-k7", ((rows + 2 * halo, 8192),),
                        SEED_LARGE_8192, 64, 7, 1.5, 0.1, (8192, 8192), 3 * rows - halo)


def uneven_512(n: int = 512) -> Workload:
    """n images with each side log-uniform in [64, 2048], k5 sigma 1.0."""
    sizes = tuple(log_uniform_sizes(n, 64, 2048, SEED_UNEVEN_512))
    return Workload(f"uneven-{n}-64..2048-k5", sizes, SEED_UNEVEN_512, 8,
                    5, 1.0)


def serving_sizes(n: int = 20000):
    """Request image sizes for the serving workload (sides in [64, 4096])."""
    return log_uniform_sizes(n, 64, 4096, SEED_SERVING)


def poisson_arrivals(n: int, rate: float, seed: int = SEED_SERVING):
    """n arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 1]))
    return np.cumsum(rng.exponential(1.0 / rate, n))


SERVING_POOL = 16
SERVING_POOL_SIDE = 4096


def serving_pool(n: int = SERVING_POOL, side: int = SERVING_POOL_SIDE):
    """The pre-generated source images that serving requests are cut from
    (generating a fresh image per request would cost more than serving it)."""
    return [image(side, side, SEED_SERVING, 1000 + j, 16) for j in range(n)]


def serving_requests(n: int = 20000, pool: int = SERVING_POOL,
                     side: int = SERVING_POOL_SIDE):
    """n requests as (pool index, y0, x0, h, w): the sizes of serving_sizes,
    cut from a pool image at seeded offsets."""
    sizes = serving_sizes(n)
    rng = np.random.default_rng(np.random.SeedSequence([SEED_SERVING, 2]))
    out = []
    for h, w in sizes:
        j = int(rng.integers(0, pool))
        y0 = int(rng.integers(0, side - h + 1))
        x0 = int(rng.integers(0, side - w + 1))
        out.append((j, y0, x0, h, w))
    return out


SEED_SRAD = 6


def speckle(H: int, W: int, config_seed: int = SEED_SRAD, index: int = 0) -> np.ndarray:
    """A positive float32 speckle image for SRAD: the piecewise-constant
    scene of image() times multiplicative gamma(4, 1/4) noise (mean 1),
    plus 0.05 so that every pixel is > 0."""
    scene = image(H, W, config_seed, index, 8).astype(np.float64)
    rng = np.random.default_rng(np.random.SeedSequence([config_seed, index, 7]))
    return (scene * rng.gamma(4.0, 0.25, (H, W)) + 0.05).astype(np.float32)
