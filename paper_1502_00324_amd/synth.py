"""Seeded synthetic grayscale images (input generator only).

Stand-ins for the paper's test photographs, which are not available: 1/f^2
spectral noise (natural-image-like spatial correlation) plus filled
rectangles at uniform gray levels (flat, zero-entropy areas that exercise the
entropy filter and produce exact ties).  This module holds none of the
encoder's arithmetic; the tests feed its bytes to the GPU path and to the
oracle alike.

Recipe, in draw order from numpy's PCG64 ``default_rng(seed)``:
  1. phases: H x W uniform on [0, 2 pi);
  2. amplitude 1/|f| on the ``fftfreq`` grid (power ~ 1/f^2), 0 at DC;
     real part of the inverse FFT, rescaled linearly to [0, 255];
  3. per rectangle: width in [max(2, W//32), W//4], height likewise from H,
     top-left x in [0, W-w], y in [0, H-h], gray in [0, 255] (all integer,
     inclusive), painted in order;
  4. np.rint, clip to [0, 255], uint8.
"""
from __future__ import annotations

import hashlib

import numpy as np


def make_image(seed: int, width: int, height: int, n_rect: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    fy = np.fft.fftfreq(height)[:, None]
    fx = np.fft.fftfreq(width)[None, :]
    f = np.sqrt(fx * fx + fy * fy)
    amp = np.zeros_like(f)
    amp[f > 0] = 1.0 / f[f > 0]
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(height, width))
    img = np.real(np.fft.ifft2(amp * np.exp(1j * phase)))
    lo, hi = img.min(), img.max()
    img = (img - lo) * (255.0 / (hi - lo)) if hi > lo else np.zeros_like(img)
    for _ in range(n_rect):
        w = int(rng.integers(max(2, width // 32), max(2, width // 4), endpoint=True))
        h = int(rng.integers(max(2, height // 32), max(2, height // 4), endpoint=True))
        x = int(rng.integers(0, width - w, endpoint=True))
        y = int(rng.integers(0, height - h, endpoint=True))
        g = int(rng.integers(0, 255, endpoint=True))
        img[y:y + h, x:x + w] = g
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def batch_shapes(seeds, sides=tuple(range(128, 1025, 64)), shape_seed: int = 4242):
    """(width, height) per image of a mixed-size batch: side uniform from
    ``sides``, aspect uniform from {1:1, 2:1}; 2:1 means (side, side // 2)."""
    rng = np.random.default_rng(shape_seed)
    out = []
    for _ in seeds:
        s = int(rng.choice(sides))
        wide = bool(rng.integers(0, 2))
        out.append((s, s // 2) if wide else (s, s))
    return out


def sha256(img: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(img).tobytes()).hexdigest()
