"""Seeded synthetic F2M instances: integer 2-D city coordinates.

The paper benchmarks on the VLSI and TSP-Art collections (Sec. 5.3); those
files are not used here.  These generators produce inputs of the same shape
(integer 2-D coordinates, n from 10^3 to 2*10^5) from a seed, for the
uniform and Gaussian-cluster families, plus small structured families
(lattices, separated triangles, duplicates) used as test cases.

This module holds no arithmetic of the method itself: it only draws
coordinates.  Both the oracle's tests and the GPU path's tests use it.

Every generator returns a C-contiguous int32 array of shape (n, 2) holding
(x, y) per city.
"""
from __future__ import annotations

import hashlib
import math

import numpy as np

__all__ = [
    "uniform", "clustered", "lattice", "lattice_jitter", "triangles",
    "square4", "with_duplicates", "batch_sizes", "batch", "digest",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform(n: int, side: int, seed: int) -> np.ndarray:
    """n cities with x, y drawn uniformly from the integers 0..side-1."""
    rng = _rng(seed)
    return np.ascontiguousarray(rng.integers(0, side, size=(n, 2), dtype=np.int64).astype(np.int32))


def clustered(n: int, side: int, seed: int, centres: int = 200,
              sigma_frac: float = 0.02) -> np.ndarray:
    """Gaussian clusters: `centres` centres uniform on the integer square,
    each city picks a centre uniformly and is offset by N(0, sigma^2) per
    axis, sigma = sigma_frac * side, rounded half-to-even; a city that lands
    outside [0, side) is drawn again (same centre, new offset)."""
    rng = _rng(seed)
    cen = rng.integers(0, side, size=(centres, 2), dtype=np.int64).astype(np.float64)
    pick = rng.integers(0, centres, size=n)
    sigma = sigma_frac * side
    out = np.empty((n, 2), dtype=np.int64)
    todo = np.arange(n)
    while todo.size:
        pts = np.rint(cen[pick[todo]] + rng.normal(0.0, sigma, size=(todo.size, 2)))
        ok = np.all((pts >= 0) & (pts < side), axis=1)
        out[todo[ok]] = pts[ok].astype(np.int64)
        todo = todo[~ok]
    return np.ascontiguousarray(out.astype(np.int32))


def lattice(k1: int, k2: int, s: int, origin=(0, 0)) -> np.ndarray:
    """k1 x k2 grid with spacing s (k1*k2 cities)."""
    xs, ys = np.meshgrid(np.arange(k1), np.arange(k2), indexing="ij")
    pts = np.stack([xs.ravel() * s + origin[0], ys.ravel() * s + origin[1]], axis=1)
    return np.ascontiguousarray(pts.astype(np.int32))


def lattice_jitter(k1: int, k2: int, s: int, jitter: int, seed: int) -> np.ndarray:
    """Lattice with each coordinate moved by an integer drawn from
    [-jitter, jitter]; many equal costs remain, so ties are common."""
    rng = _rng(seed)
    pts = lattice(k1, k2, s, origin=(jitter, jitter)).astype(np.int64)
    pts += rng.integers(-jitter, jitter + 1, size=pts.shape)
    return np.ascontiguousarray(pts.astype(np.int32))


def triangles(m: int, gap: int = 100000) -> np.ndarray:
    """m copies of the triangle (0,0), (10,0), (5,9), placed `gap` apart on
    a row.  Each triangle's three sides all round to cost 10."""
    tri = np.array([[0, 0], [10, 0], [5, 9]], dtype=np.int64)
    pts = np.concatenate([tri + np.array([i * gap, 0]) for i in range(m)])
    return np.ascontiguousarray(pts.astype(np.int32))


def square4(s: int = 10) -> np.ndarray:
    """The 4-point square with side s."""
    return np.array([[0, 0], [s, 0], [s, s], [0, s]], dtype=np.int32)


def with_duplicates(n: int, side: int, dup: int, seed: int) -> np.ndarray:
    """Uniform cities where the last `dup` cities repeat earlier ones
    exactly (cost 0 between the copies)."""
    rng = _rng(seed)
    pts = rng.integers(0, side, size=(n, 2), dtype=np.int64)
    src = rng.integers(0, n - dup, size=dup)
    pts[n - dup:] = pts[src]
    return np.ascontiguousarray(pts.astype(np.int32))


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Instance sizes log-uniform in [lo, hi]: floor(exp(U[ln lo, ln hi]))."""
    rng = _rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.floor(np.exp(u)).astype(np.int64)


def batch(count: int, lo: int, hi: int, seed: int, side: int = 1_000_000):
    """A batch of instances: sizes from batch_sizes, first half uniform,
    second half clustered; returns (coords concatenated, offsets[count+1])."""
    ns = batch_sizes(count, lo, hi, seed)
    parts = []
    for i, n in enumerate(ns):
        s = seed * 100003 + i
        parts.append(uniform(int(n), side, s) if i < count // 2 else clustered(int(n), side, s))
    offs = np.zeros(count + 1, dtype=np.int64)
    offs[1:] = np.cumsum(ns)
    return np.ascontiguousarray(np.concatenate(parts)), offs


def digest(coords: np.ndarray) -> str:
    """SHA-256 of the int32 little-endian coordinate bytes."""
    a = np.ascontiguousarray(coords, dtype="<i4")
    return hashlib.sha256(a.tobytes()).hexdigest()
