"""O(N^2) brute-force neighbour sets (numpy), for tiny inputs.

Two predicates, each the plain definition of "j is a neighbour of i"
(|r_ij| < 2h, j != i; Section 2.2, support 0 <= q <= 2):

* FP64: d = r_j - r_i in float64 and r^2 = (dx dx + dy dy) + dz dz, each
  operation rounded once (numpy never contracts), compared with 4h^2.
* Mixed (FP32 cell + offset): a particle's position is stored as an integer
  cell coordinate c (floor((x - origin)/cs), clamped to the grid) and an FP32
  offset o from that cell's centre, computed in float64 and rounded once.  The
  displacement is d = fl32(fl32(o_j + (c_j - c_i) cs32) - o_i) per axis and
  r^2 = fma32(dz, dz, fma32(dy, dy, fl32(dx^2))) with fma32 a fused
  multiply-add rounded once to FP32, compared with fl32(4h^2).  This is the
  decision the mixed-precision path takes, so the two sets are compared
  bit-exactly.
"""
from __future__ import annotations

from typing import Sequence, Set, Tuple

import numpy as np


def fma32(a, b, c) -> np.ndarray:
    """a * b + c for float32 arrays, rounded once to float32 (to nearest,
    ties to even).  The product is exact in float64; the float64 sum s and its
    exact error e (Knuth's two-sum) give the exact value s + e, and rounding s
    to float32 is already correct unless s lies exactly halfway between two
    float32 values with e != 0, where e decides the side."""
    a, b, c = (np.asarray(v, np.float32) for v in (a, b, c))
    p = a.astype(np.float64) * b.astype(np.float64)
    c64 = c.astype(np.float64)
    s = p + c64
    bb = s - p
    e = (p - (s - bb)) + (c64 - bb)
    r = s.astype(np.float32)
    rd = r.astype(np.float64)
    # the float32 neighbour of r on s's side, and the midpoint between them
    other = np.nextafter(r, np.where(s > rd, np.float32(np.inf), np.float32(-np.inf)))
    mid = (rd + other.astype(np.float64)) * 0.5
    fix = (s != rd) & (s == mid) & (e != 0)
    up = e > 0          # the exact value lies above the midpoint
    hi = np.maximum(r, other)
    lo = np.minimum(r, other)
    return np.where(fix, np.where(up, hi, lo), r).astype(np.float32)


def pairs_fp64(x, y, z, h: float) -> Set[Tuple[int, int]]:
    x, y, z = (np.asarray(a, np.float64) for a in (x, y, z))
    dx = x[None, :] - x[:, None]
    dy = y[None, :] - y[:, None]
    dz = z[None, :] - z[:, None]
    r2 = (dx * dx + dy * dy) + dz * dz
    ok = r2 < 4.0 * h * h
    np.fill_diagonal(ok, False)
    i, j = np.nonzero(ok)
    return set(zip(i.tolist(), j.tolist()))


def cell_coords(v, o: float, cs: float, n: int) -> np.ndarray:
    f = np.floor((np.asarray(v, np.float64) - o) / cs)
    f = np.where(np.isnan(f), 0.0, f)
    return np.clip(f, 0, n - 1).astype(np.int64)


def upper_half(v, o: float, cs: float, n: int) -> np.ndarray:
    """1 where the position lies in the upper half of its (unclamped) cell
    along this axis, 0 elsewhere and where the cell index is clamped."""
    t = (np.asarray(v, np.float64) - o) / cs
    f = np.floor(t)
    ok = (f >= 0) & (f <= n - 1)
    return (ok & (t - f >= 0.5)).astype(np.int64)


def cells_and_offsets(x, y, z, origin: Sequence[float], cs: float,
                      dims: Sequence[int]):
    cs_ = float(cs)
    out_c, out_o = [], []
    for v, o, n in zip((x, y, z), origin, dims):
        c = cell_coords(v, o, cs_, n)
        t = np.asarray(v, np.float64) - o
        ctr = (c.astype(np.float64) + 0.5) * cs_
        out_c.append(c)
        out_o.append((t - ctr).astype(np.float32))
    return out_c, out_o


def pairs_mixed(x, y, z, h: float, origin, cs: float, dims, stencil: bool = False
                ) -> Set[Tuple[int, int]]:
    """Every pair the FP32 cell + offset predicate accepts, over all cells
    (stencil=True: only pairs whose cells differ by at most one per axis, the
    27 cells a cell-list search visits)."""
    (cx, cy, cz), (ox, oy, oz) = cells_and_offsets(x, y, z, origin, cs, dims)
    cs32 = np.float64(np.float32(cs))
    d = []
    for c, o in ((cx, ox), (cy, oy), (cz, oz)):
        dc = (c[None, :] - c[:, None]).astype(np.float64)
        shifted = (o[None, :].astype(np.float64) + dc * cs32).astype(np.float32)
        d.append(shifted - o[:, None])            # float32 - float32
    dx, dy, dz = d
    r2 = fma32(dz, dz, fma32(dy, dy, dx * dx))     # all float32
    assert r2.dtype == np.float32
    ok = r2 < np.float32(4.0 * h * h)
    near = ((np.abs(cx[None, :] - cx[:, None]) <= 1)
            & (np.abs(cy[None, :] - cy[:, None]) <= 1)
            & (np.abs(cz[None, :] - cz[:, None]) <= 1))
    if stencil:
        ok &= near
    np.fill_diagonal(ok, False)
    i, j = np.nonzero(ok)
    return set(zip(i.tolist(), j.tolist()))


def adversarial_cloud(seed: int, params, n_random: int = 600):
    """Tiny point set with the hard cases: points exactly on cell faces,
    pairs at exactly 2h along an axis, coincident points, points outside the
    grid on every side, and a random filler."""
    rng = np.random.default_rng(seed)
    o = np.asarray(params["origin"], np.float64)
    cs = float(params["cell_size"])
    dims = np.asarray(params["dims"])
    h = float(params["h"])
    hi = o + dims * cs
    pts = [rng.uniform(o + cs, hi - cs, size=(n_random, 3))]
    # on cell faces
    k = rng.integers(1, dims - 1, size=(40, 3))
    face = o + k * cs
    jit = rng.uniform(0, cs, size=(40, 3))
    for ax in range(3):
        q = o + k * cs + jit
        q[:, ax] = face[:, ax]
        pts.append(q)
    # pairs exactly 2h apart along each axis, and just inside / outside
    base = rng.uniform(o + 2 * cs, hi - 2 * cs, size=(20, 3))
    for ax in range(3):
        for dd in (2.0 * h, np.nextafter(2.0 * h, 0.0), np.nextafter(2.0 * h, 4.0 * h)):
            q = base.copy()
            q[:, ax] += dd
            pts.append(base.copy())
            pts.append(q)
    # coincident points
    c = rng.uniform(o + cs, hi - cs, size=(10, 3))
    pts += [c, c.copy()]
    # outside the grid on every side (clamped for binning)
    for ax in range(3):
        q = rng.uniform(o + cs, hi - cs, size=(8, 3))
        q[:, ax] = o[ax] - rng.uniform(0.0, 0.5 * h, size=8)
        pts.append(q)
        q2 = q.copy()
        q2[:, ax] = hi[ax] + rng.uniform(0.0, 0.5 * h, size=8)
        pts.append(q2)
        pts.append(q2 + np.array([0.3 * h, 0.2 * h, 0.1 * h]))
    p = np.concatenate(pts, axis=0)
    return p[:, 0].copy(), p[:, 1].copy(), p[:, 2].copy()
