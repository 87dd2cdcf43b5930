"""Oracle of the BOS displacement check of section 4 (Fig. 4 and eq. 9).

Test infrastructure only (see the package docstring).  Three pieces, each a plain definition:

* ``dot_mean_hits``: per dot, the mean sensor hit of its rays that deposit on the sensor (the
  paper averages the displacements of the rays of one dot; with the same rays traced with and
  without the field, the difference of the two means is that average over the rays deposited in
  both renders).
* ``dot_map``: the scattered per-dot displacements placed on a regular grid by bilinear
  weights.  READING: each dot spreads weight (1 - t)(1 - u), t(1 - u), (1 - t)u, tu onto the four
  nodes around it (t, u its fractional position in the grid cell); a node's value is the
  weighted mean of the displacements it received, empty nodes are NaN.  Weights and weighted
  displacements are summed as integers in units of 2^-32 (round half to even), so the result does
  not depend on the order of the dots.
* ``theory_map``: eq. 9 on the same grid (``orc_bos_theory_map`` in oracle.c).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import DEPOSITED, _ptr, lib

Q24 = float(2 ** 24)
Q32 = float(2 ** 32)


def dot_mean_hits(o, src, rays_per_src, n_threads=0, which=None):
    """Traces every ray of the sources ``which`` (default: all) with the oracle scene ``o``;
    returns (mean [n][2] of the sensor hits of the deposited rays in pixels, NaN where none;
    deposited count [n]) for those sources."""
    src = np.ascontiguousarray(src, dtype=np.float32)
    which = np.arange(src.shape[0]) if which is None else np.asarray(which, dtype=np.int64)
    n = len(which)
    ids = (which[:, None] * int(rays_per_src) + np.arange(int(rays_per_src))[None, :]).ravel().astype(np.int64)
    r = o.trace_ids(src, rays_per_src, ids, n_threads=n_threads)
    dep = (r["status"] == DEPOSITED).reshape(n, rays_per_src)
    px = r["sensor_px"].reshape(n, rays_per_src, 2)
    cnt = dep.sum(axis=1)
    mean = np.full((n, 2), np.nan)
    for s in range(n):
        if cnt[s]:
            mean[s] = px[s][dep[s]].mean(axis=0)
    return mean, cnt


def means_from_sums(sums):
    """Mean hit of each source from per-source sums (int64 [n][4]: sum_x, sum_y, hits, 0 with
    the sums in units of 2^-24 pixel): (sum * 2^-24) / hits in FP64, NaN where hits = 0."""
    out = np.full((len(sums), 2), np.nan)
    for s in range(len(sums)):
        h = int(sums[s][2])
        if h:
            out[s, 0] = (float(int(sums[s][0])) / Q24) / float(h)
            out[s, 1] = (float(int(sums[s][1])) / Q24) / float(h)
    return out


def dot_map(xy, disp, grid):
    """Bilinear map of per-dot displacements.  xy: dot positions [n][2] (m, float32 values as
    in the source list), disp: [n][2] pixels (rows with a NaN are skipped), grid: (x0, y0, dx, dy,
    nx, ny, z_dots).  Returns float32 [ny][nx][2]."""
    x0, y0, dx, dy, nx, ny = grid[:6]
    nx, ny = int(nx), int(ny)
    sw = [[0] * nx for _ in range(ny)]
    sd = [[[0, 0] for _ in range(nx)] for _ in range(ny)]
    for (px, py), (ddx, ddy) in zip(np.asarray(xy, dtype=np.float64), np.asarray(disp, dtype=np.float64)):
        if not (np.isfinite(ddx) and np.isfinite(ddy)):
            continue
        fx = (float(px) - x0) / dx
        fy = (float(py) - y0) / dy
        if not (fx > -1.0 and fy > -1.0 and fx < nx and fy < ny):
            continue
        i = int(np.floor(fx))
        j = int(np.floor(fy))
        t = fx - i
        u = fy - j
        for di, dj, w in ((0, 0, (1.0 - t) * (1.0 - u)), (1, 0, t * (1.0 - u)),
                          (0, 1, (1.0 - t) * u), (1, 1, t * u)):
            ii, jj = i + di, j + dj
            if 0 <= ii < nx and 0 <= jj < ny:
                sw[jj][ii] += round(w * Q32)
                sd[jj][ii][0] += round((w * float(ddx)) * Q32)
                sd[jj][ii][1] += round((w * float(ddy)) * Q32)
    out = np.full((ny, nx, 2), np.nan, dtype=np.float32)
    for j in range(ny):
        for i in range(nx):
            if sw[j][i]:
                out[j, i, 0] = float(sd[j][i][0]) / float(sw[j][i])
                out[j, i, 1] = float(sd[j][i][1]) / float(sw[j][i])
    return out


def theory_map(o, grid, samples):
    """Eq. 9 at the grid nodes (pixels), float64 [ny][nx][2]."""
    x0, y0, dx, dy, nx, ny, z_dots = grid
    out = np.zeros((int(ny), int(nx), 2))
    l = lib()
    l.orc_bos_theory_map.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p]
    l.orc_bos_theory_map(o.h, x0, y0, dx, dy, int(nx), int(ny), z_dots, int(samples), _ptr(out))
    return out


def magnification(o, z_obj):
    """Paraxial lateral magnification of the object plane z_obj."""
    out = np.zeros(2)
    l = lib()
    l.orc_paraxial.argtypes = [C.c_void_p, C.c_double, C.c_void_p]
    l.orc_paraxial(o.h, z_obj, _ptr(out))
    return float(out[1])

