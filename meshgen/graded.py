"""Graded coastal workload: a conforming triangulation of a 2:1-balanced
quadtree refined toward a seeded fractal coastline and three river channels
(no solver arithmetic).

Domain: 80 x 60 root cells of 15.36 km (1228.8 km x 921.6 km).  A cell is
split while its size exceeds h(d) = min(15.36 km, 30 m + gamma d), d the
distance from the cell to the nearest coastline or river point, down to
level 9 (30 m).  The tree is then 2:1 balanced across cell sides and every
leaf is cut into a fan of triangles around its centre through its corners
and the midpoints of sides shared with finer neighbours, which makes the
mesh conforming.

Bathymetry (positive down) from the signed distance to the coast plus
seeded multi-octave noise: ocean to about -4000 m, land rising to +50 m
above the coastline with noise that fades out near the rivers (valleys),
river channels 300 m wide, 3 m below the smooth land profile and at least
3 m below the datum at the coast.  Manning 0.02 in the
ocean and rivers, 0.05 on land.  The tidal ocean boundary is every domain
boundary edge in the ocean (south side and the ocean parts of the west and
east sides), slot 0: 0.5 m amplitude, 44,712 s period.  Each river enters
through the north boundary edges of its channel (slots 1-3) with
q = -1 m^2/s.  Gridded rain on an 11.12 km (0.1 degree) lattice: 20 Gaussian
cells, peak 20-100 mm/h, radius 20-80 km, hourly records drifting 5 m/s.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from .generators import LAND, OCEAN, RIVER, Mesh, Scenario, default_params, gridded_field, seed_for

ROOT = 15360.0
NRX, NRY = 80, 60
LMAX = 9                       # 15360 / 2^9 = 30 m


class Features:
    """Seeded coastline y = yc(x) and river polylines."""

    def __init__(self, seed):
        rng = np.random.default_rng(seed)
        self.Lx, self.Ly = NRX * ROOT, NRY * ROOT
        # coastline: mean at 62% of the height, fractal wiggle (power
        # spectrum slope -2: amplitude halves per octave; 7 octaves,
        # wavelengths from 400 km down to 6.25 km)
        k = 2 * np.pi / (400e3 / 2.0 ** np.arange(7))
        self.c_amp = 60e3 / 2.0 ** np.arange(7)
        self.c_k = k
        self.c_ph = rng.uniform(0, 2 * np.pi, 7)
        self.y0 = 0.62 * self.Ly
        # rivers: start on the north boundary, wander south to the coast
        self.rivers = []
        xs = rng.uniform(0.15, 0.85, 3) * self.Lx
        for r in range(3):
            x, y = xs[r], self.Ly
            pts = [(x, y)]
            while y > self.coast(np.array([x]))[0] - 2e3:
                y -= 2000.0
                x += rng.normal(0.0, 700.0)
                x = min(max(x, 0.05 * self.Lx), 0.95 * self.Lx)
                pts.append((x, y))
            self.rivers.append(np.array(pts))
        # bathymetry noise: random plane waves, amplitude ~ 1 / wavenumber
        self.n_k = 2 * np.pi / (300e3 / 2.0 ** np.arange(8))
        self.n_th = rng.uniform(0, np.pi, (8, 3))
        self.n_ph = rng.uniform(0, 2 * np.pi, (8, 3))

    def coast(self, x):
        y = np.full_like(np.asarray(x, dtype=np.float64), self.y0)
        for a, k, p in zip(self.c_amp, self.c_k, self.c_ph):
            y = y + a * np.sin(k * x + p)
        return y

    def noise(self, x, y):
        f = np.zeros_like(x)
        for o in range(8):
            for w in range(3):
                kx, ky = np.cos(self.n_th[o, w]), np.sin(self.n_th[o, w])
                f = f + np.cos(self.n_k[o] * (kx * x + ky * y) + self.n_ph[o, w]) / 2.0 ** o
        return f / 3.0

    def sample_points(self, spacing=15.0):
        x = np.arange(0.0, self.Lx + spacing, spacing)
        pts = [np.stack([x, self.coast(x)], 1)]
        for r in self.rivers:
            seg = []
            for a, b in zip(r[:-1], r[1:]):
                n = max(2, int(np.hypot(*(b - a)) / spacing) + 1)
                t = np.linspace(0.0, 1.0, n)[:, None]
                seg.append(a[None] * (1 - t) + b[None] * t)
            pts.append(np.concatenate(seg))
        return np.concatenate(pts)

    def river_points(self, r, spacing=15.0):
        pts = []
        for a, b in zip(self.rivers[r][:-1], self.rivers[r][1:]):
            n = max(2, int(np.hypot(*(b - a)) / spacing) + 1)
            t = np.linspace(0.0, 1.0, n)[:, None]
            pts.append(a[None] * (1 - t) + b[None] * t)
        return np.concatenate(pts)

    def river_tree(self, spacing=15.0):
        return cKDTree(np.concatenate([self.river_points(r, spacing) for r in range(len(self.rivers))]))


def _key(i, j):
    return (np.asarray(i, dtype=np.int64) << 32) | np.asarray(j, dtype=np.int64)


def build_tree(feat: Features, gamma: float, *, lmax: int = LMAX, hmin: float = 30.0, window=(0, 0, NRX, NRY)):
    """Leaves per level: list of (i, j) int64 arrays after refinement and
    2:1 balancing.  ``window`` = (first root column, first root row, number
    of columns, number of rows) of the root grid."""
    tree = cKDTree(feat.sample_points())
    rx0, ry0, nrx, nry = window
    ii, jj = np.meshgrid(np.arange(rx0, rx0 + nrx), np.arange(ry0, ry0 + nry), indexing="ij")
    cur_i, cur_j = ii.ravel().astype(np.int64), jj.ravel().astype(np.int64)
    leaves = [None] * (lmax + 1)
    for L in range(lmax + 1):
        s = ROOT / 2 ** L
        if L == lmax:
            leaves[L] = (cur_i, cur_j)
            break
        cx, cy = (cur_i + 0.5) * s, (cur_j + 0.5) * s
        d, _ = tree.query(np.stack([cx, cy], 1))
        dmin = np.maximum(d - 0.7072 * s, 0.0)
        h = np.minimum(ROOT, hmin + gamma * dmin)
        split = s > h * 1.0001
        leaves[L] = (cur_i[~split], cur_j[~split])
        si, sj = cur_i[split], cur_j[split]
        cur_i = np.concatenate([2 * si, 2 * si + 1, 2 * si, 2 * si + 1])
        cur_j = np.concatenate([2 * sj, 2 * sj, 2 * sj + 1, 2 * sj + 1])
    return balance(leaves, window)


def balance(leaves, window=(0, 0, NRX, NRY)):
    """Split leaves until every side neighbour is at most one level coarser."""
    lmax = len(leaves) - 1
    rx0, ry0, nrx, nry = window
    keys = [_key(*leaves[L]) for L in range(lmax + 1)]
    changed = True
    while changed:
        changed = False
        for L in range(lmax, 1, -1):
            if keys[L].size == 0:
                continue
            i, j = keys[L] >> 32, keys[L] & 0xFFFFFFFF
            lo_x, lo_y = rx0 * 2 ** L, ry0 * 2 ** L
            hi_x, hi_y = (rx0 + nrx) * 2 ** L, (ry0 + nry) * 2 ** L
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ni, nj = i + di, j + dj
                ok = (ni >= lo_x) & (ni < hi_x) & (nj >= lo_y) & (nj < hi_y)
                ni, nj = ni[ok], nj[ok]
                for k in range(2, L + 1):
                    M = L - k
                    if keys[M].size == 0:
                        continue
                    anc = _key(ni >> k, nj >> k)
                    hit = np.isin(anc, keys[M])
                    if hit.any():
                        bad = np.unique(anc[hit])
                        keys[M] = np.setdiff1d(keys[M], bad, assume_unique=True)
                        bi, bj = bad >> 32, bad & 0xFFFFFFFF
                        kids = np.concatenate([_key(2 * bi + a, 2 * bj + b) for a in (0, 1) for b in (0, 1)])
                        keys[M + 1] = np.union1d(keys[M + 1], kids)
                        changed = True
    return [(keys[L] >> 32, keys[L] & 0xFFFFFFFF) for L in range(lmax + 1)]


def triangulate(leaves, window=(0, 0, NRX, NRY)):
    """Conforming fan triangulation.  Returns node lattice coordinates (units
    of ROOT / 2^(lmax+1)), triangles, and the window's boundary edges."""
    lmax = len(leaves) - 1
    rx0, ry0, nrx, nry = window
    keysets = [_key(*leaves[L]) for L in range(lmax + 1)]
    all_pts = []
    all_tri_local = []
    bnd = []
    for L in range(lmax + 1):
        i, j = leaves[L]
        if i.size == 0:
            continue
        S = 2 ** (lmax + 1 - L)
        lo_x, lo_y = rx0 * 2 ** L, ry0 * 2 ** L
        hi_x, hi_y = (rx0 + nrx) * 2 ** L - 1, (ry0 + nry) * 2 ** L - 1
        # midpoint present where the neighbour across the side is subdivided
        fine = keysets[L + 1] if L < lmax else np.zeros(0, dtype=np.int64)

        def sub(ci, cj):
            # the finer leaf that touches this cell's side at its first half
            return np.isin(_key(ci, cj), fine) if fine.size else np.zeros(ci.shape, bool)
        has_b = (j > lo_y) & sub(2 * i, 2 * j - 1)
        has_r = (i < hi_x) & sub(2 * i + 2, 2 * j)
        has_t = (j < hi_y) & sub(2 * i, 2 * j + 2)
        has_l = (i > lo_x) & sub(2 * i - 1, 2 * j)
        x0, y0 = i * S, j * S
        h = S // 2
        # slots CCW: c0, b, c1, r, c2, t, c3, l ; centre
        P = np.stack([
            np.stack([x0, y0], 1), np.stack([x0 + h, y0], 1), np.stack([x0 + S, y0], 1),
            np.stack([x0 + S, y0 + h], 1), np.stack([x0 + S, y0 + S], 1), np.stack([x0 + h, y0 + S], 1),
            np.stack([x0, y0 + S], 1), np.stack([x0, y0 + h], 1), np.stack([x0 + h, y0 + h], 1)], 1)
        present = np.stack([np.ones_like(has_b), has_b, np.ones_like(has_b), has_r, np.ones_like(has_b),
                            has_t, np.ones_like(has_b), has_l], 1)
        base = sum(p.shape[0] for p in all_pts)
        all_pts.append(P.reshape(-1, 2))
        n = i.size
        idx = base + 9 * np.arange(n)[:, None] + np.arange(9)[None]
        for sidx in range(8):
            # triangle (centre, slot s, next present slot)
            nxt = (sidx + 1) % 8
            if sidx % 2 == 0:
                nxt_id = np.where(present[:, nxt], idx[:, nxt], idx[:, (sidx + 2) % 8])
                m = np.ones(n, bool)
            else:
                nxt_id = idx[:, nxt]
                m = present[:, sidx]
            all_tri_local.append(np.stack([idx[m, 8], idx[m, sidx], nxt_id[m]], 1))
        # domain boundary sides (no midpoints there)
        for side, cond, a, b in (("b", j == lo_y, 0, 2), ("r", i == hi_x, 2, 4), ("t", j == hi_y, 4, 6),
                                 ("l", i == lo_x, 6, 0)):
            if cond.any():
                bnd.append(np.stack([idx[cond, a], idx[cond, b]], 1))
    pts = np.concatenate(all_pts)
    W = NRY * 2 ** (lmax + 1) + 1
    key = pts[:, 0].astype(np.int64) * W + pts[:, 1].astype(np.int64)
    uk, inv = np.unique(key, return_inverse=True)
    xy_lat = np.stack([uk // W, uk % W], 1)
    tri = inv[np.concatenate(all_tri_local)]
    bedges = inv[np.concatenate(bnd)]
    # drop the midpoint slots of sides without a finer neighbour
    used = np.zeros(len(uk), bool)
    used[tri.ravel()] = True
    remap = np.cumsum(used) - 1
    return xy_lat[used], remap[tri].astype(np.int32), remap[bedges].astype(np.int32)


def graded_coast(gamma: float = 1.6, seed: int = seed_for(3), *, lmax: int = LMAX, hmin: float = 30.0,
           window=(0, 0, NRX, NRY), n_steps: int = 10000, name: str = "graded") -> Scenario:
    """The graded coastal workload.  With the defaults (gamma = 1.6, 30 m
    down to level 9 over the full 80 x 60 root grid) it has 3,596,698
    triangles.  ``window`` selects a block of root cells (same coast,
    rivers, bathymetry and forcing), ``lmax``/``hmin`` a coarser finest
    level, for small instances of the same construction."""
    feat = Features(seed)
    leaves = build_tree(feat, gamma, lmax=lmax, hmin=hmin, window=window)
    xy_lat, tri, bed = triangulate(leaves, window)
    xy = xy_lat.astype(np.float64) * (ROOT / 2 ** (lmax + 1))
    x, y = xy[:, 0], xy[:, 1]
    d = y - feat.coast(x)                                   # > 0 on land
    nz = feat.noise(x, y)
    rt = feat.river_tree()
    dr, _ = rt.query(xy)
    # land: a smooth rise to +50 m plus noise that fades out within 3 km of a
    # river (valleys); channels 3 m below the smooth profile, and at least
    # 3 m below the datum where they meet the sea
    rise = 49.5 * np.tanh(np.maximum(d, 0.0) / 40e3)
    zs = 0.5 + 0.6 * rise
    zland = zs + 0.4 * rise * nz * np.minimum(1.0, dr / 3e3)
    zb = np.where(d < 0.0, -4000.0 * np.tanh(-d / 150e3) - 5.0 + 150.0 * nz * np.tanh(-d / 20e3), zland)
    channel = (dr < 150.0) & (d > -1000.0)
    zb = np.where(channel, np.where(d > 0.0, zs - 3.0, np.minimum(zb, -3.0)), zb)
    zb = np.clip(zb, -4000.0, 50.0)
    hb = -zb
    fric = np.where((zb < 0.0) | channel, 0.02, 0.05)
    # boundary types: ocean where both nodes are below -10 m, river inflow
    # on the north side inside a channel, land elsewhere
    bt = np.full(len(bed), LAND, np.int32)
    bs = np.zeros(len(bed), np.int32)
    zb_e = np.maximum(zb[bed[:, 0]], zb[bed[:, 1]])
    bt[zb_e < -10.0] = OCEAN
    ytop = (window[1] + window[3]) * ROOT
    north = (y[bed[:, 0]] >= ytop - 1.0) & (y[bed[:, 1]] >= ytop - 1.0)
    mid = 0.5 * (xy[bed[:, 0]] + xy[bed[:, 1]])
    for r in range(len(feat.rivers)):
        dr_e, _ = cKDTree(feat.river_points(r)).query(mid)
        sel = north & (dr_e < 150.0)
        bt[sel] = RIVER
        bs[sel] = 1 + r
    mesh = Mesh(xy, tri, hb, fric, bed, bt, bs)
    zeta0 = np.where(hb > 0.0, 0.0, -hb)                   # sea at rest, land dry
    rng = np.random.default_rng(seed + 11)
    ddeg = 11120.0
    nxl, nyl = int(np.ceil(feat.Lx / ddeg)) + 1, int(np.ceil(feat.Ly / ddeg)) + 1
    rain = gridded_field(rng, 0.0, 0.0, ddeg, ddeg, nxl, nyl, 8, 3600.0, n_cells=20,
                         peak_range=(20.0, 100.0), radius_range=(20e3 / feat.Lx, 80e3 / feat.Lx), drift=(5.0, 0.0))
    tides = {0: (0.0, np.array([[0.5, 44712.0, 0.0]]))}
    rivers = {1 + r: (np.array([0.0]), np.array([-1.0])) for r in range(3)}
    # the step is capped at 0.5 s (the paper's large-mesh step): a window
    # without water has no wave speed
    return Scenario(name, mesh, zeta0, np.zeros_like(hb), np.zeros_like(hb),
                    default_params(flux="llf", friction="manning", limiter=True, cfl=0.3, H0=0.05, dt_max=0.5),
                    rain=rain, tides=tides, rivers=rivers, n_steps=n_steps)


def graded_small(river: int = 0, seed: int = seed_for(3), *, size=(3, 3), gamma: float = 6.0,
                 lmax: int = 6, hmin: float = 240.0) -> Scenario:
    """A few root cells of the graded workload around the mouth of one river
    (same coast, channel, bathymetry and forcing), refined to 240 m: a small
    instance of the same construction for element-by-element parity."""
    feat = Features(seed)
    mx, my = feat.rivers[river][-1]
    rx = int(mx // ROOT) - size[0] // 2
    ry = int(my // ROOT) - size[1] // 2
    rx = min(max(rx, 0), NRX - size[0])
    ry = min(max(ry, 0), NRY - size[1])
    return graded_coast(gamma, seed, lmax=lmax, hmin=hmin, window=(rx, ry, size[0], size[1]), n_steps=200,
                  name=f"graded_small_{river}")
