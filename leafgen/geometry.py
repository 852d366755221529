"""Seeded synthetic leaf cross-sections, described in micrometres and
rasterised at cell centres for any grid spacing.

These stand in for the segmented micrographs of the paper (Sec. 2.7), which
are not available.  Every random draw is made in physical units before
rasterisation, so one seed gives the same anatomy at every dx.  Shapes follow
the paper's tissue list (cuticle, epidermal cells, palisade and spongy
mesophyll, bulliform cells, vascular bundle, chloroplasts) and its chloroplast
recipe: rotated ellipses with a = mu_a + sigma_a (2 r1 - 1),
b = a [1 + (r2 - 0.5)], theta ~ U[0, 2 pi), inserted until they cover a target
fraction of the mesophyll (eqs. 35-36).

Output: uint8 label map [ny][nx], row-major, j = 0 at the bottom, x periodic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

AIR = 0


# ---------------------------------------------------------------------------
# rasterisation helpers (positions in um, dx in um)
# ---------------------------------------------------------------------------

def _rows(y0: float, y1: float, dx: float, ny: int) -> tuple[int, int]:
    """Rows whose centre (j+1/2)dx lies in [y0, y1)."""
    j0 = max(0, int(math.ceil(y0 / dx - 0.5)))
    j1 = min(ny, int(math.ceil(y1 / dx - 0.5)))
    return j0, max(j0, j1)


def _centres(n: int, dx: float, start: int = 0) -> np.ndarray:
    return (np.arange(start, start + n) + 0.5) * dx


def fill_band(lab: np.ndarray, dx: float, y0: float, y1: float, label: int) -> None:
    j0, j1 = _rows(y0, y1, dx, lab.shape[0])
    lab[j0:j1] = label


def _periodic_dx(x: np.ndarray, cx: float, Lx: float) -> np.ndarray:
    d = x - cx
    return d - Lx * np.round(d / Lx)


def ellipse(lab: np.ndarray, dx: float, cx: float, cy: float, a: float, b: float, theta: float,
            label: int, only: tuple[int, ...] | None = None, rim: tuple[float, int] | None = None,
            inside_mask: np.ndarray | None = None) -> None:
    """Rasterise a rotated ellipse (semi-axes a, b) with periodic x.

    only: overwrite only pixels whose current label is in this set.
    rim: (thickness, label) paints a rim of roughly that thickness inside the
    boundary with a second label."""
    ny, nx = lab.shape
    Lx = nx * dx
    r = max(a, b)
    j0, j1 = _rows(cy - r, cy + r, dx, ny)
    if j1 <= j0:
        return
    i0 = int(math.floor((cx - r) / dx - 0.5))
    i1 = int(math.ceil((cx + r) / dx - 0.5)) + 1
    cols = np.arange(i0, i1) % nx
    if len(cols) > nx:
        cols = np.arange(nx)
    xs = (cols + 0.5) * dx
    ys = _centres(j1 - j0, dx, j0)
    X = _periodic_dx(xs, cx, Lx)[None, :]
    Y = (ys - cy)[:, None]
    c, s = math.cos(theta), math.sin(theta)
    u = (X * c + Y * s) / a
    v = (-X * s + Y * c) / b
    rr = np.sqrt(u * u + v * v)
    inside = rr < 1.0
    sub = lab[j0:j1][:, cols]
    if only is not None:
        inside &= np.isin(sub, only)
    if inside_mask is not None:
        inside &= inside_mask[j0:j1][:, cols]
    new = np.where(inside, label, sub)
    if rim is not None:
        t, rim_label = rim
        edge = inside & (rr > 1.0 - t / min(a, b))
        new = np.where(edge, rim_label, new)
    lab[j0:j1, cols] = new


def rect_cells(lab: np.ndarray, dx: float, y0: float, y1: float, widths: np.ndarray, x_off: float,
               wall_t: float, wall_label: int, fill_label: int) -> None:
    """A band [y0, y1) of rectangular cells with the given widths (sum = Lx),
    starting at x_off, walls of thickness wall_t around every cell."""
    ny, nx = lab.shape
    Lx = nx * dx
    j0, j1 = _rows(y0, y1, dx, ny)
    if j1 <= j0:
        return
    edges = x_off + np.concatenate([[0.0], np.cumsum(widths)])
    xs = (np.arange(nx) + 0.5) * dx
    # distance to the nearest vertical wall (periodic)
    dmin = np.full(nx, np.inf)
    for e in edges[:-1]:
        dmin = np.minimum(dmin, np.abs(_periodic_dx(xs, e % Lx, Lx)))
    vwall = dmin < wall_t / 2
    ys = _centres(j1 - j0, dx, j0)
    hwall = (ys - y0 < wall_t / 2) | (y1 - ys < wall_t / 2)
    band = np.where(vwall[None, :] | hwall[:, None], wall_label, fill_label).astype(np.uint8)
    lab[j0:j1] = band


def _widths(rng: np.random.Generator, Lx: float, lo: float, hi: float) -> np.ndarray:
    w = []
    while sum(w) < Lx:
        w.append(rng.uniform(lo, hi))
    w = np.array(w)
    if len(w) > 1 and w.sum() - w[-1] >= Lx - lo / 2:
        w = w[:-1]
    return w * (Lx / w.sum())


def voronoi_band(lab: np.ndarray, dx: float, y0: float, y1: float, seeds: np.ndarray, sx: float,
                 sy: float, wall_t: float, wall_label: int, fill_label: int, chunk: int = 256) -> None:
    """Anisotropic Voronoi cells in [y0, y1): distance metric scaled by (1/sx, 1/sy),
    walls where a pixel lies within wall_t/2 (physical) of a cell bisector.
    seeds: (N, 2) array of (x, y) in um, periodic in x."""
    ny, nx = lab.shape
    Lx = nx * dx
    j0, j1 = _rows(y0, y1, dx, ny)
    xs = (np.arange(nx) + 0.5) * dx
    A = np.array([1.0 / sx, 1.0 / sy])
    sd = seeds * A
    for jc in range(j0, j1, chunk):
        je = min(j1, jc + chunk)
        ys = _centres(je - jc, dx, jc)
        # nearest two seeds in scaled metric (brute force over seeds; few hundred seeds)
        best1 = np.full((je - jc, nx), np.inf)
        best2 = np.full((je - jc, nx), np.inf)
        arg1 = np.zeros((je - jc, nx), np.int32)
        arg2 = np.zeros((je - jc, nx), np.int32)
        for k, (sxk, syk) in enumerate(seeds):
            if abs(syk - ys.mean()) > (ys[-1] - ys[0]) / 2 + 3 * sy:
                continue
            ddx = _periodic_dx(xs, sxk, Lx)[None, :] * A[0]
            ddy = (ys - syk)[:, None] * A[1]
            d2 = ddx * ddx + ddy * ddy
            lt1 = d2 < best1
            lt2 = (~lt1) & (d2 < best2)
            best2 = np.where(lt1, best1, np.where(lt2, d2, best2))
            arg2 = np.where(lt1, arg1, np.where(lt2, k, arg2))
            best1 = np.where(lt1, d2, best1)
            arg1 = np.where(lt1, k, arg1)
        # physical distance to the bisector of the two nearest seeds
        s1 = seeds[arg1]
        s2 = seeds[arg2]
        ddx12 = _periodic_dx(s2[..., 0], 0.0, Lx) - _periodic_dx(s1[..., 0], 0.0, Lx)
        ddx12 = ddx12 - Lx * np.round(ddx12 / Lx)
        n_sc = np.stack([ddx12 * A[0], (s2[..., 1] - s1[..., 1]) * A[1]], -1)  # scaled normal
        # point relative to s1 in scaled coordinates
        px = _periodic_dx(xs[None, :], 0.0, Lx) - s1[..., 0]
        px = px - Lx * np.round(px / Lx)
        py = ys[:, None] - s1[..., 1]
        z = np.stack([px * A[0], py * A[1]], -1)
        nn = np.sqrt((n_sc ** 2).sum(-1))
        along = (z * n_sc).sum(-1) / np.maximum(nn, 1e-12)
        gap = nn / 2 - along                      # scaled distance to the bisector
        phys_norm = np.sqrt((n_sc[..., 0] * A[0]) ** 2 + (n_sc[..., 1] * A[1]) ** 2) / np.maximum(nn, 1e-12)
        dist = gap / np.maximum(phys_norm, 1e-12)
        band = np.where(dist < wall_t / 2, wall_label, fill_label).astype(np.uint8)
        ywall = (ys - y0 < wall_t / 2) | (y1 - ys < wall_t / 2)
        band[ywall] = wall_label
        lab[jc:je] = band


def chloroplasts(lab: np.ndarray, dx: float, rng: np.random.Generator, y0: float, y1: float,
                 host_label: int, label: int, fraction: float, mu_a: float, sigma_a: float,
                 mes_area_px: int, max_tries: int = 20000) -> None:
    """Eqs. 35-36: rotated ellipses inside host (cytoplasm) pixels of [y0, y1) until
    they cover `fraction` of the mesophyll area (mes_area_px pixels)."""
    ny, nx = lab.shape
    Lx = nx * dx
    target = fraction * mes_area_px
    j0, j1 = _rows(y0, y1, dx, ny)
    if not (lab[j0:j1] == host_label).any():
        return
    target = min(target, int((lab[j0:j1] == host_label).sum()) + int((lab[j0:j1] == label).sum()))
    covered = int((lab[j0:j1] == label).sum())
    tries = 0
    while covered < target and tries < max_tries:
        tries += 1
        r1, r2 = rng.random(), rng.random()
        a = mu_a + sigma_a * (2 * r1 - 1)
        b = a * (1 + (r2 - 0.5))
        th = rng.uniform(0, 2 * math.pi)
        cx = rng.uniform(0, Lx)
        cy = rng.uniform(y0, y1)
        ellipse(lab, dx, cx, cy, a, b, th, label, only=(host_label,))
        if tries % 16 == 0:
            covered = int((lab[j0:j1] == label).sum())


# ---------------------------------------------------------------------------
# leaves
# ---------------------------------------------------------------------------

@dataclass
class DicotLayers:
    cuticle: float = 2.0
    upper_epidermis: float = 18.0
    palisade: float = 60.0
    spongy: float = 50.0
    lower_epidermis: float = 14.0
    wall: float = 0.3
    epi_width: tuple = (15.0, 25.0)
    low_epi_width: tuple = (12.0, 20.0)
    palisade_cell: tuple = (10.0, 40.0)
    spongy_axes: tuple = (4.0, 10.0)
    spongy_cover: float = 0.70
    chl_mu: float = 2.0           # 4 um discs
    chl_sigma: float = 0.5
    chl_fraction: float = 0.20
    hypha_width: tuple = (2.0, 3.0)
    hypha_spacing: float = 12.0

    @property
    def thickness(self) -> float:
        return 2 * self.cuticle + self.upper_epidermis + self.palisade + self.spongy + self.lower_epidermis

    def scaled(self, **kw) -> "DicotLayers":
        d = dict(self.__dict__)
        d.update(kw)
        return DicotLayers(**d)


# dicot labels (see materials.DICOT_LABELS)
D_CUT, D_WEPI, D_WPAL, D_WSPO, D_CYT, D_CHL, D_HYP = 1, 2, 3, 4, 5, 6, 7


def dicot(nx: int, ny: int, dx_nm: float, seed: int, diseased: bool = False,
          layers: DicotLayers | None = None, leaf_top_um: float | None = None,
          hypha_seed: int | None = None) -> np.ndarray:
    """Synthetic dicot cross-section, top to bottom: air, cuticle, upper
    epidermis (rectangular cells), palisade (vertically elongated Voronoi cells),
    spongy mesophyll (random ellipses with ~30 % air), lower epidermis, cuticle,
    air.  Chloroplasts fill ~20 % of the mesophyll.  `diseased` adds melanised
    hyphae through the cuticle and upper epidermis."""
    L = layers or DicotLayers()
    dx = dx_nm * 1e-3
    Lx, Ly = nx * dx, ny * dx
    rng = np.random.default_rng(seed)
    lab = np.zeros((ny, nx), np.uint8)
    top = leaf_top_um if leaf_top_um is not None else (Ly + L.thickness) / 2
    y = top
    # cuticle (top)
    fill_band(lab, dx, y - L.cuticle, y, D_CUT)
    y -= L.cuticle
    # upper epidermis
    w = _widths(rng, Lx, *L.epi_width)
    rect_cells(lab, dx, y - L.upper_epidermis, y, w, rng.uniform(0, Lx), L.wall, D_WEPI, D_CYT)
    epi_bottom = y - L.upper_epidermis
    y = epi_bottom
    # palisade
    pal_top, pal_bot = y, y - L.palisade
    sx, sy = L.palisade_cell
    seeds = []
    nxs = max(1, int(round(Lx / sx)))
    nys = max(1, int(round(L.palisade / sy)))
    for a in range(nys):
        for b in range(nxs):
            seeds.append(((b + 0.5 + rng.uniform(-0.3, 0.3) + 0.5 * (a % 2)) * Lx / nxs % Lx,
                          pal_bot + (a + 0.5 + rng.uniform(-0.2, 0.2)) * L.palisade / nys))
    voronoi_band(lab, dx, pal_bot, pal_top, np.array(seeds), sx, sy, L.wall, D_WPAL, D_CYT)
    y = pal_bot
    # spongy mesophyll: air with random elliptical cells
    spo_top, spo_bot = y, y - L.spongy
    fill_band(lab, dx, spo_bot, spo_top, AIR)
    band_area = Lx * L.spongy
    j0, j1 = _rows(spo_bot, spo_top, dx, ny)
    n_try = 0
    while n_try < 10000:
        n_try += 1
        a = rng.uniform(*L.spongy_axes)
        b = rng.uniform(*L.spongy_axes)
        th = rng.uniform(0, math.pi)
        cx = rng.uniform(0, Lx)
        cy = rng.uniform(spo_bot + min(a, b) * 0.5, spo_top - min(a, b) * 0.5)
        mask = np.zeros_like(lab, dtype=bool)
        mask[j0:j1] = True
        ellipse(lab, dx, cx, cy, a, b, th, D_CYT, only=(AIR,), rim=(L.wall, D_WSPO), inside_mask=mask)
        if n_try % 4 == 0:
            cover = float((lab[j0:j1] != AIR).mean()) if j1 > j0 else 1.0
            if cover >= L.spongy_cover:
                break
    y = spo_bot
    # lower epidermis and cuticle
    w = _widths(rng, Lx, *L.low_epi_width)
    rect_cells(lab, dx, y - L.lower_epidermis, y, w, rng.uniform(0, Lx), L.wall, D_WEPI, D_CYT)
    y -= L.lower_epidermis
    fill_band(lab, dx, y - L.cuticle, y, D_CUT)
    # chloroplasts in mesophyll cytoplasm (palisade + spongy)
    jm0, jm1 = _rows(spo_bot, pal_top, dx, ny)
    mes_area = (jm1 - jm0) * nx
    chloroplasts(lab, dx, rng, spo_bot, pal_top, D_CYT, D_CHL, L.chl_fraction,
                 L.chl_mu, L.chl_sigma, mes_area)
    if diseased:
        hr = np.random.default_rng(hypha_seed if hypha_seed is not None else seed + 1000003)
        count = max(1, int(hr.poisson(Lx / L.hypha_spacing)))
        for _ in range(count):
            wdt = hr.uniform(*L.hypha_width)
            cx = hr.uniform(0, Lx)
            jj0, jj1 = _rows(epi_bottom, top, dx, ny)
            xs = (np.arange(nx) + 0.5) * dx
            cols = np.abs(_periodic_dx(xs, cx, Lx)) < wdt / 2
            lab[jj0:jj1, cols] = D_HYP
    return lab


# monocot labels (see materials.MONOCOT_LABELS)
M_CUT, M_WALL, M_ECYT, M_MCYT, M_CHL, M_VASC = 1, 2, 3, 4, 5, 6


def monocot(nx: int, ny: int, dx_nm: float, seed: int) -> np.ndarray:
    """Synthetic monocot cross-section: cuticle 1 um; upper epidermis of 4 um
    cells with one group of 3-5 inflated bulliform cells (~5 x 10 um); mesophyll
    of staggered rounded-rectangle cells (~5 x 8 um, ~5 % air) aligned as if
    vein-parallel; one vascular bundle (~8 um ellipse); lower epidermis 3 um;
    cuticle 1 um.  Chloroplasts fill ~20 % of the mesophyll."""
    dx = dx_nm * 1e-3
    Lx, Ly = nx * dx, ny * dx
    rng = np.random.default_rng(seed)
    lab = np.zeros((ny, nx), np.uint8)
    cut, epi, mes, lepi, wall = 1.0, 5.0, 16.0, 3.0, 0.3
    thick = 2 * cut + epi + mes + lepi
    top = (Ly + thick) / 2
    y = top
    fill_band(lab, dx, y - cut, y, M_CUT)
    y -= cut
    # upper epidermis: regular 4 um cells, bulliform group replaces a few of them
    n_bull = int(rng.integers(3, 6))
    widths = list(_widths(rng, Lx - n_bull * 5.0, 3.5, 4.5)) if Lx > n_bull * 5.0 + 4 else []
    ins = int(rng.integers(0, max(1, len(widths))))
    widths = widths[:ins] + [5.0] * n_bull + widths[ins:]
    widths = np.array(widths) * (Lx / sum(widths))
    x_off = rng.uniform(0, Lx)
    rect_cells(lab, dx, y - epi, y, widths, x_off, wall, M_WALL, M_ECYT)
    # bulliform cells extend 10 um down into the mesophyll band
    edges = x_off + np.concatenate([[0.0], np.cumsum(widths)])
    bull_lo, bull_hi = edges[ins], edges[ins + n_bull]
    epi_bot = y - epi
    y = epi_bot
    mes_top, mes_bot = y, y - mes
    # mesophyll: staggered rounded rectangles in air
    fill_band(lab, dx, mes_bot, mes_top, 0)
    cw, ch = 5.0, 8.0
    n_rows = max(1, int(round(mes / ch)))
    rh = mes / n_rows
    xs = (np.arange(nx) + 0.5) * dx
    for r in range(n_rows):
        yb, yt = mes_bot + r * rh, mes_bot + (r + 1) * rh
        ncell = max(1, int(round(Lx / cw)))
        wdt = Lx / ncell
        off = (0.5 * wdt * (r % 2)) + rng.uniform(-0.3, 0.3)
        j0, j1 = _rows(yb, yt, dx, ny)
        ys = _centres(j1 - j0, dx, j0)
        # rounded rectangle: inset 0.12 um gap (≈5 % air), corner radius 1 um
        gap = 0.12
        px = ((xs - off) % wdt)[None, :]
        py = (ys - yb)[:, None]
        hx_, hy_ = wdt / 2 - gap, rh / 2 - gap
        qx = np.abs(px - wdt / 2) - (hx_ - 1.0)
        qy = np.abs(py - rh / 2) - (hy_ - 1.0)
        outside = np.sqrt(np.maximum(qx, 0) ** 2 + np.maximum(qy, 0) ** 2) + np.minimum(np.maximum(qx, qy), 0) - 1.0
        cell = outside < 0
        wallp = cell & (outside > -wall)
        band = np.where(wallp, M_WALL, np.where(cell, M_MCYT, 0)).astype(np.uint8)
        lab[j0:j1] = band
    # bulliform cells overwrite the top 5 um of the mesophyll under their group
    j0, j1 = _rows(epi_bot - 5.0, epi_bot, dx, ny)
    bw = (bull_hi - bull_lo) / n_bull
    rect_cells_sub = np.zeros((j1 - j0, nx), np.uint8)
    cols = np.zeros(nx, bool)
    for b in range(n_bull):
        x0 = (bull_lo + b * bw) % Lx
        d = _periodic_dx(xs, x0 + bw / 2, Lx)
        inside = np.abs(d) < bw / 2
        cols |= inside
        wall_c = inside & (np.abs(np.abs(d) - bw / 2) < wall / 2)
        rect_cells_sub[:, inside] = M_ECYT
        rect_cells_sub[:, wall_c] = M_WALL
    ys = _centres(j1 - j0, dx, j0)
    rect_cells_sub[(ys - (epi_bot - 5.0)) < wall / 2] = np.where(cols, M_WALL, rect_cells_sub[(ys - (epi_bot - 5.0)) < wall / 2])
    lab[j0:j1, cols] = rect_cells_sub[:, cols]
    # remove the epidermal floor wall under the bulliform group (one tall cell)
    jw0, jw1 = _rows(epi_bot - wall / 2, epi_bot + wall / 2, dx, ny)
    inner = cols.copy()
    for b in range(n_bull):
        x0 = (bull_lo + b * bw) % Lx
        d = _periodic_dx(xs, x0 + bw / 2, Lx)
        inner &= ~((np.abs(d) < bw / 2) & (np.abs(np.abs(d) - bw / 2) < wall / 2))
    lab[jw0:jw1, inner] = M_ECYT
    # vascular bundle
    vx = rng.uniform(0, Lx)
    vy = (mes_top + mes_bot) / 2 - 1.0
    ellipse(lab, dx, vx, vy, 4.0, 3.5, 0.0, M_VASC, rim=(wall, M_WALL))
    y = mes_bot
    w = _widths(rng, Lx, 3.0, 5.0)
    rect_cells(lab, dx, y - lepi, y, w, rng.uniform(0, Lx), wall, M_WALL, M_ECYT)
    y -= lepi
    fill_band(lab, dx, y - cut, y, M_CUT)
    jm0, jm1 = _rows(mes_bot, mes_top, dx, ny)
    chloroplasts(lab, dx, rng, mes_bot, mes_top, M_MCYT, M_CHL, 0.20, 1.0, 0.25, (jm1 - jm0) * nx)
    return lab


def slab(nx: int, ny: int, row_lo: int, row_hi: int, label: int = 1) -> np.ndarray:
    """x-invariant slab occupying rows [row_lo, row_hi)."""
    lab = np.zeros((ny, nx), np.uint8)
    lab[row_lo:row_hi] = label
    return lab


def random_blocks(nx: int, ny: int, seed: int, n_labels: int, row_lo: int, row_hi: int,
                  block: tuple[int, int] = (4, 4)) -> np.ndarray:
    """Random piecewise-constant label map in rows [row_lo, row_hi), air elsewhere.
    Labels drawn uniformly from 0..n_labels-1 on blocks of (by, bx) cells."""
    rng = np.random.default_rng(seed)
    by, bx = block
    nby = -(-(row_hi - row_lo) // by)
    nbx = -(-nx // bx)
    blk = rng.integers(0, n_labels, size=(nby, nbx)).astype(np.uint8)
    full = np.kron(blk, np.ones((by, bx), np.uint8))[: row_hi - row_lo, :nx]
    lab = np.zeros((ny, nx), np.uint8)
    lab[row_lo:row_hi] = full
    return lab
