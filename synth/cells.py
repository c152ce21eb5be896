"""Seeded unit-cell generators for the synthetic workloads.

Every cell is a square lattice of side 1 m (rows of ``lattice`` are h1, h2),
rasterised on an ``nx x ny`` pixel grid whose first index runs along h1.
``phase[i, j]`` is the phase id of pixel (i, j); ``props[p] = (E [Pa], nu,
rho [kg/m^3])`` are the isotropic properties of phase p.  Nothing here knows
about plane waves or eigenproblems.

Seeds: numpy ``Generator(PCG64(SeedSequence([13106380, cfg, item])))``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Cell", "rng_for", "SQUARE", "circle_cell", "voronoi_phase_map", "random_iso_props",
    "inclusion_phase_map", "grf_phase_map", "layered_cell", "kpath_gxmg",
    "config0", "config1", "config2", "config3", "config4_cells", "workload",
    "INCLUSION_PROPS", "MATRIX_PROPS",
]

SQUARE = np.array([[1.0, 0.0], [0.0, 1.0]])

# the two-phase material pair of the simple inclusion workload
INCLUSION_PROPS = (70e9, 0.33, 2700.0)   # stiff inclusion
MATRIX_PROPS = (3.5e9, 0.35, 1180.0)     # compliant matrix


@dataclasses.dataclass
class Cell:
    lattice: np.ndarray          # [2,2] rows h1, h2 (metres)
    phase: np.ndarray            # [nx, ny] int32, i along h1
    props: np.ndarray            # [P, 3] (E, nu, rho)

    @property
    def n_phases(self) -> int:
        return int(self.props.shape[0])

    @property
    def nx(self) -> int:
        return int(self.phase.shape[0])

    @property
    def ny(self) -> int:
        return int(self.phase.shape[1])


def rng_for(cfg: int, item: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([13106380, cfg, item])))


def _pixel_centres(nx: int, ny: int):
    fx = (np.arange(nx) + 0.5) / nx
    fy = (np.arange(ny) + 0.5) / ny
    return np.meshgrid(fx, fy, indexing="ij")


def circle_cell(n: int = 16, r: float = 0.3, inc=INCLUSION_PROPS, mat=MATRIX_PROPS) -> Cell:
    """Circular inclusion of radius r (fraction of a) centred in the cell.

    A pixel is inclusion (phase 1) when its centre lies inside the circle.
    """
    x, y = _pixel_centres(n, n)
    inside = (x - 0.5) ** 2 + (y - 0.5) ** 2 < r * r
    phase = inside.astype(np.int32)
    props = np.array([mat, inc], dtype=np.float64)
    return Cell(SQUARE.copy(), phase, props)


def random_iso_props(n: int, rng: np.random.Generator) -> np.ndarray:
    """E log-uniform in [1, 200] GPa, nu uniform in [0.2, 0.4], rho log-uniform in [1000, 8000]."""
    E = np.exp(rng.uniform(np.log(1e9), np.log(200e9), n))
    nu = rng.uniform(0.2, 0.4, n)
    rho = np.exp(rng.uniform(np.log(1000.0), np.log(8000.0), n))
    return np.stack([E, nu, rho], axis=1)


def voronoi_phase_map(nx: int, ny: int, sites: np.ndarray) -> np.ndarray:
    """Periodic Voronoi partition: each pixel centre takes the nearest site
    (minimum-image distance on the unit torus); ties go to the lowest index."""
    x, y = _pixel_centres(nx, ny)
    px = x.reshape(-1, 1)
    py = y.reshape(-1, 1)
    best = np.full(px.shape[0], np.inf)
    arg = np.zeros(px.shape[0], dtype=np.int64)
    chunk = 256
    for s0 in range(0, sites.shape[0], chunk):
        sx = sites[s0:s0 + chunk, 0][None, :]
        sy = sites[s0:s0 + chunk, 1][None, :]
        dx = np.abs(px - sx)
        dx = np.minimum(dx, 1.0 - dx)
        dy = np.abs(py - sy)
        dy = np.minimum(dy, 1.0 - dy)
        d2 = dx * dx + dy * dy
        a = np.argmin(d2, axis=1)           # first minimum = lowest index within chunk
        v = d2[np.arange(d2.shape[0]), a]
        better = v < best                   # strict: earlier chunks win ties
        best[better] = v[better]
        arg[better] = a[better] + s0
    return arg.reshape(nx, ny).astype(np.int32)


def inclusion_phase_map(n: int, shape: str, phi: float) -> np.ndarray:
    """Centred inclusion (phase 1) of a circle, square or cross with nominal fill phi."""
    x, y = _pixel_centres(n, n)
    x = x - 0.5
    y = y - 0.5
    if shape == "circle":
        r = np.sqrt(phi / np.pi)
        inside = x * x + y * y < r * r
    elif shape == "square":
        h = 0.5 * np.sqrt(phi)
        inside = (np.abs(x) < h) & (np.abs(y) < h)
    elif shape == "cross":
        w = 0.8 - np.sqrt(0.64 - phi)
        bar1 = (np.abs(x) < 0.4) & (np.abs(y) < 0.5 * w)
        bar2 = (np.abs(y) < 0.4) & (np.abs(x) < 0.5 * w)
        inside = bar1 | bar2
    else:
        raise ValueError(shape)
    return inside.astype(np.int32)


def grf_phase_map(n: int, ell: float, phi: float, rng: np.random.Generator) -> np.ndarray:
    """Binary cell from a periodic Gaussian random field.

    White N(0,1) noise is filtered in Fourier space by exp(-pi^2 ell^2 |f|^2)
    (f in cycles/pixel, correlation length ell pixels); the round(phi n^2)
    largest values become phase 1 (stable ordering on ties).
    """
    noise = rng.standard_normal((n, n))
    f = np.fft.fftfreq(n)
    fx, fy = np.meshgrid(f, f, indexing="ij")
    filt = np.exp(-np.pi ** 2 * ell ** 2 * (fx ** 2 + fy ** 2))
    field = np.real(np.fft.ifft2(np.fft.fft2(noise) * filt))
    k = int(round(phi * n * n))
    order = np.argsort(-field.reshape(-1), kind="stable")
    out = np.zeros(n * n, dtype=np.int32)
    out[order[:k]] = 1
    return out.reshape(n, n)


def layered_cell(fractions, props, nx: int) -> Cell:
    """1-D stack of layers along h1 (phase depends on H1 only), ny = 1.

    ``fractions`` are layer thicknesses in pixels along h1 and must sum to nx.
    """
    fr = list(fractions)
    if sum(fr) != nx:
        raise ValueError("layer widths must sum to nx")
    col = np.concatenate([np.full(w, p, dtype=np.int32) for p, w in enumerate(fr)])
    phase = col.reshape(nx, 1)
    return Cell(SQUARE.copy(), phase, np.asarray(props, dtype=np.float64))


def kpath_gxmg(n_k: int) -> np.ndarray:
    """n_k points equally spaced in arc length on Gamma(0,0)-X(1/2,0)-M(1/2,1/2)-Gamma.

    Coordinates are fractional (Q1, Q2) with k = Q1 q1 + Q2 q2; both ends are
    Gamma.  Corners appear only when they fall on the grid.
    """
    corners = np.array([[0.0, 0.0], [0.5, 0.0], [0.5, 0.5], [0.0, 0.0]])
    seg = np.linalg.norm(np.diff(corners, axis=0), axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    if n_k == 1:
        return corners[:1].copy()
    s = np.linspace(0.0, cum[-1], n_k)
    out = np.empty((n_k, 2))
    for t, si in enumerate(s):
        k = min(int(np.searchsorted(cum, si, side="right")) - 1, len(seg) - 1)
        u = (si - cum[k]) / seg[k]
        out[t] = corners[k] + u * (corners[k + 1] - corners[k])
    return out


# --------------------------------------------------------------------------
# The five synthetic workloads
# --------------------------------------------------------------------------

def config0():
    """Simple cell: r = 0.3 circle on 16x16, 7x7 plane waves, 30 k, 6 bands."""
    return dict(cell=circle_cell(16, 0.3), M=3, Q=kpath_gxmg(30), n_bands=6)


def config1():
    """1132 Voronoi phases on 64x64, 21x21 plane waves, 60 k, 18 bands."""
    rng = rng_for(1, 0)
    sites = rng.uniform(0.0, 1.0, (1132, 2))
    props = random_iso_props(1132, rng)
    phase = voronoi_phase_map(64, 64, sites)
    return dict(cell=Cell(SQUARE.copy(), phase, props), M=10, Q=kpath_gxmg(60), n_bands=18)


def config2(n_cells: int = 256):
    """Seeded two-phase inclusion cells on 32x32 with cutoff M uniform in 5..12."""
    items = []
    for c in range(n_cells):
        rng = rng_for(2, c)
        shape = ("circle", "square", "cross")[int(rng.integers(0, 3))]
        phi = float(rng.uniform(0.1, 0.6))
        M = int(rng.integers(5, 13))
        props = random_iso_props(2, rng)
        phase = inclusion_phase_map(32, shape, phi)
        items.append(dict(cell=Cell(SQUARE.copy(), phase, props), M=M, shape=shape, phi=phi))
    return dict(cells=items, Q=kpath_gxmg(40), n_bands=10)


def config3():
    """4096 Voronoi phases on 128x128, 31x31 plane waves, 60 k, 24 bands."""
    rng = rng_for(3, 0)
    sites = rng.uniform(0.0, 1.0, (4096, 2))
    props = random_iso_props(4096, rng)
    phase = voronoi_phase_map(128, 128, sites)
    return dict(cell=Cell(SQUARE.copy(), phase, props), M=15, Q=kpath_gxmg(60), n_bands=24)


def config4_cells(start: int, stop: int):
    """Binary GRF cells (32x32, ell = 4 px) with fill uniform in [0.2, 0.8].

    Phase 1 is the stiff inclusion material, phase 0 the compliant matrix.
    Returns a uint8 array [stop-start, 32, 32].
    """
    out = np.empty((stop - start, 32, 32), dtype=np.uint8)
    for t, c in enumerate(range(start, stop)):
        rng = rng_for(4, c)
        phi = float(rng.uniform(0.2, 0.8))
        out[t] = grf_phase_map(32, 4.0, phi, rng)
    return out


def workload(name: str):
    return {"c0": config0, "c1": config1, "c2": config2, "c3": config3}[name]()
