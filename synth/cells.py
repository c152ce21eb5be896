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
    "INCLUSION_PROPS", "MATRIX_PROPS", "PolygonCell", "iso_from_c11_c44", "hex_lattice",
    "hex_cylinder_cell", "hex_steel_epoxy", "kpath_xgjx", "hex_graded_1132", "random_voigt_props",
    "voigt_rows_to_matrices",
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


def random_voigt_props(n: int, rng: np.random.Generator, dim: int = 2) -> np.ndarray:
    """Rows of a random symmetric positive-definite engineering-Voigt
    compliance matrix (stress order 11, 22, 12 in the plane; 11, 22, 33, 23,
    13, 12 in space) with every normal-shear coupling non-zero, scaled like
    a 10-300 GPa solid, as its upper triangle row by row, then rho
    log-uniform in [1000, 8000] kg/m^3: 7 values per row in the plane, 22 in
    space."""
    ns = 3 if dim == 2 else 6
    iu = np.triu_indices(ns)
    rows = []
    for _ in range(n):
        B = rng.normal(size=(ns, ns))
        W = (B @ B.T + ns * np.eye(ns)) * 10.0 ** rng.uniform(-11.5, -10.5)
        rho = np.exp(rng.uniform(np.log(1000.0), np.log(8000.0)))
        rows.append(np.concatenate([W[iu], [rho]]))
    return np.array(rows)


def voigt_rows_to_matrices(rows: np.ndarray, dim: int = 2):
    """Per-phase symmetric compliance matrices and densities from rows in the
    layout of ``random_voigt_props``."""
    ns = 3 if dim == 2 else 6
    iu = np.triu_indices(ns)
    rows = np.asarray(rows, dtype=np.float64)
    W = np.zeros((rows.shape[0], ns, ns))
    for p, r in enumerate(rows):
        W[p][iu] = r[:-1]
        W[p] = W[p] + np.triu(W[p], 1).T
    return W, rows[:, -1].copy()


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
# Polygon cells on the hexagonal lattice (the paper's Sec. 5 example geometry)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class PolygonCell:
    lattice: np.ndarray          # [2,2] rows h1, h2 (metres)
    polygons: list               # [n_i, 2] Cartesian vertices; CCW adds, CW subtracts
    poly_phase: np.ndarray       # [n_polys] int32
    props: np.ndarray            # [P, 3] (E, nu, rho)

    @property
    def n_phases(self) -> int:
        return int(self.props.shape[0])


def iso_from_c11_c44(c11: float, c44: float, rho: float):
    """(E, nu, rho) of an isotropic solid given C11 = lambda + 2 mu, C44 = mu."""
    mu = c44
    lam = c11 - 2.0 * c44
    E = mu * (3.0 * lam + 2.0 * mu) / (lam + mu)
    nu = lam / (2.0 * (lam + mu))
    return (E, nu, rho)


# steel cylinders in epoxy (Sec. 5; C11, C44 in Pa, rho in kg/m^3)
STEEL = iso_from_c11_c44(264e9, 81e9, 7780.0)
EPOXY = iso_from_c11_c44(7.54e9, 1.48e9, 1142.0)


def hex_lattice(a: float) -> np.ndarray:
    """Rows h1 = a (1, 0), h2 = a (1/2, sqrt(3)/2)."""
    return np.array([[a, 0.0], [0.5 * a, 0.5 * np.sqrt(3.0) * a]])


def _ngon(centre, radius: float, n: int, ccw: bool = True) -> np.ndarray:
    t = 2.0 * np.pi * np.arange(n) / n
    if not ccw:
        t = -t
    return np.stack([centre[0] + radius * np.cos(t), centre[1] + radius * np.sin(t)], axis=1)


def hex_cylinder_cell(a: float, d: float, inc, mat, n_gon: int = 256) -> PolygonCell:
    """One cylinder of diameter d at the centre of the primitive hexagonal cell.

    Polygons: the cell parallelogram (matrix, CCW), the cylinder as a regular
    n-gon (inclusion, CCW) and the same n-gon clockwise in the matrix phase (the
    hole).  The n-gon's circumradius gives it the disk's area, so the filling
    fraction is exact.
    """
    L = hex_lattice(a)
    h1, h2 = L[0], L[1]
    para = np.array([[0.0, 0.0], h1, h1 + h2, h2])
    centre = 0.5 * (h1 + h2)
    r = 0.5 * d
    R = r * np.sqrt(2.0 * np.pi / (n_gon * np.sin(2.0 * np.pi / n_gon)))
    polys = [para, _ngon(centre, R, n_gon, True), _ngon(centre, R, n_gon, False)]
    phase = np.array([0, 1, 0], dtype=np.int32)
    props = np.array([mat, inc], dtype=np.float64)
    return PolygonCell(L, polys, phase, props)


def hex_steel_epoxy(n_gon: int = 256) -> PolygonCell:
    """Steel cylinders (d = 4 mm) in epoxy, hexagonal lattice a = 6.023 mm (Sec. 5)."""
    return hex_cylinder_cell(6.023e-3, 4.0e-3, STEEL, EPOXY, n_gon)


def hex_graded_1132(a: float = 6.023e-3, n: int = 24, n_quads: int = 20) -> PolygonCell:
    """The 1132-element hexagonal cell of Sec. 5: every element its own phase
    with steel's stiffness (C11 = 264 GPa, C44 = 81 GPa) and the density
    rho_i = 10^6 x (x2 of the element's centroid, metres) kg/m^3.

    Mesh: the primitive cell cut into n x n small parallelograms; the first
    ``n_quads`` stay whole and the others are split into two triangles, which
    gives 2 n^2 - n_quads = 1132 elements for n = 24."""
    L = hex_lattice(a)
    h1, h2 = L[0], L[1]
    polys = []
    for i in range(n):
        for j in range(n):
            p00 = (i / n) * h1 + (j / n) * h2
            p10 = ((i + 1) / n) * h1 + (j / n) * h2
            p11 = ((i + 1) / n) * h1 + ((j + 1) / n) * h2
            p01 = (i / n) * h1 + ((j + 1) / n) * h2
            if len(polys) < n_quads:
                polys.append(np.array([p00, p10, p11, p01]))
            else:
                polys.append(np.array([p00, p10, p11]))
                polys.append(np.array([p00, p11, p01]))
    E, nu, _ = iso_from_c11_c44(264e9, 81e9, 1.0)
    props = np.array([(E, nu, 1e6 * float(np.mean(v[:, 1]))) for v in polys], dtype=np.float64)
    return PolygonCell(L, polys, np.arange(len(polys), dtype=np.int32), props)


def kpath_xgjx(n_k: int) -> np.ndarray:
    """n_k points equally spaced in arc length on X - Gamma - J - X of the
    hexagonal Brillouin zone (X: edge midpoint (1/2, 0), J: corner (2/3, 1/3),
    fractional coordinates of q1, q2 for the lattice of ``hex_lattice``)."""
    corners = np.array([[0.5, 0.0], [0.0, 0.0], [2.0 / 3.0, 1.0 / 3.0], [0.5, 0.0]])
    # arc length in Cartesian k: q1, q2 of the unit hexagonal lattice
    q = 2.0 * np.pi * np.linalg.inv(hex_lattice(1.0)).T
    cart = corners @ q
    seg = np.linalg.norm(np.diff(cart, axis=0), axis=1)
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
