"""Seeded synthetic problem generators (inputs only).

This module produces meshes, per-element orders p and density-grid sizes d,
density fields, supports and point loads.  It holds none of the method's
arithmetic (no basis, stiffness, solve or sensitivity): both the HIP library
and the CPU oracle consume its output as plain arrays.

The paper's own density fields exist only as figures, so seeded random
fields of the same character stand in for them: structured square-element
meshes, point-loaded cantilever / MBB beams (Sec. 4.1), E0 = 1, nu = 0.3,
q = 3, Emin = 1e-9 E0 (Sec. 2.2, Sec. 4.1), volume fractions in the paper's
range.

Random field z: seeded white noise smoothed by a Gaussian of length sigma
(element widths) and scaled to unit variance (``RandomField``), evaluated at
cell centres, so it does not depend on d.

Density map: rho = clip(0.5 + 0.5 z - t, rho_min, 1) with the shift t found
by bisection so that the area-weighted mean density equals the volume
fraction.  This plain field is the default of the five workload
configurations.  With ``solid_paths=True`` the cells on the load paths are
also made solid (rho = 1): a pad of radius LOAD_PAD around each point load
and a beam of half-width BEAM_HALF_WIDTH from the clamped edge to it, as the
paper's optimised designs carry every load through material to the
supports.  That eased field conditions K better; the small parity meshes and
the force inverter use it, so that a tiny mesh does not leave its load on
void material.

dp rule for mixed meshes (an element is 'solid' when z at its centre >= 0,
i.e. the [0, 1]-mapped field is >= 0.5, or, with solid_paths, it lies on a
load path): elements whose centre lies within 3
element widths of an element on the solid/void contour (one with a
4-neighbour of the other class) get p = 4, d = 5; other solid elements get
p = 2, d = 2 and other void elements p = 1, d = 1.  Then neighbouring orders
are brought within 2 of each other by raising the lower one (the smoothing
step of the dp-adaptivity algorithm, Sec. 3.3), which keeps d.
"""

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

SUP_VERTEX, SUP_EDGE_LEFT, SUP_EDGE_RIGHT, SUP_EDGE_BOTTOM, SUP_EDGE_TOP = 0, 1, 2, 3, 4

# Gaussian smoothing length (element widths) of the mixed-mesh configs; fixed
# once so that about a fifth of a 200 x 100 mesh is refined.
MIXED_SIGMA = 12.0
# Radius (element widths) of the solid pad around each point load, and the
# half-width of the solid beam that joins each load to the clamped edge.
LOAD_PAD = 2.0
BEAM_HALF_WIDTH = 2.0


@dataclass
class Problem:
    name: str
    nelx: int
    nely: int
    p: np.ndarray                      # int8 [nel], e = ey*nelx + ex
    d: np.ndarray                      # int8 [nel]
    rho: np.ndarray                    # float64 [sum d^2], element-major, cell sy*d+sx
    supports: List[Tuple[int, int, int, int]] = field(default_factory=list)  # (kind, a, b, mask)
    loads: List[Tuple[int, int, float, float, int]] = field(default_factory=list)  # (vx, vy, fx, fy, lc)
    n_load_cases: int = 1
    springs: List[Tuple[int, int, int, float]] = field(default_factory=list)  # (vx, vy, comp, k) to ground
    E0: float = 1.0
    Emin: float = 1e-9
    nu: float = 0.3
    q: float = 3.0

    @property
    def nel(self):
        return self.nelx * self.nely

    @property
    def n_cells(self):
        return int(self.rho.size)

    def cell_offsets(self):
        d = self.d.astype(np.int64)
        return np.concatenate([[0], np.cumsum(d * d)])

    def oracle_args(self):
        """Keyword arguments for the oracle's solve."""
        return dict(nelx=self.nelx, nely=self.nely, p=self.p, d=self.d, rho=self.rho,
                    supports=self.supports, loads=self.loads, n_load_cases=self.n_load_cases,
                    E0=self.E0, Emin=self.Emin, nu=self.nu, q=self.q, springs=self.springs)


class RandomField:
    """Standardised Gaussian-smoothed white noise, bilinearly interpolated.

    Seeded i.i.d. N(0, 1) noise on a grid of spacing h (element widths) that
    covers the mesh plus a margin of 4 sigma, convolved with a Gaussian of
    standard deviation sigma (periodic on the padded grid) and scaled to unit
    variance; values at arbitrary points by bilinear interpolation.
    """

    def __init__(self, seed, sigma, nelx, nely, h=0.5):
        from scipy import ndimage

        rng = np.random.default_rng(seed)
        self.h = h
        self.pad = float(np.ceil(4.0 * sigma))
        nx = int(np.ceil((nelx + 2 * self.pad) / h)) + 1
        ny = int(np.ceil((nely + 2 * self.pad) / h)) + 1
        noise = rng.standard_normal((ny, nx))
        s = sigma / h
        # unit variance: sum of squared weights of a normalised 2D Gaussian
        # kernel of std s is 1 / (4 pi s^2)
        self.grid = ndimage.gaussian_filter(noise, s, mode="wrap", truncate=4.0) * (2.0 * np.sqrt(np.pi) * s)
        self._nd = ndimage

    def __call__(self, x, y):
        x = np.asarray(x, dtype=np.float64).ravel()
        y = np.asarray(y, dtype=np.float64).ravel()
        coords = np.stack([(y + self.pad) / self.h, (x + self.pad) / self.h])
        return self._nd.map_coordinates(self.grid, coords, order=1, mode="nearest")


def cell_centres(nelx, nely, d):
    """Centres (x, y) and areas of every density cell, element-major."""
    d = np.asarray(d, dtype=np.int64).ravel()
    off = np.concatenate([[0], np.cumsum(d * d)])
    n = int(off[-1])
    xs, ys, ws = np.empty(n), np.empty(n), np.empty(n)
    els = np.arange(nelx * nely)
    for de in np.unique(d):
        de = int(de)
        sel = els[d == de]
        t = (np.arange(de) + 0.5) / de
        sx = np.tile(t, de)       # cell s = sy*d + sx
        sy = np.repeat(t, de)
        idx = off[sel][:, None] + np.arange(de * de)[None, :]
        xs[idx] = (sel % nelx)[:, None] + sx[None, :]
        ys[idx] = (sel // nelx)[:, None] + sy[None, :]
        ws[idx] = 1.0 / (de * de)
    return xs, ys, ws


def map_density(z, weights, volfrac, rho_min=1e-3, solid=None):
    """rho = clip(0.5 + 0.5 z - t, rho_min, 1) (1 on the `solid` mask), with
    t by bisection so that the area-weighted mean is volfrac."""
    wsum = weights.sum()
    if solid is None:
        solid = np.zeros(z.shape, dtype=bool)

    def field(t):
        return np.where(solid, 1.0, np.clip(0.5 + 0.5 * z - t, rho_min, 1.0))

    lo, hi = -10.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if float(np.dot(field(mid), weights) / wsum) > volfrac:
            lo = mid
        else:
            hi = mid
        if hi - lo < 1e-13:
            break
    return field(0.5 * (lo + hi))


def load_paths(x, y, loads, pad=LOAD_PAD, half_width=BEAM_HALF_WIDTH):
    """Solid mask at points (x, y): a pad of radius `pad` around each loaded
    vertex and a horizontal beam of half-width `half_width` from the clamped
    edge x = 0 to it.  The paper's optimised designs carry every load through
    material to the supports; a random field alone at a low volume fraction
    leaves the loads on void (E = Emin) with compliances of order 1e9."""
    solid = np.zeros(np.shape(x), dtype=bool)
    for vx, vy, *_ in loads:
        solid |= (x - vx) ** 2 + (y - vy) ** 2 <= pad * pad
        solid |= (np.abs(y - vy) <= half_width) & (x <= vx)
    return solid


def smooth_orders(p, nelx, nely, max_jump=2):
    """Raise the lower order until neighbouring elements differ by <= max_jump."""
    p = p.reshape(nely, nelx).copy()
    while True:
        changed = False
        for dy, dx in ((0, 1), (1, 0)):
            a = p[: nely - dy, : nelx - dx]
            b = p[dy:, dx:]
            lo_a = a < b - max_jump
            lo_b = b < a - max_jump
            if lo_a.any() or lo_b.any():
                changed = True
                a[lo_a] = b[lo_a] - max_jump
                b[lo_b] = a[lo_b] - max_jump
        if not changed:
            return p.ravel()


def dp_rule(nelx, nely, fieldfn, band=3.0, loads=()):
    """Per-element (p, d) of the mixed-mesh configs (see the module docstring);
    elements on the load paths of `loads` (empty: none) count as solid."""
    from scipy import ndimage

    ex, ey = np.meshgrid(np.arange(nelx) + 0.5, np.arange(nely) + 0.5)
    solid = (fieldfn(ex.ravel(), ey.ravel()) >= 0.0) | load_paths(ex.ravel(), ey.ravel(), loads)
    solid = solid.reshape(nely, nelx)
    contour = np.zeros_like(solid)
    contour[:, :-1] |= solid[:, :-1] != solid[:, 1:]
    contour[:, 1:] |= solid[:, :-1] != solid[:, 1:]
    contour[:-1, :] |= solid[:-1, :] != solid[1:, :]
    contour[1:, :] |= solid[:-1, :] != solid[1:, :]
    if contour.any():
        dist = ndimage.distance_transform_edt(~contour)
    else:
        dist = np.full(solid.shape, np.inf)
    refined = dist <= band
    p = np.where(refined, 4, np.where(solid, 2, 1)).ravel()
    d = np.where(refined, 5, np.where(solid, 2, 1)).ravel()
    p = smooth_orders(p, nelx, nely)
    return p.astype(np.int8), d.astype(np.int8)


def cantilever_supports():
    return [(SUP_EDGE_LEFT, 0, 0, 3)]


def mbb_20x10(seed=1):
    """MBB half-beam, 20 x 10, p = 1, d = 2, rho = 0.5 + U[-0.4, 0.4] per cell;
    u_x = 0 on the left edge (symmetry), u_y = 0 at the bottom-right vertex,
    unit downward load at the top-left vertex."""
    nelx, nely = 20, 10
    rng = np.random.default_rng(seed)
    p = np.full(nelx * nely, 1, np.int8)
    d = np.full(nelx * nely, 2, np.int8)
    rho = 0.5 + rng.uniform(-0.4, 0.4, size=nelx * nely * 4)
    sup = [(SUP_EDGE_LEFT, 0, 0, 1), (SUP_VERTEX, nelx, 0, 2)]
    loads = [(0, nely, 0.0, -1.0, 0)]
    return Problem("mbb20x10_p1d2", nelx, nely, p, d, rho, sup, loads, 1)


def cantilever_uniform(nelx=160, nely=80, p=3, d=4, sigma=8.0, volfrac=0.4, seed=2, solid_paths=False):
    """Clamped-left cantilever with uniform (p, d), density from the random
    field (length scale sigma) mapped to [0.001, 1] at mean volfrac, unit
    downward load at the mid-right vertex (solid_paths: see the module
    docstring)."""
    pa = np.full(nelx * nely, p, np.int8)
    da = np.full(nelx * nely, d, np.int8)
    fld = RandomField(seed, sigma, nelx, nely)
    x, y, w = cell_centres(nelx, nely, da)
    loads = [(nelx, nely // 2, 0.0, -1.0, 0)]
    rho = map_density(fld(x, y), w, volfrac, solid=load_paths(x, y, loads) if solid_paths else None)
    return Problem(f"cantilever{nelx}x{nely}_p{p}d{d}", nelx, nely, pa, da, rho,
                   cantilever_supports(), loads, 1)


def mixed_cantilever(nelx=200, nely=100, volfrac=0.5, seed=3, load_vy=None, sigma=MIXED_SIGMA,
                     solid_paths=False):
    """Clamped-left cantilever on a dp-mixed mesh from the dp rule; point loads
    f_y = -1 at the given right-edge vertices (one load case each);
    solid_paths: see the module docstring."""
    fld = RandomField(seed, sigma, nelx, nely)
    if load_vy is None:
        load_vy = [nely // 2]
    loads = [(nelx, int(vy), 0.0, -1.0, lc) for lc, vy in enumerate(load_vy)]
    paths = loads if solid_paths else ()
    p, d = dp_rule(nelx, nely, fld, loads=paths)
    x, y, w = cell_centres(nelx, nely, d)
    rho = map_density(fld(x, y), w, volfrac, solid=load_paths(x, y, paths) if solid_paths else None)
    return Problem(f"mixed{nelx}x{nely}", nelx, nely, p, d, rho, cantilever_supports(), loads,
                   len(load_vy))


def force_inverter(nelx=40, nely=20, p=2, d=4, volfrac=0.45, seed=7, sigma=4.0):
    """Force inverter of Sec. 4.1 as the half model symmetric about its bottom
    edge (the paper's 40 x 20 initial mesh of Q2 elements with 4 x 4 design
    points; E0 = 1, nu = 0.3, q = 3): u_y = 0 on the bottom edge, the top-left
    vertex clamped (the support segment of 0.01 L is shorter than an element),
    input force f_in = 1 in +x at the bottom-left vertex with a spring
    k_in = 1, output at the bottom-right vertex with a spring k_out = 0.001,
    both in x.  Load case 0 is f_in; load case 1 is the unit load at the
    output DOF, the right-hand side z of the adjoint solve (K is symmetric).
    The objective is z^T u = u_x at the output (Eq. (1)).  Density: the
    random field at mean volfrac, solid along the load paths.
    Returns the Problem; its attributes in_dof and out_dof are (vx, vy, comp)."""
    pa = np.full(nelx * nely, p, np.int8)
    da = np.full(nelx * nely, d, np.int8)
    fld = RandomField(seed, sigma, nelx, nely)
    x, y, w = cell_centres(nelx, nely, da)
    loads = [(0, 0, 1.0, 0.0, 0), (nelx, 0, 1.0, 0.0, 1)]
    rho = map_density(fld(x, y), w, volfrac, solid=load_paths(x, y, loads))
    sup = [(SUP_EDGE_BOTTOM, 0, 0, 2), (SUP_VERTEX, 0, nely, 3)]
    springs = [(0, 0, 0, 1.0), (nelx, 0, 0, 0.001)]
    pr = Problem(f"inverter{nelx}x{nely}_p{p}d{d}", nelx, nely, pa, da, rho, sup, loads, 2, springs)
    pr.in_dof = (0, 0, 0)
    pr.out_dof = (nelx, 0, 0)
    return pr


def mixed_200x100(seed=3, solid_paths=False):
    return mixed_cantilever(200, 100, 0.5, seed, solid_paths=solid_paths)


def batch_instances(n=64, first_seed=100, lo=20, hi=160, solid_paths=False):
    """Uneven batch: nelx = 2 round(exp(U[ln lo, ln hi])), nely = nelx / 2,
    dp rule, mean density 0.5, 1-3 load cases at distinct right-edge vertices
    (solid_paths: see the module docstring)."""
    out = []
    for k in range(n):
        seed = first_seed + k
        rng = np.random.default_rng(seed)
        nelx = 2 * int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
        nely = nelx // 2
        nl = int(rng.integers(1, 4))
        vys = rng.choice(np.arange(1, nely), size=nl, replace=False)
        prob = mixed_cantilever(nelx, nely, 0.5, seed, load_vy=sorted(int(v) for v in vys),
                                solid_paths=solid_paths)
        prob.name = f"batch{k}_{nelx}x{nely}"
        out.append(prob)
    return out


def autograd_400x200(seed=5, solid_paths=False):
    """400 x 200 mixed mesh, mean density 0.2, three load cases at right-edge
    vertices nely/4, nely/2, 3 nely/4."""
    nelx, nely = 400, 200
    return mixed_cantilever(nelx, nely, 0.2, seed, load_vy=[nely // 4, nely // 2, 3 * nely // 4],
                            solid_paths=solid_paths)


def small_mixed(nelx, nely, seed, volfrac=0.5, sigma=3.0, n_loads=1, solid_paths=True):
    """Small mixed-mesh cantilever for parity tests (same dp rule, shorter
    field length so a small mesh still has all four (p, d) groups; solid load
    paths by default, so that a load is not left on void)."""
    nl = n_loads
    vys = [max(1, (k + 1) * nely // (nl + 1)) for k in range(nl)]
    return mixed_cantilever(nelx, nely, volfrac, seed, load_vy=vys, sigma=sigma, solid_paths=solid_paths)


def uniform_random(nelx, nely, p, d, seed, supports=None, loads=None, n_load_cases=1,
                   lo=0.1, hi=1.0):
    """Uniform (p, d) mesh with i.i.d. uniform densities (small parity cases)."""
    rng = np.random.default_rng(seed)
    pa = np.full(nelx * nely, p, np.int8) if np.isscalar(p) else np.asarray(p, np.int8)
    da = np.full(nelx * nely, d, np.int8) if np.isscalar(d) else np.asarray(d, np.int8)
    n_cells = int((da.astype(np.int64) ** 2).sum())
    rho = rng.uniform(lo, hi, size=n_cells)
    if supports is None:
        supports = cantilever_supports()
    if loads is None:
        loads = [(nelx, nely // 2, 0.0, -1.0, 0)]
    return Problem(f"uniform{nelx}x{nely}", nelx, nely, pa, da, rho, supports, loads, n_load_cases)


def config(k, solid_paths=False):
    """The five workload configurations, by number 1..5 (4 returns a list).
    Default: the plain random density field; solid_paths=True gives the eased
    field with solid load paths (configs 2-5; config 1 has i.i.d. densities)."""
    if k == 1:
        return mbb_20x10()
    if k == 2:
        return cantilever_uniform(solid_paths=solid_paths)
    if k == 3:
        return mixed_200x100(solid_paths=solid_paths)
    if k == 4:
        return batch_instances(solid_paths=solid_paths)
    if k == 5:
        return autograd_400x200(solid_paths=solid_paths)
    raise ValueError(k)
