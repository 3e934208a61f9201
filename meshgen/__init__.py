"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module produces inputs only: structured tetrahedral meshes (Kuhn split
of a hexahedral index grid), Lagrange P1/P2 node numbering, nodal temperature
fields, body forces and Dirichlet masks.  It holds none of the finite-element
or solver arithmetic.

Geometry follows the paper's setting of conforming Lagrange spaces on
tetrahedral meshes (Sec. 3.1); the paper's own meshes (Sec. 4.1) are
proprietary, so structured stand-ins of the same element types are generated.

Conventions
-----------
* Kuhn split: each hex of the index grid is cut into 6 tetrahedra around the
  (0,0,0)-(1,1,1) diagonal, one per permutation of the three axes; every cell
  is stored positively oriented.
* P2 cells list 10 nodes: v0..v3 then the edge midpoints in the order
  (01, 02, 03, 12, 13, 23).
* P2 nodes of an n-grid are the P1 nodes of the 2n-grid (every point of the
  doubled grid is a vertex, an edge midpoint, a face-diagonal midpoint or the
  hex centre); midside nodes sit at the midpoint of the *straight* physical
  edge.
* Node numbering is lexicographic with the third logical axis fastest:
  cube (x, y, z) -> id = (i*NY + j)*NZ + k; disc (theta slowest, then r, then
  z fastest) -> id = (j*NR + i)*NZ + k.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

# Permutations of the logical axes, one Kuhn tetrahedron each (fixed order).
_PERMS = list(itertools.permutations(range(3)))
_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


@dataclasses.dataclass
class Mesh:
    """A tetrahedral mesh: coords[N][3] float64, cells[C][4 or 10] int32."""

    coords: np.ndarray
    cells: np.ndarray
    degree: int
    # logical grid index of each node on the (degree * n) grid, [N][3] int64
    grid_index: np.ndarray
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_dof(self) -> int:
        return 3 * self.n_nodes


def _kuhn_local():
    """Local corner offsets (4 x 3) of the 6 Kuhn tets of the unit hex,
    positively oriented: odd permutations get v1 and v2 swapped."""
    tets = []
    for p in _PERMS:
        e = np.eye(3, dtype=np.int64)
        v0 = np.zeros(3, np.int64)
        v1 = v0 + e[p[0]]
        v2 = v1 + e[p[1]]
        v3 = np.ones(3, np.int64)
        vs = [v0, v1, v2, v3]
        det = np.linalg.det(np.array([v1 - v0, v2 - v0, v3 - v0], dtype=float).T)
        if det < 0:
            vs = [v0, v2, v1, v3]
        tets.append(np.array(vs))
    return np.array(tets)  # [6][4][3]


def cube_mesh(n: int, degree: int = 1) -> Mesh:
    """Unit cube [0,1]^3 with n^3 hexes split 6 tets each, P1 or P2."""
    assert degree in (1, 2)
    m = degree * n + 1  # points per axis on the node grid
    idx = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), -1).reshape(-1, 3)
    coords = idx.astype(np.float64) / float(degree * n)

    def node_id(g):
        return (g[..., 0] * m + g[..., 1]) * m + g[..., 2]

    # hex storage order for the cube: x slowest, then y, then z.
    n0 = n1 = n2 = n
    local = _kuhn_local()
    h0, h1, h2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    corners = np.stack([h0.ravel(), h1.ravel(), h2.ravel()], axis=1)
    vert = (corners[:, None, None, :] + local[None]).reshape(-1, 4, 3)
    if degree == 1:
        g = vert
    else:
        mids = np.stack([vert[:, a] + vert[:, b] for a, b in _EDGES], axis=1)
        g = np.concatenate([2 * vert, mids], axis=1)
    cells = node_id(g).astype(np.int32)
    return Mesh(coords=coords, cells=np.ascontiguousarray(cells), degree=degree,
                grid_index=idx.astype(np.int64), name=f"cube{n}_p{degree}")


@dataclasses.dataclass(frozen=True)
class DiscGeom:
    r_in: float = 0.1
    r_out: float = 0.5
    thickness: float = 0.05


def disc_mesh(nr: int, nth: int, nz: int, degree: int = 1, geom: DiscGeom = DiscGeom()) -> Mesh:
    """Hollow cylinder (turbine-disc proxy), index grid (i, j, k) ->
    (r_in + i*dr, 2*pi*j/nth, k*dz), periodic in j, Kuhn split.

    Logical axes for the split are (r, theta, z); nodes are numbered theta
    slowest, then r, then z fastest.
    """
    assert degree in (1, 2)
    d = degree
    NR, NT, NZ = d * nr + 1, d * nth, d * nz + 1
    jj, ii, kk = np.meshgrid(np.arange(NT), np.arange(NR), np.arange(NZ), indexing="ij")
    grid = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.int64)  # (r, th, z) index

    dr = (geom.r_out - geom.r_in) / nr
    dth = 2.0 * math.pi / nth
    dz = geom.thickness / nz

    def vertex_xyz(iv, jv, kv):
        r = geom.r_in + iv * dr
        th = jv * dth
        return np.stack([r * np.cos(th), r * np.sin(th), kv * dz], axis=-1)

    # node physical coordinates: midpoint of the straight edge lo-hi
    lo = grid // d
    hi = (grid + d - 1) // d
    hi_j = hi[:, 1] % nth
    coords = 0.5 * (vertex_xyz(lo[:, 0], lo[:, 1], lo[:, 2]) + vertex_xyz(hi[:, 0], hi_j, hi[:, 2]))

    def node_id(g):
        return (g[..., 1] * NR + g[..., 0]) * NZ + g[..., 2]

    local = _kuhn_local()
    hj, hi_, hk = np.meshgrid(np.arange(nth), np.arange(nr), np.arange(nz), indexing="ij")
    corners = np.stack([hi_.ravel(), hj.ravel(), hk.ravel()], axis=1)
    vert = (corners[:, None, None, :] + local[None]).reshape(-1, 4, 3)
    if d == 1:
        g = vert.copy()
    else:
        mids = np.stack([vert[:, a] + vert[:, b] for a, b in _EDGES], axis=1)
        g = np.concatenate([2 * vert, mids], axis=1)
    g[..., 1] %= NT
    cells = node_id(g).astype(np.int32)
    return Mesh(coords=np.ascontiguousarray(coords), cells=np.ascontiguousarray(cells), degree=d,
                grid_index=grid, name=f"disc{nr}x{nth}x{nz}_p{d}")


# ---------------------------------------------------------------------------
# Dirichlet masks
# ---------------------------------------------------------------------------

def clamp_mask(mesh: Mesh, node_sel: np.ndarray) -> np.ndarray:
    """mask[N][3] uint8 with all three components of the selected nodes set."""
    mask = np.zeros((mesh.n_nodes, 3), np.uint8)
    mask[node_sel] = 1
    return mask


def cube_clamp_x0(mesh: Mesh) -> np.ndarray:
    return clamp_mask(mesh, mesh.grid_index[:, 0] == 0)


def disc_clamp_bore(mesh: Mesh) -> np.ndarray:
    return clamp_mask(mesh, mesh.grid_index[:, 0] == 0)


# ---------------------------------------------------------------------------
# Temperature fields and body forces (seeded)
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Bumps:
    amp: np.ndarray
    width: np.ndarray
    centre: np.ndarray  # [K][3]


def draw_bumps(rng: np.random.Generator, k: int, amp_max: float, geom: DiscGeom = DiscGeom()) -> Bumps:
    """k Gaussian hot spots; centres uniform in the annulus volume.
    Draw order: amplitudes, widths, r^2, theta, z (each as a length-k array)."""
    amp = rng.uniform(0.0, amp_max, k)
    width = rng.uniform(0.02, 0.1, k)
    rc = np.sqrt(rng.uniform(geom.r_in ** 2, geom.r_out ** 2, k))
    th = rng.uniform(0.0, 2.0 * math.pi, k)
    zc = rng.uniform(0.0, geom.thickness, k)
    centre = np.stack([rc * np.cos(th), rc * np.sin(th), zc], axis=1)
    return Bumps(amp, width, centre)


def bump_sum(coords: np.ndarray, b: Bumps) -> np.ndarray:
    out = np.zeros(coords.shape[0])
    for a, w, c in zip(b.amp, b.width, b.centre):
        d2 = ((coords - c[None, :]) ** 2).sum(axis=1)
        out += a * np.exp(-d2 / (2.0 * w * w))
    return out


def disc_temperature_ramp(mesh: Mesh, seed: int = 0, n_bumps: int = 8, amp_max: float = 200.0,
                          geom: DiscGeom = DiscGeom()) -> np.ndarray:
    """Radial ramp 300 -> 900 K from bore to rim plus seeded Gaussian hot spots."""
    rng = np.random.default_rng(seed)
    r = np.hypot(mesh.coords[:, 0], mesh.coords[:, 1])
    T = 300.0 + 600.0 * (r - geom.r_in) / (geom.r_out - geom.r_in)
    return T + bump_sum(mesh.coords, draw_bumps(rng, n_bumps, amp_max, geom))


def disc_temperature_bumps(mesh: Mesh, seed: int, T_ref: float = 300.0, amp_max: float = 500.0,
                           geom: DiscGeom = DiscGeom()) -> np.ndarray:
    """T_ref plus a seeded sum of 4..16 Gaussian bumps (load-case family)."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(4, 17))
    return T_ref + bump_sum(mesh.coords, draw_bumps(rng, k, amp_max, geom))


def body_force_case(mesh: Mesh, seed: int) -> np.ndarray | None:
    """Seeded body force for the learned-guess data set: zero for half of the
    seeds (even seed -> None), otherwise a uniform force of random direction
    with magnitude U[0.5e9, 2e9] N/m^3 (displacement comparable to the
    thermal one for steel-like material)."""
    if seed % 2 == 0:
        return None
    rng = np.random.default_rng(seed + 7_777_777)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    mag = rng.uniform(0.5e9, 2.0e9)
    return np.tile(d * mag, (mesh.n_nodes, 1))


def random_unit(rng, n):
    return rng.uniform(-1.0, 1.0, n)


# ---------------------------------------------------------------------------
# Boundary faces, material regions and boundary pressure
# ---------------------------------------------------------------------------
# A face opposite each local vertex of a tetrahedron (local vertex triples).
_TET_FACES = [(1, 2, 3), (0, 3, 2), (0, 1, 3), (0, 2, 1)]
# Edge nodes of a P2 face in the order 01, 02, 12 of the face's vertices.
_FACE_EDGES = [(0, 1), (0, 2), (1, 2)]


def boundary_faces(mesh: Mesh, select=None) -> np.ndarray:
    """Triangles that belong to exactly one cell, ordered so that
    (x1 - x0) x (x2 - x0) points out of that cell: [F][3] vertex ids (P1), or
    [F][6] with the edge nodes 01, 02, 12 of that vertex order (P2), sorted
    by their vertex triple.  `select(centroids [F][3]) -> bool[F]` keeps a
    subset."""
    cells = mesh.cells.astype(np.int64)
    tri = np.array(_TET_FACES)
    verts = cells[:, tri]                                  # [C,4,3] local triple -> global ids
    key = np.sort(verts, axis=2).reshape(-1, 3)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    once = np.nonzero(cnt[inv.ravel()] == 1)[0]
    c_of, f_of = once // 4, once % 4
    v = verts[c_of, f_of]                                  # [F,3]
    x = mesh.coords[v]
    nrm = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    opp = mesh.coords[cells[c_of, f_of]]                   # local vertex f is opposite face f
    flip = np.einsum("fi,fi->f", nrm, x.mean(axis=1) - opp) < 0
    v[flip] = v[flip][:, [0, 2, 1]]
    if mesh.degree == 2:
        # edge node of global vertices (a, b) in cell c: its local edge index
        loc = np.argmax(cells[c_of][:, None, :4] == v[:, :, None], axis=2)  # [F,3] local vertex of each face vertex
        edge_ids = {e: i for i, e in enumerate(_EDGES)}
        mids = np.empty((v.shape[0], 3), np.int64)
        for k, (a, b) in enumerate(_FACE_EDGES):
            la, lb = loc[:, a], loc[:, b]
            lo, hi = np.minimum(la, lb), np.maximum(la, lb)
            e = np.array([edge_ids[(int(p), int(q))] for p, q in zip(lo, hi)], dtype=np.int64)
            mids[:, k] = cells[c_of, 4 + e]
        v = np.concatenate([v, mids], axis=1)
    order = np.lexsort(np.sort(v[:, :3], axis=1).T[::-1])
    v = v[order]
    if select is not None:
        v = v[np.asarray(select(mesh.coords[v[:, :3]].mean(axis=1)), dtype=bool)]
    return np.ascontiguousarray(v.astype(np.int32))


@dataclasses.dataclass
class Materials:
    """Temperature tables [n_materials][n_points] (T ascending) of E, nu and
    alpha_L, and the material of every cell."""
    T: np.ndarray
    E: np.ndarray
    nu: np.ndarray
    alpha: np.ndarray
    cell_material: np.ndarray


def turbine_material_tables():
    """Three illustrative metals sampled at 250..1000 K (the paper shows
    normalised temperature curves only): stiffness falling and expansion and
    Poisson ratio rising with temperature."""
    Tp = np.linspace(250.0, 1000.0, 6)
    s = (Tp - 250.0) / 750.0
    rows = []
    for E0, a0, dE, da in ((205e9, 1.15e-5, 0.28, 0.38), (195e9, 1.30e-5, 0.22, 0.30), (215e9, 1.05e-5, 0.33, 0.45)):
        rows.append((E0 * (1.0 - dE * s * (1.0 + 0.4 * s)), np.full_like(s, 0.0) + 0.29 + 0.03 * s,
                     a0 * (1.0 + da * s * (1.0 - 0.2 * s))))
    E = np.array([r[0] for r in rows])
    nu = np.array([r[1] for r in rows])
    alpha = np.array([r[2] for r in rows])
    return np.tile(Tp, (3, 1)), E, nu, alpha


def disc_materials(mesh: Mesh, geom: DiscGeom = DiscGeom()) -> Materials:
    """Hub, web and rim of the disc as three materials by the radius of the
    cell centroid (radial thirds)."""
    c = mesh.coords[mesh.cells[:, :4].astype(np.int64)].mean(axis=1)
    r = np.hypot(c[:, 0], c[:, 1])
    t = (r - geom.r_in) / (geom.r_out - geom.r_in)
    cm = np.minimum(2, (3.0 * t).astype(np.int64)).astype(np.int32)
    Tp, E, nu, alpha = turbine_material_tables()
    return Materials(Tp, E, nu, alpha, np.ascontiguousarray(cm))


def disc_pressure_faces(mesh: Mesh, p_rim: float = 4.0e7, p_top: float = -5.0e6, geom: DiscGeom = DiscGeom()):
    """Boundary pressure of the disc: traction p_rim n on the outer rim (blade
    pull, outward) and p_top n on the upper face (gas pressure, compressive).
    Returns (faces, p)."""
    faces = boundary_faces(mesh)
    x = mesh.coords[faces[:, :3].astype(np.int64)]
    rim = np.all(np.hypot(x[..., 0], x[..., 1]) > geom.r_out * (1 - 1e-6), axis=1)
    top = np.all(x[..., 2] > geom.thickness * (1 - 1e-9), axis=1)
    keep = rim | top
    p = np.where(rim, p_rim, p_top)[keep]
    return np.ascontiguousarray(faces[keep]), np.ascontiguousarray(p.astype(np.float64))


@dataclasses.dataclass
class ThermalMaterials:
    """Temperature tables [n_materials][n_points] (T ascending) of the thermal
    conductivity kappa (W/(m K)) and specific heat c_v (J/(kg K)), the density
    rho [n_materials] (kg/m^3), and the material of every cell."""
    T: np.ndarray
    kappa: np.ndarray
    cv: np.ndarray
    rho: np.ndarray
    cell_material: np.ndarray


def turbine_thermal_tables():
    """Three illustrative metals sampled at 250..1000 K (the paper shows
    normalised conductivity and specific-heat curves only): conductivity
    falling for the first, rising for the other two, specific heat rising."""
    Tp = np.linspace(250.0, 1000.0, 6)
    s = (Tp - 250.0) / 750.0
    kappa = np.array([26.0 * (1.0 - 0.25 * s), 14.0 * (1.0 + 0.6 * s), 21.0 * (1.0 + 0.35 * s * (1.0 - 0.3 * s))])
    cv = np.array([450.0 * (1.0 + 0.35 * s), 430.0 * (1.0 + 0.45 * s), 470.0 * (1.0 + 0.3 * s)])
    rho = np.array([7850.0, 8190.0, 7750.0])
    return np.tile(Tp, (3, 1)), kappa, cv, rho


def disc_thermal_materials(mesh: Mesh, geom: DiscGeom = DiscGeom()) -> ThermalMaterials:
    """Hub, web and rim (radial thirds of the cell centroid, as
    disc_materials) with the thermal tables above."""
    cm = disc_materials(mesh, geom).cell_material
    Tp, kappa, cv, rho = turbine_thermal_tables()
    return ThermalMaterials(Tp, kappa, cv, rho, cm)


@dataclasses.dataclass
class RobinFaces:
    """Heat-transfer boundary faces (the triangles of boundary_faces), with a
    heat-transfer coefficient h >= 0 (W/(m^2 K)) and an exterior temperature
    T_bc (K) per face."""
    faces: np.ndarray
    h: np.ndarray
    T_bc: np.ndarray


def disc_robin_faces(mesh: Mesh, geom: DiscGeom = DiscGeom(), T_rim=900.0, T_bore=350.0, T_side=600.0,
                     h_rim=1500.0, h_bore=800.0, h_side=150.0) -> RobinFaces:
    """Every boundary face of the disc exchanges heat: hot gas at the rim,
    cooling air in the bore, and a moderate exchange on the two flat faces."""
    faces = boundary_faces(mesh)
    x = mesh.coords[faces[:, :3].astype(np.int64)]
    r = np.hypot(x[..., 0], x[..., 1])
    rim = np.all(r > geom.r_out * (1 - 1e-6), axis=1)
    bore = np.all(r < geom.r_in * (1 + 1e-6), axis=1)
    h = np.where(rim, h_rim, np.where(bore, h_bore, h_side))
    Tb = np.where(rim, T_rim, np.where(bore, T_bore, T_side))
    return RobinFaces(faces, np.ascontiguousarray(h, dtype=np.float64), np.ascontiguousarray(Tb, dtype=np.float64))


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    mesh: Mesh
    E: float
    nu: float
    alpha: float
    T_ref: float
    T: np.ndarray
    f: np.ndarray | None
    mask: np.ndarray
    name: str


def cube_problem(n: int = 16, degree: int = 1) -> Problem:
    """Unit cube, E=1, nu=0.3, alpha=1e-3, uniform dT=1, clamped at x=0, f=0."""
    m = cube_mesh(n, degree)
    return Problem(m, 1.0, 0.3, 1e-3, 300.0, np.full(m.n_nodes, 301.0), None,
                   cube_clamp_x0(m), f"cube{n}_p{degree}")


def disc_problem(nr: int, nth: int, nz: int, degree: int = 2, seed: int = 0) -> Problem:
    """Steel disc: E=200e9, nu=0.3, alpha=1.2e-5, ramp + 8 hot spots, bore clamped."""
    m = disc_mesh(nr, nth, nz, degree)
    return Problem(m, 200e9, 0.3, 1.2e-5, 300.0, disc_temperature_ramp(m, seed), None,
                   disc_clamp_bore(m), f"disc{nr}x{nth}x{nz}_p{degree}")


# Full-size workload grids (nr, ntheta, nz, degree)
DISC_P2_12M = (96, 416, 12, 2)     # 4,014,400 nodes, 12,043,200 DOF
DISC_P1_2M = (104, 452, 13, 1)     # 664,440 nodes, 1,993,320 DOF
DISC_P1_1M = (80, 344, 11, 1)      # 334,368 nodes, 1,003,104 DOF


def multi_mesh_sizes(n_mesh: int = 32, seed0: int = 2000, lo: float = 1e4, hi: float = 5e5):
    """Grids of the multi-mesh batch: target DOF log-uniform in [lo, hi];
    (nr, ntheta, nz) = round(s * (8, 34.7, 1)), nz >= 2, P1."""
    out = []
    for m in range(n_mesh):
        rng = np.random.default_rng(seed0 + m)
        target = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        # DOF ~ 3 * (8s+1) * 34.7s * (s+1) ~ 3*277.6 s^3
        s = (target / (3 * 8 * 34.7)) ** (1.0 / 3.0)
        nr = max(2, int(round(8 * s)))
        nth = max(8, int(round(34.7 * s)))
        nz = max(2, int(round(s)))
        out.append((nr, nth, nz, seed0 + m))
    return out
