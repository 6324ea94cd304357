"""Seeded synthetic workloads and inputs, shared by the tests, the bench and the oracle.

This module holds configuration data only -- grid sizes, velocity grids, gas
constants and boundary conditions -- plus seeded random inputs.  It contains
none of the method's arithmetic, so both the GPU binding and the CPU oracle can
read the same case description without sharing any computation.

The workloads stand in for the paper's test problems, whose meshes and
reference data are not published: a 3-D lid-driven cavity for the 2-D cavity
of Sec. 5.1, and a cube in a Ma = 5 stream for the Apollo reentry capsule of
Sec. 5.2.  Velocities are in units of the most probable speed sqrt(2 R T0),
lengths in the cavity side (or the block side).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

WALL = 0
INFLOW = 1

MONATOMIC = 0
DIATOMIC = 1

# Nitrogen (Sec. 5): internal degrees of freedom, rotational collision number,
# viscosity index and the heat-flux relaxation rates A_tt, A_tr, A_rt, A_rr.
N2_DR = 2.0
N2_ZR = 3.5
N2_OMEGA = 0.74
N2_A = (0.786, -0.201, -0.059, 0.842)


@dataclasses.dataclass
class Boundary:
    kind: int = WALL
    u: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    T: float = 1.0
    rho: float = 1.0


@dataclasses.dataclass
class Case:
    """One problem: uniform hex cells, tensor velocity grid, gas, boundaries.

    ``bcs`` has 7 entries: the box faces -x, +x, -y, +y, -z, +z and the surface
    of solid cells.  ``solid`` is a uint8 array of nx*ny*nz (x fastest) or None.
    """
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    ly: float
    lz: float
    nv: Tuple[int, int, int]
    vmin: Tuple[float, float, float]
    vmax: Tuple[float, float, float]
    Kn: float
    omega: float = 0.75
    species: int = MONATOMIC
    dr: float = 0.0
    Zr: float = 1.0
    A: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    inv_dt: float = 0.0
    conservative: int = 1
    macro_cfl: float = 10.0
    # spatial order of the explicit interface values of the kinetic update
    # (1 first-order upwind; 2 least-squares reconstruction with the
    # Venkatakrishnan limiter, eps^2 = (limiter_k h)^3 times the square of
    # the stencil's largest |f|, limiter_k < 0: none).  K = 0.3 to 1 suits the
    # cavities; the strict K = 0 switches at smooth extrema (FP32 and FP64
    # then part by 1e-4); the Mach-5 block flows lose positivity in the wake
    # at second order beyond the smallest grids whatever K, so they run first
    # order
    order: int = 1
    limiter_k: float = 1.0
    # macroscopic boundary flux of the GSIS correction: 0 the kinetic flux plus
    # the change of the cell Maxwellian's flux, 1 the same with the Grad-13
    # distributions of the iterate's state, stress and heat fluxes (Sec. 3.3)
    wall_flux: int = 0
    bcs: List[Boundary] = dataclasses.field(default_factory=lambda: [Boundary() for _ in range(7)])
    solid: Optional[np.ndarray] = None
    init: Tuple[float, Tuple[float, float, float], float, float] = (1.0, (0.0, 0.0, 0.0), 1.0, 1.0)
    # optional node positions per axis (strictly increasing, nv[a] each); None:
    # nv[a] uniform nodes on [vmin[a], vmax[a]]
    nodes: Optional[Tuple[Optional[np.ndarray], Optional[np.ndarray], Optional[np.ndarray]]] = None
    # optional general velocity set, [n][4] = (xi_x, xi_y, xi_z, w): one node per
    # velocity cell of a refined or unstructured mesh, its weight the cell's
    # volume; replaces the tensor grid (nv, vmin, vmax and nodes are then unused)
    velocity_list: Optional[np.ndarray] = None
    # optional unstructured spatial mesh (SpatialMesh): replaces the box of
    # nx x ny x nz hex cells (nx then holds the cell count, ny = nz = 1, and
    # solid cells are simply not part of the mesh)
    mesh: Optional["SpatialMesh"] = None
    # iteration plan of the workload
    passes: int = 10
    gsis: bool = False
    macro_iters: int = 300
    tol: float = 1e-6
    max_iters: int = 100

    @property
    def ncell(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def nvel(self) -> int:
        if self.velocity_list is not None:
            return int(self.velocity_list.shape[0])
        return self.nv[0] * self.nv[1] * self.nv[2]

    @property
    def nfluid(self) -> int:
        return self.ncell - (0 if self.solid is None else int(self.solid.sum()))

    def solid_mask(self) -> np.ndarray:
        if self.solid is None:
            return np.zeros(self.ncell, dtype=np.uint8)
        return np.ascontiguousarray(self.solid, dtype=np.uint8)


def cavity(n: int, m: int, Kn: float, lid: float = 0.1, vmax: float = 4.0, omega: float = 0.75,
           name: str = "cavity", lid_axis: int = 0, **kw) -> Case:
    """Lid-driven cubic cavity: n^3 cells on the unit cube, m^3 nodes on [-vmax, vmax]^3,
    diffuse walls at T = 1, the z = 1 face moving with speed ``lid`` along ``lid_axis``."""
    bcs = [Boundary(WALL, (0.0, 0.0, 0.0), 1.0) for _ in range(7)]
    u = [0.0, 0.0, 0.0]
    u[lid_axis] = lid
    bcs[5] = Boundary(WALL, tuple(u), 1.0)
    return Case(name=name, nx=n, ny=n, nz=n, lx=1.0, ly=1.0, lz=1.0, nv=(m, m, m),
                vmin=(-vmax,) * 3, vmax=(vmax,) * 3, Kn=Kn, omega=omega, bcs=bcs, **kw)


def free_stream_speed(Ma: float, gamma: float) -> float:
    """Speed of a Mach-Ma stream at T = 1 in units of sqrt(2 R T0): Ma sqrt(gamma/2)."""
    return Ma * math.sqrt(gamma / 2.0)


def block_flow(nx: int, ny: int, nz: int, block: Tuple[Tuple[int, int], Tuple[int, int], Tuple[int, int]],
               m: int, vmax: float, Kn: float, Ma: float = 5.0, species: int = MONATOMIC,
               omega: float = 0.75, name: str = "block", **kw) -> Case:
    """A solid block of masked cells in a uniform stream along +x.

    The block side is the length scale (h = 1 / block cells along x; 1/16 for an
    empty block), every box face lets in the free-stream Maxwellian, the block
    surface is a diffuse wall at T_w = 1."""
    bx = block[0][1] - block[0][0]
    h = 1.0 / (bx if bx > 0 else 16)
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    solid[block[2][0]:block[2][1], block[1][0]:block[1][1], block[0][0]:block[0][1]] = 1
    gamma = 5.0 / 3.0 if species == MONATOMIC else (5.0 + N2_DR) / (3.0 + N2_DR)
    U = free_stream_speed(Ma, gamma)
    bcs = [Boundary(INFLOW, (U, 0.0, 0.0), 1.0, 1.0) for _ in range(6)]
    bcs.append(Boundary(WALL, (0.0, 0.0, 0.0), 1.0))
    extra = {}
    if species == DIATOMIC:
        extra = dict(dr=N2_DR, Zr=N2_ZR, A=N2_A)
        omega = N2_OMEGA
    return Case(name=name, nx=nx, ny=ny, nz=nz, lx=nx * h, ly=ny * h, lz=nz * h, nv=(m, m, m),
                vmin=(-vmax,) * 3, vmax=(vmax,) * 3, Kn=Kn, omega=omega, species=species,
                bcs=bcs, solid=solid.reshape(-1), init=(1.0, (U, 0.0, 0.0), 1.0, 1.0), **extra, **kw)


# ----------------------------------------------------------------- workloads
def stretched_nodes(n: int, vmax: float, s: float) -> np.ndarray:
    """n nodes on [-vmax, vmax] clustered at the origin: vmax sinh(s t) / sinh(s)
    for t uniform on [-1, 1] (s -> 0 gives the uniform grid)."""
    t = np.linspace(-1.0, 1.0, n)
    return vmax * np.sinh(s * t) / np.sinh(s)


def with_nodes(case: Case, nodes) -> Case:
    """The case on a tensor grid with the given per-axis nodes (vmin/vmax follow)."""
    case.nodes = tuple(None if x is None else np.asarray(x, dtype=np.float64) for x in nodes)
    vmin, vmax, nv = list(case.vmin), list(case.vmax), list(case.nv)
    for a, x in enumerate(case.nodes):
        if x is not None:
            vmin[a], vmax[a], nv[a] = float(x[0]), float(x[-1]), int(x.size)
    case.vmin, case.vmax, case.nv = tuple(vmin), tuple(vmax), tuple(nv)
    return case


def refined_velocity_mesh(center, radius: float, refine, H: float, r: int = 2) -> np.ndarray:
    """A locally refined velocity mesh of Sec. 3.1 as a node list [n][4].

    The ball |xi - center| <= radius is tiled by cubes of side H on a lattice
    aligned with the origin; a cube is kept when its centre lies in the ball.
    A kept cube that overlaps one of the refinement cubes (centre c, half
    side L, given as ``refine = [(c, L), ...]``) is split into r^3 cubes of
    side H / r, each kept when its own centre lies in the ball.  A node is the
    centre of a cube and its weight the cube's volume.  Nodes are ordered by
    (z, y, x) of their centres."""
    center = np.asarray(center, dtype=np.float64)
    lo = np.floor((center - radius) / H).astype(int)
    hi = np.ceil((center + radius) / H).astype(int)
    ax = [np.arange(lo[a], hi[a]) for a in range(3)]
    K = np.stack(np.meshgrid(ax[0], ax[1], ax[2], indexing="ij"), axis=-1).reshape(-1, 3)
    cen = (K + 0.5) * H
    inside = np.sum((cen - center) ** 2, axis=1) <= radius * radius
    cen = cen[inside]
    split = np.zeros(cen.shape[0], dtype=bool)
    for c, L in refine:
        c = np.asarray(c, dtype=np.float64)
        split |= np.all(np.abs(cen - c) < 0.5 * H + L, axis=1)   # the two cubes overlap
    coarse = cen[~split]
    off = (np.arange(r) + 0.5) / r - 0.5
    sub = np.stack(np.meshgrid(off, off, off, indexing="ij"), axis=-1).reshape(-1, 3) * H
    fine = (cen[split][:, None, :] + sub[None, :, :]).reshape(-1, 3)
    fine = fine[np.sum((fine - center) ** 2, axis=1) <= radius * radius]
    xi = np.concatenate([coarse, fine])
    w = np.concatenate([np.full(coarse.shape[0], H ** 3), np.full(fine.shape[0], (H / r) ** 3)])
    order = np.lexsort((xi[:, 0], xi[:, 1], xi[:, 2]))
    return np.ascontiguousarray(np.column_stack([xi[order], w[order]]))


def hypersonic_velocity_mesh(Ma: float, gamma: float, H: float, r: int = 2, T_inf: float = 1.0,
                             T_w: float = 1.0) -> np.ndarray:
    """The velocity mesh of Sec. 3.1 for a stream along +x at Mach Ma (units of
    sqrt(2 R T_inf)): the ball centred at U_s = U_inf / (density ratio of the
    normal shock) with radius 5 sqrt(R T_s), T_s the largest of the stagnation,
    wall and free-stream temperatures, refined (cells of side H / r) on the
    cubes of half side 3 sqrt(R T_inf) about U_inf and 3 sqrt(R T_w) about 0."""
    U = free_stream_speed(Ma, gamma) * math.sqrt(T_inf)
    ratio = (gamma + 1.0) * Ma * Ma / (2.0 + (gamma - 1.0) * Ma * Ma)
    Tm = T_inf * (1.0 + 0.5 * (gamma - 1.0) * Ma * Ma)
    Ts = max(Tm, T_w, T_inf)
    srt = lambda T: math.sqrt(0.5 * T)   # sqrt(R T) in units of sqrt(2 R T0)
    return refined_velocity_mesh((U / ratio, 0.0, 0.0), 5.0 * srt(Ts),
                                 [((U, 0.0, 0.0), 3.0 * srt(T_inf)), ((0.0, 0.0, 0.0), 3.0 * srt(T_w))], H, r)


def with_velocity_list(case: Case, nodes: np.ndarray, name: Optional[str] = None) -> Case:
    """The case on the general velocity set ``nodes`` ([n][4])."""
    case.velocity_list = np.ascontiguousarray(nodes, dtype=np.float64)
    if name:
        case.name = name
    return case


def c1() -> Case:
    """16^3 cavity, 16^3 nodes on [-4,4]^3, Kn = 0.1, lid 0.1, 10 source iterations, FP64."""
    return cavity(16, 16, 0.1, name="c1_cavity16_v16", passes=10)


def c2() -> Case:
    """48^3 cavity, 32^3 nodes, Kn = 0.01, GSIS until the relative change of rho, u and T < 1e-6;
    600 inner macroscopic iterations per correction (the shortest time to converge measured)."""
    return cavity(48, 32, 0.01, name="c2_cavity48_v32_gsis", gsis=True, passes=1, max_iters=200, macro_iters=600)


def c3() -> Case:
    """Ma = 5 past a 16^3 block in 96x64x64 cells, 40^3 nodes on [-12,12]^3, Kn = 0.05, 20 passes."""
    return block_flow(96, 64, 64, ((40, 56), (24, 40), (24, 40)), 40, 12.0, 0.05,
                      name="c3_block96x64x64_v40", passes=20)


def c3r() -> Case:
    """The Ma = 5 block flow of c3 (96x64x64 cells, Kn = 0.05, 20 passes) on the
    refined velocity mesh of Sec. 3.1: the ball of radius 10.8 about the
    post-shock velocity, cells of side 1.0, and 0.5 in the refinement cubes
    about the free-stream and wall velocities (7788 nodes)."""
    c = block_flow(96, 64, 64, ((40, 56), (24, 40), (24, 40)), 40, 12.0, 0.05,
                   name="c3r_block96x64x64_refined7788", passes=20)
    return with_velocity_list(c, hypersonic_velocity_mesh(5.0, 5.0 / 3.0, 1.0, 2))


def c4() -> Case:
    """Diatomic N2 (Rykov, Z = 3.5), Ma = 5 past a 16^3 block in 64x48x48 cells, 32^3 nodes, GSIS;
    1000 inner macroscopic iterations per correction (the shortest time to converge measured)."""
    return block_flow(64, 48, 48, ((24, 40), (16, 32), (16, 32)), 32, 12.0, 0.05, species=DIATOMIC,
                      name="c4_n2_block64x48x48_v32_gsis", gsis=True, passes=1, macro_iters=1000)


def c5(seed: int = 2310_18916, ncases: int = 64) -> List[Case]:
    """64 cavities: n ~ U{8..32} cells/side, m ~ U{12..24} nodes/side, Kn = 10^U(-3,0),
    lid ~ U(0.05, 0.3); draws in case order as (n, m, log10 Kn, lid)."""
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(ncases):
        n = int(rng.integers(8, 33))
        m = int(rng.integers(12, 25))
        kn = float(10.0 ** rng.uniform(-3.0, 0.0))
        lid = float(rng.uniform(0.05, 0.3))
        cases.append(cavity(n, m, kn, lid=lid, name=f"c5_case{i}", gsis=True, max_iters=50))
    return cases


def small(case: Case, n: Optional[int] = None, m: Optional[int] = None) -> Case:
    """A reduced copy of a workload with the same physics (for full-field parity)."""
    c = dataclasses.replace(case)
    if case.solid is not None:
        raise ValueError("use small_block for masked cases")
    if n is not None:
        c.nx = c.ny = c.nz = n
    if m is not None:
        c.nv = (m, m, m)
    return c


def small_block(species: int = MONATOMIC, n: Tuple[int, int, int] = (12, 9, 10), blk=((4, 7), (3, 6), (4, 6)),
                m: int = 10, vmax: float = 12.0, Kn: float = 0.05, name: str = "block_small", **kw) -> Case:
    """Reduced block flow: same physics as c3/c4 on a coarse grid with a ragged block."""
    c = block_flow(n[0], n[1], n[2], blk, m, vmax, Kn, species=species, name=name, **kw)
    return c


# -------------------------------------------------------------- random data
def random_vdf(case: Case, seed: int, dtype=np.float64) -> Tuple[np.ndarray, Optional[np.ndarray]]:
    """Positive random VDFs in the canonical [cell][node] layout (node x fastest):
    a Maxwellian-like envelope in node index times U(0.5, 1.5) noise."""
    rng = np.random.default_rng(seed)
    shape = (case.ncell, case.nvel)
    if case.velocity_list is not None:
        xi = case.velocity_list[:, :3]
        vm = float(np.abs(xi).max())
        env = np.exp(-np.sum(xi ** 2, axis=1) / (1.0 + 0.25 * vm ** 2 / 16.0))
    else:
        axes = [np.linspace(case.vmin[a], case.vmax[a], case.nv[a]) for a in range(3)]
        xz, xy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        env = np.exp(-(xx ** 2 + xy ** 2 + xz ** 2) / (1.0 + 0.25 * max(case.vmax) ** 2 / 16.0)).reshape(-1)
    f0 = (env[None, :] * rng.uniform(0.5, 1.5, size=shape)).astype(dtype)
    f1 = None
    if case.species == DIATOMIC:
        f1 = (env[None, :] * rng.uniform(0.5, 1.5, size=shape)).astype(dtype)
    if case.solid is not None:
        f0[case.solid.astype(bool)] = 0
        if f1 is not None:
            f1[case.solid.astype(bool)] = 0
    return f0, f1


# ------------------------------------------------------- unstructured meshes
# Cell kinds of a lattice mesh: every cube of the lattice is kept whole or cut
# into tetrahedra, pyramids or prisms.
TET, PYRAMID, PRISM, HEX = 0, 1, 2, 3


@dataclasses.dataclass
class SpatialMesh:
    """A finite-volume mesh of convex polyhedral cells (Sec. 3.2: cells i of
    volume V_i, interfaces ij of area S_ij with unit normal n from i to j).

    ``face_cell[f] = (owner, neighbour)``, the neighbour a cell index or
    ``-1 - slot`` for a boundary face of boundary slot 0..6 (the box faces
    -x, +x, -y, +y, -z, +z, then the surface of a solid body);
    ``face_geom[f] = (area, n_x, n_y, n_z)`` with n the unit normal pointing
    out of the owner; ``centroid`` the cell centroids and ``face_center`` the
    face centroids (the macroscopic correction's gradients and distances);
    ``kind`` the cell kind (reports)."""
    volume: np.ndarray
    face_cell: np.ndarray
    face_geom: np.ndarray
    centroid: np.ndarray
    kind: np.ndarray
    face_center: Optional[np.ndarray] = None

    @property
    def ncell(self) -> int:
        return int(self.volume.shape[0])

    @property
    def nface(self) -> int:
        return int(self.face_cell.shape[0])


def _cube_cells():
    """Cells of one lattice cube by kind, each a list of boundary triangles over
    the cube's local points: corner b = bx + 2 by + 4 bz (0..7) and the centre
    (8).  A cube face is always cut along the diagonal from its (0, 0) to its
    (1, 1) corner in the face's own axes (the lower axis first), the cut the
    Kuhn tetrahedra make, so that any two kinds meet on matching triangles."""
    def face_tris(a, s):
        b, c = [x for x in range(3) if x != a]
        def pt(ub, uc):
            bits = [0, 0, 0]
            bits[a], bits[b], bits[c] = s, ub, uc
            return bits[0] + 2 * bits[1] + 4 * bits[2]
        return [(pt(0, 0), pt(1, 0), pt(1, 1)), (pt(0, 0), pt(0, 1), pt(1, 1))]

    def face_edges(a, s):
        b, c = [x for x in range(3) if x != a]
        def pt(ub, uc):
            bits = [0, 0, 0]
            bits[a], bits[b], bits[c] = s, ub, uc
            return bits[0] + 2 * bits[1] + 4 * bits[2]
        ring = [pt(0, 0), pt(1, 0), pt(1, 1), pt(0, 1)]
        return [(ring[k], ring[(k + 1) % 4]) for k in range(4)]

    faces = [(a, s) for a in range(3) for s in (0, 1)]
    hexcell = [[t for a, s in faces for t in face_tris(a, s)]]
    tets = []
    for p in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        v1 = 1 << p[0]
        v2 = v1 | (1 << p[1])
        v = (0, v1, v2, 7)
        tets.append([(v[0], v[1], v[2]), (v[0], v[1], v[3]), (v[0], v[2], v[3]), (v[1], v[2], v[3])])
    pyramids = []
    for a, s in faces:
        pyramids.append(face_tris(a, s) + [(e0, e1, 8) for e0, e1 in face_edges(a, s)])
    diag = [(0, 3, 7), (0, 4, 7)]                      # the cut x = y through the z edges
    prism_a = [(0, 1, 3), (4, 5, 7)] + face_tris(1, 0) + face_tris(0, 1) + diag   # x >= y
    prism_b = [(0, 2, 3), (4, 6, 7)] + face_tris(0, 0) + face_tris(1, 1) + diag   # x <= y
    return {TET: tets, PYRAMID: pyramids, PRISM: [prism_a, prism_b], HEX: hexcell}


def lattice_mesh(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float, split=TET,
                 solid: Optional[np.ndarray] = None) -> SpatialMesh:
    """An unstructured mesh on the nx x ny x nz lattice of the box [0,lx]x[0,ly]x[0,lz]:
    cube (i, j, k) is cut by ``split`` (one kind for all, or an int array of
    shape (nz, ny, nx)) into 6 Kuhn tetrahedra, 6 pyramids about its centre, 2
    triangular prisms, or kept as one hexahedron; cubes flagged in ``solid``
    (shape (nz, ny, nx) or flat, x fastest) are left out and their faces
    become the solid surface (slot 6).  Cells are numbered cube by cube (x
    fastest); coplanar triangles between the same two cells (or the same cell
    and slot) are merged into one face."""
    h = np.array([lx / nx, ly / ny, lz / nz])
    kinds = np.broadcast_to(np.asarray(split, dtype=np.int64), (nz, ny, nx)).reshape(-1)
    keep = np.ones(nx * ny * nz, dtype=bool)
    if solid is not None:
        keep = np.asarray(solid).reshape(-1) == 0
    cube = np.flatnonzero(keep)
    ci, cj, ck = cube % nx, (cube // nx) % ny, cube // (nx * ny)
    nvl = (nx + 1) * (ny + 1) * (nz + 1)
    bits = np.array([[b & 1, (b >> 1) & 1, (b >> 2) & 1] for b in range(8)])
    # global ids of the 9 local points of every kept cube; the centres follow the lattice points
    pid = np.empty((cube.size, 9), dtype=np.int64)
    for b in range(8):
        pid[:, b] = (ci + bits[b, 0]) + (nx + 1) * ((cj + bits[b, 1]) + (ny + 1) * (ck + bits[b, 2]))
    pid[:, 8] = nvl + np.arange(cube.size)
    lat = np.stack(np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij"),
                   axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    pts = np.concatenate([lat * h, (np.stack([ci, cj, ck], axis=1) + 0.5) * h])
    lat_i = np.concatenate([lat, np.full((cube.size, 3), -1)])   # lattice indices (-1: a centre)
    table = _cube_cells()
    ncell_of = np.array([len(table[k]) for k in (TET, PYRAMID, PRISM, HEX)])
    kc = kinds[cube]
    first = np.concatenate([[0], np.cumsum(ncell_of[kc])])   # first cell of every kept cube
    tri_cell, tri_v = [], []
    for k in (TET, PYRAMID, PRISM, HEX):
        sel = np.flatnonzero(kc == k)
        if sel.size == 0:
            continue
        for lc, tris in enumerate(table[k]):
            for t in tris:
                tri_cell.append(first[sel] + lc)
                tri_v.append(pid[sel][:, list(t)])
    tri_cell = np.concatenate(tri_cell)
    tri_v = np.concatenate(tri_v)
    ncell = int(first[-1])
    kind = np.empty(ncell, dtype=np.int8)
    for k in (TET, PYRAMID, PRISM, HEX):
        sel = np.flatnonzero(kc == k)
        for lc in range(ncell_of[k]):
            kind[first[sel] + lc] = k
    # a point inside every cell (the mean of its triangles' vertices: inside a
    # convex cell), triangle geometry, then volume and centroid from the
    # pyramids the triangles span with that point
    tp = pts[tri_v]
    ref = np.zeros((ncell, 3))
    np.add.at(ref, tri_cell, tp.sum(axis=1))
    ref /= np.bincount(tri_cell, minlength=ncell)[:, None] * 3
    cr = np.cross(tp[:, 1] - tp[:, 0], tp[:, 2] - tp[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area[:, None])
    tc = tp.mean(axis=1)
    flip = np.einsum("ij,ij->i", nrm, tc - ref[tri_cell]) < 0
    nrm[flip] *= -1.0                                   # out of the triangle's own cell
    pv = area * np.einsum("ij,ij->i", nrm, tc - ref[tri_cell]) / 3.0
    vol = np.zeros(ncell)
    np.add.at(vol, tri_cell, pv)
    cen = np.zeros((ncell, 3))
    np.add.at(cen, tri_cell, pv[:, None] * (0.75 * tc + 0.25 * ref[tri_cell]))
    cen /= vol[:, None]
    # pair the triangles: equal vertex sets are the two sides of one interface
    key = np.sort(tri_v, axis=1)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0]))
    ks = key[order]
    same = np.all(ks[1:] == ks[:-1], axis=1)
    a_idx = order[:-1][same]
    b_idx = order[1:][same]
    paired = np.zeros(tri_cell.size, dtype=bool)
    paired[a_idx] = paired[b_idx] = True
    lone = np.flatnonzero(~paired)
    li = lat_i[tri_v[lone]]                             # [n, 3 vertices, 3 axes]
    slot = np.full(lone.size, 6)
    for a, n_a in enumerate((nx, ny, nz)):
        slot[np.all(li[:, :, a] == 0, axis=1)] = 2 * a
        slot[np.all(li[:, :, a] == n_a, axis=1)] = 2 * a + 1
    owner = np.concatenate([tri_cell[a_idx], tri_cell[lone]])
    other = np.concatenate([tri_cell[b_idx], -1 - slot])
    geom = np.concatenate([np.column_stack([area[a_idx], nrm[a_idx]]), np.column_stack([area[lone], nrm[lone]])])
    # merge coplanar triangles of the same (owner, other) pair
    nkey = np.round(geom[:, 1:] * 1e9).astype(np.int64)
    mk = np.column_stack([owner, other, nkey])
    uq, inv = np.unique(mk, axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    fa = np.zeros(uq.shape[0])
    np.add.at(fa, inv, geom[:, 0])
    tcs = np.concatenate([tc[a_idx], tc[lone]])
    fcen = np.zeros((uq.shape[0], 3))
    np.add.at(fcen, inv, geom[:, :1] * tcs)
    fcen /= fa[:, None]
    rep = np.zeros(uq.shape[0], dtype=np.int64)
    rep[inv[::-1]] = np.arange(inv.size)[::-1]          # first triangle of every face
    fn = geom[rep, 1:]
    fc = np.column_stack([owner[rep], other[rep]]).astype(np.int32)
    fo = np.lexsort((fc[:, 1], fc[:, 0]))
    return SpatialMesh(volume=vol, face_cell=np.ascontiguousarray(fc[fo]),
                       face_geom=np.ascontiguousarray(np.column_stack([fa, fn])[fo]),
                       centroid=cen, kind=kind, face_center=np.ascontiguousarray(fcen[fo]))


def tensor_velocity_list(nv, vmin, vmax) -> np.ndarray:
    """The uniform tensor grid of a case as a node list [n][4], x fastest,
    trapezoid weights (products of the 1-D weights)."""
    ax, wt = [], []
    for a in range(3):
        x = np.linspace(vmin[a], vmax[a], nv[a])
        d = (vmax[a] - vmin[a]) / (nv[a] - 1)
        w = np.full(nv[a], d)
        w[0] = w[-1] = 0.5 * d
        ax.append(x)
        wt.append(w)
    X = np.stack(np.meshgrid(ax[0], ax[1], ax[2], indexing="ij"), axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    W = (wt[0][None, None, :] * wt[1][None, :, None] * wt[2][:, None, None]).reshape(-1)
    return np.ascontiguousarray(np.column_stack([X, W]))


def on_mesh(case: Case, mesh: SpatialMesh, name: Optional[str] = None) -> Case:
    """The case on the unstructured spatial mesh ``mesh`` (same gas, velocity
    set and boundary slots; a tensor velocity grid becomes its node list)."""
    c = dataclasses.replace(case)
    c.mesh = mesh
    c.nx, c.ny, c.nz = mesh.ncell, 1, 1
    c.solid = None
    c.order = 1
    if c.velocity_list is None:
        c.velocity_list = tensor_velocity_list(c.nv, c.vmin, c.vmax)
    if name:
        c.name = name
    return c


def c3t() -> Case:
    """The Ma = 5 block flow of c3r (Kn = 0.05, the refined velocity mesh of
    Sec. 3.1, 7788 nodes) on an unstructured spatial mesh: the 48x32x32 lattice
    of the same box (cubes of twice the c3 cell side), every cube cut into six
    tetrahedra, the block's 8^3 cubes left out (291,840 tetrahedra; the
    block's surface is slot 6)."""
    base = c3r()
    solid = np.zeros((32, 32, 48), dtype=np.uint8)
    solid[12:20, 12:20, 20:28] = 1
    mesh = lattice_mesh(48, 32, 32, base.lx, base.ly, base.lz, split=TET, solid=solid)
    return on_mesh(base, mesh, name="c3t_block48x32x32_tet_refined7788")
