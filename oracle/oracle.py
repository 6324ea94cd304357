"""ctypes loader for the FP64 CPU oracle (gsis_oracle.c).

TEST INFRASTRUCTURE: only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import this module.  The product path never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gsis_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, OpenMP over independent nodes/cells)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared", SRC, "-o", LIB, "-lm"]
        subprocess.run(cmd, check=True)
    return LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
        ("nv", C.c_int * 3), ("vmin", C.c_double * 3), ("vmax", C.c_double * 3),
        ("species", C.c_int), ("Kn", C.c_double), ("omega", C.c_double),
        ("dr", C.c_double), ("Zr", C.c_double), ("A", C.c_double * 4),
        ("inv_dt", C.c_double), ("conservative", C.c_int), ("macro_cfl", C.c_double),
        ("bc_kind", C.c_int * 7), ("bc_u", (C.c_double * 3) * 7), ("bc_T", C.c_double * 7),
        ("bc_rho", C.c_double * 7),
        ("nodes", C.POINTER(C.c_double) * 3),
        ("order", C.c_int), ("limiter_k", C.c_double),
        ("nlist", C.c_int), ("node_list", C.POINTER(C.c_double)),
        ("ucells", C.c_int), ("ufaces", C.c_int), ("uvol", C.POINTER(C.c_double)),
        ("uface_cell", C.POINTER(C.c_int)), ("uface_geom", C.POINTER(C.c_double)),
        ("ucenter", C.POINTER(C.c_double)), ("ufcenter", C.POINTER(C.c_double)),
        ("wall_flux", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        D = C.POINTER(C.c_double)
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Cfg), C.c_void_p]
        L.orc_free.argtypes = [P]
        L.orc_ncell.argtypes = [P]
        L.orc_nv.argtypes = [P]
        L.orc_status.argtypes = [P]
        L.orc_step.argtypes = [P, C.c_int]
        L.orc_init_maxwellian.argtypes = [P, C.c_double, D, C.c_double, C.c_double]
        L.orc_set_vdf.argtypes = [P, D, D]
        L.orc_get_vdf.argtypes = [P, D, D]
        L.orc_replace_vdf.argtypes = [P, D, D]
        L.orc_moments.argtypes = [P, D]
        L.orc_residual.argtypes = [P, D]
        L.orc_gsis_correct.argtypes = [P, C.c_int]
        L.orc_gsis_precondition.argtypes = [P, C.c_int, C.c_int]
        L.orc_ref_dist.argtypes = [P, C.c_int, D, D]
        L.orc_invtau.argtypes = [P, C.c_int]
        L.orc_invtau.restype = C.c_double
        L.orc_boundary_values.argtypes = [P, C.c_int, C.c_int, D, D]
        L.orc_face_values.argtypes = [P, C.c_int, C.c_int, C.c_int, D]
        L.orc_flux_divergence.argtypes = [P, C.c_int, C.c_int, C.c_int, D]
        L.orc_umesh_grad.argtypes = [P, D, D]
        L.orc_total_mass.argtypes = [P]
        L.orc_total_mass.restype = C.c_double
        L.orc_ref_components.argtypes = [C.POINTER(_Cfg), C.c_double, D, C.c_double, C.c_double, D, D,
                                         C.c_int, D, D]
        L.orc_conductivities.argtypes = [C.POINTER(_Cfg), D]
        L.orc_last_macro_W.argtypes = [P, D]
        L.orc_stream_create.restype = P
        L.orc_stream_create.argtypes = [C.POINTER(_Cfg), C.c_void_p]
        L.orc_stream_free.argtypes = [P]
        L.orc_stream_init_maxwellian.argtypes = [P, C.c_double, D, C.c_double, C.c_double]
        L.orc_stream_step.argtypes = [P, C.c_int]
        L.orc_stream_gsis_correct.argtypes = [P, C.c_int]
        L.orc_stream_moments.argtypes = [P, D]
        L.orc_stream_residual.argtypes = [P, D]
        L.orc_stream_status.argtypes = [P]
        L.orc_nsf_face.argtypes = [P, D, C.c_int, C.c_int, D]
        L.orc_g13_vdf.argtypes = [C.POINTER(_Cfg), C.c_double, D, C.c_double, C.c_double, D, C.c_int, D, D, D]
        L.orc_model_face_flux.argtypes = [P, D, D, C.c_int, C.c_int, D]
        L.orc_g13_wall_stress.argtypes = [P, D, C.c_int, D]
        L.orc_first_pass_nodes.argtypes = [C.POINTER(_Cfg), C.c_void_p, C.c_double, D, C.c_double, C.c_double,
                                           C.POINTER(C.c_int), C.c_int, D, D]
        _lib = L
    return _lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def g13_vdf(case, rho, u, Tt, Tr, sq, xi):
    """Grad-13 distributions (f0, f1) of Eq. (G13_VDF) of the state (rho, u,
    Tt, Tr) with sq = (sigma xx yy zz xy xz yz, q, qr) at velocities xi[n][3]."""
    cfg = make_cfg(case)
    xi = np.ascontiguousarray(xi, dtype=np.float64).reshape(-1, 3)
    u = np.ascontiguousarray(u, dtype=np.float64)
    sq = np.ascontiguousarray(sq, dtype=np.float64)
    f0 = np.empty(xi.shape[0])
    f1 = np.empty(xi.shape[0])
    lib().orc_g13_vdf(C.byref(cfg), rho, _dp(u), Tt, Tr, _dp(sq), xi.shape[0], _dp(xi), _dp(f0), _dp(f1))
    return f0, f1


def make_cfg(case) -> _Cfg:
    c = _Cfg()
    c.nx, c.ny, c.nz = case.nx, case.ny, case.nz
    c.lx, c.ly, c.lz = case.lx, case.ly, case.lz
    for a in range(3):
        c.nv[a] = case.nv[a]
        c.vmin[a] = case.vmin[a]
        c.vmax[a] = case.vmax[a]
    c.species = case.species
    c.Kn, c.omega = case.Kn, case.omega
    c.dr, c.Zr = case.dr, case.Zr
    for k in range(4):
        c.A[k] = case.A[k]
    c.inv_dt = case.inv_dt
    c.conservative = case.conservative
    c.macro_cfl = case.macro_cfl
    c.order = case.order
    c.limiter_k = case.limiter_k
    c.wall_flux = getattr(case, "wall_flux", 0)
    for b, bc in enumerate(case.bcs):
        c.bc_kind[b] = bc.kind
        for a in range(3):
            c.bc_u[b][a] = bc.u[a]
        c.bc_T[b] = bc.T
        c.bc_rho[b] = bc.rho
    # explicit node positions: the arrays live on the config object (the C side
    # copies them when it creates its state)
    c._keep = []
    mesh = getattr(case, "mesh", None)
    if mesh is not None:
        vol = np.ascontiguousarray(mesh.volume, dtype=np.float64)
        fc = np.ascontiguousarray(mesh.face_cell, dtype=np.int32)
        fg = np.ascontiguousarray(mesh.face_geom, dtype=np.float64)
        c._keep += [vol, fc, fg]
        c.ucells, c.ufaces = mesh.ncell, mesh.nface
        c.uvol = vol.ctypes.data_as(C.POINTER(C.c_double))
        c.uface_cell = fc.ctypes.data_as(C.POINTER(C.c_int))
        c.uface_geom = fg.ctypes.data_as(C.POINTER(C.c_double))
        if mesh.face_center is not None:
            cc = np.ascontiguousarray(mesh.centroid, dtype=np.float64)
            fcc = np.ascontiguousarray(mesh.face_center, dtype=np.float64)
            c._keep += [cc, fcc]
            c.ucenter = cc.ctypes.data_as(C.POINTER(C.c_double))
            c.ufcenter = fcc.ctypes.data_as(C.POINTER(C.c_double))
    if getattr(case, "velocity_list", None) is not None:
        t = np.ascontiguousarray(case.velocity_list, dtype=np.float64)
        c._keep.append(t)
        c.nlist = t.shape[0]
        c.node_list = t.ctypes.data_as(C.POINTER(C.c_double))
        return c
    for a in range(3):
        x = axis_nodes(case, a, explicit_only=True)
        if x is not None:
            x = np.ascontiguousarray(x, dtype=np.float64)
            c._keep.append(x)
            c.nodes[a] = x.ctypes.data_as(C.POINTER(C.c_double))
    return c


class Oracle:
    """One problem state held by the C oracle (canonical [cell][node] FP64 VDFs)."""

    def __init__(self, case):
        self.case = case
        self._cfg = make_cfg(case)
        self._mask = case.solid_mask()
        self.h = lib().orc_create(C.byref(self._cfg), self._mask.ctypes.data_as(C.c_void_p))
        if not self.h:
            raise ValueError("oracle rejected the configuration")
        self.ncell = case.ncell
        self.nv = case.nvel
        self.nmom = 18 if case.species == 1 else 14

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def init_maxwellian(self, rho=None, u=None, T=None, Tr=None):
        r0, u0, T0, Tr0 = self.case.init
        rho = r0 if rho is None else rho
        u = np.array(u0 if u is None else u, dtype=np.float64)
        T = T0 if T is None else T
        Tr = Tr0 if Tr is None else Tr
        lib().orc_init_maxwellian(self.h, rho, _dp(u), T, Tr)

    def step(self, n: int = 1) -> int:
        return lib().orc_step(self.h, n)

    def gsis_correct(self, iters: int) -> int:
        return lib().orc_gsis_correct(self.h, iters)

    def precondition(self, macro_steps: int = 1000, kinetic_steps: int = 10) -> int:
        """Alg. 1, line 1: Euler macroscopic steps, the VDF corrected to their
        result, then kinetic passes."""
        return lib().orc_gsis_precondition(self.h, macro_steps, kinetic_steps)

    def status(self) -> int:
        return lib().orc_status(self.h)

    def moments(self) -> np.ndarray:
        out = np.empty((self.ncell, self.nmom), dtype=np.float64)
        lib().orc_moments(self.h, _dp(out))
        return out

    def residual(self) -> np.ndarray:
        e = np.empty(3, dtype=np.float64)
        lib().orc_residual(self.h, _dp(e))
        return e

    def get_vdf(self):
        f0 = np.empty((self.ncell, self.nv), dtype=np.float64)
        f1 = np.empty_like(f0) if self.case.species == 1 else None
        lib().orc_get_vdf(self.h, _dp(f0), _dp(f1))
        return f0, f1

    def set_vdf(self, f0: np.ndarray, f1: Optional[np.ndarray] = None):
        f0 = np.ascontiguousarray(f0, dtype=np.float64)
        f1 = None if f1 is None else np.ascontiguousarray(f1, dtype=np.float64)
        lib().orc_set_vdf(self.h, _dp(f0), _dp(f1))

    def replace_vdf(self, f0: np.ndarray, f1: Optional[np.ndarray] = None):
        """Replace the VDF keeping the residual snapshot of the state before."""
        f0 = np.ascontiguousarray(f0, dtype=np.float64)
        f1 = None if f1 is None else np.ascontiguousarray(f1, dtype=np.float64)
        lib().orc_replace_vdf(self.h, _dp(f0), _dp(f1))

    def ref_dist(self, cell: int):
        g0 = np.empty(self.nv)
        g1 = np.empty(self.nv)
        lib().orc_ref_dist(self.h, cell, _dp(g0), _dp(g1))
        return g0, (g1 if self.case.species == 1 else None)

    def invtau(self, cell: int) -> float:
        return lib().orc_invtau(self.h, cell)

    def boundary_values(self, cell: int, d: int):
        b0 = np.empty(self.nv)
        b1 = np.empty(self.nv)
        bc = lib().orc_boundary_values(self.h, cell, d, _dp(b0), _dp(b1))
        return bc, b0, b1

    def last_macro_W(self) -> np.ndarray:
        """[cell][6] W^{n+1} = (rho, rho u, E, Er) of the last macroscopic solve."""
        out = np.empty((self.ncell, 6))
        if lib().orc_last_macro_W(self.h, _dp(out)) != 0:
            raise RuntimeError("no macroscopic solve yet")
        return out

    def nsf_face(self, W: np.ndarray, cell: int, a: int) -> np.ndarray:
        """NSF closure (sigma_xa, sigma_ya, sigma_za, q_a, qr_a) of the macroscopic
        solve at the face between `cell` and its +a neighbour for the field W[cell][6]."""
        W = np.ascontiguousarray(W, dtype=np.float64)
        out = np.empty(5)
        if lib().orc_nsf_face(self.h, _dp(W), cell, a, _dp(out)) != 0:
            raise ValueError("not an interior fluid face")
        return out

    def umesh_grad(self, W: np.ndarray) -> np.ndarray:
        """[cell][3][3] least-squares velocity gradients (d u_b / d x_c) of the
        unstructured macroscopic solve for the field W[cell][6]."""
        W = np.ascontiguousarray(W, dtype=np.float64)
        G = np.empty((self.ncell, 9))
        if lib().orc_umesh_grad(self.h, _dp(W), _dp(G)) != 0:
            raise ValueError("no unstructured mesh with centroids")
        return G.reshape(-1, 3, 3)

    def total_mass(self) -> float:
        return lib().orc_total_mass(self.h)

    def g13_wall_stress(self, Wm, cell: int) -> np.ndarray:
        """(sigma xx yy zz xy xz yz, q, qr) the Grad-13 wall flux takes at
        `cell` for the iterate Wm[ncell][6], the current VDF being f^{n+1/2}."""
        Wm = np.ascontiguousarray(Wm, dtype=np.float64)
        out = np.empty(12)
        if lib().orc_g13_wall_stress(self.h, _dp(Wm), cell, _dp(out)) != 0:
            raise ValueError("not a fluid cell")
        return out

    def model_face_flux(self, W6, cell: int, d: int, sq=None) -> np.ndarray:
        """Flux (mass, momentum, energy, Er) out of boundary face d of `cell`
        whose conservative state is W6, with that face's boundary rule: of the
        cell's Maxwellian (sq None) or of its Grad-13 distributions with
        sq = (sigma xx yy zz xy xz yz, q, qr)."""
        W6 = np.ascontiguousarray(W6, dtype=np.float64)
        sqa = None if sq is None else np.ascontiguousarray(sq, dtype=np.float64)
        out = np.empty(6)
        if lib().orc_model_face_flux(self.h, _dp(W6), _dp(sqa), cell, d, _dp(out)) != 0:
            raise ValueError("not a boundary face of a fluid cell")
        return out

    def face_values(self, v: int, which: int = 0, order: int = 2) -> np.ndarray:
        """[cell][6] value of canonical node v at each face of each cell
        (order 2: the limited reconstruction on faces between fluid cells)."""
        out = np.empty((self.ncell, 6))
        lib().orc_face_values(self.h, v, which, order, _dp(out))
        return out

    def flux_divergence(self, v: int, which: int = 0, order: int = 2) -> np.ndarray:
        """[cell] (1/V) sum_j xi_n f_ij S_ij of canonical node v."""
        out = np.empty(self.ncell)
        lib().orc_flux_divergence(self.h, v, which, order, _dp(out))
        return out


class StreamOracle:
    """The oracle's iteration without the VDF in memory (source iteration,
    first order): per-cell moment sums and per-face outgoing fluxes only, so
    it serves the full-size workloads.  Same calls as Oracle."""

    def __init__(self, case):
        self.case = case
        self._cfg = make_cfg(case)
        self._mask = case.solid_mask()
        self.h = lib().orc_stream_create(C.byref(self._cfg), self._mask.ctypes.data_as(C.c_void_p))
        if not self.h:
            raise ValueError("streaming oracle needs inv_dt = 0 and order 1")
        self.ncell = case.ncell
        self.nmom = 18 if case.species == 1 else 14

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_stream_free(self.h)
            self.h = None

    def init_maxwellian(self):
        rho, u, T, Tr = self.case.init
        u = np.ascontiguousarray(u, dtype=np.float64)
        lib().orc_stream_init_maxwellian(self.h, rho, _dp(u), T, Tr)

    def step(self, n: int = 1) -> int:
        return lib().orc_stream_step(self.h, n)

    def gsis_correct(self, iters: int) -> int:
        return lib().orc_stream_gsis_correct(self.h, iters)

    def status(self) -> int:
        return lib().orc_stream_status(self.h)

    def moments(self) -> np.ndarray:
        out = np.empty((self.ncell, self.nmom), dtype=np.float64)
        lib().orc_stream_moments(self.h, _dp(out))
        return out

    def residual(self) -> np.ndarray:
        e = np.empty(3, dtype=np.float64)
        lib().orc_stream_residual(self.h, _dp(e))
        return e


def ref_components(case, rho, u, Tt, Tr, qt, qr, xi: np.ndarray) -> np.ndarray:
    """Uncorrected (g0t, g0r, g1t, g1r) at points xi[n,3] from given moments."""
    cfg = make_cfg(case)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    n = xi.shape[0]
    out = np.empty((n, 4))
    u = np.asarray(u, dtype=np.float64)
    qt = np.asarray(qt, dtype=np.float64)
    qr = np.asarray(qr, dtype=np.float64)
    lib().orc_ref_components(C.byref(cfg), rho, _dp(u), Tt, Tr, _dp(qt), _dp(qr), n, _dp(xi), _dp(out))
    return out


def conductivities(case) -> np.ndarray:
    """(k_t, k_r) of the oracle's macroscopic heat fluxes."""
    cfg = make_cfg(case)
    out = np.empty(2)
    lib().orc_conductivities(C.byref(cfg), _dp(out))
    return out


def first_pass_nodes(case, nodes):
    """f^{n+1/2} after one pass from the case's uniform initial Maxwellian, at
    canonical nodes only: ([k][cell] f0, [k][cell] f1 or None, status).  Needs no
    VDF in memory, so it serves the full-size workloads."""
    cfg = make_cfg(case)
    nodes = np.ascontiguousarray(nodes, dtype=np.int32)
    nn, n = nodes.size, case.ncell
    out0 = np.zeros((nn, n))
    out1 = np.zeros((nn, n)) if case.species == 1 else None
    mask = np.ascontiguousarray(case.solid_mask(), dtype=np.uint8)
    rho, u, T, Tr = case.init
    u = np.ascontiguousarray(u, dtype=np.float64)
    st = lib().orc_first_pass_nodes(C.byref(cfg), mask.ctypes.data_as(C.c_void_p), rho, _dp(u), T, Tr,
                                    nodes.ctypes.data_as(C.POINTER(C.c_int)), nn, _dp(out0), _dp(out1))
    return out0, out1, st


def axis_nodes(case, a, explicit_only=False):
    """The nodes of axis a: the case's explicit array, else uniform on [vmin, vmax]
    (None for that with explicit_only)."""
    nodes = getattr(case, "nodes", None)
    if nodes is not None and nodes[a] is not None:
        return np.asarray(nodes[a], dtype=np.float64)
    if explicit_only:
        return None
    return np.linspace(case.vmin[a], case.vmax[a], case.nv[a])


def node_grid(case):
    """Nodes (n,3) and weights (n,) in canonical order: a node list as given, else
    the tensor grid (x fastest) with trapezoid weights."""
    lst = getattr(case, "velocity_list", None)
    if lst is not None:
        lst = np.asarray(lst, dtype=np.float64)
        return lst[:, :3].copy(), lst[:, 3].copy()
    axes, wts = [], []
    for a in range(3):
        x = axis_nodes(case, a, explicit_only=True)
        if x is None:
            x = np.linspace(case.vmin[a], case.vmax[a], case.nv[a])
            d = (case.vmax[a] - case.vmin[a]) / (case.nv[a] - 1)
            w = np.full(case.nv[a], d)
            w[0] *= 0.5
            w[-1] *= 0.5
        else:
            # trapezoid rule on the given nodes: half of each neighbouring gap
            w = 0.5 * (np.append(x[1:], x[-1]) - np.insert(x[:-1], 0, x[0]))
        axes.append(x)
        wts.append(w)
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    WZ, WY, WX = np.meshgrid(wts[2], wts[1], wts[0], indexing="ij")
    xi = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)
    return xi, (WX * WY * WZ).reshape(-1)
