"""Python face of libgsis: the same calls as include/gsis.h, argument marshalling only.

Device memory and streams come from PyTorch (ROCm): the workspace is a torch
uint8 tensor on the GPU and device work goes to torch's current stream.  Every
step of the kinetic path runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import numpy as np

from . import _lib
from .inputs import Case, DIATOMIC


class GsisError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {_lib.STATUS.get(status, status)}: {message}")


def make_config(case: Case, dtype: str = "fp64") -> _lib.Config:
    c = _lib.Config()
    c.nx, c.ny, c.nz = case.nx, case.ny, case.nz
    if case.mesh is not None:      # the box is replaced by gsis_set_spatial_mesh
        c.nx = c.ny = c.nz = 1
    c.lx, c.ly, c.lz = case.lx, case.ly, case.lz
    c.nvx, c.nvy, c.nvz = case.nv
    for a in range(3):
        c.vmin[a] = case.vmin[a]
        c.vmax[a] = case.vmax[a]
    c.species = case.species
    c.Kn, c.omega = case.Kn, case.omega
    c.dr, c.Zr = case.dr, case.Zr
    for k in range(4):
        c.A[k] = case.A[k]
    c.inv_dt = case.inv_dt
    c.vdf_dtype = {"fp64": 0, "fp32": 1}[dtype]
    c.conservative = case.conservative
    c.macro_cfl = case.macro_cfl
    c.order = case.order
    c.limiter_k = case.limiter_k
    return c


def tile_shapes():
    """Compiled sweep tiles as (tx, ty, precision bits)."""
    buf = (C.c_int * 96)()
    n = C.c_int()
    st = _lib.lib().gsis_tile_shapes(buf, 32, C.byref(n))
    if st:
        raise GsisError(st, "gsis_tile_shapes", "")
    return [(buf[3 * k], buf[3 * k + 1], buf[3 * k + 2]) for k in range(n.value)]


class Context:
    """A gsis_ctx without device memory: creation, mask, boundaries, workspace size.
    Touches no GPU (usable on a CPU-only host)."""

    def __init__(self, case: Case, dtype: str = "fp64"):
        self.case = case
        self.dtype = dtype
        self.L = _lib.lib()
        self._cfg = make_config(case, dtype)
        h = C.c_void_p()
        st = self.L.gsis_create(C.byref(h), C.byref(self._cfg))
        if st:
            raise GsisError(st, "gsis_create", "invalid configuration")
        self.h = h
        if case.solid is not None:
            mask = case.solid_mask()
            self._check(self.L.gsis_set_solid_mask(self.h, mask.ctypes.data_as(C.c_void_p), mask.size),
                        "gsis_set_solid_mask")
        for face, bc in enumerate(case.bcs):
            u = (C.c_double * 3)(*bc.u)
            self._check(self.L.gsis_set_boundary(self.h, face, bc.kind, u, bc.T, bc.rho), "gsis_set_boundary")
        if case.wall_flux:
            self._check(self.L.gsis_set_wall_flux(self.h, case.wall_flux), "gsis_set_wall_flux")
        if case.nodes is not None:
            for a, x in enumerate(case.nodes):
                if x is None:
                    continue
                x = np.ascontiguousarray(x, dtype=np.float64)
                self._check(self.L.gsis_set_velocity_nodes(self.h, a, x.ctypes.data_as(C.c_void_p), x.size),
                            "gsis_set_velocity_nodes")
        if case.velocity_list is not None:
            t = np.ascontiguousarray(case.velocity_list, dtype=np.float64)
            self._vlist = t
            self._check(self.L.gsis_set_velocity_list(self.h, t.ctypes.data_as(C.c_void_p), t.shape[0]),
                        "gsis_set_velocity_list")
        if case.mesh is not None:
            m = case.mesh
            vol = np.ascontiguousarray(m.volume, dtype=np.float64)
            fc = np.ascontiguousarray(m.face_cell, dtype=np.int32)
            fg = np.ascontiguousarray(m.face_geom, dtype=np.float64)
            cc = fcc = None
            if m.face_center is not None:
                cc = np.ascontiguousarray(m.centroid, dtype=np.float64)
                fcc = np.ascontiguousarray(m.face_center, dtype=np.float64)
            ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
            self._check(self.L.gsis_set_spatial_mesh(self.h, vol.size, ptr(vol), fc.shape[0], ptr(fc), ptr(fg),
                                                     ptr(cc), ptr(fcc)),
                        "gsis_set_spatial_mesh")

    def _check(self, st: int, where: str):
        if st:
            msg = self.L.gsis_last_error(self.h)
            raise GsisError(st, where, msg.decode() if msg else "")

    def workspace_size(self) -> int:
        n = C.c_size_t()
        self._check(self.L.gsis_workspace_size(self.h, C.byref(n)), "gsis_workspace_size")
        return n.value

    def close(self):
        if getattr(self, "h", None):
            self.L.gsis_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver(Context):
    """A bound context on the current GPU (torch workspace, torch stream)."""

    def __init__(self, case: Case, dtype: str = "fp64", tile: Optional[Tuple[int, int, int, int]] = None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libgsis needs a GPU; none is visible")
        super().__init__(case, dtype)
        self.torch = torch
        if tile is not None:
            self.set_tile(*tile)
        nbytes = self.workspace_size()
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self._check(self.L.gsis_bind_workspace(self.h, C.c_void_p(self.ws.data_ptr()), nbytes), "gsis_bind_workspace")
        self._check(self.L.gsis_set_stream(self.h, C.c_void_p(torch.cuda.current_stream().cuda_stream)),
                    "gsis_set_stream")
        self.nmom = _lib.NMOM[case.species]

    def set_tile(self, tx: int, ty: int, tz: int, block: int):
        self._check(self.L.gsis_set_tile(self.h, tx, ty, tz, block), "gsis_set_tile")

    def get_tile(self):
        t = (C.c_int * 4)()
        self._check(self.L.gsis_get_tile(self.h, t), "gsis_get_tile")
        return tuple(t)

    def autotune(self, reps: int = 2):
        """Time the next pass's sweep under every compiled configuration and keep the
        fastest; returns [((tx, ty, tz, block), ms), ...]."""
        cfg = (C.c_int * 512)()
        ms = (C.c_double * 128)()
        n = C.c_int()
        self._check(self.L.gsis_autotune(self.h, reps, cfg, ms, 128, C.byref(n)), "gsis_autotune")
        return [((cfg[4 * k], cfg[4 * k + 1], cfg[4 * k + 2], cfg[4 * k + 3]), ms[k]) for k in range(n.value)]

    def init_maxwellian(self, rho=None, u=None, T=None, Tr=None):
        r0, u0, T0, Tr0 = self.case.init
        rho = r0 if rho is None else rho
        u = (C.c_double * 3)(*(u0 if u is None else u))
        T = T0 if T is None else T
        Tr = Tr0 if Tr is None else Tr
        self._check(self.L.gsis_init_maxwellian(self.h, rho, u, T, Tr), "gsis_init_maxwellian")

    def kinetic_step(self, npasses: int = 1):
        self._check(self.L.gsis_kinetic_step(self.h, npasses), "gsis_kinetic_step")

    def gsis_correct(self, inner_iters: int):
        self._check(self.L.gsis_gsis_correct(self.h, inner_iters), "gsis_gsis_correct")

    def precondition(self, macro_steps: int = 1000, kinetic_steps: int = 10):
        """Alg. 1, line 1: Euler macroscopic steps, the VDF corrected to their
        result, then kinetic passes."""
        self._check(self.L.gsis_precondition(self.h, macro_steps, kinetic_steps), "gsis_precondition")

    def moments(self) -> np.ndarray:
        # through a contiguous device buffer: the library's strided copy straight
        # into pageable host memory goes row by row
        return self.moments_device().cpu().numpy()

    def moments_host_copy(self) -> np.ndarray:
        """gsis_moments straight into host memory (the library's own copy)."""
        out = np.empty((self.case.ncell, self.nmom), dtype=np.float64)
        self._check(self.L.gsis_moments(self.h, out.ctypes.data_as(C.c_void_p), 0), "gsis_moments")
        return out

    def moments_device(self):
        out = self.torch.empty((self.case.ncell, self.nmom), dtype=self.torch.float64, device="cuda")
        self._check(self.L.gsis_moments(self.h, C.c_void_p(out.data_ptr()), 1), "gsis_moments")
        return out

    def residual(self) -> np.ndarray:
        eps = (C.c_double * 3)()
        self._check(self.L.gsis_residual(self.h, eps), "gsis_residual")
        return np.array(eps[:])

    def residual_noalloc(self) -> np.ndarray:
        """gsis_residual_noalloc: the same criterion with the library's static
        partial-sum array instead of the workspace's (allocates nothing)."""
        eps = (C.c_double * 3)()
        self._check(self.L.gsis_residual_noalloc(self.h, eps), "gsis_residual_noalloc")
        return np.array(eps[:])

    def get_vdf(self):
        t = self.torch
        shape = (self.case.ncell, self.case.nvel)
        f0 = t.empty(shape, dtype=t.float64, device="cuda")
        f1 = t.empty(shape, dtype=t.float64, device="cuda") if self.case.species == DIATOMIC else None
        self._check(self.L.gsis_get_vdf(self.h, C.c_void_p(f0.data_ptr()),
                                        C.c_void_p(f1.data_ptr()) if f1 is not None else None), "gsis_get_vdf")
        return f0, f1

    def set_vdf(self, f0, f1=None):
        t = self.torch
        f0 = t.as_tensor(f0, dtype=t.float64).to("cuda").contiguous()
        f1 = None if f1 is None else t.as_tensor(f1, dtype=t.float64).to("cuda").contiguous()
        self._check(self.L.gsis_set_vdf(self.h, C.c_void_p(f0.data_ptr()),
                                        C.c_void_p(f1.data_ptr()) if f1 is not None else None), "gsis_set_vdf")
        t.cuda.current_stream().synchronize()

    def state_size(self) -> int:
        n = C.c_size_t()
        self._check(self.L.gsis_state_size(self.h, C.byref(n)), "gsis_state_size")
        return n.value

    def get_state(self):
        blob = self.torch.empty(self.state_size(), dtype=self.torch.uint8, device="cuda")
        self._check(self.L.gsis_get_state(self.h, C.c_void_p(blob.data_ptr())), "gsis_get_state")
        return blob

    def set_state(self, blob):
        self._check(self.L.gsis_set_state(self.h, C.c_void_p(blob.data_ptr())), "gsis_set_state")

    def get_vdf_nodes(self, nodes):
        nodes = np.ascontiguousarray(nodes, dtype=np.int32)
        out = self.torch.empty((nodes.size, self.case.ncell), dtype=self.torch.float64, device="cuda")
        self._check(self.L.gsis_get_vdf_nodes(self.h, nodes.ctypes.data_as(C.POINTER(C.c_int)), nodes.size,
                                              C.c_void_p(out.data_ptr())), "gsis_get_vdf_nodes")
        return out

    def profile(self, enable: bool = True):
        self._check(self.L.gsis_profile_enable(self.h, int(enable)), "gsis_profile_enable")

    def profile_read(self, reset: bool = True):
        """{phase: (milliseconds, calls)} measured with HIP events on the bound stream."""
        ms = (C.c_double * len(_lib.PHASES))()
        calls = (C.c_longlong * len(_lib.PHASES))()
        self._check(self.L.gsis_profile_read(self.h, ms, calls, int(reset)), "gsis_profile_read")
        return {name: (ms[k], calls[k]) for k, name in enumerate(_lib.PHASES)}

    def pass_count(self) -> int:
        n = C.c_longlong()
        self._check(self.L.gsis_pass_count(self.h, C.byref(n)), "gsis_pass_count")
        return n.value

    def synchronize(self):
        self.torch.cuda.current_stream().synchronize()


class BatchMember(Solver):
    """One case of a Batch: a context bound inside the batch's workspace.  The
    per-case calls of Solver work on it, on the batch's stream."""

    def __init__(self, ctx: Context, batch: "Batch"):
        import torch
        self.torch = torch
        self.case, self.dtype, self.L, self._cfg = ctx.case, ctx.dtype, ctx.L, ctx._cfg
        self.h = ctx.h
        self._ctx = ctx          # owns the handle
        self._batch = batch      # keeps the workspace alive
        self.nmom = _lib.NMOM[ctx.case.species]

    def get_vdf(self):
        with self.torch.cuda.stream(self._batch.stream):
            out = super().get_vdf()
        self._batch.synchronize()
        return out

    def moments_device(self):
        with self.torch.cuda.stream(self._batch.stream):
            out = super().moments_device()
        self._batch.synchronize()
        return out

    def synchronize(self):
        self._batch.synchronize()

    def close(self):
        self.h = None            # the context destroys the handle


class Batch:
    """Independent cases iterated together (gsis_batch_*): one launch per kernel
    covers every case, and a GSIS iteration replays as one captured HIP graph.
    Device memory and the (non-null) stream come from PyTorch."""

    def __init__(self, cases, dtype: str = "fp32", tile: Optional[Tuple[int, int, int, int]] = None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libgsis needs a GPU; none is visible")
        self.torch = torch
        self.L = _lib.lib()
        self.cases = list(cases)
        self.ctxs = [Context(c, dtype) for c in self.cases]
        arr = (C.c_void_p * len(self.ctxs))(*[c.h.value for c in self.ctxs])
        h = C.c_void_p()
        st = self.L.gsis_batch_create(C.byref(h), arr, len(self.ctxs))
        if st:
            raise GsisError(st, "gsis_batch_create", "cases must share precision and gas and use inv_dt = 0 and order 1")
        self.h = h
        self.stream = torch.cuda.Stream()
        self._check(self.L.gsis_batch_set_stream(self.h, C.c_void_p(self.stream.cuda_stream)), "gsis_batch_set_stream")
        if tile is not None:
            self.set_tile(*tile)
        n = C.c_size_t()
        self._check(self.L.gsis_batch_workspace_size(self.h, C.byref(n)), "gsis_batch_workspace_size")
        self.ws = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        torch.cuda.current_stream().synchronize()
        self._check(self.L.gsis_batch_bind_workspace(self.h, C.c_void_p(self.ws.data_ptr()), n.value),
                    "gsis_batch_bind_workspace")
        self.members = [BatchMember(c, self) for c in self.ctxs]

    def _check(self, st: int, where: str):
        if st:
            msg = self.L.gsis_batch_last_error(self.h)
            raise GsisError(st, where, msg.decode() if msg else "")

    def __len__(self):
        return len(self.members)

    def __getitem__(self, i) -> BatchMember:
        return self.members[i]

    def set_tile(self, tx: int, ty: int, tz: int, block: int):
        self._check(self.L.gsis_batch_set_tile(self.h, tx, ty, tz, block), "gsis_batch_set_tile")

    def get_tile(self):
        t = (C.c_int * 4)()
        self._check(self.L.gsis_batch_get_tile(self.h, t), "gsis_batch_get_tile")
        return tuple(t)

    def autotune(self, reps: int = 2):
        cfg = (C.c_int * 512)()
        ms = (C.c_double * 128)()
        n = C.c_int()
        self._check(self.L.gsis_batch_autotune(self.h, reps, cfg, ms, 128, C.byref(n)), "gsis_batch_autotune")
        return [((cfg[4 * k], cfg[4 * k + 1], cfg[4 * k + 2], cfg[4 * k + 3]), ms[k]) for k in range(n.value)]

    def init_maxwellian(self, rho=None, u=None, T=None, Tr=None):
        """With no arguments every case starts from the Maxwellian of its own
        initial state (Case.init); with arguments every case from that one
        state (missing ones: rho = 1, u = 0, T = Tr = 1)."""
        own = rho is None and u is None and T is None and Tr is None
        rho = 1.0 if rho is None else rho
        u = (0.0, 0.0, 0.0) if u is None else u
        T = 1.0 if T is None else T
        Tr = 1.0 if Tr is None else Tr
        self._check(self.L.gsis_batch_init_maxwellian(self.h, rho, (C.c_double * 3)(*u), T, Tr),
                    "gsis_batch_init_maxwellian")
        if own:
            for m in self.members:
                r0, u0, T0, Tr0 = m.case.init
                if (r0, tuple(u0), T0, Tr0) != (rho, tuple(u), T, Tr):
                    m.init_maxwellian()     # the case's context, on the batch's stream
            self.synchronize()

    def run(self, iters: int, inner_iters: int, graph: bool = True):
        self._check(self.L.gsis_batch_run(self.h, iters, inner_iters, int(graph)), "gsis_batch_run")

    def residuals(self, max_iters: int = 1024) -> np.ndarray:
        """[iteration, case, (rho, |u|, Tt)] of the recorded iterations, oldest first."""
        out = np.empty((max_iters, len(self), 3), dtype=np.float64)
        n = C.c_int()
        self._check(self.L.gsis_batch_residuals(self.h, out.ctypes.data_as(C.POINTER(C.c_double)), max_iters,
                                                C.byref(n)), "gsis_batch_residuals")
        return out[:n.value].copy()

    def last_run_ms(self) -> float:
        ms = C.c_double()
        self._check(self.L.gsis_batch_last_run_ms(self.h, C.byref(ms)), "gsis_batch_last_run_ms")
        return ms.value

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "h", None):
            self.stream.synchronize()
            self.L.gsis_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
