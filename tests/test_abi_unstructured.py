"""Host-side checks of gsis_set_spatial_mesh (no GPU: argument validation
and the velocity classes and sweep levels happen before any device work)."""
import ctypes as C

import numpy as np
import pytest

from paper_2310_18916_amd import inputs as I
from paper_2310_18916_amd import _lib
from paper_2310_18916_amd.gsis import Context, GsisError, make_config

EINVAL, ESTATE = -1, -2


def raw_ctx(case, with_list=True):
    L = _lib.lib()
    cfg = make_config(case)
    cfg.nx = cfg.ny = cfg.nz = 1
    h = C.c_void_p()
    assert L.gsis_create(C.byref(h), C.byref(cfg)) == 0
    if with_list:
        t = np.ascontiguousarray(I.tensor_velocity_list(case.nv, case.vmin, case.vmax))
        assert L.gsis_set_velocity_list(h, t.ctypes.data_as(C.c_void_p), t.shape[0]) == 0
    return L, h


def set_mesh(L, h, vol, fc, fg, cc=None, fcc=None):
    vol = np.ascontiguousarray(vol, dtype=np.float64)
    fc = np.ascontiguousarray(fc, dtype=np.int32)
    fg = np.ascontiguousarray(fg, dtype=np.float64)
    ptr = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.c_void_p)
    keep = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (cc, fcc)]
    return L.gsis_set_spatial_mesh(h, vol.size, vol.ctypes.data_as(C.c_void_p), fc.shape[0],
                                   fc.ctypes.data_as(C.c_void_p), fg.ctypes.data_as(C.c_void_p),
                                   None if keep[0] is None else keep[0].ctypes.data_as(C.c_void_p),
                                   None if keep[1] is None else keep[1].ctypes.data_as(C.c_void_p))


def test_lattice_meshes_are_accepted():
    base = I.small_block(n=(6, 5, 5), blk=((2, 4), (2, 3), (2, 3)), m=6)
    for split in (I.TET, I.PYRAMID, I.PRISM, I.HEX, np.random.default_rng(2).integers(0, 4, (5, 5, 6))):
        case = I.on_mesh(base, I.lattice_mesh(6, 5, 5, base.lx, base.ly, base.lz, split=split, solid=base.solid))
        assert Context(case).workspace_size() > 0


def test_bad_meshes_are_rejected():
    base = I.cavity(2, 4, 0.5)
    m = I.lattice_mesh(2, 2, 2, 1.0, 1.0, 1.0, split=I.TET)
    cases = []
    fg = m.face_geom.copy(); fg[3, 1:] *= 1.1                       # not a unit normal
    cases.append((m.volume, m.face_cell, fg))
    vol = m.volume.copy(); vol[0] = 0.0                             # zero volume
    cases.append((vol, m.face_cell, m.face_geom))
    fc = m.face_cell.copy(); fc[0, 1] = m.ncell                     # neighbour out of range
    cases.append((m.volume, fc, m.face_geom))
    fc = m.face_cell.copy(); fc[0, 1] = -8                          # boundary slot 7
    cases.append((m.volume, fc, m.face_geom))
    keep = np.ones(m.nface, dtype=bool); keep[5] = False            # a cell left open
    cases.append((m.volume, m.face_cell[keep], m.face_geom[keep]))
    for vol, fc, fg in cases:
        L, h = raw_ctx(base)
        assert set_mesh(L, h, vol, fc, fg) == EINVAL
        L.gsis_destroy(h)


def test_bad_centroids_are_rejected():
    """Centroids come in pairs, and a face's centroid distance along its normal
    must be positive (a cell centroid on the wrong side of a face)."""
    base = I.cavity(2, 4, 0.5)
    m = I.lattice_mesh(2, 2, 2, 1.0, 1.0, 1.0, split=I.TET)
    L, h = raw_ctx(base)
    assert set_mesh(L, h, m.volume, m.face_cell, m.face_geom, m.centroid, None) == EINVAL
    L.gsis_destroy(h)
    bad = m.centroid.copy()
    bad[0] = m.centroid[m.face_cell[0, 1]] if m.face_cell[0, 1] >= 0 else bad[0] + 10.0
    L, h = raw_ctx(base)
    assert set_mesh(L, h, m.volume, m.face_cell, m.face_geom, bad, m.face_center) == EINVAL
    L.gsis_destroy(h)
    L, h = raw_ctx(base)
    assert set_mesh(L, h, m.volume, m.face_cell, m.face_geom, m.centroid, m.face_center) == 0
    L.gsis_destroy(h)


def test_cyclic_mesh_is_rejected():
    """Three unit cells in a ring, each leaving along +x into the next (every
    cell closed: one face out along +x, one in): nodes with xi_x > 0 have no
    sweep order."""
    base = I.cavity(1, 4, 0.5)
    vol = np.ones(3)
    fc = np.array([[0, 1], [1, 2], [2, 0]])
    fg = np.array([[1, 1, 0, 0]] * 3, dtype=float)
    L, h = raw_ctx(base)
    assert set_mesh(L, h, vol, fc, fg) == EINVAL
    assert b"cycle" in L.gsis_last_error(h)
    L.gsis_destroy(h)


def test_order_of_calls():
    base = I.cavity(2, 4, 0.5)
    m = I.lattice_mesh(2, 2, 2, 1.0, 1.0, 1.0, split=I.TET)
    L, h = raw_ctx(base, with_list=False)
    assert set_mesh(L, h, m.volume, m.face_cell, m.face_geom) == ESTATE      # no velocity list yet
    L.gsis_destroy(h)
    L, h = raw_ctx(base)
    assert set_mesh(L, h, m.volume, m.face_cell, m.face_geom) == 0
    assert set_mesh(L, h, m.volume, m.face_cell, m.face_geom) == ESTATE      # twice
    t = np.ascontiguousarray(I.tensor_velocity_list(base.nv, base.vmin, base.vmax))
    assert L.gsis_set_velocity_list(h, t.ctypes.data_as(C.c_void_p), t.shape[0]) == ESTATE
    mask = np.zeros(8, dtype=np.uint8)
    assert L.gsis_set_solid_mask(h, mask.ctypes.data_as(C.c_void_p), mask.size) == ESTATE
    L.gsis_destroy(h)
    so = I.cavity(2, 4, 0.5, order=2)
    L, h = raw_ctx(so)
    assert set_mesh(L, h, m.volume, m.face_cell, m.face_geom) == ESTATE      # second order
    L.gsis_destroy(h)


def test_workspace_holds_the_sweep_schedule():
    """The workspace grows with the classes x cells sweep entries; a mesh
    through the Python binding sizes it without a GPU."""
    base = I.cavity(3, 6, 0.5)
    small = Context(I.on_mesh(base, I.lattice_mesh(3, 3, 3, 1.0, 1.0, 1.0, split=I.HEX))).workspace_size()
    tets = Context(I.on_mesh(base, I.lattice_mesh(3, 3, 3, 1.0, 1.0, 1.0, split=I.TET))).workspace_size()
    assert tets > small


def test_wall_flux_model_validation():
    """gsis_set_wall_flux: unknown models are EINVAL; both models are accepted
    on a box and, in either order of the calls, on an unstructured mesh."""
    base = I.small_block(n=(6, 5, 5), blk=((2, 4), (2, 3), (2, 3)), m=6)
    L = _lib.lib()
    cfg = make_config(base)
    h = C.c_void_p()
    assert L.gsis_create(C.byref(h), C.byref(cfg)) == 0
    assert L.gsis_set_wall_flux(h, 2) == EINVAL
    assert L.gsis_set_wall_flux(h, -1) == EINVAL
    assert L.gsis_set_wall_flux(h, 1) == 0
    assert L.gsis_set_wall_flux(h, 0) == 0
    L.gsis_destroy(h)
    mesh = I.lattice_mesh(2, 2, 2, 1.0, 1.0, 1.0, split=I.TET)
    L, h = raw_ctx(base)
    assert set_mesh(L, h, mesh.volume, mesh.face_cell, mesh.face_geom, mesh.centroid, mesh.face_center) == 0
    assert L.gsis_set_wall_flux(h, 1) == 0
    assert L.gsis_set_wall_flux(h, 3) == EINVAL
    L.gsis_destroy(h)
    L, h = raw_ctx(base)
    assert L.gsis_set_wall_flux(h, 1) == 0
    assert set_mesh(L, h, mesh.volume, mesh.face_cell, mesh.face_geom, mesh.centroid, mesh.face_center) == 0
    L.gsis_destroy(h)
