"""Host-side checks of the C-ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments and out-of-order calls before any
device work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2310_18916_amd import _lib
from paper_2310_18916_amd import gsis as G
from paper_2310_18916_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libgsis.so not built")


def header_symbols():
    text = open(os.path.join(ROOT, "include", "gsis.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsis_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = header_symbols()
    assert len(names) >= 20
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.SIGNATURES) == names


def test_phase_names_match_header():
    """gsis_profile_read fills GSIS_NPHASE entries: the binding's phase list
    (which sizes its arrays) has exactly that many, in the header's order."""
    text = open(os.path.join(ROOT, "include", "gsis.h")).read()
    n = int(re.search(r"GSIS_NPHASE\s*=\s*(\d+)", text).group(1))
    assert len(_lib.PHASES) == n
    for k, name in enumerate(_lib.PHASES):
        assert re.search(rf"GSIS_PHASE_{name.upper()}\s*=\s*{k}\b", text), name


def _cfg(**kw):
    c = G.make_config(I.cavity(4, 6, 0.1))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def _create(cfg):
    h = C.c_void_p()
    st = _lib.lib().gsis_create(C.byref(h), C.byref(cfg))
    return st, h


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("nvy", 1), ("Kn", 0.0), ("Kn", -1.0), ("lx", 0.0), ("species", 2), ("vdf_dtype", 3),
    ("conservative", 2), ("inv_dt", -1.0), ("macro_cfl", 0.0), ("nz", 5000),
    ("order", 3), ("order", -1), ("limiter_k", float("nan")), ("limiter_k", float("inf")),
])
def test_create_rejects_bad_config(field, value):
    st, h = _create(_cfg(**{field: value}))
    assert st == -1 and not h.value


def test_create_rejects_inverted_velocity_range_and_singular_A():
    c = _cfg()
    c.vmin[0], c.vmax[0] = 1.0, -1.0
    assert _create(c)[0] == -1
    c = _cfg(species=1, dr=2.0, Zr=3.5)
    for k, v in enumerate([1.0, 2.0, 0.5, 1.0]):   # det = 0
        c.A[k] = v
    assert _create(c)[0] == -1


def test_mask_boundary_and_order_checks():
    L = _lib.lib()
    st, h = _create(_cfg())
    assert st == 0
    try:
        bad = np.zeros(10, dtype=np.uint8)
        assert L.gsis_set_solid_mask(h, bad.ctypes.data_as(C.c_void_p), bad.size) == -1
        allsolid = np.ones(64, dtype=np.uint8)
        assert L.gsis_set_solid_mask(h, allsolid.ctypes.data_as(C.c_void_p), 64) == -1
        assert b"solid" in L.gsis_last_error(h)
        u = (C.c_double * 3)(0, 0, 0)
        assert L.gsis_set_boundary(h, 7, 0, u, 1.0, 1.0) == -1
        assert L.gsis_set_boundary(h, 0, 5, u, 1.0, 1.0) == -1
        assert L.gsis_set_boundary(h, 0, 0, u, 0.0, 1.0) == -1
        assert L.gsis_set_boundary(h, 0, 1, u, 1.0, -1.0) == -1
        assert L.gsis_set_boundary(h, 0, 1, u, 1.0, 1.0) == 0
        # device calls before a workspace is bound
        assert L.gsis_init_maxwellian(h, 1.0, u, 1.0, 1.0) == -2
        assert L.gsis_kinetic_step(h, 1) == -2
        assert L.gsis_gsis_correct(h, 1) == -2
        assert L.gsis_precondition(h, 10, 1) == -2
        eps = (C.c_double * 3)()
        assert L.gsis_residual(h, eps) == -2
        out = np.empty(64 * 14)
        assert L.gsis_moments(h, out.ctypes.data_as(C.c_void_p), 0) == -2
        n = C.c_size_t()
        assert L.gsis_workspace_size(h, C.byref(n)) == 0
        vdf = 64 * 216 * 8
        assert n.value > vdf
        # the mask is frozen once the workspace is sized
        ok = np.zeros(64, dtype=np.uint8)
        assert L.gsis_set_solid_mask(h, ok.ctypes.data_as(C.c_void_p), 64) == -2
        assert L.gsis_bind_workspace(h, C.c_void_p(255), n.value) == -1         # misaligned
        assert L.gsis_bind_workspace(h, C.c_void_p(256), n.value - 1) == -3     # too small
        assert L.gsis_bind_workspace(h, None, n.value) == -1
    finally:
        L.gsis_destroy(h)


def test_workspace_grows_with_precision_and_species():
    sizes = {}
    for dt in ("fp32", "fp64"):
        sizes[dt] = G.Context(I.cavity(6, 8, 0.1), dt).workspace_size()
    assert sizes["fp64"] - sizes["fp32"] >= 6 ** 3 * 8 ** 3 * 4
    mono = G.Context(I.small_block(), "fp32").workspace_size()
    dia = G.Context(I.small_block(species=I.DIATOMIC), "fp32").workspace_size()
    case = I.small_block()
    assert dia - mono >= case.ncell * case.nvel * 4


def test_second_order_adds_two_vdf_buffers():
    """Order 2 keeps the sweep's per-point term (one row more: the sink of
    dead cells) and the limiter of every point: two VDF-sized buffers per VDF."""
    import dataclasses
    for dt, esz in (("fp32", 4), ("fp64", 8)):
        for case in (I.cavity(6, 8, 0.1), I.small_block(species=I.DIATOMIC, m=6)):
            one = G.Context(case, dt).workspace_size()
            two = G.Context(dataclasses.replace(case, order=2), dt).workspace_size()
            nvdf = 2 if case.species == I.DIATOMIC else 1
            want = nvdf * (2 * case.ncell + 1) * case.nvel * esz
            assert want <= two - one <= want + 4 * 256, (dt, case.name)


def test_tile_shapes_and_set_tile_validation():
    shapes = G.tile_shapes()
    assert (8, 8, 32) in shapes and (4, 4, 64) in shapes
    ctx = G.Context(I.cavity(6, 8, 0.1), "fp32")
    L = ctx.L
    assert L.gsis_set_tile(ctx.h, 8, 8, 4, 128) == 0
    assert L.gsis_set_tile(ctx.h, 5, 5, 4, 128) == -1     # not compiled
    assert L.gsis_set_tile(ctx.h, 8, 8, 0, 128) == -1
    assert L.gsis_set_tile(ctx.h, 8, 8, 4, 100) == -1     # block must be 64, 128 or 256
    assert L.gsis_set_tile(ctx.h, 8, 8, 4, 32) == -1
    assert L.gsis_set_tile(ctx.h, 16, 16, 4, 256) == -1   # not compiled
    # 16 x 8 is a 2 x 2 grid of 8 x 4 waves: the block is exactly its four waves
    assert (16, 8, 32) in shapes and (8, 8, 64) in shapes
    assert L.gsis_set_tile(ctx.h, 16, 8, 4, 128) == -1
    assert L.gsis_set_tile(ctx.h, 16, 8, 4, 256) == 0
    assert L.gsis_set_tile(ctx.h, 8, 4, 16, 256) == 0
    tile = (C.c_int * 4)()
    assert L.gsis_get_tile(ctx.h, tile) == 0 and tuple(tile) == (8, 4, 16, 256)
    # the diatomic gas keeps two register planes: the 8x8 slab is not compiled for it
    dia = G.Context(I.small_block(species=I.DIATOMIC), "fp32")
    assert dia.L.gsis_set_tile(dia.h, 8, 8, 8, 128) == -1
    assert dia.L.gsis_set_tile(dia.h, 8, 4, 8, 128) == 0
    assert dia.L.gsis_set_tile(dia.h, 16, 8, 8, 256) == 0    # wave grid of 8 x 4 slabs
    f64 = G.Context(I.cavity(6, 8, 0.1), "fp64")
    assert f64.L.gsis_set_tile(f64.h, 8, 8, 8, 128) == -1    # 2 x 2 waves of 4 x 4: block 256 only
    assert f64.L.gsis_set_tile(f64.h, 8, 8, 8, 256) == 0
    assert f64.L.gsis_set_tile(f64.h, 8, 4, 8, 128) == 0


def _batch(ctxs):
    arr = (C.c_void_p * len(ctxs))(*[c.h.value for c in ctxs])
    h = C.c_void_p()
    st = _lib.lib().gsis_batch_create(C.byref(h), arr, len(ctxs))
    return st, h


def test_batch_create_rejects_mixed_or_invalid_cases():
    L = _lib.lib()
    a = G.Context(I.cavity(4, 6, 0.1), "fp32")
    b = G.Context(I.cavity(5, 7, 0.3), "fp32")
    c64 = G.Context(I.cavity(4, 6, 0.1), "fp64")
    dia = G.Context(I.small_block(species=I.DIATOMIC, m=6), "fp32")
    fin = G.Context(I.cavity(4, 6, 0.1, inv_dt=2.0), "fp32")
    assert _batch([a, c64])[0] == -1          # precision differs
    assert _batch([a, dia])[0] == -1          # gas differs
    assert _batch([a, fin])[0] == -1          # finite pseudo time step
    import dataclasses
    ho = G.Context(dataclasses.replace(I.cavity(4, 6, 0.1), order=2), "fp32")
    assert _batch([a, ho])[0] == -1           # second-order right-hand side
    assert _batch([a, a])[0] == -1            # a case twice
    h = C.c_void_p()
    assert L.gsis_batch_create(C.byref(h), None, 1) == -1
    assert L.gsis_batch_create(C.byref(h), (C.c_void_p * 1)(a.h.value), 0) == -1
    st, bh = _batch([a, b])
    assert st == 0 and bh.value
    assert L.gsis_batch_destroy(bh) == 0


def test_batch_host_checks_before_device_work():
    """Sizes, tile validation and call order, all on the host."""
    L = _lib.lib()
    cases = [I.cavity(4, 6, 0.1), I.cavity(6, 9, 0.05), I.cavity(5, 8, 0.2)]
    ctxs = [G.Context(c, "fp32") for c in cases]
    st, bh = _batch(ctxs)
    assert st == 0
    n = C.c_size_t()
    assert L.gsis_batch_workspace_size(bh, C.byref(n)) == 0
    assert n.value >= sum(c.workspace_size() for c in ctxs)
    assert L.gsis_batch_set_tile(bh, 5, 5, 4, 128) != 0      # not compiled
    assert L.gsis_batch_set_tile(bh, 8, 4, 8, 256) == 0
    t = (C.c_int * 4)()
    assert L.gsis_batch_get_tile(bh, t) == 0 and tuple(t) == (8, 4, 8, 256)
    assert L.gsis_batch_run(bh, 1, 10, 0) == -2               # not initialised
    assert L.gsis_batch_run(bh, -1, 10, 0) == -2
    cnt = C.c_int()
    eps = (C.c_double * 30)()
    assert L.gsis_batch_residuals(bh, eps, 10, C.byref(cnt)) == -2   # not bound
    ms = C.c_double()
    assert L.gsis_batch_last_run_ms(bh, C.byref(ms)) == -2
    assert L.gsis_batch_bind_workspace(bh, None, n.value) == -1
    assert L.gsis_batch_bind_workspace(bh, C.c_void_p(256), 16) == -3   # smaller than required
    assert L.gsis_batch_destroy(bh) == 0


def test_velocity_nodes_validation():
    L = _lib.lib()
    st, h = _create(_cfg())            # 4^3 cells, 6 nodes per axis
    assert st == 0
    try:
        good = np.linspace(-3.0, 4.0, 6)
        P = lambda a: a.ctypes.data_as(C.c_void_p)
        assert L.gsis_set_velocity_nodes(h, 3, P(good), 6) == -1          # axis
        assert L.gsis_set_velocity_nodes(h, 0, P(good), 5) == -1          # count
        assert L.gsis_set_velocity_nodes(h, 0, None, 6) == -1
        bad = good.copy()
        bad[3] = bad[2]
        assert L.gsis_set_velocity_nodes(h, 1, P(bad), 6) == -1           # not strictly increasing
        bad[3] = np.nan
        assert L.gsis_set_velocity_nodes(h, 1, P(bad), 6) == -1
        assert L.gsis_set_velocity_nodes(h, 2, P(good), 6) == 0
        n = C.c_size_t()
        assert L.gsis_workspace_size(h, C.byref(n)) == 0
        assert L.gsis_set_velocity_nodes(h, 2, P(good), 6) == -2          # frozen once sized
    finally:
        L.gsis_destroy(h)


def test_velocity_list_validation():
    """A general node list: argument checks, the node count it sets (the
    workspace follows it), its exclusion from batches and from per-axis nodes."""
    L = _lib.lib()
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    nodes = I.hypersonic_velocity_mesh(5.0, 5.0 / 3.0, 2.0, 2)
    n = nodes.shape[0]
    st, h = _create(_cfg())
    st2, h2 = _create(_cfg())
    assert st == 0 and st2 == 0
    try:
        assert L.gsis_set_velocity_list(h, None, n) == -1
        assert L.gsis_set_velocity_list(h, P(nodes), 1) == -1            # fewer than 2 nodes
        bad = nodes.copy()
        bad[7, 3] = 0.0
        assert L.gsis_set_velocity_list(h, P(bad), n) == -1              # weight must be > 0
        bad = nodes.copy()
        bad[3, 1] = np.inf
        assert L.gsis_set_velocity_list(h, P(bad), n) == -1
        sz = [C.c_size_t(), C.c_size_t()]
        assert L.gsis_workspace_size(h2, C.byref(sz[0])) == 0            # 6^3 = 216 nodes
        assert L.gsis_set_velocity_list(h, P(nodes), n) == 0
        good = np.linspace(-3.0, 4.0, 6)
        assert L.gsis_set_velocity_nodes(h, 0, P(good), 6) == -2         # not a tensor grid now
        assert L.gsis_workspace_size(h, C.byref(sz[1])) == 0
        assert sz[1].value > sz[0].value * (n / 216) * 0.5
        assert L.gsis_set_velocity_list(h, P(nodes), n) == -2            # frozen once sized
    finally:
        L.gsis_destroy(h)
        L.gsis_destroy(h2)
    a = G.Context(I.cavity(4, 6, 0.1), "fp32")
    lst = G.Context(I.with_velocity_list(I.cavity(4, 6, 0.1), nodes), "fp32")
    assert _batch([a, lst])[0] == -1


def test_noalloc_residual_checks_before_device_work():
    """gsis_residual_noalloc refuses contexts beyond its static array (more than
    4096 blocks of 256 cells) before anything else, and otherwise checks the
    state as gsis_residual does."""
    L = _lib.lib()
    eps = (C.c_double * 3)()
    st, h = _create(_cfg(nx=128, ny=128, nz=64))        # 1,048,576 cells: the largest accepted
    assert st == 0
    try:
        assert L.gsis_residual_noalloc(h, eps) == -2    # accepted size, not initialised
    finally:
        L.gsis_destroy(h)
    st, h = _create(_cfg(nx=128, ny=128, nz=65))        # one plane more
    assert st == 0
    try:
        assert L.gsis_residual_noalloc(h, eps) == -1
        assert b"at most 1048576 cells" in L.gsis_last_error(h)
    finally:
        L.gsis_destroy(h)
    assert L.gsis_residual_noalloc(None, eps) == -1


def test_build_keeps_packed_fp32_off():
    """Every HIP source is compiled with the packed-FP32 instructions disabled
    (-Xclang -target-feature -Xclang -packed-fp32-ops, in that order)."""
    from paper_2310_18916_amd.csrc import build as B
    f = B.COMPILE_FLAGS
    i = f.index("-packed-fp32-ops")
    assert f[i - 3:i + 1] == ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    assert "--offload-arch=gfx950" in f
