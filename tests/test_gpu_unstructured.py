"""GPU parity on unstructured spatial meshes (Sec. 3.2 on cells with
volumes and faces with areas and normals), through the C-ABI
(gsis_set_spatial_mesh), against the FP64 oracle.

Meshes: the lattice meshes of the workload generator -- six Kuhn tetrahedra
per cube, or every cube cut at random into tetrahedra, pyramids, prisms or
kept whole -- for a lid-driven cavity, the Mach-5 block flow (inflow faces, a
solid body as a hole with diffuse walls), the diatomic block flow, a block
flow on a refined velocity mesh and a finite time step.  Bars: one pass from
a seeded random VDF, FP64 1e-12 and FP32 3e-6 relative per point; several
passes from the initial Maxwellian, FP64 1e-12 and FP32 1e-5 on rho, u, T,
and the volume-weighted residual; GSIS iterations (kinetic pass and the
GSIS-II correction on the mesh) against the oracle, FP64 1e-12 and FP32 1e-5;
a mesh of whole hexahedra against the box path on the GPU, kinetic passes and
GSIS; repeated runs bit for bit.
"""
import dataclasses
import sys

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2310_18916_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2310_18916_amd.gsis import GsisError, Solver  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def mixed(n, seed):
    return np.random.default_rng(seed).integers(0, 4, size=(n[2], n[1], n[0]))


def block_mesh(base, n, split):
    return I.lattice_mesh(*n, base.lx, base.ly, base.lz, split=split, solid=base.solid)


def make_cases():
    cav = I.cavity(4, 8, 0.1, lid=0.3)
    blk = I.small_block(n=(8, 6, 6), blk=((3, 5), (2, 4), (2, 4)), m=8)
    dia = I.small_block(species=I.DIATOMIC, n=(6, 5, 5), blk=((2, 4), (2, 3), (2, 3)), m=8)
    ref = I.with_velocity_list(I.small_block(n=(6, 5, 5), blk=((2, 4), (2, 3), (2, 3)), m=8),
                               I.hypersonic_velocity_mesh(5.0, 5.0 / 3.0, 2.0, 2))
    dt = I.cavity(4, 7, 0.2, lid=0.2, inv_dt=0.5)
    return {
        "tet_cavity": I.on_mesh(cav, I.lattice_mesh(4, 4, 4, 1.0, 1.0, 1.0, split=I.TET)),
        "mixed_block": I.on_mesh(blk, block_mesh(blk, (8, 6, 6), mixed((8, 6, 6), 11))),
        "n2_mixed_block": I.on_mesh(dia, block_mesh(dia, (6, 5, 5), mixed((6, 5, 5), 12))),
        "tet_block_refined": I.on_mesh(ref, block_mesh(ref, (6, 5, 5), I.TET)),
        "mixed_cavity_dt": I.on_mesh(dt, I.lattice_mesh(4, 4, 4, 1.0, 1.0, 1.0, split=mixed((4, 4, 4), 13))),
    }


CASES = make_cases()


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def field_errors(mg, mo):
    return {"rho": rel(mg[:, 0], mo[:, 0]), "T": rel(mg[:, 4], mo[:, 4]),
            "u": np.abs(mg[:, 1:4] - mo[:, 1:4]).max() / max(np.abs(mo[:, 1:4]).max(), 1e-300)}


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_unstructured_one_pass(name, dtype):
    case = CASES[name]
    say(f"[umesh pass] {name} {dtype}: {case.mesh.ncell} cells, {case.mesh.nface} faces, {case.nvel} nodes")
    f0, f1 = I.random_vdf(case, seed=31)
    if dtype == "fp32":
        f0 = f0.astype(np.float32).astype(np.float64)
        f1 = None if f1 is None else f1.astype(np.float32).astype(np.float64)
    s = Solver(case, dtype)
    s.set_vdf(f0, f1)
    s.kinetic_step(1)
    g0, g1 = s.get_vdf()
    o = Oracle(case)
    o.set_vdf(f0, f1)
    assert o.step(1) == 0
    o0, o1 = o.get_vdf()
    tol = 1e-12 if dtype == "fp64" else 3e-6
    e0 = rel(g0.cpu().numpy(), o0)
    say(f"  f0 error {e0:.3e}")
    assert e0 <= tol
    if o1 is not None:
        e1 = rel(g1.cpu().numpy(), o1)
        say(f"  f1 error {e1:.3e}")
        assert e1 <= tol


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_unstructured_passes(name, dtype):
    case = CASES[name]
    say(f"[umesh passes] {name} {dtype}")
    s = Solver(case, dtype)
    o = Oracle(case)
    s.init_maxwellian()
    o.init_maxwellian()
    s.kinetic_step(4)
    assert o.step(4) == 0
    eg, eo = s.residual(), o.residual()
    e = field_errors(s.moments(), o.moments())
    say(f"  errors {e}; residual {eg} oracle {eo}")
    tol = 1e-12 if dtype == "fp64" else 1e-5
    assert max(e.values()) <= tol
    assert np.abs(eg - eo).max() <= (1e-9 if dtype == "fp64" else 1e-3) * np.abs(eo).max()


def test_hex_mesh_matches_the_box_path():
    """Whole hexahedra as an unstructured mesh and the same cells as the box:
    the two GPU paths agree to rounding after several passes."""
    say("[umesh hex vs box]")
    base = I.small_block(n=(8, 6, 6), blk=((3, 5), (2, 4), (2, 4)), m=8)
    box = I.with_velocity_list(base, I.tensor_velocity_list(base.nv, base.vmin, base.vmax))
    hexc = I.on_mesh(box, block_mesh(box, (8, 6, 6), I.HEX))
    a, b = Solver(box, "fp64"), Solver(hexc, "fp64")
    a.init_maxwellian()
    b.init_maxwellian()
    a.kinetic_step(3)
    b.kinetic_step(3)
    fluid = ~box.solid_mask().astype(bool)
    e = field_errors(b.moments(), a.moments()[fluid])
    say(f"  errors {e}")
    assert max(e.values()) <= 1e-12


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_unstructured_runs_repeat_bit_for_bit(dtype):
    case = CASES["mixed_block"]
    say(f"[umesh repeat] {dtype}")
    out = []
    for _ in range(2):
        s = Solver(case, dtype)
        s.init_maxwellian()
        s.kinetic_step(3)
        out.append(s.get_vdf()[0].cpu().numpy())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["tet_cavity", "mixed_block", "n2_mixed_block", "tet_block_refined"])
def test_unstructured_gsis(name, dtype):
    case = CASES[name]
    say(f"[umesh gsis] {name} {dtype}")
    s = Solver(case, dtype)
    o = Oracle(case)
    s.init_maxwellian()
    o.init_maxwellian()
    for _ in range(2):
        s.kinetic_step(1)
        assert o.step(1) == 0
        s.gsis_correct(25)
        assert o.gsis_correct(25) == 0
    s.kinetic_step(1)
    assert o.step(1) == 0
    eg, eo = s.residual(), o.residual()
    e = field_errors(s.moments(), o.moments())
    say(f"  errors {e}; residual {eg} oracle {eo}")
    tol = 1e-12 if dtype == "fp64" else 1e-5
    assert max(e.values()) <= tol
    assert np.abs(eg - eo).max() <= (1e-9 if dtype == "fp64" else 1e-3) * np.abs(eo).max()


def test_hex_mesh_gsis_matches_the_box_path():
    """GSIS on whole hexahedra given as an unstructured mesh and on the box:
    the two GPU solves agree to rounding."""
    say("[umesh hex gsis vs box]")
    base = I.small_block(n=(8, 6, 6), blk=((3, 5), (2, 4), (2, 4)), m=8)
    box = I.with_velocity_list(base, I.tensor_velocity_list(base.nv, base.vmin, base.vmax))
    hexc = I.on_mesh(box, block_mesh(box, (8, 6, 6), I.HEX))
    a, b = Solver(box, "fp64"), Solver(hexc, "fp64")
    a.init_maxwellian()
    b.init_maxwellian()
    for _ in range(2):
        a.kinetic_step(1)
        b.kinetic_step(1)
        a.gsis_correct(30)
        b.gsis_correct(30)
    a.kinetic_step(1)
    b.kinetic_step(1)
    fluid = ~box.solid_mask().astype(bool)
    e = field_errors(b.moments(), a.moments()[fluid])
    say(f"  errors {e}")
    assert max(e.values()) <= 1e-12


@pytest.mark.parametrize("name", ["mixed_cavity_dt", "n2_mixed_block"])
def test_unstructured_precondition(name):
    """The initial field of Alg. 1 on the mesh: Euler macroscopic steps (no
    stress, heat flux or high-order terms, the boundary flux of the iterate's
    own Maxwellian), the VDF corrected to them, then kinetic passes."""
    case = CASES[name]
    say(f"[umesh precondition] {name}")
    s = Solver(case, "fp64")
    o = Oracle(case)
    s.init_maxwellian()
    o.init_maxwellian()
    s.precondition(40, 2)
    assert o.precondition(40, 2) == 0
    e = field_errors(s.moments(), o.moments())
    say(f"  errors {e}")
    assert max(e.values()) <= 1e-12


def test_unstructured_refusals():
    say("[umesh refusals]")
    case = CASES["tet_cavity"]
    s = Solver(case, "fp64")
    s.init_maxwellian()
    s.kinetic_step(1)
    for call in (lambda: s.autotune(1), lambda: s.set_tile(4, 4, 4, 128)):
        with pytest.raises(GsisError) as ei:
            call()
        assert ei.value.status == -2
    bare = dataclasses.replace(case, mesh=dataclasses.replace(case.mesh, face_center=None))
    t = Solver(bare, "fp64")
    t.init_maxwellian()
    t.kinetic_step(1)
    with pytest.raises(GsisError) as ei:
        t.gsis_correct(5)
    assert ei.value.status == -2
