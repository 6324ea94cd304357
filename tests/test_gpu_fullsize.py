"""GPU checks at the full workload sizes, through the C-ABI.

The oracle cannot hold these VDFs, so parity is taken on sampled outputs it
can compute one by one: the first pass from the uniform initial Maxwellian at
selected velocity nodes, for every cell (oracle.first_pass_nodes), after the
pass run by the autotuner in the launch configuration bench.py uses.  Beyond
the first pass, properties that hold at any size are checked: mirror symmetry
of the cavity and the agreement of the FP32 and FP64 paths, with first- and
second-order right-hand sides.
"""
import sys

import numpy as np
import pytest

from oracle.oracle import first_pass_nodes, node_grid
from paper_2310_18916_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2310_18916_amd.gsis import Solver  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sample_nodes(case, extra=6, seed=7):
    """The fastest and the slowest node of every octant, plus seeded random nodes."""
    xi, _ = node_grid(case)
    octant = (xi[:, 0] < 0) * 1 + (xi[:, 1] < 0) * 2 + (xi[:, 2] < 0) * 4
    speed = (xi * xi).sum(1)
    picks = set()
    for o in range(8):
        idx = np.nonzero(octant == o)[0]
        if idx.size:
            picks.add(int(idx[np.argmax(speed[idx])]))
            picks.add(int(idx[np.argmin(speed[idx])]))
    rng = np.random.default_rng(seed)
    picks.update(int(v) for v in rng.integers(0, case.nvel, extra))
    return np.array(sorted(picks), dtype=np.int32)


def first_pass_parity(case, dtype, tol):
    nodes = sample_nodes(case)
    s = Solver(case, dtype)
    s.init_maxwellian()
    if case.mesh is None:
        s.autotune(reps=1)                   # the first pass, in bench.py's configuration
        tile = s.get_tile()
    else:
        s.kinetic_step(1)                    # an unstructured mesh: no tiles
        tile = "(unstructured)"
    g = s.get_vdf_nodes(nodes).cpu().numpy()
    del s
    torch.cuda.empty_cache()
    o0, _, st = first_pass_nodes(case, nodes)
    assert st == 0
    fluid = ~case.solid_mask().astype(bool)
    err = np.abs(g[:, fluid] - o0[:, fluid]).max() / np.abs(o0[:, fluid]).max()
    say(f"  {case.name} {dtype} tile {tile}: {nodes.size} nodes x {int(fluid.sum())} cells, error {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("workload,dtype,tol", [("c2", "fp64", 1e-13), ("c2", "fp32", 3e-6),
                                                ("c3", "fp32", 3e-6), ("c3", "fp64", 1e-13),
                                                ("c4", "fp32", 3e-6), ("c4", "fp64", 1e-13),
                                                ("c3r", "fp32", 3e-6), ("c3r", "fp64", 1e-13),
                                                ("c3t", "fp32", 3e-6), ("c3t", "fp64", 1e-12)])
def test_full_size_first_pass_matches_oracle(workload, dtype, tol):
    say(f"[full-size first pass] {workload} {dtype}")
    first_pass_parity(getattr(I, workload)(), dtype, tol)


def test_c2_gsis_mirror_symmetry():
    """The lid moves along x, so the cavity is symmetric under y -> 1 - y with
    u_y -> -u_y; after GSIS iterations at full size the fields must be too."""
    say("[c2 symmetry]")
    case = I.c2()
    s = Solver(case, "fp64")
    s.init_maxwellian()
    s.autotune(reps=1)
    for _ in range(3):
        s.gsis_correct(case.macro_iters)
        s.kinetic_step(1)
    m = s.moments().reshape(case.nz, case.ny, case.nx, -1)
    mir = m[:, ::-1, :, :].copy()
    mir[..., 2] *= -1.0                     # u_y
    for k, name in ((0, "rho"), (4, "T"), (1, "ux"), (3, "uz")):
        d = np.abs(m[..., k] - mir[..., k]).max() / np.abs(m[..., k]).max()
        say(f"  {name} asymmetry {d:.2e}")
        assert d <= 1e-10
    d = np.abs(m[..., 2] - mir[..., 2]).max() / np.abs(m[..., 1]).max()
    say(f"  uy asymmetry {d:.2e}")
    assert d <= 1e-10


def test_c2_second_order_symmetry_and_precision():
    """The second-order right-hand side at full size (Venkatakrishnan K = 1):
    after GSIS iterations the c2 fields keep the cavity's mirror symmetry
    (FP64), and the FP32 path tracks the FP64 one within 1e-5."""
    import dataclasses
    say("[c2 second order]")
    case = dataclasses.replace(I.c2(), order=2, limiter_k=1.0)
    res = {}
    for dtype in ("fp64", "fp32"):
        s = Solver(case, dtype, tile=(8, 8, 32, 256) if dtype == "fp64" else (16, 8, 32, 256))
        s.init_maxwellian()
        for _ in range(3):
            s.kinetic_step(1)
            s.gsis_correct(case.macro_iters)
        res[dtype] = s.moments()
        del s
        torch.cuda.empty_cache()
    m = res["fp64"].reshape(case.nz, case.ny, case.nx, -1)
    mir = m[:, ::-1, :, :].copy()
    mir[..., 2] *= -1.0
    for k, name in ((0, "rho"), (4, "T"), (1, "ux"), (3, "uz")):
        d = np.abs(m[..., k] - mir[..., k]).max() / np.abs(m[..., k]).max()
        say(f"  {name} asymmetry {d:.2e}")
        assert d <= 1e-10
    a, b = res["fp32"], res["fp64"]
    errs = {"rho": np.abs(a[:, 0] - b[:, 0]).max() / np.abs(b[:, 0]).max(),
            "T": np.abs(a[:, 4] - b[:, 4]).max() / np.abs(b[:, 4]).max(),
            "u": np.abs(a[:, 1:4] - b[:, 1:4]).max() / np.abs(b[:, 1:4]).max()}
    say(f"  fp32 vs fp64 {errs}")
    assert max(errs.values()) <= 1e-5


@pytest.mark.parametrize("workload,steps", [("c3", 20), ("c4", 3)])
def test_full_size_fp32_tracks_fp64(workload, steps):
    """The FP32 path against the FP64 path at full size: 20 passes of the
    supersonic block (c3), 3 GSIS iterations of the diatomic block (c4)."""
    say(f"[fp32 vs fp64] {workload}")
    case = getattr(I, workload)()
    res = {}
    for dtype in ("fp64", "fp32"):
        s = Solver(case, dtype)
        s.init_maxwellian()
        for _ in range(steps):
            s.kinetic_step(1)
            if case.gsis:
                s.gsis_correct(case.macro_iters)
        res[dtype] = s.moments()
        del s
        torch.cuda.empty_cache()
    fluid = ~case.solid_mask().astype(bool)
    a, b = res["fp32"][fluid], res["fp64"][fluid]
    assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
    errs = {"rho": np.abs(a[:, 0] - b[:, 0]).max() / np.abs(b[:, 0]).max(),
            "T": np.abs(a[:, 4] - b[:, 4]).max() / np.abs(b[:, 4]).max(),
            "u": np.abs(a[:, 1:4] - b[:, 1:4]).max() / np.abs(b[:, 1:4]).max()}
    if case.species == I.DIATOMIC:
        errs["Tr"] = np.abs(a[:, 14] - b[:, 14]).max() / np.abs(b[:, 14]).max()
    say(f"  {errs}")
    assert max(errs.values()) <= 1e-5
