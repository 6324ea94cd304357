"""Writes the full-size oracle fields that tests/test_gpu_fullsize_oracle.py
compares the GPU with: the 48^3 x 32^3 cavity (three GSIS iterations), the
Mach-5 block flow at 96x64x64 x 40^3 (two source-iteration passes), the
nitrogen block flow at 64x48x48 x 32^3 (a GSIS iteration and a pass) and the
Mach-5 block flow on 291,840 tetrahedra with the 7788-node refined velocity
mesh (two passes; and a GSIS iteration followed by a pass), and the cavity
again with the Grad-13 wall flux of the correction (three GSIS iterations),
each from its uniform initial Maxwellian, FP64.

Calls only the CPU oracle (its streaming mode, which holds no VDF; the
tetrahedral mesh, which the streaming mode does not take, through the
stored-VDF mode: 18 GB of host memory) and the seeded workload definitions.  The files keep, per recorded stage, the moments
of a fixed sample of fluid cells (half of them next to a wall, solid or
inflow face), the largest |value| of every moment over all fluid cells (the
denominators of the parity norm) and the residual against the previous
record (the first against the initial state).

    python tests/golden/make_fullsize.py c2 c3 c4 c3t c3t_gsis c2_g13     (about two hours on 8 cores)
"""
import dataclasses
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.oracle import Oracle, StreamOracle  # noqa: E402
from paper_2310_18916_amd import inputs as I  # noqa: E402

MACRO_ITERS = 300
NSAMPLE = 1024          # cells drawn among all fluid cells, and as many among boundary-adjacent ones
# operations of each workload: a kinetic pass, a GSIS-II correction, or a record of the state
PLANS = {
    "c2": ["pass", "correct", "record", "pass", "correct", "pass", "correct", "record"],
    "c3": ["pass", "record", "pass", "record"],
    "c4": ["pass", "correct", "record", "pass", "record"],
    "c3t": ["pass", "record", "pass", "record"],
    "c3t_gsis": ["pass", "correct", "record", "pass", "record"],
    "c2_g13": ["pass", "correct", "record", "pass", "correct", "pass", "correct", "record"],
}


def workload(name):
    if name == "c2_g13":    # the cavity with the Grad-13 wall flux of the correction
        return dataclasses.replace(I.c2(), wall_flux=1)
    return {"c2": I.c2, "c3": I.c3, "c4": I.c4, "c3t": I.c3t, "c3t_gsis": I.c3t}[name]()


def sample_cells(case, seed):
    """Fluid cells: NSAMPLE uniform draws and NSAMPLE among cells with a
    boundary (wall, solid or inflow) face, without repeats, sorted."""
    rng = np.random.default_rng(seed)
    if case.mesh is not None:
        fc = case.mesh.face_cell
        ed = np.unique(fc[fc[:, 1] < 0, 0])
        a = rng.choice(case.mesh.ncell, size=min(NSAMPLE, case.mesh.ncell), replace=False)
        b = rng.choice(ed, size=min(NSAMPLE, ed.size), replace=False)
        return np.unique(np.concatenate([a, b])).astype(np.int64)
    n = (case.nx, case.ny, case.nz)
    solid = case.solid_mask().reshape(n[2], n[1], n[0]).astype(bool)
    fluid = ~solid
    edge = np.zeros_like(fluid)
    pad = np.pad(solid, 1, constant_values=True)
    for ax in range(3):
        for sh in (-1, 1):
            edge |= np.roll(pad, sh, axis=ax)[1:-1, 1:-1, 1:-1]
    edge &= fluid
    fl = np.flatnonzero(fluid.reshape(-1))
    ed = np.flatnonzero(edge.reshape(-1))
    a = rng.choice(fl, size=min(NSAMPLE, fl.size), replace=False)
    b = rng.choice(ed, size=min(NSAMPLE, ed.size), replace=False)
    return np.unique(np.concatenate([a, b])).astype(np.int64)


def run(name):
    case = workload(name)
    cells = sample_cells(case, seed=2310_18916 + sum(map(ord, name)))
    fluid = ~case.solid_mask().astype(bool)
    o = Oracle(case) if case.mesh is not None else StreamOracle(case)
    o.init_maxwellian()
    o.residual()
    mom, fmax, eps, tags = [], [], [], []
    t0 = time.time()
    for k, op in enumerate(PLANS[name]):
        if op == "pass":
            st = o.step(1)
        elif op == "correct":
            st = o.gsis_correct(MACRO_ITERS)
        else:
            # the residual against the previous record (or the initial state)
            st = o.status()
            eps.append(o.residual())
            m = o.moments()
            mom.append(m[cells])
            fmax.append(np.abs(m[fluid]).max(axis=0))
            tags.append(k)
        if st != 0:
            raise RuntimeError(f"{name}: oracle status {st} at step {k} ({op})")
        print(f"{name}: {op} done at {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, f"fullsize_{name}.npz")
    np.savez_compressed(out, plan=np.array(PLANS[name]), record_at=np.array(tags), cells=cells,
                        moments=np.array(mom), field_max=np.array(fmax), eps=np.array(eps),
                        macro_iters=MACRO_ITERS, workload=case.name)
    print(f"wrote {out} ({os.path.getsize(out)} bytes)", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["c2", "c3", "c4"]:
        run(name)
