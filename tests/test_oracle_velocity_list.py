"""Pins of the oracle on general velocity sets (Sec. 3.1: locally refined or
unstructured velocity meshes, one node per velocity cell, weight = volume).

The oracle's arithmetic is the same on a node list as on a tensor grid (every
sum runs over its node table), so the list path is pinned by (a) bitwise
identity with the tensor path when the list spells out a tensor grid, (b)
invariance under a reordering of the list, (c) exact conservation of the
corrected reference distribution on a refined mesh, (d) zero wall mass flux
and GSIS mass conservation on a refined mesh, and (e) the geometry and
quadrature of the refined meshes themselves, against numbers worked out by
hand from the Sec. 3.1 recipe.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2310_18916_amd import inputs as I


def as_list(case, perm=None):
    xi, w = O.node_grid(case)
    t = np.column_stack([xi, w])
    if perm is not None:
        t = t[perm]
    return I.with_velocity_list(dataclasses.replace(case), t)


def run(o, plan):
    o.init_maxwellian()
    for op in plan:
        assert (o.step(1) if op == "pass" else o.gsis_correct(20)) == 0
    return o


@pytest.mark.parametrize("which", ["cavity", "n2_block", "second_order"])
def test_tensor_grid_as_a_list_is_bitwise_the_tensor_path(which):
    case = {"cavity": I.cavity(5, 9, 0.05, lid=0.2),
            "n2_block": I.small_block(species=I.DIATOMIC, m=8),
            "second_order": I.cavity(5, 8, 0.1, lid=0.2, order=2)}[which]
    plan = ["pass", "correct", "pass"]
    a = run(O.Oracle(case), plan)
    b = run(O.Oracle(as_list(case)), plan)
    fa, ga = a.get_vdf()
    fb, gb = b.get_vdf()
    assert np.array_equal(fa, fb)
    if ga is not None:
        assert np.array_equal(ga, gb)
    fl = ~case.solid_mask().astype(bool)
    assert np.array_equal(a.moments()[fl], b.moments()[fl])
    assert np.array_equal(a.residual(), b.residual())


def test_reordered_list_permutes_the_vdf():
    """Canonical node k is entry k of the list: shuffling the list shuffles the
    VDF's node axis and leaves the moments alone (up to summation order)."""
    case = as_list(I.small_block(m=8))
    perm = np.random.default_rng(5).permutation(case.nvel)
    shuf = I.with_velocity_list(dataclasses.replace(case), case.velocity_list[perm])
    plan = ["pass", "correct", "pass"]
    a = run(O.Oracle(case), plan)
    b = run(O.Oracle(shuf), plan)
    fa, _ = a.get_vdf()
    fb, _ = b.get_vdf()
    assert np.abs(fb - fa[:, perm]).max() <= 1e-12 * fa.max()
    fl = ~case.solid_mask().astype(bool)
    ma, mb = a.moments()[fl], b.moments()[fl]
    for cols in ([0], [1, 2, 3], [4]):
        assert np.abs(ma[:, cols] - mb[:, cols]).max() <= 1e-12 * np.abs(ma[:, cols]).max()


def test_collision_conserves_on_a_refined_mesh():
    """The corrected reference distribution has the discrete mass, momentum and
    energy of f on a non-tensor mesh too (random positive f)."""
    L = I.hypersonic_velocity_mesh(5.0, 5.0 / 3.0, 2.0, 2)
    case = I.with_velocity_list(I.cavity(2, 4, 0.1), L)
    o = O.Oracle(case)
    f0, f1 = I.random_vdf(case, seed=11)
    o.set_vdf(f0, f1)
    xi, w = O.node_grid(case)
    x2 = (xi * xi).sum(1)
    for cell in range(case.ncell):
        g0, _ = o.ref_dist(cell)
        d0 = g0 - f0[cell]
        scale = (w * f0[cell] * (1 + x2)).sum()
        assert abs((w * d0).sum()) < 1e-13 * scale
        for a in range(3):
            assert abs((w * xi[:, a] * d0).sum()) < 1e-13 * scale
        assert abs((w * x2 * d0).sum()) < 1e-13 * scale


def test_walls_and_gsis_conserve_mass_on_a_refined_mesh():
    """Closed cavity on a refined mesh: every diffuse-wall face carries zero
    discrete mass flux (outgoing f plus the scaled wall Maxwellian), and the
    GSIS correction moves the total mass only by the quadrature error of the
    discrete Maxwellians of Eq. (updatef)."""
    L = I.refined_velocity_mesh((0.0, 0.0, 0.0), 5.0 * math.sqrt(0.5), [((0.1, 0.0, 0.0), 1.0)], 0.6, 2)
    case = I.with_velocity_list(I.cavity(4, 4, 0.05, lid=0.1), L)
    o = O.Oracle(case)
    f0, _ = I.random_vdf(case, seed=4)
    o.set_vdf(f0)
    xi, w = O.node_grid(case)
    nwall = 0
    for c in range(case.ncell):
        for d in range(6):
            bc, b0, _ = o.boundary_values(c, d)
            if bc < 0:
                continue
            xn = xi[:, d // 2] * (1 if d % 2 else -1)
            face = np.where(xn > 0, f0[c], b0)
            assert abs((w * xn * face).sum()) <= 1e-14 * (w * np.abs(xn) * face).sum()
            nwall += 1
    assert nwall == 6 * 16
    # the discrete Maxwellian M(1, 0, 1) on this mesh has mass 0.982: its
    # quadrature error, which the correction's mass change follows and which
    # shrinks as the mesh is refined
    drift = []
    for H in (0.6, 0.3):
        L = I.refined_velocity_mesh((0.0, 0.0, 0.0), 5.0 * math.sqrt(0.5), [((0.1, 0.0, 0.0), 1.0)], H, 2)
        o = O.Oracle(I.with_velocity_list(I.cavity(4, 4, 0.05, lid=0.1), L))
        o.init_maxwellian()
        assert o.step(2) == 0
        m1 = o.total_mass()
        assert o.gsis_correct(30) == 0
        drift.append(abs(o.total_mass() - m1) / m1)
    assert drift[0] <= 1e-5 and drift[1] <= drift[0] / 2


def test_refined_mesh_geometry_follows_sec_3_1():
    """Mach 5, gamma = 5/3, T_inf = T_w = 1, units sqrt(2 R T_inf):
    U_inf = 5 sqrt(5/6) = 4.5644; the normal-shock density ratio is
    (8/3) 25 / (2 + (2/3) 25) = 25/7, so U_s = 7 U_inf / 25 = 1.27802;
    T_m = 1 + 25/3 = 28/3 = T_s, so the radius is 5 sqrt(14/3) = 10.8012
    (sqrt(R T) = sqrt(T/2)); both refinement cubes have half side
    3 sqrt(1/2) = 2.1213."""
    H, r = 1.0, 2
    L = I.hypersonic_velocity_mesh(5.0, 5.0 / 3.0, H, r)
    xi, w = L[:, :3], L[:, 3]
    Us = np.array([7.0 * 5.0 * math.sqrt(5.0 / 6.0) / 25.0, 0.0, 0.0])
    R = 5.0 * math.sqrt(14.0 / 3.0)
    assert np.all(np.linalg.norm(xi - Us, axis=1) <= R)
    # coarse cubes of volume H^3, fine ones (H/r)^3, and nothing else
    fine = np.isclose(w, (H / r) ** 3, rtol=0, atol=1e-15)
    assert np.all(fine | np.isclose(w, H ** 3, rtol=0, atol=1e-15))
    # the cells tile the ball up to the shell of cubes cut by its surface
    V = 4.0 / 3.0 * math.pi * R ** 3
    assert abs(w.sum() - V) <= 4.0 * math.pi * R * R * (math.sqrt(3.0) / 2.0) * H
    # every point of each refinement cube lies in a fine cell
    rng = np.random.default_rng(3)
    for c in ((5.0 * math.sqrt(5.0 / 6.0), 0.0, 0.0), (0.0, 0.0, 0.0)):
        p = np.asarray(c) + rng.uniform(-1, 1, size=(400, 3)) * 3.0 * math.sqrt(0.5)
        d = np.abs(p[:, None, :] - xi[fine][None, :, :]).max(axis=2)
        assert np.all(d.min(axis=1) <= 0.5 * H / r + 1e-12)
    # no node on a coordinate plane: every node has a definite octant
    assert np.all(xi != 0.0)


@pytest.mark.parametrize("u,T,tol", [((5.0 * math.sqrt(5.0 / 6.0), 0.0, 0.0), 1.0, 1e-3),
                                     ((0.0, 0.0, 0.0), 1.0, 1e-3)])
def test_refined_mesh_integrates_its_maxwellians(u, T, tol):
    """The free-stream and wall Maxwellians, which the refinement cubes cover to
    3 sigma, keep density, velocity and temperature within 1e-3 on the
    hybrid mesh of side 1.0 / 0.5 (midpoint rule on the velocity cells)."""
    L = I.hypersonic_velocity_mesh(5.0, 5.0 / 3.0, 1.0, 2)
    xi, w = L[:, :3], L[:, 3]
    M = (math.pi * T) ** -1.5 * np.exp(-((xi - np.asarray(u)) ** 2).sum(1) / T)
    rho = (w * M).sum()
    uu = (w[:, None] * xi * M[:, None]).sum(0) / rho
    Tt = (2.0 / 3.0) * (w * M * ((xi - uu) ** 2).sum(1)).sum() / rho
    assert abs(rho - 1.0) <= tol
    assert np.abs(uu - np.asarray(u)).max() <= tol
    assert abs(Tt / T - 1.0) <= tol


def test_stream_and_sampled_first_pass_on_a_node_list():
    """The streaming oracle and the sampled first pass, which the full-size
    parity checks use, run on node lists as on tensor grids."""
    L = I.hypersonic_velocity_mesh(5.0, 5.0 / 3.0, 2.0, 2)
    case = I.with_velocity_list(I.small_block(m=8), L)
    full, stream = O.Oracle(case), O.StreamOracle(case)
    for o in (full, stream):
        o.init_maxwellian()
        assert o.step(1) == 0 and o.gsis_correct(20) == 0 and o.step(1) == 0
    fl = ~case.solid_mask().astype(bool)
    mf, ms = full.moments()[fl], stream.moments()[fl]
    for cols in ([0], [1, 2, 3], [4]):
        assert np.abs(mf[:, cols] - ms[:, cols]).max() <= 1e-13 * np.abs(mf[:, cols]).max()
    o = O.Oracle(case)
    o.init_maxwellian()
    o.step(1)
    f0, _ = o.get_vdf()
    nodes = np.array([0, 5, case.nvel // 2, case.nvel - 1])
    s0, _, st = O.first_pass_nodes(case, nodes)
    assert st == 0
    assert np.array_equal(s0[:, fl], f0[fl][:, nodes].T)
