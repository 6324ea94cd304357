"""Host logic of the convergence criterion (Sec. 5, Eq. (convergence_critertion))
and of the divergence watch, compiled from the library's own header with g++
and driven on the CPU: the relative changes, the noise floor of the velocity
denominator, and that a forced growth of u is reported as divergence once u
has a reference computed against a real (above-floor) denominator."""
import math
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2310_18916_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("resid") / "resid_host")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "resid_host_driver.cpp"), "-o", exe], check=True)
    return exe


def run(exe, rows):
    text = "\n".join(" ".join(repr(float(x)) if i else str(int(x)) for i, x in enumerate(r)) for r in rows) + "\n"
    out = subprocess.run([exe], input=text, capture_output=True, text=True, check=True).stdout.split("\n")
    res = []
    for line in out:
        if line.strip():
            v = line.split()
            res.append(([float(x) for x in v[:3]], [int(x) for x in v[3:6]], int(v[6])))
    return res


def sums(drho, du, dT, rho, u, T, n=1000):
    """Residual sums of n cells with uniform changes and states."""
    return [n * drho ** 2, n * du ** 2, n * dT ** 2, n * rho ** 2, n * u ** 2, n * T ** 2]


def test_relative_change_and_absolute_below_floor(driver):
    n = 1000
    (e, rel, d), = run(driver, [[0] + sums(1e-3, 2e-4, 3e-3, 1.0, 0.1, 1.2, n)])
    assert rel == [1, 1, 1] and d == 0
    assert math.isclose(e[0], 1e-3, rel_tol=1e-12)
    assert math.isclose(e[1], 2e-3, rel_tol=1e-12)
    assert math.isclose(e[2], 3e-3 / 1.2, rel_tol=1e-12)
    # a gas at rest: u^{n-1} is rounding noise (1e-17 thermal speeds), far below
    # the FP64 floor (1e3 eps)^2 sum T^2: the absolute change is reported
    (e, rel, d), = run(driver, [[0] + sums(1e-3, 1e-17, 3e-3, 1.0, 1e-17, 1.2, n)])
    assert rel == [1, 0, 1]
    assert math.isclose(e[1], math.sqrt(n) * 1e-17, rel_tol=1e-12)
    # the FP32 floor is larger: u of 1e-7 thermal speeds is noise there, not in FP64
    rows = [[p] + sums(1e-3, 1e-6, 3e-3, 1.0, 1e-7, 1.0, n) for p in (0, 1)]
    (_, rel64, _), (_, rel32, _) = run(driver, rows)
    assert rel64[1] == 1 and rel32[1] == 0
    # zero denominators (no fluid cell) never divide
    (e, rel, d), = run(driver, [[0, 0, 0, 0, 0, 0, 0]])
    assert e == [0.0, 0.0, 0.0] and rel == [0, 0, 0] and d == 0


def test_forced_growth_of_u_is_divergence_after_a_start_at_rest(driver):
    """A cavity started at rest: the first call's u denominator is noise (no
    reference taken from it), the second has a real one and sets the
    reference; a later growth of u beyond 1e6 times that reference diverges.
    With the previous rule (reference = the first value, whatever its
    denominator) the noise-over-noise first value hid this growth."""
    rows = [
        [0] + sums(1e-2, 1e-2, 1e-2, 1.0, 1e-18, 1.0),     # first: u at rest, absolute change 0.3
        [0] + sums(1e-3, 1e-4, 1e-3, 1.0, 1e-2, 1.0),      # reference for u: 1e-2
        [0] + sums(1e-4, 1e-5, 1e-4, 1.0, 1e-2, 1.0),      # converging
        [0] + sums(1e-4, 1e6, 1e-4, 1.0, 1e-2, 1.0),       # u jumps: 1e8 = 1e10 times the reference
    ]
    res = run(driver, rows)
    assert res[0][1][1] == 0 and res[0][2] == 0
    assert math.isclose(res[1][0][1], 1e-2, rel_tol=1e-12) and res[1][2] == 0
    assert res[2][2] == 0
    assert res[3][2] == 1
    # the previous rule divided by the noise (1e-2 / 1e-18 = 1e16) and took that
    # as the reference: the jump to 1e8 stayed far below 1e6 times it
    old_first = math.sqrt(rows[0][2] / rows[0][5])
    assert math.isclose(old_first, 1e16, rel_tol=1e-9)
    assert res[3][0][1] < 1e6 * old_first


def test_growth_below_the_factor_is_not_divergence(driver):
    rows = [[0] + sums(1e-3, 1e-4, 1e-3, 1.0, 1e-2, 1.0)] + \
           [[0] + sums(1e-3 * 10 ** k, 1e-4, 1e-3, 1.0, 1e-2, 1.0) for k in range(1, 6)]
    res = run(driver, rows)
    assert [r[2] for r in res] == [0] * 6
    res = run(driver, rows + [[0] + sums(1e-3 * 1e6 * 1.01, 1e-4, 1e-3, 1.0, 1e-2, 1.0)])
    assert res[-1][2] == 1
