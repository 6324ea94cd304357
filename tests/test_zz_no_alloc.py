"""gsis_residual_noalloc (the allocation-free residual, partial sums in the
library's static device array) against gsis_residual (partial sums in the
workspace), through the C-ABI: two identical contexts step identically, one
reports through each entry point, and the results must be bitwise equal --
on two calls in a row on one GPU, the second on a smaller problem (the
static array then still holds the first call's partial sums beyond the
second call's range), and again on a later iteration of each."""
import sys

import numpy as np
import pytest

from paper_2310_18916_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2310_18916_amd.gsis import Solver  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair(case, dtype):
    a, b = Solver(case, dtype), Solver(case, dtype)
    for s in (a, b):
        s.init_maxwellian()
    return a, b


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_noalloc_residual_equals_workspace_residual(dtype):
    big = I.cavity(24, 6, 0.05, lid=0.2)        # 13,824 cells: 54 blocks of the reduction
    small = I.small_block(m=8)                  # 1,080 cells with a solid block: 5 blocks
    pairs = [("big", _pair(big, dtype)), ("small", _pair(small, dtype))]
    for it in range(2):
        for name, (a, b) in pairs:
            say(f"[noalloc] {dtype} {name} iteration {it}")
            for s in (a, b):
                s.kinetic_step(1)
                s.gsis_correct(20)
            ea = a.residual()
            eb = b.residual_noalloc()
            say(f"  workspace {ea} static {eb}")
            assert np.array_equal(ea, eb), (name, it, ea, eb)
            assert np.all(np.isfinite(eb)) and np.all(eb > 0)
            # the snapshot the variant takes is the same as the workspace path's
            assert np.array_equal(a.moments(), b.moments(), equal_nan=True)   # NaN in solid cells
