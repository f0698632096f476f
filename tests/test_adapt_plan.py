"""The library's adaptation rule (adg_adapt_plan, host only) against the
oracle's plain version, on a refined mesh with seeded indicators.  Runs on
the CPU: the library is loaded but no device work is done."""
import numpy as np
import pytest

import oracle
import paper_1806_07984_amd as A
from paper_1806_07984_amd import inputs


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plan_matches_oracle(seed):
    n, L = (4, 3, 3), 2
    ref = inputs.sphere_refine_list(n, 2, radius=0.3)
    om = oracle.Mesh(1, n, max_level=L, refine=ref)
    cells = om.cells()
    rng = np.random.Generator(np.random.PCG64(seed))
    eta = rng.uniform(0.0, 1.0, size=om.nc)
    # make some full sibling groups quiet so that merges happen
    kids = np.nonzero(cells[:, 0] == 2)[0]
    eta[kids[: 27 * 2]] = 0.01
    desc = A.instance(1, n, max_level=L, refine=ref)
    for tr, tc in ((0.9, 0.05), (0.5, 0.2), (2.0, 0.0)):
        got = A.adapt_plan(desc, eta, tr, tc)
        want = oracle.adapt_plan(cells, ref, eta, tr, tc, L)
        assert np.array_equal(got, want), (tr, tc)
    # the plan is a valid mesh description for both sides
    rows = A.adapt_plan(desc, eta, 0.9, 0.05)
    om2 = oracle.Mesh(1, n, max_level=L, refine=rows)
    assert om2.nc > 0
