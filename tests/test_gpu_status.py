"""The step's only error path for bad states: a non-physical state (rho <= 0,
p <= 0 or a non-finite value) met on the device is latched, reported once by
adg_get_status (ADG_ERR_NONPHYSICAL) and then cleared.  The cases are those
where the oracle flags the state itself; every kernel exits normally.

Paper: Eq. 1 (the Euler system, whose pressure and sound speed need rho > 0
and p > 0); the status contract is the library's."""
import numpy as np
import pytest

import oracle
import paper_1806_07984_amd as A
from paper_1806_07984_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NONPHYSICAL = 5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)).cuda()


def expect_nonphysical(gm):
    with pytest.raises(A.AdgError) as e:
        gm.status()
    assert e.value.code == NONPHYSICAL, str(e.value)
    gm.status()  # the latch is cleared by the report


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_sharp_blast_without_limiter_is_reported(precision):
    """The nodal step profile of the blast overshoots to negative density in
    the first face projections (the oracle reports the same step), then a
    physical run on the same handle reports OK."""
    n = (3, 3, 3)
    ref = inputs.sphere_refine_list(n, 2, radius=0.2)
    om = oracle.Mesh(2, n, max_level=2, refine=ref)
    gm = A.Mesh(A.instance(2, n, max_level=2, refine=ref), precision)
    u0 = inputs.blast(om.node_coords())
    assert om.run(u0, 1)[2] == 1
    ws = gm.empty_workspace()
    u = dev(u0)
    print(f"[status] sharp blast {precision}", flush=True)
    gm.step(u, 1, ws)
    expect_nonphysical(gm)
    good = dev(inputs.density_wave(om.node_coords()))
    gm.step(good, 2, ws)
    gm.status()
    assert torch.isfinite(good).all()
    gm.close()


@pytest.mark.parametrize("what", ["negative density", "negative pressure", "nan"])
def test_bad_node_is_reported_by_the_cfl_reduction(what):
    """One bad node in an otherwise smooth state: the oracle's CFL flags it,
    the library's gives dt = 0 and reports NONPHYSICAL, for both entry
    points that start from u (adg_cfl and adg_step)."""
    p, n = 3, (4, 3, 5)
    om = oracle.Mesh(p, n)
    u0 = inputs.density_wave(om.node_coords())
    c, a = 17, 9
    if what == "negative density":
        u0[0, c, a] = -0.3
    elif what == "negative pressure":
        u0[4, c, a] = 0.5 * (u0[1, c, a] ** 2 + u0[2, c, a] ** 2 + u0[3, c, a] ** 2) / u0[0, c, a] - 0.1
    else:
        u0[2, c, a] = np.nan
    assert om.cfl(u0)[1] == 1
    for precision in ("fp64", "fp32"):
        gm = A.Mesh(A.instance(p, n), precision)
        dt = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        gm.cfl(dev(u0), dt)
        expect_nonphysical(gm)
        assert float(dt.item()) == 0.0
        u = dev(u0)
        gm.step(u, 1, gm.empty_workspace())
        expect_nonphysical(gm)
        gm.close()
