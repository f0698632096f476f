"""Dynamic adaptivity on the GPU against the oracle: the refinement indicator,
the volumetric transfer between meshes, and whole adaptation steps inside a
run (mass conserved through the transfer).  FP64 data throughout (the state
is FP64 in both precisions)."""
import numpy as np
import pytest

import oracle
import paper_1806_07984_amd as A
from paper_1806_07984_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)).cuda()


@pytest.mark.parametrize("p", [1, 3, 4, 6])
def test_indicator_matches_oracle(p):
    n = (3, 3, 2)
    ref = inputs.sphere_refine_list(n, 2, radius=0.25)
    om = oracle.Mesh(p, n, max_level=2, refine=ref)
    gm = A.Mesh(A.instance(p, n, max_level=2, refine=ref), "fp64")
    u0 = inputs.blast_smooth(om.node_coords(), width=1.0 / 27, radius=0.25)
    eta = gm.indicator(dev(u0)).cpu().numpy()
    want = om.indicator(u0)
    print(f"[indicator] p={p} cells={om.nc} max eta {want.max():.3f}", flush=True)
    assert np.abs(eta - want).max() <= 1e-12 * want.max()


@pytest.mark.parametrize("p", [2, 3, 5])
def test_transfer_matches_oracle(p):
    n = (3, 3, 3)
    # a: centre cell refined, its centre child refined again; b: two other
    # cells refined, one child of them refined again.  a -> b coarsens over
    # two levels, refines over one and two levels, and copies the rest.
    ref_a = np.array([[0, 1, 1, 1], [1, 4, 4, 4]], dtype=np.int32)
    ref_b = np.array([[0, 0, 0, 0], [0, 2, 1, 0], [1, 7, 4, 1]], dtype=np.int32)
    om_a = oracle.Mesh(p, n, max_level=2, refine=ref_a)
    om_b = oracle.Mesh(p, n, max_level=2, refine=ref_b)
    gm_a = A.Mesh(A.instance(p, n, max_level=2, refine=ref_a), "fp64")
    gm_b = A.Mesh(A.instance(p, n, max_level=2, refine=ref_b), "fp64")
    u_a = inputs.density_wave_noisy(om_a.node_coords(), seed=40 + p, noise=0.05)
    print(f"[transfer] p={p} cells {om_a.nc} -> {om_b.nc}", flush=True)
    for src_o, dst_o, src_g, dst_g, u in ((om_a, om_b, gm_a, gm_b, u_a),):
        want = src_o.transfer_to(u, dst_o)
        got = src_g.transfer_to(dev(u), dst_g).cpu().numpy().reshape(want.shape)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
        # and back
        back_w = dst_o.transfer_to(want, src_o)
        back_g = dst_g.transfer_to(dev(want), src_g).cpu().numpy().reshape(back_w.shape)
        assert np.abs(back_g - back_w).max() <= 1e-12 * np.abs(back_w).max()
        # identical meshes: copy
        assert torch.equal(src_g.transfer_to(dev(u), src_g), dev(u))
    # different base grids are refused
    other = A.Mesh(A.instance(p, (3, 3, 2)), "fp64")
    with pytest.raises(A.AdgError) as e:
        gm_a.transfer_to(dev(u_a), other)
    assert e.value.code == 1


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_adaptive_run_matches_oracle(precision):
    """Smoothed blast on 3^3 base cells, p = 3, max_level 2: 2 steps, adapt,
    2 steps, adapt, 2 steps.  Plan, mesh and state follow the oracle's
    adaptation (rule, transfer, run); mass is conserved through every
    adaptation."""
    n, p, L = (3, 3, 3), 3, 2
    tr, tc = 0.08, 0.02
    tol = 1e-12 if precision == "fp64" else 2e-5
    desc = A.instance(p, n, max_level=L, refine=np.zeros((0, 4), dtype=np.int32))
    om = oracle.Mesh(p, n, max_level=L)
    gm = A.Mesh(desc, precision)
    u_o = inputs.blast_smooth(om.node_coords(), width=1.0 / 9, radius=0.25)
    u_g = dev(u_o)
    rows = np.zeros((0, 4), dtype=np.int32)
    ws = gm.empty_workspace()
    for stage in range(3):
        gm.step(u_g, 2, ws)
        torch.cuda.synchronize()
        gm.status()
        u_o, _, rc = om.run(u_o, 2)
        assert rc == 0
        mass_before = om.integral(u_o)
        if stage == 2:
            break
        eta_o = om.indicator(u_o)
        rows_o = oracle.adapt_plan(om.cells(), rows, eta_o, tr, tc, L)
        new_g, u_g2 = A.adapt(gm, u_g, tr, tc)
        rows = new_g.descs[0]["refine"]
        assert np.array_equal(rows, rows_o), stage
        om2 = oracle.Mesh(p, n, max_level=L, refine=rows)
        u_o = om.transfer_to(u_o, om2)
        om = om2
        assert np.array_equal(new_g.cells(), om.cells())
        mass_after = om.integral(u_o)
        # exact up to the rounding of summing ~10^5-10^6 node terms per integral
        assert np.allclose(mass_after, mass_before, rtol=1e-12, atol=1e-15)
        print(f"[adapt] {precision} stage {stage}: cells {gm.info['n_cells']} -> {new_g.info['n_cells']}", flush=True)
        gm.close()
        gm, u_g = new_g, u_g2
        ws = gm.empty_workspace()
        e = np.abs(u_g.cpu().numpy().reshape(u_o.shape) - u_o).max() / np.abs(u_o).max()
        assert e <= tol, (stage, e)
    assert len(rows) > 0
    e = np.abs(u_g.cpu().numpy().reshape(u_o.shape) - u_o).max() / np.abs(u_o).max()
    print(f"   final max relative deviation {e:.2e}", flush=True)
    assert e <= tol


def test_handle_plan_and_chunked_transfer_match_oracle():
    """adg_adapt_plan_mesh (leaves and rows kept by the handle) gives the
    oracle's plan, and the transfer onto the planned mesh matches the oracle
    on a mesh large enough (81,953 cells) for the host tables to be built in
    many chunks on several threads."""
    p, n, L = 2, (9, 9, 9), 2
    ref = inputs.sphere_refine_list(n, 2, radius=0.3)
    om = oracle.Mesh(p, n, max_level=L, refine=ref)
    gm = A.Mesh(A.instance(p, n, max_level=L, refine=ref), "fp64")
    u0 = inputs.blast_smooth(om.node_coords(), width=1.0 / 27, radius=0.3)
    eta = om.indicator(u0)
    tr, tc = float(np.quantile(eta, 0.9)), float(np.quantile(eta, 0.6))
    rows = gm.adapt_plan(eta, tr, tc)
    assert np.array_equal(rows, oracle.adapt_plan(om.cells(), ref, eta, tr, tc, L))
    assert np.array_equal(rows, A.adapt_plan(gm.descs[0], eta, tr, tc))
    om2 = oracle.Mesh(p, n, max_level=L, refine=rows)
    gm2 = A.Mesh(A.instance(p, n, max_level=L, refine=rows), "fp64")
    print(f"[plan+transfer] cells {om.nc} -> {om2.nc}", flush=True)
    assert om2.nc != om.nc
    want = om.transfer_to(u0, om2)
    got = gm.transfer_to(dev(u0), gm2).cpu().numpy().reshape(want.shape)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
    # a uniform handle plans too (no rows yet)
    gu = A.Mesh(A.instance(p, (3, 3, 3), max_level=1), "fp64")
    e = np.zeros(27)
    e[13] = 1.0
    assert np.array_equal(gu.adapt_plan(e, 0.5, 0.1), np.array([[0, 1, 1, 1]], dtype=np.int32))
    for m in (gm, gm2, gu):
        m.close()
