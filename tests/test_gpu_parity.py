"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same
seeded inputs: every phase separately (each fed the oracle's own inputs) and
whole runs.  Bars: relative L2 per variable <= 1e-12 for FP64 and <= 2e-5 for
the FP32 form.

Paper: Eq. 3-4 and Alg. 1 (predictor, Riemann, corrector), Sec. 2.3 (AMR)."""
import numpy as np
import pytest

import oracle
import paper_1806_07984_amd as A
from paper_1806_07984_amd import inputs
from helpers import rel_l2_blocks, rel_l2_per_var, solution_weights

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 2e-5}


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def make_pair(order, n, precision, max_level=0, refine=None):
    om = oracle.Mesh(order, n, max_level=max_level, refine=refine)
    gm = A.Mesh(A.instance(order, n, max_level=max_level, refine=refine), precision)
    return om, gm


def check_phases(om, gm, u0, n_base, precision):
    tol = TOL[precision]
    print(f"[phases] p={om.N - 1} n={n_base} cells={om.nc} {precision}", flush=True)
    assert np.array_equal(gm.cells(), om.cells())
    xyz = gm.node_coords().cpu().numpy().reshape(3, om.nc, -1)
    assert np.abs(xyz - om.node_coords()).max() < 1e-14
    W = solution_weights(om, n_base)

    u = dev(u0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    gm.cfl(u, dt)
    dt_ref, st = om.cfl(u0)
    assert st == 0
    assert abs(dt.item() - dt_ref) <= 1e-14 * dt_ref

    # predictor (both sides use the oracle's dt)
    dt.fill_(dt_ref)
    us, tr = gm.empty_u(), gm.empty_traces()
    gm.predictor(u, dt, us, tr)
    us_ref, tr_ref = om.predictor(u0, dt_ref)
    e = rel_l2_per_var(us.cpu().numpy(), us_ref, W)
    assert e.max() <= tol, ("ustar", e)
    et = rel_l2_blocks(tr.cpu().numpy().reshape(tr_ref.shape), tr_ref, 3)
    assert et.max() <= tol, ("traces", et)

    # Riemann on identical traces (rounded to the path's precision first)
    tr_in = dev(tr_ref, gm.real_dtype)
    fs = gm.empty_fside()
    gm.riemann(tr_in, fs)
    fs_ref, bad = om.riemann(tr_in.double().cpu().numpy().reshape(tr_ref.shape))
    assert bad == 0
    ef = rel_l2_blocks(fs.cpu().numpy().reshape(fs_ref.shape), fs_ref, 2)
    assert ef.max() <= tol, ("fside", ef)

    # corrector on identical u* and face fluxes
    fs_in = dev(fs_ref, gm.real_dtype)
    un = gm.empty_u()
    gm.corrector(dev(us_ref), fs_in, dt, un)
    un_ref = om.corrector(us_ref, fs_in.double().cpu().numpy().reshape(fs_ref.shape), dt_ref)
    e = rel_l2_per_var(un.cpu().numpy(), un_ref, W)
    assert e.max() <= (1e-13 if precision == "fp64" else 1e-12), ("corrector", e)
    gm.status()


def check_run(om, gm, u0, n_base, precision, nsteps, two_streams=False):
    tol = TOL[precision]
    print(f"[run] p={om.N - 1} n={n_base} cells={om.nc} {precision} steps={nsteps} two={two_streams}",
          flush=True)
    u = dev(u0)
    ws = gm.empty_workspace()
    hist = torch.zeros(nsteps, dtype=torch.float64, device="cuda")
    if two_streams:
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        s1.wait_stream(torch.cuda.current_stream())
        gm.step(u, nsteps, ws, hist, stream_skeleton=s1, stream_enclave=s2)
        torch.cuda.current_stream().wait_stream(s1)
    else:
        gm.step(u, nsteps, ws, hist)
    torch.cuda.synchronize()
    gm.status()
    u_ref, hist_ref, rc = om.run(u0, nsteps)
    assert rc == 0
    assert np.abs(hist.cpu().numpy() / hist_ref - 1).max() <= (1e-12 if precision == "fp64" else 1e-5)
    e = rel_l2_per_var(u.cpu().numpy(), u_ref, solution_weights(om, n_base))
    print("   rel L2 per variable:", e, flush=True)
    assert e.max() <= tol, e
    return u


# --------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_density_wave_9cubed_p3(precision):
    """9^3 periodic mesh, p = 3, density wave with seeded node noise, 10 steps."""
    n = (9, 9, 9)
    om, gm = make_pair(3, n, precision)
    u0 = inputs.density_wave_noisy(om.node_coords(), seed=1, noise=0.01)
    check_phases(om, gm, u0, n, precision)
    check_run(om, gm, u0, n, precision, 10)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5, 6])
def test_orders_ragged_mesh_fp64(p):
    n = (5, 3, 2)
    om, gm = make_pair(p, n, "fp64")
    u0 = inputs.density_wave_noisy(om.node_coords(), seed=10 + p, noise=0.05)
    check_phases(om, gm, u0, n, "fp64")
    check_run(om, gm, u0, n, "fp64", 3)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_orders_ragged_mesh_fp32(p):
    n = (4, 3, 5)
    om, gm = make_pair(p, n, "fp32")
    u0 = inputs.density_wave_noisy(om.node_coords(), seed=20 + p, noise=0.05)
    check_phases(om, gm, u0, n, "fp32")
    check_run(om, gm, u0, n, "fp32", 3)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_amr_blast(p, precision):
    """3^3 base cells, two levels of 3:1 refinement in a sphere (level jumps
    of 1 and 2), smoothed blast wave; phases, runs, and the two-stream
    schedule bit-for-bit equal to the single-stream one."""
    n = (3, 3, 3)
    ref = inputs.sphere_refine_list(n, 2, radius=0.2)
    om, gm = make_pair(p, n, precision, max_level=2, refine=ref)
    assert gm.info["n_hanging_faces"] > 0 and gm.info["n_skeleton_cells"] > 0
    u0 = inputs.blast_smooth(om.node_coords(), width=1.0 / 27, radius=0.2)
    check_phases(om, gm, u0, n, precision)
    u1 = check_run(om, gm, u0, n, precision, 3)
    u2 = check_run(om, gm, u0, n, precision, 3, two_streams=True)
    assert torch.equal(u1, u2)


def test_amr_density_wave_fp64():
    """Smooth wave crossing level transitions (9^3 base, one level)."""
    n = (9, 9, 9)
    ref = inputs.sphere_refine_list(n, 1, radius=0.2)
    om, gm = make_pair(3, n, "fp64", max_level=1, refine=ref)
    u0 = inputs.density_wave_noisy(om.node_coords(), seed=3, noise=0.01)
    check_phases(om, gm, u0, n, "fp64")
    check_run(om, gm, u0, n, "fp64", 4)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_step_to_end_time(precision):
    """adg_step with an end time: every step takes min(dt_cfl, t_end - t), the
    last one lands on t_end, further steps of the call have dt = 0 and change
    nothing; the state matches the oracle's run to the same end time, and the
    step-by-step phase loop with the same clamp gives the same bits."""
    n, p, T = (5, 4, 3), 3, 0.0123
    om, gm = make_pair(p, n, precision)
    u0 = inputs.density_wave_noisy(om.node_coords(), seed=8, noise=0.01)
    ref, dts_ref, rc = om.run(u0, 200, t_end=T)
    assert rc == 0
    used = int(np.count_nonzero(dts_ref))
    u = dev(u0)
    hist = torch.full((used + 3,), -1.0, dtype=torch.float64, device="cuda")
    gm.step(u, used + 3, gm.empty_workspace(), dt_hist=hist, t_end=T)
    torch.cuda.synchronize()
    gm.status()
    h = hist.cpu().numpy()
    print(f"[t_end] {precision}: {used} steps, last dt {h[used - 1]:.3e}, sum {h.sum():.17g}", flush=True)
    assert np.all(h[used:] == 0.0) and np.all(h[:used] > 0.0)
    assert abs(h.sum() - T) <= 1e-15
    assert np.abs(h[:used] - dts_ref[:used]).max() <= (1e-13 if precision == "fp64" else 1e-6) * T
    e = rel_l2_per_var(u.cpu().numpy(), ref, solution_weights(om, n))
    assert e.max() <= TOL[precision], e
    # the phase entry points with the clamp done on the host
    v = dev(u0)
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    us, tr, fs = gm.empty_u(), gm.empty_traces(), gm.empty_fside()
    t = 0.0
    for k in range(used):
        gm.cfl(v, dt)
        d = float(dt.item())
        if d >= T - t:
            d = T - t
        dt.fill_(d)
        gm.predictor(v, dt, us, tr)
        gm.riemann(tr, fs)
        gm.corrector(us, fs, dt, v)
        t += d
        assert d == h[k], (k, d, h[k])
    assert torch.equal(u, v)
    gm.close()



@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n", [(6, 5, 7), (1, 4, 2), (3, 1, 1), (13, 17, 11)])
def test_face_fusion_same_bits(precision, n):
    """adg_step with the Riemann problems inside the corrector (the default for
    one uniform p = 3 instance) against the separate face and corrector
    kernels: the same bits after several steps, including the step sizes, on
    meshes with unequal and single-cell axes (a cell that is its own
    periodic neighbour) and with partial cell tiles along every axis (13 x 17
    x 11: tiles of 8 x 9 x 9); and the oracle's run to the stated bar."""
    om, gm = make_pair(3, n, precision)
    u0 = inputs.density_wave_noisy(om.node_coords(), seed=31, noise=0.02)
    steps = 4
    runs = []
    for fuse in (True, False):
        gm.set_face_fusion(fuse)
        u = dev(u0)
        hist = torch.zeros(steps, dtype=torch.float64, device="cuda")
        gm.step(u, steps, gm.empty_workspace(), dt_hist=hist)
        gm.status()
        runs.append((u, hist))
    print(f"[face fusion] {precision} n={n}", flush=True)
    assert torch.equal(runs[0][1], runs[1][1])
    assert torch.equal(runs[0][0], runs[1][0])
    ref, _, rc = om.run(u0, steps)
    assert rc == 0
    e = rel_l2_per_var(runs[0][0].cpu().numpy(), ref, solution_weights(om, n))
    assert e.max() <= TOL[precision], e
    gm.close()
