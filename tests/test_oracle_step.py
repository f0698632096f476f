"""Pins of the oracle's ADER-DG step against what the method fixes: closed
forms, a textbook special case, invariants and the convergence order.

Paper: Sec. 2.1-2.3 (predictor, Riemann, corrector, AMR), Eq. 3-4, Alg. 1.
Each test names the property it pins; none re-types the oracle's formulas."""
import math

import numpy as np
import pytest

import oracle
from paper_1806_07984_amd import inputs

G = 1.4


def weights3(N):
    w = oracle.gauss_legendre(N)[1]
    return np.einsum("i,j,k->kji", w, w, w).reshape(-1)


def totals(mesh, u, n_base):
    """Integral of every conserved variable over the periodic box."""
    lev = mesh.cells()[:, 0].astype(np.float64)
    vol = (1.0 / np.prod(n_base)) / 27.0 ** lev
    return (u * weights3(mesh.N)[None, None, :]).sum(axis=2) @ vol


def euler_flux_np(u, d):
    rho, m = u[0], u[1:4]
    p = (G - 1) * (u[4] - 0.5 * (m ** 2).sum(axis=0) / rho)
    v = m[d] / rho
    f = np.stack([m[d], v * m[0], v * m[1], v * m[2], v * (u[4] + p)])
    f[1 + d] += p
    return f


def speed_np(u, d):
    rho, m = u[0], u[1:4]
    p = (G - 1) * (u[4] - 0.5 * (m ** 2).sum(axis=0) / rho)
    return np.abs(m[d] / rho) + np.sqrt(G * p / rho)


# --------------------------------------------------------------------------
# time step size
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0, 2, 3])
def test_cfl_closed_form(p):
    n = 5
    m = oracle.Mesh(p, (n, n, n))
    u = inputs.conserved(np.ones((m.nc, m.N ** 3)), (1.0, 1.0, 1.0), 1.0)
    dt, st = m.cfl(u)
    assert st == 0
    lam = 3 * (1.0 + math.sqrt(1.4)) * n
    assert abs(dt - 0.4 / ((2 * p + 1) * lam)) < 1e-15


@pytest.mark.parametrize("p", [0, 2, 4])
def test_free_stream(p):
    m = oracle.Mesh(p, (3, 4, 2))
    u0 = inputs.conserved(np.full((m.nc, m.N ** 3), 1.2), (0.3, -0.2, 0.1), 0.9)
    u, _, rc = m.run(u0, 2)
    assert rc == 0
    assert np.abs(u - u0).max() < 1e-14


def test_cfl_flags_unphysical():
    m = oracle.Mesh(1, (2, 2, 2))
    u = inputs.conserved(np.ones((m.nc, m.N ** 3)), (0.0, 0.0, 0.0), 1.0)
    u[0, 3, 2] = -1.0
    assert m.cfl(u)[1] == 1
    u[0, 3, 2] = np.nan
    assert m.cfl(u)[1] == 1


# --------------------------------------------------------------------------
# predictor
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [0, 1, 3, 5])
def test_predictor_constant_state(p):
    m = oracle.Mesh(p, (3, 2, 2))
    u = inputs.conserved(np.full((m.nc, m.N ** 3), 1.3), (0.2, -0.4, 0.7), 0.8)
    us, tr = m.predictor(u, 1e-2)
    # (u* differs from u by the volume term; the face terms of the corrector
    # cancel it, which test_free_stream pins)
    for s in range(6):
        d = s // 2
        assert np.allclose(tr[s, 0], u[:, :, :m.N ** 2], atol=1e-14)
        f = euler_flux_np(u[:, :, :m.N ** 2], d)
        assert np.allclose(tr[s, 1], f, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_predictor_linear_advection_closed_form(p):
    """For data varying along x only, with constant velocity and pressure, the
    Euler system is linear advection; the discrete space-time solution is the
    translated polynomial q(tau, xi) = rho_h(xi - nu tau), nu = u_x dt/dx, and
    its time average on the faces follows in closed form."""
    N = p + 1
    n = 4
    m = oracle.Mesh(p, (n, 1, 1))
    xyz = m.node_coords()
    vel = (0.7, 0.3, -0.2)
    u = inputs.density_wave(xyz, amp=0.3, vel=vel, wavevec=(1.0, 0.0, 0.0), p=1.0)
    dt = 0.3 / n
    nu = vel[0] * dt * n
    us, tr = m.predictor(u, dt)
    xi = oracle.gauss_legendre(N)[0]
    tx, tw = np.polynomial.legendre.leggauss(40)
    tau, tw = 0.5 * (tx + 1), 0.5 * tw
    for c in range(n):
        rho_nodes = u[0, c].reshape(N, N, N)[0, 0, :]  # along x (same for all y, z)
        poly = np.polynomial.Polynomial.fit(xi, rho_nodes, p, domain=[0, 1], window=[0, 1]) if p > 0 else None
        for s, xf in ((0, 0.0), (1, 1.0)):
            exact = (tw * poly(xf - nu * tau)).sum()
            assert np.allclose(tr[s, 0, 0, c], exact, atol=2e-13, rtol=0)
            # normal flux of the density is u_x rho
            assert np.allclose(tr[s, 1, 0, c], vel[0] * exact, atol=2e-13, rtol=0)
        # y and z faces see the time average at the x nodes
        avg = np.array([(tw * poly(x - nu * tau)).sum() for x in xi])
        face = tr[2, 0, 0, c].reshape(N, N)  # index = a_x + N a_z
        assert np.allclose(face, avg[None, :], atol=2e-13, rtol=0)


def test_predictor_volume_term_has_zero_cell_integral():
    """The weak-form volume term integrates to zero over each cell (the
    derivative of the constant test function vanishes)."""
    m = oracle.Mesh(3, (3, 3, 3))
    u = inputs.density_wave_noisy(m.node_coords(), seed=5, noise=0.05)
    us, _ = m.predictor(u, 2e-3)
    W = weights3(m.N)
    assert np.allclose((us * W).sum(axis=2), (u * W).sum(axis=2), atol=1e-14, rtol=0)


# --------------------------------------------------------------------------
# Riemann solver
# --------------------------------------------------------------------------

def test_riemann_consistency():
    """F(u, u) = f(u): equal traces on both sides give the physical flux."""
    p = 2
    m = oracle.Mesh(p, (3, 3, 3))
    N2 = m.N ** 2
    rng = np.random.Generator(np.random.PCG64(11))
    q = inputs.conserved(rng.uniform(0.8, 1.2, size=(N2,)), (0.3, -0.1, 0.2), 1.0)
    tr = np.zeros((6, 2, 5, m.nc, N2))
    for s in range(6):
        tr[s, 0] = q[:, None, :]
        tr[s, 1] = euler_flux_np(q, s // 2)[:, None, :]
    fs, bad = m.riemann(tr)
    assert bad == 0
    for s in range(6):
        assert np.allclose(fs[s], euler_flux_np(q, s // 2)[:, None, :], atol=1e-15, rtol=0)


# --------------------------------------------------------------------------
# whole step
# --------------------------------------------------------------------------

def textbook_fv_step(u, n, dt):
    """First-order finite volumes with the Rusanov flux on a periodic grid,
    u[5, nz, ny, nx]."""
    out = u.copy()
    for d in range(3):
        ax = 3 - d  # numpy axis of physical axis d
        uR = np.roll(u, -1, axis=ax)
        s = np.maximum(speed_np(u, d), speed_np(uR, d))
        F = 0.5 * (euler_flux_np(u, d) + euler_flux_np(uR, d)) - 0.5 * s * (uR - u)
        out -= dt * n[d] * (F - np.roll(F, 1, axis=ax))
    return out


def test_p0_is_first_order_rusanov_fv():
    n = (5, 4, 3)
    m = oracle.Mesh(0, n)
    rng = np.random.Generator(np.random.PCG64(7))
    rho = rng.uniform(0.7, 1.3, size=m.nc)
    vel = [rng.uniform(-0.5, 0.5, size=m.nc) for _ in range(3)]
    pr = rng.uniform(0.6, 1.4, size=m.nc)
    u = inputs.conserved(rho, vel, pr)[:, :, None]
    dt = 1e-2
    out, _, rc = m.run(u, 1, dt_fixed=dt)
    assert rc == 0
    ref = textbook_fv_step(u[:, :, 0].reshape(5, n[2], n[1], n[0]), n, dt)
    assert np.allclose(out[:, :, 0], ref.reshape(5, -1), atol=1e-14, rtol=0)


@pytest.mark.parametrize("p", [1, 3])
def test_density_wave_keeps_velocity_and_pressure(p):
    m = oracle.Mesh(p, (4, 4, 4))
    u0 = inputs.density_wave(m.node_coords())
    u, _, rc = m.run(u0, 3)
    assert rc == 0
    vel = u[1:4] / u[0]
    pr = (G - 1) * (u[4] - 0.5 * (u[1:4] ** 2).sum(axis=0) / u[0])
    assert np.abs(vel - 1.0).max() < 1e-14
    assert np.abs(pr - 1.0).max() < 1e-14


@pytest.mark.parametrize("p", [0, 2, 3])
def test_conservation_uniform(p):
    m = oracle.Mesh(p, (4, 3, 5))
    u0 = inputs.density_wave_noisy(m.node_coords(), seed=3, noise=0.05)
    t0 = totals(m, u0, (4, 3, 5))
    u, _, rc = m.run(u0, 3)
    assert rc == 0
    assert np.allclose(totals(m, u, (4, 3, 5)), t0, atol=1e-14, rtol=0)


def test_shift_invariance():
    """A cyclic shift by whole cells commutes with the step, bit for bit."""
    n = (4, 3, 3)
    m = oracle.Mesh(2, n)
    u0 = inputs.density_wave_noisy(m.node_coords(), seed=9, noise=0.05)
    u1, _, _ = m.run(u0, 2, dt_fixed=3e-3)

    def shift(u):
        v = u.reshape(5, n[2], n[1], n[0], -1)
        return np.roll(v, 1, axis=3).reshape(u.shape)
    u2, _, _ = m.run(shift(u0), 2, dt_fixed=3e-3)
    assert np.array_equal(u2, shift(u1))


def test_axis_permutation_invariance():
    """Swapping the x and y axes (and the two momenta) commutes with the step."""
    n = 3
    m = oracle.Mesh(2, (n, n, n))
    N = m.N
    u0 = inputs.density_wave_noisy(m.node_coords(), seed=4, noise=0.05)
    u0[1] *= 1.3  # break the symmetry between the momenta
    u0[4] += 0.5 * ((1.3 ** 2 - 1) * (u0[1] / 1.3) ** 2) / u0[0]

    def swap(u):
        v = u.reshape(5, n, n, n, N, N, N)  # var, k, j, i, a2, a1, a0
        v = v.transpose(0, 1, 3, 2, 4, 6, 5)
        v = v[[0, 2, 1, 3, 4]]
        return np.ascontiguousarray(v).reshape(u.shape)
    u1, _, _ = m.run(u0, 2, dt_fixed=2e-3)
    u2, _, _ = m.run(swap(u0), 2, dt_fixed=2e-3)
    assert np.allclose(u2, swap(u1), atol=1e-14, rtol=0)


@pytest.mark.parametrize("p,axis", [(1, 0), (2, 1), (3, 2), (4, 0)])
def test_convergence_order_1d(p, axis):
    """Density wave along one axis: L2 error against the exact solution
    decreases with order ~p+1 (Sec. 2.1: same polynomial order in space and
    time)."""
    T = 0.05
    errs = []
    for n in (12, 24):
        nn = [1, 1, 1]
        nn[axis] = n
        m = oracle.Mesh(p, nn)
        wv = [0.0, 0.0, 0.0]
        wv[axis] = 1.0
        xyz = m.node_coords()
        u, _, rc = m.run(inputs.density_wave(xyz, wavevec=wv), 10 ** 6, t_end=T)
        assert rc == 0
        ue = inputs.density_wave(xyz, wavevec=wv, t=T)
        errs.append(math.sqrt(((u[0] - ue[0]) ** 2 * weights3(m.N)).sum() / m.nc))
    order = math.log2(errs[0] / errs[1])
    assert order > p + 0.8, (errs, order)


def test_convergence_order_3d():
    T = 0.03
    errs = []
    for n in (4, 8):
        m = oracle.Mesh(3, (n, n, n))
        xyz = m.node_coords()
        u, _, rc = m.run(inputs.density_wave(xyz), 10 ** 6, t_end=T)
        assert rc == 0
        ue = inputs.density_wave(xyz, t=T)
        errs.append(math.sqrt(((u[0] - ue[0]) ** 2 * weights3(m.N)).sum() / m.nc))
    assert math.log2(errs[0] / errs[1]) > 3.5, errs


# --------------------------------------------------------------------------
# adaptive meshes
# --------------------------------------------------------------------------

def amr_mesh(p, n=3, levels=2, radius=0.2):
    ref = inputs.sphere_refine_list((n, n, n), levels, radius=radius)
    return oracle.Mesh(p, (n, n, n), max_level=levels, refine=ref), ref


def test_amr_mesh_structure():
    m, ref = amr_mesh(2)
    cells = m.cells()
    kind, nbr = m.sides()
    # every refined cell became 27 children: count
    assert m.nc == 27 + 26 * ref.shape[0]
    # ordering by (level, k, j, i)
    key = cells[:, 0].astype(np.int64) * 10 ** 9 + cells[:, 3] * 10 ** 6 + cells[:, 2] * 10 ** 3 + cells[:, 1]
    assert np.all(np.diff(key) > 0)
    # the volume adds up to the box
    assert abs((1.0 / 27 / 27.0 ** cells[:, 0]).sum() - 1.0) < 1e-12
    # conforming sides are mutual, hanging faces point to coarser cells
    for c in range(m.nc):
        for s in range(6):
            if kind[c, s] == oracle.SIDE_CONFORMING:
                o = nbr[c, s]
                assert nbr[o, s ^ 1] == c and kind[o, s ^ 1] == oracle.SIDE_CONFORMING
            elif kind[c, s] == oracle.SIDE_FINE:
                assert cells[nbr[c, s], 0] < cells[c, 0]
    # level jumps of two exist (no 2:1 balancing)
    jumps = {int(cells[c, 0] - cells[nbr[c, s], 0]) for c in range(m.nc) for s in range(6)
             if kind[c, s] == oracle.SIDE_FINE}
    assert jumps == {1, 2}


def test_amr_sphere_counts_27():
    """Level populations of the 27^3 sphere-refined mesh with two levels."""
    ref = inputs.sphere_refine_list((27, 27, 27), 2, radius=0.25)
    lev0 = (ref[:, 0] == 0).sum()
    lev1 = (ref[:, 0] == 1).sum()
    assert 27 ** 3 - lev0 == 17868
    assert 27 * lev0 - lev1 == 10268
    assert 27 * lev1 == 1045899


@pytest.mark.parametrize("p", [1, 3])
def test_amr_free_stream(p):
    m, _ = amr_mesh(p)
    u0 = inputs.conserved(np.full((m.nc, m.N ** 3), 1.2), (0.3, -0.2, 0.1), 0.9)
    u, _, rc = m.run(u0, 2)
    assert rc == 0
    assert np.abs(u - u0).max() < 1e-14


@pytest.mark.parametrize("p", [1, 2])
def test_amr_conservation(p):
    m, _ = amr_mesh(p)
    u0 = inputs.blast_smooth(m.node_coords(), width=1.0 / 27, radius=0.2)
    t0 = totals(m, u0, (3, 3, 3))
    u, _, rc = m.run(u0, 2)
    assert rc == 0
    assert np.allclose(totals(m, u, (3, 3, 3)), t0, atol=1e-14, rtol=0)


def test_amr_refined_smooth_wave_converges():
    """A smooth wave crossing refinement boundaries still converges at high
    order when the base mesh is refined (hanging-face coupling is consistent)."""
    T = 0.02
    errs = []
    for n in (3, 6):
        ref = inputs.sphere_refine_list((n, n, n), 1, radius=0.2)
        m = oracle.Mesh(2, (n, n, n), max_level=1, refine=ref)
        xyz = m.node_coords()
        u, _, rc = m.run(inputs.density_wave(xyz), 10 ** 6, t_end=T)
        assert rc == 0
        ue = inputs.density_wave(xyz, t=T)
        lev = m.cells()[:, 0]
        vol = 27.0 ** (-lev.astype(float))
        errs.append(math.sqrt((((u[0] - ue[0]) ** 2 * weights3(m.N)).sum(axis=1) * vol).sum() / n ** 3))
    assert math.log2(errs[0] / errs[1]) > 2.0, errs


def test_sharp_blast_is_flagged_unphysical():
    """Without a limiter the nodal step profile of the blast overshoots to
    negative density in the face projections of the first step; the step
    reports it instead of producing NaNs."""
    m, _ = amr_mesh(2)
    u0 = inputs.blast(m.node_coords())
    dt, st = m.cfl(u0)
    assert st == 0
    _, tr = m.predictor(u0, dt)
    assert tr[:, 0, 0].min() < 0.0
    assert m.riemann(tr)[1] == 1
    assert m.run(u0, 1)[2] == 1


def test_sample_reproduces_polynomials():
    """Point values of the discrete solution are exact for data that is a
    polynomial of degree <= p along each axis inside every cell."""
    p, n = 3, (3, 2, 4)
    m = oracle.Mesh(p, n)
    xyz = m.node_coords()
    poly = lambda x, y, z: 1.0 + 0.3 * x ** 3 - 0.2 * x * y ** 2 + 0.1 * z ** 3 * y
    u = np.zeros((5, m.nc, m.N ** 3))
    u[0] = poly(*xyz)
    rng = np.random.Generator(np.random.PCG64(17))
    pts = rng.uniform(0.0, 1.0, size=(200, 3))
    pts[0] = (0.0, 0.0, 0.0)
    pts[1] = (1.0, 1.0, 1.0)
    assert np.allclose(m.sample(u, pts), poly(pts[:, 0], pts[:, 1], pts[:, 2]), atol=1e-13, rtol=0)


def test_run_sched_matches_fixed_dt():
    m = oracle.Mesh(2, (3, 3, 3))
    u0 = inputs.density_wave_noisy(m.node_coords(), seed=8, noise=0.02)
    a, _, _ = m.run(u0, 3, dt_fixed=2e-3)
    b, rc = m.run_sched(u0, [2e-3] * 3)
    assert rc == 0 and np.array_equal(a, b)
