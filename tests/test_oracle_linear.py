"""Pins of the oracle's linear (elastic-wave) variant with the
Cauchy-Kowalevski predictor (Sec. 2.4: a linear PDE is integrated in time
by Cauchy-Kowalevski; Sec. 6: the seismic benchmark).

What fixes it independently of the oracle's own code:
  * the flux matrices: eigenvalues +-c_p, +-c_s (twice), 0 (three times);
  * the truncated Taylor series in time is what p Picard iterations from the
    time-constant start produce (the Picard predictor is the Euler path's
    algorithm with the linear flux);
  * for data that vary along one axis only, the series ends and the time
    average is exact: closed form for a P-wave profile g(x - c_p t);
  * plane P- and S-waves travel at c_p and c_s in +x: the discrete solution
    converges to the exact one at about order p + 1;
  * constant states are preserved; the elastic energy does not grow
    (Rusanov is dissipative)."""
import numpy as np
import pytest

import oracle

RNG = np.random.Generator(np.random.PCG64(11))


def materials(nc, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    return np.stack([r.uniform(1.0, 3.0, nc), r.uniform(1.0, 2.0, nc), r.uniform(0.5, 1.5, nc)])


def test_flux_matrix_eigenvalues():
    for mat in ((2.0, 1.5, 1.0), (2.7, 3.0, 0.3), (1.0, 0.0, 1.0)):
        rho, lam, mu = mat
        cp, cs = np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho)
        want = np.sort([-cp, -cs, -cs, 0, 0, 0, cs, cs, cp])
        for d in range(3):
            ev = np.sort(np.linalg.eigvals(oracle.lin_flux_matrix(mat, d)).real)
            assert np.allclose(ev, want, atol=1e-12)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5])
def test_ck_is_p_picard_iterations(p):
    m = oracle.Mesh(p, (3, 2, 2))
    N = p + 1
    mat = materials(m.nc, 20 + p)
    u = RNG.standard_normal((9, m.nc, N ** 3))
    dt = m.lin_cfl(mat)
    a, ta = m.lin_predictor(mat, u, dt, ck=True)
    b, tb = m.lin_predictor(mat, u, dt, ck=False, npic=p)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
    assert np.abs(ta - tb).max() <= 1e-13 * np.abs(ta).max()
    if p > 0:  # one more iteration brings in higher time derivatives: a different predictor
        c, _ = m.lin_predictor(mat, u, dt, ck=False, npic=p + 1)
        assert np.abs(a - c).max() > 1e-8


def pwave(xyz, mat, t, k=1):
    rho, lam, mu = mat
    cp = np.sqrt((lam + 2 * mu) / rho)
    f = np.sin(2 * np.pi * k * (xyz[0] - cp * t))
    q = np.zeros((9,) + xyz[0].shape)
    q[6] = f
    q[0] = -(lam + 2 * mu) / cp * f
    q[1] = q[2] = -lam / cp * f
    return q


def swave(xyz, mat, t):
    rho, lam, mu = mat
    cs = np.sqrt(mu / rho)
    f = np.sin(2 * np.pi * (xyz[0] - cs * t))
    q = np.zeros((9,) + xyz[0].shape)
    q[7] = f                 # v_y
    q[3] = -mu / cs * f      # s_xy
    return q


@pytest.mark.parametrize("p", [1, 2, 3])
def test_time_average_exact_for_one_axis_polynomial(p):
    """g(x) = x^p along x only: the Taylor series ends, and the predictor's
    face value of the time average at the +x face equals
    (1/dt) int_0^dt r g(x_R - c_p t) dt in closed form."""
    mat0 = (2.0, 1.5, 1.0)
    n = (3, 1, 1)
    m = oracle.Mesh(p, n)
    xyz = m.node_coords()
    mat = np.array(mat0)[:, None] * np.ones((3, m.nc))
    rho, lam, mu = mat0
    cp = np.sqrt((lam + 2 * mu) / rho)
    r = np.zeros(9)
    r[6], r[0], r[1], r[2] = 1.0, -(lam + 2 * mu) / cp, -lam / cp, -lam / cp
    u = r[:, None, None] * (xyz[0] ** p)[None]
    dt = m.lin_cfl(mat)
    _, tr = m.lin_predictor(mat, u, dt)
    cells = m.cells()
    for c in range(m.nc):
        xR = (cells[c, 1] + 1) / n[0]
        avg = (xR ** (p + 1) - (xR - cp * dt) ** (p + 1)) / ((p + 1) * cp * dt)
        got = tr[1, 0, :, c, :]  # side +x, state, [9, N^2]
        assert np.allclose(got, r[:, None] * avg, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("wave", ["p", "s"])
def test_plane_waves_converge(wave):
    mat0 = (2.0, 1.5, 1.0)
    T = 0.05
    for p, min_order in ((2, 2.7), (3, 3.5)):
        errs = []
        for n in (8, 16):
            m = oracle.Mesh(p, (n, 1, 1))
            xyz = m.node_coords()
            mat = np.array(mat0)[:, None] * np.ones((3, m.nc))
            exact = pwave if wave == "p" else swave
            dt = m.lin_cfl(mat)
            k = int(np.ceil(T / dt))
            u, _ = m.lin_run(mat, exact(xyz, mat0, 0.0), k, dt_fixed=T / k)
            errs.append(np.abs(u - exact(xyz, mat0, T)).max())
        order = np.log2(errs[0] / errs[1])
        assert errs[1] < 2e-2 and order > min_order, (wave, p, errs, order)


def test_constant_state_and_energy():
    p, n = 3, (4, 3, 3)
    m = oracle.Mesh(p, n)
    mat = np.array([2.0, 1.5, 1.0])[:, None] * np.ones((3, m.nc))
    const = RNG.standard_normal(9)[:, None, None] * np.ones((9, m.nc, (p + 1) ** 3))
    u, _ = m.lin_run(mat, const, 3)
    assert np.abs(u - const).max() <= 1e-13 * np.abs(const).max()
    # a smooth random field: energy never grows from step to step
    xyz = m.node_coords()
    u = np.stack([np.sin(2 * np.pi * (xyz[0] + k * xyz[1] + 0.5 * k * xyz[2]) + k) for k in range(9)])
    e = [m.lin_energy(mat, u)]
    for _ in range(4):
        u, _ = m.lin_run(mat, u, 1)
        e.append(m.lin_energy(mat, u))
    assert all(b <= a * (1 + 1e-14) for a, b in zip(e, e[1:])) and e[-1] < e[0]
