"""Pins of the oracle's Rusanov face speed and of its tangent-linear model
and adjoint of one step at a fixed dt.

Paper: Sec. 2.4 (the Riemann solver needs the flux and one estimate of the
largest eigenvalue per face), Eq. 4 (one step), Sec. 2.3 (hanging faces:
interpolation and its weighted transpose).  The tangent is pinned by central
differences of the oracle's own forward step and, at p = 0, by automatic
differentiation of an independent textbook finite-volume step; the adjoint by
the dot-product identity <J v, w> = <v, J^T w>."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1806_07984_amd import inputs

G = 1.4


def amr_mesh(p, n=3, levels=2, radius=0.2):
    ref = inputs.sphere_refine_list((n, n, n), levels, radius=radius)
    return oracle.Mesh(p, (n, n, n), max_level=levels, refine=ref)


def one_face_traces(QL, FL, QR, FR, d, N2):
    """Traces of a 1x1x1 periodic mesh whose only face normal to d has the
    left state (QL, FL) on the cell's plus side and the right state (QR, FR)
    on its minus side; the faces of the other axes see one state twice."""
    tr = np.zeros((6, 2, 5, 1, N2))
    rest = inputs.conserved(np.ones(N2), (0.0, 0.0, 0.0), 1.0)
    for s in range(6):
        dd = s // 2
        if dd == d:
            continue
        tr[s, 0, :, 0] = rest
        tr[s, 1, :, 0] = 0.0
        tr[s, 1, 1 + dd, 0] = 1.0  # pressure in the normal momentum flux
    tr[2 * d + 1, 0, :, 0], tr[2 * d + 1, 1, :, 0] = QL, FL
    tr[2 * d, 0, :, 0], tr[2 * d, 1, :, 0] = QR, FR
    return tr


# --------------------------------------------------------------------------
# Rusanov: one speed per face (Sec. 2.4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [0, 1, 2])
def test_rusanov_one_speed_per_face_hand_case(d):
    """States at rest, rho = 1: c = sqrt(gamma p).  Left pressure 1/gamma
    (c = 1) except node 2 with 4/gamma (c = 2), right pressure 0.25/gamma
    (c = 1/2).  The face speed is 2 at every node; a per-node speed would be
    1 away from node 2 and halve the energy diffusion there."""
    p = 1
    m = oracle.Mesh(p, (1, 1, 1))
    N2 = m.N ** 2
    pl = np.full(N2, 1.0 / G)
    pl[2] = 4.0 / G
    pr = np.full(N2, 0.25 / G)
    QL = inputs.conserved(np.ones(N2), (0.0, 0.0, 0.0), pl)
    QR = inputs.conserved(np.ones(N2), (0.0, 0.0, 0.0), pr)
    FL = np.zeros((5, N2))
    FR = np.zeros((5, N2))
    FL[1 + d] = pl  # flux of a state at rest: pressure in the normal momentum
    FR[1 + d] = pr
    fs, bad = m.riemann(one_face_traces(QL, FL, QR, FR, d, N2))
    assert bad == 0
    # by hand: F* = (F_L + F_R)/2 - s (Q_R - Q_L)/2 with s = 2 on every node;
    # Q_R - Q_L is (p_R - p_L)/(gamma - 1) in the energy only
    want = np.zeros((5, N2))
    want[1 + d] = 0.5 * (pl + pr)
    want[4] = (pl - pr) / (G - 1.0)  # = -(2/2)(p_R - p_L)/(gamma - 1)
    assert np.allclose(want[4, [0, 1, 3]], 0.75 / (G * 0.4), rtol=0, atol=1e-15)
    assert abs(want[4, 2] - 3.75 / (G * 0.4)) < 1e-14
    for s in (2 * d, 2 * d + 1):
        assert np.allclose(fs[s, :, 0], want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_rusanov_mirror_antisymmetry(d):
    """Reflecting the face normal swaps the sides and negates the normal
    momentum (operator M); the normal flux of a reflected state is -M f, so
    F*(M Q_R, -M F_R; M Q_L, -M F_L) = -M F*(Q_L, F_L; Q_R, F_R), exactly."""
    p = 3
    m = oracle.Mesh(p, (1, 1, 1))
    N2 = m.N ** 2
    rng = np.random.Generator(np.random.PCG64(40 + d))
    def state():
        return inputs.conserved(rng.uniform(0.5, 1.5, N2), [rng.uniform(-0.7, 0.7, N2) for _ in range(3)],
                                rng.uniform(0.5, 1.5, N2))
    QL, QR = state(), state()
    FL, FR = rng.standard_normal((5, N2)), rng.standard_normal((5, N2))
    M = np.ones(5)
    M[1 + d] = -1.0
    fs, bad = m.riemann(one_face_traces(QL, FL, QR, FR, d, N2))
    fm, bad2 = m.riemann(one_face_traces(M[:, None] * QR, -M[:, None] * FR, M[:, None] * QL, -M[:, None] * FL, d, N2))
    assert bad == 0 and bad2 == 0
    assert np.array_equal(fm[2 * d + 1], -M[:, None, None] * fs[2 * d + 1])


def test_rusanov_face_speed_from_both_sides():
    """The speed is taken over both sides: moving the fast node from the left
    state to the right state leaves F* unchanged where Q_L = Q_R."""
    p = 1
    m = oracle.Mesh(p, (1, 1, 1))
    N2 = m.N ** 2
    base = np.full(N2, 1.0 / G)
    fast = base.copy()
    fast[3] = 9.0 / G  # c = 3
    Z = np.zeros((5, N2))
    QA = inputs.conserved(np.ones(N2), (0.0, 0.0, 0.0), fast)
    QB = inputs.conserved(np.ones(N2), (0.0, 0.0, 0.0), base)
    f1, _ = m.riemann(one_face_traces(QA, Z, QB, Z, 0, N2))
    f2, _ = m.riemann(one_face_traces(QB, Z, QA, Z, 0, N2))
    # only node 3 has a jump; the speed 3 enters there with opposite signs
    jump = (9.0 - 1.0) / G / (G - 1.0)
    assert abs(f1[1, 4, 0, 3] - 1.5 * jump) < 1e-13
    assert abs(f2[1, 4, 0, 3] + 1.5 * jump) < 1e-13
    assert np.all(f1[1, 4, 0, :3] == 0.0) and np.all(f2[1, 4, 0, :3] == 0.0)


# --------------------------------------------------------------------------
# tangent-linear model of one step
# --------------------------------------------------------------------------

def _setup(p, amr, seed=5):
    m = amr_mesh(p) if amr else oracle.Mesh(p, (3, 3, 3))
    u0 = inputs.density_wave_noisy(m.node_coords(), seed=seed, noise=0.02)
    dt, st = m.cfl(u0)
    assert st == 0
    return m, u0, dt


def test_tlm_keeps_the_forward_step():
    m, u0, dt = _setup(2, True)
    v = inputs.directions(u0.shape, 1, seed=9)[0]
    u1, _, rc = m.step_tlm(u0, dt, v)
    ref, rc2 = m.run_sched(u0, [dt])
    assert rc == 0 and rc2 == 0 and np.array_equal(u1, ref)


@pytest.mark.parametrize("p,amr,epsr", [(0, False, 1e-6), (1, False, 1e-6), (2, False, 1e-6), (3, False, 1e-6),
                                        (1, True, 1e-7), (2, True, 1e-7)])
def test_tlm_matches_central_differences(p, amr, epsr):
    """(S(u + e v) - S(u - e v)) / 2e against the tangent.  The noisy state
    keeps every face's fastest node well ahead of the next one, so no
    maximiser switches inside the difference interval; the agreement is then
    limited by rounding (e = epsr |u| / |v|)."""
    m, u0, dt = _setup(p, amr)
    for k, v in enumerate(inputs.directions(u0.shape, 2, seed=11 + p)):
        _, jv, rc = m.step_tlm(u0, dt, v)
        assert rc == 0
        eps = epsr * np.linalg.norm(u0) / np.linalg.norm(v)
        up, _ = m.run_sched(u0 + eps * v, [dt])
        um, _ = m.run_sched(u0 - eps * v, [dt])
        fd = (up - um) / (2 * eps)
        err = np.linalg.norm(fd - jv) / np.linalg.norm(jv)
        assert err < 1e-8, (k, err)


def test_tlm_several_directions_at_once():
    m, u0, dt = _setup(2, True)
    V = inputs.directions(u0.shape, 3, seed=21)
    _, JV, rc = m.step_tlm(u0, dt, V)
    assert rc == 0
    for k in range(3):
        _, jv, _ = m.step_tlm(u0, dt, V[k])
        assert np.array_equal(jv, JV[k])


def _torch_fv_step(u, n, dt):
    """First-order finite volumes with the Rusanov flux on a periodic grid,
    u[5, nz, ny, nx] (torch, float64): the textbook scheme p = 0 reduces to."""
    def flux(q, d):
        rho, m = q[0], q[1:4]
        p = (G - 1) * (q[4] - 0.5 * (m ** 2).sum(0) / rho)
        v = m[d] / rho
        f = torch.stack([m[d], v * m[0], v * m[1], v * m[2], v * (q[4] + p)])
        return f + torch.nn.functional.one_hot(torch.tensor(1 + d), 5).to(q)[:, None, None, None] * p
    def speed(q, d):
        rho, m = q[0], q[1:4]
        p = (G - 1) * (q[4] - 0.5 * (m ** 2).sum(0) / rho)
        return torch.abs(m[d] / rho) + torch.sqrt(G * p / rho)
    out = u.clone()
    for d in range(3):
        ax = 3 - d
        uR = torch.roll(u, -1, dims=ax)
        s = torch.maximum(speed(u, d), speed(uR, d))
        F = 0.5 * (flux(u, d) + flux(uR, d)) - 0.5 * s * (uR - u)
        out = out - dt * n[d] * (F - torch.roll(F, 1, dims=ax))
    return out


def test_tlm_p0_equals_autodiff_of_textbook_fv():
    """At p = 0 the step is the textbook Rusanov finite-volume scheme; its
    derivative by torch's forward-mode autodiff matches the oracle's tangent."""
    n = (5, 4, 3)
    m = oracle.Mesh(0, n)
    rng = np.random.Generator(np.random.PCG64(71))
    u = inputs.conserved(rng.uniform(0.7, 1.3, m.nc), [rng.uniform(-0.5, 0.5, m.nc) for _ in range(3)],
                         rng.uniform(0.6, 1.4, m.nc))[:, :, None]
    v = rng.standard_normal(u.shape)
    dt = 1e-2
    _, jv, rc = m.step_tlm(u, dt, v)
    assert rc == 0
    shp = (5, n[2], n[1], n[0])
    ut = torch.from_numpy(u[:, :, 0].reshape(shp).copy())
    vt = torch.from_numpy(v[:, :, 0].reshape(shp).copy())
    _, jt = torch.func.jvp(lambda x: _torch_fv_step(x, n, dt), (ut,), (vt,))
    assert np.allclose(jv[:, :, 0], jt.numpy().reshape(5, -1), rtol=0, atol=1e-13)


# --------------------------------------------------------------------------
# adjoint of one step
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p,amr", [(0, False), (1, False), (3, False), (1, True), (2, True), (3, True)])
def test_adjoint_dot_product(p, amr):
    """<J v, w> = <v, J^T w> between the tangent and the adjoint."""
    m, u0, dt = _setup(p, amr, seed=13)
    V = inputs.directions(u0.shape, 3, seed=31)
    W = inputs.directions(u0.shape, 3, seed=32)
    _, JV, rc = m.step_tlm(u0, dt, V)
    assert rc == 0
    for k in range(3):
        jtw, rc = m.step_adj(u0, dt, W[k])
        assert rc == 0
        a = float((JV[k] * W[k]).sum())
        b = float((V[k] * jtw).sum())
        assert abs(a - b) <= 1e-13 * max(abs(a), np.linalg.norm(JV[k]) * np.linalg.norm(W[k]) * 1e-2), (a, b)


def test_sample_adjoint_dot_product():
    m = oracle.Mesh(3, (3, 2, 4))
    rng = np.random.Generator(np.random.PCG64(5))
    u = rng.standard_normal((5, m.nc, m.N ** 3))
    pts = rng.uniform(0.0, 1.0, size=(50, 3))
    w = rng.standard_normal(50)
    a = float(m.sample(u, pts) @ w)
    b = float((u * m.sample_adj(pts, w)).sum())
    assert abs(a - b) < 1e-13 * abs(a)


def test_loss_gradient_chain():
    """Gradient of J = 1/2 sum_s (rho_h(x_s, T) - rho*_s)^2 after 3 steps by
    the adjoint chain, against the tangent chain and central differences of
    the forward run (the config-5 loss, on a small mesh)."""
    m = oracle.Mesh(2, (4, 4, 4))
    u0 = inputs.density_wave_noisy(m.node_coords(), seed=7, noise=0.01)
    pts = inputs.sample_points(40, seed=1)
    tgt = inputs.sample_targets(40, seed=2)
    _, dts, rc = m.run(u0, 3)
    assert rc == 0
    states = [u0]
    for dt in dts:
        states.append(m.run_sched(states[-1], [dt])[0])
    r = m.sample(states[-1], pts) - tgt
    g = m.sample_adj(pts, r)
    for n in range(len(dts) - 1, -1, -1):
        g, rc = m.step_adj(states[n], dts[n], g)
        assert rc == 0
    loss = lambda u: 0.5 * float(((m.sample(m.run_sched(u, dts)[0], pts) - tgt) ** 2).sum())
    for v in inputs.directions(u0.shape, 2, seed=44):
        x, dv = u0, v
        for dt in dts:
            x, dv, rc = m.step_tlm(x, dt, dv)
        dj = float(r @ m.sample(dv, pts))
        assert abs(dj - float((g * v).sum())) < 1e-12 * abs(dj)
        eps = 1e-6 * np.linalg.norm(u0) / np.linalg.norm(v)
        fd = (loss(u0 + eps * v) - loss(u0 - eps * v)) / (2 * eps)
        assert abs(fd - dj) < 1e-6 * abs(dj), (fd, dj)


# --------------------------------------------------------------------------
# convergence across a level jump of two
# --------------------------------------------------------------------------

def box_refine(n):
    """Level 0: the base cells of the middle third [1/3, 2/3]^3; level 1: the
    children of those on the boundary layer of that box.  Level-2 cells then
    touch level-0 cells (jumps of 2) and level-1 cells (jumps of 1)."""
    lo, hi = n // 3, 2 * n // 3
    rows = [(0, i, j, k) for k in range(lo, hi) for j in range(lo, hi) for i in range(lo, hi)]
    L, H = 3 * lo, 3 * hi
    for k in range(L, H):
        for j in range(L, H):
            for i in range(L, H):
                if min(i - L, j - L, k - L, H - 1 - i, H - 1 - j, H - 1 - k) == 0:
                    rows.append((1, i, j, k))
    return np.array(rows, dtype=np.int32)


def test_two_level_jump_converges():
    """A density wave crossing faces with level jumps of 1 and 2 converges at
    about order p + 1 (p = 3) when the base mesh is refined: the r = 9
    interpolation and restriction are consistent."""
    p, T = 3, 0.01
    errs = []
    for n in (3, 6):
        m = oracle.Mesh(p, (n, n, n), max_level=2, refine=box_refine(n))
        kind, nbr = m.sides()
        cells = m.cells()
        jumps = {int(cells[c, 0] - cells[nbr[c, s], 0]) for c in range(m.nc) for s in range(6)
                 if kind[c, s] == oracle.SIDE_FINE}
        assert jumps == {1, 2}
        xyz = m.node_coords()
        u, _, rc = m.run(inputs.density_wave(xyz), 10 ** 6, t_end=T)
        assert rc == 0
        ue = inputs.density_wave(xyz, t=T)
        w = oracle.gauss_legendre(m.N)[1]
        W = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
        vol = 27.0 ** (-cells[:, 0].astype(float)) / n ** 3
        errs.append(math.sqrt(((((u[0] - ue[0]) ** 2) * W).sum(axis=1) * vol).sum()))
    assert math.log2(errs[0] / errs[1]) > p + 0.8, errs
