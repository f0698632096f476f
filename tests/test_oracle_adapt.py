"""Pins of the oracle's dynamic-adaptivity pieces (Sec. 2.3, dynamic
adaptivity): the refinement indicator, the volumetric transfer between two
meshes (refinement interpolates volumetric data, coarsening merges 27 cells)
and the adaptation rule.

What fixes them independently of the oracle's own code:
  * indicator of a linear density = dx_d * |gradient| (closed form);
  * the transfer of a polynomial of degree <= p onto a finer mesh is that
    polynomial at the new nodes (the fine space contains it);
  * projecting back onto the original mesh returns the original data (the
    L2 projection onto a space that contains the data is the identity);
  * coarsening conserves every integral (constants lie in the coarse space),
    for arbitrary data;
  * copy on identical meshes; refusal when a target cell is only partly
    covered;
  * the plan on hand-made cases."""
import numpy as np
import pytest

import oracle


def poly(xyz, deg, seed):
    """A random polynomial of total degree <= deg in x, y, z (5 variables)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y, z = xyz
    out = np.zeros((5,) + x.shape)
    for v in range(5):
        for i in range(deg + 1):
            for j in range(deg + 1 - i):
                for k in range(deg + 1 - i - j):
                    out[v] += rng.uniform(-1, 1) * x ** i * y ** j * z ** k
    return out


def refine_rows(n, count, seed, level=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.choice(n ** 3 * 27 ** level, size=count, replace=False)
    e = n * 3 ** level
    return np.array([[level, p % e, (p // e) % e, p // (e * e)] for p in sorted(pick)], dtype=np.int32)


def test_indicator_of_linear_density():
    n, p = (3, 4, 2), 3
    m = oracle.Mesh(p, n, hi=(1.0, 2.0, 0.5))
    xyz = m.node_coords()
    g = np.array([0.7, -1.3, 2.1])
    u = np.zeros((5, m.nc, m.N ** 3))
    u[0] = 1.0 + g[0] * xyz[0] + g[1] * xyz[1] + g[2] * xyz[2]
    dx = np.array([1.0 / 3, 2.0 / 4, 0.5 / 2])
    eta = m.indicator(u)
    assert np.allclose(eta, np.max(np.abs(g) * dx), rtol=1e-12, atol=0)
    # only the density enters
    u[1:] = np.random.Generator(np.random.PCG64(1)).standard_normal(u[1:].shape)
    assert np.allclose(m.indicator(u), eta, rtol=1e-14, atol=0)


@pytest.mark.parametrize("p", [1, 3, 4])
def test_refinement_is_exact_and_projection_returns(p):
    n = (3, 3, 3)
    coarse = oracle.Mesh(p, n, max_level=2)
    rows1 = refine_rows(3, 5, seed=p)
    fine = oracle.Mesh(p, n, max_level=2, refine=rows1)
    u_c = poly(coarse.node_coords(), p, seed=10 + p)
    u_f = coarse.transfer_to(u_c, fine)
    assert np.allclose(u_f, poly(fine.node_coords(), p, seed=10 + p), rtol=0, atol=1e-12)
    back = fine.transfer_to(u_f, coarse)
    assert np.allclose(back, u_c, rtol=0, atol=1e-12)
    # two levels at once: a level-0 cell straight to level-2 cells, and back
    rows2 = np.concatenate([rows1[:1], [[1, 3 * rows1[0, 1], 3 * rows1[0, 2], 3 * rows1[0, 3]]]]).astype(np.int32)
    finer = oracle.Mesh(p, n, max_level=2, refine=rows2)
    u_ff = coarse.transfer_to(u_c, finer)
    assert np.allclose(u_ff, poly(finer.node_coords(), p, seed=10 + p), rtol=0, atol=1e-12)
    assert np.allclose(finer.transfer_to(u_ff, coarse), u_c, rtol=0, atol=1e-12)


@pytest.mark.parametrize("p", [2, 3])
def test_coarsening_conserves_integrals(p):
    n = (3, 2, 3)
    rows = refine_rows(3, 4, seed=20 + p)
    rows = rows[(rows[:, 2] < 2)]
    fine = oracle.Mesh(p, n, max_level=1, refine=rows)
    coarse = oracle.Mesh(p, n, max_level=1)
    rng = np.random.Generator(np.random.PCG64(30 + p))
    u = 1.0 + rng.uniform(-0.5, 0.5, size=(5, fine.nc, fine.N ** 3))
    t0 = fine.integral(u)
    t1 = coarse.integral(fine.transfer_to(u, coarse))
    assert np.allclose(t1, t0, rtol=1e-13, atol=0)
    # refinement conserves them too (exact evaluation of the coarse polynomial)
    uc = fine.transfer_to(u, coarse)
    assert np.allclose(fine.integral(coarse.transfer_to(uc, fine)), coarse.integral(uc), rtol=1e-13, atol=0)


def test_copy_and_partial_cover():
    m = oracle.Mesh(2, (2, 2, 2), max_level=1, refine=[[0, 1, 0, 1]])
    u = np.random.Generator(np.random.PCG64(3)).standard_normal((5, m.nc, 27))
    assert np.array_equal(m.transfer_to(u, m), u)
    # a target mesh of a different base grid is not covered cell by cell
    other = oracle.Mesh(2, (3, 2, 2))
    with pytest.raises(AssertionError):
        m.transfer_to(u, other)


def test_plan_rule():
    n, L = 3, 2
    rows = np.array([[0, 1, 1, 1]], dtype=np.int32)
    m = oracle.Mesh(1, (n, n, n), max_level=L, refine=rows)
    cells = m.cells()
    eta = np.full(m.nc, 0.5)
    # nothing crosses the thresholds: same mesh
    assert np.array_equal(oracle.adapt_plan(cells, rows, eta, 1.0, 0.1, L), rows)
    # one level-0 leaf above the threshold is split
    i0 = int(np.nonzero((cells[:, 0] == 0) & (cells[:, 1] == 0) & (cells[:, 2] == 0) & (cells[:, 3] == 0))[0][0])
    e2 = eta.copy()
    e2[i0] = 2.0
    assert np.array_equal(oracle.adapt_plan(cells, rows, e2, 1.0, 0.1, L), [[0, 0, 0, 0], [0, 1, 1, 1]])
    # all 27 children of the refined cell below the coarsening threshold: merged
    kids = cells[:, 0] == 1
    e3 = eta.copy()
    e3[kids] = 0.01
    assert oracle.adapt_plan(cells, rows, e3, 1.0, 0.1, L).shape == (0, 4)
    # one child above it: kept
    e3[np.nonzero(kids)[0][5]] = 0.2
    assert np.array_equal(oracle.adapt_plan(cells, rows, e3, 1.0, 0.1, L), rows)
    # a child above the refinement threshold is split (level 1 < max_level)
    e4 = eta.copy()
    k7 = np.nonzero(kids)[0][7]
    e4[k7] = 3.0
    out = oracle.adapt_plan(cells, rows, e4, 1.0, 0.1, L)
    assert out.tolist() == [[0, 1, 1, 1], [1] + cells[k7, 1:].tolist()]
    # nothing is split at max_level
    m2 = oracle.Mesh(1, (n, n, n), max_level=1, refine=rows)
    c2 = m2.cells()
    e5 = np.full(m2.nc, 5.0)
    out = oracle.adapt_plan(c2, rows, e5, 1.0, 0.1, 1)
    assert all(r[0] == 0 for r in out) and len(out) == 27
