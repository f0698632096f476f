"""Dynamic adaptivity at the benchmark's size (27^3 base cells, two levels
of refinement in the sphere, p = 4, FP32 form, 1,074,035 cells): one
adaptation of the smoothed blast after two steps.

The plan equals the oracle's rule applied to the library's own indicator
values; mass is conserved through the transfer; and sampled new cells
equal the oracle's transfer computed on their own box alone.  A new cell's
data depend only on the old leaves covering it, so the oracle rebuilds that
box as a one-cell mesh with the same sub-refinement (or takes the one old
leaf that contains it) and transfers it."""
import numpy as np
import pytest

import oracle
import paper_1806_07984_amd as A
from paper_1806_07984_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def totals(u, cells, N, n0):
    w = oracle.gauss_legendre(N)[1]
    W = torch.from_numpy(np.einsum("i,j,k->kji", w, w, w).reshape(-1)).cuda()
    vol = torch.from_numpy((1.0 / n0 ** 3) / 27.0 ** cells[:, 0].astype(np.float64)).cuda()
    return ((u.view(5, -1, N ** 3) * W).sum(dim=2) * vol).sum(dim=1).cpu().numpy()


def test_adaptation_full_size():
    n0, p, L = 27, 4, 2
    N = p + 1
    n = (n0, n0, n0)
    ref = inputs.sphere_refine_list(n, L, radius=0.25)
    gm = A.Mesh(A.instance(p, n, max_level=L, refine=ref), "fp32")
    xyz = gm.node_coords().cpu().numpy().reshape(3, -1)
    u = torch.from_numpy(inputs.blast_smooth(xyz, width=1.0 / (n0 * 9)).reshape(-1)).cuda()
    del xyz
    ws = gm.empty_workspace()
    gm.step(u, 2, ws)
    torch.cuda.synchronize()
    gm.status()
    tr, tc = 0.05, 0.005
    cells_old = gm.cells()
    eta = gm.indicator(u).cpu().numpy()
    new, u_new = A.adapt(gm, u, tr, tc)
    torch.cuda.synchronize()
    cells_new = new.cells()
    rows_new = new.descs[0]["refine"]
    print(f"[adapt full size] cells {len(cells_old)} -> {len(cells_new)}", flush=True)
    assert np.array_equal(rows_new, oracle.adapt_plan(cells_old, ref, eta, tr, tc, L))
    t0, t1 = totals(u, cells_old, N, n0), totals(u_new, cells_new, N, n0)
    assert np.allclose(t1[[0, 4]], t0[[0, 4]], rtol=1e-12, atol=0)
    assert np.abs(t1[1:4] - t0[1:4]).max() <= 1e-12

    old_index = {tuple(c): i for i, c in enumerate(cells_old.tolist())}
    ref_rows = np.asarray(ref)
    uo = u.view(5, -1, N ** 3)
    un = u_new.view(5, -1, N ** 3)
    rng = np.random.Generator(np.random.PCG64(3))
    # sample new cells that are not plain copies: coarsened and refined ones
    moved = [i for i, c in enumerate(cells_new.tolist()) if tuple(c) not in old_index]
    assert len(moved) > 100
    for c in np.sort(rng.choice(moved, size=16, replace=False)):
        lt, I, J, K = (int(x) for x in cells_new[c])
        h = 1.0 / (n0 * 3 ** lt)
        # the old leaf containing the new cell, if any
        src = None
        for l2 in range(lt - 1, -1, -1):
            r = 3 ** (lt - l2)
            key = (l2, I // r, J // r, K // r)
            if key in old_index:
                src = (l2, old_index[key])
                break
        if src is not None:
            l2, s = src
            r = 3 ** (lt - l2)
            H = 1.0 / (n0 * 3 ** l2)
            # one old cell; the new cell as the matching leaf of a chain of refinements
            om_old = oracle.Mesh(p, (1, 1, 1), hi=(H, H, H))
            chain, pos = [], (I - r * (I // r), J - r * (J // r), K - r * (K // r))
            for lev in range(lt - l2):
                f = 3 ** (lt - l2 - lev)
                chain.append([lev, pos[0] // f, pos[1] // f, pos[2] // f])
            om_new = oracle.Mesh(p, (1, 1, 1), hi=(H, H, H), max_level=lt - l2, refine=chain)
            want_all = om_old.transfer_to(uo[:, s:s + 1, :].double().cpu().numpy(), om_new)
            target = (lt - l2,) + pos
        else:
            # finer old leaves inside the new cell: their refine rows relative to it
            rel = []
            for (l, i, j, k) in ref_rows.tolist():
                if l < lt:
                    continue
                r = 3 ** (l - lt)
                if (i // r, j // r, k // r) == (I, J, K):
                    rel.append([l - lt, i - r * I, j - r * J, k - r * K])
            rel = np.array(sorted(rel, key=lambda q: (q[0], q[3], q[2], q[1])), dtype=np.int32).reshape(-1, 4)
            om_old = oracle.Mesh(p, (1, 1, 1), hi=(h, h, h), max_level=L - lt, refine=rel)
            sub = om_old.cells()
            idx = [old_index[(lt + q[0], q[1] + I * 3 ** q[0], q[2] + J * 3 ** q[0], q[3] + K * 3 ** q[0])]
                   for q in sub.tolist()]
            uo_sub = uo[:, torch.tensor(idx, device="cuda"), :].double().cpu().numpy()
            om_new = oracle.Mesh(p, (1, 1, 1), hi=(h, h, h))
            want_all = om_old.transfer_to(uo_sub, om_new)
            target = (0, 0, 0, 0)
        tcells = om_new.cells().tolist()
        want = want_all[:, tcells.index(list(target)), :]
        got = un[:, c, :].double().cpu().numpy()
        err = np.abs(got - want).max() / np.abs(want).max()
        assert err <= 1e-12, (c, src is not None, err)
    new.close()
    gm.close()
