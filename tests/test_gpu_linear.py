"""The linear variant (elastic waves, Cauchy-Kowalevski predictor) on the GPU
against the oracle: the predictor for orders 0-6 on random data with a
different material in every cell, whole runs, and at the benchmark's size
(81^3, p = 3) a plane P-wave against its exact solution and a constant state
kept exactly.  FP64 throughout."""
import numpy as np
import pytest

import oracle
import paper_1806_07984_amd as A

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a, dtype=np.float64)).reshape(-1)).cuda()


def materials(nc, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    return np.stack([r.uniform(1.0, 3.0, nc), r.uniform(1.0, 2.0, nc), r.uniform(0.5, 1.5, nc)])


def rel(got, want):
    return np.abs(got - want).max() / np.abs(want).max()


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5, 6])
def test_predictor_matches_oracle(p):
    n = (3, 4, 2)
    N = p + 1
    om = oracle.Mesh(p, n)
    mat = materials(om.nc, 30 + p)
    u = np.random.Generator(np.random.PCG64(p)).standard_normal((9, om.nc, N ** 3))
    print(f"[linear predictor] p={p}", flush=True)
    lm = A.LinMesh(p, n)
    md = dev(mat)
    dt = lm.dt(md)
    dt_o = om.lin_cfl(mat)
    assert abs(dt.item() - dt_o) <= 1e-14 * dt_o
    us, tr = lm.predictor(md, dev(u), dt)
    us_o, tr_o = om.lin_predictor(mat, u, dt.item())
    assert rel(us.cpu().numpy().reshape(us_o.shape), us_o) <= 1e-12
    assert rel(tr.cpu().numpy().reshape(tr_o.shape), tr_o) <= 1e-12
    lm.close()


@pytest.mark.parametrize("p", [1, 3, 5])
def test_run_matches_oracle(p):
    n = (5, 4, 3)
    N = p + 1
    om = oracle.Mesh(p, n)
    mat = materials(om.nc, 40 + p)
    xyz = om.node_coords()
    u0 = np.stack([np.sin(2 * np.pi * (xyz[0] + k * xyz[1] - 0.5 * k * xyz[2]) + k) for k in range(9)])
    print(f"[linear run] p={p}", flush=True)
    want, dt_o = om.lin_run(mat, u0, 5)
    lm = A.LinMesh(p, n)
    u = dev(u0)
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    lm.step(dev(mat), u, 5, lm.empty_workspace(), dt_out=dt)
    torch.cuda.synchronize()
    assert abs(dt.item() - dt_o) <= 1e-14 * dt_o
    assert rel(u.cpu().numpy().reshape(want.shape), want) <= 1e-12
    lm.close()


@pytest.mark.parametrize("n", [(5, 4, 3), (1, 4, 2), (3, 1, 1), (13, 17, 11)])
def test_face_fusion_same_bits(n):
    """adg_lin_step at p = 3 with the faces inside the corrector (the default)
    against the separate face and corrector kernels: the same bits after
    several steps, on meshes with unequal and single-cell axes and with
    partial cell tiles along every axis; and the oracle's run to the bar."""
    p, steps = 3, 4
    om = oracle.Mesh(p, n)
    mat = materials(om.nc, 50)
    xyz = om.node_coords()
    u0 = np.stack([np.sin(2 * np.pi * (xyz[0] + k * xyz[1] - 0.5 * k * xyz[2]) + k) for k in range(9)])
    print(f"[linear face fusion] n={n}", flush=True)
    lm = A.LinMesh(p, n)
    md = dev(mat)
    runs = []
    for fuse in (True, False):
        lm.set_face_fusion(fuse)
        u = dev(u0)
        lm.step(md, u, steps, lm.empty_workspace())
        runs.append(u)
    torch.cuda.synchronize()
    assert torch.equal(runs[0], runs[1])
    want, _ = om.lin_run(mat, u0, steps)
    assert rel(runs[0].cpu().numpy().reshape(want.shape), want) <= 1e-12
    lm.close()


def test_full_size_plane_wave_and_constant_state():
    """81^3, p = 3, the benchmark's launch configuration: a plane P-wave along
    x after 20 steps against the exact solution (the discretisation error at
    this resolution, not a rounding bound), and a constant state kept to
    rounding."""
    p, n = 3, (81, 81, 81)
    lm = A.LinMesh(p, n)
    nc = lm.info["n_cells"]
    N = p + 1
    rho, lam, mu = 2.0, 1.5, 1.0
    cp = np.sqrt((lam + 2 * mu) / rho)
    mat = torch.tensor([rho, lam, mu], dtype=torch.float64, device="cuda")[:, None].repeat(1, nc).contiguous()
    xi, _ = oracle.gauss_legendre(N)
    i = torch.arange(nc, device="cuda") % n[0]
    x = ((i[:, None] + torch.tensor(xi, device="cuda")[None, :]) / n[0])        # [nc, N] along x
    x = x[:, None, None, :].expand(nc, N, N, N).reshape(nc, N ** 3)
    r = torch.zeros(9, dtype=torch.float64, device="cuda")
    r[6], r[0], r[1], r[2] = 1.0, -(lam + 2 * mu) / cp, -lam / cp, -lam / cp
    u = (r[:, None, None] * torch.sin(2 * np.pi * x)[None]).contiguous()
    ws = lm.empty_workspace()
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    print("[linear full size] plane wave 20 steps", flush=True)
    lm.step(mat, u, 20, ws, dt_out=dt)
    torch.cuda.synchronize()
    T = 20 * dt.item()
    exact = r[:, None, None] * torch.sin(2 * np.pi * (x - cp * T))[None]
    err = (u - exact).abs().max().item() / r.abs().max().item()
    print(f"   T = {T:.4e}, max error {err:.3e}", flush=True)
    assert err < 1e-5
    const = torch.from_numpy(np.random.Generator(np.random.PCG64(5)).standard_normal(9)).cuda()
    uc = const[:, None, None].repeat(1, nc, N ** 3).contiguous()
    u0 = uc.clone()
    lm.step(mat, uc, 3, ws)
    torch.cuda.synchronize()
    assert (uc - u0).abs().max().item() <= 1e-13 * const.abs().max().item()
    lm.close()


def test_refusals():
    with pytest.raises(A.AdgError) as e:
        A.LinMesh(7, (2, 2, 2))
    assert e.value.code == 2  # UNSUPPORTED
    with pytest.raises(A.AdgError) as e:
        A.LinMesh(2, (0, 2, 2))
    assert e.value.code == 1  # INVALID_ARG
