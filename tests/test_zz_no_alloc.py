"""adg_step_noalloc: the step with the library's static workspace gives the
same bits as adg_step with a caller workspace, on two calls in a row (the
second on a smaller mesh, so stale contents of the static array from the
first call would show), and refuses meshes whose workspace does not fit."""
import numpy as np
import pytest

import paper_1806_07984_amd as A
from paper_1806_07984_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def initial_state(mesh, seed):
    xyz = mesh.node_coords().cpu().numpy().reshape(3, -1)
    return torch.from_numpy(inputs.density_wave_noisy(xyz, seed=seed, noise=0.01).reshape(-1)).cuda()


def both_ways(desc, precision, steps, seed):
    mesh = A.Mesh(desc, precision)
    assert mesh.info["workspace_bytes"] <= A.NOALLOC_WORKSPACE_BYTES
    u0 = initial_state(mesh, seed)
    ref, got = u0.clone(), u0.clone()
    h_ref = torch.zeros(steps, dtype=torch.float64, device="cuda")
    h_got = torch.full((steps,), -1.0, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    mesh.step(ref, steps, mesh.empty_workspace(), dt_hist=h_ref, stream_skeleton=s, stream_enclave=s)
    mesh.step_noalloc(got, steps, dt_hist=h_got, stream=s)
    torch.cuda.synchronize()
    mesh.status()
    print(f"noalloc {precision} cells={mesh.info['n_cells']} steps={steps} "
          f"max|diff|={float((got - ref).abs().max()):.3e}", flush=True)
    assert torch.equal(got, ref)
    assert torch.equal(h_got, h_ref)
    assert float(h_ref.min()) > 0.0
    mesh.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_matches_step_two_calls(precision):
    """9^3 at p = 3 for 3 steps, then 5 x 4 x 3 at p = 2 for 2 steps."""
    both_ways(A.instance(3, (9, 9, 9)), precision, 3, seed=31)
    both_ways(A.instance(2, (5, 4, 3)), precision, 2, seed=32)


def test_noalloc_adaptive_then_smaller():
    """Hanging faces with level jumps of 1 and 2 (3^3 base, two levels), then
    a smaller uniform mesh."""
    ref = inputs.sphere_refine_list((3, 3, 3), 2, radius=0.2)
    both_ways(A.instance(2, (3, 3, 3), max_level=2, refine=ref), "fp64", 2, seed=33)
    both_ways(A.instance(1, (3, 2, 2)), "fp64", 2, seed=34)


def test_noalloc_refuses_a_mesh_too_large():
    mesh = A.Mesh(A.instance(3, (27, 27, 27)), "fp64")
    assert mesh.info["workspace_bytes"] > A.NOALLOC_WORKSPACE_BYTES
    u = mesh.empty_u()
    with pytest.raises(A.AdgError) as e:
        mesh.step_noalloc(u, 1)
    assert e.value.code == 6
    mesh.close()
