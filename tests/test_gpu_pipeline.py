"""The pipelined step (predictors chunk by chunk on one stream, the faces and
correctors of finished chunks on another) against the sequential step: the
same per-cell and per-face arithmetic, so the states and the dt histories must
agree bit for bit, eager and graph-captured, with one caller stream or two."""
import numpy as np
import pytest

import oracle
import paper_1806_07984_amd as A
from paper_1806_07984_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(gm, u0, steps, two_streams=False):
    u = torch.from_numpy(u0.copy()).cuda()
    ws = gm.empty_workspace()
    hist = torch.zeros(steps, dtype=torch.float64, device="cuda")
    if two_streams:
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        s1.wait_stream(torch.cuda.current_stream())
        s2.wait_stream(torch.cuda.current_stream())
        gm.step(u, steps, ws, hist, stream_skeleton=s1, stream_enclave=s2)
        torch.cuda.current_stream().wait_stream(s1)
        torch.cuda.current_stream().wait_stream(s2)
    else:
        gm.step(u, steps, ws, hist)
    torch.cuda.synchronize()
    gm.status()
    return u, hist


@pytest.mark.parametrize("order,precision", [(3, "fp32"), (3, "fp64"), (2, "fp64"), (4, "fp32"), (1, "fp32")])
def test_pipelined_step_is_bitwise_identical(order, precision):
    n = (12, 10, 9)
    gm = A.Mesh(A.instance(order, n), precision)
    u0 = inputs.density_wave_noisy(oracle.Mesh(order, n).node_coords(), seed=31, noise=0.02).reshape(-1)
    steps = 4
    gm.set_pipeline(False)
    gm.set_options(use_graph=False, batched=False)
    ref_u, ref_h = run(gm, u0, steps)
    for pipe in (0, 1, 2):
        for graph in (False, True):
            for two in (False, True):
                print(f"[pipeline] p={order} {precision} pipe={pipe} graph={graph} two_streams={two}", flush=True)
                gm.set_pipeline(pipe)
                gm.set_options(use_graph=graph, batched=False)
                u, h = run(gm, u0, steps, two)
                assert torch.equal(u, ref_u), (pipe, graph, two)
                assert torch.equal(h, ref_h), (pipe, graph, two)


def test_pipeline_large_mesh_and_refusals():
    # a mesh of 68,921 cells (chunks of ~8,600 cells, several corrector blocks each)
    big = A.Mesh(A.instance(3, (41, 41, 41)), "fp32")
    u0 = inputs.density_wave(big.node_coords().cpu().numpy().reshape(3, -1)).reshape(-1)
    u_seq, h_seq = run(big, u0, 2)
    big.set_pipeline(True)
    u_pipe, h_pipe = run(big, u0, 2)
    assert torch.equal(u_pipe, u_seq) and torch.equal(h_pipe, h_seq)
    big.close()
    # not available with hanging faces or several instances
    ref = inputs.sphere_refine_list((6, 6, 6), 1, radius=0.2)
    amr = A.Mesh(A.instance(2, (6, 6, 6), max_level=1, refine=ref), "fp64")
    with pytest.raises(A.AdgError) as e:
        amr.set_pipeline(True)
    assert e.value.code == 2
    two = A.Mesh([A.instance(2, (4, 4, 4)), A.instance(3, (3, 3, 3))], "fp64")
    with pytest.raises(A.AdgError) as e:
        two.set_pipeline(True)
    assert e.value.code == 2
