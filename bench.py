"""Benchmark of the ADER-DG step on one MI355X.

Workload: 3-D compressible Euler, p = 3 (4^3 Gauss-Legendre nodes per cell),
uniform periodic 81^3 mesh (531,441 cells, 170,061,120 DoFs), density wave
rho = 1 + 0.2 sin(2 pi (x+y+z)), velocity (1,1,1), pressure 1, plus seeded
U[-0.01, 0.01] noise on the nodal density; CFL 0.4, Rusanov faces.

The timed region runs K whole steps through adg_step (CFL reduction,
predictor, Riemann, corrector, all on the device; dt never leaves the GPU) for
the FP32 form (predictor, face data and Riemann in FP32; u, u*, dt and the
corrector accumulation in FP64) and for the plain FP64 path.  Per-kernel
durations come from HIP events the library records around every launch on
the launch's own stream during the timed region.

`value` is the plain FP64 path's DoF-updates/s (the paper's precision); the
FP32 form is reported beside it under `paths`, each path with the roofline
of its predictor kernel and a whole-step figure (algorithmic HBM bytes of the
three phases per step over the measured time per step, against 8 TB/s).

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_BASE = 81
ORDER = 3
SEED = 2026
PEAK = {"hbm_GBs": 8000.0, "fp64_TFs": 78.6, "fp32_TFs": 157.3}


def predictor_flops_per_node(N, npic):
    """Algorithmic flops of the predictor per spatial node (FMA = 2 flops,
    division = 1).  A Picard iteration from a general iterate costs N flux
    evaluations (29 flops) + 3 derivative contractions (2N each) per variable
    and time node + the time solve (2N per variable and time node).  The first
    iteration starts from the time-constant state u, so its N time nodes share
    one flux evaluation and one set of contractions, and the time solve
    reduces to the row sums of the time matrix (2 flops per variable and time
    node).  Then the epilogue (N flux evaluations, time averages of the state
    and the 3 fluxes, volume term) and the face projections (12 arrays x 5
    variables x N^2 face nodes x 2N per cell)."""
    per_iter = N * (29 + 5 * (3 * 2 * N + 5 + 2 * N)) + 5 * N
    first_iter = 29 + 5 * (3 * 2 * N + 5) + 5 * 2 * N
    epilogue = N * (29 + 5 * 2 + 15 * 2) + 5 * (3 * 2 * N + 6)
    traces = 12 * 5 * N * N * 2 * N / N ** 3
    iters = first_iter + (npic - 1) * per_iter if npic > 0 else 0
    return iters + epilogue + traces


def predictor_bytes_per_cell(N, real_bytes):
    """HBM bytes of the predictor per cell: read u, write u* (FP64), write the
    face projections (12 arrays x 5 variables x N^2 reals)."""
    return 2 * 5 * N ** 3 * 8 + 12 * 5 * N ** 2 * real_bytes


def step_bytes_per_cell(N, real_bytes, fused=True):
    """Algorithmic HBM bytes of one whole step per cell of a uniform periodic
    mesh (3 faces per cell): the predictor (read u, write u* and the 12 face
    projection arrays), then either (fused, the step at p = 3) one kernel that
    solves every cell's face problems and runs its corrector (read u* and the
    12 face projection arrays once, write u), or the separate Riemann solves
    (read both sides' state and normal flux projections, write the flux both
    sides see) and corrector (read u* and the 6 face fluxes, write u).  The
    next step's CFL maximum is fused into the corrector; the CFL final
    reduction reads one value per corrector block."""
    pred = predictor_bytes_per_cell(N, real_bytes)
    if fused:
        return pred + 2 * 5 * N ** 3 * 8 + 12 * 5 * N ** 2 * real_bytes
    riem = 3 * 6 * 5 * N ** 2 * real_bytes
    corr = 2 * 5 * N ** 3 * 8 + 6 * 5 * N ** 2 * real_bytes
    return pred + riem + corr


def cpu_baseline(budget_s=12.0):
    """The oracle (plain FP64 C, OpenMP over cells) on a bounded sample of the
    same workload: 27^3 cells, p = 3, same initial state recipe."""
    import oracle
    from paper_1806_07984_amd import inputs
    n = 27
    om = oracle.Mesh(ORDER, (n, n, n))
    u = inputs.density_wave_noisy(om.node_coords(), seed=SEED, noise=0.01)
    dofs = om.nc * 5 * (ORDER + 1) ** 3
    steps, t0 = 0, time.perf_counter()
    while True:
        u, _, rc = om.run(u, 1)
        steps += 1
        el = time.perf_counter() - t0
        if rc != 0 or el >= budget_s:
            break
    return {"value": dofs * steps / el, "unit": "DoF-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} step(s) of a 27^3 periodic mesh, p=3, density wave + node noise "
                      f"({dofs} DoFs/step), {el:.1f} s"}


def load_traffic(kernel_name):
    """HBM traffic of a kernel from committed rocprofv3 --pmc summaries, if
    they were taken on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel_name)
    if not rec:
        return None
    src = open(os.path.join(ROOT, "paper_1806_07984_amd", "csrc", "kernels.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("kernels_sha"):
        return None
    return rec["bytes_per_launch"]


def run_path(A, precision, u0, steps, warmup):
    """Timed region: `steps` steps with HIP events around the predictor
    launches only (their average duration is the roofline's kernel time).
    Then the same number of steps again with every phase timed, for the
    per-phase breakdown (its events add a little time, so it is not the
    figure of merit)."""
    import torch
    mesh = A.Mesh(A.instance(ORDER, (N_BASE,) * 3), precision)
    u = u0.clone()
    ws = mesh.empty_workspace()
    s = torch.cuda.current_stream()
    mesh.step(u, warmup, ws, stream_skeleton=s, stream_enclave=s)
    torch.cuda.synchronize()
    mesh.profile(True, predictor_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mesh.step(u, steps, ws, stream_skeleton=s, stream_enclave=s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = mesh.profile_read()
    mesh.profile(True)
    mesh.step(u, steps, ws, stream_skeleton=s, stream_enclave=s)
    phases = mesh.profile_read()
    mesh.profile(False)
    mesh.status()
    ms_step = (t1 - t0) * 1e3 / steps
    dofs = mesh.info["n_dofs"]
    N = ORDER + 1
    pm, pc = prof["predictor"]
    avg = pm / max(pc, 1)
    nc = mesh.info["n_cells"]
    flops = predictor_flops_per_node(N, N) * nc * N ** 3
    res = {
        "value": dofs * steps / (t1 - t0),
        "ms_per_step": ms_step,
        "phases_ms_per_step": {k: v[0] / steps for k, v in phases.items()},
        "predictor": {"avg_ms": avg, "flops_per_launch": flops, "tflops": flops / (avg * 1e-3) / 1e12,
                      "bytes_per_launch": predictor_bytes_per_cell(N, mesh.info["real_bytes"]) * nc},
    }
    mesh.close()
    del ws, u
    torch.cuda.empty_cache()
    return res


def run_amr(A, steps=50, sharp=False):
    """Adaptive mesh: 27^3 base cells, two levels of 3:1 refinement in the
    sphere |x - c| <= 0.25 (1,074,035 cells), p = 4, FP32 form.  The blast
    wave with its interface smoothed over one finest cell (sharp=False), or
    the sharp blast with the a-posteriori subcell limiter (sharp=True).  The
    limiter acts on cells of the finest level only (no resolution transition
    cuts an FV region), so the sharp blast's discontinuity sits one level-1
    cell inside the refined sphere: radius 0.25 - 1/81.
    Timed both ways: the skeleton/enclave split on the handle's two streams
    (two different caller streams passed), and every phase on one stream."""
    import torch
    from paper_1806_07984_amd import inputs
    n = (27, 27, 27)
    ref = inputs.sphere_refine_list(n, 2, radius=0.25)
    mesh = A.Mesh(A.instance(4, n, max_level=2, refine=ref), "fp32")
    xyz = mesh.node_coords().cpu().numpy().reshape(3, -1)
    state = inputs.blast(xyz, radius=0.25 - 1.0 / 81) if sharp else inputs.blast_smooth(xyz, width=1.0 / (27 * 9))
    u0 = torch.from_numpy(state.reshape(-1)).cuda()
    del xyz, state
    if sharp:
        mesh.set_limiter(1, 1e-4, 1e-3)
    ws = mesh.empty_workspace()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    times = {}
    for mode in ("two streams", "one stream"):
        u = u0.clone()
        a, b = (s1, s2) if mode == "two streams" else (cur, cur)
        a.wait_stream(cur)
        b.wait_stream(cur)
        mesh.step(u, 1, ws, stream_skeleton=a, stream_enclave=b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mesh.step(u, steps, ws, stream_skeleton=a, stream_enclave=b)
        torch.cuda.synchronize()
        times[mode] = time.perf_counter() - t0
        mesh.status()
    el = times["two streams"]
    info = mesh.info
    out = {"value": info["n_dofs"] * steps / el, "unit": "DoF-updates/s", "ms_per_step": el * 1e3 / steps,
           "steps": steps, "cells": info["n_cells"], "dofs": info["n_dofs"],
           "hanging_faces": info["n_hanging_faces"], "skeleton_cells": info["n_skeleton_cells"],
           "state": "sharp blast, subcell limiter" if sharp else "blast smoothed over one finest cell",
           "path": "fp32, skeleton/enclave split on two streams",
           "ms_per_step_by_streams": {k: v * 1e3 / steps for k, v in times.items()}}
    if sharp:
        nl, nr, fl = mesh.limiter_stats(flags=True)
        out["limited_cells_last_step"] = nl
        out["rerun_cells_last_step"] = nr
        out["troubled_not_limitable_last_step"] = int(((fl == 3) | (fl == 4)).sum().item())
    else:
        # the first new handle in a process also creates hardware queues for
        # its two streams (a few ms, once); two repeats show the steady cost
        out["adaptation"] = adapt_once(A, mesh, u, 0.05, 0.005)
        out["adaptation"]["total_ms_repeats"] = [out["adaptation"]["total_ms"]] + [
            adapt_once(A, mesh, u, 0.05, 0.005)["total_ms"] for _ in range(2)]
    mesh.close()
    del u, u0, ws
    torch.cuda.empty_cache()
    return out


def adapt_once(A, mesh, u, theta_refine, theta_coarsen):
    """One adaptation step of the state after the timed steps: indicator
    (device), plan (host, from the leaves the handle keeps), the new handle
    (host mesh build and uploads) and the volumetric transfer (host table,
    device kernel), timed each."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    eta = mesh.indicator(u).cpu().numpy()
    t1 = time.perf_counter()
    rows = mesh.adapt_plan(eta, theta_refine, theta_coarsen)
    t2 = time.perf_counter()
    new = A.Mesh(dict(mesh.descs[0], refine=rows), mesh.precision)
    t3 = time.perf_counter()
    u_new = mesh.transfer_to(u, new)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    res = {"theta_refine": theta_refine, "theta_coarsen": theta_coarsen, "cells_before": mesh.info["n_cells"],
           "cells_after": new.info["n_cells"], "indicator_ms": (t1 - t0) * 1e3, "plan_ms": (t2 - t1) * 1e3,
           "new_mesh_ms": (t3 - t2) * 1e3, "transfer_ms": (t4 - t3) * 1e3, "total_ms": (t4 - t0) * 1e3}
    new.close()
    del u_new
    return res


def run_batch(A, steps=10, seed=0):
    """64 periodic instances, edges in {9,15,21,27,45} and orders 2..6 drawn
    from a seed, density waves with amplitudes in [0.05, 0.3]; FP32 form,
    one persistent predictor launch over all instances, autotuned cells per
    work item, hipGraph-captured step."""
    import torch
    from paper_1806_07984_amd import inputs
    draws = inputs.batch_instances(64, seed=seed)
    mesh = A.Mesh([A.instance(d["order"], (d["edge"],) * 3) for d in draws], "fp32")
    xyz = mesh.node_coords().cpu().numpy()
    u0 = np.zeros(mesh.info["u_elems"])
    for g, d in zip(mesh.instances, draws):
        nn = g["n_cells"] * (g["order"] + 1) ** 3
        x = xyz[3 * g["u_offset"] // 5: 3 * g["u_offset"] // 5 + 3 * nn].reshape(3, nn)
        u0[g["u_offset"]: g["u_offset"] + 5 * nn] = inputs.density_wave(x, amp=d["amp"]).reshape(-1)
    del xyz
    u = torch.from_numpy(u0).cuda()
    del u0
    ws = mesh.empty_workspace()
    mesh.autotune(u, ws)
    res = {}
    for mode, name in ((1, "one persistent predictor launch per order"),
                       (2, "one persistent predictor launch for all orders")):
        mesh.set_options(use_graph=True, batched=mode)
        mesh.step(u, 1, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mesh.step(u, steps, ws)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        mesh.status()
        res[mode] = (el, name)
    best = min(res, key=lambda k: res[k][0])
    el = res[best][0]
    out = {"value": mesh.info["n_dofs"] * steps / el, "unit": "DoF-updates/s", "ms_per_step": el * 1e3 / steps,
           "steps": steps, "instances": 64, "dofs": mesh.info["n_dofs"],
           "tuning_cells_per_item": {f"p={N - 1}": c for N, c in mesh.tuning().items() if 3 <= N <= 7},
           "path": "fp32, graph, " + res[best][1],
           "ms_per_step_by_mode": {v[1]: v[0] * 1e3 / steps for v in res.values()}}
    mesh.close()
    del u, ws
    torch.cuda.empty_cache()
    return out


def run_uniform(A, order, n, steps=10, warmup=10):
    """The headline's workload at another order: a periodic n^3 mesh with about
    the same number of degrees of freedom, the density wave with seeded node
    noise, both precisions (the generic predictor and the separate face and
    corrector kernels at p != 3).  DoF-updates/s and ms per step of plain
    launches."""
    import torch
    from paper_1806_07984_amd import inputs
    out = {"order": order, "cells": n ** 3, "dofs": 5 * n ** 3 * (order + 1) ** 3}
    for prec in ("fp64", "fp32"):
        mesh = A.Mesh(A.instance(order, (n,) * 3), prec)
        xyz = mesh.node_coords().cpu().numpy().reshape(3, -1)
        u = torch.from_numpy(inputs.density_wave_noisy(xyz, seed=SEED, noise=0.01).reshape(-1)).cuda()
        del xyz
        ws = mesh.empty_workspace()
        s = torch.cuda.current_stream()
        mesh.step(u, warmup, ws, stream_skeleton=s, stream_enclave=s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mesh.step(u, steps, ws, stream_skeleton=s, stream_enclave=s)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mesh.status()
        out[prec] = {"value": out["dofs"] * steps / dt, "ms_per_step": dt * 1e3 / steps}
        mesh.close()
        del u, ws
    torch.cuda.empty_cache()
    out["value"] = out["fp64"]["value"]
    out["unit"] = "DoF-updates/s"
    return out


def run_limiter(A, steps=20, warmup=10):
    """A-posteriori subcell limiter: uniform periodic 81^3 mesh, p = 3, the
    discontinuous spherical blast wave (rho, p = 1, 1 inside radius 0.25,
    0.125, 0.1 outside, at rest), delta0 = 1e-4, eps = 1e-3; both precisions.
    Timed: `steps` limited steps (plain launches, one stream); then the same
    again with every phase timed for the breakdown."""
    import torch
    from paper_1806_07984_amd import inputs
    n = (N_BASE,) * 3
    probe = A.Mesh(A.instance(ORDER, n), "fp64")
    xyz = probe.node_coords().cpu().numpy().reshape(3, -1)
    probe.close()
    u0 = torch.from_numpy(inputs.blast(xyz).reshape(-1)).cuda()
    del xyz
    out = {"workload": "blast_p3_81cubed_limited", "unit": "DoF-updates/s", "steps": steps}
    for precision in ("fp32", "fp64"):
        mesh = A.Mesh(A.instance(ORDER, n), precision)
        mesh.set_options(use_graph=False, batched=0)
        mesh.set_limiter(1, 1e-4, 1e-3)
        u = u0.clone()
        ws = mesh.empty_workspace()
        s = torch.cuda.current_stream()
        mesh.step(u, warmup, ws, stream_skeleton=s, stream_enclave=s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mesh.step(u, steps, ws, stream_skeleton=s, stream_enclave=s)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        nl, nr = mesh.limiter_stats()
        mesh.profile(True)
        mesh.step(u, steps, ws, stream_skeleton=s, stream_enclave=s)
        phases = mesh.profile_read()
        mesh.profile(False)
        mesh.status()
        out[precision] = {"value": mesh.info["n_dofs"] * steps / el, "ms_per_step": el * 1e3 / steps,
                          "limited_cells_last_step": nl, "rerun_cells_last_step": nr,
                          "cells": mesh.info["n_cells"],
                          "phases_ms_per_step": {k: v[0] / steps for k, v in phases.items()}}
        mesh.close()
        del u, ws
        torch.cuda.empty_cache()
    out["value"] = out["fp32"]["value"]
    return out


def run_linear(A, steps=20, warmup=10):
    """Linear variant: elastic waves, uniform periodic 81^3 mesh, p = 3,
    Cauchy-Kowalevski predictor, FP64.  Synthetic layered medium (a softer
    layer, rho, lambda, mu = 2.0, 2.0, 1.0, for z > 0.75 over rho, lambda,
    mu = 2.7, 4.0, 2.0) and a Gaussian velocity pulse of width 0.05 at the
    centre (stands in for the point-source benchmark, whose data are not
    here).  Timed with events around `steps` steps."""
    import torch
    n = (N_BASE,) * 3
    p = ORDER
    N = p + 1
    lm = A.LinMesh(p, n)
    nc = lm.info["n_cells"]
    c = torch.arange(nc, device="cuda")
    k = c // (n[0] * n[1])
    soft = (k + 0.5) / n[2] > 0.75
    def layered(top, below):
        return torch.where(soft, torch.tensor(top, dtype=torch.float64, device="cuda"),
                           torch.tensor(below, dtype=torch.float64, device="cuda"))
    mat = torch.stack([layered(2.0, 2.7), layered(2.0, 4.0), layered(1.0, 2.0)]).contiguous()
    xi = torch.tensor(_gl_nodes(N), device="cuda")
    i, j = c % n[0], (c // n[0]) % n[1]

    def coord(idx, m):
        return (idx[:, None] + xi[None, :]) / m
    x = coord(i, n[0])[:, None, None, :].expand(nc, N, N, N).reshape(nc, -1)
    y = coord(j, n[1])[:, None, :, None].expand(nc, N, N, N).reshape(nc, -1)
    z = coord(k, n[2])[:, :, None, None].expand(nc, N, N, N).reshape(nc, -1)
    r2 = (x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2
    u = torch.zeros(9, nc, N ** 3, dtype=torch.float64, device="cuda")
    pulse = torch.exp(-r2 / 0.05 ** 2)
    u[6], u[7], u[8] = pulse, 0.5 * pulse, -0.25 * pulse
    del x, y, z, r2, pulse
    ws = lm.empty_workspace()
    lm.step(mat, u, warmup, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lm.step(mat, u, steps, ws)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    assert torch.isfinite(u).all().item()
    dofs = 9 * nc * N ** 3
    out = {"workload": "elastic_p3_81cubed_layered", "value": dofs * 1e3 / ms, "unit": "DoF-updates/s",
           "ms_per_step": ms, "steps": steps, "cells": nc, "dofs": dofs, "path": "fp64, Cauchy-Kowalevski",
           "predictor_bytes_per_cell": 9 * N ** 3 * 8 * 2 + 24 + 6 * 2 * 9 * N * N * 8}
    lm.close()
    del u, ws, mat
    torch.cuda.empty_cache()
    return out


def _gl_nodes(N):
    """Gauss-Legendre nodes on [0, 1] (numpy), for placing the pulse."""
    import numpy as np
    x, _ = np.polynomial.legendre.leggauss(N)
    return (x + 1.0) / 2.0


def run_adjoint(A, n=27, steps=20, k=5, n_pts=512):
    """Differentiation workload: 27^3 cells, p = 3, FP64, 20 steps; loss =
    sampled density misfit at 512 seeded points; gradient with respect to
    the whole initial state through the hand-written adjoint, checkpoint
    every 5 steps.  Reports the forward time (20 steps) and the gradient
    time (forward with checkpoints, segment recomputation and the adjoint
    steps) and their ratio."""
    import torch
    from paper_1806_07984_amd import inputs, rollout
    mesh = A.Mesh(A.instance(ORDER, (n, n, n)), "fp64")
    xyz = mesh.node_coords().cpu().numpy().reshape(3, -1)
    u0 = torch.from_numpy(inputs.density_wave_noisy(xyz, seed=7, noise=0.01).reshape(-1)).cuda()
    pts = torch.from_numpy(inputs.sample_points(n_pts, seed=1)).cuda().contiguous()
    target = torch.from_numpy(inputs.sample_targets(n_pts, seed=2)).cuda()
    sched = rollout.dt_schedule(mesh, u0, steps)  # also warms up
    rollout.loss_and_grad(mesh, u0, pts, target, steps, k=k, dt_sched=sched)
    torch.cuda.synchronize()
    u = u0.clone()
    ws = mesh.empty_workspace()
    t0 = time.perf_counter()
    mesh.step(u, steps, ws)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    J, g, _ = rollout.loss_and_grad(mesh, u0, pts, target, steps, k=k, dt_sched=sched)
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    mesh.status()
    out = {"forward_ms": t_fwd * 1e3, "gradient_ms": t_grad * 1e3, "gradient_over_forward": t_grad / t_fwd,
           "steps": steps, "checkpoint_every": k, "cells": n ** 3, "dofs": mesh.info["n_dofs"],
           "loss": float(J), "path": "fp64"}
    mesh.close()
    del u, ws, g
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["fp64", "fp32"], default=None,
                    help="run one path only (for profiling runs)")
    ap.add_argument("--no-extra", action="store_true", help="skip the AMR and batch workloads")
    ap.add_argument("--extra-only", choices=["amr", "amr_sharp", "batch", "adjoint", "limiter", "linear", "uniform_p4",
                                             "uniform_p5"],
                    default=None,
                    help="run only one of the other workloads and print its JSON (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB buffer 3 times (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": 2 * a.numel() * 8, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design, not a measured path.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1806_07984_amd as A
    from paper_1806_07984_amd import inputs

    A.load()
    if args.extra_only:
        res = {"amr": run_amr, "amr_sharp": lambda A: run_amr(A, sharp=True), "batch": run_batch,
               "uniform_p4": lambda A: run_uniform(A, 4, 65), "uniform_p5": lambda A: run_uniform(A, 5, 54),
               "adjoint": run_adjoint, "limiter": run_limiter, "linear": run_linear}[args.extra_only](A)
        print(json.dumps({"workload": args.extra_only, **res}))
        return
    # initial state: node coordinates from the library, analytic state + seeded noise on the host
    probe = A.Mesh(A.instance(ORDER, (N_BASE,) * 3), "fp64")
    xyz = probe.node_coords().cpu().numpy().reshape(3, -1)
    probe.close()
    u0 = torch.from_numpy(inputs.density_wave_noisy(xyz, seed=SEED, noise=0.01).reshape(-1)).cuda()
    del xyz

    paths = ["fp64", "fp32"] if args.only is None else [args.only]
    res = {p: run_path(A, p, u0, args.steps, args.warmup) for p in paths}
    head_prec = "fp64" if "fp64" in res else "fp32"
    head = res[head_prec]
    kernels = {"fp64": "adg::k_predictor4_f64", "fp32": "adg::k_predictor4_mfma"}
    nc = N_BASE ** 3
    N = ORDER + 1

    def roofline(prec):
        pr = res[prec]["predictor"]
        peak = PEAK["fp64_TFs"] if prec == "fp64" else PEAK["fp32_TFs"]
        return {"bound": "alu", "achieved": pr["tflops"], "peak": peak, "unit": "TFLOP/s",
                "frac": pr["tflops"] / peak, "traffic": load_traffic(f"predictor_{prec}"),
                "kernel": kernels[prec], "avg_launch_ms": pr["avg_ms"],
                "flops_per_launch": pr["flops_per_launch"], "bytes_per_launch": pr["bytes_per_launch"],
                "hbm_GBs_algorithmic": pr["bytes_per_launch"] / (pr["avg_ms"] * 1e-3) / 1e9}

    def whole_step(prec):
        b = step_bytes_per_cell(N, 8 if prec == "fp64" else 4) * nc
        ms = res[prec]["ms_per_step"]
        gbs = b / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "bytes_per_step": b, "achieved": gbs, "peak": PEAK["hbm_GBs"], "unit": "GB/s",
                "frac": gbs / PEAK["hbm_GBs"]}
    out = {
        "metric": "DoF-updates/s, 3D Euler ADER-DG p=3-5: FP64 plain vs FP32-MFMA batched; % roofline",
        "value": head["value"],
        "unit": "DoF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_prec == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "euler3d_aderdg_p3_periodic_81cubed_density_wave_noise", "order": ORDER,
                   "cells": N_BASE ** 3, "dofs": 5 * N_BASE ** 3 * (ORDER + 1) ** 3, "path": head_prec,
                   "parallelism": "single-gpu"},
        "roofline": roofline(head_prec),
        "whole_step_roofline": whole_step(head_prec),
        "paths": {k: {"value": v["value"], "ms_per_step": v["ms_per_step"],
                      "dtype": "f64" if k == "fp64" else "f32+f64",
                      "phases_ms_per_step": v["phases_ms_per_step"],
                      "roofline": roofline(k), "whole_step_roofline": whole_step(k)} for k, v in res.items()},
    }
    if not args.no_extra:
        out["other_workloads"] = {"uniform_p4_65cubed": run_uniform(A, 4, 65),
                                  "uniform_p5_54cubed": run_uniform(A, 5, 54),
                                  "amr_blast_p4_27cubed_2levels": run_amr(A),
                                  "amr_sharp_blast_p4_27cubed_2levels_limited": run_amr(A, steps=20, sharp=True),
                                  "batch64_p2to6_seed0": run_batch(A),
                                  "adjoint_p3_27cubed_20steps": run_adjoint(A),
                                  "limiter_blast_p3_81cubed": run_limiter(A),
                                  "elastic_p3_81cubed_layered": run_linear(A)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
