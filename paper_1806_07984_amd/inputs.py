"""Seeded synthetic inputs for the ADER-DG step (initial states, meshes, samples).

This module holds no arithmetic of the method: it evaluates analytic initial
states at node coordinates that the caller supplies, draws seeded random
numbers (NumPy PCG64) and describes refinement patterns geometrically.  Both
the product path and the oracle receive exactly the arrays it returns.

Workloads (3-D compressible Euler, gamma = 1.4, periodic unit cube):
  * density wave   rho = 1 + A sin(2 pi k.(x - v t)), v = (1,1,1), p = 1;
  * node noise     seeded U[-a, a] added to the primitive density at each node,
                   velocity and pressure unchanged;
  * blast wave     rho = 1, p = 1 inside |x - c| < R, rho = 0.125, p = 0.1
                   outside, zero velocity; optionally with the interface
                   smoothed by a tanh profile;
  * sphere refinement: a cell is split 3x3x3 when its closed box meets the
                   closed ball |x - c| <= R, recursively up to max_level.
"""
import numpy as np

GAMMA = 1.4


def conserved(rho, vel, p, gamma=GAMMA):
    """(rho, m1, m2, m3, E) stacked on a new leading axis from primitives."""
    rho = np.asarray(rho, dtype=np.float64)
    v = [np.broadcast_to(np.asarray(vel[d], dtype=np.float64), rho.shape) for d in range(3)]
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    m = [rho * v[d] for d in range(3)]
    E = p / (gamma - 1.0) + 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    return np.stack([rho, m[0], m[1], m[2], E])


def density_wave(xyz, amp=0.2, vel=(1.0, 1.0, 1.0), wavevec=(1.0, 1.0, 1.0), p=1.0, t=0.0,
                 gamma=GAMMA):
    """Smooth density wave advected with constant velocity and pressure.

    xyz: array [3, ...] of node coordinates.  Returns [5, ...]."""
    xyz = np.asarray(xyz, dtype=np.float64)
    phase = sum(wavevec[d] * (xyz[d] - vel[d] * t) for d in range(3))
    rho = 1.0 + amp * np.sin(2.0 * np.pi * phase)
    return conserved(rho, vel, p, gamma)


def density_wave_noisy(xyz, seed, noise=0.01, amp=0.2, vel=(1.0, 1.0, 1.0), p=1.0, gamma=GAMMA):
    """Density wave plus seeded uniform [-noise, noise] on the nodal density."""
    xyz = np.asarray(xyz, dtype=np.float64)
    phase = xyz[0] + xyz[1] + xyz[2]
    rho = 1.0 + amp * np.sin(2.0 * np.pi * phase)
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = rho + rng.uniform(-noise, noise, size=rho.shape)
    return conserved(rho, vel, p, gamma)


def blast(xyz, center=(0.5, 0.5, 0.5), radius=0.25, inside=(1.0, 1.0), outside=(0.125, 0.1),
          gamma=GAMMA):
    """Spherical blast wave, evaluated at the nodes (strict inequality inside)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    r2 = sum((xyz[d] - center[d]) ** 2 for d in range(3))
    ins = r2 < radius * radius
    rho = np.where(ins, inside[0], outside[0])
    p = np.where(ins, inside[1], outside[1])
    return conserved(rho, (0.0, 0.0, 0.0), p, gamma)


def blast_smooth(xyz, width, center=(0.5, 0.5, 0.5), radius=0.25, inside=(1.0, 1.0),
                 outside=(0.125, 0.1), gamma=GAMMA, velocity=(0.0, 0.0, 0.0)):
    """Blast wave whose interface is smoothed by a tanh profile of the given
    width: s = (1 - tanh((r - R)/width))/2, value = outside + s (inside - outside)
    for density and pressure; a uniform velocity (zero by default)."""
    xyz = np.asarray(xyz, dtype=np.float64)
    r = np.sqrt(sum((xyz[d] - center[d]) ** 2 for d in range(3)))
    s = 0.5 * (1.0 - np.tanh((r - radius) / width))
    rho = outside[0] + s * (inside[0] - outside[0])
    p = outside[1] + s * (inside[1] - outside[1])
    return conserved(rho, velocity, p, gamma)


def sphere_refine_list(n, max_level, center=(0.5, 0.5, 0.5), radius=0.25, lo=(0.0, 0.0, 0.0),
                       hi=(1.0, 1.0, 1.0)):
    """(level, i, j, k) of every cell to split, level by level.

    A cell is split when its closed box intersects the closed ball; children
    of split cells are tested again on the next level."""
    n = np.asarray(n, dtype=np.int64)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    c = np.asarray(center, dtype=np.float64)
    out = []
    # candidates at level 0: every base cell
    ii = np.stack(np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij"),
                  axis=-1).reshape(-1, 3)
    for lev in range(max_level):
        h = (hi - lo) / (n * 3 ** lev)
        blo = lo + ii * h
        bhi = blo + h
        nearest = np.clip(c, blo, bhi)
        hit = ((nearest - c) ** 2).sum(axis=1) <= radius * radius
        sel = ii[hit]
        if sel.shape[0] == 0:
            break
        out.append(np.concatenate([np.full((sel.shape[0], 1), lev), sel], axis=1))
        # children of the split cells
        off = np.stack(np.meshgrid(np.arange(3), np.arange(3), np.arange(3), indexing="ij"),
                       axis=-1).reshape(-1, 3)
        ii = (3 * sel[:, None, :] + off[None, :, :]).reshape(-1, 3)
    if not out:
        return np.zeros((0, 4), dtype=np.int32)
    return np.ascontiguousarray(np.concatenate(out, axis=0), dtype=np.int32)


def batch_instances(n_inst=64, seed=0, edges=(9, 15, 21, 27, 45), orders=(2, 3, 4, 5, 6),
                    amp_range=(0.05, 0.3)):
    """Seeded draws for a batch of independent periodic instances:
    list of dicts (edge, order, amp)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.choice(np.asarray(edges), size=n_inst)
    p = rng.choice(np.asarray(orders), size=n_inst)
    a = rng.uniform(amp_range[0], amp_range[1], size=n_inst)
    return [dict(edge=int(e[i]), order=int(p[i]), amp=float(a[i])) for i in range(n_inst)]


def sample_points(n_pts=512, seed=1):
    """Seeded sample points x_s ~ U[0,1)^3, shape [n_pts, 3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=(n_pts, 3))


def sample_targets(n_pts=512, seed=2, lo=0.8, hi=1.2):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=n_pts)


def directions(shape, count, seed=3):
    """Seeded standard-normal perturbation directions, [count, *shape]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=(count,) + tuple(shape))
