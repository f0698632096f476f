"""Shared test helpers: error metrics and side-by-side runs of the HIP path
(through the C ABI) and the oracle on identical seeded inputs."""
import numpy as np

import oracle

NV = 5


def rel_l2_per_var(x, ref, weights=None, floor_var=0):
    """Relative L2 error per variable (leading axis), with the norm of a
    variable floored at 1e-3 times the norm of variable floor_var so that
    variables that vanish (zero momentum) do not blow up the ratio."""
    x = np.asarray(x, dtype=np.float64).reshape(NV, -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(NV, -1)
    w = np.ones(x.shape[1]) if weights is None else np.asarray(weights).reshape(-1)
    nr = np.sqrt((ref ** 2 * w).sum(axis=1))
    ne = np.sqrt(((x - ref) ** 2 * w).sum(axis=1))
    return ne / np.maximum(nr, 1e-3 * nr[floor_var])


def solution_weights(mesh_oracle, n_base):
    """Quadrature weight x cell volume of every node, [n_cells * N^3]."""
    N = mesh_oracle.N
    w = oracle.gauss_legendre(N)[1]
    W = np.einsum("i,j,k->kji", w, w, w).reshape(-1)
    lev = mesh_oracle.cells()[:, 0].astype(np.float64)
    vol = (1.0 / np.prod(n_base)) / 27.0 ** lev
    return (vol[:, None] * W[None, :]).reshape(-1)


def rel_l2_blocks(x, ref, lead):
    """Relative L2 error of every block along the first `lead` axes, with a
    floor of 1e-3 times the largest block norm (for face arrays whose
    components can vanish)."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    shp = ref.shape[:lead]
    x = x.reshape(int(np.prod(shp)), -1)
    ref = ref.reshape(int(np.prod(shp)), -1)
    nr = np.sqrt((ref ** 2).sum(axis=1))
    ne = np.sqrt(((x - ref) ** 2).sum(axis=1))
    return (ne / np.maximum(nr, 1e-3 * nr.max())).reshape(shp)
