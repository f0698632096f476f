"""Plain FP64 CPU oracle of the ADER-DG step (ctypes binding of adg_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of
the benchmark use this package; the product library never imports it, and it
imports nothing from the product.

Arrays use the layouts documented at the top of adg_oracle.c (they are the
same documented layouts the product's C ABI uses, so results compare element
by element).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NV = 5
SIDE_CONFORMING, SIDE_FINE, SIDE_COARSE = 0, 1, 2


def build():
    """Compile the oracle with gcc (OpenMP over independent cells)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, P, P]
        L.orc_basis.argtypes = [ctypes.c_int, P, P, P, P, P, P, P]
        L.orc_transfer.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        L.orc_mesh_build.restype = P
        L.orc_mesh_build.argtypes = [ctypes.c_int, P, P, P, ctypes.c_int, ctypes.c_long, P]
        L.orc_mesh_free.argtypes = [P]
        L.orc_mesh_ncells.restype = ctypes.c_long
        L.orc_mesh_ncells.argtypes = [P]
        L.orc_mesh_cells.argtypes = [P, P]
        L.orc_mesh_sides.argtypes = [P, P, P]
        L.orc_node_coords.argtypes = [P, P]
        L.orc_cfl.restype = ctypes.c_double
        L.orc_cfl.argtypes = [P, ctypes.c_double, ctypes.c_double, P, P]
        L.orc_predictor.argtypes = [P, ctypes.c_double, ctypes.c_int, ctypes.c_double, P, P, P]
        L.orc_riemann.restype = ctypes.c_int
        L.orc_riemann.argtypes = [P, ctypes.c_double, P, P]
        L.orc_corrector.argtypes = [P, ctypes.c_double, P, P, P]
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, P, ctypes.c_int, P]
        L.orc_run_sched.restype = ctypes.c_int
        L.orc_run_sched.argtypes = [P, ctypes.c_double, ctypes.c_int, P, P, ctypes.c_int]
        L.orc_sample.restype = ctypes.c_int
        L.orc_sample.argtypes = [P, P, P, ctypes.c_long, P]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_step_tlm.restype = ctypes.c_int
        L.orc_step_tlm.argtypes = [P, ctypes.c_double, ctypes.c_int, ctypes.c_double, P, ctypes.c_int, P]
        L.orc_step_adj.restype = ctypes.c_int
        L.orc_step_adj.argtypes = [P, ctypes.c_double, ctypes.c_int, ctypes.c_double, P, P, P]
        L.orc_sample_adj.restype = ctypes.c_int
        L.orc_sample_adj.argtypes = [P, P, ctypes.c_long, P, P]
        L.orc_lin_flux_matrix.argtypes = [P, ctypes.c_int, P]
        L.orc_lin_predictor.argtypes = [P, P, ctypes.c_double, ctypes.c_int, ctypes.c_int, P, P, P]
        L.orc_lin_riemann.argtypes = [P, P, P, P]
        L.orc_lin_corrector.argtypes = [P, ctypes.c_double, P, P, P]
        L.orc_lin_cfl.restype = ctypes.c_double
        L.orc_lin_cfl.argtypes = [P, P, ctypes.c_double]
        L.orc_lin_run.restype = ctypes.c_int
        L.orc_lin_run.argtypes = [P, P, ctypes.c_double, ctypes.c_double, P, ctypes.c_int, P]
        L.orc_lin_energy.restype = ctypes.c_double
        L.orc_lin_energy.argtypes = [P, P, P]
        L.orc_indicator.argtypes = [P, P, P]
        L.orc_volume_transfer.restype = ctypes.c_int
        L.orc_volume_transfer.argtypes = [P, P, P, P]
        L.orc_integral.argtypes = [P, P, P]
        L.orc_subcell_ops.restype = ctypes.c_int
        L.orc_subcell_ops.argtypes = [ctypes.c_int, P, P, P]
        L.orc_limiter_detect.restype = ctypes.c_int
        L.orc_limiter_detect.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, P, P, P]
        L.orc_limited_step.restype = ctypes.c_int
        L.orc_limited_step.argtypes = [P, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int, P, P]
        L.orc_run_limited.restype = ctypes.c_int
        L.orc_run_limited.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_int, P, ctypes.c_int, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def gauss_legendre(N):
    xi, w = np.zeros(N), np.zeros(N)
    assert lib().orc_gauss_legendre(N, _p(xi), _p(w)) == 0
    return xi, w


def basis(N):
    """dict with xi, w, D, L, R, Kinv, Kw (see adg_oracle.c)."""
    xi, w, L, R = (np.zeros(N) for _ in range(4))
    D, Kinv, Kw = (np.zeros((N, N)) for _ in range(3))
    assert lib().orc_basis(N, _p(xi), _p(w), _p(D), _p(L), _p(R), _p(Kinv), _p(Kw)) == 0
    return dict(xi=xi, w=w, D=D, L=L, R=R, Kinv=Kinv, Kw=Kw)


def transfer(N, r, s):
    P, Rm = np.zeros((N, N)), np.zeros((N, N))
    assert lib().orc_transfer(N, r, s, _p(P), _p(Rm)) == 0
    return P, Rm


class Mesh:
    """Leaf mesh of a periodic box: base grid n, recursive 3x3x3 refinement."""

    def __init__(self, order, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), max_level=0, refine=None):
        self.order = int(order)
        self.N = self.order + 1
        n = np.asarray(n, dtype=np.int32)
        lo = _f64(lo)
        hi = _f64(hi)
        ref = np.zeros((0, 4), dtype=np.int32) if refine is None else np.ascontiguousarray(refine, dtype=np.int32)
        h = lib().orc_mesh_build(self.N, _p(n), _p(lo), _p(hi), int(max_level), ref.shape[0], _p(ref))
        if not h:
            raise ValueError("oracle: invalid mesh description")
        self._h = h
        self.nc = lib().orc_mesh_ncells(h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_mesh_free(self._h)
            self._h = None

    def cells(self):
        out = np.zeros((self.nc, 4), dtype=np.int32)
        lib().orc_mesh_cells(self._h, _p(out))
        return out

    def sides(self):
        kind = np.zeros((self.nc, 6), dtype=np.int32)
        nbr = np.zeros((self.nc, 6), dtype=np.int64)
        lib().orc_mesh_sides(self._h, _p(kind), _p(nbr))
        return kind, nbr

    def node_coords(self):
        xyz = np.zeros((3, self.nc, self.N ** 3))
        lib().orc_node_coords(self._h, _p(xyz))
        return xyz

    def cfl(self, u, gamma=1.4, cfl=0.4):
        u = _f64(u)
        st = np.zeros(1, dtype=np.int32)
        dt = lib().orc_cfl(self._h, gamma, cfl, _p(u), _p(st))
        return dt, int(st[0])

    def predictor(self, u, dt, gamma=1.4, npic=None):
        u = _f64(u)
        npic = self.N if npic is None else npic
        us = np.zeros_like(u)
        tr = np.zeros((6, 2, NV, self.nc, self.N ** 2))
        lib().orc_predictor(self._h, gamma, int(npic), float(dt), _p(u), _p(us), _p(tr))
        return us, tr

    def riemann(self, traces, gamma=1.4):
        traces = _f64(traces)
        fs = np.zeros((6, NV, self.nc, self.N ** 2))
        bad = lib().orc_riemann(self._h, gamma, _p(traces), _p(fs))
        return fs, int(bad)

    def corrector(self, ustar, fside, dt):
        ustar, fside = _f64(ustar), _f64(fside)
        un = np.zeros_like(ustar)
        lib().orc_corrector(self._h, float(dt), _p(ustar), _p(fside), _p(un))
        return un

    def run(self, u, nsteps, gamma=1.4, cfl=0.4, npic=None, dt_fixed=0.0, t_end=0.0):
        """Returns (u_final, dt_history, status)."""
        u = np.array(u, dtype=np.float64, copy=True, order="C")
        npic = self.N if npic is None else npic
        hist = np.zeros(max(nsteps, 1))
        rc = lib().orc_run(self._h, gamma, cfl, int(npic), float(dt_fixed), float(t_end), _p(u),
                           int(nsteps), _p(hist))
        return u, hist[:nsteps], int(rc)


def _run_sched(self, u, dt_sched, gamma=1.4, npic=None):
    """Steps with a prescribed dt per step; returns (u_final, status)."""
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    dts = np.ascontiguousarray(dt_sched, dtype=np.float64)
    npic = self.N if npic is None else npic
    rc = lib().orc_run_sched(self._h, gamma, int(npic), _p(dts), _p(u), int(dts.shape[0]))
    return u, int(rc)


def _sample(self, u, pts):
    """Density at points [n, 3] (base-level meshes)."""
    u = _f64(u)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    out = np.zeros(pts.shape[0])
    assert lib().orc_sample(self._h, _p(u), _p(pts), pts.shape[0], _p(out)) == 0
    return out


def _sample_adj(self, pts, wbar, ubar=None):
    """Transpose of sample(): adds wbar_s phi_a(x_s) into the density part of
    ubar (a new zero array if None) and returns it."""
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    wbar = _f64(wbar)
    ubar = np.zeros((NV, self.nc, self.N ** 3)) if ubar is None else np.ascontiguousarray(ubar, dtype=np.float64)
    assert lib().orc_sample_adj(self._h, _p(pts), pts.shape[0], _p(wbar), _p(ubar)) == 0
    return ubar


def _step_tlm(self, u, dt, du, gamma=1.4, npic=None):
    """One step at the fixed dt together with its tangent-linear model.

    du: one direction [5, nc, N^3] or K directions [K, 5, nc, N^3].
    Returns (u_next, du_next of the same shape as du, status); du_next is the
    derivative of the step at u applied to du (face speed differentiated at
    its first maximiser)."""
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    du = np.asarray(du, dtype=np.float64)
    single = du.ndim == 3
    d = np.array(du[None] if single else du, dtype=np.float64, copy=True, order="C")
    npic = self.N if npic is None else npic
    rc = lib().orc_step_tlm(self._h, gamma, int(npic), float(dt), _p(u), int(d.shape[0]), _p(d))
    return u, (d[0] if single else d), int(rc)


def _step_adj(self, u, dt, ubar, gamma=1.4, npic=None):
    """Adjoint of one step at the fixed dt: (d u_next / d u)^T ubar at u.
    Returns (ubar_n, status)."""
    u = _f64(u)
    ubar = _f64(ubar)
    out = np.zeros_like(ubar)
    npic = self.N if npic is None else npic
    rc = lib().orc_step_adj(self._h, gamma, int(npic), float(dt), _p(u), _p(ubar), _p(out))
    return out, int(rc)


def _indicator(self, u):
    """Refinement indicator per cell: max over nodes and axes of the density
    derivative in the cell's reference coordinate (change across the cell)."""
    u = _f64(u)
    out = np.zeros(self.nc)
    lib().orc_indicator(self._h, _p(u), _p(out))
    return out


def _transfer_to(self, u, other):
    """Volumetric data of mesh `other` from this mesh's u (copy, evaluation of
    a coarser cell's polynomial, or L2 projection of finer cells)."""
    u = _f64(u)
    out = np.zeros((5, other.nc, other.N ** 3))
    rc = lib().orc_volume_transfer(self._h, _p(u), other._h, _p(out))
    assert rc == 0, "a cell of the target mesh is only partly covered"
    return out


def _integral(self, u):
    """Integral of every variable over the box."""
    u = _f64(u)
    out = np.zeros(5)
    lib().orc_integral(self._h, _p(u), _p(out))
    return out


def _run_limited(self, u, nsteps, gamma=1.4, cfl=0.4, npic=None, dt_fixed=0.0, delta0=1e-4, eps=1e-3,
                 force=False):
    """Steps with the a-posteriori subcell limiter.  Returns (u_final,
    dt_history, troubled cells per step, flags of the last step, status);
    flags: 1 limited, 2 corrector re-run next to a limited cell, 3 troubled
    but not limitable (a hanging side, adaptive meshes), 0 else."""
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    npic = self.N if npic is None else npic
    hist = np.zeros(max(nsteps, 1))
    nt = np.zeros(max(nsteps, 1), dtype=np.int64)
    flags = np.zeros(self.nc, dtype=np.int32)
    rc = lib().orc_run_limited(self._h, gamma, cfl, int(npic), float(dt_fixed), float(delta0), float(eps),
                               int(bool(force)), _p(u), int(nsteps), _p(hist), _p(nt), _p(flags))
    return u, hist[:nsteps], nt[:nsteps], flags, int(rc)


def _limiter_detect(self, u_old, u_cand, gamma=1.4, delta0=1e-4, eps=1e-3):
    """Troubled flags of a candidate given the old solution: 1 troubled,
    3 troubled with a hanging side (adaptive meshes: cannot be limited), 0
    else."""
    u_old, u_cand = _f64(u_old), _f64(u_cand)
    flags = np.zeros(self.nc, dtype=np.int32)
    rc = lib().orc_limiter_detect(self._h, gamma, float(delta0), float(eps), _p(u_old), _p(u_cand), _p(flags))
    assert rc == 0, rc
    return flags


def subcell_ops(N):
    """(A [ns, N], least-squares inverse [N, ns], face projection B [N, ns])
    of the subcell limiter, ns = 2N - 1."""
    ns = 2 * N - 1
    A, Ap, B = np.zeros((ns, N)), np.zeros((N, ns)), np.zeros((N, ns))
    assert lib().orc_subcell_ops(N, _p(A), _p(Ap), _p(B)) == 0
    return A, Ap, B


NL = 9  # elastic unknowns: s_xx, s_yy, s_zz, s_xy, s_yz, s_xz, v_x, v_y, v_z


def lin_flux_matrix(mat, d):
    """A_d (9 x 9) of the elastic system for material (rho, lambda, mu)."""
    A = np.zeros((NL, NL))
    lib().orc_lin_flux_matrix(_p(_f64(mat)), int(d), _p(A))
    return A


def _lin_predictor(self, mat, u, dt, ck=True, npic=None):
    """(ustar [9, nc, N^3], traces [6, 2, 9, nc, N^2]); material [3, nc]."""
    mat, u = _f64(mat), _f64(u)
    us = np.zeros((NL, self.nc, self.N ** 3))
    tr = np.zeros((6, 2, NL, self.nc, self.N ** 2))
    lib().orc_lin_predictor(self._h, _p(mat), float(dt), int(bool(ck)), int(self.N if npic is None else npic),
                            _p(u), _p(us), _p(tr))
    return us, tr


def _lin_riemann(self, mat, traces):
    fs = np.zeros((6, NL, self.nc, self.N ** 2))
    lib().orc_lin_riemann(self._h, _p(_f64(mat)), _p(_f64(traces)), _p(fs))
    return fs


def _lin_corrector(self, ustar, fside, dt):
    un = np.zeros_like(_f64(ustar))
    lib().orc_lin_corrector(self._h, float(dt), _p(_f64(ustar)), _p(_f64(fside)), _p(un))
    return un


def _lin_run(self, mat, u, nsteps, cfl=0.4, dt_fixed=0.0):
    """Elastic steps (Cauchy-Kowalevski predictor); returns (u, dt)."""
    u = np.array(u, dtype=np.float64, copy=True, order="C")
    dt = np.zeros(1)
    rc = lib().orc_lin_run(self._h, _p(_f64(mat)), float(cfl), float(dt_fixed), _p(u), int(nsteps), _p(dt))
    assert rc == 0, rc
    return u, float(dt[0])


def _lin_cfl(self, mat, cfl=0.4):
    return lib().orc_lin_cfl(self._h, _p(_f64(mat)), float(cfl))


def _lin_energy(self, mat, u):
    return lib().orc_lin_energy(self._h, _p(_f64(mat)), _p(_f64(u)))


Mesh.lin_predictor = _lin_predictor
Mesh.lin_riemann = _lin_riemann
Mesh.lin_corrector = _lin_corrector
Mesh.lin_run = _lin_run
Mesh.lin_cfl = _lin_cfl
Mesh.lin_energy = _lin_energy
Mesh.run_limited = _run_limited
Mesh.limiter_detect = _limiter_detect
Mesh.run_sched = _run_sched
Mesh.sample = _sample
Mesh.sample_adj = _sample_adj
Mesh.step_tlm = _step_tlm
Mesh.step_adj = _step_adj
Mesh.indicator = _indicator
Mesh.transfer_to = _transfer_to
Mesh.integral = _integral


def adapt_plan(cells, refine, eta, theta_refine, theta_coarsen, max_level):
    """The next refine list (rows (level, i, j, k), sorted by (level, k, j, i))
    from the current one, written out plainly (test reference).

    cells: [nc, 4] (level, i, j, k) of the leaves; refine: rows of the current
    mesh; eta: indicator per leaf.  A leaf with eta > theta_refine below
    max_level is split; a parent whose 27 children are all leaves, none split
    now, all with eta < theta_coarsen, is merged (its row is dropped)."""
    rows = {tuple(int(x) for x in r) for r in np.asarray(refine, dtype=np.int64).reshape(-1, 4)}
    leaf = {tuple(int(x) for x in c): i for i, c in enumerate(np.asarray(cells).reshape(-1, 4))}
    split = {c for c, i in leaf.items() if eta[i] > theta_refine and c[0] < max_level}
    merged = set()
    for r in rows:
        l, i, j, k = r
        kids = [(l + 1, 3 * i + a, 3 * j + b, 3 * k + c) for c in range(3) for b in range(3) for a in range(3)]
        if all(q in leaf and q not in split and eta[leaf[q]] < theta_coarsen for q in kids):
            merged.add(r)
    new = (rows - merged) | split
    return np.array(sorted(new, key=lambda r: (r[0], r[3], r[2], r[1])), dtype=np.int32).reshape(-1, 4)


def num_threads():
    return lib().orc_num_threads()
