"""MI355X-native ADER-DG time step for the 3-D compressible Euler equations.

Thin Python binding of the C ABI in include/adg.h (libadg.so, built in-tree by
``python -m paper_1806_07984_amd.build``).  This module only marshals
arguments: every phase of the step runs in the library's HIP kernels.  PyTorch
supplies device memory and streams.  If the library is missing, loading fails
with an error; there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadg.so")

NV = 5
FP64, FP32_MFMA = 0, 1
NOALLOC_WORKSPACE_BYTES = 64 * 1024 * 1024  # ADG_NOALLOC_WORKSPACE_BYTES

STATUS = {0: "OK", 1: "INVALID_ARG", 2: "UNSUPPORTED", 3: "OOM", 4: "HIP", 5: "NONPHYSICAL", 6: "WORKSPACE"}

EXPORTS = ["adg_init_mesh", "adg_free_mesh", "adg_mesh_info", "adg_instance_info", "adg_mesh_cells",
           "adg_node_coords", "adg_cfl", "adg_predictor", "adg_riemann", "adg_corrector", "adg_step",
           "adg_profile", "adg_profile_read", "adg_get_status", "adg_last_error", "adg_autotune",
           "adg_tuning", "adg_set_options", "adg_step_adjoint", "adg_sample", "adg_sample_adjoint",
           "adg_set_switch_tape", "adg_set_pipeline", "adg_indicator", "adg_adapt_plan", "adg_transfer",
           "adg_set_limiter", "adg_limiter_stats", "adg_lin_init", "adg_lin_free", "adg_lin_info", "adg_lin_dt",
           "adg_lin_predictor", "adg_lin_step", "adg_step_noalloc", "adg_adapt_plan_mesh",
           "adg_step_record", "adg_step_adjoint_tape", "adg_set_face_fusion", "adg_lin_set_face_fusion"]
PHASES = ["cfl", "predictor", "hanging", "riemann", "corrector", "limiter"]


class AdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"adg error {STATUS.get(code, code)}: {msg}")
        self.code = code


class InstanceDesc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("periodic_mask", ctypes.c_uint32), ("max_level", ctypes.c_int32),
                ("n_refine", ctypes.c_int64), ("refine", ctypes.c_void_p), ("gamma", ctypes.c_double),
                ("cfl", ctypes.c_double), ("picard_iters", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_int32), ("n_cells", ctypes.c_int64), ("n_dofs", ctypes.c_int64),
                ("u_elems", ctypes.c_int64), ("trace_elems", ctypes.c_int64), ("fside_elems", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("n_conforming_faces", ctypes.c_int64),
                ("n_hanging_faces", ctypes.c_int64), ("n_skeleton_cells", ctypes.c_int64),
                ("real_bytes", ctypes.c_int32), ("adjoint_workspace_bytes", ctypes.c_int64),
                ("adjoint_tape_bytes", ctypes.c_int64)]


class InstanceGeom(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("n_cells", ctypes.c_int64), ("cell_offset", ctypes.c_int64),
                ("u_offset", ctypes.c_int64), ("trace_offset", ctypes.c_int64), ("fside_offset", ctypes.c_int64)]


class LinDesc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("cfl", ctypes.c_double)]


_lib = None


def load():
    """Load libadg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_1806_07984_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "adg_init_mesh": [ctypes.POINTER(InstanceDesc), I32, I32, ctypes.POINTER(P)],
        "adg_free_mesh": [P],
        "adg_mesh_info": [P, ctypes.POINTER(Info)],
        "adg_instance_info": [P, I32, ctypes.POINTER(InstanceGeom)],
        "adg_mesh_cells": [P, P],
        "adg_node_coords": [P, P, P],
        "adg_cfl": [P, P, P, P],
        "adg_predictor": [P, P, P, P, P, P],
        "adg_riemann": [P, P, P, P],
        "adg_corrector": [P, P, P, P, P, P],
        "adg_step": [P, P, I32, ctypes.c_double, P, P, P, P],
        "adg_step_noalloc": [P, P, I32, ctypes.c_double, P, P],
        "adg_get_status": [P],
        "adg_profile": [P, I32],
        "adg_profile_read": [P, P, P],
        "adg_autotune": [P, P, P, P],
        "adg_tuning": [P, P],
        "adg_set_options": [P, I32, I32],
        "adg_set_pipeline": [P, I32],
        "adg_step_adjoint": [P, P, P, P, P, P, P],
        "adg_step_record": [P, P, P, P, P, P, P],
        "adg_set_face_fusion": [P, I32],
        "adg_step_adjoint_tape": [P, P, P, P, P, P, P, P],
        "adg_set_switch_tape": [P, P, I32],
        "adg_sample": [P, P, P, I64, P, P],
        "adg_sample_adjoint": [P, P, P, I64, P, P],
        "adg_indicator": [P, P, P, P],
        "adg_adapt_plan": [P, P, ctypes.c_double, ctypes.c_double, P, I64, P],
        "adg_adapt_plan_mesh": [P, P, ctypes.c_double, ctypes.c_double, P, I64, P],
        "adg_transfer": [P, P, P, P, P],
        "adg_set_limiter": [P, I32, ctypes.c_double, ctypes.c_double],
        "adg_limiter_stats": [P, P, P, P, P],
        "adg_lin_init": [ctypes.POINTER(LinDesc), ctypes.POINTER(P)],
        "adg_lin_free": [P],
        "adg_lin_info": [P, P, P, P, P, P],
        "adg_lin_dt": [P, P, P, P],
        "adg_lin_predictor": [P, P, P, P, P, P, P],
        "adg_lin_step": [P, P, P, I32, P, P, P],
        "adg_lin_set_face_fusion": [P, I32],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = None if name == "adg_free_mesh" else ctypes.c_int
    L.adg_last_error.restype = ctypes.c_char_p
    L.adg_last_error.argtypes = []
    _lib = L
    return L


def _check(code):
    if code != 0:
        raise AdgError(code, load().adg_last_error().decode())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, dtype, numel, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def instance(order, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), max_level=0, refine=None, gamma=1.4, cfl=0.4,
             picard_iters=0):
    """Descriptor of one periodic box (see adg_instance_desc)."""
    return dict(order=order, n=tuple(n), lo=tuple(lo), hi=tuple(hi), max_level=max_level, refine=refine,
                gamma=gamma, cfl=cfl, picard_iters=picard_iters)


def _fill_desc(a, d):
    """Fills the InstanceDesc a from the dict d; returns the refine array that
    must stay alive while a is used."""
    ref = np.zeros((0, 4), dtype=np.int32) if d.get("refine") is None else \
        np.ascontiguousarray(d["refine"], dtype=np.int32).reshape(-1, 4)
    a.order = d["order"]
    a.n[:] = list(d["n"])
    a.lo[:] = list(d.get("lo", (0.0, 0.0, 0.0)))
    a.hi[:] = list(d.get("hi", (1.0, 1.0, 1.0)))
    a.periodic_mask = 7
    a.max_level = d.get("max_level", 0)
    a.n_refine = ref.shape[0]
    a.refine = ref.ctypes.data if ref.shape[0] else None
    a.gamma = d.get("gamma", 1.4)
    a.cfl = d.get("cfl", 0.4)
    a.picard_iters = d.get("picard_iters", 0)
    return ref


def adapt_plan(desc, eta, theta_refine, theta_coarsen):
    """Refine rows [n, 4] (int32) of the next mesh (adg_adapt_plan; host only).
    desc: the instance dict of the current mesh; eta: indicator per cell."""
    L = load()
    a = InstanceDesc()
    keep = _fill_desc(a, desc)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    n = ctypes.c_int64(0)
    # at most the current rows plus one per cell above the refinement threshold
    cap = keep.shape[0] + int(np.count_nonzero(eta > theta_refine))
    out = np.zeros((max(cap, 1), 4), dtype=np.int32)
    _check(L.adg_adapt_plan(ctypes.byref(a), eta.ctypes.data, float(theta_refine), float(theta_coarsen),
                            out.ctypes.data, out.shape[0], ctypes.byref(n)))
    del keep
    return out[: n.value]


def adapt(mesh, u, theta_refine, theta_coarsen, stream=None):
    """One adaptation step of a single-instance handle: indicator, plan, new
    handle, transfer of the state.  Returns (new_mesh, new_u); the old handle
    is left open (close it when done)."""
    import torch
    eta = mesh.indicator(u, stream=stream)
    rows = mesh.adapt_plan(eta.cpu().numpy(), theta_refine, theta_coarsen)
    desc = dict(mesh.descs[0], refine=rows)
    new = Mesh(desc, mesh.precision)
    u_new = torch.empty(new.info["u_elems"], dtype=torch.float64, device=u.device)
    mesh.transfer_to(u, new, u_new, stream=stream)
    return new, u_new


class Mesh:
    """Handle over one or more instances (adg_init_mesh).

    precision: "fp64" (ADG_FP64) or "fp32" (ADG_FP32_MFMA)."""

    def __init__(self, descs, precision="fp64"):
        L = load()
        if isinstance(descs, dict):
            descs = [descs]
        self.precision = precision
        prec = {"fp64": FP64, "fp32": FP32_MFMA}[precision]
        arr = (InstanceDesc * len(descs))()
        self._keep = [_fill_desc(arr[i], d) for i, d in enumerate(descs)]
        self.descs = [dict(d) for d in descs]
        h = ctypes.c_void_p()
        _check(L.adg_init_mesh(arr, len(descs), prec, ctypes.byref(h)))
        self._h = h
        info = Info()
        _check(L.adg_mesh_info(self._h, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in Info._fields_}
        self.instances = []
        for i in range(len(descs)):
            g = InstanceGeom()
            _check(L.adg_instance_info(self._h, i, ctypes.byref(g)))
            self.instances.append({k: getattr(g, k) for k, _ in InstanceGeom._fields_})
        self.n_instances = len(descs)

    def close(self):
        if getattr(self, "_h", None):
            load().adg_free_mesh(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- sizes and allocation ------------------------------------------------
    @property
    def real_dtype(self):
        import torch
        return torch.float64 if self.precision == "fp64" else torch.float32

    def empty_u(self, device="cuda"):
        import torch
        return torch.empty(self.info["u_elems"], dtype=torch.float64, device=device)

    def empty_traces(self, device="cuda"):
        import torch
        return torch.empty(self.info["trace_elems"], dtype=self.real_dtype, device=device)

    def empty_fside(self, device="cuda"):
        import torch
        return torch.empty(self.info["fside_elems"], dtype=self.real_dtype, device=device)

    def empty_workspace(self, device="cuda"):
        import torch
        return torch.empty(self.info["workspace_bytes"], dtype=torch.uint8, device=device)

    def cells(self):
        out = np.zeros((self.info["n_cells"], 4), dtype=np.int32)
        _check(load().adg_mesh_cells(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    # -- calls ---------------------------------------------------------------
    def node_coords(self, stream=None):
        import torch
        xyz = torch.empty(3 * self.info["u_elems"] // NV, dtype=torch.float64, device="cuda")
        _check(load().adg_node_coords(self._h, _ptr(xyz, torch.float64, None, "xyz"), _stream(stream)))
        return xyz

    def cfl(self, u, dt, stream=None):
        import torch
        _check(load().adg_cfl(self._h, _ptr(u, torch.float64, self.info["u_elems"], "u"),
                              _ptr(dt, torch.float64, self.n_instances, "dt"), _stream(stream)))

    def predictor(self, u, dt, ustar, traces, stream=None):
        import torch
        n = self.info["u_elems"]
        _check(load().adg_predictor(self._h, _ptr(u, torch.float64, n, "u"),
                                    _ptr(dt, torch.float64, self.n_instances, "dt"),
                                    _ptr(ustar, torch.float64, n, "ustar"),
                                    _ptr(traces, self.real_dtype, self.info["trace_elems"], "traces"),
                                    _stream(stream)))

    def riemann(self, traces, fside, stream=None):
        _check(load().adg_riemann(self._h, _ptr(traces, self.real_dtype, self.info["trace_elems"], "traces"),
                                  _ptr(fside, self.real_dtype, self.info["fside_elems"], "fside"),
                                  _stream(stream)))

    def corrector(self, ustar, fside, dt, uout, stream=None):
        import torch
        n = self.info["u_elems"]
        _check(load().adg_corrector(self._h, _ptr(ustar, torch.float64, n, "ustar"),
                                    _ptr(fside, self.real_dtype, self.info["fside_elems"], "fside"),
                                    _ptr(dt, torch.float64, self.n_instances, "dt"),
                                    _ptr(uout, torch.float64, n, "uout"), _stream(stream)))

    def step(self, u, n_steps, ws, dt_hist=None, stream_skeleton=None, stream_enclave=None, t_end=0.0):
        """n_steps whole steps in place on u (adg_step); t_end > 0 stops the
        run at that time, measured from the state's time at the call."""
        import torch
        hist = ctypes.c_void_p(0) if dt_hist is None else \
            _ptr(dt_hist, torch.float64, n_steps * self.n_instances, "dt_hist")
        s1 = _stream(stream_skeleton)
        s2 = _stream(stream_enclave) if stream_enclave is not None else s1
        if ws.numel() < self.info["workspace_bytes"]:
            raise ValueError("workspace too small")
        _check(load().adg_step(self._h, _ptr(u, torch.float64, self.info["u_elems"], "u"), int(n_steps),
                               float(t_end), hist, ctypes.c_void_p(ws.data_ptr()), s1, s2))

    def step_noalloc(self, u, n_steps, dt_hist=None, stream=None, t_end=0.0):
        """n_steps whole steps in place on u with the library's static
        workspace instead of a caller buffer (adg_step_noalloc)."""
        import torch
        hist = ctypes.c_void_p(0) if dt_hist is None else \
            _ptr(dt_hist, torch.float64, n_steps * self.n_instances, "dt_hist")
        _check(load().adg_step_noalloc(self._h, _ptr(u, torch.float64, self.info["u_elems"], "u"), int(n_steps),
                                       float(t_end), hist, _stream(stream)))

    def autotune(self, u, ws, stream=None):
        """Pick the cells per work item of every order by timing (adg_autotune)."""
        import torch
        _check(load().adg_autotune(self._h, _ptr(u, torch.float64, self.info["u_elems"], "u"),
                                   ctypes.c_void_p(ws.data_ptr()), _stream(stream)))

    def tuning(self):
        out = np.zeros(8, dtype=np.int32)
        _check(load().adg_tuning(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return {N: int(out[N - 1]) for N in range(1, 9)}

    def set_options(self, use_graph=True, batched=None):
        """batched: 0 per-instance launches, 1 one persistent launch per order,
        2 one persistent launch for all orders (None: 1 if the handle can batch)."""
        if batched is None:
            batched = 1 if (self.n_instances > 1 and self.info["n_hanging_faces"] == 0) else 0
        _check(load().adg_set_options(self._h, 1 if use_graph else 0, int(batched)))

    def set_pipeline(self, mode):
        """Pipelined step over cell chunks (single instance, no hanging faces):
        0/False off, 1/True predictor and face/corrector streams, 2 one stream."""
        _check(load().adg_set_pipeline(self._h, int(mode)))

    def set_face_fusion(self, enable):
        """Riemann problems solved inside the corrector (adg_set_face_fusion;
        one uniform instance at p = 3; on by default, same bits either way)."""
        _check(load().adg_set_face_fusion(self._h, int(bool(enable))))

    def set_limiter(self, mode, delta0=1e-4, eps=1e-3):
        """A-posteriori subcell limiter: 0/False off, 1/True on, 2 every cell
        limited (test hook); delta0, eps: relaxation of the bounds."""
        _check(load().adg_set_limiter(self._h, int(mode), float(delta0), float(eps)))

    def limiter_stats(self, flags=False, stream=None, device="cuda"):
        """(limited cells, cells whose corrector ran again) of the last step,
        plus the per-cell flags (int32 tensor: 1 limited, 2 re-run, 0 else)
        if flags; synchronises the stream."""
        import torch
        nl = ctypes.c_int64(0)
        nr = ctypes.c_int64(0)
        f = torch.empty(self.info["n_cells"], dtype=torch.int32, device=device) if flags else None
        _check(load().adg_limiter_stats(self._h, ctypes.byref(nl), ctypes.byref(nr),
                                        ctypes.c_void_p(f.data_ptr()) if flags else None, _stream(stream)))
        return (nl.value, nr.value, f) if flags else (nl.value, nr.value)

    def profile(self, enable, predictor_only=False):
        """Enable (and clear) or disable HIP-event timing of every phase (or of
        the predictor launches only)."""
        _check(load().adg_profile(self._h, (2 if predictor_only else 1) if enable else 0))

    def profile_read(self):
        """{phase: (milliseconds summed over launches, launch count)}; synchronises."""
        ms = np.zeros(len(PHASES))
        cnt = np.zeros(len(PHASES), dtype=np.int64)
        _check(load().adg_profile_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                       cnt.ctypes.data_as(ctypes.c_void_p)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PHASES)}

    def set_switch_tape(self, tape, mode):
        """mode 0 off, 1 record, 2 replay; tape: int16 tensor of n_conforming_faces."""
        import torch
        ptr = ctypes.c_void_p(0) if tape is None else _ptr(tape, torch.int16, self.info["n_conforming_faces"], "tape")
        _check(load().adg_set_switch_tape(self._h, ptr, int(mode)))

    def empty_adjoint_workspace(self, device="cuda"):
        import torch
        return torch.empty(self.info["adjoint_workspace_bytes"], dtype=torch.uint8, device=device)

    def step_adjoint(self, u, dt, ubar_next, ubar, ws, stream=None):
        """ubar = (d step(u; dt) / du)^T ubar_next at fixed dt (adg_step_adjoint)."""
        import torch
        n = self.info["u_elems"]
        if ws.numel() < self.info["adjoint_workspace_bytes"]:
            raise ValueError("adjoint workspace too small")
        _check(load().adg_step_adjoint(self._h, _ptr(u, torch.float64, n, "u"),
                                       _ptr(dt, torch.float64, self.n_instances, "dt"),
                                       _ptr(ubar_next, torch.float64, n, "ubar_next"),
                                       _ptr(ubar, torch.float64, n, "ubar"), ctypes.c_void_p(ws.data_ptr()),
                                       _stream(stream)))

    def empty_tape(self, device="cuda"):
        import torch
        return torch.empty(self.info["adjoint_tape_bytes"], dtype=torch.uint8, device=device)

    def step_record(self, u, dt, u_next, tape, ws, stream=None):
        """u_next = step(u; dt) at fixed dt, keeping what its adjoint reads in
        tape (adg_step_record); u_next may be u, or None for the tape only;
        tape None: a plain step at the fixed dt."""
        import torch
        n = self.info["u_elems"]
        if ws.numel() < self.info["adjoint_workspace_bytes"] or (
                tape is not None and tape.numel() < self.info["adjoint_tape_bytes"]):
            raise ValueError("tape or adjoint workspace too small")
        if tape is None and u_next is None:
            raise ValueError("a step without a tape needs u_next")
        _check(load().adg_step_record(self._h, _ptr(u, torch.float64, n, "u"),
                                      _ptr(dt, torch.float64, self.n_instances, "dt"),
                                      None if u_next is None else _ptr(u_next, torch.float64, n, "u_next"),
                                      None if tape is None else ctypes.c_void_p(tape.data_ptr()),
                                      ctypes.c_void_p(ws.data_ptr()), _stream(stream)))

    def step_adjoint_tape(self, u, dt, tape, ubar_next, ubar, ws, stream=None):
        """step_adjoint of the step recorded in tape from the same u and dt
        (adg_step_adjoint_tape)."""
        import torch
        n = self.info["u_elems"]
        if tape.numel() < self.info["adjoint_tape_bytes"] or ws.numel() < self.info["adjoint_workspace_bytes"]:
            raise ValueError("tape or adjoint workspace too small")
        _check(load().adg_step_adjoint_tape(self._h, _ptr(u, torch.float64, n, "u"),
                                            _ptr(dt, torch.float64, self.n_instances, "dt"),
                                            ctypes.c_void_p(tape.data_ptr()),
                                            _ptr(ubar_next, torch.float64, n, "ubar_next"),
                                            _ptr(ubar, torch.float64, n, "ubar"), ctypes.c_void_p(ws.data_ptr()),
                                            _stream(stream)))

    def sample(self, u, pts, out, stream=None):
        """Density at points pts [n, 3] (adg_sample)."""
        import torch
        _check(load().adg_sample(self._h, _ptr(u, torch.float64, self.info["u_elems"], "u"),
                                 _ptr(pts, torch.float64, None, "pts"), pts.shape[0],
                                 _ptr(out, torch.float64, pts.shape[0], "out"), _stream(stream)))

    def sample_adjoint(self, pts, wbar, ubar, stream=None):
        """ubar[density] += sum_s wbar[s] phi(x_s) (adg_sample_adjoint)."""
        import torch
        _check(load().adg_sample_adjoint(self._h, _ptr(pts, torch.float64, None, "pts"),
                                         _ptr(wbar, torch.float64, pts.shape[0], "wbar"), pts.shape[0],
                                         _ptr(ubar, torch.float64, self.info["u_elems"], "ubar"),
                                         _stream(stream)))

    def indicator(self, u, eta=None, stream=None):
        """Refinement indicator per cell (adg_indicator); returns eta (FP64)."""
        import torch
        if eta is None:
            eta = torch.empty(self.info["n_cells"], dtype=torch.float64, device=u.device)
        _check(load().adg_indicator(self._h, _ptr(u, torch.float64, self.info["u_elems"], "u"),
                                    _ptr(eta, torch.float64, self.info["n_cells"], "eta"), _stream(stream)))
        return eta

    def adapt_plan(self, eta, theta_refine, theta_coarsen):
        """Refine rows [n, 4] (int32) of the next mesh of this single-instance
        handle (adg_adapt_plan_mesh; host only, eta on the host)."""
        eta = np.ascontiguousarray(eta, dtype=np.float64)
        if eta.shape != (self.info["n_cells"],):
            raise ValueError("eta needs one value per cell")
        n = ctypes.c_int64(0)
        ref = self.descs[0].get("refine")
        n_rows = 0 if ref is None else np.asarray(ref).reshape(-1, 4).shape[0]
        # at most the current rows plus one per cell above the refinement threshold
        cap = n_rows + int(np.count_nonzero(eta > theta_refine))
        out = np.zeros((max(cap, 1), 4), dtype=np.int32)
        _check(load().adg_adapt_plan_mesh(self._h, eta.ctypes.data, float(theta_refine), float(theta_coarsen),
                                          out.ctypes.data, out.shape[0], ctypes.byref(n)))
        return out[: n.value]

    def transfer_to(self, u, other, u_other=None, stream=None):
        """State of handle `other` from this handle's u (adg_transfer)."""
        import torch
        if u_other is None:
            u_other = torch.empty(other.info["u_elems"], dtype=torch.float64, device=u.device)
        _check(load().adg_transfer(self._h, _ptr(u, torch.float64, self.info["u_elems"], "u"), other._h,
                                   _ptr(u_other, torch.float64, other.info["u_elems"], "u_other"),
                                   _stream(stream)))
        return u_other

    def status(self):
        """Synchronises; raises AdgError(NONPHYSICAL) if a bad state was met."""
        _check(load().adg_get_status(self._h))


class LinMesh:
    """Linear variant: elastic waves (9 unknowns) on a uniform periodic box
    with the Cauchy-Kowalevski predictor (adg_lin_*).  material: float64
    tensor [3, n_cells] (rho, lambda, mu); u: float64 [9, n_cells, N^3]."""

    def __init__(self, order, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), cfl=0.4):
        L = load()
        d = LinDesc()
        d.order = int(order)
        for a in range(3):
            d.n[a], d.lo[a], d.hi[a] = int(n[a]), float(lo[a]), float(hi[a])
        d.cfl = float(cfl)
        h = ctypes.c_void_p()
        _check(L.adg_lin_init(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.N = int(order) + 1
        vals = [ctypes.c_int64(0) for _ in range(5)]
        _check(L.adg_lin_info(self._h, *[ctypes.byref(v) for v in vals]))
        self.info = dict(zip(["n_cells", "u_elems", "trace_elems", "fside_elems", "workspace_bytes"],
                             [v.value for v in vals]))

    def close(self):
        if getattr(self, "_h", None):
            load().adg_lin_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_workspace(self, device="cuda"):
        import torch
        return torch.empty(self.info["workspace_bytes"], dtype=torch.uint8, device=device)

    def dt(self, material, stream=None):
        import torch
        out = torch.empty(1, dtype=torch.float64, device=material.device)
        _check(load().adg_lin_dt(self._h, _ptr(material, torch.float64, 3 * self.info["n_cells"], "material"),
                                 _ptr(out, torch.float64, 1, "dt"), _stream(stream)))
        return out

    def predictor(self, material, u, dt, stream=None):
        """(ustar, traces) of the Cauchy-Kowalevski predictor at the dt in the
        one-element device tensor dt."""
        import torch
        ustar = torch.empty(self.info["u_elems"], dtype=torch.float64, device=u.device)
        traces = torch.empty(self.info["trace_elems"], dtype=torch.float64, device=u.device)
        _check(load().adg_lin_predictor(self._h, _ptr(material, torch.float64, 3 * self.info["n_cells"], "material"),
                                        _ptr(u, torch.float64, self.info["u_elems"], "u"),
                                        _ptr(dt, torch.float64, 1, "dt"), ctypes.c_void_p(ustar.data_ptr()),
                                        ctypes.c_void_p(traces.data_ptr()), _stream(stream)))
        return ustar, traces

    def set_face_fusion(self, enable):
        """Faces inside the corrector at p = 3 (adg_lin_set_face_fusion; on by
        default, the same bits either way)."""
        _check(load().adg_lin_set_face_fusion(self._h, int(bool(enable))))

    def step(self, material, u, n_steps, ws, dt_out=None, stream=None):
        import torch
        _check(load().adg_lin_step(self._h, _ptr(material, torch.float64, 3 * self.info["n_cells"], "material"),
                                   _ptr(u, torch.float64, self.info["u_elems"], "u"), int(n_steps),
                                   ctypes.c_void_p(0) if dt_out is None else _ptr(dt_out, torch.float64, 1, "dt_out"),
                                   ctypes.c_void_p(ws.data_ptr()), _stream(stream)))
