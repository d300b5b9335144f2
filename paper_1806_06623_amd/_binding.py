"""ctypes binding of the C ABI in include/sphpoisson.h (argument marshalling only)."""
import ctypes
import os

import numpy as np
# torch first: it maps its own HIP runtime (libamdhip64.so.7), and the library
# must bind to that same runtime instance.  Loading the library first would map
# a second HIP/HSA runtime from /opt/rocm next to torch's, and device handles
# (streams, memory) of one are unknown to the other.
import torch  # noqa: F401

# SPP_LIB names another build of the same library (the host-sanitized one of
# the host-side tests); by default the library next to this file
LIB_PATH = os.environ.get("SPP_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsphpoisson.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_1806_06623_amd/build.py` "
        "(there is no CPU fallback)")

lib = ctypes.CDLL(LIB_PATH)

_c_int, _c_double, _c_size_t, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)

lib.spp_grid_create.argtypes = [_c_int, _dp, _c_int, _dp, _c_int, _c_int, ctypes.POINTER(_vp)]
lib.spp_grid_create.restype = _c_int
lib.spp_grid_destroy.argtypes = [_vp]
lib.spp_grid_destroy.restype = None
lib.spp_plan_create.argtypes = [_vp, ctypes.POINTER(_vp)]
lib.spp_plan_create.restype = _c_int
lib.spp_plan_destroy.argtypes = [_vp]
lib.spp_plan_destroy.restype = None
lib.spp_plan_device_bytes.argtypes = [_vp, ctypes.POINTER(_c_size_t), ctypes.POINTER(_c_size_t)]
lib.spp_plan_device_bytes.restype = _c_int
lib.spp_plan_upload.argtypes = [_vp, _vp, _vp]
lib.spp_plan_upload.restype = _c_int
lib.spp_solve.argtypes = [_vp, _vp, _vp, _c_double, _vp, _vp]
lib.spp_solve.restype = _c_int
lib.spp_solve_noalloc.argtypes = [_vp, _vp, _vp, _c_double, _vp]
lib.spp_solve_noalloc.restype = _c_int
lib.spp_solve_profiled.argtypes = [_vp, _vp, _vp, _c_double, _vp, _vp, _dp]
lib.spp_solve_profiled.restype = _c_int
lib.spp_face_fluxes.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
lib.spp_face_fluxes.restype = _c_int
lib.spp_plan_workspace_bytes.argtypes = [_vp, _c_int, ctypes.POINTER(_c_size_t)]
lib.spp_plan_workspace_bytes.restype = _c_int
lib.spp_solve_mixed.argtypes = [_vp, _c_int, _c_int, _c_int, _vp, _vp, _c_double, _vp, _vp]
lib.spp_solve_mixed.restype = _c_int
lib.spp_momentum_source.argtypes = [_vp, _vp, _c_double, _vp, _vp, _vp, _vp, _vp]
lib.spp_momentum_source.restype = _c_int
lib.spp_residual.argtypes = [_vp, _vp, _vp, _c_double, _vp, _vp, _vp]
lib.spp_residual.restype = _c_int
lib.spp_plan_scale_lowprec_basis.argtypes = [_vp, _c_double]
lib.spp_plan_scale_lowprec_basis.restype = _c_int


class _SolveInfo(ctypes.Structure):
    _fields_ = [("refine_iters", _c_int), ("first_residual_rel", _c_double), ("last_residual_rel", _c_double),
                ("not_contracted", _c_int), ("fell_back_fp64", _c_int), ("nonfinite", _c_int)]


lib.spp_solve_status.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_SolveInfo)]
lib.spp_solve_status.restype = _c_int
lib.spp_batch_status.argtypes = [_vp, _c_int, _vp, ctypes.POINTER(_SolveInfo)]
lib.spp_batch_status.restype = _c_int


def _info_dict(st, info):
    d = {f: getattr(info, f) for f, _ in _SolveInfo._fields_}
    d["status"] = STATUS_NAMES.get(st, st)
    return d
lib.spp_autotune_projection.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_c_int)]
lib.spp_autotune_projection.restype = _c_int
_vpp = ctypes.POINTER(_vp)
lib.spp_batch_workspace_bytes.argtypes = [_c_int, _vpp, _c_int, ctypes.POINTER(_c_size_t)]
lib.spp_batch_workspace_bytes.restype = _c_int
lib.spp_batch_create.argtypes = [_c_int, _vpp, _vpp, _vpp, _dp, _c_int, _c_int, _c_int, _vp, _vp, ctypes.POINTER(_vp)]
lib.spp_batch_create.restype = _c_int
lib.spp_batch_describe.argtypes = [_vp, ctypes.c_char_p, _c_size_t, ctypes.POINTER(_c_size_t)]
lib.spp_batch_describe.restype = _c_int
lib.spp_batch_launch.argtypes = [_vp, _vp]
lib.spp_batch_launch.restype = _c_int
lib.spp_batch_destroy.argtypes = [_vp]
lib.spp_batch_destroy.restype = None
lib.spp_solve_batched.argtypes = [_c_int, _vpp, _vpp, _vpp, _dp, _c_int, _c_int, _vp, _vp]
lib.spp_solve_batched.restype = _c_int


class _Request(ctypes.Structure):
    _fields_ = [("plan_index", _c_int), ("rho_dev", _vp), ("phi_dev", _vp), ("G", _c_double),
                ("request_id", ctypes.c_longlong), ("ready_event", _vp), ("precision", _c_int),
                ("n_refine", _c_int)]


class _Completion(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_longlong), ("plan_index", _c_int), ("t_arrival", _c_double),
                ("t_admit", _c_double), ("t_done", _c_double), ("status", _c_int)]


lib.spp_server_create.argtypes = [_c_int, _vpp, _vp, _c_size_t, _c_int, ctypes.POINTER(_vp)]
lib.spp_server_create.restype = _c_int
lib.spp_server_submit.argtypes = [_vp, ctypes.POINTER(_Request), _c_double]
lib.spp_server_submit.restype = _c_int
lib.spp_server_poll.argtypes = [_vp, ctypes.POINTER(_Completion), _c_int, ctypes.POINTER(_c_int)]
lib.spp_server_poll.restype = _c_int
lib.spp_server_drain.argtypes = [_vp, _c_double]
lib.spp_server_drain.restype = _c_int
lib.spp_server_now.argtypes = [_vp, ctypes.POINTER(_c_double)]
lib.spp_server_now.restype = _c_int
lib.spp_server_destroy.argtypes = [_vp]
lib.spp_server_destroy.restype = None
lib.spp_plan_parity_split.argtypes = [_vp, ctypes.POINTER(_c_int)]
lib.spp_plan_parity_split.restype = _c_int
lib.spp_plan_set_path.argtypes = [_vp, _c_int]
lib.spp_plan_set_path.restype = _c_int
lib.spp_plan_get_path.argtypes = [_vp, ctypes.POINTER(_c_int)]
lib.spp_plan_get_path.restype = _c_int
lib.spp_theta_eigensystem.argtypes = [_vp, _c_int, _dp, _dp]
lib.spp_theta_eigensystem.restype = _c_int
lib.spp_plan_kernels.argtypes = [_vp, ctypes.c_char_p, _c_size_t, ctypes.POINTER(_c_size_t)]
lib.spp_plan_kernels.restype = _c_int
lib.spp_plan_shape.argtypes = [_vp, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_int)]
lib.spp_plan_shape.restype = _c_int
lib.spp_last_error.argtypes = []
lib.spp_last_error.restype = ctypes.c_char_p
lib.spp_stream_copy.argtypes = [_vp, _vp, _c_size_t, _vp]
lib.spp_stream_copy.restype = _c_int

precision_codes = {"fp64": 0, "mixed_fp32": 1, "mixed_bf16x3": 2}
inner_codes = {"auto": 0, "zero_flux": 1, "regular": 2}
STATUS_NAMES = {0: "ok", -1: "einval", -2: "enotsup", -3: "edevice", -4: "enomem", -5: "estate",
                -6: "enonfinite", -7: "enoconv"}


class SphPoissonError(RuntimeError):
    def __init__(self, status, where):
        msg = lib.spp_last_error().decode(errors="replace")
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def _check(status, where):
    if status != 0:
        raise SphPoissonError(status, where)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def stream_copy(src, dst, stream=None):
    """Enqueue spp_stream_copy of the contiguous CUDA tensor src into dst (same
    number of bytes, a multiple of 16) on ``stream`` (default: the current
    torch stream): the streaming-rate reference of the memory-bound kernels
    (include/spp_reference.h)."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("stream_copy: contiguous CUDA tensors required")
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy: src and dst differ in size")
    _check(lib.spp_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                               _stream_ptr(stream)), "spp_stream_copy")


class Plan:
    """Grid + set-up (host eigensolves) + device-resident tables.

    ``Plan(r_if, th_if, nphi)`` creates the grid and the plan, allocates the
    plan buffer and one workspace as torch uint8 tensors on ``device`` and
    uploads the tables.  ``solve(rho)`` enqueues one solve on the current
    torch stream and returns Phi (float64, same shape as rho).
    """

    def __init__(self, r_if, th_if, nphi, device="cuda", inner="auto"):
        import torch
        r_if, rp = _f64(r_if)
        th_if, tp = _f64(th_if)
        self.nr, self.nth, self.nphi = r_if.size - 1, th_if.size - 1, int(nphi)
        grid = _vp()
        _check(lib.spp_grid_create(self.nr, rp, self.nth, tp, self.nphi, inner_codes[inner], ctypes.byref(grid)),
               "spp_grid_create")
        plan = _vp()
        try:
            _check(lib.spp_plan_create(grid, ctypes.byref(plan)), "spp_plan_create")
        finally:
            lib.spp_grid_destroy(grid)
        self._plan = plan
        pb, wb = _c_size_t(), _c_size_t()
        _check(lib.spp_plan_device_bytes(plan, ctypes.byref(pb), ctypes.byref(wb)), "spp_plan_device_bytes")
        self.plan_bytes, self.workspace_bytes = pb.value, wb.value
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        with torch.cuda.device(self.device):
            self._plan_dev = torch.empty(self.plan_bytes, dtype=torch.uint8, device=self.device)
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
            _check(lib.spp_plan_upload(plan, _vp(self._plan_dev.data_ptr()), _stream_ptr(None)),
                   "spp_plan_upload")

    PATHS = {"auto": 0, "staged": 1, "fused": 2}

    @property
    def path(self):
        """Kernel path of the FP64 solves: "staged" (five kernels) or "fused"
        (folded FFT, one per-mode kernel, folded inverse FFT)."""
        v = _c_int()
        _check(lib.spp_plan_get_path(self._plan, ctypes.byref(v)), "spp_plan_get_path")
        return {1: "staged", 2: "fused"}[v.value]

    @path.setter
    def path(self, name):
        _check(lib.spp_plan_set_path(self._plan, self.PATHS[name]), "spp_plan_set_path")

    @property
    def parity_split(self):
        on = _c_int()
        _check(lib.spp_plan_parity_split(self._plan, ctypes.byref(on)), "spp_plan_parity_split")
        return bool(on.value)

    @property
    def kernels(self):
        """Kernels one FP64 solve launches, in order (see spp_plan_kernels)."""
        need = _c_size_t()
        _check(lib.spp_plan_kernels(self._plan, None, 0, ctypes.byref(need)), "spp_plan_kernels")
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.spp_plan_kernels(self._plan, buf, need.value, None), "spp_plan_kernels")
        return buf.value.decode().split(";")

    @property
    def shape(self):
        return (self.nr, self.nth, self.nphi)

    def _check_field(self, t, name):
        import torch
        if (not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous()
                or tuple(t.shape) != self.shape or t.device != self.device):
            raise ValueError(f"{name} must be a contiguous float64 tensor of shape {self.shape} on {self.device}")

    def _check_workspace(self, ws, need):
        import torch
        if (not isinstance(ws, torch.Tensor) or not ws.is_contiguous() or ws.device != self.device
                or ws.numel() * ws.element_size() < need):
            raise ValueError(f"workspace must be a contiguous tensor of at least {need} bytes on {self.device}")

    def new_workspace(self):
        import torch
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)

    def solve(self, rho, G=1.0, out=None, workspace=None, stream=None):
        import torch
        if rho.dtype != torch.float64 or not rho.is_contiguous() or tuple(rho.shape) != self.shape:
            raise ValueError(f"rho must be a contiguous float64 tensor of shape {self.shape}")
        if rho.device != self.device:
            raise ValueError("rho must live on the plan's device")
        if out is None:
            out = torch.empty_like(rho)
        self._check_field(out, "out")
        ws = self.workspace if workspace is None else workspace
        self._check_workspace(ws, self.workspace_bytes)
        _check(lib.spp_solve(self._plan, _vp(rho.data_ptr()), _vp(out.data_ptr()), float(G),
                             _vp(ws.data_ptr()), _stream_ptr(stream)), "spp_solve")
        return out

    def solve_noalloc(self, rho, G=1.0, out=None, stream=None):
        """spp_solve_noalloc: the solve with the library's own device scratch
        as workspace (no allocation by the library; `out` is allocated here
        when not given).  Calls overlapping on one device race."""
        import torch
        self._check_field(rho, "rho")
        if out is None:
            out = torch.empty_like(rho)
        self._check_field(out, "out")
        _check(lib.spp_solve_noalloc(self._plan, _vp(rho.data_ptr()), _vp(out.data_ptr()), float(G),
                                     _stream_ptr(stream)), "spp_solve_noalloc")
        return out

    def face_fluxes(self, phi, out=None, workspace=None, stream=None):
        """Face fluxes (Fr, Ft, Fp) of grad Phi through the r, theta and phi
        faces of every cell (see spp_face_fluxes); three float64 tensors of
        Phi's shape, written on the current torch stream."""
        import torch
        if phi.dtype != torch.float64 or not phi.is_contiguous() or tuple(phi.shape) != self.shape:
            raise ValueError(f"phi must be a contiguous float64 tensor of shape {self.shape}")
        if phi.device != self.device:
            raise ValueError("phi must live on the plan's device")
        if out is None:
            out = tuple(torch.empty_like(phi) for _ in range(3))
        fr, ft, fp = out
        for t, name in ((fr, "out[0]"), (ft, "out[1]"), (fp, "out[2]")):
            self._check_field(t, name)
        ws = self.workspace if workspace is None else workspace
        self._check_workspace(ws, self.workspace_bytes)
        _check(lib.spp_face_fluxes(self._plan, _vp(phi.data_ptr()), _vp(fr.data_ptr()), _vp(ft.data_ptr()),
                                   _vp(fp.data_ptr()), _vp(ws.data_ptr()), _stream_ptr(stream)), "spp_face_fluxes")
        return fr, ft, fp

    def workspace_bytes_for(self, precision):
        b = _c_size_t()
        _check(lib.spp_plan_workspace_bytes(self._plan, precision_codes[precision], ctypes.byref(b)),
               "spp_plan_workspace_bytes")
        return b.value

    def solve_mixed(self, rho, G=1.0, precision="mixed_fp32", n_refine=1, out=None, workspace=None,
                    stream=None, fallback_fp64=True):
        """Mixed-precision solve with FP64 refinement (see spp_solve_mixed)."""
        import torch
        self._check_field(rho, "rho")
        if out is None:
            out = torch.empty_like(rho)
        self._check_field(out, "out")
        need = self.workspace_bytes_for(precision)
        if workspace is None:
            if getattr(self, "_mixed_ws", None) is None or self._mixed_ws.numel() < need:
                self._mixed_ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            workspace = self._mixed_ws
        self._check_workspace(workspace, need)
        _check(lib.spp_solve_mixed(self._plan, precision_codes[precision], int(n_refine), int(bool(fallback_fp64)),
                                   _vp(rho.data_ptr()), _vp(out.data_ptr()), float(G), _vp(workspace.data_ptr()),
                                   _stream_ptr(stream)), "spp_solve_mixed")
        return out

    @property
    def mixed_workspace(self):
        """The workspace solve_mixed allocated for itself (None before its first call)."""
        return getattr(self, "_mixed_ws", None)

    def status(self, workspace=None, noalloc=False, stream=None):
        """spp_solve_status of the last solve on `workspace` (default: the
        plan's own workspace; noalloc=True: the no-allocation scratch).
        Synchronises the stream; returns a dict with the status name and the
        spp_solve_info fields."""
        if noalloc:
            ptr = None
        else:
            ws = self.workspace if workspace is None else workspace
            ptr = _vp(ws.data_ptr())
        info = _SolveInfo()
        st = lib.spp_solve_status(self._plan, ptr, _stream_ptr(stream), ctypes.byref(info))
        if st not in (0, -6, -7):
            _check(st, "spp_solve_status")
        d = {f: getattr(info, f) for f, _ in _SolveInfo._fields_}
        d["status"] = STATUS_NAMES.get(st, st)
        return d

    def momentum_source(self, phi, G=1.0, out=None, workspace=None, stream=None):
        """Force on every cell from the gravitational stress tensor
        (spp_momentum_source): three float64 tensors (Fx, Fy, Fz) of Phi's
        shape."""
        import torch
        self._check_field(phi, "phi")
        if out is None:
            out = tuple(torch.empty_like(phi) for _ in range(3))
        for t, name in zip(out, ("out[0]", "out[1]", "out[2]")):
            self._check_field(t, name)
        ws = self.workspace if workspace is None else workspace
        self._check_workspace(ws, self.workspace_bytes)
        _check(lib.spp_momentum_source(self._plan, _vp(phi.data_ptr()), float(G), _vp(out[0].data_ptr()),
                                       _vp(out[1].data_ptr()), _vp(out[2].data_ptr()), _vp(ws.data_ptr()),
                                       _stream_ptr(stream)), "spp_momentum_source")
        return out

    def residual(self, rho, phi, G=1.0, out=None, workspace=None, stream=None):
        """r = 4 pi G rho - L Phi in FP64 (spp_residual)."""
        import torch
        self._check_field(rho, "rho")
        self._check_field(phi, "phi")
        if out is None:
            out = torch.empty_like(phi)
        self._check_field(out, "out")
        ws = self.workspace if workspace is None else workspace
        self._check_workspace(ws, self.workspace_bytes)
        _check(lib.spp_residual(self._plan, _vp(rho.data_ptr()), _vp(phi.data_ptr()), float(G), _vp(out.data_ptr()),
                                _vp(ws.data_ptr()), _stream_ptr(stream)), "spp_residual")
        return out

    def scale_lowprec_basis(self, factor):
        """Test hook: scale the low-precision eigenvector images and upload the
        plan again (spp_plan_scale_lowprec_basis)."""
        _check(lib.spp_plan_scale_lowprec_basis(self._plan, float(factor)), "spp_plan_scale_lowprec_basis")
        with torch.cuda.device(self.device):
            _check(lib.spp_plan_upload(self._plan, _vp(self._plan_dev.data_ptr()), _stream_ptr(None)),
                   "spp_plan_upload")

    def solve_profiled(self, rho, out, G=1.0, stream=None):
        """One solve with per-stage HIP-event timing; blocks until done.

        Returns the five stage durations in ms (forward FFT, forward
        projection, radial solves, inverse projection, inverse FFT).
        """
        self._check_field(rho, "rho")
        self._check_field(out, "out")
        st = np.zeros(5)
        _check(lib.spp_solve_profiled(self._plan, _vp(rho.data_ptr()), _vp(out.data_ptr()), float(G),
                                      _vp(self.workspace.data_ptr()), _stream_ptr(stream),
                                      st.ctypes.data_as(_dp)), "spp_solve_profiled")
        return st

    def autotune(self, stream=None):
        """Time the projection tile candidates for this shape; returns rows per wave tile."""
        rows = _c_int()
        _check(lib.spp_autotune_projection(self._plan, _vp(self.workspace.data_ptr()), _stream_ptr(stream),
                                           ctypes.byref(rows)), "spp_autotune_projection")
        return rows.value

    def theta_eigensystem(self, m):
        H = np.empty((self.nth, self.nth))
        lam = np.empty(self.nth)
        _check(lib.spp_theta_eigensystem(self._plan, int(m), H.ctypes.data_as(_dp), lam.ctypes.data_as(_dp)),
               "spp_theta_eigensystem")
        return lam, H

    def __del__(self):
        p = getattr(self, "_plan", None)
        if p is not None and p.value:
            lib.spp_plan_destroy(p)
            self._plan = None


class Batch:
    """Many solves captured once into one HIP graph (see spp_batch_create).

    ``plans[r]``, ``rhos[r]``, ``phis[r]`` and ``Gs[r]`` describe solve r; the
    tensors are kept alive by the batch.  ``launch()`` replays all solves;
    ``description`` names the classes and the tuner's choices.
    """

    def __init__(self, plans, rhos, phis, Gs, precision="fp64", n_refine=1, autotune=True, stream=None):
        import torch
        n = len(plans)
        if not (len(rhos) == len(phis) == len(Gs) == n) or n == 0:
            raise ValueError("plans, rhos, phis and Gs must have the same non-zero length")
        for p, x, y in zip(plans, rhos, phis):
            for t in (x, y):
                if (t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != p.shape
                        or t.device != p.device):
                    raise ValueError(f"tensors must be contiguous float64 of shape {p.shape} on {p.device}")
        self._keep = (list(plans), list(rhos), list(phis))
        self.n = n
        self._plans = (_vp * n)(*[p._plan for p in plans])
        self._rho = (_vp * n)(*[x.data_ptr() for x in rhos])
        self._phi = (_vp * n)(*[y.data_ptr() for y in phis])
        self._G = (ctypes.c_double * n)(*[float(g) for g in Gs])
        prec = precision_codes[precision]
        wb = _c_size_t()
        _check(lib.spp_batch_workspace_bytes(n, self._plans, prec, ctypes.byref(wb)), "spp_batch_workspace_bytes")
        self.workspace = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=plans[0].device)
        b = _vp()
        _check(lib.spp_batch_create(n, self._plans, self._rho, self._phi, self._G, prec, int(n_refine),
                                    int(bool(autotune)), _vp(self.workspace.data_ptr()), _stream_ptr(stream),
                                    ctypes.byref(b)), "spp_batch_create")
        self._batch = b

    @property
    def description(self):
        need = _c_size_t()
        _check(lib.spp_batch_describe(self._batch, None, 0, ctypes.byref(need)), "spp_batch_describe")
        buf = ctypes.create_string_buffer(need.value)
        _check(lib.spp_batch_describe(self._batch, buf, need.value, None), "spp_batch_describe")
        return buf.value.decode()

    def status(self, r, stream=None):
        info = _SolveInfo()
        st = lib.spp_batch_status(self._batch, int(r), _stream_ptr(stream), ctypes.byref(info))
        if st not in (0, -6, -7):
            _check(st, "spp_batch_status")
        return _info_dict(st, info)

    def launch(self, stream=None):
        _check(lib.spp_batch_launch(self._batch, _stream_ptr(stream)), "spp_batch_launch")

    def __del__(self):
        b = getattr(self, "_batch", None)
        if b is not None and b.value:
            lib.spp_batch_destroy(b)
            self._batch = None


class Server:
    """Serving loop with continuous batching (see spp_server_create).

    ``Server(plans, pool_bytes, n_slots)`` allocates the workspace pool as a
    torch uint8 tensor on the plans' device.  ``submit`` queues a request
    (tensors are kept alive until its completion is polled); ``poll`` returns
    completion records as dicts; ``drain`` waits for all submitted requests.
    """

    def __init__(self, plans, pool_bytes, n_slots=8):
        import torch
        self.plans = list(plans)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.plans[0].device)
        arr = (_vp * len(self.plans))(*[p._plan for p in self.plans])
        s = _vp()
        _check(lib.spp_server_create(len(self.plans), arr, _vp(self.pool.data_ptr()), self.pool.numel(),
                                     int(n_slots), ctypes.byref(s)), "spp_server_create")
        self._s = s
        # requests in flight, keyed by the binding's own sequence number (the
        # tag the library sees): caller tags may repeat
        self._live = {}
        self._seq = 0

    def now(self):
        t = _c_double()
        _check(lib.spp_server_now(self._s, ctypes.byref(t)), "spp_server_now")
        return t.value

    def submit(self, plan_index, rho, phi, G=1.0, request_id=0, not_before=0.0, stream=None,
               precision="fp64", n_refine=1):
        """Queue one solve (precision "fp64" or "mixed_fp32").  An event
        recorded on `stream` (default: the current torch stream) after the work
        queued so far makes the slot stream wait until rho is written."""
        import torch
        if not 0 <= int(plan_index) < len(self.plans):
            raise ValueError(f"plan_index must be in [0, {len(self.plans)})")
        plan = self.plans[int(plan_index)]
        plan._check_field(rho, "rho")
        plan._check_field(phi, "phi")
        ready = torch.cuda.Event()
        ready.record(stream if stream is not None else torch.cuda.current_stream(plan.device))
        seq = self._seq
        self._seq += 1
        req = _Request(int(plan_index), _vp(rho.data_ptr()), _vp(phi.data_ptr()), float(G), seq,
                       _vp(ready.cuda_event), precision_codes[precision], int(n_refine))
        _check(lib.spp_server_submit(self._s, ctypes.byref(req), float(not_before)), "spp_server_submit")
        self._live[seq] = (int(request_id), rho, phi, ready)

    def poll(self, max_out=4096):
        buf = (_Completion * max_out)()
        n = _c_int()
        _check(lib.spp_server_poll(self._s, buf, max_out, ctypes.byref(n)), "spp_server_poll")
        out = []
        for c in buf[:n.value]:
            tag = self._live.pop(int(c.request_id), (int(c.request_id),))[0]
            out.append(dict(request_id=tag, plan_index=c.plan_index, t_arrival=c.t_arrival,
                            t_admit=c.t_admit, t_done=c.t_done, status=c.status))
        return out

    def drain(self, timeout_s=120.0):
        _check(lib.spp_server_drain(self._s, float(timeout_s)), "spp_server_drain")

    def close(self):
        s = getattr(self, "_s", None)
        if s is not None and s.value:
            lib.spp_server_destroy(s)
            self._s = None

    def __del__(self):
        self.close()
