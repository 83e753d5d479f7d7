"""Python binding of libmsm (include/msm.h): argument marshalling only.

Every step of the MSM runs in the HIP kernels of ``libmsm.so``; this module
passes torch tensors' device pointers and the current HIP stream across the
C ABI.  There is no CPU fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsm.so")

MSM_FP32, MSM_FP64 = 0, 1
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "cutoff too large", 4: "grid",
          5: "out of domain", 6: "non-finite", 7: "capacity", 8: "HIP error", 9: "out of memory",
          10: "no device"}

_lib = None

# every symbol declared in include/msm.h
EXPORTS = ("msm_plan_create", "msm_plan_create_kernel", "msm_plan_create_cell",
           "msm_plan_create_cell_kernel", "msm_plan_set_cell",
           "msm_plan_create_host", "msm_plan_destroy", "msm_plan_describe",
           "msm_plan_get_stencil", "msm_plan_grid_dims", "msm_workspace_bytes",
           "msm_energy_forces", "msm_energy_forces_noalloc", "msm_backward", "msm_backward_full",
           "msm_plan_status", "msm_plan_set_skin", "msm_plan_skin_stats",
           "msm_energy_forces_cell_gradient",
           "msm_plan_get_grid",
           "msm_batch_plan_create", "msm_batch_plan_create_kernel", "msm_batch_energy_forces",
           "msm_status_string",
           "msm_plan_set_profiling", "msm_plan_get_profile", "msm_plan_set_profile_stages",
           "msm_md_create", "msm_md_destroy", "msm_md_set_state", "msm_md_run",
           "msm_md_get_state", "msm_md_energies")


class MSMError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: libmsm status {code} ({STATUS.get(code, '?')})")


def lib():
    """Loads libmsm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2510_05961_amd.build`")
        # torch ships its own libamdhip64.so.7; loading torch first makes
        # libmsm bind to that same HIP runtime (one runtime per process).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P, i, u, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint, ctypes.c_double, ctypes.c_size_t
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.msm_plan_create.argtypes = [pp, P, u, i, d, d, i, i, i, i]
        L.msm_plan_create_host.argtypes = [pp, P, u, i, d, d, i, i, i, i]
        L.msm_plan_create_cell.argtypes = [pp, P, u, i, d, d, i, i, i, i]
        L.msm_plan_create_kernel.argtypes = [pp, i, P, u, i, d, d, i, i, i, i]
        L.msm_plan_create_cell_kernel.argtypes = [pp, i, P, u, i, d, d, i, i, i, i]
        L.msm_plan_set_cell.argtypes = [P, P]
        L.msm_plan_destroy.argtypes = [P]
        L.msm_plan_describe.argtypes = [P, ctypes.c_char_p, sz]
        L.msm_plan_get_stencil.argtypes = [P, i, P, P, sz]
        L.msm_plan_grid_dims.argtypes = [P, i, P]
        L.msm_workspace_bytes.argtypes = [P, i, i]
        L.msm_workspace_bytes.restype = sz
        L.msm_energy_forces.argtypes = [P, i, P, P, P, P, P, P, P]
        L.msm_energy_forces_noalloc.argtypes = [P, i, P, P, P, P, P, P, P]
        L.msm_backward.argtypes = [P, i, P, P, P, P, P, P, P, P]
        L.msm_backward_full.argtypes = [P, i, P, P, P, P, P, P, P, P, P]
        L.msm_plan_set_skin.argtypes = [P, d]
        L.msm_energy_forces_cell_gradient.argtypes = [P, i, P, P, P, P, P, P, P]
        L.msm_plan_skin_stats.argtypes = [P, ctypes.POINTER(ctypes.c_longlong),
                                          ctypes.POINTER(ctypes.c_longlong), P]
        L.msm_plan_status.argtypes = [P, P]
        L.msm_plan_get_grid.argtypes = [P, i, i, P, P]
        L.msm_batch_plan_create.argtypes = [pp, i, P, P, u, i, d, d, i, i, i]
        L.msm_batch_plan_create_kernel.argtypes = [pp, i, i, P, P, u, i, d, d, i, i, i]
        L.msm_batch_energy_forces.argtypes = [P, P, P, P, P, P, P, P, P]
        L.msm_plan_set_profiling.argtypes = [P, i]
        L.msm_plan_get_profile.argtypes = [P, ctypes.c_char_p, sz, i]
        L.msm_plan_set_profile_stages.argtypes = [P, ctypes.c_char_p]
        L.msm_md_create.argtypes = [pp, P, i, d, d, d, d, d, i]
        L.msm_md_destroy.argtypes = [P]
        L.msm_md_set_state.argtypes = [P, P, P, P, P, P]
        L.msm_md_run.argtypes = [P, i, i, P]
        L.msm_md_get_state.argtypes = [P, P, P, P, P]
        L.msm_md_energies.argtypes = [P, P, i, ctypes.POINTER(ctypes.c_int)]
        L.msm_status_string.argtypes = [i]
        L.msm_status_string.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "msm_workspace_bytes" and name != "msm_status_string":
                getattr(L, name).restype = i
        _lib = L
    return _lib


def _check(code, where):
    if code != 0:
        raise MSMError(code, where)


def _flat9(cell):
    rows = [list(r) for r in cell]
    assert len(rows) == 3 and all(len(r) == 3 for r in rows)
    return [x for r in rows for x in r]


def _dbl3(v):
    return (ctypes.c_double * 3)(*[float(x) for x in v])


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """An MSM plan for one orthorhombic box (msm_plan_create)."""

    def __init__(self, box, periodic_mask, order, h, cutoff, levels, precision=MSM_FP32,
                 max_n=1, quasi_degree=-1, device=True, cell=None, kernel=1):
        """cell: rows a, b, c of a triclinic cell (msm_plan_create_cell; box is
        then ignored and periodic_mask must be 7).  kernel: the power nu of
        k(r) = r^-nu (1 Coulomb, 6 dispersion: msm_plan_create_kernel, or
        msm_plan_create_cell_kernel with a cell)."""
        self._h = ctypes.c_void_p()
        if kernel != 1 and cell is not None:
            c9 = (ctypes.c_double * 9)(*[float(x) for x in _flat9(cell)])
            _check(lib().msm_plan_create_cell_kernel(ctypes.byref(self._h), int(kernel), c9,
                                                     int(periodic_mask), int(order), float(h),
                                                     float(cutoff), int(levels), int(precision),
                                                     int(max_n), int(quasi_degree)),
                   "msm_plan_create_cell_kernel")
            box = (1.0, 1.0, 1.0)
        elif kernel != 1:
            _check(lib().msm_plan_create_kernel(ctypes.byref(self._h), int(kernel), _dbl3(box),
                                                int(periodic_mask), int(order), float(h),
                                                float(cutoff), int(levels), int(precision),
                                                int(max_n), int(quasi_degree)),
                   "msm_plan_create_kernel")
        elif cell is not None:
            c9 = (ctypes.c_double * 9)(*[float(x) for x in _flat9(cell)])
            _check(lib().msm_plan_create_cell(ctypes.byref(self._h), c9, int(periodic_mask),
                                              int(order), float(h), float(cutoff), int(levels),
                                              int(precision), int(max_n), int(quasi_degree)),
                   "msm_plan_create_cell")
            box = (1.0, 1.0, 1.0)
        else:
            f = lib().msm_plan_create if device else lib().msm_plan_create_host
            _check(f(ctypes.byref(self._h), _dbl3(box), int(periodic_mask), int(order),
                     float(h), float(cutoff), int(levels), int(precision), int(max_n),
                     int(quasi_degree)), "msm_plan_create")
        self.cell = cell
        self.box = tuple(float(b) for b in box)
        self.periodic_mask = int(periodic_mask)
        self.order, self.levels = int(order), int(levels)
        self.precision = int(precision)
        self.max_n = int(max_n)
        self.device = device

    def close(self):
        if self._h:
            lib().msm_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == MSM_FP64 else torch.float32

    def describe(self):
        buf = ctypes.create_string_buffer(1 << 20)
        _check(lib().msm_plan_describe(self._h, buf, len(buf)), "msm_plan_describe")
        return json.loads(buf.value.decode())

    def stencil(self, level):
        """(len[3], off[3], K[len_z, len_y, len_x]) as numpy FP64."""
        import numpy as np
        dims = (ctypes.c_int * 6)()
        _check(lib().msm_plan_get_stencil(self._h, level, dims, None, 0), "get_stencil")
        ln, off = list(dims[:3]), list(dims[3:])
        K = np.zeros((ln[2], ln[1], ln[0]))
        _check(lib().msm_plan_get_stencil(self._h, level, dims,
                                          K.ctypes.data_as(ctypes.c_void_p), K.size),
               "get_stencil")
        return ln, off, K

    def grid_dims(self, level):
        n = (ctypes.c_int * 3)()
        _check(lib().msm_plan_grid_dims(self._h, level, n), "grid_dims")
        return tuple(n)

    def set_cell(self, cell):
        """msm_plan_set_cell: a new triclinic cell (stencils rebuilt)."""
        c9 = (ctypes.c_double * 9)(*[float(x) for x in _flat9(cell)])
        _check(lib().msm_plan_set_cell(self._h, c9), "msm_plan_set_cell")
        self.cell = cell

    def set_skin(self, skin):
        _check(lib().msm_plan_set_skin(self._h, float(skin)), "msm_plan_set_skin")

    def skin_stats(self, stream=None):
        """(calls, rebuilds) since set_skin."""
        c, r = ctypes.c_longlong(), ctypes.c_longlong()
        _check(lib().msm_plan_skin_stats(self._h, ctypes.byref(c), ctypes.byref(r),
                                         _stream(stream)), "msm_plan_skin_stats")
        return c.value, r.value

    def workspace_bytes(self, n):
        return int(lib().msm_workspace_bytes(self._h, int(n), 0))

    def energy_forces(self, pos, q, ws=None, want_forces=True, want_dEdq=True, stream=None,
                      out=None):
        """Forward pass on the device; returns (energy[1] f64, forces|None, dEdq|None)."""
        import torch
        n = q.shape[0]
        assert pos.is_cuda and q.is_cuda and pos.dtype == self.dtype and q.dtype == self.dtype
        assert pos.is_contiguous() and q.is_contiguous() and tuple(pos.shape) == (n, 3)
        if out is None:
            E = torch.empty(1, dtype=torch.float64, device=pos.device)
            F = torch.empty((n, 3), dtype=self.dtype, device=pos.device) if want_forces else None
            dq = torch.empty(n, dtype=self.dtype, device=pos.device) if want_dEdq else None
        else:
            E, F, dq = out
        _check(lib().msm_energy_forces(self._h, n, _ptr(pos), _ptr(q), _ptr(ws), _ptr(E),
                                       _ptr(F), _ptr(dq), _stream(stream)), "msm_energy_forces")
        return E, F, dq

    def energy_forces_cell_gradient(self, pos, q, stream=None):
        """(E, F, dEdq, dE/dH [3, 3] f64) of a triclinic plan; dE/dH at fixed
        Cartesian positions, H with the lattice vectors as columns."""
        import torch
        n = q.shape[0]
        E = torch.empty(1, dtype=torch.float64, device=pos.device)
        F = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        dq = torch.empty(n, dtype=self.dtype, device=pos.device)
        G = torch.empty((3, 3), dtype=torch.float64, device=pos.device)
        _check(lib().msm_energy_forces_cell_gradient(self._h, n, _ptr(pos), _ptr(q), _ptr(E),
                                                     _ptr(F), _ptr(dq), _ptr(G),
                                                     _stream(stream)),
               "msm_energy_forces_cell_gradient")
        return E, F, dq, G

    def energy_forces_noalloc(self, pos, q, out, ws=None, stream=None):
        """msm_energy_forces_noalloc into the caller's outputs out = (E[1] f64,
        F [n,3] or None, dEdq [n] or None); the call allocates nothing."""
        n = q.shape[0]
        assert pos.is_cuda and q.is_cuda and pos.dtype == self.dtype and q.dtype == self.dtype
        assert pos.is_contiguous() and q.is_contiguous() and tuple(pos.shape) == (n, 3)
        E, F, dq = out
        _check(lib().msm_energy_forces_noalloc(self._h, n, _ptr(pos), _ptr(q), _ptr(ws), _ptr(E),
                                               _ptr(F), _ptr(dq), _stream(stream)),
               "msm_energy_forces_noalloc")
        return E, F, dq

    def backward(self, pos, q, ws, gE=None, gF=None, gdEdq=None, stream=None):
        import torch
        n = q.shape[0]
        gpos = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
        gq = torch.empty(n, dtype=self.dtype, device=pos.device)
        if gdEdq is None:
            _check(lib().msm_backward(self._h, n, _ptr(pos), _ptr(q), _ptr(ws), _ptr(gE),
                                      _ptr(gF), _ptr(gpos), _ptr(gq), _stream(stream)),
                   "msm_backward")
        else:
            _check(lib().msm_backward_full(self._h, n, _ptr(pos), _ptr(q), _ptr(ws), _ptr(gE),
                                           _ptr(gF), _ptr(gdEdq), _ptr(gpos), _ptr(gq),
                                           _stream(stream)), "msm_backward_full")
        return gpos, gq

    def status(self, stream=None):
        return int(lib().msm_plan_status(self._h, _stream(stream)))

    def set_profiling(self, on=True):
        _check(lib().msm_plan_set_profiling(self._h, int(bool(on))), "set_profiling")

    def set_profile_stages(self, stages=None):
        """Record only these stages (iterable of names; None: all)."""
        arg = None if not stages else ",".join(stages).encode()
        _check(lib().msm_plan_set_profile_stages(self._h, arg), "set_profile_stages")

    def profile(self, reset=False):
        """{stage: {"ms": total, "launches": n}} since the last reset."""
        buf = ctypes.create_string_buffer(1 << 16)
        _check(lib().msm_plan_get_profile(self._h, buf, len(buf), int(bool(reset))), "get_profile")
        return json.loads(buf.value.decode())

    def grid(self, level, which):
        import torch
        n = self.grid_dims(level)
        out = torch.empty((n[2], n[1], n[0]), dtype=self.dtype, device="cuda")
        _check(lib().msm_plan_get_grid(self._h, level, which, _ptr(out), _stream()), "get_grid")
        return out


class BatchPlan:
    """Many free-space systems in one launch sequence (msm_batch_plan_create)."""

    def __init__(self, boxes, levels, order, h, cutoff, precision=MSM_FP32, max_total_n=1,
                 quasi_degree=-1, periodic_mask=0, kernel=1):
        """boxes: [n_sys, 3] edge lengths, or [n_sys] edges of cubes; kernel:
        the power nu of k(r) = r^-nu (1 Coulomb, 6 dispersion)."""
        import numpy as np
        self._h = ctypes.c_void_p()
        b = np.asarray(boxes, dtype=np.float64)
        if b.ndim == 1:
            b = np.stack([b, b, b], axis=1)
        b = np.ascontiguousarray(b)
        lv = np.ascontiguousarray(levels, dtype=np.int32)
        self.n_sys = len(b)
        if kernel == 1:
            _check(lib().msm_batch_plan_create(ctypes.byref(self._h), self.n_sys,
                                               b.ctypes.data_as(ctypes.c_void_p),
                                               lv.ctypes.data_as(ctypes.c_void_p),
                                               int(periodic_mask), int(order),
                                               float(h), float(cutoff), int(precision),
                                               int(max_total_n), int(quasi_degree)),
                   "msm_batch_plan_create")
        else:
            _check(lib().msm_batch_plan_create_kernel(ctypes.byref(self._h), int(kernel),
                                                      self.n_sys,
                                                      b.ctypes.data_as(ctypes.c_void_p),
                                                      lv.ctypes.data_as(ctypes.c_void_p),
                                                      int(periodic_mask), int(order),
                                                      float(h), float(cutoff), int(precision),
                                                      int(max_total_n), int(quasi_degree)),
                   "msm_batch_plan_create_kernel")
        self.precision = int(precision)

    close = Plan.close
    __del__ = Plan.__del__
    dtype = Plan.dtype
    describe = Plan.describe
    status = Plan.status
    set_profiling = Plan.set_profiling
    set_profile_stages = Plan.set_profile_stages
    profile = Plan.profile

    def energy_forces(self, offsets, pos, q, stream=None, out=None):
        """offsets: int32 cuda [n_sys+1]; returns (energies f64 [n_sys], F, dEdq)."""
        import torch
        n = q.shape[0]
        assert offsets.dtype == torch.int32 and offsets.is_cuda
        assert pos.dtype == self.dtype and q.dtype == self.dtype
        if out is None:
            E = torch.empty(self.n_sys, dtype=torch.float64, device=pos.device)
            F = torch.empty((n, 3), dtype=self.dtype, device=pos.device)
            dq = torch.empty(n, dtype=self.dtype, device=pos.device)
        else:
            E, F, dq = out
        _check(lib().msm_batch_energy_forces(self._h, _ptr(offsets), _ptr(pos), _ptr(q), None, _ptr(E),
                                             _ptr(F), _ptr(dq), _stream(stream)),
               "msm_batch_energy_forces")
        return E, F, dq


class MD:
    """Velocity-Verlet dynamics of charged Lennard-Jones particles around a
    plan (msm_md_*): state on the device in the plan's precision."""

    def __init__(self, plan, n, dt, epsilon, sigma, cutoff, switch_on, log_steps=0):
        self._h = ctypes.c_void_p()
        _check(lib().msm_md_create(ctypes.byref(self._h), plan._h, int(n), float(dt),
                                   float(epsilon), float(sigma), float(cutoff),
                                   float(switch_on), int(log_steps)), "msm_md_create")
        self.plan, self.n, self.log_steps = plan, int(n), int(log_steps)

    def close(self):
        if self._h:
            lib().msm_md_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, pos, vel, q, mass, stream=None):
        for t in (pos, vel, q, mass):
            assert t.is_cuda and t.dtype == self.plan.dtype and t.is_contiguous()
        _check(lib().msm_md_set_state(self._h, _ptr(pos), _ptr(vel), _ptr(q), _ptr(mass),
                                      _stream(stream)), "msm_md_set_state")

    def run(self, nsteps, graph=True, stream=None):
        _check(lib().msm_md_run(self._h, int(nsteps), 1 if graph else 0, _stream(stream)),
               "msm_md_run")

    def state(self, stream=None):
        import torch
        pos = torch.empty((self.n, 3), dtype=self.plan.dtype, device="cuda")
        vel, F = torch.empty_like(pos), torch.empty_like(pos)
        _check(lib().msm_md_get_state(self._h, _ptr(pos), _ptr(vel), _ptr(F), _stream(stream)),
               "msm_md_get_state")
        return pos, vel, F

    def energies(self):
        """[steps, 3] numpy array: kinetic, Lennard-Jones, MSM energy after
        each step."""
        import numpy as np
        buf = np.zeros((max(self.log_steps, 1), 3))
        steps = ctypes.c_int()
        _check(lib().msm_md_energies(self._h, buf.ctypes.data_as(ctypes.c_void_p),
                                     self.log_steps, ctypes.byref(steps)), "msm_md_energies")
        return buf[:min(steps.value, self.log_steps)]


def _autograd_function():
    import torch

    class MSMFunction(torch.autograd.Function):
        """(pos, q) -> (E, F, dEdq), differentiable in all three outputs."""

        @staticmethod
        def forward(ctx, pos, q, plan):
            ws = torch.empty(plan.workspace_bytes(q.shape[0]), dtype=torch.uint8,
                             device=pos.device)
            E, F, dq = plan.energy_forces(pos, q, ws=ws)
            ctx.set_materialize_grads(False)  # unused outputs: NULL cotangents, no extra passes
            ctx.plan = plan
            ctx.save_for_backward(pos, q, ws)
            return E, F, dq

        @staticmethod
        def backward(ctx, gE, gF, gdq):
            pos, q, ws = ctx.saved_tensors
            plan = ctx.plan
            gE = gE.to(torch.float64).contiguous() if gE is not None else None
            gF = gF.to(plan.dtype).contiguous() if gF is not None else None
            gdq = gdq.to(plan.dtype).contiguous() if gdq is not None else None
            gpos, gq = plan.backward(pos, q, ws, gE=gE, gF=gF, gdEdq=gdq)
            return gpos, gq, None

    return MSMFunction


_MSMFunction = None


def energy_forces(pos, q, plan):
    """Differentiable forward: returns (E [1] float64, F [n,3], dEdq [n])."""
    global _MSMFunction
    if _MSMFunction is None:
        _MSMFunction = _autograd_function()
    return _MSMFunction.apply(pos, q, plan)
