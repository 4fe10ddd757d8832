"""Python binding of the C ABI: argument marshalling only.

Every step of a solve runs inside libieti.so (host planning in C++, the solve
in HIP kernels on gfx950).  PyTorch supplies device memory and streams.
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np

from . import _abi
from ._abi import IetiOptions, IetiPatch, IetiStats, check, lib


def default_options(**overrides) -> IetiOptions:
    opt = IetiOptions()
    lib().ieti_default_options(C.byref(opt))
    for k, v in overrides.items():
        if not hasattr(opt, k):
            raise KeyError(k)
        if k == "tune_cache" and isinstance(v, str):
            v = v.encode()
        setattr(opt, k, v)
    return opt


def options_for(wl, **overrides) -> IetiOptions:
    """Options implied by a workload description (local solver, MG precision, primal set, tolerances)."""
    o = dict(
        local_solver={"exact": _abi.IETI_LOCAL_EXACT, "exact_mg": _abi.IETI_LOCAL_EXACT_MG,
                      "mg_saddle": _abi.IETI_LOCAL_MG_SADDLE}.get(wl.local_solver, _abi.IETI_LOCAL_MG),
        mg_precision=int(wl.mg_precision),
        primal={"vertices": _abi.IETI_PRIMAL_VERTICES, "edges": _abi.IETI_PRIMAL_EDGES,
                "vertices+edges": _abi.IETI_PRIMAL_VERTICES | _abi.IETI_PRIMAL_EDGES}[wl.primal],
        tol=float(wl.tol),
        inner_tol=float(wl.inner_tol),
    )
    o.update(overrides)
    return default_options(**o)


class _PatchArray:
    """Keeps the numpy buffers alive while the C struct array points into them."""

    def __init__(self, patches: Sequence):
        self.keep = []
        self.arr = (IetiPatch * len(patches))()
        for i, p in enumerate(patches):
            s = self.arr[i]
            s.dim = p.dim
            for d in range(p.dim):
                kn = np.ascontiguousarray(p.knots[d], dtype=np.float64)
                self.keep.append(kn)
                s.degree[d] = int(p.degree[d])
                s.n_knots[d] = len(kn)
                s.knots[d] = kn.ctypes.data_as(C.POINTER(C.c_double))
            ct = np.ascontiguousarray(p.ctrl, dtype=np.float64)
            self.keep.append(ct)
            s.ctrl = ct.ctypes.data_as(C.POINTER(C.c_double))

    def __len__(self):
        return len(self.arr)


def _primal_arg(primal_vertices):
    if primal_vertices is None:
        return None, 0, None
    pv = np.ascontiguousarray(primal_vertices, dtype=np.float64)
    return pv.ctypes.data_as(C.POINTER(C.c_double)), int(pv.shape[0]), pv


class Plan:
    """Host-only plan (topology, numbering, multigrid hierarchy, FP64 operator data)."""

    def __init__(self, patches: Sequence, options: IetiOptions | None = None, primal_vertices=None):
        self._pa = _PatchArray(patches)
        opt = options if options is not None else default_options()
        pvp, npv, self._pv = _primal_arg(primal_vertices)
        h = C.c_void_p()
        check(lib().ieti_plan_create(self._pa.arr, len(self._pa), pvp, npv, C.byref(opt), C.byref(h)),
              "ieti_plan_create")
        self.h = h
        self.dim = patches[0].dim

    def __del__(self):
        if getattr(self, "h", None):
            lib().ieti_plan_destroy(self.h)
            self.h = None

    def sizes(self) -> dict:
        v = [C.c_int64() for _ in range(5)]
        ml = C.c_int32()
        check(lib().ieti_plan_sizes(self.h, *[C.byref(x) for x in v], C.byref(ml)), "ieti_plan_sizes")
        names = ["ndof_torn", "ndof_global", "n_lambda", "n_primal", "n_qp"]
        out = {k: int(x.value) for k, x in zip(names, v)}
        out["max_levels"] = int(ml.value)
        return out

    def array(self, which: int, patch: int = 0, level: int = 0, dtype=np.float64) -> np.ndarray:
        cnt = C.c_int64()
        check(lib().ieti_plan_array(self.h, which, patch, level, None, C.byref(cnt)), "ieti_plan_array")
        out = np.empty(cnt.value, dtype=dtype)
        check(lib().ieti_plan_array(self.h, which, patch, level, out.ctypes.data_as(C.c_void_p), C.byref(cnt)),
              "ieti_plan_array")
        return out

    def device_bytes(self) -> int:
        """Device bytes a serving slot reserves for a request with this plan."""
        b = C.c_size_t()
        check(lib().ieti_plan_device_bytes(self.h, C.byref(b)), "ieti_plan_device_bytes")
        return int(b.value)

    def quadrature(self) -> np.ndarray:
        n = self.sizes()["n_qp"]
        x = np.empty((n, self.dim), dtype=np.float64)
        check(lib().ieti_plan_quadrature(self.h, x.ctypes.data_as(C.POINTER(C.c_double))), "ieti_plan_quadrature")
        return x


class Solver:
    """Device solver handle: ieti_setup once, ieti_solve per right-hand side."""

    def __init__(self, patches: Sequence, options: IetiOptions | None = None, primal_vertices=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the IETI-DP solver runs only on the device")
        self._pa = _PatchArray(patches)
        opt = options if options is not None else default_options()
        if stream is not None:
            opt.stream = C.c_void_p(stream.cuda_stream)
        pvp, npv, self._pv = _primal_arg(primal_vertices)
        h = C.c_void_p()
        check(lib().ieti_setup(self._pa.arr, len(self._pa), pvp, npv, C.byref(opt), C.byref(h)), "ieti_setup")
        self.h = h
        self.dim = patches[0].dim
        nq, nt, nb = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib().ieti_sizes(self.h, C.byref(nq), C.byref(nt), C.byref(nb)), "ieti_sizes")
        self.n_qp, self.ndof_torn, self.device_bytes = int(nq.value), int(nt.value), int(nb.value)

    def close(self):
        if getattr(self, "h", None):
            lib().ieti_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def profile(self, enable: bool = True):
        check(lib().ieti_profile_enable(self.h, 1 if enable else 0), "ieti_profile_enable")

    def profile_query(self, kernel: int) -> dict:
        n, ms, b = C.c_int64(), C.c_double(), C.c_double()
        check(lib().ieti_profile_query(self.h, kernel, C.byref(n), C.byref(ms), C.byref(b)), "ieti_profile_query")
        return {"launches": int(n.value), "ms": float(ms.value), "bytes": float(b.value)}

    def quadrature(self, device: bool = True):
        import torch
        if device:
            x = torch.empty((self.n_qp, self.dim), dtype=torch.float64, device="cuda")
            ptr = C.c_void_p(x.data_ptr())
        else:
            x = np.empty((self.n_qp, self.dim), dtype=np.float64)
            ptr = x.ctypes.data_as(C.c_void_p)
        n = C.c_int64()
        check(lib().ieti_quadrature(self.h, ptr, 1 if device else 0, C.byref(n)), "ieti_quadrature")
        return x

    def solve(self, f_qp, u=None, raise_on_noconv: bool = True, no_alloc: bool = False):
        """f_qp: float64 CUDA tensor of n_qp values; returns (u, stats dict).  no_alloc: call
        ieti_solve_noalloc (scratch in the library's static per-GPU array) instead of ieti_solve."""
        import torch
        if not (isinstance(f_qp, torch.Tensor) and f_qp.is_cuda and f_qp.dtype == torch.float64
                and f_qp.numel() == self.n_qp and f_qp.is_contiguous()):
            raise ValueError("f_qp must be a contiguous float64 CUDA tensor with n_qp entries")
        if u is None:
            u = torch.empty(self.ndof_torn, dtype=torch.float64, device=f_qp.device)
        st = IetiStats()
        fn = lib().ieti_solve_noalloc if no_alloc else lib().ieti_solve
        rc = fn(self.h, C.c_void_p(f_qp.data_ptr()), C.c_void_p(u.data_ptr()), C.byref(st))
        if rc != _abi.IETI_OK and not (rc == _abi.IETI_ENOCONV and not raise_on_noconv):
            check(rc, "ieti_solve_noalloc" if no_alloc else "ieti_solve")
        return u, st.as_dict()


def quadrature_points(patches: Sequence) -> np.ndarray:
    """Physical quadrature points of a set of patches (host, no planning)."""
    pa = _PatchArray(patches)
    n = C.c_int64()
    check(lib().ieti_quadrature_points(pa.arr, len(pa), None, C.byref(n)), "ieti_quadrature_points")
    x = np.empty((n.value, patches[0].dim), dtype=np.float64)
    check(lib().ieti_quadrature_points(pa.arr, len(pa), x.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)),
          "ieti_quadrature_points")
    return x


class Server:
    """Request loop: independent solves admitted by free slots and HBM budget, overlapping on the device."""

    def __init__(self, options: IetiOptions | None = None, slots: int = 4):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the IETI-DP server runs only on the device")
        torch.cuda.init()
        opt = options if options is not None else default_options()
        h = C.c_void_p()
        check(lib().ieti_server_create(C.byref(opt), slots, C.byref(h)), "ieti_server_create")
        self.h = h
        self._live = {}

    def submit(self, patches: Sequence, f_qp: np.ndarray) -> int:
        pa = _PatchArray(patches)
        f = np.ascontiguousarray(f_qp, dtype=np.float64)
        nt = sum(int(np.prod([len(k) - d - 1 for k, d in zip(p.knots, p.degree)])) for p in patches)
        u = np.empty(nt, dtype=np.float64)
        t = C.c_int64()
        check(lib().ieti_server_submit(self.h, pa.arr, len(pa), f.ctypes.data_as(C.POINTER(C.c_double)), f.size,
                                       u.ctypes.data_as(C.POINTER(C.c_double)), C.byref(t)), "ieti_server_submit")
        self._live[t.value] = u
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        """None while pending, else (status, u, stats, (t_submit, t_admit, t_done) in ms)."""
        st = IetiStats()
        times = (C.c_double * 3)()
        rc = lib().ieti_server_poll(self.h, ticket, 1 if wait else 0, C.byref(st), times)
        if rc == _abi.IETI_PENDING:
            return None
        u = self._live.pop(ticket)
        return rc, u, st.as_dict(), tuple(times)

    def load(self):
        q, r, b = C.c_int32(), C.c_int32(), C.c_size_t()
        check(lib().ieti_server_load(self.h, C.byref(q), C.byref(r), C.byref(b)), "ieti_server_load")
        return int(q.value), int(r.value), int(b.value)

    def close(self):
        if getattr(self, "h", None):
            lib().ieti_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()
