"""ctypes binding of libcbs.so (argument marshalling only).

Every operation runs in the HIP library; this module converts torch tensors to
device pointers and the current torch stream to a hipStream_t.  There is no
fallback: if the library is missing, loading fails with an error.

Fields are packed 1-D complex tensors on the GPU: instance i occupies
elements [off_i, off_i + n_i^2) with off_i = sum_{j<i} n_j^2, row-major [y][x].
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbs.so")

CBS_OK = 0
CBS_NOT_CONVERGED = 1
CBS_ERR_ARG = -1
CBS_ERR_SIZE = -2
CBS_ERR_ILLCOND = -3
CBS_ERR_WORKSPACE = -4
CBS_ERR_HIP = -5
CBS_C64 = 0
CBS_C128 = 1
FLAG_NO_GUARD = 1
FLAG_ONE_STREAM = 2
FLAG_DIRICHLET = 4
FLAG_UNDAMPED = 8
INST_RUNNING, INST_CONVERGED, INST_MAX_ITERS, INST_DIVERGED = 0, 1, 2, 3

SUPPORTED_SIZES = (16, 32, 64, 128, 192, 256, 288, 384, 512, 1024)
# Dirichlet instance sizes n (interior points): 2(n + 1) is a supported FFT length
# n with 2(n+1) an FFT size, and n = 64 (direct DST-I)
SUPPORTED_DIRICHLET = tuple(sorted([m // 2 - 1 for m in SUPPORTED_SIZES] + [64]))

# Every symbol include/cbs.h declares, with its ctypes signature.
_vp, _i32, _u32, _f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_double
SIGNATURES = {
    "cbs_setup": (_i32, [ctypes.POINTER(_vp), _i32, _vp, _vp, _vp, _vp, _i32, _i32, _u32, _vp]),
    "cbs_setup_ws": (_i32, [ctypes.POINTER(_vp), _i32, _vp, _vp, _vp, _vp, _i32, _i32, _u32, _vp,
                            ctypes.c_size_t, _vp]),
    "cbs_setup_cdr": (_i32, [ctypes.POINTER(_vp), _i32, _vp, _vp, _vp, _vp, _i32, _vp]),
    "cbs_setup_cdr_ws": (_i32, [ctypes.POINTER(_vp), _i32, _vp, _vp, _vp, _vp, _i32, _vp, ctypes.c_size_t,
                                _vp]),
    "cbs_workspace_size_cdr": (_i32, [_i32, _vp, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    "cbs_workspace_size": (_i32, [_i32, _vp, _i32, _i32, _u32, ctypes.POINTER(ctypes.c_size_t)]),
    "cbs_plan_info": (_i32, [_vp, _vp, _vp, _vp]),
    "cbs_plan_layout": (_i32, [_vp, _vp, _vp, _vp]),
    "cbs_apply": (_i32, [_vp, _vp, _vp, _vp, _vp]),
    "cbs_residual": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cbs_sweep": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "cbs_sweep_checkpoints": (_i32, [_vp, _vp, _vp, _i32, _vp]),
    "cbs_npbs_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "cbs_helmholtz_residual": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "cbs_relres": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "cbs_iterate": (_i32, [_vp, _vp, _vp, _i32, _f64, _i32, _i32, _vp, _vp, _vp, _i32, _vp]),
    "fgmres_solve": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _f64, _vp, _vp, _vp, _vp]),
    "cbs_iterate_async": (_i32, [_vp, _vp, _vp, _i32, _f64, _i32, _i32, _vp, _vp, _vp, _vp]),
    "fgmres_solve_async": (_i32, [_vp, _vp, _vp, _i32, _i32, _i32, _f64, _vp, _vp, _vp, _vp]),
    "cbs_adjoint_step": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cbs_born_adjoint": (_i32, [_vp, _vp, _vp, _vp]),
    "cbs_metric_matched_grad": (_i32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cbs_loss_seed": (_i32, [_vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "cbs_autotune": (_i32, [_vp, _vp, _vp]),
    "cbs_set_tile": (_i32, [_vp, _i32, _i32]),
    "cbs_set_col_threads": (_i32, [_vp, _i32]),
    "cbs_apply_static": (_i32, [_i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp]),
    "cbs_destroy": (None, [_vp]),
    "cbs_last_error": (ctypes.c_char_p, []),
    "cbs_version": (ctypes.c_char_p, []),
}

_lib = None


class CbsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cbs status {status}: {msg}")
        self.status = status


_deferred = []  # (plan handle, workspace) released after a graph capture


def _capturing() -> bool:
    try:
        return torch.cuda.is_available() and torch.cuda.is_current_stream_capturing()
    except Exception:
        return False


def _release(h, ws):
    if _capturing():
        _deferred.append((h, ws))
        return
    release_deferred()
    _lib.cbs_destroy(h)


def release_deferred():
    """Destroy plans whose release was deferred during a graph capture."""
    while _deferred and not _capturing():
        h, _ = _deferred.pop()
        _lib.cbs_destroy(h)


def load(path: str = LIB_PATH):
    """Load libcbs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libcbs.so not found at {path}; build it with "
                           "`python -m paper_2603_18527_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().cbs_last_error().decode()


def _check(st: int, allow_not_converged: bool = False) -> int:
    if st == CBS_OK or (allow_not_converged and st == CBS_NOT_CONVERGED):
        return st
    raise CbsError(st, last_error())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def workspace_size(sizes: Sequence[int], dtype: int = CBS_C64, max_restart: int = 0,
                   dirichlet: bool = False) -> int:
    """Device bytes of a plan's workspace (cbs_workspace_size; host only)."""
    n_arr = (ctypes.c_int32 * len(sizes))(*[int(n) for n in sizes])
    out = ctypes.c_size_t()
    _check(load().cbs_workspace_size(len(sizes), n_arr, int(dtype), int(max_restart),
                                     FLAG_DIRICHLET if dirichlet else 0, ctypes.byref(out)))
    return int(out.value)


# Limits of cbs_apply_static's fixed scratch (include/cbs.h).
STATIC_MAX_BATCH = 16
STATIC_MAX_BYTES = 16 << 20


def apply_static(k2: torch.Tensor, sizes: Sequence[int], k0sq, eps, u=None, s=None, out=None,
                 stream=None) -> torch.Tensor:
    """y = G(V u + s) through cbs_apply_static: no plan and no device
    allocation in the library (its scratch is a fixed device array).  k0sq and
    eps are per instance and must be given; out (optional) is the result
    tensor, else one is allocated here by torch."""
    sizes = [int(n) for n in sizes]
    cells = sum(n * n for n in sizes)
    dtype = CBS_C64 if k2.dtype == torch.complex64 else CBS_C128
    for name, t in (("k2", k2), ("u", u), ("s", s), ("out", out)):
        if t is not None and (t.dtype != k2.dtype or t.numel() != cells or not t.is_cuda
                              or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous packed CUDA tensor of dtype {k2.dtype}")
    y = torch.empty(cells, dtype=k2.dtype, device=k2.device) if out is None else out
    b = len(sizes)
    n_arr = (ctypes.c_int32 * b)(*sizes)
    k0_arr = (ctypes.c_double * b)(*[float(v) for v in _expand(k0sq, b)])
    eps_arr = (ctypes.c_double * b)(*[float(v) for v in _expand(eps, b)])
    _check(load().cbs_apply_static(b, n_arr, _ptr(k2), k0_arr, eps_arr, dtype, _ptr(u), _ptr(s), _ptr(y),
                                   _stream(stream)))
    return y


def workspace_size_cdr(sizes: Sequence[int], dtype: int = CBS_C64) -> int:
    """Device bytes of a convection-diffusion-reaction plan's workspace."""
    n_arr = (ctypes.c_int32 * len(sizes))(*[int(n) for n in sizes])
    out = ctypes.c_size_t()
    _check(load().cbs_workspace_size_cdr(len(sizes), n_arr, int(dtype), ctypes.byref(out)))
    return int(out.value)


def offsets(sizes: Sequence[int]) -> List[int]:
    out, o = [], 0
    for n in sizes:
        out.append(o)
        o += n * n
    return out


def pack(fields: Sequence, dtype=torch.complex64, device="cuda") -> torch.Tensor:
    """Concatenate (n, n) arrays/tensors into one packed device tensor."""
    parts = [torch.as_tensor(np.asarray(f) if not torch.is_tensor(f) else f).reshape(-1) for f in fields]
    return torch.cat([p.to(dtype) for p in parts]).to(device).contiguous()


def unpack(t: torch.Tensor, sizes: Sequence[int]) -> List[torch.Tensor]:
    out = []
    for n, o in zip(sizes, offsets(sizes)):
        out.append(t[o:o + n * n].reshape(n, n))
    return out


class Plan:
    """A batch of Helmholtz instances on the GPU (cbs_setup)."""

    def __init__(self, k2: torch.Tensor, sizes: Sequence[int], k0sq=None, eps=None,
                 dtype: int = CBS_C64, max_restart: int = 0, guard: bool = True, stream=None,
                 lanes: bool = True, torch_workspace: bool = True, dirichlet: bool = False,
                 undamped: bool = False):
        """torch_workspace: the plan's device memory is one torch tensor
        (cbs_setup_ws); False lets the library allocate it (cbs_setup).
        dirichlet: instances are n x n interiors of the unit square with
        homogeneous Dirichlet boundaries (five-point FD, DST-I reference).
        undamped (Dirichlet only): eps = 0, the reference L_D - k0^2 itself
        (no sweeps; FGMRES with sweeps=0)."""
        lib = load()
        release_deferred()
        self.sizes = [int(n) for n in sizes]
        self.batch = len(self.sizes)
        self.dtype = dtype
        self.tdtype = torch.complex64 if dtype == CBS_C64 else torch.complex128
        self.cells = sum(n * n for n in self.sizes)
        if k2.dtype != self.tdtype or k2.numel() != self.cells or not k2.is_cuda:
            raise ValueError("k2 must be a packed CUDA tensor of the plan dtype")
        k2 = k2.contiguous()
        n_arr = (ctypes.c_int32 * self.batch)(*self.sizes)
        k0_arr = None if k0sq is None else (ctypes.c_double * self.batch)(
            *[float("nan") if v is None else float(v) for v in _expand(k0sq, self.batch)])
        eps_arr = None if eps is None else (ctypes.c_double * self.batch)(
            *[0.0 if v is None else float(v) for v in _expand(eps, self.batch)])
        h = ctypes.c_void_p()
        flags = ((0 if guard else FLAG_NO_GUARD) | (0 if lanes else FLAG_ONE_STREAM)
                 | (FLAG_DIRICHLET if dirichlet else 0) | (FLAG_UNDAMPED if undamped else 0))
        self.dirichlet = bool(dirichlet)
        self.undamped = bool(undamped)
        self._ws = None
        if torch_workspace:
            self._ws = torch.empty(workspace_size(self.sizes, dtype, max_restart, dirichlet), dtype=torch.uint8,
                                   device="cuda")
            self._ws_stream = torch.cuda.current_stream()
            st = lib.cbs_setup_ws(ctypes.byref(h), self.batch, n_arr, _ptr(k2), k0_arr, eps_arr, dtype,
                                  int(max_restart), flags, _ptr(self._ws), self._ws.numel(),
                                  _stream(stream))
        else:
            st = lib.cbs_setup(ctypes.byref(h), self.batch, n_arr, _ptr(k2), k0_arr, eps_arr, dtype,
                               int(max_restart), flags, _stream(stream))
        _check(st)
        self._h = h
        self.max_restart = int(max_restart)
        cells = ctypes.c_int64()
        k0o = (ctypes.c_double * self.batch)()
        epso = (ctypes.c_double * self.batch)()
        _check(lib.cbs_plan_info(h, ctypes.byref(cells), k0o, epso))
        self.k0sq = list(k0o)
        self.eps = list(epso)

    def __del__(self):
        # cbs_destroy waits for the plan's own streams.  The workspace tensor
        # goes back to torch's allocator, which orders its reuse after the
        # work already queued on the streams the plan was called on
        # (record_stream in _st), so no device-wide synchronisation is needed.
        # A plan collected while a graph is being captured on this thread's
        # stream (the collector can run inside the capture) is released
        # later: stream synchronisation would invalidate the capture.
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _release(h, getattr(self, "_ws", None))
            self._h = None
        self._ws = None

    def close(self):
        self.__del__()

    # -- helpers
    def _st(self, stream):
        """hipStream_t of a call; the workspace is marked in use on streams
        other than the one it was allocated on."""
        st = torch.cuda.current_stream() if stream is None else stream
        ws = getattr(self, "_ws", None)
        if ws is not None and st != self._ws_stream:
            ws.record_stream(st)
        return ctypes.c_void_p(st.cuda_stream)

    def _field(self, t, name):
        if t is None:
            return None
        if t.dtype != self.tdtype or t.numel() != self.cells or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous packed CUDA tensor of dtype {self.tdtype}")
        return t

    def empty(self) -> torch.Tensor:
        return torch.empty(self.cells, dtype=self.tdtype, device="cuda")

    def zeros(self) -> torch.Tensor:
        return torch.zeros(self.cells, dtype=self.tdtype, device="cuda")

    # -- operations
    def apply(self, u, s, out=None, stream=None):
        y = self.empty() if out is None else self._field(out, "out")
        _check(load().cbs_apply(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                _ptr(y), self._st(stream)))
        return y

    def residual(self, u, s, rhs=None, out=None, norms=True, store=True, stream=None):
        r = (self.empty() if out is None else self._field(out, "out")) if store else None
        n2 = torch.empty(self.batch, dtype=torch.float64, device="cuda") if norms else None
        _check(load().cbs_residual(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                   _ptr(self._field(rhs, "rhs")), _ptr(r), _ptr(n2), self._st(stream)))
        return r, n2

    def helmholtz_residual(self, u, s, out=None, norms=True, store=True, stream=None):
        """r = s - A u (physical residual) and per-instance sums |r|^2."""
        r = (self.empty() if out is None else self._field(out, "out")) if store else None
        n2 = torch.empty(self.batch, dtype=torch.float64, device="cuda") if norms else None
        _check(load().cbs_helmholtz_residual(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                             _ptr(r), _ptr(n2), self._st(stream)))
        return r, n2

    def relres(self, u, s, stop="born", stream=None) -> torch.Tensor:
        """Per-instance relative residual (FP64, on the device): "born" is
        ||G(V u + s) - u|| / ||G s||, "physical" the paper's rTol
        ||s - A u|| / ||s|| (cbs_relres)."""
        if stop not in _STOPS:
            raise ValueError(f"stop must be one of {sorted(_STOPS)}")
        out = torch.empty(self.batch, dtype=torch.float64, device="cuda")
        _check(load().cbs_relres(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")), _STOPS[stop],
                                 _ptr(out), self._st(stream)))
        return out

    def physical_relres(self, u, s, stream=None):
        """The paper's rTol = ||s - A u|| / ||s|| per instance, as a list."""
        return self.relres(u, s, "physical", stream).cpu().tolist()

    def sweep(self, u, s, count=1, norms=False, stream=None):
        n2 = torch.empty(self.batch, dtype=torch.float64, device="cuda") if norms else None
        _check(load().cbs_sweep(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                int(count), _ptr(n2), self._st(stream)))
        return n2

    def sweep_checkpoints(self, u0, s, count, stream=None):
        """cbs_sweep_checkpoints: (count + 1, cells) tensor of u_0..u_count."""
        u0 = self._field(u0, "u0")
        u_all = torch.empty((int(count) + 1, self.cells), dtype=self.tdtype, device="cuda")
        u_all[0].copy_(u0)
        _check(load().cbs_sweep_checkpoints(self._h, _ptr(u_all), _ptr(self._field(s, "s")), int(count),
                                            self._st(stream)))
        return u_all

    def npbs_step(self, u, s, wf, wloc=None, count=1, stream=None):
        """count NPBS steps in place with the linear Fourier layer
        M(r) = F^-1(wf * F r) + wloc * r (wf packed per instance on the DFT bins)."""
        _check(load().cbs_npbs_step(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                    _ptr(self._field(wf, "wf")), _ptr(self._field(wloc, "wloc")),
                                    int(count), self._st(stream)))
        return u

    def iterate(self, u, s, max_sweeps=2500, rtol=1e-6, check_every=50, use_graph=True, stream=None,
                stop="born"):
        """stop: "born" (preconditioned residual) or "physical" (rTol = ||s - A u|| / ||s||)."""
        if stop not in _STOPS:
            raise ValueError(f"stop must be one of {sorted(_STOPS)}")
        it = (ctypes.c_int32 * self.batch)()
        rel = (ctypes.c_double * self.batch)()
        stat = (ctypes.c_int32 * self.batch)()
        _check(load().cbs_iterate(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                  int(max_sweeps), float(rtol), int(check_every), _STOPS[stop],
                                  it, rel, stat,
                                  1 if use_graph else 0, self._st(stream)), allow_not_converged=True)
        return list(it), list(rel), list(stat)

    def fgmres(self, u, s, restart=30, sweeps=4, max_iters=2500, rtol=1e-6, stream=None):
        it = (ctypes.c_int32 * self.batch)()
        rel = (ctypes.c_double * self.batch)()
        stat = (ctypes.c_int32 * self.batch)()
        _check(load().fgmres_solve(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                   int(restart), int(sweeps), int(max_iters), float(rtol), it, rel, stat,
                                   self._st(stream)), allow_not_converged=True)
        return list(it), list(rel), list(stat)

    def iterate_async(self, u, s, max_sweeps=2500, rtol=1e-6, check_every=50, stop="born", stream=None):
        """cbs_iterate_async: stream-ordered, no host synchronisation; returns
        device tensors (iters int32, relres float64, status int32)."""
        if stop not in _STOPS:
            raise ValueError(f"stop must be one of {sorted(_STOPS)}")
        it = torch.empty(self.batch, dtype=torch.int32, device="cuda")
        rel = torch.empty(self.batch, dtype=torch.float64, device="cuda")
        stat = torch.empty(self.batch, dtype=torch.int32, device="cuda")
        _check(load().cbs_iterate_async(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                        int(max_sweeps), float(rtol), int(check_every), _STOPS[stop],
                                        _ptr(it), _ptr(rel), _ptr(stat), self._st(stream)))
        return it, rel, stat

    def fgmres_async(self, u, s, restart=30, sweeps=4, max_iters=2500, rtol=1e-6, stream=None):
        """fgmres_solve_async: stream-ordered; device tensors (iters, relres, status)."""
        it = torch.empty(self.batch, dtype=torch.int32, device="cuda")
        rel = torch.empty(self.batch, dtype=torch.float64, device="cuda")
        stat = torch.empty(self.batch, dtype=torch.int32, device="cuda")
        _check(load().fgmres_solve_async(self._h, _ptr(self._field(u, "u")), _ptr(self._field(s, "s")),
                                         int(restart), int(sweeps), int(max_iters), float(rtol),
                                         _ptr(it), _ptr(rel), _ptr(stat), self._st(stream)))
        return it, rel, stat

    def metric_matched_grad(self, x, s, scale=None, grad=None, stream=None):
        """(loss, grad): loss_i = ||G s - (I - G V) x||^2 (float64, device) and
        grad = -2 scale_i R^H (G s - R x) (cbs_metric_matched_grad); scale is
        a float64 device tensor [batch] or None (= 1)."""
        g = self.empty() if grad is None else self._field(grad, "grad")
        loss = torch.empty(self.batch, dtype=torch.float64, device="cuda")
        if scale is not None:
            scale = scale.to(device="cuda", dtype=torch.float64).contiguous()
            if scale.numel() != self.batch:
                raise ValueError("scale: one value per instance")
        _check(load().cbs_metric_matched_grad(self._h, _ptr(self._field(x, "x")), _ptr(self._field(s, "s")),
                                              _ptr(scale), _ptr(loss), _ptr(g), self._st(stream)))
        return loss, g

    def born_adjoint(self, e, out=None, stream=None):
        """R^H e for R = I - G V (cbs_born_adjoint)."""
        y = self.empty() if out is None else self._field(out, "out")
        _check(load().cbs_born_adjoint(self._h, _ptr(self._field(e, "e")), _ptr(y), self._st(stream)))
        return y

    def adjoint_step(self, u_m, s, lam_in, lam_out, grad_k2, stream=None):
        _check(load().cbs_adjoint_step(self._h, _ptr(self._field(u_m, "u_m")), _ptr(self._field(s, "s")),
                                       _ptr(self._field(lam_in, "lam_in")), _ptr(self._field(lam_out, "lam_out")),
                                       _ptr(self._field(grad_k2, "grad_k2")), self._st(stream)))

    def loss_seed(self, u_k, s, weight="gamma", lam_out=None, grad_k2=None, stream=None):
        """weight: "gamma" (W = gamma), "one" (W = 1) or "physical" (s - A u_K);
        True / False stand for "gamma" / "one"."""
        lam = self.empty() if lam_out is None else self._field(lam_out, "lam_out")
        grad = self.zeros() if grad_k2 is None else self._field(grad_k2, "grad_k2")
        loss = torch.empty(self.batch, dtype=torch.float64, device="cuda")
        _check(load().cbs_loss_seed(self._h, _ptr(self._field(u_k, "u_k")), _ptr(self._field(s, "s")),
                                    _weight_code(weight), _ptr(loss), _ptr(lam), _ptr(grad),
                                    self._st(stream)))
        return loss, lam, grad

    def autotune(self, stream=None) -> List[int]:
        """Per-size-class column tile autotuning; returns the width per instance."""
        t = (ctypes.c_int32 * self.batch)()
        _check(load().cbs_autotune(self._h, t, self._st(stream)))
        return list(t)

    def layout(self):
        """(lane streams used by sweep chains, column tile width per instance)."""
        lanes = ctypes.c_int32()
        t = (ctypes.c_int32 * self.batch)()
        _check(load().cbs_plan_layout(self._h, ctypes.byref(lanes), t, None))
        return int(lanes.value), list(t)

    def col_threads(self) -> int:
        """Threads per workgroup of the plan's column launches (256 or 512)."""
        thr = ctypes.c_int32()
        _check(load().cbs_plan_layout(self._h, None, None, ctypes.byref(thr)))
        return int(thr.value)

    def set_col_threads(self, threads: int):
        _check(load().cbs_set_col_threads(self._h, int(threads)))

    def set_tile(self, columns: int, n: int = 0):
        _check(load().cbs_set_tile(self._h, int(n), int(columns)))


class CdrPlan(Plan):
    """A batch of periodic convection-diffusion-reaction instances
    -div(kappa grad u) + v . grad u + sigma u = s (cbs_setup_cdr).

    kappa_sigma: packed complex tensor, real part kappa, imaginary part sigma;
    velocity: packed complex tensor, real part vx, imaginary part vy (x is the
    fast axis); background: per instance (kappa0, vx0, vy0, sigma0).  apply,
    residual, born_adjoint and helmholtz_residual (here s - A u with the CDR
    operator; also as physical_residual) run on it."""

    def __init__(self, kappa_sigma: torch.Tensor, velocity: torch.Tensor, sizes: Sequence[int],
                 background, dtype: int = CBS_C64, stream=None):
        lib = load()
        self.sizes = [int(n) for n in sizes]
        self.batch = len(self.sizes)
        self.dtype = dtype
        self.tdtype = torch.complex64 if dtype == CBS_C64 else torch.complex128
        self.cells = sum(n * n for n in self.sizes)
        for name, t in (("kappa_sigma", kappa_sigma), ("velocity", velocity)):
            if t.dtype != self.tdtype or t.numel() != self.cells or not t.is_cuda:
                raise ValueError(f"{name} must be a packed CUDA tensor of the plan dtype")
        bg = [tuple(float(v) for v in b) for b in _expand(background, self.batch)]
        if any(len(b) != 4 for b in bg):
            raise ValueError("background: (kappa0, vx0, vy0, sigma0) per instance")
        n_arr = (ctypes.c_int32 * self.batch)(*self.sizes)
        bg_arr = (ctypes.c_double * (4 * self.batch))(*[v for b in bg for v in b])
        h = ctypes.c_void_p()
        self.dirichlet = False
        self.undamped = False
        self._ws = torch.empty(workspace_size_cdr(self.sizes, dtype), dtype=torch.uint8, device="cuda")
        self._ws_stream = torch.cuda.current_stream()
        _check(lib.cbs_setup_cdr_ws(ctypes.byref(h), self.batch, n_arr, _ptr(kappa_sigma.contiguous()),
                                    _ptr(velocity.contiguous()), bg_arr, dtype, _ptr(self._ws),
                                    self._ws.numel(), _stream(stream)))
        self._h = h
        self.max_restart = 0
        self.background = bg
        self.k0sq = [b[0] for b in bg]
        self.eps = [b[3] for b in bg]

    def physical_residual(self, u, s, out=None, norms=True, store=True, stream=None):
        """r = s - A u with the CDR operator, and per-instance sums |r|^2."""
        return self.helmholtz_residual(u, s, out=out, norms=norms, store=store, stream=stream)


class MetricMatchedLoss(torch.autograd.Function):
    """ell_b = || G s - (I - G V) x ||^2 per instance: the residual of the
    metric-matched objective (Sec. 4.2; Eq. cdr_bs_loss for CDR plans) for a
    network output x (with s the residual being preconditioned).  Backward:
    dl/dx = -2 R^H (G s - R x) by cbs_metric_matched_grad (PyTorch's convention)."""

    @staticmethod
    def forward(ctx, x, plan, s):
        x = x.detach().contiguous()
        _, n2 = plan.residual(x, s, store=False)
        ctx.plan = plan
        ctx.x = x
        ctx.s = s
        return n2

    @staticmethod
    def backward(ctx, gout):
        # the library recomputes the residual and forms -2 gout_i R^H r
        _, gx = ctx.plan.metric_matched_grad(ctx.x, ctx.s, scale=gout)
        ctx.plan = None
        return gx, None, None


def metric_matched_loss(x, plan, s):
    """Per-instance || G s - (I - G V) x ||^2 (float64), differentiable in x."""
    return MetricMatchedLoss.apply(x, plan, s)


_WEIGHTS = {"one": 0, "gamma": 1, "physical": 2}
_STOPS = {"born": 0, "physical": 1}


def _weight_code(weight) -> int:
    if isinstance(weight, bool):
        return 1 if weight else 0
    if weight not in _WEIGHTS:
        raise ValueError(f"weight must be one of {sorted(_WEIGHTS)}")
    return _WEIGHTS[weight]


def _expand(v, n):
    if isinstance(v, (list, tuple, np.ndarray)):
        if len(v) != n:
            raise ValueError("per-instance parameter has the wrong length")
        return list(v)
    return [v] * n


class BornResidualLoss(torch.autograd.Function):
    """ell = sum_b || W (G s - (I - G V) u_K) ||^2 after K CBS steps from u0
    (the metric-matched residual of Sec. 4.2 with W = gamma or W = 1), or
    ell = sum_b || s - A u_K ||^2 with weight "physical" (the residual that
    L_dir, Sec. 4, and L_bs^{l2}, Sec. 4.2, measure).

    Forward keeps the checkpoints u_0..u_K; backward runs the hand-written
    adjoint (cbs_adjoint_step) from the seed computed by cbs_loss_seed.
    Returns per-instance losses (float64).  Gradients w.r.t. u0 and the packed
    complex k2 follow PyTorch's convention d/dRe + i d/dIm; eps and k0^2 are
    constants (taken from the plan built on k2 in forward).
    """

    @staticmethod
    def forward(ctx, u0, k2, s, sizes, steps, weight, k0sq, eps):
        dtype = CBS_C128 if k2.dtype == torch.complex128 else CBS_C64
        plan = Plan(k2.detach(), sizes, k0sq=k0sq, eps=eps, dtype=dtype)
        if int(steps) > 0:
            # one fused chain that keeps every iterate (cbs_sweep_checkpoints)
            u_all = plan.sweep_checkpoints(u0.detach(), s, int(steps))
            us = [u_all[k] for k in range(int(steps) + 1)]
        else:
            us = [u0.detach().clone()]
        loss, lam, grad = plan.loss_seed(us[-1], s, weight)
        ctx.plan = plan
        ctx.us = us
        ctx.s = s
        ctx.lam = lam
        ctx.grad = grad
        return loss

    @staticmethod
    def backward(ctx, gout):
        plan, us, s = ctx.plan, ctx.us, ctx.s
        lam, grad = ctx.lam, ctx.grad
        for m in range(len(us) - 2, -1, -1):
            plan.adjoint_step(us[m], s, lam, lam, grad)
        scale = torch.repeat_interleave(gout.to(torch.float64),
                                        torch.tensor([n * n for n in plan.sizes], device=gout.device))
        scale = scale.to(lam.real.dtype)
        gu = lam * scale
        gk = grad * scale
        ctx.plan = None
        return gu, gk, None, None, None, None, None, None


def born_residual_loss(u0, k2, s, sizes, steps=8, weight="gamma", k0sq=None, eps=None):
    """weight: "gamma", "one" or "physical" (see BornResidualLoss)."""
    _weight_code(weight)
    return BornResidualLoss.apply(u0, k2, s, list(sizes), int(steps), weight, k0sq, eps)
