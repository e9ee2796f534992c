"""Python binding of libslnk.so, the MI355X (gfx950) semi-Lagrangian Newton--Krylov path.

Argument marshalling only: every step of the method runs in the HIP library behind the C ABI of
include/slnk.h.  Fields are torch tensors on the GPU (float32 for the mixed-precision context,
float64 for the FP64 context); PyTorch provides device memory and the stream, nothing else.
There is no CPU fallback: without the built library every call raises.
"""

from __future__ import annotations

import ctypes
import os

__all__ = ["Context", "Context3", "BatchContext", "UNet", "library_path", "load_library", "SolveOpts", "STATUS"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

STATUS = {0: "SLNK_OK", 1: "SLNK_EINVAL", 2: "SLNK_ENOMEM", 3: "SLNK_EDEVICE", 4: "SLNK_ENAN",
          5: "SLNK_ELINESEARCH", 6: "SLNK_ENEGCURV", 7: "SLNK_EMAXIT", 8: "SLNK_ECHEB_DIVERGED"}
REG = {"h1": 1, "h2": 2, "h3": 3}
PREC = {"fp64": 0, "mixed": 1}
PC = {"reg": 1, "2l": 2}
HESSIAN = {"gn": 0, "fn": 1}
PROJ = {"none": 0, "leray": 1}
TRANSPORT = {"sl": 0, "rk2a": 1}
COARSE = {"cheb": 0, "pcg": 1}
REPORT_MAX = 64


class Params(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int), ("n2", ctypes.c_int), ("nt", ctypes.c_int), ("reg", ctypes.c_int),
                ("beta", ctypes.c_double), ("prec", ctypes.c_int), ("pc", ctypes.c_int),
                ("cheb_iters", ctypes.c_int), ("lanczos_steps", ctypes.c_int),
                ("emax_safety", ctypes.c_double), ("lanczos_seed", ctypes.c_ulonglong), ("use_graphs", ctypes.c_int),
                ("batch", ctypes.c_int), ("sl_path", ctypes.c_int), ("hessian", ctypes.c_int),
                ("proj", ctypes.c_int), ("coarse_solver", ctypes.c_int), ("coarse_eps", ctypes.c_double),
                ("transport", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("max_newton", ctypes.c_int), ("gtol_rel", ctypes.c_double), ("gtol_abs", ctypes.c_double),
                ("max_pcg", ctypes.c_int), ("armijo_c1", ctypes.c_double), ("max_halvings", ctypes.c_int)]


class SolveReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("newton_iters", ctypes.c_int), ("pcg_iters", ctypes.c_int),
                ("matvecs", ctypes.c_int), ("coarse_matvecs", ctypes.c_int), ("line_search_evals", ctypes.c_int),
                ("g0_inf", ctypes.c_double), ("g0_two", ctypes.c_double), ("emin", ctypes.c_double),
                ("emax", ctypes.c_double), ("grel", ctypes.c_double * (REPORT_MAX + 1)),
                ("J", ctypes.c_double * (REPORT_MAX + 1)), ("pcg", ctypes.c_int * (REPORT_MAX + 1)),
                ("time_total_ms", ctypes.c_double), ("time_gradient_ms", ctypes.c_double),
                ("time_pcg_ms", ctypes.c_double), ("time_precond_ms", ctypes.c_double),
                ("time_linesearch_ms", ctypes.c_double), ("time_to_stop_ms", ctypes.c_double),
                ("fallback", ctypes.c_int), ("cheb_reestimates", ctypes.c_int)]


class Params3(ctypes.Structure):
    _fields_ = [("n1", ctypes.c_int), ("n2", ctypes.c_int), ("n3", ctypes.c_int), ("nt", ctypes.c_int),
                ("reg", ctypes.c_int), ("beta", ctypes.c_double), ("prec", ctypes.c_int), ("proj", ctypes.c_int),
                ("sl_path", ctypes.c_int), ("pc", ctypes.c_int), ("cheb_iters", ctypes.c_int),
                ("lanczos_steps", ctypes.c_int), ("emax_safety", ctypes.c_double), ("lanczos_seed", ctypes.c_ulonglong),
                ("hessian", ctypes.c_int), ("coarse_solver", ctypes.c_int), ("coarse_eps", ctypes.c_double),
                ("transport", ctypes.c_int)]


class UNetParams(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int), ("width", ctypes.c_int), ("levels", ctypes.c_int),
                ("base_channels", ctypes.c_int), ("max_batch", ctypes.c_int), ("seed", ctypes.c_ulonglong),
                ("start_kmax", ctypes.c_int)]


EXPORTS = ["slnk_default_params", "slnk_default_opts", "slnk_create", "slnk_destroy", "slnk_last_error",
           "slnk_workspace_bytes", "slnk_set_images", "slnk_transport_state", "slnk_transport_state_noalloc", "slnk_objective", "slnk_gradient",
           "slnk_hessian_matvec", "slnk_split_matvec", "slnk_precond_apply", "slnk_get_cheb_bounds",
           "slnk_get_field", "slnk_set_cheb_emax", "slnk_time_kernel", "slnk_newton_solve", "slnk_batch_create", "slnk_batch_destroy",
           "slnk_batch_last_error", "slnk_batch_bucket_info", "slnk_batch_set_images", "slnk_batch_gradient",
           "slnk_batch_hessian_matvec", "slnk_batch_newton_solve", "slnk_batch_autotune", "slnk_unet_default_params",
           "slnk_unet_create", "slnk_unet_destroy", "slnk_unet_last_error", "slnk_unet_param_count",
           "slnk_unet_get_params", "slnk_unet_set_params", "slnk_unet_get_grads", "slnk_unet_forward",
           "slnk_unet_train_step", "slnk_unet_conv_variants", "slnk_set_images_learned", "slnk_newton_solve_learned"]
# include/slnk3.h
EXPORTS3 = ["slnk3_default_params", "slnk3_create", "slnk3_destroy", "slnk3_last_error", "slnk3_workspace_bytes",
            "slnk3_set_images", "slnk3_transport_state", "slnk3_objective", "slnk3_gradient",
            "slnk3_hessian_matvec", "slnk3_precond_apply", "slnk3_split_matvec", "slnk3_get_cheb_bounds",
            "slnk3_newton_solve"]


def library_path() -> str:
    return os.path.join(_HERE, "libslnk.so")


def load_library():
    """Load libslnk.so (built by paper_1604_02153_amd.build); raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1604_02153_amd.build`")
    lib = ctypes.CDLL(path)
    P, V = ctypes.POINTER, ctypes.c_void_p
    sig = {
        "slnk_default_params": (None, [P(Params)]),
        "slnk_default_opts": (None, [P(SolveOpts)]),
        "slnk_create": (ctypes.c_int, [P(Params), V, P(V)]),
        "slnk_destroy": (None, [V]),
        "slnk_last_error": (ctypes.c_char_p, [V]),
        "slnk_workspace_bytes": (ctypes.c_ulonglong, [V]),
        "slnk_set_images": (ctypes.c_int, [V, V, V]),
        "slnk_transport_state": (ctypes.c_int, [V, V, V, V]),
        "slnk_transport_state_noalloc": (ctypes.c_int, [P(Params), V, V, V, V, ctypes.c_char_p, ctypes.c_size_t]),
        "slnk_objective": (ctypes.c_int, [V, V, P(ctypes.c_double)]),
        "slnk_gradient": (ctypes.c_int, [V, V, V, P(ctypes.c_double)]),
        "slnk_hessian_matvec": (ctypes.c_int, [V, V, V]),
        "slnk_split_matvec": (ctypes.c_int, [V, V, V]),
        "slnk_precond_apply": (ctypes.c_int, [V, V, V]),
        "slnk_get_cheb_bounds": (ctypes.c_int, [V, P(ctypes.c_double), P(ctypes.c_double)]),
        "slnk_get_field": (ctypes.c_int, [V, ctypes.c_int, V]),
        "slnk_set_cheb_emax": (ctypes.c_int, [V, P(ctypes.c_double)]),
        "slnk_time_kernel": (ctypes.c_int, [V, ctypes.c_int, ctypes.c_int, P(ctypes.c_double)]),
        "slnk_newton_solve": (ctypes.c_int, [V, V, P(SolveOpts), P(SolveReport)]),
        "slnk_batch_create": (ctypes.c_int, [P(Params), ctypes.c_int, P(ctypes.c_int), P(ctypes.c_int), V, P(V)]),
        "slnk_batch_destroy": (None, [V]),
        "slnk_batch_last_error": (ctypes.c_char_p, [V]),
        "slnk_batch_bucket_info": (ctypes.c_int, [V, ctypes.c_int] + [P(ctypes.c_int)] * 5),
        "slnk_batch_set_images": (ctypes.c_int, [V, P(V), P(V)]),
        "slnk_batch_gradient": (ctypes.c_int, [V, P(V), P(V), P(ctypes.c_double)]),
        "slnk_batch_hessian_matvec": (ctypes.c_int, [V, P(V), P(V)]),
        "slnk_batch_newton_solve": (ctypes.c_int, [V, P(V), P(SolveOpts), P(SolveReport)]),
        "slnk_batch_autotune": (ctypes.c_int, [V, P(V), ctypes.c_int, P(ctypes.c_double)]),
        "slnk_unet_default_params": (None, [P(UNetParams)]),
        "slnk_unet_create": (ctypes.c_int, [P(UNetParams), V, P(V)]),
        "slnk_unet_destroy": (None, [V]),
        "slnk_unet_last_error": (ctypes.c_char_p, [V]),
        "slnk_unet_param_count": (ctypes.c_longlong, [V]),
        "slnk_unet_get_params": (ctypes.c_int, [V, V]),
        "slnk_unet_set_params": (ctypes.c_int, [V, V]),
        "slnk_unet_get_grads": (ctypes.c_int, [V, V]),
        "slnk_unet_forward": (ctypes.c_int, [V, ctypes.c_int, V, V, V, V]),
        "slnk_unet_train_step": (ctypes.c_int, [V, ctypes.c_int, V, V, V, V, ctypes.c_double, P(ctypes.c_double),
                                                P(ctypes.c_double)]),
        "slnk_unet_conv_variants": (None, [P(ctypes.c_longlong), ctypes.c_int]),
        "slnk_set_images_learned": (ctypes.c_int, [V, V, V, V]),
        "slnk_newton_solve_learned": (ctypes.c_int, [V, V, V, P(SolveOpts), P(SolveReport)]),
        "slnk3_default_params": (None, [P(Params3)]),
        "slnk3_create": (ctypes.c_int, [P(Params3), V, P(V)]),
        "slnk3_destroy": (None, [V]),
        "slnk3_last_error": (ctypes.c_char_p, [V]),
        "slnk3_workspace_bytes": (ctypes.c_ulonglong, [V]),
        "slnk3_set_images": (ctypes.c_int, [V, V, V]),
        "slnk3_transport_state": (ctypes.c_int, [V, V, V, V]),
        "slnk3_objective": (ctypes.c_int, [V, V, P(ctypes.c_double)]),
        "slnk3_gradient": (ctypes.c_int, [V, V, V, P(ctypes.c_double)]),
        "slnk3_hessian_matvec": (ctypes.c_int, [V, V, V]),
        "slnk3_precond_apply": (ctypes.c_int, [V, V, V]),
        "slnk3_split_matvec": (ctypes.c_int, [V, V, V]),
        "slnk3_get_cheb_bounds": (ctypes.c_int, [V, P(ctypes.c_double), P(ctypes.c_double)]),
        "slnk3_newton_solve": (ctypes.c_int, [V, V, P(SolveOpts), P(SolveReport)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


class SlnkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    load_library().slnk_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """A batch of same-size registration problems on the current GPU (see include/slnk.h for every
    call).  With batch == 1 fields have their plain shapes ([n1, n2], [2, n1, n2]) and scalar
    results are numbers; with batch B > 1 every field carries a leading item axis of length B and
    scalar results are lists of B values."""

    def __init__(self, n1, n2, nt, reg="h2", beta=1e-3, prec="mixed", pc="2l", cheb_iters=10,
                 lanczos_steps=30, emax_safety=1.05, lanczos_seed=0x5EED, use_graphs=True, stream=None,
                 batch=1, sl_path=0, hessian="gn", proj="none", coarse_solver="cheb", coarse_eps=0.1,
                 transport="sl"):
        import torch
        lib = load_library()
        p = Params()
        lib.slnk_default_params(ctypes.byref(p))
        p.n1, p.n2, p.nt = int(n1), int(n2), int(nt)
        p.reg = REG[reg] if isinstance(reg, str) else int(reg)
        p.beta = float(beta)
        p.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        p.pc = PC[pc] if isinstance(pc, str) else int(pc)
        p.cheb_iters, p.lanczos_steps = int(cheb_iters), int(lanczos_steps)
        p.emax_safety, p.lanczos_seed = float(emax_safety), int(lanczos_seed)
        p.use_graphs = 1 if use_graphs else 0
        p.batch = int(batch)
        p.sl_path = int(sl_path)
        p.hessian = HESSIAN[hessian] if isinstance(hessian, str) else int(hessian)
        p.proj = PROJ[proj] if isinstance(proj, str) else int(proj)
        p.coarse_solver = COARSE[coarse_solver] if isinstance(coarse_solver, str) else int(coarse_solver)
        p.coarse_eps = float(coarse_eps)
        p.transport = TRANSPORT[transport] if isinstance(transport, str) else int(transport)
        self.batch = p.batch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.dtype = torch.float64 if p.prec == 0 else torch.float32
        self.shape = (p.n1, p.n2)
        self.params = p
        self._lib = lib
        self._ctx = ctypes.c_void_p()
        self._check(lib.slnk_create(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self._ctx)))

    # -- helpers --------------------------------------------------------------------------------
    def _check(self, st):
        if st != 0:
            msg = self._lib.slnk_last_error(self._ctx).decode() if self._ctx else ""
            raise SlnkError(st, msg)

    def _ptr(self, t, ncomp):
        shape = self.shape if ncomp == 1 else (ncomp,) + self.shape
        if self.batch > 1 or (t.dim() == len(shape) + 1):
            shape = (self.batch,) + shape
        if not t.is_cuda or t.dtype != self.dtype or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {self.dtype} CUDA tensor of shape {shape}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")
        return ctypes.c_void_p(t.data_ptr())

    def close(self):
        if self._ctx:
            self._lib.slnk_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI ---------------------------------------------------------------------------------
    def workspace_bytes(self) -> int:
        return int(self._lib.slnk_workspace_bytes(self._ctx))

    def set_images(self, m_R, m_T):
        self._check(self._lib.slnk_set_images(self._ctx, self._ptr(m_R, 1), self._ptr(m_T, 1)))

    def transport_state(self, v, m0, m1):
        self._check(self._lib.slnk_transport_state(self._ctx, self._ptr(v, 2), self._ptr(m0, 1), self._ptr(m1, 1)))

    def _scalars(self, arr):
        vals = list(arr)
        return vals[0] if self.batch == 1 else vals

    def objective(self, v):
        J = (ctypes.c_double * self.batch)()
        self._check(self._lib.slnk_objective(self._ctx, self._ptr(v, 2), J))
        return self._scalars(J)

    def gradient(self, v, g):
        J = (ctypes.c_double * self.batch)()
        self._check(self._lib.slnk_gradient(self._ctx, self._ptr(v, 2), self._ptr(g, 2), J))
        return self._scalars(J)

    def hessian_matvec(self, vt, out):
        self._check(self._lib.slnk_hessian_matvec(self._ctx, self._ptr(vt, 2), self._ptr(out, 2)))

    def split_matvec(self, s, out):
        self._check(self._lib.slnk_split_matvec(self._ctx, self._ptr(s, 2), self._ptr(out, 2)))

    def precond_apply(self, r, z):
        self._check(self._lib.slnk_precond_apply(self._ctx, self._ptr(r, 2), self._ptr(z, 2)))

    def cheb_bounds(self):
        a, b = (ctypes.c_double * self.batch)(), (ctypes.c_double * self.batch)()
        self._check(self._lib.slnk_get_cheb_bounds(self._ctx, a, b))
        if self.batch == 1:
            return a[0], b[0]
        return list(zip(a, b))

    def set_cheb_emax(self, emax):
        """Chebyshev upper bound(s) of P_2L in place of the Lanczos estimate (one float per item)."""
        vals = [float(emax)] if self.batch == 1 and not hasattr(emax, "__len__") else [float(x) for x in emax]
        if len(vals) != self.batch:
            raise ValueError(f"expected {self.batch} values")
        self._check(self._lib.slnk_set_cheb_emax(self._ctx, (ctypes.c_double * self.batch)(*vals)))

    def get_field(self, which, out):
        ncomp = 2 if which in (1, 2) else 1
        self._check(self._lib.slnk_get_field(self._ctx, int(which), self._ptr(out, ncomp)))

    def time_kernel(self, which, reps) -> float:
        """Average duration (ms) of one launch of a hot-path kernel: reps launches back to back
        between two HIP events on the library's stream."""
        ms = ctypes.c_double()
        self._check(self._lib.slnk_time_kernel(self._ctx, int(which), int(reps), ctypes.byref(ms)))
        return ms.value

    def newton_solve(self, v, opts: SolveOpts | None = None, **kw):
        """Newton--Krylov solve in place; one report dict (batch 1) or a list of B dicts."""
        if opts is None:
            opts = default_opts(**kw)
        reps = (SolveReport * self.batch)()
        st = self._lib.slnk_newton_solve(self._ctx, self._ptr(v, 2), ctypes.byref(opts), reps)
        if st not in (0, 5, 7, 8):  # reported per item: failed line search, Newton limit, indefinite P_2L
            self._check(st)
        out = [self._report(r) for r in reps]
        return out[0] if self.batch == 1 else out

    def set_images_learned(self, unet, m_R, m_T):
        """set_images with the network: its head gives e_max (no Lanczos) and its start is kept."""
        self._check(self._lib.slnk_set_images_learned(self._ctx, unet._u, self._ptr(m_R, 1), self._ptr(m_T, 1)))

    def newton_solve_learned(self, unet, v, opts: SolveOpts | None = None, **kw):
        """Warm start v = unet(m_R, m_T) (written into v), then the Newton--Krylov solve."""
        if opts is None:
            opts = default_opts(**kw)
        reps = (SolveReport * self.batch)()
        st = self._lib.slnk_newton_solve_learned(self._ctx, unet._u, self._ptr(v, 2), ctypes.byref(opts), reps)
        if st not in (0, 5, 7, 8):  # reported per item: failed line search, Newton limit, indefinite P_2L
            self._check(st)
        out = [self._report(r) for r in reps]
        return out[0] if self.batch == 1 else out

    @staticmethod
    def _report(rep) -> dict:
        k = rep.newton_iters
        return {
            "status": STATUS.get(rep.status, rep.status), "newton_iters": k, "pcg_iters": rep.pcg_iters, "matvecs": rep.matvecs,
            "coarse_matvecs": rep.coarse_matvecs, "line_search_evals": rep.line_search_evals,
            "g0_inf": rep.g0_inf, "g0_two": rep.g0_two, "emin": rep.emin, "emax": rep.emax,
            "grel": list(rep.grel[: k + 1]), "J": list(rep.J[: k + 1]), "pcg": list(rep.pcg[:k]),
            "time_total_ms": rep.time_total_ms, "time_gradient_ms": rep.time_gradient_ms,
            "time_pcg_ms": rep.time_pcg_ms, "time_precond_ms": rep.time_precond_ms,
            "time_linesearch_ms": rep.time_linesearch_ms, "time_to_stop_ms": rep.time_to_stop_ms,
            "fallback": bool(rep.fallback), "cheb_reestimates": rep.cheb_reestimates,
        }


class Context3:
    """One registration problem on a periodic n1 x n2 x n3 volume (include/slnk3.h): scalar fields
    [n1, n2, n3], velocities [3, n1, n2, n3] (float32 for prec="mixed", float64 for "fp64")."""

    def __init__(self, n1, n2, n3, nt, reg="h2", beta=1e-3, prec="mixed", proj="none", sl_path=0, pc="reg",
                 cheb_iters=10, lanczos_steps=30, emax_safety=1.05, lanczos_seed=0x5EED, hessian="gn",
                 coarse_solver="cheb", coarse_eps=0.1, transport="sl", stream=None):
        import torch
        lib = load_library()
        p = Params3()
        lib.slnk3_default_params(ctypes.byref(p))
        p.n1, p.n2, p.n3, p.nt = int(n1), int(n2), int(n3), int(nt)
        p.reg = REG[reg] if isinstance(reg, str) else int(reg)
        p.beta = float(beta)
        p.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        p.proj = PROJ[proj] if isinstance(proj, str) else int(proj)
        p.sl_path = int(sl_path)
        p.pc = PC[pc] if isinstance(pc, str) else int(pc)
        p.cheb_iters, p.lanczos_steps = int(cheb_iters), int(lanczos_steps)
        p.emax_safety, p.lanczos_seed = float(emax_safety), int(lanczos_seed)
        p.hessian = HESSIAN[hessian] if isinstance(hessian, str) else int(hessian)
        p.coarse_solver = COARSE[coarse_solver] if isinstance(coarse_solver, str) else int(coarse_solver)
        p.coarse_eps = float(coarse_eps)
        p.transport = TRANSPORT[transport] if isinstance(transport, str) else int(transport)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.dtype = torch.float64 if p.prec == 0 else torch.float32
        self.shape = (p.n1, p.n2, p.n3)
        self.params = p
        self._lib = lib
        self._ctx = ctypes.c_void_p()
        self._check(lib.slnk3_create(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self._ctx)))

    def _check(self, st):
        if st != 0:
            msg = self._lib.slnk3_last_error(self._ctx).decode() if self._ctx else ""
            raise SlnkError(st, msg)

    def _ptr(self, t, ncomp):
        shape = self.shape if ncomp == 1 else (ncomp,) + self.shape
        if not t.is_cuda or t.dtype != self.dtype or tuple(t.shape) != shape or not t.is_contiguous():
            raise ValueError(f"expected a contiguous {self.dtype} CUDA tensor of shape {shape}, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")
        return ctypes.c_void_p(t.data_ptr())

    def close(self):
        if self._ctx:
            self._lib.slnk3_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self) -> int:
        return int(self._lib.slnk3_workspace_bytes(self._ctx))

    def set_images(self, m_R, m_T):
        self._check(self._lib.slnk3_set_images(self._ctx, self._ptr(m_R, 1), self._ptr(m_T, 1)))

    def transport_state(self, v, m0, m1):
        self._check(self._lib.slnk3_transport_state(self._ctx, self._ptr(v, 3), self._ptr(m0, 1),
                                                    self._ptr(m1, 1)))

    def objective(self, v) -> float:
        J = ctypes.c_double()
        self._check(self._lib.slnk3_objective(self._ctx, self._ptr(v, 3), ctypes.byref(J)))
        return J.value

    def gradient(self, v, g) -> float:
        J = ctypes.c_double()
        self._check(self._lib.slnk3_gradient(self._ctx, self._ptr(v, 3), self._ptr(g, 3), ctypes.byref(J)))
        return J.value

    def hessian_matvec(self, vt, out):
        self._check(self._lib.slnk3_hessian_matvec(self._ctx, self._ptr(vt, 3), self._ptr(out, 3)))

    def precond_apply(self, r, z):
        self._check(self._lib.slnk3_precond_apply(self._ctx, self._ptr(r, 3), self._ptr(z, 3)))

    def split_matvec(self, s, out):
        self._check(self._lib.slnk3_split_matvec(self._ctx, self._ptr(s, 3), self._ptr(out, 3)))

    def cheb_bounds(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.slnk3_get_cheb_bounds(self._ctx, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def newton_solve(self, v, opts: SolveOpts | None = None, **kw):
        """Newton--Krylov solve (the GN or FN matvec; P_REG or P_2L) in place; the report as a dict."""
        if opts is None:
            opts = default_opts(**kw)
        rep = SolveReport()
        st = self._lib.slnk3_newton_solve(self._ctx, self._ptr(v, 3), ctypes.byref(opts), ctypes.byref(rep))
        if st not in (0, 5, 7, 8):  # failed line search, Newton limit, indefinite P_2L: reported
            self._check(st)
        return Context._report(rep)


def transport_state_noalloc(v, m0, m1, nt, sl_path=0, stream=None):
    """State transport of m0 by v over nt SL steps into m1 (include/slnk.h,
    slnk_transport_state_noalloc): no context and no device allocation.  Tensors on one CUDA device,
    float32 (mixed precision) or float64, v [B][2][n1][n2] or [2][n1][n2], m0 and m1 the matching
    scalar fields."""
    import torch
    lib = load_library()
    batched = v.dim() == 4
    B = v.shape[0] if batched else 1
    n1, n2 = v.shape[-2], v.shape[-1]
    dt = v.dtype
    if dt not in (torch.float32, torch.float64):
        raise ValueError("v must be float32 or float64")
    want = {id(v): (B, 2, n1, n2) if batched else (2, n1, n2), id(m0): (B, n1, n2) if batched else (n1, n2),
            id(m1): (B, n1, n2) if batched else (n1, n2)}
    for t in (v, m0, m1):
        if not t.is_cuda or t.dtype != dt or tuple(t.shape) != want[id(t)] or not t.is_contiguous():
            raise ValueError(f"expected contiguous {dt} CUDA tensors of shapes {list(want.values())}")
    p = Params()
    lib.slnk_default_params(ctypes.byref(p))
    p.n1, p.n2, p.nt, p.batch, p.sl_path = int(n1), int(n2), int(nt), int(B), int(sl_path)
    p.prec = 0 if dt == torch.float64 else 1
    if stream is None:
        stream = torch.cuda.current_stream()
    msg = ctypes.create_string_buffer(256)
    st = lib.slnk_transport_state_noalloc(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream),
                                          ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(m0.data_ptr()),
                                          ctypes.c_void_p(m1.data_ptr()), msg, 256)
    if st != 0:
        raise SlnkError(st, msg.value.decode())


class BatchContext:
    """Independent problems of uneven grid sizes (include/slnk.h, ragged batches).  sizes is a
    list of (n1, n2) per pair; every per-pair argument is a list of tensors (pair order)."""

    def __init__(self, sizes, nt, reg="h2", beta=1e-3, prec="mixed", pc="2l", cheb_iters=10, lanczos_steps=30,
                 emax_safety=1.05, lanczos_seed=0x5EED, use_graphs=True, sl_path=0, stream=None, hessian="gn",
                 proj="none", coarse_solver="cheb", coarse_eps=0.1, transport="sl"):
        import torch
        lib = load_library()
        p = Params()
        lib.slnk_default_params(ctypes.byref(p))
        p.nt = int(nt)
        p.reg = REG[reg] if isinstance(reg, str) else int(reg)
        p.beta = float(beta)
        p.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        p.pc = PC[pc] if isinstance(pc, str) else int(pc)
        p.cheb_iters, p.lanczos_steps = int(cheb_iters), int(lanczos_steps)
        p.emax_safety, p.lanczos_seed = float(emax_safety), int(lanczos_seed)
        p.use_graphs, p.sl_path = (1 if use_graphs else 0), int(sl_path)
        p.hessian = HESSIAN[hessian] if isinstance(hessian, str) else int(hessian)
        p.proj = PROJ[proj] if isinstance(proj, str) else int(proj)
        p.coarse_solver = COARSE[coarse_solver] if isinstance(coarse_solver, str) else int(coarse_solver)
        p.coarse_eps = float(coarse_eps)
        p.transport = TRANSPORT[transport] if isinstance(transport, str) else int(transport)
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        self.npairs = len(self.sizes)
        n1 = (ctypes.c_int * self.npairs)(*[a for a, _ in self.sizes])
        n2 = (ctypes.c_int * self.npairs)(*[b for _, b in self.sizes])
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.dtype = torch.float64 if p.prec == 0 else torch.float32
        self._lib = lib
        self._b = ctypes.c_void_p()
        self._check(lib.slnk_batch_create(ctypes.byref(p), self.npairs, n1, n2, ctypes.c_void_p(stream.cuda_stream),
                                          ctypes.byref(self._b)))

    def _check(self, st):
        if st != 0:
            msg = self._lib.slnk_batch_last_error(self._b).decode() if self._b else ""
            raise SlnkError(st, msg)

    def _ptrs(self, ts, ncomp):
        if len(ts) != self.npairs:
            raise ValueError(f"expected {self.npairs} tensors, got {len(ts)}")
        out = (ctypes.c_void_p * self.npairs)()
        for p, (t, (a, b)) in enumerate(zip(ts, self.sizes)):
            shape = (a, b) if ncomp == 1 else (ncomp, a, b)
            if not t.is_cuda or t.dtype != self.dtype or tuple(t.shape) != shape or not t.is_contiguous():
                raise ValueError(f"pair {p}: expected a contiguous {self.dtype} CUDA tensor of shape {shape}")
            out[p] = t.data_ptr()
        return out

    def close(self):
        if self._b:
            self._lib.slnk_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def buckets(self):
        """[(n1, n2, pairs, sl_path, use_graphs)] per bucket."""
        c = ctypes.c_int()
        self._check(self._lib.slnk_batch_bucket_info(self._b, -1, None, None, ctypes.byref(c), None, None))
        out = []
        for k in range(c.value):
            v = [ctypes.c_int() for _ in range(5)]
            self._check(self._lib.slnk_batch_bucket_info(self._b, k, *[ctypes.byref(x) for x in v]))
            out.append(tuple(x.value for x in v))
        return out

    def set_images(self, m_R, m_T):
        self._check(self._lib.slnk_batch_set_images(self._b, self._ptrs(m_R, 1), self._ptrs(m_T, 1)))

    def gradient(self, v, g):
        J = (ctypes.c_double * self.npairs)()
        self._check(self._lib.slnk_batch_gradient(self._b, self._ptrs(v, 2), self._ptrs(g, 2), J))
        return list(J)

    def hessian_matvec(self, vt, out):
        self._check(self._lib.slnk_batch_hessian_matvec(self._b, self._ptrs(vt, 2), self._ptrs(out, 2)))

    def autotune(self, vt, reps=5):
        nb = len(self.buckets())
        best = (ctypes.c_double * nb)()
        self._check(self._lib.slnk_batch_autotune(self._b, self._ptrs(vt, 2), int(reps), best))
        return list(best)

    def newton_solve(self, v, opts: SolveOpts | None = None, **kw):
        if opts is None:
            opts = default_opts(**kw)
        reps = (SolveReport * self.npairs)()
        st = self._lib.slnk_batch_newton_solve(self._b, self._ptrs(v, 2), ctypes.byref(opts), reps)
        if st not in (0, 5, 7, 8):  # reported per item: failed line search, Newton limit, indefinite P_2L
            self._check(st)
        return [Context._report(r) for r in reps]


class UNet:
    """The learned warm start (include/slnk.h): a periodic conv U-Net on BF16 matrix cores.
    Images are float32 CUDA tensors [batch, H, W]; velocities [batch, 2, H, W]."""

    def __init__(self, height=256, width=256, levels=4, base_channels=32, max_batch=16, seed=0xC0FFEE, stream=None,
                 start_kmax=8):
        import torch
        lib = load_library()
        p = UNetParams()
        lib.slnk_unet_default_params(ctypes.byref(p))
        p.height, p.width, p.levels = int(height), int(width), int(levels)
        p.base_channels, p.max_batch, p.seed = int(base_channels), int(max_batch), int(seed)
        p.start_kmax = int(start_kmax)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.params = p
        self._lib = lib
        self._u = ctypes.c_void_p()
        st = lib.slnk_unet_create(ctypes.byref(p), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(self._u))
        if st != 0:
            raise SlnkError(st, "slnk_unet_create failed (sizes, channels or memory)")
        self.n_params = int(lib.slnk_unet_param_count(self._u))

    def _check(self, st):
        if st != 0:
            raise SlnkError(st, self._lib.slnk_unet_last_error(self._u).decode())

    def _ptr(self, t, shape):
        import torch
        if not t.is_cuda or t.dtype != torch.float32 or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"expected a contiguous float32 CUDA tensor of shape {tuple(shape)}, got "
                             f"{t.dtype} {tuple(t.shape)}")
        return ctypes.c_void_p(t.data_ptr())

    def close(self):
        if self._u:
            self._lib.slnk_unet_destroy(self._u)
            self._u = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        import numpy as np
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(self._lib.slnk_unet_get_params(self._u, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_params(self, w):
        import numpy as np
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.shape != (self.n_params,):
            raise ValueError(f"expected {self.n_params} parameters, got {w.shape}")
        self._check(self._lib.slnk_unet_set_params(self._u, w.ctypes.data_as(ctypes.c_void_p)))

    def get_grads(self):
        import numpy as np
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(self._lib.slnk_unet_get_grads(self._u, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    @staticmethod
    def conv_variant_counts(reset=True) -> dict:
        """Launches of each convolution kernel variant in this process since the last reset, keyed
        by (pixels per output tile, ways the channel reduction is split) for the direct kernel and
        ("lds", output channels per block) for the LDS-tiled one."""
        c = (ctypes.c_longlong * 8)()
        load_library().slnk_unet_conv_variants(c, 1 if reset else 0)
        out = {(16 * mw, ks): int(c[3 * (mw - 1) + j]) for mw in (1, 2) for j, ks in enumerate((1, 2, 4))}
        out[("lds", 32)], out[("lds", 64)] = int(c[6]), int(c[7])
        return out

    def forward(self, m_R, m_T, v, head=None):
        b, h, w = m_R.shape
        hp = self._ptr(head, (b,)) if head is not None else None
        self._check(self._lib.slnk_unet_forward(self._u, int(b), self._ptr(m_R, (b, h, w)), self._ptr(m_T, (b, h, w)),
                                                self._ptr(v, (b, 2, h, w)), hp))

    def train_step(self, m_R, m_T, v_target, lr, head_target=None):
        """One step; returns the velocity loss (or (loss, head_loss) with a head target)."""
        b, h, w = m_R.shape
        loss, hloss = ctypes.c_double(), ctypes.c_double()
        vp = self._ptr(v_target, (b, 2, h, w)) if v_target is not None else None
        hp = self._ptr(head_target, (b,)) if head_target is not None else None
        self._check(self._lib.slnk_unet_train_step(self._u, int(b), self._ptr(m_R, (b, h, w)),
                                                   self._ptr(m_T, (b, h, w)), vp, hp, float(lr), ctypes.byref(loss),
                                                   ctypes.byref(hloss)))
        return loss.value if head_target is None else (loss.value, hloss.value)

    def save(self, path):
        """Parameters as a raw little-endian float32 file with a small text header."""
        import numpy as np
        w = self.get_params()
        p = self.params
        with open(path, "wb") as f:
            hdr = f"SLNKUNET1 {p.height} {p.width} {p.levels} {p.base_channels} {self.n_params}\n".encode()
            f.write(hdr)
            f.write(w.astype("<f4").tobytes())

    def load(self, path):
        """Parameters from save(); a file holding only the convolution layers (no head) leaves the
        head's current values in place."""
        import numpy as np
        with open(path, "rb") as f:
            hdr = f.readline().decode().split()
            p = self.params
            want = ["SLNKUNET1", str(p.height), str(p.width), str(p.levels), str(p.base_channels)]
            if hdr[:5] != want or len(hdr) != 6 or int(hdr[5]) > self.n_params:
                raise ValueError(f"{path}: header {hdr} does not match this network {want + [str(self.n_params)]}")
            w = np.frombuffer(f.read(), dtype="<f4")
        if w.size != int(hdr[5]):
            raise ValueError(f"{path}: {w.size} values, header says {hdr[5]}")
        full = self.get_params()
        full[: w.size] = w
        self.set_params(full)
