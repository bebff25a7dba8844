"""Python binding of the sfdp C ABI (include/sfdp.h): argument marshalling only.

Every computation runs in the native library ``libsfdp.so`` (HIP kernels for
gfx950).  Arrays are torch tensors on the GPU; complex vectors are
``torch.complex128`` (interleaved re/im in memory, as the ABI expects).  There
is no fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfdp.so")

SFDP_FP64, SFDP_MIXED, SFDP_MIXED_IFACE = 0, 1, 2
STATUS = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_NOCONV", -4: "E_DEVICE", -5: "E_STATE"}
Q_SINV, Q_SBB, Q_PHI, Q_COARSE, Q_COARSE_INV = 0, 1, 2, 3, 4

EXPORTS = [
    "sfdp_ctx_create", "sfdp_ctx_destroy", "sfdp_last_error", "sfdp_abi_version", "sfdp_problem_create",
    "sfdp_problem_sizes", "sfdp_problem_destroy", "sfdp_set_beta", "sfdp_solve_range_space",
    "sfdp_apply_schur_inv", "sfdp_feti_solve", "sfdp_apply_operator", "sfdp_kkt_residual",
    "sfdp_inspect", "sfdp_interface_apply", "sfdp_timing_enable", "sfdp_kernel_times",
    "sfdp_batch_create", "sfdp_batch_destroy", "sfdp_batch_sizes", "sfdp_batch_set_beta",
    "sfdp_batch_solve_range_space", "sfdp_server_create", "sfdp_server_submit", "sfdp_server_poll",
    "sfdp_server_stats", "sfdp_server_destroy", "sfdp_set_coarse_space", "sfdp_batch_inspect",
    "sfdp_solve_full_space", "sfdp_set_tuning", "sfdp_kkt_residual_noalloc", "sfdp_set_graphs",
    "sfdp_set_setup_arithmetic", "sfdp_elastic_create", "sfdp_elastic_pressure_load", "sfdp_elastic_forward",
    "sfdp_set_gmres_launch",
]


class SfdpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sfdp {STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("tol_kkt", ctypes.c_double), ("tol_inner", ctypes.c_double),
                ("max_outer", ctypes.c_int), ("max_krylov", ctypes.c_int), ("factors", ctypes.c_int),
                ("batch", ctypes.c_int), ("schur_block", ctypes.c_int), ("tol_inner_first", ctypes.c_double),
                ("host_ptrs", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("rel_kkt", ctypes.c_double), ("rel_kkt_first", ctypes.c_double),
                ("imag_ratio", ctypes.c_double), ("outer_steps", ctypes.c_int),
                ("krylov_total", ctypes.c_int), ("krylov_its", ctypes.c_int * 16),
                ("n_feti", ctypes.c_int), ("minres_its", ctypes.c_int),
                ("constr_viol", ctypes.c_double), ("eta_blk", ctypes.c_double),
                ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {"rel_kkt": self.rel_kkt, "rel_kkt_first": self.rel_kkt_first,
                "constr_viol": self.constr_viol, "eta_blk": self.eta_blk,
                "t_setup_ms": self.t_setup_ms, "t_solve_ms": self.t_solve_ms,
                "imag_ratio": self.imag_ratio, "outer_steps": self.outer_steps,
                "krylov_total": self.krylov_total, "n_feti": self.n_feti,
                "krylov_its": list(self.krylov_its)[: min(self.n_feti, 16)],
                "minres_its": self.minres_its}


class Request(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_elem", ctypes.c_int), ("sub_elem", ctypes.c_int),
                ("beta", ctypes.c_double), ("nrhs", ctypes.c_int), ("ybar", ctypes.c_void_p),
                ("yc", ctypes.c_void_p), ("y", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("lam", ctypes.c_void_p), ("mode", ctypes.c_int)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("setups", ctypes.c_int64), ("evictions", ctypes.c_int64), ("ticks", ctypes.c_int64),
                ("resident", ctypes.c_int64), ("device_bytes", ctypes.c_int64), ("mean_ms", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("solo_in_flight_max", ctypes.c_int64)]


class Timing(ctypes.Structure):
    _fields_ = [("gmres_ms", ctypes.c_double), ("local_ms", ctypes.c_double),
                ("gmres_launches", ctypes.c_int64), ("gmres_iters", ctypes.c_int64),
                ("local_launches", ctypes.c_int64), ("gmres_rhs_iters", ctypes.c_int64),
                ("gmres_width", ctypes.c_int), ("gmres_resident", ctypes.c_int)]


class Sizes(ctypes.Structure):
    _fields_ = [("n_free", ctypes.c_int64), ("n_bdry", ctypes.c_int64), ("n_sub", ctypes.c_int64),
                ("n_mult", ctypes.c_int64), ("n_corner", ctypes.c_int64),
                ("max_delta", ctypes.c_int64), ("resident_bytes", ctypes.c_int64),
                ("n_coarse", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsfdp.so and declare the ABI; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is not built; run python -m paper_1312_5653_amd.build")
    lib = ctypes.CDLL(path)
    P, I, D, VP = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    lib.sfdp_ctx_create.argtypes = [I, ctypes.c_size_t, VP, ctypes.POINTER(P)]
    lib.sfdp_ctx_destroy.argtypes = [P]
    lib.sfdp_ctx_destroy.restype = ctypes.c_int
    lib.sfdp_last_error.restype = ctypes.c_char_p
    lib.sfdp_abi_version.restype = ctypes.c_int
    lib.sfdp_abi_version.argtypes = []
    lib.sfdp_problem_create.argtypes = [P, I, I, I, I, ctypes.POINTER(P)]
    lib.sfdp_problem_sizes.argtypes = [P, ctypes.POINTER(Sizes)]
    lib.sfdp_set_coarse_space.argtypes = [P, I]
    lib.sfdp_problem_destroy.argtypes = [P]
    lib.sfdp_problem_destroy.restype = None
    lib.sfdp_set_beta.argtypes = [P, D]
    lib.sfdp_solve_range_space.argtypes = [P, I, VP, VP, VP, VP, VP, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    lib.sfdp_set_tuning.argtypes = [I]
    lib.sfdp_set_graphs.argtypes = [I]
    lib.sfdp_set_gmres_launch.argtypes = [I]
    lib.sfdp_set_setup_arithmetic.argtypes = [I]
    lib.sfdp_solve_full_space.argtypes = [P, I, VP, VP, VP, VP, VP, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    lib.sfdp_apply_schur_inv.argtypes = [P, I, VP, VP, ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    lib.sfdp_feti_solve.argtypes = [P, I, I, VP, VP, ctypes.POINTER(Opts), ctypes.POINTER(I)]
    lib.sfdp_apply_operator.argtypes = [P, ctypes.c_char, I, VP, VP, VP]
    lib.sfdp_kkt_residual.argtypes = [P, I, VP, VP, VP, VP, VP, ctypes.POINTER(D)]
    lib.sfdp_kkt_residual_noalloc.argtypes = [P, I, VP, VP, VP, VP, VP, VP]
    lib.sfdp_inspect.argtypes = [P, I, I, VP, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.sfdp_interface_apply.argtypes = [P, ctypes.c_char, VP, VP]
    lib.sfdp_timing_enable.argtypes = [P, I]
    lib.sfdp_kernel_times.argtypes = [P, ctypes.POINTER(Timing)]
    lib.sfdp_batch_create.argtypes = [P, I, ctypes.POINTER(I), I, I, ctypes.POINTER(P)]
    lib.sfdp_batch_destroy.argtypes = [P]
    lib.sfdp_batch_destroy.restype = None
    lib.sfdp_batch_sizes.argtypes = [P, I, ctypes.POINTER(Sizes)]
    lib.sfdp_batch_inspect.argtypes = [P, I, I, I, VP, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.sfdp_batch_set_beta.argtypes = [P, ctypes.POINTER(D)]
    VPP = ctypes.POINTER(ctypes.c_void_p)
    lib.sfdp_batch_solve_range_space.argtypes = [P, ctypes.POINTER(I), VPP, VPP, VPP, VPP, VPP,
                                                 ctypes.POINTER(Opts), ctypes.POINTER(Info)]
    lib.sfdp_elastic_create.argtypes = [P, I, I, I, D, D, I, ctypes.POINTER(P)]
    lib.sfdp_elastic_pressure_load.argtypes = [P, D, VP]
    lib.sfdp_elastic_forward.argtypes = [P, I, VP, VP, ctypes.POINTER(Opts), ctypes.POINTER(I)]
    lib.sfdp_server_create.argtypes = [P, I, ctypes.POINTER(Opts), ctypes.POINTER(P)]
    lib.sfdp_server_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.sfdp_server_poll.argtypes = [P, ctypes.c_uint64, I, ctypes.POINTER(Info), ctypes.POINTER(D)]
    lib.sfdp_server_stats.argtypes = [P, ctypes.POINTER(ServerInfo)]
    lib.sfdp_server_destroy.argtypes = [P]
    lib.sfdp_server_destroy.restype = None
    for name in ("sfdp_ctx_create", "sfdp_problem_create", "sfdp_problem_sizes", "sfdp_set_beta",
                 "sfdp_solve_range_space", "sfdp_apply_schur_inv", "sfdp_feti_solve",
                 "sfdp_apply_operator", "sfdp_kkt_residual", "sfdp_kkt_residual_noalloc",
                 "sfdp_inspect", "sfdp_interface_apply",
                 "sfdp_timing_enable", "sfdp_kernel_times", "sfdp_batch_create", "sfdp_batch_sizes",
                 "sfdp_batch_set_beta", "sfdp_batch_solve_range_space", "sfdp_server_create",
                 "sfdp_server_submit", "sfdp_server_poll", "sfdp_server_stats", "sfdp_set_graphs", "sfdp_set_tuning",
                 "sfdp_set_setup_arithmetic", "sfdp_elastic_create", "sfdp_elastic_pressure_load",
                 "sfdp_elastic_forward", "sfdp_set_gmres_launch"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(st: int, allow_noconv: bool = False):
    if st == 0 or (allow_noconv and st == -3):
        return st
    raise SfdpError(st, _lib.sfdp_last_error().decode())


def _ptr(t, host=False):
    """Address of a contiguous CUDA tensor (host=True: of a CPU tensor, for the
    calls that stage host arrays)."""
    if t is None:
        return None
    if not t.is_contiguous() or t.is_cuda == host:
        raise ValueError("arrays must be contiguous " + ("CPU" if host else "CUDA") + " tensors")
    if host and _lib.sfdp_abi_version() < 2:
        raise RuntimeError("this libsfdp.so predates host-array staging; rebuild it")
    return ctypes.c_void_p(t.data_ptr())


def _opts(tol_kkt=0.0, tol_inner=0.0, max_outer=0, max_krylov=0, batch=0, factors=0, schur_block=0,
          tol_inner_first=0.0, host_ptrs=0):
    return Opts(tol_kkt, tol_inner, max_outer, max_krylov, factors, batch, schur_block, tol_inner_first,
                host_ptrs)


def _host(t):
    """1 when t is a host (CPU) tensor: the library stages it (sfdp_opts.host_ptrs)."""
    return 1 if t.device.type == "cpu" else 0


class Context:
    """One GPU; work is ordered on torch's current stream at creation time."""

    def __init__(self, device: int = 0, mem_budget: int = 0):
        import torch
        lib = load_library()
        torch.cuda.set_device(device)
        stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        _check(lib.sfdp_ctx_create(device, mem_budget, ctypes.c_void_p(stream), ctypes.byref(h)))
        self._h = h
        self.device = device

    def close(self):
        """Free the context; raises SfdpError (E_STATE) while problems, batches or
        servers made from it are still open (close those first)."""
        if self._h:
            _check(_lib.sfdp_ctx_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """A 2D unit-square Q1 instance split into (n_elem/sub_elem)^2 subdomains."""

    def __init__(self, ctx: Context, dim: int, n_elem: int, sub_elem: int, precision: int = SFDP_FP64):
        h = ctypes.c_void_p()
        _check(_lib.sfdp_problem_create(ctx._h, dim, n_elem, sub_elem, precision, ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.dim, self.n_elem, self.sub_elem, self.precision = dim, n_elem, sub_elem, precision
        s = Sizes()
        _check(_lib.sfdp_problem_sizes(h, ctypes.byref(s)))
        self.sizes = {f: getattr(s, f) for f, _ in Sizes._fields_}
        self.n_free = s.n_free
        self.n_bdry = s.n_bdry

    def close(self):
        if self._h:
            _lib.sfdp_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refresh_sizes(self):
        s = Sizes()
        _check(_lib.sfdp_problem_sizes(self._h, ctypes.byref(s)))
        self.sizes = {f: getattr(s, f) for f, _ in Sizes._fields_}
        return self.sizes

    def set_coarse_space(self, edge_averages: bool):
        """Edge-augmented (True, the default) or corner-only coarse space; takes
        effect at the next set_beta."""
        _check(_lib.sfdp_set_coarse_space(self._h, int(bool(edge_averages))))

    def set_beta(self, beta: float):
        _check(_lib.sfdp_set_beta(self._h, float(beta)))
        self.beta = beta

    def solve_range_space(self, ybar, yc=None, y=None, u=None, lam=None, **opts):
        import torch
        nrhs = 1 if ybar.dim() == 1 else ybar.shape[0]
        y = torch.empty_like(ybar) if y is None else y
        u = torch.empty_like(ybar) if u is None else u
        lam = torch.empty_like(ybar) if lam is None else lam
        infos = (Info * nrhs)()
        o = _opts(**{"host_ptrs": _host(ybar), **opts})
        h = bool(o.host_ptrs)
        st = _lib.sfdp_solve_range_space(self._h, nrhs, _ptr(ybar, h), _ptr(yc, h), _ptr(y, h), _ptr(u, h),
                                         _ptr(lam, h),
                                         ctypes.byref(o), infos)
        _check(st, allow_noconv=True)
        return y, u, lam, [i.as_dict() for i in infos], st

    def solve_full_space(self, ybar, yc=None, y=None, u=None, lam=None, **opts):
        """Full-space method: MINRES with the block-diagonal Schur preconditioner
        inside FP64 refinement (same arguments and results as solve_range_space);
        schur_block=1 uses the Pearson-Wathen approximation S_p for its S block."""
        import torch
        nrhs = 1 if ybar.dim() == 1 else ybar.shape[0]
        y = torch.empty_like(ybar) if y is None else y
        u = torch.empty_like(ybar) if u is None else u
        lam = torch.empty_like(ybar) if lam is None else lam
        infos = (Info * nrhs)()
        o = _opts(**{"host_ptrs": _host(ybar), **opts})
        h = bool(o.host_ptrs)
        st = _lib.sfdp_solve_full_space(self._h, nrhs, _ptr(ybar, h), _ptr(yc, h), _ptr(y, h), _ptr(u, h),
                                        _ptr(lam, h),
                                        ctypes.byref(o), infos)
        _check(st, allow_noconv=True)
        return y, u, lam, [i.as_dict() for i in infos], st

    def apply_schur_inv(self, r, z=None, **opts):
        """z = S^-1 r (schur_block=1: z = S_p^-1 r) for real r."""
        import torch
        nrhs = 1 if r.dim() == 1 else r.shape[0]
        z = torch.empty_like(r) if z is None else z
        infos = (Info * nrhs)()
        o = _opts(**{"host_ptrs": _host(r), **opts})
        h = bool(o.host_ptrs)
        _check(_lib.sfdp_apply_schur_inv(self._h, nrhs, _ptr(r, h), _ptr(z, h), ctypes.byref(o), infos))
        return z, [i.as_dict() for i in infos]

    def feti_solve(self, f, conj_z: bool = False, x=None, **opts):
        import torch
        nrhs = 1 if f.dim() == 1 else f.shape[0]
        x = torch.empty_like(f) if x is None else x
        its = (ctypes.c_int * nrhs)()
        o = _opts(**{"host_ptrs": _host(f), **opts})
        h = bool(o.host_ptrs)
        _check(_lib.sfdp_feti_solve(self._h, int(conj_z), nrhs, _ptr(f, h), _ptr(x, h), ctypes.byref(o), its))
        return x, list(its)[:nrhs]

    def apply_operator(self, which: str, x, xc=None, y=None):
        import torch
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        y = torch.empty_like(x) if y is None else y
        _check(_lib.sfdp_apply_operator(self._h, which.encode(), nrhs, _ptr(x), _ptr(xc), _ptr(y)))
        return y

    def kkt_residual(self, ybar, yc, y, u, lam):
        nrhs = 1 if ybar.dim() == 1 else ybar.shape[0]
        rel = (ctypes.c_double * nrhs)()
        _check(_lib.sfdp_kkt_residual(self._h, nrhs, _ptr(ybar), _ptr(yc), _ptr(y), _ptr(u), _ptr(lam), rel))
        return list(rel)

    def kkt_residual_noalloc(self, ybar, yc, y, u, lam, rel):
        """The allocation-free form: rel is a caller-owned float64 device tensor of
        nrhs entries, written in stream order (no wait)."""
        nrhs = 1 if ybar.dim() == 1 else ybar.shape[0]
        _check(_lib.sfdp_kkt_residual_noalloc(self._h, nrhs, _ptr(ybar), _ptr(yc), _ptr(y), _ptr(u), _ptr(lam),
                                              _ptr(rel)))
        return rel

    def inspect(self, what: int, sub: int = 0):
        import torch
        r, c = ctypes.c_int(), ctypes.c_int()
        _check(_lib.sfdp_inspect(self._h, what, sub, None, ctypes.byref(r), ctypes.byref(c)))
        out = torch.zeros((r.value, c.value), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        _check(_lib.sfdp_inspect(self._h, what, sub, _ptr(out), ctypes.byref(r), ctypes.byref(c)))
        return out

    def interface_apply(self, which: str, x):
        import torch
        n = self.sizes["n_mult"]
        y = torch.zeros(n, dtype=torch.complex128, device=x.device)
        _check(_lib.sfdp_interface_apply(self._h, which.encode(), _ptr(x), _ptr(y)))
        return y

    def timing_enable(self, enable=True):
        """True / 1: time the GMRES and subdomain-solve launches; 2: the GMRES launches only; 0 off."""
        _check(_lib.sfdp_timing_enable(self._h, int(enable)))

    def kernel_times(self):
        t = Timing()
        _check(_lib.sfdp_kernel_times(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in Timing._fields_}


class ElasticProblem(Problem):
    """The solid cantilever of Sec. 6.2: the box [0, length] x [0, 1]^2 of n
    cells per unit length, clamped at x = 0, trilinear elasticity elements
    (three dofs per node), (length n / sub_elem) x (n / sub_elem)^2 cubic
    subdomains.  young = poisson = 0 take the paper's rubber."""

    def __init__(self, ctx: Context, n: int, sub_elem: int, length: int = 3, young: float = 0.0,
                 poisson: float = 0.0, precision: int = SFDP_FP64):
        h = ctypes.c_void_p()
        _check(_lib.sfdp_elastic_create(ctx._h, n, sub_elem, length, float(young), float(poisson), precision,
                                        ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.dim, self.n_elem, self.sub_elem, self.precision = 3, n, sub_elem, precision
        self.length = length
        s = Sizes()
        _check(_lib.sfdp_problem_sizes(h, ctypes.byref(s)))
        self.sizes = {f: getattr(s, f) for f, _ in Sizes._fields_}
        self.n_free = s.n_free
        self.n_bdry = s.n_bdry

    def pressure_load(self, pressure: float):
        """Nodal forces of a uniform pressure on the bottom face (float64 tensor)."""
        import torch
        f = torch.zeros(self.n_free, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        _check(_lib.sfdp_elastic_pressure_load(self._h, float(pressure), _ptr(f)))
        return f

    def forward(self, f, u=None, **opts):
        """u = K^-1 f by FETI-DP on the stiffness alone; returns (u, GMRES iterations)."""
        import torch
        nrhs = 1 if f.dim() == 1 else f.shape[0]
        u = torch.empty_like(f) if u is None else u
        its = (ctypes.c_int * nrhs)()
        o = _opts(**{"host_ptrs": _host(f), **opts})
        h = bool(o.host_ptrs)
        _check(_lib.sfdp_elastic_forward(self._h, nrhs, _ptr(f, h), _ptr(u, h), ctypes.byref(o), its))
        return u, list(its)[:nrhs]


class Batch:
    """Independent 2D instances (n_elem[i] cells per side, one beta each) whose
    set-up and solves run over all instances in one launch per kernel."""

    def __init__(self, ctx: Context, n_elem, sub_elem: int, precision: int = SFDP_FP64):
        self.n_elem = [int(v) for v in n_elem]
        arr = (ctypes.c_int * len(self.n_elem))(*self.n_elem)
        h = ctypes.c_void_p()
        _check(_lib.sfdp_batch_create(ctx._h, len(self.n_elem), arr, sub_elem, precision, ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self.sizes = []
        for i in range(len(self.n_elem)):
            sz = Sizes()
            _check(_lib.sfdp_batch_sizes(h, i, ctypes.byref(sz)))
            self.sizes.append({f: getattr(sz, f) for f, _ in Sizes._fields_})

    def close(self):
        if self._h:
            _lib.sfdp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_beta(self, betas):
        arr = (ctypes.c_double * len(self.n_elem))(*[float(b) for b in betas])
        _check(_lib.sfdp_batch_set_beta(self._h, arr))

    def inspect(self, i: int, what: int, sub: int = 0):
        """Set-up operator of instance i (as Problem.inspect)."""
        import torch
        r, c = ctypes.c_int(), ctypes.c_int()
        _check(_lib.sfdp_batch_inspect(self._h, i, what, sub, None, ctypes.byref(r), ctypes.byref(c)))
        out = torch.zeros((r.value, c.value), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        _check(_lib.sfdp_batch_inspect(self._h, i, what, sub, _ptr(out), ctypes.byref(r), ctypes.byref(c)))
        return out

    def solve_range_space(self, ybars, ycs=None, **opts):
        """ybars[i]: (nrhs_i, n_free_i) or (n_free_i,) CUDA tensor, or None for
        no work; returns lists y, u, lam (like ybars), infos per instance, status."""
        import torch
        n = len(self.n_elem)
        nr = []
        outs = []
        ptr = lambda t: t.data_ptr() if t is not None else None
        P = lambda vals: (ctypes.c_void_p * n)(*vals)
        for i in range(n):
            yb = ybars[i]
            if yb is None:
                nr.append(0)
                outs.append((None, None, None))
                continue
            if not yb.is_cuda or not yb.is_contiguous():
                raise ValueError("arrays must be contiguous CUDA tensors")
            nr.append(1 if yb.dim() == 1 else yb.shape[0])
            outs.append(tuple(torch.empty_like(yb) for _ in range(3)))
        yc_p = P([ptr(ycs[i]) if ycs is not None and ycs[i] is not None else None for i in range(n)])
        infos = (Info * max(sum(nr), 1))()
        o = _opts(**opts)
        st = _lib.sfdp_batch_solve_range_space(
            self._h, (ctypes.c_int * n)(*nr), P([ptr(b) for b in ybars]), yc_p,
            P([ptr(t[0]) for t in outs]), P([ptr(t[1]) for t in outs]), P([ptr(t[2]) for t in outs]),
            ctypes.byref(o), infos)
        _check(st, allow_noconv=True)
        res, k = [], 0
        for i in range(n):
            res.append([infos[k + j].as_dict() for j in range(nr[i])])
            k += nr[i]
        return [t[0] for t in outs], [t[1] for t in outs], [t[2] for t in outs], res, st


class Server:
    """Continuous-batching request loop on one context (a worker thread owns the
    context's stream while the server lives)."""

    def __init__(self, ctx: Context, precision: int = SFDP_MIXED, **opts):
        h = ctypes.c_void_p()
        o = _opts(**opts)
        _check(_lib.sfdp_server_create(ctx._h, precision, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.ctx = ctx
        self._live = {}

    def submit(self, n_elem: int, sub_elem: int, beta: float, ybar, yc=None, dim: int = 2,
               full_space: bool = False):
        """ybar: (nrhs, n_free) or (n_free,) CUDA tensor whose values are ready
        (the caller synchronises after producing them); kept alive until polled.
        dim 3 or full_space (the full-space method) take the server's solo lane.
        Returns a ticket; the outputs are allocated here."""
        import torch
        if not ybar.is_cuda or not ybar.is_contiguous():
            raise ValueError("arrays must be contiguous CUDA tensors")
        nrhs = 1 if ybar.dim() == 1 else ybar.shape[0]
        y, u, lam = (torch.empty_like(ybar) for _ in range(3))
        req = Request(dim, n_elem, sub_elem, float(beta), nrhs, ybar.data_ptr(),
                      yc.data_ptr() if yc is not None else None, y.data_ptr(), u.data_ptr(), lam.data_ptr(),
                      int(full_space))
        t = ctypes.c_uint64()
        _check(_lib.sfdp_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)))
        self._live[t.value] = (ybar, yc, y, u, lam, nrhs)
        return t.value

    def poll(self, ticket: int, wait: bool = True):
        """None while pending (wait=False); else (y, u, lam, infos, latency_ms, status)."""
        ybar, yc, y, u, lam, nrhs = self._live[ticket]
        infos = (Info * nrhs)()
        lat = ctypes.c_double()
        st = _lib.sfdp_server_poll(self._h, ticket, int(wait), infos, ctypes.byref(lat))
        if st == -5 and not wait:
            return None
        del self._live[ticket]
        if st not in (0, -3):
            raise SfdpError(st, _lib.sfdp_last_error().decode())
        return y, u, lam, [i.as_dict() for i in infos], lat.value, st

    def stats(self):
        si = ServerInfo()
        _check(_lib.sfdp_server_stats(self._h, ctypes.byref(si)))
        return {f: getattr(si, f) for f, _ in ServerInfo._fields_}

    def close(self):
        if self._h:
            _lib.sfdp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_tuning(enable: bool):
    """Launch-variant autotuning on (default) or off; either forgets earlier choices."""
    load_library()
    _check(_lib.sfdp_set_tuning(int(bool(enable))))


def force_variant(c: int):
    """Run launch variant c of every kernel that has it (tests); set_tuning restores."""
    load_library()
    _check(_lib.sfdp_set_tuning(2 + int(c)))


def set_graphs(enable: bool):
    """Graph replay of the refinement steps of single 2D problems on or off (default)."""
    load_library()
    _check(_lib.sfdp_set_graphs(int(bool(enable))))


def set_gmres_launch(mode: int):
    """GMRES launch form of single-problem range-space solves: 1 (default) plain
    launch with a co-residency check and cooperative fallback, 0 cooperative
    always, 2 the plain launch with no wait in its check (forces the fallback)."""
    load_library()
    _check(_lib.sfdp_set_gmres_launch(int(mode)))


def set_setup_arithmetic(bits: int):
    """64 (default) or 32: arithmetic of the set-up's line factorization and line
    solves for complex64-storage problems, from the next set-up on."""
    load_library()
    _check(_lib.sfdp_set_setup_arithmetic(int(bits)))
