"""Python binding of libsgbt (stochastic Galerkin solves with block-triangular preconditioning).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libsgbt.so`` (see ``include/sgbt.h`` for the C ABI).  PyTorch
provides device memory (tensors) and the stream.  The binding fails loudly
when the library is missing; there is no fallback path.

Block vectors are (N, P) tensors, node-major: row i is interior node i
(x fastest), column a is chaos mode a in graded order.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# SGBT_LIBRARY selects another build of the same library (the LDS-poison debug build)
LIB_PATH = os.environ.get("SGBT_LIBRARY") or os.path.join(_HERE, "libsgbt.so")

SG_OK, SG_WNOTCOERCIVE = 0, 1
SG_EINVAL, SG_ENOMEM, SG_EHIP, SG_ENOTCONV, SG_ENAN, SG_EBREAKDOWN = -1, -2, -3, -4, -5, -6
SG_F64, SG_F32, SG_MIXED = 0, 1, 2
SG_COLOUR_FOUR, SG_COLOUR_RB, SG_COLOUR_LEX = 0, 1, 2
SG_DISC_Q1, SG_DISC_P1 = 0, 1
DISCRETIZATIONS = {"q1": SG_DISC_Q1, "p1": SG_DISC_P1}

EXPORTED = ["sg_setup", "sg_query", "sg_get_cell_coeffs", "sg_rhs", "sg_apply", "sg_residual", "sg_vcycle",
            "sg_precond_diag", "sg_precond_tri", "sg_precond_sym", "sg_precond_split", "sg_solve", "sg_qoi", "sg_qoi_noalloc", "sg_qoi_grad",
            "sg_setup_host", "sg_sync",
            "sg_destroy", "sg_last_error"]


class Options(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int), ("m", ctypes.c_int), ("p", ctypes.c_int),
                ("sigma", ctypes.c_double), ("corr_len", ctypes.c_double), ("colour_mode", ctypes.c_int),
                ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("coarsest_cells", ctypes.c_int),
                ("discretization", ctypes.c_int)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("precond", ctypes.c_int), ("prec", ctypes.c_int),
                ("restart", ctypes.c_int), ("max_it", ctypes.c_int), ("rtol", ctypes.c_double),
                ("use_x0", ctypes.c_int), ("timing", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("status", ctypes.c_int),
                ("n_hist", ctypes.c_int), ("rel_res_true", ctypes.c_double),
                ("rel_res_hist", ctypes.c_double * 1024), ("t_total_ms", ctypes.c_double),
                ("t_apply_ms", ctypes.c_double), ("t_prec_ms", ctypes.c_double), ("t_orth_ms", ctypes.c_double),
                ("n_apply", ctypes.c_int), ("n_prec", ctypes.c_int)]

    def as_dict(self):
        return dict(iters=self.iters, restarts=self.restarts, status=self.status,
                    rel_res_true=self.rel_res_true, hist=list(self.rel_res_hist[:self.n_hist]),
                    t_total_ms=self.t_total_ms, t_apply_ms=self.t_apply_ms, t_prec_ms=self.t_prec_ms,
                    t_orth_ms=self.t_orth_ms, n_apply=self.n_apply, n_prec=self.n_prec)


_lib = None


def load_library():
    """Load libsgbt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python paper_1304_1755_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    sig = {
        "sg_setup": (ctypes.c_int, [ctypes.POINTER(Options), dp, dp, vp, ctypes.POINTER(vp)]),
        "sg_query": (ctypes.c_int, [vp, ip, ip, ip, ip, dp, dp]),
        "sg_get_cell_coeffs": (ctypes.c_int, [vp, dp]),
        "sg_rhs": (ctypes.c_int, [vp, vp]),
        "sg_apply": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "sg_residual": (ctypes.c_int, [vp, vp, vp, vp]),
        "sg_vcycle": (ctypes.c_int, [vp, vp, ctypes.c_int, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "sg_precond_diag": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "sg_precond_tri": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "sg_precond_sym": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "sg_precond_split": (ctypes.c_int, [vp, vp, vp, ctypes.c_int]),
        "sg_solve": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]),
        "sg_qoi": (ctypes.c_int, [vp, vp, dp, dp]),
        "sg_qoi_noalloc": (ctypes.c_int, [vp, vp, vp, vp]),
        "sg_qoi_grad": (ctypes.c_int, [vp, vp, ctypes.POINTER(SolveOpts), dp, dp, dp, dp,
                                       ctypes.POINTER(SolveInfo)]),
        "sg_setup_host": (ctypes.c_int, [ctypes.POINTER(Options), dp, dp, dp, dp, dp, dp, dp, dp]),
        "sg_sync": (ctypes.c_int, [vp]),
        "sg_destroy": (None, [vp]),
        "sg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsgbt error {code}: {msg}")
        self.code = code


def _check(code, allow=(SG_OK,)):
    if code not in allow:
        raise SGError(code, load_library().sg_last_error().decode())
    return code


def _dptr(arr):
    import numpy as np
    a = np.ascontiguousarray(arr, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def solve_options(solver="fgmres", precond="tri", prec=SG_F64, restart=30, max_it=500, rtol=1e-8,
                  use_x0=False, timing=False):
    return SolveOpts(solver={"fgmres": 0, "pcg": 1, "gpcg": 2, "bgs": 3, "gmres_left": 4}[solver],
                     precond={"diag": 0, "tri": 1, "sym": 2, "tri2x2": 3, "sym2x2": 4}[precond], prec=prec,
                     restart=restart, max_it=max_it, rtol=rtol, use_x0=int(use_x0), timing=int(timing))


def setup_host(n, m, p, sigma, corr_len=0.5, a0_nodal=None, kl_amp=None, coarsest=8, disc="q1"):
    """Run the library's host-side setup only (no device) and return its tables.

    disc "q1": bilinear elements, f = 1; "p1": the triangulation, load and
    variance-one law of Sec. 6 (cell rows then hold the 2 n^2 triangles).
    """
    import numpy as np
    lib = load_library()
    opt = Options(n_cells=n, m=m, p=p, sigma=sigma, corr_len=corr_len, colour_mode=0, nu1=2, nu2=2,
                  coarsest_cells=coarsest, discretization=DISCRETIZATIONS[disc])
    nel = n * n * (2 if disc == "p1" else 1)
    a0k, a0p = _dptr(a0_nodal) if a0_nodal is not None else (None, None)
    ak, ap = _dptr(kl_amp) if kl_amp is not None else (None, None)
    N, N1, Nc = (n - 1) ** 2, (n // 2 - 1) ** 2, (coarsest - 1) ** 2
    out = dict(cell=np.empty((m + 1) * nel), fine=np.empty(N * 9), l1=np.full(max(N1, 1) * 9, np.nan),
               cinv=np.empty(Nc * Nc), lam=np.empty(max(m, 1)), amin=np.empty(1))
    P = ctypes.POINTER(ctypes.c_double)
    code = lib.sg_setup_host(ctypes.byref(opt), a0p, ap, *[out[k].ctypes.data_as(P) for k in
                                                           ("cell", "fine", "l1", "cinv", "lam", "amin")])
    _check(code, allow=(SG_OK, SG_WNOTCOERCIVE))
    return dict(cell=out["cell"].reshape(m + 1, nel), fine=out["fine"].reshape(N, 9),
                l1=out["l1"][:N1 * 9].reshape(N1, 9), cinv=out["cinv"].reshape(Nc, Nc), lam=out["lam"][:m],
                a_min_h=float(out["amin"][0]), code=code)


class Problem:
    """One stochastic Galerkin system A = sum_k G_k (x) K_k on the current HIP device.

    disc "q1": bilinear elements on the unit square with f = 1; "p1": the
    setting of Sec. 6 (linear elements, f = 2 (1/2 - x^2 - y^2), unit-variance
    uniform xi_k; pass corr_len=1.0 for the paper's L).
    """

    def __init__(self, n, m, p, sigma, corr_len=0.5, a0_nodal=None, kl_amp=None, colour="four", nu1=2, nu2=2,
                 coarsest=8, stream=None, disc="q1"):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("libsgbt needs a HIP device")
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opt = Options(n_cells=n, m=m, p=p, sigma=sigma, corr_len=corr_len,
                      colour_mode={"four": SG_COLOUR_FOUR, "rb": SG_COLOUR_RB, "lex": SG_COLOUR_LEX}[colour], nu1=nu1, nu2=nu2,
                      coarsest_cells=coarsest, discretization=DISCRETIZATIONS[disc])
        a0p = amp = None
        a0_keep = amp_keep = None
        if a0_nodal is not None:
            a0_keep, a0p = _dptr(a0_nodal)
            assert a0_keep.size == (n + 1) ** 2
        if kl_amp is not None:
            amp_keep, amp = _dptr(kl_amp)
            assert amp_keep.size == m
        ctx = ctypes.c_void_p()
        self.warning = _check(lib.sg_setup(ctypes.byref(opt), a0p, amp, ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(ctx)), allow=(SG_OK, SG_WNOTCOERCIVE))
        self._ctx = ctx
        self.n, self.m, self.p, self.sigma, self.disc = n, m, p, sigma, disc
        Nv, Pv = ctypes.c_int(), ctypes.c_int()
        offs = (ctypes.c_int * (p + 2))()
        mi = (ctypes.c_int * max(1, 256 * max(m, 1)))()
        lam = (ctypes.c_double * max(1, m))()
        amin = ctypes.c_double()
        _check(lib.sg_query(ctx, ctypes.byref(Nv), ctypes.byref(Pv), offs, mi, lam, ctypes.byref(amin)))
        self.N, self.P = Nv.value, Pv.value
        self.offsets = list(offs)
        self.multi_index = [tuple(mi[a * m:(a + 1) * m]) for a in range(self.P)]
        self.kl_lambda = list(lam[:m])
        self.a_min_h = amin.value

    # -- helpers
    def _t(self, x, dtype, shape=None):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == dtype and x.is_contiguous()):
            raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
        if shape is not None and tuple(x.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(x.shape)}")
        return ctypes.c_void_p(x.data_ptr())

    def empty(self, dtype=torch.float64, width=None):
        return torch.empty((self.N, self.P if width is None else width), dtype=dtype, device=self.device)

    def cell_coeffs(self):
        import numpy as np
        nel = self.n * self.n * (2 if self.disc == "p1" else 1)
        out = np.empty((self.m + 1) * nel)
        _check(load_library().sg_get_cell_coeffs(self._ctx, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out.reshape(self.m + 1, nel)

    # -- hot path
    def rhs(self, F=None):
        F = self.empty() if F is None else F
        _check(load_library().sg_rhs(self._ctx, self._t(F, torch.float64, (self.N, self.P))))
        return F

    def apply(self, U, Y=None, prec=SG_F64):
        din = torch.float32 if prec == SG_MIXED else torch.float64
        Y = self.empty() if Y is None else Y
        _check(load_library().sg_apply(self._ctx, self._t(U, din, (self.N, self.P)),
                                       self._t(Y, torch.float64, (self.N, self.P)), prec))
        return Y

    def residual(self, F, U, R=None):
        R = self.empty() if R is None else R
        shp = (self.N, self.P)
        _check(load_library().sg_residual(self._ctx, self._t(F, torch.float64, shp), self._t(U, torch.float64, shp),
                                          self._t(R, torch.float64, shp)))
        return R

    def vcycle(self, f, u=None, prec=SG_F64):
        dt = torch.float32 if prec == SG_F32 else torch.float64
        if f.dim() != 2 or f.shape[0] != self.N:
            raise ValueError("f must be (N, width)")
        u = torch.empty_like(f) if u is None else u
        _check(load_library().sg_vcycle(self._ctx, self._t(f, dt), f.shape[1], self._t(u, dt, f.shape),
                                        u.shape[1], f.shape[1], prec))
        return u

    def precond(self, R, Z=None, kind="tri", prec=SG_F64):
        dz = torch.float32 if prec == SG_MIXED else torch.float64
        Z = self.empty(dz) if Z is None else Z
        lib = load_library()
        shp = (self.N, self.P)
        if kind in ("tri2x2", "sym2x2"):
            if prec != SG_F64:
                raise ValueError("the 2x2 split preconditioners run in double only")
            _check(lib.sg_precond_split(self._ctx, self._t(R, torch.float64, shp), self._t(Z, dz, shp),
                                        int(kind == "sym2x2")))
            return Z
        fn = {"tri": lib.sg_precond_tri, "diag": lib.sg_precond_diag, "sym": lib.sg_precond_sym}[kind]
        _check(fn(self._ctx, self._t(R, torch.float64, shp), self._t(Z, dz, shp), prec))
        return Z

    def solve(self, F=None, U=None, **kw):
        F = self.rhs() if F is None else F
        U = self.empty() if U is None else U
        o = solve_options(**kw)
        info = SolveInfo()
        shp = (self.N, self.P)
        code = load_library().sg_solve(self._ctx, self._t(F, torch.float64, shp), self._t(U, torch.float64, shp),
                                       ctypes.byref(o), ctypes.byref(info))
        _check(code, allow=(SG_OK, SG_ENOTCONV))
        return U, info.as_dict()

    def qoi(self, U):
        import numpy as np
        q = np.empty(self.P)
        J = ctypes.c_double()
        _check(load_library().sg_qoi(self._ctx, self._t(U, torch.float64, (self.N, self.P)),
                                     q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(J)))
        return J.value, q

    def qoi_noalloc(self, U, q, J):
        """sg_qoi_noalloc: q (P) and J (1) are float64 device tensors the caller owns."""
        _check(load_library().sg_qoi_noalloc(self._ctx, self._t(U, torch.float64, (self.N, self.P)),
                                             self._t(q, torch.float64, (self.P,)), self._t(J, torch.float64, (1,))))
        return q, J

    def qoi_grad(self, U, **kw):
        import numpy as np
        o = solve_options(**kw)
        J, ds = ctypes.c_double(), ctypes.c_double()
        damp = np.zeros(max(1, self.m))
        da0 = np.zeros(self.N)
        info = SolveInfo()
        dp = ctypes.POINTER(ctypes.c_double)
        _check(load_library().sg_qoi_grad(self._ctx, self._t(U, torch.float64, (self.N, self.P)), ctypes.byref(o),
                                          ctypes.byref(J), ctypes.byref(ds), damp.ctypes.data_as(dp),
                                          da0.ctypes.data_as(dp), ctypes.byref(info)), allow=(SG_OK, SG_ENOTCONV))
        return dict(J=J.value, dsigma=ds.value, damp=damp[:self.m].copy(), da0=da0, adj_info=info.as_dict())

    def sync(self):
        _check(load_library().sg_sync(self._ctx))

    def close(self):
        if getattr(self, "_ctx", None):
            load_library().sg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SGQoI(torch.autograd.Function):
    """J(sigma, s, a0) = E[Q] + Var[Q] of the subdomain mean Q of the SG solution.

    forward builds the system for the given parameters and solves it;
    backward returns the adjoint gradient computed by the library
    (sg_qoi_grad).  Inputs are CPU float64 tensors: sigma (scalar), s (m
    amplitudes) and a0_interior ((n-1)^2 values of the nodal mean field at the
    interior vertices, x fastest).  The boundary vertices of a0 are data, not
    parameters: cfg["a0_boundary"] (an (n+1)^2 array whose interior entries
    are ignored) or 1 when absent.  Every input that enters J receives its
    exact gradient.
    """

    @staticmethod
    def forward(ctx, sigma, amps, a0_interior, cfg):
        import numpy as np
        n = cfg["n"]
        if a0_interior.numel() != (n - 1) ** 2:
            raise ValueError(f"a0_interior must hold (n-1)^2 = {(n - 1) ** 2} values")
        full = np.ones((n + 1, n + 1))
        if cfg.get("a0_boundary") is not None:
            full[:] = np.asarray(cfg["a0_boundary"], dtype=np.float64).reshape(n + 1, n + 1)
        full[1:n, 1:n] = a0_interior.detach().cpu().numpy().reshape(n - 1, n - 1)
        prob = Problem(n, cfg["m"], cfg["p"], float(sigma), corr_len=cfg.get("corr_len", 0.5),
                       a0_nodal=full.ravel(), kl_amp=amps.detach().cpu().numpy(),
                       coarsest=cfg.get("coarsest", 8))
        solve_kw = cfg.get("solve", {})
        U, _info = prob.solve(**solve_kw)
        J, _q = prob.qoi(U)
        ctx.prob, ctx.U, ctx.solve_kw = prob, U, solve_kw
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gout):
        g = ctx.prob.qoi_grad(ctx.U, **ctx.solve_kw)
        ctx.prob.close()
        ctx.prob = ctx.U = None
        return (gout * torch.tensor(g["dsigma"], dtype=torch.float64),
                gout * torch.from_numpy(g["damp"]), gout * torch.from_numpy(g["da0"]), None)
