"""Thin Python binding of libsignkrylov over torch device tensors.

Only argument marshalling lives here: torch provides device memory
(tensors, the workspace) and the current stream; every step of the
computation runs in the library's HIP kernels.  Field layout is the
library's: complex tensors of shape (12, V) (component-major, site fastest)
and links of shape (4, 3, 3, V).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L

__all__ = ["WilsonOperator", "SignResult", "kl_poles", "wilson_apply", "arnoldi_cycle",
           "multishift_fom_restart", "deflate_project", "sign_apply", "BatchedSignSolver", "SkError",
           "direct_sign_apply", "OverlapOperator"]

SkError = L.SkError


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _need(t, dtype, numel=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _cplx_host(arr):
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.complex128))
    buf = (C.c_double * (2 * a.size))(*a.view(np.float64))
    return buf, a.size


class WilsonOperator:
    """H_W = gamma5 D_W(mu) on a lattice with device-resident links.

    links: complex128 CUDA tensor (4, 3, 3, V); links64 (optional) the
    complex64 copy used by complex-float calls."""

    def __init__(self, links, dims, kappa, mu, antiperiodic_t=True, links64=None):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.n = 12 * self.V
        _need(links, torch.complex128, 36 * self.V, "links")
        if links64 is not None:
            _need(links64, torch.complex64, 36 * self.V, "links64")
        self.links = links
        self.links64 = links64
        self.kappa = float(kappa)
        self.mu = float(mu)
        self.antiperiodic_t = bool(antiperiodic_t)
        self.device = links.device

    def struct(self, mu=None):
        s = L.SkOperator()
        for i in range(4):
            s.dims[i] = self.dims[i]
        s.t_antiperiodic = 1 if self.antiperiodic_t else 0
        s.kappa = self.kappa
        s.mu = self.mu if mu is None else float(mu)
        s.links = self.links.data_ptr()
        s.links_c64 = self.links64.data_ptr() if self.links64 is not None else None
        return s

    def with_mu(self, mu):
        return WilsonOperator(self.links, self.dims, self.kappa, mu, self.antiperiodic_t, self.links64)

    def ensure_c64(self):
        """Create the complex-float copy of the links (library kernel)."""
        if self.links64 is None:
            lib = L.load()
            self.links64 = torch.empty(36 * self.V, dtype=torch.complex64, device=self.device)
            L.check(lib.sk_links_to_c64(_ptr(self.links), _ptr(self.links64), self.V, _stream()))
        return self


def kl_poles(s, c):
    """First-order poles/weights of the Kenney-Laub g_s(c x) (library routine)."""
    lib = L.load()
    sg = (C.c_double * (4 * s))()
    om = (C.c_double * (4 * s))()
    L.check(lib.kl_poles(int(s), float(c), sg, om))
    a = np.frombuffer(sg, dtype=np.float64).copy().view(np.complex128)
    b = np.frombuffer(om, dtype=np.float64).copy().view(np.complex128)
    return a, b


def wilson_apply(op: WilsonOperator, v, adjoint=False, out=None):
    lib = L.load()
    dt = L.SK_C128 if v.dtype == torch.complex128 else L.SK_C64
    _need(v, v.dtype, op.n, "v")
    if out is None:
        out = torch.empty_like(v)
    s = op.struct()
    L.check(lib.wilson_apply(C.byref(s), dt, _ptr(v), _ptr(out), 1 if adjoint else 0, _stream()))
    return out


def arnoldi_cycle(op: WilsonOperator, v0, k):
    """Returns (V (k+1, n), H (k+1, k) complex128, k_done)."""
    lib = L.load()
    dt = L.SK_C128 if v0.dtype == torch.complex128 else L.SK_C64
    _need(v0, v0.dtype, op.n, "v0")
    V = torch.empty((k + 1, op.n), dtype=v0.dtype, device=v0.device)
    V[0].copy_(v0.reshape(-1))
    H = torch.empty((k, k + 1), dtype=torch.complex128, device=v0.device)  # column-major (k+1) x k
    s = op.struct()
    ws = _workspace(lib.arnoldi_cycle_workspace_bytes(C.byref(s), k), v0.device)
    kd = C.c_int(0)
    L.check(lib.arnoldi_cycle(C.byref(s), dt, _ptr(V), _ptr(H), k, C.byref(kd), _ptr(ws),
                              ws.numel(), _stream()))
    return V, H.transpose(0, 1), kd.value


def multishift_fom_restart(H, k, sigma, omega, beta, rho, V, x, X_shift=None):
    """One multishift FOM update (in place on rho, x, X_shift); returns ||u||."""
    lib = L.load()
    sg, N = _cplx_host(sigma)
    om, _ = _cplx_host(omega)
    dt = L.SK_C128 if V.dtype == torch.complex128 else L.SK_C64
    n = x.numel()
    Hc = H.transpose(0, 1).contiguous()   # column-major storage
    ws = _workspace(lib.multishift_fom_restart_workspace_bytes(k, N), x.device)
    upd = C.c_double(0.0)
    L.check(lib.multishift_fom_restart(k, n, dt, _ptr(Hc), N, sg, om, _ptr(beta), _ptr(rho),
                                       _ptr(V), _ptr(x), _ptr(X_shift), C.byref(upd), _ptr(ws),
                                       ws.numel(), _stream()))
    return upd.value


def deflate_project(R, Lv, v, F=None):
    """Returns (r = (I - R L^H) v, coeff = L^H v, x_P = R F coeff or None)."""
    lib = L.load()
    m, n = R.shape
    r = torch.empty_like(v)
    coeff = torch.empty(m, dtype=torch.complex128, device=v.device)
    xp = torch.empty_like(v) if F is not None else None
    Fc = F.transpose(0, 1).contiguous() if F is not None else None
    ws = _workspace(lib.deflate_project_workspace_bytes(m, n), v.device)
    L.check(lib.deflate_project(m, n, _ptr(R), _ptr(Lv), _ptr(Fc), _ptr(v), _ptr(r), _ptr(xp),
                                _ptr(coeff), _ptr(ws), ws.numel(), _stream()))
    return r, coeff, xp


def deflation_eigensolve(op: WilsonOperator, m, nev_extra=16, ncv=0, key="abs", tol=1e-11,
                         max_restarts=2000, keep=0):
    """The m eigenpairs of H_W nearest zero as an oblique projector:
    returns (R (m, n), L (m, n), F (m, m) = sign(T_m), lambda (numpy), stats)."""
    lib = L.load()
    p = L.SkEigParams()
    p.m, p.nev_extra, p.ncv = int(m), int(nev_extra), int(ncv)
    p.key = 0 if key == "abs" else 1
    p.tol, p.max_restarts, p.keep = float(tol), int(max_restarts), int(keep)
    s = op.struct()
    nb = lib.deflation_eigensolve_workspace_bytes(C.byref(s), C.byref(p))
    if nb == 0:
        raise SkError(L.SK_ERR_ARG, "invalid eigensolver parameters")
    ws = _workspace(nb, op.device)
    R = torch.empty((m, op.n), dtype=torch.complex128, device=op.device)
    Lv = torch.empty_like(R)
    Fc = torch.empty((m, m), dtype=torch.complex128, device=op.device)   # column-major
    lam = (C.c_double * (2 * m))()
    st = L.SkEigStats()
    L.check(lib.deflation_eigensolve(C.byref(s), C.byref(p), _ptr(R), _ptr(Lv), _ptr(Fc), lam,
                                     C.byref(st), _ptr(ws), ws.numel(), _stream()))
    lamv = np.frombuffer(lam, dtype=np.float64).copy().view(np.complex128)
    stats = {"restarts": tuple(st.restarts), "matvecs": st.matvecs, "resid": tuple(st.resid),
             "gap": st.gap, "key_window": st.key_window}
    return R, Lv, Fc.transpose(0, 1).contiguous(), lamv, stats


def _host_cplx(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    return a, a.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))


def dense_schur(A, key="re", count=None):
    """Library's host Schur form: A = Q T Q^H with `count` eigenvalues of
    smallest key first (key: "re", "abs", "absre")."""
    lib = L.load()
    n = A.shape[0]
    Af, pa = _host_cplx(np.asarray(A, dtype=np.complex128).reshape(-1, order="F"))
    T = np.zeros(n * n, dtype=np.complex128)
    Q = np.zeros(n * n, dtype=np.complex128)
    kmap = {"re": 0, "abs": 1, "absre": 2}
    L.check(lib.sk_dense_schur(n, pa, T.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                               Q.view(np.float64).ctypes.data_as(C.POINTER(C.c_double)),
                               kmap[key], n if count is None else int(count)))
    return T.reshape(n, n, order="F"), Q.reshape(n, n, order="F")


def dense_sign(A):
    lib = L.load()
    n = A.shape[0]
    Af, pa = _host_cplx(np.asarray(A, dtype=np.complex128).reshape(-1, order="F"))
    S = np.zeros(n * n, dtype=np.complex128)
    L.check(lib.sk_dense_sign(n, pa, S.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))))
    return S.reshape(n, n, order="F")


@dataclass
class SignResult:
    x: torch.Tensor
    status: int
    cycles: int
    cycles_c64: int
    matvecs: int
    converged: bool
    breakdown: bool
    update_norms: np.ndarray = field(default_factory=lambda: np.zeros(0))
    betas: np.ndarray = field(default_factory=lambda: np.zeros(0))
    leaks: np.ndarray = field(default_factory=lambda: np.zeros(0))
    X_shift: torch.Tensor | None = None
    rho_hist: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))
    shift_resid: np.ndarray | None = None
    shift_resid_implicit: np.ndarray | None = None
    resid_ok: bool | None = None
    seconds: float = 0.0


class SignSolver:
    """Holds the parameters and workspace of repeated sign_apply calls."""

    def __init__(self, op: WilsonOperator, sigma, omega, k, tol=1e-9, max_cycles=500,
                 R=None, Lv=None, F=None, project_each_cycle=True, precision="fp64",
                 keep_shift_solutions=False, hist_cap=4096, mixed_switch=0.0, resid_tol=0.0,
                 residuals=False, method="fom", seed=-1):
        self.lib = L.load()
        if precision in ("mixed", "mixed_c64_only"):
            op.ensure_c64()
            if precision == "mixed_c64_only":
                mixed_switch = 1.0
        self.op = op
        self._sg, self.N = _cplx_host(sigma)
        self._om, _ = _cplx_host(omega)
        self.k = int(k)
        self.m = 0 if R is None else int(R.shape[0])
        if self.m:
            _need(R, torch.complex128, self.m * op.n, "R")
            _need(Lv, torch.complex128, self.m * op.n, "L")
            F = F.transpose(0, 1).contiguous()   # column-major
            _need(F, torch.complex128, self.m * self.m, "F")
        self.R, self.Lv, self.F = R, Lv, F
        self.X = (torch.empty((self.N, op.n), dtype=torch.complex128, device=op.device)
                  if keep_shift_solutions else None)
        p = L.SkSignParams()
        p.npoles = self.N
        p.sigma = C.cast(self._sg, C.POINTER(C.c_double))
        p.omega = C.cast(self._om, C.POINTER(C.c_double))
        p.k = self.k
        p.max_cycles = int(max_cycles)
        p.tol = float(tol)
        p.m = self.m
        p.R = R.data_ptr() if self.m else None
        p.L = Lv.data_ptr() if self.m else None
        p.F = self.F.data_ptr() if self.m else None
        p.project_each_cycle = 1 if project_each_cycle else 0
        p.precision = L.SK_PREC_FP64 if precision == "fp64" else L.SK_PREC_MIXED
        p.mixed_switch = float(mixed_switch)
        p.X_shift = self.X.data_ptr() if self.X is not None else None
        p.resid_tol = float(resid_tol)
        p.method = {"fom": L.SK_METHOD_FOM, "gmres": L.SK_METHOD_GMRES}[method]
        p.seed = int(seed)
        self.params = p
        self.residuals = bool(residuals)
        self.opstruct = op.struct()
        nb = self.lib.sign_apply_workspace_bytes(C.byref(self.opstruct), C.byref(p))
        if nb == 0:
            raise SkError(L.SK_ERR_ARG, "invalid parameters for sign_apply")
        self.ws = _workspace(nb, op.device)
        self.hist_cap = hist_cap
        self._hu = (C.c_double * hist_cap)()
        self._hb = (C.c_double * hist_cap)()
        self._hl = (C.c_double * hist_cap)()
        self._hr = (C.c_double * (hist_cap * self.N))()
        self._sr = (C.c_double * self.N)()
        self._si = (C.c_double * self.N)()

    def __call__(self, b, x=None, raise_on_error=True):
        _need(b, torch.complex128, self.op.n, "b")
        if x is None:
            x = torch.empty_like(b)
        st = L.SkStats()
        st.hist_update = C.cast(self._hu, C.POINTER(C.c_double))
        st.hist_beta = C.cast(self._hb, C.POINTER(C.c_double))
        st.hist_leak = C.cast(self._hl, C.POINTER(C.c_double))
        st.hist_cap = self.hist_cap
        st.hist_rho = C.cast(self._hr, C.POINTER(C.c_double))
        if self.residuals:
            st.shift_resid = C.cast(self._sr, C.POINTER(C.c_double))
            st.shift_resid_implicit = C.cast(self._si, C.POINTER(C.c_double))
        status = self.lib.sign_apply(C.byref(self.opstruct), C.byref(self.params), _ptr(b), _ptr(x),
                                     C.byref(st), _ptr(self.ws), self.ws.numel(), _stream())
        if raise_on_error and status not in (L.SK_OK,):
            L.check(status)
        nc = min(st.cycles, self.hist_cap)
        checked = bool(st.resid_checked)
        return SignResult(x=x, status=status, cycles=st.cycles, cycles_c64=st.cycles_c64,
                          matvecs=st.matvecs,
                          converged=bool(st.converged), breakdown=bool(st.breakdown),
                          update_norms=np.array(self._hu[:nc]), betas=np.array(self._hb[:nc]),
                          leaks=np.array(self._hl[:nc]), X_shift=self.X,
                          rho_hist=np.array(self._hr[:nc * self.N]).reshape(nc, self.N),
                          shift_resid=np.array(self._sr[:]) if checked and self.residuals else None,
                          shift_resid_implicit=(np.array(self._si[:]) if checked and self.residuals
                                                else None),
                          resid_ok=bool(st.resid_ok) if checked else None, seconds=st.seconds)


class BatchedSignSolver:
    """sign(H_W) b for many systems in one lockstep solve (sign_apply_batched).

    systems: list of (op, deflation) with deflation None or (R, L, F) as for
    SignSolver, or of dicts {"op", "defl", "k", "sigma", "omega"} where the
    last three (optional) override the shared restart length and poles for
    that system.  sigma, omega: the shared pole set (1-D), or one row per
    system (2-D, nsys x N).  Each call takes one source per system.  Systems
    whose operators share links, dims, kappa, mu and boundary share the
    stencil's link loads."""

    def __init__(self, systems, sigma, omega, k, tol=1e-9, max_cycles=500, precision="fp64",
                 mixed_switch=0.0, project_each_cycle=True, hist_cap=4096):
        self.lib = L.load()
        entries = [s_ if isinstance(s_, dict) else {"op": s_[0], "defl": s_[1]} for s_ in systems]
        self.nsys = len(entries)
        if self.nsys < 1:
            raise ValueError("need at least one system")
        if precision in ("mixed", "mixed_c64_only"):
            for e in entries:
                e["op"].ensure_c64()
            if precision == "mixed_c64_only":
                mixed_switch = 1.0
        self.ops = [e["op"] for e in entries]
        sg = np.asarray(sigma, dtype=np.complex128)
        og = np.asarray(omega, dtype=np.complex128)
        if sg.shape != og.shape or sg.ndim not in (1, 2):
            raise ValueError("sigma and omega must have the same 1-D or 2-D shape")
        self.N = sg.shape[-1]
        if sg.ndim == 2:
            if sg.shape[0] != self.nsys:
                raise ValueError(f"need one pole row per system ({self.nsys}), got {sg.shape[0]}")
            for z, e in enumerate(entries):
                e.setdefault("sigma", sg[z])
                e.setdefault("omega", og[z])
            sg, og = sg[0], og[0]
        self._sg, _ = _cplx_host(sg)
        self._om, _ = _cplx_host(og)
        self._keep = []
        self._desc = (L.SkBatchSystem * self.nsys)()
        for z, e in enumerate(entries):
            d = self._desc[z]
            d.op = e["op"].struct()
            d.k = int(e.get("k") or 0)
            if e.get("sigma") is not None:
                ps, n_ = _cplx_host(e["sigma"])
                po, n2 = _cplx_host(e["omega"])
                if n_ != self.N or n2 != self.N:
                    raise ValueError(f"system {z}: expected {self.N} poles")
                self._keep += [ps, po]
                d.sigma = C.cast(ps, C.POINTER(C.c_double))
                d.omega = C.cast(po, C.POINTER(C.c_double))
            defl = e.get("defl")
            if defl is not None:
                R, Lv, F = defl
                m = int(R.shape[0])
                op = e["op"]
                _need(R, torch.complex128, m * op.n, "R")
                _need(Lv, torch.complex128, m * op.n, "L")
                Fc = F.transpose(0, 1).contiguous()   # column-major
                _need(Fc, torch.complex128, m * m, "F")
                self._keep += [R, Lv, Fc]
                d.m = m
                d.R, d.L, d.F = R.data_ptr(), Lv.data_ptr(), Fc.data_ptr()
        p = L.SkSignParams()
        p.npoles = self.N
        p.sigma = C.cast(self._sg, C.POINTER(C.c_double))
        p.omega = C.cast(self._om, C.POINTER(C.c_double))
        p.k = int(k)
        p.max_cycles = int(max_cycles)
        p.tol = float(tol)
        p.project_each_cycle = 1 if project_each_cycle else 0
        p.precision = L.SK_PREC_FP64 if precision == "fp64" else L.SK_PREC_MIXED
        p.mixed_switch = float(mixed_switch)
        self.params = p
        nb = self.lib.sign_apply_batched_workspace_bytes(self.nsys, self._desc, C.byref(p))
        if nb == 0:
            raise SkError(L.SK_ERR_ARG, "invalid parameters for sign_apply_batched")
        self.ws = _workspace(nb, self.ops[0].device)
        self.hist_cap = hist_cap
        self._hist = [((C.c_double * hist_cap)(), (C.c_double * hist_cap)(), (C.c_double * hist_cap)())
                      for _ in range(self.nsys)]
        self.tile = None

    def __call__(self, bs, xs=None, raise_on_error=True, kernel_times=False):
        """kernel_times: plain launches with HIP events per launch class
        (slower); the per-class times and algorithmic bytes of the live
        systems go to self.kernel_times."""
        if len(bs) != self.nsys:
            raise ValueError(f"expected {self.nsys} sources, got {len(bs)}")
        for z, b in enumerate(bs):
            _need(b, torch.complex128, self.ops[z].n, f"b[{z}]")
        if xs is None:
            xs = [torch.empty_like(b) for b in bs]
        for z, x in enumerate(xs):
            _need(x, torch.complex128, self.ops[z].n, f"x[{z}]")
            self._desc[z].b = bs[z].data_ptr()
            self._desc[z].x = x.data_ptr()
        st = (L.SkStats * self.nsys)()
        for z in range(self.nsys):
            hu, hb, hl = self._hist[z]
            st[z].hist_update = C.cast(hu, C.POINTER(C.c_double))
            st[z].hist_beta = C.cast(hb, C.POINTER(C.c_double))
            st[z].hist_leak = C.cast(hl, C.POINTER(C.c_double))
            st[z].hist_cap = self.hist_cap
        times = None
        if kernel_times:
            times = L.SkKernelTimes()
            st[0].times = C.pointer(times)
        status = self.lib.sign_apply_batched(self.nsys, self._desc, C.byref(self.params), st,
                                             _ptr(self.ws), self.ws.numel(), _stream())
        if times is not None:
            self.kernel_times = {
                name: {"ms": times.ms[i], "launches": int(times.launches[i]),
                       "avg_us": 1e3 * times.ms[i] / times.launches[i],
                       "bytes_per_launch": times.bytes[i] / times.launches[i],
                       "GBs": times.bytes[i] / (times.ms[i] * 1e-3) / 1e9 if times.ms[i] > 0 else None}
                for i, name in enumerate(L.SK_KERNEL_CLASSES) if times.launches[i]}
        if raise_on_error and status != L.SK_OK:
            L.check(status)
        a, b_, c_ = C.c_int(), C.c_int(), C.c_int()
        self.lib.sk_batched_last_tile(C.byref(a), C.byref(b_), C.byref(c_))
        self.tile = {"dot_rows_per_thread": a.value, "update_rows_per_thread": b_.value,
                     "rhs_per_stencil_block": c_.value}
        out = []
        for z in range(self.nsys):
            nc = min(st[z].cycles, self.hist_cap)
            hu, hb, hl = self._hist[z]
            out.append(SignResult(x=xs[z], status=L.SK_OK if st[z].converged else status,
                                  cycles=st[z].cycles, cycles_c64=st[z].cycles_c64,
                                  matvecs=st[z].matvecs, converged=bool(st[z].converged),
                                  breakdown=bool(st[z].breakdown),
                                  update_norms=np.array(hu[:nc]), betas=np.array(hb[:nc]),
                                  leaks=np.array(hl[:nc])))
        return out


def direct_sign_apply(op: WilsonOperator, b, k, method="arnoldi", R=None, Lv=None, F=None,
                      return_sign=False):
    """The direct projection x_P + ||(I-P)b|| V_k sign(M_k) e_1 (library).

    method "arnoldi" (M_k = H_k) or "lanczos" (two-sided Lanczos, M_k = T_k).
    Returns (x, stats dict[, sign(M_kk) as a (kk, kk) tensor])."""
    lib = L.load()
    _need(b, torch.complex128, op.n, "b")
    mth = {"arnoldi": 0, "lanczos": 1}[method]
    m = 0 if R is None else int(R.shape[0])
    Fc = None
    if m:
        _need(R, torch.complex128, m * op.n, "R")
        _need(Lv, torch.complex128, m * op.n, "L")
        Fc = F.transpose(0, 1).contiguous()
    s = op.struct()
    nb = lib.direct_sign_workspace_bytes(C.byref(s), mth, int(k), m)
    if nb == 0:
        raise SkError(L.SK_ERR_ARG, "invalid parameters for direct_sign_apply")
    ws = _workspace(nb, op.device)
    x = torch.empty_like(b)
    S = torch.empty(int(k) * int(k), dtype=torch.complex128, device=op.device) if return_sign else None
    st = L.SkDirectStats()
    L.check(lib.direct_sign_apply(C.byref(s), mth, int(k), m, _ptr(R), _ptr(Lv), _ptr(Fc), _ptr(b), _ptr(x),
                                  _ptr(S), C.byref(st), _ptr(ws), ws.numel(), _stream()))
    stats = {"k_done": st.k_done, "breakdown": bool(st.breakdown), "newton_iters": st.newton_iters,
             "newton_change": st.newton_change, "seconds": st.seconds}
    if return_sign:
        kk = st.k_done
        return x, stats, S[: kk * kk].reshape(kk, kk).transpose(0, 1)
    return x, stats


class OverlapOperator:
    """D(m) = (1 - m/2)(1 + gamma5 sign(H_W)) + m with sign(H_W) by sign_apply
    (the SignSolver's poles, restart length, deflation and precision)."""

    def __init__(self, solver: "SignSolver", mass=0.0, k_outer=30):
        if solver.X is not None:
            raise ValueError("the inner solver must not keep per-shift solutions")
        self.solver, self.mass, self.k_outer = solver, float(mass), int(k_outer)
        self.lib = L.load()
        nb = self.lib.overlap_workspace_bytes(C.byref(solver.opstruct), C.byref(solver.params), self.k_outer)
        if nb == 0:
            raise SkError(L.SK_ERR_ARG, "invalid parameters for the overlap operator")
        self.ws = _workspace(nb, solver.op.device)

    def apply(self, b):
        _need(b, torch.complex128, self.solver.op.n, "b")
        y = torch.empty_like(b)
        st = L.SkStats()
        L.check(self.lib.overlap_apply(C.byref(self.solver.opstruct), C.byref(self.solver.params), self.mass,
                                       _ptr(b), _ptr(y), C.byref(st), _ptr(self.ws), self.ws.numel(),
                                       _stream()))
        return y

    def solve(self, b, tol=1e-8, max_outer=1000, raise_on_error=True):
        _need(b, torch.complex128, self.solver.op.n, "b")
        x = torch.empty_like(b)
        st = L.SkOverlapStats()
        status = self.lib.overlap_solve(C.byref(self.solver.opstruct), C.byref(self.solver.params), self.mass,
                                        self.k_outer, int(max_outer), float(tol), _ptr(b), _ptr(x),
                                        C.byref(st), _ptr(self.ws), self.ws.numel(), _stream())
        if raise_on_error:
            L.check(status)
        return x, {"status": status, "outer_iters": st.outer_iters, "restarts": st.restarts,
                   "sign_calls": st.sign_calls, "inner_matvecs": st.inner_matvecs,
                   "rel_residual": st.rel_residual, "converged": bool(st.converged), "seconds": st.seconds}


def sign_apply(op, b, sigma, omega, k, **kw):
    return SignSolver(op, sigma, omega, k, **{k_: v for k_, v in kw.items() if k_ != "raise_on_error"})(
        b, raise_on_error=kw.get("raise_on_error", True))


def sign_apply_backward(op: WilsonOperator, b, eta, sigma, omega, k, tol=1e-12, max_cycles=1000):
    """Gradient of F = Re <eta, g(H_W) b> (no deflation, complex double).

    Returns (x = g(H_W) b, grad_theta (4, V, 8) float64, dF/dmu)."""
    lib = L.load()
    solver = SignSolver(op, sigma, omega, k, tol=tol, max_cycles=max_cycles)
    p = solver.params
    s = op.struct()
    nb = lib.sign_apply_backward_workspace_bytes(C.byref(s), C.byref(p))
    if nb == 0:
        raise SkError(L.SK_ERR_ARG, "invalid parameters for sign_apply_backward")
    ws = _workspace(nb, op.device)
    _need(b, torch.complex128, op.n, "b")
    _need(eta, torch.complex128, op.n, "eta")
    x = torch.empty_like(b)
    grad = torch.empty((4, op.V, 8), dtype=torch.float64, device=op.device)
    gmu = C.c_double(0.0)
    st = (L.SkStats * 2)()
    L.check(lib.sign_apply_backward(C.byref(s), C.byref(p), _ptr(b), _ptr(eta), _ptr(x), _ptr(grad),
                                    C.byref(gmu), st, _ptr(ws), ws.numel(), _stream()))
    return x, grad, gmu.value


class SignKrylov(torch.autograd.Function):
    """x = g(H_W(U, mu)) b with gradients for the links and mu.

    ``theta`` is the (4, V, 8) real tangent coordinate of the links at the
    current field (U -> exp(i theta^a lambda_a/2) U, evaluated at theta = 0,
    so pass zeros); ``mu`` a 0-dim float64 tensor.  For a real loss L the
    incoming gradient of the complex output is dL/dRe x + i dL/dIm x = eta,
    and L changes by Re <eta, dx>, which is what the library differentiates."""

    @staticmethod
    def forward(ctx, theta, mu, b, op, sigma, omega, k, tol, max_cycles):
        if theta.abs().max().item() != 0.0:
            raise ValueError("theta is a tangent coordinate at the current links: pass zeros")
        opm = op.with_mu(float(mu))
        res = SignSolver(opm, sigma, omega, k, tol=tol, max_cycles=max_cycles)(b)
        ctx.save_for_backward(b)
        ctx.cfg = (opm, sigma, omega, k, tol, max_cycles)
        return res.x

    @staticmethod
    def backward(ctx, grad_x):
        (b,) = ctx.saved_tensors
        opm, sigma, omega, k, tol, max_cycles = ctx.cfg
        _, g, gmu = sign_apply_backward(opm, b, grad_x.contiguous().to(torch.complex128), sigma, omega,
                                        k, tol=tol, max_cycles=max_cycles)
        return g, torch.tensor(gmu, dtype=torch.float64, device=g.device), None, None, None, None, \
            None, None, None
