"""GPU parity of the batched solver (many systems of Algorithm 1 in one
lockstep solve): every system against the oracle's x* on lattices small
enough for dense algebra, and against the single-system solver (itself
checked against the oracle) where the lattice is too large for that."""
import ctypes as C

import numpy as np
import pytest

import skinputs as si
from skinputs.configs import CONFIGS
from oracle import dirac, rational, xstar, deflation, krylov
from tests.gpu_util import make_op, to_dev, from_dev, vecs_to_dev, rel, announce, torch_dev

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-8


def _mixed_batch(with_c64=False):
    """Four systems: two sources on one 4^4 field (shared links), a ragged
    3x4x5x6 lattice with LR deflation, and a 2x3x4x5 point source."""
    import torch
    cfg = CONFIGS["c1"]
    mu = cfg.mus[0]
    sig, om = rational.kl_first_order(cfg.s, cfg.scales[mu])
    out = []
    U1 = si.gauge_links(cfg.dims, cfg.eps, si.seed_for(cfg.L, "gauge"))
    V1 = si.lattice_volume(cfg.dims)
    A1 = dirac.hw_dense(U1, cfg.dims, cfg.kappa, mu)
    op1 = make_op(U1, cfg.dims, cfg.kappa, mu, with_c64=with_c64)
    b1 = si.gaussian_source(12 * V1, si.seed_for(cfg.L, "b"))
    b2 = si.z2_source(12 * V1, si.seed_for(cfg.L, "z2", 0))
    out.append(dict(op=op1, V=V1, A=A1, b=b1, defl=None))
    out.append(dict(op=op1, V=V1, A=A1, b=b2, defl=None))
    dims = (3, 4, 5, 6)
    V2 = si.lattice_volume(dims)
    U2 = si.gauge_links(dims, 0.6, 91)
    A2 = dirac.hw_dense(U2, dims, 0.25, mu)
    R, L, lam, F = deflation.lr_dense(A2, 24)
    dev = (vecs_to_dev(R, V2), vecs_to_dev(L, V2), torch.from_numpy(F).to(torch_dev()))
    out.append(dict(op=make_op(U2, dims, 0.25, mu, with_c64=with_c64), V=V2, A=A2,
                    b=si.gaussian_source(12 * V2, 92), defl=(R, L, F), defl_dev=dev))
    dims = (2, 3, 4, 5)
    V3 = si.lattice_volume(dims)
    U3 = si.gauge_links(dims, 0.5, 93)
    A3 = dirac.hw_dense(U3, dims, 0.25, mu)
    out.append(dict(op=make_op(U3, dims, 0.25, mu, with_c64=with_c64), V=V3, A=A3,
                    b=si.point_source(12 * V3, 7, 1, 2), defl=None))
    return out, sig, om, cfg


def _solve(batch, sig, om, k, **kw):
    from paper_0910_2927_amd import api
    systems = [(s["op"], s.get("defl_dev")) for s in batch]
    solver = api.BatchedSignSolver(systems, sig, om, k, **kw)
    return solver([to_dev(s["b"], s["V"]) for s in batch])


def test_batch_of_uneven_systems_matches_oracle():
    from paper_0910_2927_amd import api
    batch, sig, om, cfg = _mixed_batch()
    announce("sign_apply_batched 4 systems (4^4 x2 shared, 3x4x5x6 m=24, 2x3x4x5) k=20 fp64")
    res = _solve(batch, sig, om, 20, tol=1e-11, max_cycles=400)
    for z, (s, r) in enumerate(zip(batch, res)):
        assert r.converged, z
        Rm = Lm = Fm = None
        if s["defl"] is not None:
            Rm, Lm, Fm = s["defl"]
        ref = xstar.xstar_dense(s["A"], s["b"], sig, om, Rm, Lm, Fm)
        err = rel(from_dev(r.x, s["V"]), ref)
        # the single-system solver on the same system
        single = api.sign_apply(s["op"], to_dev(s["b"], s["V"]), sig, om, 20, tol=1e-11,
                                max_cycles=400,
                                **({} if s["defl"] is None else
                                   dict(R=s["defl_dev"][0], Lv=s["defl_dev"][1], F=s["defl_dev"][2])))
        d = rel(from_dev(r.x, s["V"]), from_dev(single.x, s["V"]))
        print(f"system {z}: cycles={r.cycles} (single {single.cycles}) err={err:.2e} "
              f"vs single {d:.2e}")
        assert err <= TOL_FP64
        assert d <= 1e-9
        assert abs(r.cycles - single.cycles) <= 1


def test_batch_mixed_precision_reaches_fp64_accuracy():
    batch, sig, om, cfg = _mixed_batch(with_c64=True)
    announce("sign_apply_batched 4 systems mixed precision")
    res = _solve(batch, sig, om, 20, tol=1e-11, max_cycles=600, precision="mixed")
    assert any(r.cycles_c64 > 0 for r in res)
    for z, (s, r) in enumerate(zip(batch, res)):
        assert r.converged, z
        Rm = Lm = Fm = None
        if s["defl"] is not None:
            Rm, Lm, Fm = s["defl"]
        err = rel(from_dev(r.x, s["V"]), xstar.xstar_dense(s["A"], s["b"], sig, om, Rm, Lm, Fm))
        print(f"mixed system {z}: cycles={r.cycles} c64={r.cycles_c64} err={err:.2e}")
        assert err <= TOL_FP64


def test_batch_is_deterministic_and_drops_finished_systems():
    """A zero source finishes at once (x = 0) while the others go on; two
    runs give bit-identical results."""
    import torch
    batch, sig, om, cfg = _mixed_batch()
    batch[1]["b"] = np.zeros_like(batch[1]["b"])
    announce("sign_apply_batched with a zero source, twice")
    r1 = _solve(batch, sig, om, 16, tol=1e-10, max_cycles=400)
    r2 = _solve(batch, sig, om, 16, tol=1e-10, max_cycles=400)
    assert r1[1].converged and r1[1].cycles <= 1
    assert float(torch.linalg.vector_norm(r1[1].x)) == 0.0
    for a, b in zip(r1, r2):
        assert a.converged and b.converged
        assert a.cycles == b.cycles
        assert torch.equal(a.x, b.x)
    assert max(r.cycles for r in r1) > r1[1].cycles


def test_point_and_z2_sources_on_one_field_share_links():
    """The multi-source workload at 6^4: 12 point + 16 Z2 sources on one gauge
    field in one batch; each against the single-system solver, and one
    against the oracle's sparse x*."""
    from paper_0910_2927_amd import api
    dims, L = (6, 6, 6, 6), 6
    V = si.lattice_volume(dims)
    mu = 0.3
    U = si.gauge_links(dims, 0.5, si.seed_for(L, "gauge"))
    sig, om = rational.kl_first_order(10, 1.4)
    op = make_op(U, dims, 0.25, mu)
    srcs = [si.point_source(12 * V, 0, sc // 3, sc % 3) for sc in range(12)]   # one propagator
    srcs += [si.z2_source(12 * V, si.seed_for(L, "z2", i)) for i in range(16)]
    announce("sign_apply_batched 6^4, 28 sources on one field, k=30")
    solver = api.BatchedSignSolver([(op, None)] * len(srcs), sig, om, 30, tol=1e-10, max_cycles=300)
    res = solver([to_dev(b, V) for b in srcs])
    for z in (0, 5, 11, 12, 20, 27):
        single = api.sign_apply(op, to_dev(srcs[z], V), sig, om, 30, tol=1e-10, max_cycles=300)
        d = rel(from_dev(res[z].x, V), from_dev(single.x, V))
        print(f"source {z}: cycles={res[z].cycles} (single {single.cycles}) vs single {d:.2e}")
        assert res[z].converged and d <= 1e-8
    # oracle: Algorithm 1 on the CPU to a tight tolerance, its per-shift
    # residuals checked so that it stands for x* (a sparse LU per pole at
    # n = 15552 would take minutes)
    announce("oracle restarted FOM on the CPU, 6^4 Z2 source")
    A = dirac.hw_csr(U, dims, 0.25, mu)
    ref, info = krylov.restarted_fom_lr(lambda v: A @ v, srcs[12], sig, om, 30, tol_update=1e-13,
                                        max_cycles=600, keep_shift_solutions=True)
    assert info["converged"]
    for i in range(len(sig)):
        r = A @ info["X"][i] - sig[i] * info["X"][i] - srcs[12]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(srcs[12])
    err = rel(from_dev(res[12].x, V), ref)
    print(f"Z2 source vs oracle: {err:.2e}")
    assert err <= 1e-8


def test_batched_argument_errors():
    from paper_0910_2927_amd import _lib, api
    lib = _lib.load()
    batch, sig, om, cfg = _mixed_batch()
    ops = (_lib.SkOperator * 2)(batch[0]["op"].struct(), batch[2]["op"].struct())
    p = _lib.SkSignParams()
    sg, N = api._cplx_host(sig)
    og, _ = api._cplx_host(om)
    p.npoles, p.k, p.max_cycles, p.tol = N, 10, 10, 1e-8
    p.sigma = C.cast(sg, C.POINTER(C.c_double))
    p.omega = C.cast(og, C.POINTER(C.c_double))
    assert lib.sign_apply_batched_workspace_bytes(2, ops, None, C.byref(p)) > 0
    b0, b1 = to_dev(batch[0]["b"], batch[0]["V"]), to_dev(batch[2]["b"], batch[2]["V"])
    x0 = b0.clone()
    bp = (C.c_void_p * 2)(b0.data_ptr(), b1.data_ptr())
    xp = (C.c_void_p * 2)(x0.data_ptr(), x0.data_ptr())   # two systems, one solution buffer
    ws = api._workspace(lib.sign_apply_batched_workspace_bytes(2, ops, None, C.byref(p)), b0.device)
    st = lib.sign_apply_batched(2, ops, bp, xp, None, None, None, None, C.byref(p), None,
                                C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == _lib.SK_ERR_ARG and b"share" in lib.sk_last_error()
    m = (C.c_int * 2)(0, 4)
    x1 = b1.clone()
    xp = (C.c_void_p * 2)(x0.data_ptr(), x1.data_ptr())
    st = lib.sign_apply_batched(2, ops, bp, xp, m, None, None, None, C.byref(p), None,
                                C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == _lib.SK_ERR_ARG
    st = lib.sign_apply_batched(2, ops, bp, xp, None, None, None, None, C.byref(p), None,
                                C.c_void_p(ws.data_ptr()), 16, None)
    assert st == _lib.SK_ERR_WORKSPACE
