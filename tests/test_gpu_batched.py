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
    out.append(dict(op=op1, V=V1, A=A1, b=b1, defl=None, sig=sig, om=om))
    out.append(dict(op=op1, V=V1, A=A1, b=b2, defl=None, sig=sig, om=om))
    dims = (3, 4, 5, 6)
    V2 = si.lattice_volume(dims)
    U2 = si.gauge_links(dims, 0.6, 91)
    A2 = dirac.hw_dense(U2, dims, 0.25, mu)
    R, L, lam, F = deflation.lr_dense(A2, 24)
    dev = (vecs_to_dev(R, V2), vecs_to_dev(L, V2), torch.from_numpy(F).to(torch_dev()))
    out.append(dict(op=make_op(U2, dims, 0.25, mu, with_c64=with_c64), V=V2, A=A2,
                    b=si.gaussian_source(12 * V2, 92), defl=(R, L, F), defl_dev=dev))
    out[-1]["sig"], out[-1]["om"] = rational.kl_first_order(cfg.s, 1.5)   # its own pole scale
    dims = (2, 3, 4, 5)
    V3 = si.lattice_volume(dims)
    U3 = si.gauge_links(dims, 0.5, 93)
    A3 = dirac.hw_dense(U3, dims, 0.25, mu)
    out.append(dict(op=make_op(U3, dims, 0.25, mu, with_c64=with_c64), V=V3, A=A3,
                    b=si.point_source(12 * V3, 7, 1, 2), defl=None))
    out[-1]["sig"], out[-1]["om"] = rational.kl_first_order(cfg.s, 1.2)
    return out, sig, om, cfg


def _solve(batch, sig, om, k, **kw):
    from paper_0910_2927_amd import api
    systems = [(s["op"], s.get("defl_dev")) for s in batch]
    solver = api.BatchedSignSolver(systems, np.stack([s["sig"] for s in batch]),
                                   np.stack([s["om"] for s in batch]), k, **kw)
    return solver([to_dev(s["b"], s["V"]) for s in batch])


def test_batch_of_uneven_systems_matches_oracle():
    """Two sources on one field, a deflated ragged lattice and a point source,
    each lattice with its own pole scale."""
    from paper_0910_2927_amd import api
    batch, sig, om, cfg = _mixed_batch()
    announce("sign_apply_batched 4 systems (4^4 x2 shared, 3x4x5x6 m=24, 2x3x4x5) k=20 fp64")
    res = _solve(batch, sig, om, 20, tol=1e-11, max_cycles=400)
    for z, (s, r) in enumerate(zip(batch, res)):
        assert r.converged, z
        Rm = Lm = Fm = None
        if s["defl"] is not None:
            Rm, Lm, Fm = s["defl"]
        ref = xstar.xstar_dense(s["A"], s["b"], s["sig"], s["om"], Rm, Lm, Fm)
        err = rel(from_dev(r.x, s["V"]), ref)
        # the single-system solver on the same system
        single = api.sign_apply(s["op"], to_dev(s["b"], s["V"]), s["sig"], s["om"], 20, tol=1e-11,
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
        err = rel(from_dev(r.x, s["V"]), xstar.xstar_dense(s["A"], s["b"], s["sig"], s["om"], Rm, Lm, Fm))
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


def test_per_kernel_timing_gives_the_same_iterates():
    """With per-kernel timing the cycles run as plain launches stamped by
    HIP events instead of graph replays: bit-identical results in mixed
    precision (all three cycle kinds), and every launch class reports its
    launches with the algorithmic bytes of the systems live in each cycle."""
    import torch
    from paper_0910_2927_amd import api
    batch, sig, om, cfg = _mixed_batch(with_c64=True)
    systems = [(s["op"], s.get("defl_dev")) for s in batch]
    solver = api.BatchedSignSolver(systems, np.stack([s["sig"] for s in batch]),
                                   np.stack([s["om"] for s in batch]), 16, tol=1e-10, max_cycles=400,
                                   precision="mixed")
    bs = [to_dev(s["b"], s["V"]) for s in batch]
    announce("sign_apply_batched graph replay vs timed plain launches (mixed)")
    r1 = solver(bs)
    r2 = solver(bs, kernel_times=True)
    for a, b in zip(r1, r2):
        assert a.converged and b.converged and a.cycles == b.cycles and a.cycles_c64 == b.cycles_c64
        assert torch.equal(a.x, b.x)
    assert 0 < r1[0].cycles_c64 < r1[0].cycles
    kt = solver.kernel_times
    for cls in ("stencil", "gs_dot", "gs_upd_dot", "gs_upd_norm", "small", "sol_update", "project"):
        assert kt[cls]["launches"] > 0 and kt[cls]["ms"] > 0
    cycles = max(r.cycles for r in r1)
    assert kt["small"]["launches"] == cycles
    assert kt["stencil"]["launches"] == 16 * cycles
    # the stencil's bytes: every system steps at every j < 16 while it is
    # live; links once per gauge field (the first two systems share one)
    c64 = r1[0].cycles_c64
    nb = 0.0
    for j, sys_ in enumerate(batch):
        n = 12 * sys_["V"]
        for cyc in range(r1[j].cycles):
            c = 8 if cyc >= r1[0].cycles - c64 else 16
            nb += 16 * 2.0 * n * c
    fields = [batch[0], batch[2], batch[3]]
    for f, owner in zip(fields, (0, 2, 3)):
        n = 12 * f["V"]
        live = max(r1[owner].cycles, r1[1].cycles) if owner == 0 else r1[owner].cycles
        for cyc in range(live):
            c = 8 if cyc >= r1[0].cycles - c64 else 16
            nb += 16 * 3.0 * n * c
    assert abs(kt["stencil"]["bytes_per_launch"] * kt["stencil"]["launches"] - nb) <= 1e-9 * nb


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
    b0, b1 = to_dev(batch[0]["b"], batch[0]["V"]), to_dev(batch[2]["b"], batch[2]["V"])
    x0, x1 = b0.clone(), b1.clone()
    sys_ = (_lib.SkBatchSystem * 2)()
    sys_[0].op, sys_[1].op = batch[0]["op"].struct(), batch[2]["op"].struct()
    sys_[0].b, sys_[1].b = b0.data_ptr(), b1.data_ptr()
    sys_[0].x, sys_[1].x = x0.data_ptr(), x0.data_ptr()   # two systems, one solution buffer
    p = _lib.SkSignParams()
    sg, N = api._cplx_host(sig)
    og, _ = api._cplx_host(om)
    p.npoles, p.k, p.max_cycles, p.tol = N, 10, 10, 1e-8
    p.sigma = C.cast(sg, C.POINTER(C.c_double))
    p.omega = C.cast(og, C.POINTER(C.c_double))
    nb = lib.sign_apply_batched_workspace_bytes(2, sys_, C.byref(p))
    assert nb > 0
    ws = api._workspace(nb, b0.device)
    st = lib.sign_apply_batched(2, sys_, C.byref(p), None, C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == _lib.SK_ERR_ARG and b"share" in lib.sk_last_error()
    sys_[1].x = x1.data_ptr()
    sys_[1].m = 4                        # deflation without vectors
    st = lib.sign_apply_batched(2, sys_, C.byref(p), None, C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert st == _lib.SK_ERR_ARG
    sys_[1].m = 0
    st = lib.sign_apply_batched(2, sys_, C.byref(p), None, C.c_void_p(ws.data_ptr()), 16, None)
    assert st == _lib.SK_ERR_WORKSPACE


def test_systems_with_their_own_restart_lengths():
    """Restart lengths 12, 20, 31 and 17 in one batch: each system as the
    single-system solver with its own k, and against the oracle.  The last
    one diverges (restarted FOM is not monotone; the oracle's own restarted
    FOM diverges there too): it is reported while the others converge."""
    from paper_0910_2927_amd import api, _lib
    batch, sig, om, cfg = _mixed_batch()
    ks = [12, 20, 31, 17]
    entries = [{"op": s_["op"], "defl": s_.get("defl_dev"), "k": kz, "sigma": s_["sig"],
                "omega": s_["om"]} for s_, kz in zip(batch, ks)]
    announce("sign_apply_batched 4 systems, k = 12/20/31/17")
    solver = api.BatchedSignSolver(entries, sig, om, 20, tol=1e-11, max_cycles=600)
    res = solver([to_dev(s_["b"], s_["V"]) for s_ in batch], raise_on_error=False)
    for z, (s_, r, kz) in enumerate(zip(batch[:3], res[:3], ks[:3])):
        assert r.converged, z
        single = api.sign_apply(s_["op"], to_dev(s_["b"], s_["V"]), s_["sig"], s_["om"], kz,
                                tol=1e-11, max_cycles=600,
                                **({} if s_["defl"] is None else
                                   dict(R=s_["defl_dev"][0], Lv=s_["defl_dev"][1], F=s_["defl_dev"][2])))
        Rm = Lm = Fm = None
        if s_["defl"] is not None:
            Rm, Lm, Fm = s_["defl"]
        err = rel(from_dev(r.x, s_["V"]), xstar.xstar_dense(s_["A"], s_["b"], s_["sig"], s_["om"], Rm, Lm, Fm))
        d = rel(from_dev(r.x, s_["V"]), from_dev(single.x, s_["V"]))
        print(f"k={kz}: cycles={r.cycles} (single {single.cycles}) matvecs={r.matvecs} "
              f"err={err:.2e} vs single {d:.2e}")
        assert abs(r.cycles - single.cycles) <= 1
        assert err <= TOL_FP64 and d <= 1e-9
    s3 = batch[3]
    _, info = krylov.restarted_fom_lr(lambda v: s3["A"] @ v, s3["b"], s3["sig"], s3["om"], 17,
                                      tol_update=1e-11, max_cycles=600)
    print(f"k=17: GPU converged={res[3].converged} after {res[3].cycles} cycles; "
          f"oracle converged={info['converged']} after {info['cycles']}")
    assert not info["converged"]
    assert not res[3].converged and res[3].status == _lib.SK_ERR_NOCONV


def test_row_blocking_does_not_change_results():
    """Every tile the tuner may pick gives the same solutions to rounding,
    and the tuner's pick is one of them."""
    from paper_0910_2927_amd import api, _lib
    lib = _lib.load()
    dims = (6, 6, 6, 6)
    V = si.lattice_volume(dims)
    U = si.gauge_links(dims, 0.5, 77)
    sig, om = rational.kl_first_order(8, 1.5)
    op = make_op(U, dims, 0.25, 0.3)
    srcs = [to_dev(si.z2_source(12 * V, 500 + i), V) for i in range(6)]
    outs = {}
    try:
        for tile in [(1, 1, 1), (2, 1, 4), (8, 1, 2), (4, 2, 8), (8, 4, 3), (0, 0, 0)]:
            assert lib.sk_batched_set_tile(*tile) == _lib.SK_OK
            announce(f"sign_apply_batched 6^4 x6 tile {tile}")
            solver = api.BatchedSignSolver([(op, None)] * 6, sig, om, 24, tol=1e-10, max_cycles=300)
            res = solver(srcs)
            assert all(r.converged for r in res)
            outs[tile] = [r.x.clone() for r in res]
            if tile == (0, 0, 0):
                print("tuner picked", solver.tile)
                assert solver.tile["dot_rows_per_thread"] in (1, 2, 4, 8)
                assert solver.tile["update_rows_per_thread"] in (1, 2, 4)
                assert solver.tile["rhs_per_stencil_block"] in (1, 2, 4, 8)
            else:
                assert solver.tile == {"dot_rows_per_thread": tile[0], "update_rows_per_thread": tile[1],
                                       "rhs_per_stencil_block": tile[2]}
    finally:
        lib.sk_batched_set_tile(0, 0, 0)
    ref = outs[(1, 1, 1)]
    for tile, xs in outs.items():
        for a, b in zip(xs, ref):
            d = rel(from_dev(a, V), from_dev(b, V))
            assert d <= 1e-10, (tile, d)


def test_deflated_lattices_whose_row_blocking_is_not_monotone():
    """8x8x8x4 (n = 24576, one row per thread, 96 row blocks) next to the
    larger 6x6x6x10 (n = 25920, two rows per thread, 51 row blocks): the
    deflation dots of the smaller system need more row blocks than the
    largest system; every block must still be reduced.  The projector is
    built from random orthonormal R = L (F = I, projection of the source
    only), which both solvers take as given."""
    import torch
    from paper_0910_2927_amd import api
    sig, om = rational.kl_first_order(5, 1.5)
    entries, bs, singles = [], [], []
    for dims, seed in (((8, 8, 8, 4), 41), ((6, 6, 6, 10), 42)):
        V = si.lattice_volume(dims)
        U = si.gauge_links(dims, 0.5, seed)
        op = make_op(U, dims, 0.25, 0.3)
        Q = np.linalg.qr(si.gaussian_source(12 * V * 8, seed + 7).reshape(12 * V, 8))[0]
        R = vecs_to_dev(Q, V)
        F = torch.eye(8, dtype=torch.complex128, device=R.device)
        b = to_dev(si.gaussian_source(12 * V, seed + 100), V)
        entries.append((op, (R, R, F)))
        bs.append(b)
        announce(f"sign_apply {dims} with an 8-dimensional projector")
        singles.append(api.sign_apply(op, b, sig, om, 20, tol=1e-11, max_cycles=400, R=R, Lv=R, F=F,
                                      project_each_cycle=False))
    announce("sign_apply_batched 8x8x8x4 + 6x6x6x10, m=8")
    res = api.BatchedSignSolver(entries, sig, om, 20, tol=1e-11, max_cycles=400,
                                project_each_cycle=False)(bs)
    for r, s_ in zip(res, singles):
        d = float((r.x - s_.x).norm() / s_.x.norm())
        print(f"batched vs single: {d:.2e}, cycles {r.cycles} vs {s_.cycles}")
        assert r.converged and d <= 1e-9


def test_batched_84_source_workload():
    """The batched configuration itself: 12 spin-colour point sources at site 0
    and 16 Z2 sources on each of the 6^4 (eps 0.5, m 10, k 40), 8^4 (eps 0.6,
    m 20, k 50) and 10^4 (eps 0.7, m 40, k 60) fields at mu = 0.3, 16 poles at
    each lattice's scale, GPU deflation, mixed precision switching to complex
    float at a relative update of 1e-2, all 84 systems in one batch.  Every
    system against the same source solved alone in complex double (itself
    pinned to the oracle below), and each lattice's Gaussian source, solved
    in a batch of its own with the same settings, against the oracle's full
    x*."""
    import json
    import os
    import torch
    from paper_0910_2927_amd import api
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    mu = 0.3
    tol = 1e-10
    lattices, systems, bs = [], [], []
    for name in ("c6", "c2", "c3"):
        cfg = CONFIGS[name]
        U = si.gauge_links(cfg.dims, cfg.eps, si.seed_for(cfg.L, "gauge"))
        op = make_op(U, cfg.dims, cfg.kappa, mu, with_c64=True)
        announce(f"eigensolve {name} for the batch")
        R, Lv, F, lam, st = api.deflation_eigensolve(op, cfg.m, nev_extra=16, tol=1e-12)
        sig, om = api.kl_poles(cfg.s, cfg.scales[mu])
        srcs = [si.point_source(cfg.n, 0, sc // 3, sc % 3) for sc in range(12)]
        srcs += [si.z2_source(cfg.n, si.seed_for(cfg.L, "z2", i)) for i in range(16)]
        lt = dict(cfg=cfg, op=op, defl=(R, Lv, F), sig=sig, om=om, srcs=srcs)
        lattices.append(lt)
        for b in srcs:
            systems.append({"op": op, "defl": (R, Lv, F), "k": cfg.k, "sigma": sig, "omega": om})
            bs.append(to_dev(b, cfg.V))
    assert len(systems) == 84
    announce("sign_apply_batched 84 systems, mixed, switch 1e-2")
    solver = api.BatchedSignSolver(systems, lattices[0]["sig"], lattices[0]["om"], lattices[0]["cfg"].k,
                                   tol=tol, max_cycles=400, precision="mixed", mixed_switch=1e-2)
    res = solver(bs)
    assert all(r.converged for r in res)
    assert max(r.cycles_c64 for r in res) > 0
    z = 0
    worst = []
    for lt in lattices:
        cfg = lt["cfg"]
        R, Lv, F = lt["defl"]
        single = api.SignSolver(lt["op"], lt["sig"], lt["om"], cfg.k, tol=tol, max_cycles=400, R=R, Lv=Lv, F=F)
        errs = []
        for b in bs[z:z + 28]:
            r1 = single(b)
            errs.append(float(torch.linalg.vector_norm(res[z + len(errs)].x - r1.x)
                              / torch.linalg.vector_norm(r1.x)))
        z += 28
        worst.append(max(errs))
        # the Gaussian source of the lattice against the oracle's full x*
        g = json.load(open(os.path.join(golden, f"{cfg.name}_mu{mu:g}.json")))
        bg = si.gaussian_source(cfg.n, si.seed_for(cfg.L, "b"))
        announce(f"batched Gaussian source {cfg.name}")
        rg = api.BatchedSignSolver([{"op": lt["op"], "defl": lt["defl"], "k": cfg.k, "sigma": lt["sig"],
                                     "omega": lt["om"]}], lt["sig"], lt["om"], cfg.k, tol=tol, max_cycles=400,
                                   precision="mixed", mixed_switch=1e-2)([to_dev(bg, cfg.V)])[0]
        xg = from_dev(rg.x, cfg.V)
        full = os.path.join(golden, f"{cfg.name}_mu{mu:g}_x.npy")
        if os.path.exists(full):
            eg = rel(xg, np.load(full))
        else:
            eg = rel(xg[np.array(g["sample_index"])], np.array(g["x_re"]) + 1j * np.array(g["x_im"]))
        print(f"{cfg.name}: batch vs single complex double max {max(errs):.2e}; Gaussian vs oracle {eg:.2e}")
        assert eg <= 1e-8
    assert max(worst) <= 1e-8
