#!/usr/bin/env python3
"""Throughput of sign(H_W) b by restarted multishift FOM-LR on one MI355X.

One step = one complete solve x ~ sign(H_W) b (Algorithm 1: deflated start,
restart cycles of k Arnoldi steps with CGS2, shifted Hessenberg solves,
solution update, projection step) for one synthetic source on the 10^4
lattice at mu = 0.3, with the inputs resident in device memory.  Prints one
JSON line:  value = solves per second.

    python bench.py [--steps K] [--warmup W] [--config c3] [--mu 0.3]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--mu", type=float, default=0.3)
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--tol", type=float, default=None, help="override the configuration's tolerance")
    ap.add_argument("--mixed-switch", type=float, default=None,
                    help="override the relative update at which mixed precision switches to complex float")
    ap.add_argument("--cpu-cycles", type=int, default=2,
                    help="restart cycles of the CPU oracle to time (bounded sample)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the multi-source leg (84 sources on 6^4, 8^4, 10^4)")
    ap.add_argument("--batched-only", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the 16^4 / 24^4 bandwidth sweep")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the 16^4 / 24^4 bandwidth sweep (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 512 MiB three times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE hardware counters) and exit")
    ap.add_argument("--solve-only", action="store_true",
                    help="setup, warm-up and the timed solves only (for profiler runs)")
    ap.add_argument("--no-methods", action="store_true",
                    help="skip the comparison of GMRES-LR and the direct projections at 10^4")
    ap.add_argument("--no-backward", action="store_true", help="skip the timing of the gradient")
    ap.add_argument("--batched-tile", default=None,
                    help="dot,update,rhs: fix the batched launch shapes (skips the tuner; for "
                         "profiler runs of --batched-only)")
    ap.add_argument("--batched-profile", action="store_true",
                    help="with --batched-only: stop after the warm-up and the timed batched solve "
                         "(a kernel trace then holds those two solves' launches only)")
    ap.add_argument("--batched-switch", type=float, default=1e-2,
                    help="relative update below which the batch switches to complex float "
                         "(the single-source solves keep the library's 1e-3)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# sources that define each kernel whose hardware counters are committed
_GS_SOURCES = ("dcgs2_dev.h", "dcgs2.hip", "sk_common.h", "sk_internal.h")
KERNEL_SOURCES = {"k_dc_update": _GS_SOURCES, "k_dc_dot": _GS_SOURCES,
                  "k_wilson": ("stencil_dev.h", "wilson.hip", "sk_common.h", "sk_internal.h")}

# kernel class of the per-kernel timing -> kernel name in a trace
KERNEL_NAMES = {"stencil": "k_wilson", "gs_dot": "k_dc_dot", "gs_upd_dot": "k_dc_update",
                "gs_upd_norm": "k_dc_update_final", "small": "k_fom_poles", "sol_update": "k_cx_update",
                "project": "k_cp_apply", "gs_reduce": "k_dc_reduce"}


def kernel_source_hash(kernel):
    """sha256 of the sources that define `kernel`."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, ()):
        h.update(open(os.path.join(ROOT, "paper_0910_2927_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def load_counters(path):
    """key: value lines of a committed hardware-counter summary."""
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ", "|", "`")):
            k, v = line.split(":", 1)
            v = v.strip()
            try:
                out[k.strip()] = float(v)
            except ValueError:
                out[k.strip()] = v
    return out


def kernel_times(lib, solver, b, x, stream):
    """Per-class kernel times of one solve (HIP events around each launch)."""
    import torch
    from paper_0910_2927_amd import _lib
    times = _lib.SkKernelTimes()
    st = _lib.SkStats()
    st.times = C.pointer(times)
    status = lib.sign_apply(C.byref(solver.opstruct), C.byref(solver.params), C.c_void_p(b.data_ptr()),
                            C.c_void_p(x.data_ptr()), C.byref(st), C.c_void_p(solver.ws.data_ptr()),
                            solver.ws.numel(), C.c_void_p(stream.cuda_stream))
    if status not in (_lib.SK_OK, _lib.SK_ERR_NOCONV):
        _lib.check(status)
    torch.cuda.synchronize()
    kern = {}
    for i, name in enumerate(_lib.SK_KERNEL_CLASSES):
        if times.launches[i]:
            kern[name] = {"ms": times.ms[i], "launches": int(times.launches[i]),
                          "avg_us": 1e3 * times.ms[i] / times.launches[i],
                          "bytes_per_launch": times.bytes[i] / times.launches[i],
                          "GBs": times.bytes[i] / (times.ms[i] * 1e-3) / 1e9 if times.ms[i] > 0 else None}
    return kern, st


def launch_floor(nbytes, reps=100):
    """Floors for a kernel that moves nbytes, on the GPU side of launches
    (a HIP graph of reps back-to-back kernels, replayed; HIP events around
    the replay): a one-block elementwise kernel, and a device copy whose
    read + write traffic is nbytes."""
    import torch
    tiny = torch.zeros(1, device="cuda")
    src = torch.zeros(max(1, int(nbytes) // 8), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)

    def per_launch_us(fn):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(reps):
                fn()
        g.replay()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            g.replay()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, 1e3 * e0.elapsed_time(e1) / reps)
        return best

    return {"launch_floor_us": per_launch_us(lambda: tiny.add_(1.0)),
            "copy_same_bytes_us": per_launch_us(lambda: dst.copy_(src)), "bytes": int(nbytes),
            "note": "per kernel in a replayed graph of back-to-back launches"}


def sweep_leg():
    """Stencil and Gram-Schmidt bandwidth where the basis no longer fits in
    the 256 MB last-level cache: one restart cycle (k = 16) on 16^4 and 24^4
    lattices, complex double and complex float."""
    import torch
    import skinputs as si
    from paper_0910_2927_amd import api, _lib
    lib = _lib.load()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    out = []
    for L in (16, 24):
        dims = (L, L, L, L)
        V = L ** 4
        U = si.gauge_links(dims, 0.7, si.seed_for(L, "gauge"))
        links = torch.from_numpy(si.links_soa_from_canonical(U).reshape(-1)).to(dev)
        del U
        op = api.WilsonOperator(links, dims, 0.25, 0.3, True, links64=links.to(torch.complex64))
        b = torch.from_numpy(si.soa_from_canonical(si.gaussian_source(12 * V, si.seed_for(L, "b")), V)).to(dev)
        sig, om = api.kl_poles(8, 2.0)
        # consistency at this size: the complex-float stencil against the
        # complex-double one (each pinned to the oracle on smaller lattices)
        w64 = api.wilson_apply(op, b)
        w32 = api.wilson_apply(op, b.to(torch.complex64))
        stencil_c64_vs_c128 = float(torch.linalg.vector_norm(w32.to(torch.complex128) - w64)
                                    / torch.linalg.vector_norm(w64))
        xs = {}
        for prec in ("fp64", "mixed_c64_only"):
            sv = api.SignSolver(op, sig, om, 16, tol=1e-10, max_cycles=1, precision=prec, resid_tol=1.0)
            x = torch.empty_like(b)
            kernel_times(lib, sv, b, x, stream)          # warm-up
            kern, _ = kernel_times(lib, sv, b, x, stream)
            xs[prec] = x.clone()
            row = {"lattice": f"{L}^4", "n": 12 * V, "basis": "c128" if prec == "fp64" else "c64",
                   "stencil_c64_vs_c128": stencil_c64_vs_c128}
            if prec != "fp64":
                row["cycle_c64_vs_c128"] = float(torch.linalg.vector_norm(xs[prec] - xs["fp64"])
                                                 / torch.linalg.vector_norm(xs["fp64"]))
            for name in ("stencil", "gs_dot", "gs_upd_dot"):
                row[name + "_GBs"] = kern[name]["GBs"]
                row[name + "_avg_us"] = kern[name]["avg_us"]
            out.append(row)
            log(f"sweep {L}^4 {row['basis']}: stencil {row['stencil_GBs']:.0f}, dots "
                f"{row['gs_dot_GBs']:.0f}, update {row['gs_upd_dot_GBs']:.0f} GB/s")
            del sv
        assert stencil_c64_vs_c128 < 1e-6 and out[-1]["cycle_c64_vs_c128"] < 1e-5, out[-1]
        del op, links, b, xs, w64, w32
        torch.cuda.empty_cache()
    return out


def methods_leg(op, b, sigma, omega, cfg, R, Lv, F, xstar_full, fom_value):
    """The other methods of the paper on the headline input (10^4, mu = 0.3,
    the same deflation): restarted multishift GMRES-LR with the same poles
    and restart length, and the direct projections x_P + ||(I-P)b|| V_k
    sign(M_k) e_1 by Arnoldi and by two-sided Lanczos (no rational
    approximation; error against the oracle's x*, which carries the
    rational approximation's own error, is reported as it is).  Each timed
    once after a warm-up."""
    import torch
    import skinputs as si
    from paper_0910_2927_amd import api
    out = {"fom_lr_solves_per_s": fom_value}

    def err_of(xd):
        if xstar_full is None:
            return None
        xh = si.canonical_from_soa(xd.cpu().numpy(), cfg.V)
        return float(np.linalg.norm(xh - xstar_full) / np.linalg.norm(xstar_full))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    try:
        gm = api.SignSolver(op, sigma, omega, cfg.k, tol=cfg.tol, max_cycles=cfg.max_cycles, R=R, Lv=Lv, F=F,
                            method="gmres")
        r, t = timed(lambda: gm(b, raise_on_error=False))
        out["gmres_lr"] = {"seconds": t, "cycles": r.cycles, "converged": r.converged,
                           "rel_err_vs_oracle": err_of(r.x), "status": r.status}
        log(f"methods: GMRES-LR {t * 1e3:.1f} ms, {r.cycles} cycles, converged {r.converged}")
    except Exception as e:   # noqa: BLE001 - reported, not fatal for the bench
        out["gmres_lr"] = {"error": str(e)}
    for mth in ("arnoldi", "lanczos"):
        rows = []
        for k in (64, 128, 256):
            try:
                (xd, st), t = timed(lambda: api.direct_sign_apply(op, b, k, mth, R=R, Lv=Lv, F=F))
                rows.append({"k": k, "seconds": t, "k_done": st["k_done"], "newton_iters": st["newton_iters"],
                             "rel_err_vs_oracle_xstar": err_of(xd)})
            except Exception as e:   # noqa: BLE001
                rows.append({"k": k, "error": str(e)})
        out[f"direct_{mth}"] = rows
        log(f"methods: direct {mth}: " + ", ".join(
            f"k={r_['k']} {r_.get('seconds', 0) * 1e3:.1f} ms err {r_.get('rel_err_vs_oracle_xstar')}"
            for r_ in rows))
    return out


def backward_leg():
    """The gradient of Re<eta, g(H_W) b> on the backward configuration (8^4,
    mu = 0.3, 16 poles, k = 50, complex double): two multishift solves (H_W
    and H_W^H) with per-shift solutions and the link/mu derivative kernel."""
    import torch
    import skinputs as si
    from skinputs.configs import CONFIGS
    from paper_0910_2927_amd import api
    cfg = CONFIGS["cg"]
    mu = cfg.mus[0]
    dev = torch.device("cuda:0")
    U = si.gauge_links(cfg.dims, cfg.eps, si.seed_for(cfg.L, "gauge"))
    links = torch.from_numpy(si.links_soa_from_canonical(U).reshape(-1)).to(dev)
    op = api.WilsonOperator(links, cfg.dims, cfg.kappa, mu, cfg.antiperiodic_t)
    b = torch.from_numpy(si.soa_from_canonical(si.gaussian_source(cfg.n, si.seed_for(cfg.L, "b")), cfg.V)).to(dev)
    eta = torch.from_numpy(si.soa_from_canonical(si.gaussian_source(cfg.n, si.seed_for(cfg.L, "eta")),
                                                 cfg.V)).to(dev)
    sig, om = api.kl_poles(cfg.s, cfg.scales[mu])
    api.sign_apply_backward(op, b, eta, sig, om, cfg.k, tol=cfg.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, g, gmu = api.sign_apply_backward(op, b, eta, sig, om, cfg.k, tol=cfg.tol)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    t0 = time.perf_counter()
    api.sign_apply(op, b, sig, om, cfg.k, tol=cfg.tol, max_cycles=cfg.max_cycles)
    torch.cuda.synchronize()
    tf = time.perf_counter() - t0
    log(f"backward (8^4): {t * 1e3:.1f} ms per gradient, forward alone {tf * 1e3:.1f} ms")
    return {"workload": f"cg: 8^4, eps={cfg.eps}, mu={mu}, {2 * cfg.s} poles, k={cfg.k}, complex double",
            "seconds_per_gradient": t, "seconds_forward_only": tf,
            "grad_kernel_bytes": (24 * 2 * cfg.s + 36) * 16 * cfg.V}


def batched_leg(args, log_prefix="batched"):
    """The multi-source workload: 12 spin-colour point sources at site 0 plus
    16 Z2 noise sources on each of the 6^4, 8^4 and 10^4 gauge fields (84
    independent systems, mu = 0.3), solved in one lockstep batch in mixed
    precision, against the same 84 solves one by one in complex double."""
    import torch
    import skinputs as si
    from skinputs.configs import CONFIGS
    from paper_0910_2927_amd import api

    dev = torch.device("cuda:0")
    mu = 0.3
    lattices = []
    for name in ("c6", "c2", "c3"):
        cfg = CONFIGS[name]
        c = cfg.scales.get(mu)
        if c is None:
            log(f"{log_prefix}: no pole scale for {name} at mu={mu}; leg skipped")
            return None
        U = si.gauge_links(cfg.dims, cfg.eps, si.seed_for(cfg.L, "gauge"))
        links = torch.from_numpy(si.links_soa_from_canonical(U).reshape(-1)).to(dev)
        op = api.WilsonOperator(links, cfg.dims, cfg.kappa, mu, cfg.antiperiodic_t,
                                links64=links.to(torch.complex64))
        R, Lv, F, lam, est = api.deflation_eigensolve(op, cfg.m, nev_extra=16, tol=1e-12)
        sig, om = api.kl_poles(cfg.s, c)
        srcs = [si.point_source(cfg.n, 0, sc // 3, sc % 3) for sc in range(12)]
        srcs += [si.z2_source(cfg.n, si.seed_for(cfg.L, "z2", i)) for i in range(16)]
        bd = [torch.from_numpy(si.soa_from_canonical(b, cfg.V)).to(dev) for b in srcs]
        lattices.append(dict(cfg=cfg, op=op, defl=(R, Lv, F), sig=sig, om=om, b=bd))
        log(f"{log_prefix}: {name} {cfg.dims[0]}^4 ready (m={cfg.m}, c={c}, "
            f"eigensolve {est['matvecs']} matvecs)")
    systems, bs = [], []
    for lt in lattices:
        for b in lt["b"]:
            systems.append({"op": lt["op"], "defl": lt["defl"], "k": lt["cfg"].k,
                            "sigma": lt["sig"], "omega": lt["om"]})
            bs.append(b)
    nsys = len(systems)
    tol, maxc = 1e-10, 400
    from paper_0910_2927_amd import _lib
    if args.batched_tile:
        a_, b_, c_ = (int(v) for v in args.batched_tile.split(","))
        _lib.check(_lib.load().sk_batched_set_tile(a_, b_, c_))
    solver = api.BatchedSignSolver(systems, lattices[0]["sig"], lattices[0]["om"], lattices[0]["cfg"].k,
                                   tol=tol, max_cycles=maxc, precision="mixed",
                                   mixed_switch=args.batched_switch)
    xs = [torch.empty_like(b) for b in bs]
    solver(bs, xs)                      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = solver(bs, xs)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    log(f"{log_prefix}: {nsys} systems in one batch: {tb:.3f} s "
        f"(cycles {min(r.cycles for r in res)}..{max(r.cycles for r in res)})")
    if args.batched_profile:            # the two batched solves only, for a kernel trace
        return {"systems": nsys, "batched_seconds": tb, "tile": solver.tile}
    # per launch class: HIP events that the launches stamp (plain launches,
    # one more solve), algorithmic bytes summed over the systems live in each
    # cycle
    xk = [torch.empty_like(b) for b in bs]
    solver(bs, xk, kernel_times=True)
    bkern = solver.kernel_times
    log(f"{log_prefix}: kernel classes: " + ", ".join(
        f"{k_}: {v['ms']:.1f} ms/{v['launches']} ({v['GBs'] or 0:.0f} GB/s)" for k_, v in bkern.items()))
    # the same solves one by one in complex double
    ts, errs, cyc1 = 0.0, [], []
    z = 0
    for lt in lattices:
        R, Lv, F = lt["defl"]
        single = api.SignSolver(lt["op"], lt["sig"], lt["om"], lt["cfg"].k, tol=tol, max_cycles=maxc,
                                precision="fp64", R=R, Lv=Lv, F=F)
        x1 = torch.empty_like(lt["b"][0])
        single(lt["b"][0], x1)          # warm-up per lattice
        for b in lt["b"]:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r1 = single(b, x1)
            torch.cuda.synchronize()
            ts += time.perf_counter() - t0
            cyc1.append(r1.cycles)
            errs.append(float(torch.linalg.vector_norm(xs[z] - x1) / torch.linalg.vector_norm(x1)))
            z += 1
    log(f"{log_prefix}: one by one in complex double: {ts:.3f} s; max rel diff {max(errs):.2e}")
    # parity with the oracle: the Gaussian source of each lattice, whose x*
    # the oracle stored at a sample of components, solved as one batch with
    # the same settings
    gerr = []
    gsys, gbs = [], []
    for lt in lattices:
        cfg = lt["cfg"]
        gsys.append({"op": lt["op"], "defl": lt["defl"], "k": cfg.k, "sigma": lt["sig"], "omega": lt["om"]})
        gbs.append(torch.from_numpy(si.soa_from_canonical(si.gaussian_source(cfg.n, si.seed_for(cfg.L, "b")),
                                                          cfg.V)).to(dev))
    gres = api.BatchedSignSolver(gsys, lattices[0]["sig"], lattices[0]["om"], lattices[0]["cfg"].k, tol=tol,
                                 max_cycles=maxc, precision="mixed",
                                 mixed_switch=args.batched_switch)(gbs)
    for lt, r in zip(lattices, gres):
        cfg = lt["cfg"]
        gpath = os.path.join(ROOT, "tests", "golden", f"{cfg.name}_mu{mu:g}.json")
        g = json.load(open(gpath))
        xs_ = si.canonical_from_soa(r.x.cpu().numpy(), cfg.V)[np.array(g["sample_index"])]
        ref = np.array(g["x_re"]) + 1j * np.array(g["x_im"])
        gerr.append(float(np.linalg.norm(xs_ - ref) / np.linalg.norm(ref)))
    log(f"{log_prefix}: Gaussian sources vs oracle x* samples: " + ", ".join(f"{e:.1e}" for e in gerr))
    per_lat = []
    for i, lt in enumerate(lattices):
        per_lat.append(max(errs[28 * i:28 * (i + 1)]))
    return {"workload": "12 point (site 0, every spin-colour) + 16 Z2 sources on each of the "
                        "6^4 (eps 0.5, m 10, k 40), 8^4 (eps 0.6, m 20, k 50) and 10^4 "
                        f"(eps 0.7, m 40, k 60) fields, mu={mu}, 16 poles at each lattice's "
                        f"scale, tol={tol}",
            "systems": nsys, "batched_mixed_solves_per_s": nsys / tb,
            "single_fp64_solves_per_s": nsys / ts, "ratio": ts / tb,
            "batched_seconds": tb, "single_seconds": ts,
            "mixed_switch": args.batched_switch,
            "cycles_batched": [r.cycles for r in res], "cycles_c64": [r.cycles_c64 for r in res],
            "cycles_single": cyc1,
            "max_rel_diff_vs_fp64": max(errs), "max_rel_diff_vs_fp64_per_lattice": per_lat,
            "sampled_rel_err_vs_oracle_per_lattice": gerr,
            "all_converged": all(r.converged for r in res),
            "tile": solver.tile, "kernels": bkern}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark measures one GPU (--gpus 1); the sign(H_W)b "
                                   "solve shards by source with no communication, so N GPUs run "
                                   "N independent processes of this benchmark"}))
        sys.exit(2)

    import torch
    import skinputs as si
    from skinputs.configs import CONFIGS
    from paper_0910_2927_amd import api, _lib

    if args.copy_calibration:
        nbytes = 512 << 20
        src = torch.ones(nbytes // 16, dtype=torch.complex128, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": 3}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched": batched_leg(args)}), flush=True)
        return
    if args.sweep_only:
        print(json.dumps({"bandwidth_sweep": sweep_leg()}), flush=True)
        return
    cfg = CONFIGS[args.config]
    mu = args.mu
    precision_run = args.precision or cfg.precision
    dev = torch.device("cuda:0")
    log(f"config {cfg.name} dims={cfg.dims} mu={mu} k={cfg.k} s={cfg.s} precision={precision_run}")

    # ---- inputs (seeded, synthetic), moved to HBM before timing
    U = si.gauge_links(cfg.dims, cfg.eps, si.seed_for(cfg.L, "gauge"))
    b = si.gaussian_source(cfg.n, si.seed_for(cfg.L, "b"))
    links = torch.from_numpy(si.links_soa_from_canonical(U).reshape(-1)).to(dev)
    bd = torch.from_numpy(si.soa_from_canonical(b, cfg.V)).to(dev)
    op = api.WilsonOperator(links, cfg.dims, cfg.kappa, mu, cfg.antiperiodic_t)
    c = cfg.scales.get(mu)
    if c is None:
        raise SystemExit(f"no pole scale recorded for {cfg.name} at mu={mu}")
    sigma, omega = api.kl_poles(cfg.s, c)
    # ---- deflation data on the GPU (setup: excluded from the timed solves)
    m_used = cfg.m
    eig = None
    R = Lv = F = None
    if m_used > 0:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R, Lv, F, lam, est = api.deflation_eigensolve(op, m_used, nev_extra=16, tol=1e-12)
        torch.cuda.synchronize()
        eig = {"seconds": time.perf_counter() - t0, "m": m_used, "matvecs": est["matvecs"],
               "restarts": est["restarts"], "resid": est["resid"], "gap": est["gap"],
               "lambda_min_abs": float(np.abs(lam).min()), "lambda_m_abs": float(np.abs(lam).max())}
        log(f"eigensolve m={m_used}: {eig['seconds']:.2f} s, {est['matvecs']} matvecs")
    tol = args.tol if args.tol is not None else cfg.tol
    switch = args.mixed_switch if args.mixed_switch is not None else cfg.mixed_switch
    solver = api.SignSolver(op, sigma, omega, cfg.k, tol=tol, max_cycles=cfg.max_cycles,
                            precision=precision_run, R=R, Lv=Lv, F=F, mixed_switch=switch)
    x = torch.empty_like(bd)

    # ---- warmup, then K timed solves
    for _ in range(args.warmup):
        res = solver(bd, x)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    cycles = []
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        res = solver(bd, x)
        cycles.append(res.cycles)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    sec = max(ms_total / 1e3, 1e-12)
    value = args.steps / sec
    log(f"{args.steps} solves in {sec:.4f} s (wall {wall:.4f} s); cycles/solve={cycles[-1]} "
        f"(complex float {res.cycles_c64}) matvecs={res.matvecs}")
    if args.solve_only:
        errs = {}
        gpath = os.path.join(ROOT, "tests", "golden", f"{cfg.name}_mu{mu:g}.json")
        if os.path.exists(gpath):
            g = json.load(open(gpath))
            xh = si.canonical_from_soa(x.cpu().numpy(), cfg.V)
            ref = np.array(g["x_re"]) + 1j * np.array(g["x_im"])
            errs["sampled"] = float(np.linalg.norm(xh[np.array(g["sample_index"])] - ref) / np.linalg.norm(ref))
            if os.path.exists(gpath[:-5] + "_x.npy"):
                xf = np.load(gpath[:-5] + "_x.npy")
                errs["full"] = float(np.linalg.norm(xh - xf) / np.linalg.norm(xf))
        print(json.dumps({"solve_only": True, "config": cfg.name, "mu": mu, "solves_per_s": value,
                          "ms_per_solve": 1e3 * sec / args.steps, "steps": args.steps, "tol": tol,
                          "mixed_switch": switch, "cycles": cycles[-1], "cycles_c64": res.cycles_c64,
                          "fp64_check_ok": res.resid_ok, "rel_err_vs_oracle": errs}), flush=True)
        return

    # ---- per-kernel timing (HIP events around every launch on the solve's
    # stream, plain launches): one more solve as timed, and one whose cycles
    # all use the complex-float basis, which gives the dominant kernel
    lib = _lib.load()
    kern, _ = kernel_times(lib, solver, bd, x, stream)
    log("kernel classes: " + ", ".join(f"{k_}: {v['ms']:.2f} ms/{v['launches']} "
                                       f"({v['GBs'] or 0:.0f} GB/s)" for k_, v in kern.items()))
    x64 = torch.empty_like(bd)
    solver_c64 = api.SignSolver(op, sigma, omega, cfg.k, tol=cfg.tol, max_cycles=cfg.max_cycles,
                                precision="mixed_c64_only", R=R, Lv=Lv, F=F)
    kern_c64, _ = kernel_times(lib, solver_c64, bd, x64, stream)
    # the dominant kernel: the class with the largest summed time in a solve
    # of the timed configuration (complex-double and complex-float launches
    # together, as the timed solves run them)
    dom = max(kern, key=lambda c_: kern[c_]["ms"])
    achieved = kern[dom]["GBs"]
    counters = load_counters(os.path.join(ROOT, "profiles", f"{KERNEL_NAMES[dom]}_c3_10x4_counters.txt"))
    traffic = traffic_bytes = None
    if counters and counters.get("source_sha256") == kernel_source_hash(KERNEL_NAMES[dom]):
        traffic_bytes = counters["traffic_bytes_per_launch"]
        traffic = traffic_bytes / (kern[dom]["avg_us"] * 1e-6) / 1e9
    log(f"dominant kernel {KERNEL_NAMES[dom]} ({dom}): {achieved:.0f} GB/s algorithmic, "
        f"{kern[dom]['avg_us']:.1f} us per launch, {kern[dom]['ms']:.2f} ms per solve")

    # what a kernel moving the complex-float stencil's bytes costs at least
    floors = launch_floor(kern_c64["stencil"]["bytes_per_launch"]) if "stencil" in kern_c64 else {}
    log(f"launch floor {floors.get('launch_floor_us', 0):.2f} us, copy of the stencil's bytes "
        f"{floors.get('copy_same_bytes_us', 0):.2f} us")

    # ---- parity against the oracle's stored sample, when one exists for this setup
    err = err_full = None
    gpath = os.path.join(ROOT, "tests", "golden", f"{cfg.name}_mu{mu:g}.json")
    xstar_full = None
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        if g["c"] == c and m_used == cfg.m:
            xh = si.canonical_from_soa(x.cpu().numpy(), cfg.V)
            xs = xh[np.array(g["sample_index"])]
            ref = np.array(g["x_re"]) + 1j * np.array(g["x_im"])
            err = float(np.linalg.norm(xs - ref) / np.linalg.norm(ref))
            fpath = gpath[:-5] + "_x.npy"
            if os.path.exists(fpath):
                xstar_full = np.load(fpath)
                err_full = float(np.linalg.norm(xh - xstar_full) / np.linalg.norm(xstar_full))
    log(f"parity vs the oracle's x*: every component {err_full}, sampled {err}")

    # ---- CPU baseline: the oracle's restarted FOM-LR, a bounded number of cycles
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import dirac, krylov
        A = dirac.hw_csr(U, cfg.dims, cfg.kappa, mu, cfg.antiperiodic_t)
        nc = max(1, args.cpu_cycles)
        t0 = time.perf_counter()
        # deflation vectors of the right shape for the projection's cost
        # (timing only: the oracle's own eigenpairs at this size take hours)
        Rc = Lc = Fc = None
        if m_used > 0:
            Rc = np.linalg.qr(si.gaussian_source(cfg.n * m_used, 77).reshape(cfg.n, m_used))[0]
            Lc, Fc = Rc.copy(), np.eye(m_used, dtype=complex)
        krylov.restarted_fom_lr(lambda v: A @ v, b, sigma, omega, cfg.k, R=Rc, L=Lc, F=Fc,
                                tol_update=cfg.tol, max_cycles=nc)
        tc = (time.perf_counter() - t0) / nc
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": 1.0 / (tc * cycles[-1]), "unit": "solves/s", "cores": cores,
               "kind": "oracle",
               "sample": f"{nc} restart cycles (k={cfg.k}) of the oracle's restarted FOM "
                         f"(CSR matvec, numpy CGS2) on the same 10^4 input, "
                         f"{tc:.2f} s/cycle, scaled by the {cycles[-1]} cycles a solve takes"}
        log(f"cpu oracle: {tc:.2f} s per cycle on {cores} cores")

    methods = None if args.no_methods else methods_leg(op, bd, sigma, omega, cfg, R, Lv, F, xstar_full,
                                                         value)
    backward = None if args.no_backward else backward_leg()
    batched = None if args.no_batched else batched_leg(args)
    sweep = None if args.no_sweep else sweep_leg()

    out = {
        "metric": "sign(H_W)b solves/s at 10^4, mu=0.3, rel err 1e-8; stencil HBM GB/s",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128" if precision_run == "fp64" else "c64+f64", "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.dims[0]}^4 lattice, eps={cfg.eps}, mu={mu}, "
                               f"{2 * cfg.s} poles (c={c}), k={cfg.k}, deflation m={m_used}",
                   "n": cfg.n, "k": cfg.k, "npoles": 2 * cfg.s, "m": m_used,
                   "precision": precision_run, "cycles_per_solve": cycles[-1],
                   "cycles_complex_float": res.cycles_c64,
                   "matvecs_per_solve": res.matvecs, "sampled_rel_err_vs_oracle": err,
                   "rel_err_vs_oracle": err_full,
                   "fp64_true_residual_check": {"ok": res.resid_ok},
                   "eigensolve_setup": eig},
        "stencil": {"GBs": kern.get("stencil", {}).get("GBs"),
                    "avg_us": kern.get("stencil", {}).get("avg_us"),
                    "note": "algorithmic bytes (12 in + 36 link + 12 out complex per site) / time",
                    "complex_float": {"GBs": kern_c64.get("stencil", {}).get("GBs"),
                                      "avg_us": kern_c64.get("stencil", {}).get("avg_us"),
                                      **floors}},
        "roofline": {"bound": "hbm",
                     "kernel": f"{KERNEL_NAMES[dom]} ({dom}: largest summed time in a solve of this "
                               f"configuration; complex-double and complex-float launches)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_bytes_per_launch": traffic_bytes,
                     "bytes_per_launch": kern[dom]["bytes_per_launch"],
                     "avg_us": kern[dom]["avg_us"], "launches": kern[dom]["launches"],
                     "ms_per_solve": kern[dom]["ms"]},
        "kernels": kern,
        "kernels_complex_float": kern_c64,
        "bandwidth_sweep": sweep,
        "methods": methods,
        "backward": backward,
        "cpu_baseline": cpu,
        "batched": batched,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
