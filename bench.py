"""Benchmark of the condensed-HDG hot path on one MI355X.

Workload (default): Cartesian 16^3 mesh of the unit cube with per-axis widths
perturbed by U[0.7, 1.3] and renormalised (seed 2), p = 7, lambda = 10,
tau = 1, forcing f ~ U[-1, 1] i.i.d. per node, homogeneous Dirichlet data.

One step = the whole hot path on that input, all data resident on the GPU:
right-hand side with Dirichlet lift, transform to the eigen-face basis,
Jacobi-preconditioned CG on the transformed condensed operator to a relative
residual of 1e-10 (one operator application per iteration), transform back,
and recovery of u in every element.

value = N_tr(free) x (operator applications in the step) / step time, i.e.
trace-DOF/s of the condensed operator as the CG drives it.  The JSON line also
carries the isolated apply rate, FP64 and mixed-precision time-to-1e-10, the
roofline of the dominant kernel (the fused CG apply) timed with HIP events on
its own stream, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _blas_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        return int(max([d.get("num_threads", 1) for d in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(prob, budget_s: float, cg_iters: int):
    """The oracle (dense element Schur complements, the definition of the
    operator) timed on the host cores, as three separate parts:

    * cfg1 (2^3, p = 4): setup (element systems and the assembled sparse K),
      apply (CSR matvec of K_ff) and solve (sparse direct), all measured;
    * the bench workload (16^3 perturbed, p = 7): setup of K_e for a random
      sample of elements (dense LU of the element system), the element-by-
      element apply y[Q_e] += K_e x[Q_e] over that sample with its K_e
      precomputed, both scaled to the whole mesh, and the Jacobi-CG solve
      estimated as (CG iterations of the GPU solve) x (apply + the vector
      work of one iteration, timed on full-length numpy vectors).

    `value` is the apply rate of the bench workload in trace-DOF/s."""
    import oracle
    import workloads as W
    threads = _blas_threads()
    rng = np.random.default_rng(0)
    # ---- cfg1: everything measured --------------------------------------
    tp = W.tiny()
    t0 = time.perf_counter()
    o1 = oracle.HdgOracle(tp.n, tp.widths, tp.p, tp.tau, tp.lam)
    K1 = o1.assemble_K()
    nf1 = o1.layout.n_free
    Kff1 = K1[:nf1, :nf1].tocsr()
    t_setup1 = time.perf_counter() - t0
    x1 = rng.uniform(-1, 1, nf1)
    ts = []
    for _ in range(11):
        t = time.perf_counter()
        _ = Kff1 @ x1
        ts.append(time.perf_counter() - t)
    t_apply1 = statistics.median(ts[1:])
    X = o1.volume_coords()
    T = o1.trace_coords()
    f1 = W.f_sin3(*X.T, 1.0)
    g1 = W.u_sin3(*T.T)
    ts = []
    for _ in range(4):
        t = time.perf_counter()
        _ = o1.solve(f1, g1)
        ts.append(time.perf_counter() - t)
    t_solve1 = statistics.median(ts[1:])
    # ---- bench workload: sampled setup and apply, estimated solve --------
    o = oracle.HdgOracle(prob.n, prob.widths, prob.p, prob.tau, prob.lam, cache_limit=1 << 20)
    ne, nf, na = o.layout.n_elem, o.layout.n_free, o.layout.n_all
    order = rng.permutation(ne)
    t0 = time.perf_counter()
    m = 0
    for e in order:
        o.K_e(int(e))
        o.tmap(int(e))
        m += 1
        if time.perf_counter() - t0 > 0.6 * budget_s and m >= 4:
            break
    t_setup = (time.perf_counter() - t0) / m * ne
    sample = [int(e) for e in order[:m]]
    x = rng.uniform(-1, 1, na)
    x[nf:] = 0.0
    y = np.zeros(na)
    ts = []
    for _ in range(6):
        t = time.perf_counter()
        for e in sample:
            mp = o.tmap(e)
            y[mp] += o.K_e(e) @ x[mp]
        ts.append(time.perf_counter() - t)
    t_apply = statistics.median(ts[1:]) / m * ne
    # vector work of one Jacobi-PCG iteration on N_tr(free)-long vectors
    v = [rng.uniform(-1, 1, nf) for _ in range(5)]
    xv, rv, pv, qv, dv = v
    ts = []
    for _ in range(6):
        t = time.perf_counter()
        al = 0.5 * float(rv @ rv) / float(pv @ qv)
        xv += al * pv
        rv -= al * qv
        zv = dv * rv
        be = float(rv @ zv) * 1e-3
        pv *= be
        pv += zv
        ts.append(time.perf_counter() - t)
    t_vec = statistics.median(ts[1:])
    t_solve = cg_iters * (t_apply + t_vec)
    return {"value": nf / t_apply, "unit": "trace-DOF/s", "cores": threads, "kind": "oracle",
            "sample": (f"apply: y[Q_e] += K_e x[Q_e] over {m} of {ne} elements of the 16^3 p=7 "
                       f"workload with K_e precomputed, scaled to the mesh; setup (dense K_e) "
                       f"timed on the same sample"),
            "bench_workload_s": {"setup": round(t_setup, 1), "apply": round(t_apply, 4),
                                 "solve_est": round(t_solve, 1)},
            "cfg1_s": {"setup": round(t_setup1, 4), "apply": t_apply1, "solve": round(t_solve1, 4)}}


# Algorithmic bytes of one FP64 Jacobi-PCG iteration per free trace DOF: the
# operator reads its input and writes its output once (16 B) and the CG's
# vector work takes about nine more passes over 8-byte vectors (72 B).  FP32
# halves it.  The implementation's own per-DOF traffic is listed beside it.
ALG_CG_BYTES = 88
IMPL_CG_BYTES = {"one kernel": 104, "two kernels": 104,
                 # pencil: element launch reads z, p_old, x and writes p, x and
                 # the face contributions (two per face normal to x1 or x2,
                 # one summed per face normal to x3); the update reads z,
                 # D^-1 and those contributions and writes z
                 "pencil": 91}
# committed rocprofv3 FETCH_SIZE / WRITE_SIZE summaries, one per workload
TRAFFIC_PROFILES = {
    "perturbed16_p7": os.path.join(ROOT, "profiles", "cg_iteration_perturbed16_p7_hbm_counters.md"),
    "uniform32_p8": os.path.join(ROOT, "profiles", "cg_iteration_uniform32_p8_hbm_counters.md"),
    "uniform32_p12": os.path.join(ROOT, "profiles", "cg_iteration_uniform32_p12_hbm_counters.md"),
}
KERNEL_SOURCES = ("paper_2007_11891_amd/csrc/elem_unit.hpp", "paper_2007_11891_amd/csrc/elem_kernels.hip",
                  "paper_2007_11891_amd/csrc/vec_kernels.hip", "paper_2007_11891_amd/csrc/pencil_cg.hip",
                  "paper_2007_11891_amd/csrc/pencil_unit.hpp", "paper_2007_11891_amd/csrc/cg_state.hpp",
                  "paper_2007_11891_amd/csrc/device_common.hpp")


def kernel_source_hash() -> str:
    """sha256 over the sources of the CG kernels."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernels):
    """HBM bytes per CG iteration (the sum over `kernels`, one launch each)
    from the committed counter summary of `workload` (FETCH_SIZE +
    WRITE_SIZE, each scaled by what it reads for a plain copy), or None when
    the summary is missing, does not cover a kernel, or the kernel sources
    changed since the counters were taken."""
    try:
        with open(TRAFFIC_PROFILES[workload]) as fh:
            text = fh.read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        rec = json.loads(block)
    except (KeyError, OSError, IndexError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    tot = 0
    for k in kernels:
        entry = rec.get("kernels", {}).get(k)
        if entry is None:
            return None
        tot += entry["traffic_bytes"]
    return tot


def cg_kernel_names(c, fp32: bool = False):
    """Names (as rocprofv3 prints them) of the kernels of one CG iteration in
    the context's CG form and tile shape."""
    t = c.tile_shape()
    typ = "float" if fp32 else "double"
    np_, epu = c.p + 1, t["elems_per_unit"]
    if t["cg_variant"] == 0 and not fp32:
        return [f"elem_apply_kernel<{typ}, {np_}, {epu}, 2, 0>"]
    if t["cg_variant"] == 2:   # the FP32 inner CG follows the FP64 pencil form
        return [f"pencil_apply_kernel<{typ}, {np_}, {epu}>", f"pencil_update_kernel<{typ}>"]
    units = -(-c.n_elem // epu)
    upb = -(-units // min(units, 2048))
    return [f"elem_apply_kernel<{typ}, {np_}, {epu}, 1, {1 if upb > 1 else 0}>",
            f"cg_update_kernel<{typ}>"]


def cg_iteration_roofline(c, W, torch, dev, fp32: bool = False, reps: int = 50,
                          workload: str | None = None):
    """One CG iteration in the CG form and tile shape the solve runs (FP32:
    the form of the mixed-precision inner CG, the pencil form when the FP64
    CG runs it, else the two-kernel form), mean time per
    iteration over back-to-back launches (HIP events on the context stream),
    as an HBM roofline entry at the algorithmic 88 B per free DOF (44 in
    FP32), with the implementation's own bytes and the counted traffic."""
    import paper_2007_11891_amd as pkg
    nf = c.sizes.n_free
    cgv = c.tile_shape()["cg_variant"]
    if fp32:
        form, which = (("pencil", pkg.TIME_PENCIL_ITER_F32) if cgv == 2 else
                       ("two kernels", pkg.TIME_CG2_ITER_F32))
    elif cgv == 0:
        form, which = "one kernel", pkg.TIME_CG1_ITER_F64
    elif cgv == 2:
        form, which = "pencil", pkg.TIME_PENCIL_ITER_F64
    else:
        form, which = "two kernels", pkg.TIME_CG2_ITER_F64
    x = torch.as_tensor(W.random_trace(nf, 7), device=dev)
    if fp32:
        x = x.float()
    # one discarded timing first: after the host-side set-up above the first
    # timed launches of a context ran ~6 % slow (366-370 against 345-351 us at
    # 32^3, p = 12, in four contexts of one process), the later ones steady
    c.time_kernel(which, x, max(10, reps // 2))
    t = c.time_kernel(which, x, reps)
    scale = 0.5 if fp32 else 1.0
    alg = ALG_CG_BYTES * scale * nf
    impl = IMPL_CG_BYTES[form] * scale * nf
    ach = alg / (t * 1e-3) / 1e9
    kernels = cg_kernel_names(c, fp32)
    traffic = None if (fp32 or workload is None) else measured_traffic(workload, kernels)
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernels": kernels, "cg_form": form, "avg_us": round(t * 1e3, 3),
            "alg_bytes": int(alg), "impl_bytes": int(impl),
            "impl_GBs": round(impl / (t * 1e-3) / 1e9, 1)}


def bench_mixed(pkg, W, torch, dev, reps: int = 3):
    """FP32-inner / FP64-outer vs plain FP64, time to relative residual 1e-10
    on the 32^3 unit-cube mesh, p in {4, 8, 12}, lambda in {1e-2, 1, 1e2},
    u = sin(2 pi x) cos(3 pi y) exp(z) (Dirichlet data and forcing from it);
    each result with its nodal error against that u and its distance to the
    FP64 solution."""
    rows = []
    for p in (4, 8, 12):
        for lam in (1e-2, 1.0, 1e2):
            prob = W.mixed(p, lam)
            c = pkg.HdgContext(prob.n, prob.widths, prob.p, prob.tau, lam)
            c.autotune(reps=10)
            vx, tx = c.coords()
            vx, tx = vx.cpu().numpy(), tx.cpu().numpy()
            f = torch.as_tensor(W.f_mixed(*vx.T, lam), device=dev)
            g = torch.as_tensor(W.u_mixed(*tx.T), device=dev)
            u_ex = torch.as_tensor(W.u_mixed(*vx.T), device=dev)
            nf = c.sizes.n_free
            res = {}
            for name, o in (("fp64", pkg.default_opts(rtol=1e-10)),
                            ("mixed", pkg.default_opts(rtol=1e-10, mixed=1))):
                ts = []
                for _ in range(reps + 1):
                    tr = g.clone()
                    tr[:nf] = 0
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    _, uv, info = c.solve_forcing(f, tr, opts=o)
                    torch.cuda.synchronize()
                    ts.append(1e3 * (time.perf_counter() - t))
                res[name] = (statistics.median(ts[1:]), info, tr, uv)
            t64, i64, tr64, uv64 = res["fp64"]
            tmx, imx, trmx, uvmx = res["mixed"]
            nrm = float(torch.linalg.norm(u_ex))
            row = {"p": p, "lambda": lam, "n_trace_free": nf,
                   "fp64_ms": round(t64, 3), "mixed_ms": round(tmx, 3),
                   "speedup": round(t64 / tmx, 3),
                   "fp64_iters": i64["iters"], "mixed_inner_iters": imx["iters"],
                   "mixed_outer": imx["outer_iters"],
                   "fp64_rel_res": i64["rel_res"], "mixed_rel_res": imx["rel_res"],
                   "mixed_vs_fp64_trace_rel_diff":
                       float(torch.linalg.norm(trmx - tr64) / torch.linalg.norm(tr64)),
                   "fp64_nodal_error": float(torch.linalg.norm(uv64 - u_ex)) / nrm,
                   "mixed_nodal_error": float(torch.linalg.norm(uvmx - u_ex)) / nrm,
                   "fp64_iteration": cg_iteration_roofline(c, W, torch, dev, False),
                   "fp32_iteration": cg_iteration_roofline(c, W, torch, dev, True)}
            log(f"[bench] mixed 32^3 p={p} lam={lam:g}: fp64 {t64:.2f} ms ({i64['iters']} it), "
                f"mixed {tmx:.2f} ms ({imx['iters']} inner, {imx['outer_iters']} outer), "
                f"x{t64 / tmx:.2f}")
            rows.append(row)
            c.close()
            del f, g, u_ex, res
            torch.cuda.empty_cache()
    sp = [r["speedup"] for r in rows]
    return {"workload": "32^3 unit cube, u = sin(2 pi x) cos(3 pi y) exp(z); time to rel. residual "
                        "1e-10 (FP32 inner CG to 1e-2 per step + FP64 defect correction vs FP64 CG)",
            "geomean_speedup": round(float(np.exp(np.mean(np.log(sp)))), 3), "cases": rows}


# The paper's four HDG solvers (section "Summary of solution method"):
# precond code of hdg_solve_opts, timing id of one iteration, algorithmic
# bytes per free DOF and iteration.  HDG-trans: the CG form in use (one-kernel
# 104 B, two-kernel 104 B).  Nodal solvers: p and z in, p and p^ out (32 B),
# element apply (24 B), q = (M S x M S)(qa + qb) with p.q (32 B) and the
# update with z = P^-1 r (unprec 56, diag 64, block 64 B: x, p, r, q, 1/y in,
# x, r, z out).
PAPER_SOLVERS = (("trans", 1, None, 104), ("unprec", 0, 13, 144), ("diag", 2, 14, 152),
                 ("block", 3, 15, 152))


def bench_paper_case(pkg, W, torch, dev, reps: int = 3):
    """The paper's solver test: (0, 2 pi)^3, 8^3 elements, Poisson, tau_e = 25,
    five-factor k = 5 manufactured solution, stop at 1e-10, for the paper's
    four HDG solvers: iterations, time per solve (RHS + CG + recovery), time
    per degree of freedom n_e (p + 1)^3 (the paper's unit) and the time and
    roofline fraction of one iteration."""
    rows = []
    for p in (2, 4, 6, 8, 10, 12, 14, 16):
        pr = W.paper_case(p)
        c = pkg.HdgContext(pr.n, pr.widths, pr.p, pr.tau, pr.lam)
        c.autotune(reps=10)
        vx, tx = c.coords()
        vx, tx = vx.cpu().numpy(), tx.cpu().numpy()
        f = torch.as_tensor(W.f_paper(*vx.T, 0.0), device=dev)
        g = torch.as_tensor(W.u_paper(*tx.T), device=dev)
        u_ex = torch.as_tensor(W.u_paper(*vx.T), device=dev)
        nf = c.sizes.n_free
        ndof = pr.n_elem * (p + 1) ** 3
        row = {"p": p, "n_trace_free": nf}
        xr = torch.as_tensor(W.random_trace(nf, 3), device=dev)
        for name, pc, tid, bpd in PAPER_SOLVERS:
            o = pkg.default_opts(rtol=1e-10, precond=pc)
            ts = []
            for _ in range(reps + 1):
                tr = g.clone()
                tr[:nf] = 0
                torch.cuda.synchronize()
                t = time.perf_counter()
                _, uv, info = c.solve_forcing(f, tr, opts=o)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t)
            t = statistics.median(ts[1:])
            if tid is None:
                tid = 9 if c.tile_shape()["cg_variant"] == 0 else 2
            t_it = c.time_kernel(tid, xr, 50)
            gbs = bpd * nf / (t_it * 1e-3) / 1e9
            row[name] = {"iters": info["iters"], "solve_ms": round(1e3 * t, 3),
                         "us_per_dof": 1e6 * t / ndof,
                         "ns_per_dof_per_iter": 1e9 * t / ndof / max(info["iters"], 1),
                         "iteration_us": round(t_it * 1e3, 3), "iteration_bytes": bpd * nf,
                         "iteration_frac": round(gbs / HBM_PEAK_GBS, 4),
                         "max_error": float(torch.max(torch.abs(uv - u_ex)))}
        # the paper's protocol: start from the flux of a pseudo-random volume
        # field (exact values on the boundary), stop when the initial
        # residual has dropped by 1e-10
        u0 = torch.as_tensor(W.paper_initial_volume(vx, 11), device=dev)
        o = pkg.default_opts(rtol=1e-10, guess=2)
        ts = []
        for _ in range(reps + 1):
            tr = g.clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            c.hybridize(u0, tr, out=tr[:nf])
            _, uv, info = c.solve_forcing(f, tr, opts=o)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        row["trans_paper_protocol"] = {"iters": info["iters"],
                                       "solve_ms": round(1e3 * statistics.median(ts[1:]), 3),
                                       "max_error": float(torch.max(torch.abs(uv - u_ex)))}
        rows.append(row)
        log(f"[bench] paper case p={p}: " + ", ".join(
            f"{nm} {row[nm]['iters']} it {row[nm]['solve_ms']:.2f} ms" for nm, *_ in PAPER_SOLVERS)
            + f"; trans {row['trans']['us_per_dof']:.4f} us/DOF, max error "
            f"{row['trans']['max_error']:.2e}; paper protocol (random start, 1e-10 of r_0) "
            f"{row['trans_paper_protocol']['iters']} it")
        c.close()
    return {"workload": "(0, 2 pi)^3, 8^3 uniform elements, lambda = 0, tau_e = 25, u = five-factor k = 5 "
                        "solution (paper's test case), rel. residual 1e-10; solvers HDG-trans "
                        "(eigen basis, Jacobi), HDG-unprec, HDG-diag, HDG-block (nodal basis)",
            "paper_reference": "about 1 us per degree of freedom for the transformed HDG solver and "
                               "about 2.5 us for HDG-block on one Xeon E5-2680 v3 core (p >= 8); "
                               "about 100 iterations for HDG-block and HDG-trans",
            "cases": rows}


def bench_tau_sweep(pkg, W, torch, dev):
    """The paper's penalty study: its solver test case with tau_e in
    {1, 25, 625} (section "Robustness against increases in the penalty
    parameter"): iterations of HDG-trans to 1e-10 and maximum nodal error."""
    rows = []
    for tau_e in (1.0, 25.0, 625.0):
        for p in (2, 4, 8, 12, 16):
            pr = W.paper_case(p, tau_e=tau_e)
            c = pkg.HdgContext(pr.n, pr.widths, pr.p, pr.tau, pr.lam)
            vx, tx = c.coords()
            vx, tx = vx.cpu().numpy(), tx.cpu().numpy()
            f = torch.as_tensor(W.f_paper(*vx.T, 0.0), device=dev)
            g = torch.as_tensor(W.u_paper(*tx.T), device=dev)
            u_ex = torch.as_tensor(W.u_paper(*vx.T), device=dev)
            nf = c.sizes.n_free
            tr = g.clone()
            tr[:nf] = 0
            _, uv, info = c.solve_forcing(f, tr, opts=pkg.default_opts(rtol=1e-10))
            rows.append({"tau_e": tau_e, "p": p, "iters": info["iters"],
                         "max_error": float(torch.max(torch.abs(uv - u_ex)))})
            c.close()
        log("[bench] tau_e " + f"{tau_e:g}: " + ", ".join(
            f"p={r['p']} {r['iters']} it err {r['max_error']:.2e}" for r in rows if r["tau_e"] == tau_e))
    return {"workload": "paper's test case (8^3 elements, lambda = 0, k = 5) with tau_e in {1, 25, 625}, "
                        "HDG-trans to 1e-10",
            "cases": rows}


def bench_neumann(pkg, W, torch, dev, reps: int = 3):
    """Neumann sides, the exact mass matrix and initial-guess solves on the
    headline mesh (16^3 perturbed, p = 7, f ~ U[-1, 1], seed 2): the sides
    normal to x1 and x3 Neumann (g_N = 0.5), the others Dirichlet (g_D = 0);
    and all sides Dirichlet with the exact mass.  One-kernel CG iteration and
    whole solve against the lumped all-Dirichlet mesh; then the solve at
    lambda = 11 from zero and from the hybridized volume solution at
    lambda = 10 (a time step's worth of change)."""
    mask = 0b110011
    prob = W.perturbed(n=16, p=7, lam=10.0, seed=2)
    f = torch.as_tensor(prob.f_values, device=dev)
    rows = {}
    for name, m, em in (("dirichlet", 0, False), ("neumann", mask, False),
                        ("exact_mass", 0, True)):
        c = pkg.HdgContext(prob.n, prob.widths, prob.p, prob.tau, prob.lam, neumann=m,
                           exact_mass=em)
        c.autotune(reps=20)
        nf = c.sizes.n_free
        x = torch.as_tensor(W.random_trace(nf, 1), device=dev)
        c.time_kernel(9, x, 50)            # discarded: see cg_iteration_roofline
        t_it = c.time_kernel(9, x, 200)
        bc = c.zeros_trace()
        bc[nf:] = 0.5 if m else 0.0
        o = pkg.default_opts(rtol=1e-10)
        c.solve_forcing(f, bc.clone(), opts=o)
        walls = []
        for _ in range(reps):
            tr = bc.clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, uv, info = c.solve_forcing(f, tr, opts=o)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t)
        rows[name] = {"n_free": nf, "one_kernel_iteration_us": round(t_it * 1e3, 3),
                      "iters": info["iters"], "solve_ms": round(statistics.median(walls) * 1e3, 3)}
        if name == "neumann":
            ctx_n, bc_n, u_prev = c, bc, uv
        else:
            c.close()
    # initial guess: lambda 10 -> 11
    lam2 = prob.lam * 1.1
    c2 = pkg.HdgContext(prob.n, prob.widths, prob.p, prob.tau, lam2, neumann=mask)
    c2.autotune(reps=20)
    nf = c2.sizes.n_free
    nv = c2.sizes.n_vol
    res = {}
    for name, guess in (("zero", 0), ("hybridized", 1)):
        o = pkg.default_opts(rtol=1e-10, guess=guess)
        walls = []
        for _ in range(reps + 1):
            tr = bc_n.clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            if guess:
                c2.hybridize(u_prev, bc_n, out=tr[:nf])
            _, _, info = c2.solve_forcing(f, tr, want_volume=False, opts=o)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t)
        res[name] = {"iters": info["iters"], "rel_res": info["rel_res"],
                     "ms": round(statistics.median(walls[1:]) * 1e3, 3)}
    out_free = torch.empty(nf, dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c2.hybridize(u_prev, bc_n, out=out_free)
    e0.record()
    for _ in range(50):
        c2.hybridize(u_prev, bc_n, out=out_free)
    e1.record()
    torch.cuda.synchronize()
    t_h = e0.elapsed_time(e1) / 50
    hyb_bytes = 8 * nv + 16 * nf + 24 * nf     # volume read, two face slots, their sum
    res["hybridize_us"] = round(t_h * 1e3, 3)
    res["hybridize_GBs"] = round(hyb_bytes / (t_h * 1e-3) / 1e9, 1)
    log(f"[bench] neumann: {rows}; guess {res}")
    ctx_n.close()
    c2.close()
    return {"workload": "16^3 perturbed, p = 7, f~U[-1,1]; sides x1 and x3 Neumann (g_N = 0.5), "
                        "x2 Dirichlet (g_D = 0); all Dirichlet with the exact mass; CG to 1e-10",
            "boundary": rows,
            "initial_guess": {"case": "lambda 10 -> 11 everywhere; guess = hybridized volume "
                                      "solution at lambda 10", **res}}


def bench_batched(pkg, W, torch, dev, reps: int = 3):
    """256 independent unit-cube problems (n_a ~ U{4..12}, p ~ U{2..10},
    lambda log-uniform in [1e-2, 1e2], f ~ N(0,1), seed 4) in one persistent
    launch: RHS + CG to 1e-10 + recovery, replayed from one HIP graph."""
    probs = W.batched()
    b = pkg.HdgBatch([pr.n for pr in probs], [pr.p for pr in probs],
                     [float(pr.lam[0]) for pr in probs], tau=1.0)
    tiles = b.autotune(iters=10, reps=2)
    f = torch.as_tensor(np.concatenate([pr.f_values for pr in probs]), device=dev)
    tr = torch.empty(b.total_free, dtype=torch.float64, device=dev)
    uv = torch.empty(b.total_vol, dtype=torch.float64, device=dev)
    o = pkg.default_opts(rtol=1e-10, maxit=20000)
    b.solve_forcing(f, tr, uv, opts=o)            # capture + warm-up
    walls, gpus, res = [], [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, res, gms = b.solve_forcing(f, tr, uv, opts=o)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t)
        gpus.append(gms)
    wall = statistics.median(walls)
    iters = np.array([r["iters"] for r in res])
    dof_iters = float(np.sum(b.n_free * iters))
    t1 = b.time_cg(1, reps=3)
    t21 = b.time_cg(21, reps=3)
    t_it = (t21 - t1) / 20.0                     # ms per CG iteration, all problems active
    # algorithmic 88 B per free DOF and iteration; the two-phase form moves
    # 96 B (apply phase 56 B: read z, p_old, x, write p, x, qa, qb; update
    # phase 40 B: read z, qa, qb, D^-1, write z), the one-phase form 104 B,
    # the pencil form 91 B (as the single-problem pencil form)
    bytes_it = ALG_CG_BYTES * b.total_free
    impl_it = {0: 96, 1: 104, 2: IMPL_CG_BYTES["pencil"]}[b.form()] * b.total_free
    ach = bytes_it / (t_it * 1e-3) / 1e9
    log(f"[bench] batched: {len(probs)} problems, {b.total_free} free DOFs, wall {wall*1e3:.1f} ms, "
        f"max iters {iters.max()}, CG iteration {t_it*1e3:.1f} us, tiles {tiles}")
    out = {"workload": "256 unit-cube problems, n_a~U{4..12}, p~U{2..10}, lambda~logU[1e-2,1e2], "
                       "f~N(0,1), seed 4; RHS + CG to 1e-10 + recovery in one graph",
           "problems": len(probs), "total_free": int(b.total_free),
           "trace_dof_iters_per_s": dof_iters / wall, "trace_dof_per_s": b.total_free / wall,
           "wall_ms": round(wall * 1e3, 3), "gpu_ms": round(statistics.median(gpus), 3),
           "iters_min": int(iters.min()), "iters_max": int(iters.max()),
           "iters_sum": int(iters.sum()), "tiles_by_p": tiles,
           "cg_form": {0: "two phases per iteration", 1: "one element pass per iteration",
                       2: "two phases on the pencil march"}[b.form()],
           "cg_iteration_us": round(t_it * 1e3, 2),
           "roofline": {"kernel": "batch_cg_kernel (persistent, one CG iteration of every problem)",
                        "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "alg_bytes": bytes_it, "impl_bytes": impl_it,
                        "impl_GBs": round(impl_it / (t_it * 1e-3) / 1e9, 1)}}
    b.close()
    return out


def bench_adjoint(pkg, W, torch, dev, reps: int = 3):
    """Adjoint gradient on 24^3, p = 6, log-normal lambda field (seed 5):
    forward solve, then dJ/dlambda and dJ/df by the adjoint solve."""
    prob = W.adjoint()
    c = pkg.HdgContext(prob.n, prob.widths, prob.p, prob.tau, prob.lam)
    c.autotune(reps=20)
    vx, _ = c.coords()
    vx = vx.cpu().numpy()
    lam_nodes = np.repeat(prob.lam, (prob.p + 1) ** 3)
    f = torch.as_tensor(W.lambda_forcing_sin3(*vx.T, lam_nodes), device=dev)
    ustar = torch.as_tensor(W.target_with_noise(W.u_sin3(*vx.T), prob.extra["noise_seed"]),
                            device=dev)
    w = pkg.tables(prob.p, prob.tau)["w"]
    wk = np.kron(w, np.kron(w, w))
    h = prob.widths
    Md = np.concatenate([h[0][i] * h[1][j] * h[2][k] / 8.0 * wk
                         for k in range(prob.n[2]) for j in range(prob.n[1]) for i in range(prob.n[0])])
    Md = torch.as_tensor(Md, device=dev)
    o = pkg.default_opts(rtol=1e-10, maxit=20000)
    tr = c.zeros_trace()
    fw, ad, info, ainfo = [], [], None, None
    for _ in range(reps + 1):
        tr.zero_()
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, uv, info = c.solve_forcing(f, tr, opts=o)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dl, df, ainfo = c.adjoint(f, tr, Md * (uv - ustar), opts=o)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fw.append(t1 - t)
        ad.append(t2 - t1)
    fw_ms = 1e3 * statistics.median(fw[1:])
    ad_ms = 1e3 * statistics.median(ad[1:])
    nf = c.sizes.n_free
    log(f"[bench] adjoint 24^3 p6: forward {fw_ms:.2f} ms ({info['iters']} it), "
        f"adjoint {ad_ms:.2f} ms ({ainfo['iters']} it)")
    out = {"workload": "24^3 uniform, p=6, lambda log-normal(0,1) per element, seed 5; "
                       "J = 1/2 |u - u*|_M^2, u* = sin sin sin + 1% noise",
           "n_lambda": int(prob.n_elem), "n_trace_free": int(nf),
           "forward_ms": round(fw_ms, 3), "adjoint_ms": round(ad_ms, 3),
           "forward_iters": info["iters"], "adjoint_iters": ainfo["iters"],
           "gradients_per_s": 1e3 / ad_ms,
           "adjoint_trace_dof_per_s": nf * ainfo["iters"] / (ad_ms * 1e-3),
           "cg_iteration": cg_iteration_roofline(c, W, torch, dev, False)}
    c.close()
    return out


def hbm_size_iteration(pkg, W, torch, dev, p: int):
    """The FP64 CG iteration on the 32^3 uniform unit-cube mesh at degree p
    (lambda = 1): vectors of 66 MB (p = 8) and 137 MB (p = 12), past the
    256 MB Infinity Cache once a few of them are live, so that the bytes come
    from HBM."""
    prob = W.mixed(p, 1.0)
    c = pkg.HdgContext(prob.n, prob.widths, prob.p, prob.tau, 1.0)
    c.autotune(reps=10)
    r = cg_iteration_roofline(c, W, torch, dev, False, reps=50, workload=f"uniform32_p{p}")
    r["workload"] = f"32^3 uniform, p={p}, lambda=1, N_tr(free)={c.sizes.n_free}"
    c.close()
    torch.cuda.empty_cache()
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16)
    ap.add_argument("--p", type=int, default=7)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the isolated kernel timings (for counter collection)")
    ap.add_argument("--reps", type=int, default=200)
    ap.add_argument("--tile", type=int, default=0,
                    help="--kernels-only: tile variant (no autotuning, so that every counter pass "
                         "times the same launches)")
    ap.add_argument("--ks", type=int, default=0,
                    help="--kernels-only: pencil segment length (0: whole columns)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched persistent CG timed over 1 and 21 iterations, form 0, "
                         "tile variant 0 (for counter collection)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-paper-case", action="store_true")
    ap.add_argument("--no-neumann", action="store_true")
    ap.add_argument("--no-hbm-size", action="store_true")
    ap.add_argument("--detail", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                    help="file for the full record (every section); the last stdout line is the "
                         "compact headline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"path is a design note, not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    import paper_2007_11891_amd as pkg

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    if args.kernels_only:
        # isolated kernels of one workload, for counter collection (rocprofv3
        # --pmc): the bench mesh by default, --n 32 --p 12 for the uniform
        # 32^3 mesh
        if args.n == 16 and args.p == 7:
            prob = W.perturbed(n=16, p=7, lam=10.0, seed=2)
        else:
            prob = W.mixed(args.p, 1.0) if args.n == 32 else W.perturbed(n=args.n, p=args.p,
                                                                          lam=10.0, seed=2)
        ctx = pkg.HdgContext(prob.n, prob.widths, prob.p, prob.tau, float(np.ravel(prob.lam)[0]))
        ctx.set_tile(args.tile)
        ctx.set_cg_segment(args.ks)
        tile = ctx.tile_shape()
        log(f"[bench] kernels-only n={prob.n} p={prob.p}: tile variant {args.tile}, pencil segment "
            f"{args.ks or 'whole columns'}, CG form {tile['cg_variant']}, kernels "
            f"{cg_kernel_names(ctx)}")
        nf = ctx.sizes.n_free
        x64 = torch.as_tensor(W.random_trace(nf, 1), device=dev)
        y64 = torch.empty_like(x64)
        chosen = {0: pkg.TIME_CG1_ITER_F64, 1: pkg.TIME_CG2_ITER_F64,
                  2: pkg.TIME_PENCIL_ITER_F64}[tile["cg_variant"]]
        x32 = x64.float()
        for which, name in ((pkg.TIME_APPLY_F64, "apply64"), (pkg.TIME_CG2_APPLY_F64, "cg_apply64"),
                            (pkg.TIME_CG2_UPDATE_F64, "cg_update64"),
                            (pkg.TIME_CG1_ITER_F64, "cg_onekernel64"),
                            (pkg.TIME_PENCIL_ITER_F64, "cg_pencil64"), (pkg.TIME_COPY_F64, "copy64"),
                            (chosen, "chosen CG form, again"),
                            (pkg.TIME_CG2_ITER_F32, "cg_iter32 (two kernels)"),
                            (pkg.TIME_PENCIL_ITER_F32, "cg_pencil32")):
            x = x32 if which in (pkg.TIME_CG2_ITER_F32, pkg.TIME_PENCIL_ITER_F32) else x64
            ms = ctx.time_kernel(which, x, args.reps,
                                 y=y64 if which in (pkg.TIME_COPY_F64, pkg.TIME_APPLY_F64) else None)
            log(f"[bench] {name} {ms * 1e3:.3f} us")
        # plain copy of 256 MiB (larger than L2 and the infinity cache): the
        # reference dispatch for scaling HBM byte counters
        big = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        big2 = torch.empty_like(big)
        for _ in range(3):
            big2.copy_(big)
        torch.cuda.synchronize()
        ctx.close()
        return

    if args.batch_only:
        # the persistent batched CG alone, for counter collection: the
        # dispatches are the warm-up and 3 timed launches of 1 iteration, then
        # of 21 iterations (bytes per iteration = difference / 20)
        probs = W.batched()
        b = pkg.HdgBatch([pr.n for pr in probs], [pr.p for pr in probs],
                         [float(pr.lam[0]) for pr in probs], tau=1.0)
        b.set_form(0)
        b.set_tile(0, 0)
        t1 = b.time_cg(1, reps=3)
        t21 = b.time_cg(21, reps=3)
        log(f"[bench] batch-only: {b.total_free} free DOFs, one CG iteration of every problem "
            f"{(t21 - t1) / 20 * 1e3:.1f} us")
        b.close()
        return

    prob = W.perturbed(n=args.n, p=args.p, lam=10.0, seed=2)
    log(f"[bench] workload perturbed n={prob.n} p={prob.p} lam=10 tau=1")
    ctx = pkg.HdgContext(prob.n, prob.widths, prob.p, prob.tau, prob.lam)
    nf, na, nv = ctx.sizes.n_free, ctx.sizes.n_all, ctx.sizes.n_vol
    f = torch.as_tensor(prob.f_values, device=dev)
    trace = torch.zeros(na, dtype=torch.float64, device=dev)
    u_vol = torch.empty(nv, dtype=torch.float64, device=dev)
    opts = pkg.default_opts(rtol=1e-10)
    variant, tile_times = ctx.autotune(reps=50)      # tile shape, chosen before timing
    tile = ctx.tile_shape()
    log(f"[bench] tile variant {variant} ({tile['elems_per_unit']} elements / "
        f"{tile['threads_per_unit']} threads per unit), CG form {tile['cg_variant']}, "
        f"times {[round(t * 1e3, 2) for t in tile_times]} us")

    def step():
        trace.zero_()
        return ctx.solve_forcing(f, trace, u_vol=u_vol, opts=opts)

    for _ in range(args.warmup):
        _, _, info = step()
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, info = step()
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    iters = infos[-1]["iters"]
    applies = statistics.mean(i["iters"] for i in infos)
    value = nf * applies / (elapsed / args.steps)
    log(f"[bench] step {ms_per_step:.3f} ms, CG iters {iters}, rel_res {infos[-1]['rel_res']:.2e}")

    # ---- the dominant kernel: one CG iteration (HIP events, context stream) --
    roof = cg_iteration_roofline(ctx, W, torch, dev, False, reps=args.reps, workload="perturbed16_p7"
                                 if (args.n, args.p) == (16, 7) else None)
    log(f"[bench] CG iteration {roof['avg_us']:.2f} us ({roof['cg_form']}), "
        f"{roof['achieved']:.0f} GB/s at 88 B/DOF, frac {roof['frac']:.3f}; "
        f"{roof['impl_GBs']:.0f} GB/s at the implementation's bytes")
    # ---- isolated kernels ---------------------------------------------------
    x64 = torch.as_tensor(W.random_trace(nf, 1), device=dev)
    x32 = x64.float()
    y64 = torch.empty_like(x64)
    y32 = torch.empty_like(x32)
    reps = args.reps
    t_apply64 = ctx.time_kernel(pkg.TIME_APPLY_F64, x64, reps, y=y64)
    t_apply32 = ctx.time_kernel(pkg.TIME_APPLY_F32, x32, reps, y=y32)
    t_elem64 = ctx.time_kernel(pkg.TIME_ELEM_APPLY_F64, x64, reps)
    t_cg_apply = ctx.time_kernel(pkg.TIME_CG2_APPLY_F64, x64, reps)
    t_cg_update = ctx.time_kernel(pkg.TIME_CG2_UPDATE_F64, x64, reps)
    t_cg_iter = ctx.time_kernel(pkg.TIME_CG2_ITER_F64, x64, reps)
    t_cg_iter32 = ctx.time_kernel(pkg.TIME_CG2_ITER_F32, x32, reps)
    t_one = ctx.time_kernel(pkg.TIME_CG1_ITER_F64, x64, reps)
    t_one32 = ctx.time_kernel(pkg.TIME_CG1_ITER_F32, x32, reps)
    log(f"[bench] apply64 {t_apply64*1e3:.2f} us (element kernel {t_elem64*1e3:.2f}) "
        f"apply32 {t_apply32*1e3:.2f} us cg_apply {t_cg_apply*1e3:.2f} us "
        f"cg_update {t_cg_update*1e3:.2f} us cg_iter {t_cg_iter*1e3:.2f} us "
        f"cg_iter32 {t_cg_iter32*1e3:.2f} us one-kernel {t_one*1e3:.2f} us")
    # the paper's nodal-basis solvers at the same size: one CG iteration each
    nodal_iteration = {}
    for name, pc, tid, bpd in PAPER_SOLVERS[1:]:
        t_it = ctx.time_kernel(tid, x64, reps)
        gbs = bpd * nf / (t_it * 1e-3) / 1e9
        nodal_iteration[name] = {"avg_us": round(t_it * 1e3, 3), "impl_bytes": bpd * nf,
                                 "impl_GBs": round(gbs, 1),
                                 "impl_frac": round(gbs / HBM_PEAK_GBS, 4)}
    log("[bench] nodal-basis CG iteration: " + ", ".join(
        f"{k} {v['avg_us']:.2f} us ({v['impl_frac']:.3f})" for k, v in nodal_iteration.items()))
    # hdg_apply in the eigen basis as it runs (element kernel + sum of the two
    # face contributions); algorithmic 16 B per free DOF (8 in FP32)
    apply_bytes = 16 * nf
    apply_only = {"trace_dof_per_s_fp64": nf / (t_apply64 * 1e-3),
                  "trace_dof_per_s_fp32": nf / (t_apply32 * 1e-3),
                  "avg_us_fp64": round(t_apply64 * 1e3, 3),
                  "avg_us_fp32": round(t_apply32 * 1e3, 3),
                  "element_kernel_us_fp64": round(t_elem64 * 1e3, 3),
                  "alg_GBs_fp64": round(apply_bytes / (t_apply64 * 1e-3) / 1e9, 1),
                  "frac_fp64": round(apply_bytes / (t_apply64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "alg_GBs_fp32": round(apply_bytes / 2 / (t_apply32 * 1e-3) / 1e9, 1)}

    hbm = {}
    if not args.no_hbm_size:
        for p in (8, 12):
            hbm[f"p{p}"] = hbm_size_iteration(pkg, W, torch, dev, p)
            log(f"[bench] 32^3 p={p} CG iteration {hbm[f'p{p}']['avg_us']:.1f} us "
                f"({hbm[f'p{p}']['cg_form']}), frac {hbm[f'p{p}']['frac']:.3f} at 88 B/DOF")

    mixed = None if args.no_mixed else bench_mixed(pkg, W, torch, dev)
    batched = None if args.no_batch else bench_batched(pkg, W, torch, dev)
    adjoint = None if args.no_adjoint else bench_adjoint(pkg, W, torch, dev)
    paper_case = None if args.no_paper_case else bench_paper_case(pkg, W, torch, dev)
    tau_sweep = None if args.no_paper_case else bench_tau_sweep(pkg, W, torch, dev)
    neumann = None if args.no_neumann else bench_neumann(pkg, W, torch, dev)

    cpu = None
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(prob, args.cpu_budget, iters)
        log(f"[bench] cpu baseline {cpu['value']:.3e} trace-DOF/s on {cpu['cores']} threads")

    config = {"workload": f"perturbed Cartesian {prob.n[0]}x{prob.n[1]}x{prob.n[2]}, p={prob.p}, "
                          f"lambda=10, tau=1, f~U[-1,1], g_D=0; step = RHS + Jacobi-PCG to 1e-10 + "
                          f"recovery",
              "n_elem": prob.n_elem, "p": prob.p, "n_trace_free": nf, "n_trace_all": na,
              "n_vol": nv, "cg_iters": iters, "rel_res": infos[-1]["rel_res"]}
    head = {
        "metric": "trace-DOF/s of condensed HDG apply; time-to-1e-10 CG, mixed vs FP64",
        "value": value, "unit": "trace-DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": config,
    }
    detail = dict(head)
    detail.update({
        "roofline": roof, "hbm_size_iteration": hbm, "cpu_baseline": cpu,
        "apply_only": apply_only, "nodal_solver_iteration": nodal_iteration,
        "cg_iteration_us": {"two_kernel_fp64": round(t_cg_iter * 1e3, 3),
                            "two_kernel_fp32": round(t_cg_iter32 * 1e3, 3),
                            "fused_apply_fp64": round(t_cg_apply * 1e3, 3),
                            "update_fp64": round(t_cg_update * 1e3, 3),
                            "one_kernel_fp64": round(t_one * 1e3, 3),
                            "one_kernel_fp32": round(t_one32 * 1e3, 3)},
        "tile": {"variant": variant, "elems_per_unit": tile["elems_per_unit"],
                 "threads_per_unit": tile["threads_per_unit"], "cg_variant": tile["cg_variant"],
                 "autotune_cg_iter_us": [round(t * 1e3, 3) for t in tile_times]},
        "mixed_precision": mixed, "batched": batched, "adjoint": adjoint,
        "paper_case": paper_case, "tau_sweep": tau_sweep, "neumann": neumann,
    })
    try:
        os.makedirs(os.path.dirname(args.detail), exist_ok=True)
        with open(args.detail, "w") as fh:
            json.dump(detail, fh, indent=1)
        log(f"[bench] full record: {args.detail}")
    except OSError as exc:
        log(f"[bench] could not write {args.detail}: {exc}")
    # sections on stderr, one line each, for logs that keep only the streams
    for k in ("apply_only", "mixed_precision", "batched", "adjoint", "neumann"):
        if detail.get(k) is not None:
            log(f"[bench] {k}: " + json.dumps(detail[k], separators=(",", ":"))[:4000])

    # ---- compact headline: the last stdout line ----------------------------
    keep = ("bound", "achieved", "peak", "unit", "frac", "traffic")
    roofline = {k: roof[k] for k in keep}
    roofline.update({"kernel": " + ".join(roof["kernels"]), "avg_launch_us": roof["avg_us"],
                     "alg_bytes_per_dof": ALG_CG_BYTES,
                     "impl_bytes_per_dof": IMPL_CG_BYTES[roof["cg_form"]],
                     "impl_GBs": roof["impl_GBs"]})
    if hbm:
        roofline["hbm_size"] = {k: {"workload": v["workload"], "avg_us": v["avg_us"],
                                    "achieved": v["achieved"], "frac": v["frac"],
                                    "traffic": v["traffic"], "cg_form": v["cg_form"]}
                                for k, v in hbm.items()}
    extras = {"apply_only_fp64": {"trace_dof_per_s": round(apply_only["trace_dof_per_s_fp64"], 1),
                                  "frac_16B": apply_only["frac_fp64"]}}
    if mixed:
        extras["mixed_geomean_speedup"] = mixed["geomean_speedup"]
    if batched:
        extras["batched"] = {"trace_dof_iters_per_s": round(batched["trace_dof_iters_per_s"], 1),
                             "frac": batched["roofline"]["frac"]}
    if adjoint:
        extras["adjoint_gradients_per_s"] = round(adjoint["gradients_per_s"], 2)
    head["config"] = {"workload": config["workload"], "n_trace_free": nf, "cg_iters": iters}
    head["roofline"] = roofline
    head["cpu_baseline"] = None if cpu is None else {
        k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample", "bench_workload_s", "cfg1_s")}
    head["extras"] = extras
    line = json.dumps(head, separators=(",", ":"))
    print(line, flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
