"""Benchmark: Stokes solves/s of the SIP-DG block-preconditioned solver on one
MI355X at a true relative residual of 1e-8, with the SIP viscous operator
throughput, solve latency, a roofline figure for the dominant kernel, the
oracle's accuracy checks and the FP64 CPU oracle as baseline.

Headline workload (one step): B = 16 distinct seeded variants of the
64 x 64 element, Q_4^2-Q_3 single-inclusion Stokes problem (problem 0 is the
centred disk of radius 0.25; the others move the centre within 0.1 and draw
the radius from [0.2, 0.3]; viscosity 1e4 inside, 1 outside, force (0, -1)
on elements fully inside, free slip on all sides), set up and solved in one
batched problem object with right-preconditioned FGMRES, the upper
block-triangular preconditioner and inner CG (rtol 1e-3) with the
hp-multilevel preconditioner.  The FP64 rounding floor of the true residual
lies above 1e-8 at this size, so the solves use extended iterative
refinement (double-FP64 iterate and residual): a solve counts only when it
reports status 0 and a residual of at most 1e-8.  Inputs are resident in HBM
before the timed region; setup is inside the step.

Other legs (each reported in the same JSON line): single-problem latency;
the 256 x 256 random-inclusion viscous solves at k = 3..6 with BF16 factors;
a batch of 512 random-field viscous solves with the batching and precision
levers isolated; a Poisson-arrival serving trace against the plain FP64
per-request path; the oracle's long-double residual and error of sampled
results; the oracle's own solver timed on the host cores.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--prec fp64|fp32|bf16] ...
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N, K, ETA_IN = 64, 4, 1e4
RTOL = 1e-8
PRECS = {"fp64": (0, 0), "fp32": (1, 1), "bf16": (1, 2)}  # (prec_apply, prec_smoother)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return model, n


def kernel_time_us(torch, fn, reps):
    """Average duration of one launch, HIP events on the current stream (the
    problem's stream: problems are created on torch's current stream)."""
    for _ in range(5):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    t1.synchronize()
    return t0.elapsed_time(t1) * 1e3 / reps


def ok(st):
    return st["status"] == 0 and st["rel_residual"] <= RTOL


# ---------------------------------------------------------------------------
# oracle work in background processes (host CPU, one thread each): it runs
# while the GPU legs continue and is collected at the end
# ---------------------------------------------------------------------------
def _one_thread():
    from threadpoolctl import threadpool_limits
    return threadpool_limits(1)


def _oracle_c2(args):
    """Long-double residual and error estimate of the headline's problem 0."""
    eta, f, uh, ul, ph, pl = args
    _one_thread()
    from oracle import refine as rf
    from oracle.mesh import Mesh
    t0 = time.perf_counter()
    eu, ep, res = rf.stokes_error_estimate(Mesh(N, N, K), eta, f, uh, ph, ul, pl, inner_rtol=1e-3)
    return {"problem": "headline problem 0 (centred disk r = 0.25)", "oracle_rel_residual_longdouble": res,
            "velocity_rel_error": eu, "pressure_rel_error": ep, "oracle_seconds": time.perf_counter() - t0,
            "method": "long-double residual of the FP64 pair; error = K^-1 r by the oracle's FGMRES/hp-MG "
                      "iteration to 1e-8 on the error equation"}


def _oracle_viscous(args):
    """Refined reference and long-double residual of one viscous request."""
    n, k, eta, f, uh, ul = args
    _one_thread()
    from oracle import refine as rf
    from oracle.mesh import Mesh
    m = Mesh(n, n, k)
    ref = rf.solve_viscous_ext(m, eta, f)
    err = float(np.linalg.norm((uh.astype(np.longdouble) + ul.astype(np.longdouble) - ref).astype(np.float64))
                / np.linalg.norm(ref.astype(np.float64)))
    return {"n": n, "k": k, "oracle_rel_residual_longdouble": rf.viscous_residual(m, eta, f, uh, ul),
            "velocity_rel_error": err}


def _oracle_stokes(args):
    n, k, eta, f, uh, ph = args
    _one_thread()
    from oracle import refine as rf
    from oracle.mesh import Mesh
    m = Mesh(n, n, k)
    u, p = rf.solve_stokes_ext(m, eta, f, method="lu")
    eu = float(np.linalg.norm(uh - u.astype(np.float64)) / np.linalg.norm(u.astype(np.float64)))
    ep = float(np.linalg.norm(ph - p.astype(np.float64)) / np.linalg.norm(p.astype(np.float64)))
    return {"n": n, "k": k, "oracle_rel_residual_longdouble": rf.stokes_residual(m, eta, f, uh, ph),
            "velocity_rel_error": eu, "pressure_rel_error": ep}


def _oracle_sample(seed, outer_its):
    """The oracle's FP64 Stokes solver (the paper's algorithm: FGMRES, block
    preconditioner, inner CG with the hp-multigrid cycle) on one headline
    variant, one thread: setup, then `outer_its` outer iterations.  Returns
    (setup s, seconds of the outer iterations, inner CG iterations in them)."""
    _one_thread()
    import oracle.assemble as asm
    from oracle.mesh import Mesh
    from oracle.multigrid import StokesSolver, fgmres
    from paper_1607_03777_amd import inputs as gen
    pr = gen.c2_variant(seed)
    m = Mesh(N, N, K)
    t0 = time.perf_counter()
    S = StokesSolver(m, pr.eta, inner_rtol=1e-3)
    F, G = asm.assemble_rhs(m, pr.eta, pr.f)
    t1 = time.perf_counter()
    fgmres(S.matvec, np.concatenate([F, G]), S.prec, 1e-30, restart=30, maxit=outer_its, project=S.project)
    return t1 - t0, time.perf_counter() - t1, int(sum(S.inner_its))


def cpu_baseline(pool_cores, gpu_inner, gpu_outer, sample_its=3):
    """The oracle timed on the host cores on a bounded sample of the headline
    workload, scaled to solves/s by the oracle's own cost per inner
    iteration: setup + (time per inner CG iteration incl. its share of the
    outer work) x (inner iterations one solve needs, the GPU's count for the
    same problem; the oracle's FP64 residual cannot itself reach 1e-8 here).
    Run on 1 core and, concurrently on distinct variants, on every core."""
    model, ncpu = host_cpu()
    one = _oracle_sample(0, sample_its)
    per_inner = one[1] / max(one[2], 1)
    v1 = 1.0 / (one[0] + per_inner * gpu_inner)
    with mp.get_context("spawn").Pool(pool_cores) as pool:
        t0 = time.perf_counter()
        res = pool.starmap(_oracle_sample, [(s, sample_its) for s in range(pool_cores)])
        wall = time.perf_counter() - t0
    per_all = [r[0] + r[1] / max(r[2], 1) * gpu_inner for r in res]
    v_all = sum(1.0 / t for t in per_all)
    return {
        "value": v_all, "unit": "solves/s", "cores": pool_cores, "kind": "oracle",
        "sample": (f"oracle FP64 Stokes solver (paper's algorithm, one thread per process): setup + "
                   f"{sample_its} outer FGMRES iterations on headline variants; seconds per inner CG iteration "
                   f"(incl. its share of the outer work) scaled to the {gpu_inner} inner iterations of one "
                   f"solve ({gpu_outer} outer) plus setup; {pool_cores} processes on distinct variants at once "
                   f"for the all-core figure"),
        "one_core_solves_per_s": v1, "setup_s": one[0], "s_per_inner_it": per_inner,
        "sample_wall_s": wall, "cpu_model": model, "host_cpus": ncpu,
    }


# ---------------------------------------------------------------------------
# legs
# ---------------------------------------------------------------------------
def c3_leg(sdg, ctx, torch, ks, prec):
    """256 x 256 random-inclusion viscous solves (16 disks, log10 viscosity
    U[-3, 3]), FP32 operator and BF16 block factors in the cycle (FP32 where
    the setup finds BF16 too coarse for the blocks), FGMRES with extended
    refinement, rtol 1e-8; one solve per k, setup included."""
    from paper_1607_03777_amd import inputs as gen
    out = []
    pa, ps = PRECS[prec]
    for k in ks:
        pr = gen.random_inclusions(256, k, seed=k)
        eta = torch.as_tensor(pr.eta, device="cuda")
        f = torch.as_tensor(pr.f.reshape(-1), device="cuda")
        u = torch.zeros(pr.nu, dtype=torch.float64, device="cuda")
        ul = torch.zeros_like(u)
        opts = sdg.make_options(rtol=RTOL, max_it=3000, restart=30, viscous_krylov=1, refine=1,
                                prec_apply=pa, prec_smoother=ps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = sdg.sdg_problem_create(ctx, sdg.make_mesh(256, 256, k), opts, eta, sdg.current_stream())
        factors = {0: "fp64", 1: "fp32", 2: "bf16"}[sdg.sdg_problem_smoother_precision(h)]
        rc, st = sdg.sdg_solve_viscous_ext_dev(h, f, None, u, ul)
        sdg.sdg_problem_destroy(h)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        log(f"[bench] C3 256x256 k={k}: {t:.2f} s status={st['status']} its={st['outer_its']} "
            f"resid={st['rel_residual']:.2e} factors {factors}")
        out.append({"k": k, "seconds": t, "velocity_dofs": pr.nu, "dof_per_s": pr.nu / t, "status": st["status"],
                    "smoother_factors": factors,
                    "converged": ok(st), "krylov_its": st["outer_its"], "rel_residual": st["rel_residual"],
                    "setup_ms": st["setup_ms"]})
    return {"workload": "viscous-256x256-16-random-inclusions-log10eta-U[-3,3]-rtol1e-8",
            "cycle_precision": prec, "krylov": "fgmres(30) + extended refinement", "solves": out}


# Table 4 of the paper (six inclusions, Delta eta = 1e6, GCR both loops,
# outer rtol 1e-6, inner 1e-3; one Ivy Bridge core, FP64): outer
# iterations, (average, maximum) inner iterations, seconds
TABLE4_1E6 = {(64, 1): (17, 3.4, 6, 0.98), (128, 1): (17, 3.6, 8, 4.92), (256, 1): (19, 4.1, 10, 25.43),
              (64, 2): (20, 6.7, 11, 9.50), (128, 2): (18, 6.8, 12, 35.47), (256, 2): (18, 6.9, 13, 145.18),
              (64, 3): (20, 8.9, 16, 36.28), (128, 3): (21, 8.7, 16, 151.37), (256, 3): (24, 9.0, 17, 715.33)}


def sinker_leg(sdg, ctx, torch, sizes, ks):
    """The six sedimenting inclusions of Section 8.3 (Delta eta = 1e6,
    density 1.2, g = 10, Neumann top, Navier elsewhere) with the paper's
    solver settings: GCR for the Stokes and the viscous solve, outer rtol
    1e-6 and inner 1e-3, FP64, h-coarsening down to 16 x 16 (one level less
    than for SolCx, as in the paper).  Iteration counts and time next to Table 4
    (another machine: context only)."""
    from paper_1607_03777_amd import inputs as gen
    rows = []
    for n in sizes:
        for k in ks:
            pr = gen.six_sinkers(n, k, eta2=1e6)
            eta = torch.as_tensor(pr.eta, device="cuda")
            f = torch.as_tensor(pr.f.reshape(-1), device="cuda")
            u = torch.zeros(pr.nu, dtype=torch.float64, device="cuda")
            p = torch.zeros(pr.np_, dtype=torch.float64, device="cuda")
            opts = sdg.make_options(rtol=1e-6, inner_rtol=1e-3, max_it=400, outer_krylov=1, viscous_krylov=2,
                                    coarsest_n=16)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = sdg.sdg_problem_create(ctx, sdg.make_mesh(n, n, k, pr.bc), opts, eta, sdg.current_stream())
            rc, st = sdg.sdg_solve_stokes_dev(h, f, None, u, p)
            sdg.sdg_problem_destroy(h)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            t4 = TABLE4_1E6.get((n, k))
            row = {"n": n, "k": k, "seconds": t, "status": st["status"], "outer_its": st["outer_its"],
                   "inner_avg": st["inner_its_total"] / max(st["outer_its"], 1), "inner_max": st["inner_its_max"],
                   "rel_residual": st["rel_residual"]}
            if t4:
                row["paper_table4"] = {"outer_its": t4[0], "inner_avg": t4[1], "inner_max": t4[2], "seconds": t4[3]}
            rows.append(row)
            log(f"[bench] sinkers {n}x{n} k={k}: {t:.2f} s outer {st['outer_its']} inner avg {row['inner_avg']:.1f} "
                f"max {st['inner_its_max']} status {st['status']}" + (f" (Table 4: {t4})" if t4 else ""))
    return {"workload": "six-sinkers-eta1e6-gcr-rtol1e-6-inner1e-3", "runs": rows}


def sweep_leg(sdg, ctx, torch, full):
    """Sections 8.1 and 8.2 with the paper's solver settings (FGMRES rtol
    1e-6 on the Stokes system, inner CG rtol 1e-3, a 16 x 16 coarsest
    h-level as its level counts imply, FP64 with the extended refinement,
    which contrast 1e8 needs to reach 1e-6, Section 8.3.1): the SolCx-shaped field
    (jump along x = 0.5) at k = 2, contrast 1 and 1e6, with the Q_1 coarse
    space on even meshes and the Q_0 one on odd meshes, and the 2 x 2
    checkerboard at k = 1..3, contrast 1e3, 1e6, 1e8, with this library's
    own smooth force; per solve the outer and inner iteration counts and
    the time with setup, next to Tables 2 and 3 (context, one core of the
    paper's machine)."""
    from paper_1607_03777_amd import inputs as gen
    tables = json.load(open(os.path.join(ROOT, "tests", "golden", "solcx_tables.json")))
    t2, t3 = tables["table2_solcx_k2"], tables["table3_checkerboard"]
    cases = [("solcx", 2, d, n) for d in (1.0, 1e6) for n in (64, 128, 256, 512)]
    cases += [("solcx-q0", 2, d, n) for d in (1.0, 1e6) for n in (65, 129, 257, 513)]
    cases += [("checker", k, d, n) for d in (1e3, 1e6, 1e8) for k in (1, 2, 3)
              for n in ((64, 128, 256, 512, 1024) if full else (64, 256))]
    if not full:
        cases += [("checker", 1, d, 1024) for d in (1e3, 1e6, 1e8)]
    rows = []
    for shape, k, d, n in cases:
        pr = (gen.checkerboard if shape == "checker" else gen.solcx_like)(n, k, d)
        eta = torch.as_tensor(pr.eta, device="cuda")
        f = torch.as_tensor(pr.f.reshape(-1), device="cuda")
        u = torch.zeros(pr.nu, dtype=torch.float64, device="cuda")
        p = torch.zeros(pr.np_, dtype=torch.float64, device="cuda")
        ul, pl = torch.zeros_like(u), torch.zeros_like(p)
        opts = sdg.make_options(rtol=1e-6, inner_rtol=1e-3, max_it=400, coarsest_n=16, refine=1,
                                coarse_space=1 if shape == "solcx-q0" else 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = sdg.sdg_problem_create(ctx, sdg.make_mesh(n, n, k), opts, eta, sdg.current_stream())
        rc, st = sdg.sdg_solve_stokes_ext_dev(h, f, None, u, ul, p, pl)
        sdg.sdg_problem_destroy(h)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        dkey = "1" if d == 1.0 else f"1e{int(round(np.log10(d)))}"
        if shape == "solcx":
            paper = t2.get(str(n), {}).get(dkey)
        elif shape == "solcx-q0":
            paper = tables["table2_solcx_k2_q0"]["A_hp(Q0)"].get(str(n), {}).get(dkey)
        else:
            paper = t3.get(dkey, {}).get(str(n), {}).get(str(k))
        row = {"shape": shape, "k": k, "deta": d, "n": n, "seconds": t, "status": st["status"],
               "outer_its": st["outer_its"], "inner_avg": st["inner_its_total"] / max(st["outer_its"], 1),
               "inner_max": st["inner_its_max"], "rel_residual": st["rel_residual"]}
        if paper:
            row["paper"] = {"outer_its": paper[0], "inner_avg": paper[1], "inner_max": paper[2], "seconds": paper[3]}
        rows.append(row)
        log(f"[bench] {shape} k={k} deta={d:g} {n}x{n}: {t:.2f} s outer {st['outer_its']} inner avg "
            f"{row['inner_avg']:.1f} max {st['inner_its_max']} status {st['status']}" + (f" (paper: {paper})" if paper else ""))
    return {"workload": "solcx-shaped-and-checkerboard-fgmres1e-6-inner1e-3-coarsest16", "runs": rows}


def batched_leg(sdg, ctx, torch, nreq, pool):
    """Batching form: nreq independent viscous solves, n in {16, 32, 64,
    128}, k in 2..5, log10 viscosity a Gaussian random field (correlation
    length 0.1, std 1.5), smooth random force, rtol 1e-8 with extended
    refinement (CG corrections).  Runs in this process that isolate the
    levers: the heterogeneous batch call (chunks of 64 requests) with the
    FP32 and the FP64 cycle; one request at a time (one-shot calls, no
    batching) with the FP32 cycle, and with the FP64 cycle (the plain FP64
    per-request path).  The same requests through the request server run
    in a child process (served_runs)."""
    from paper_1607_03777_amd import inputs as gen
    probs = [gen.grf_problem(seed) for seed in range(nreq)]
    dofs = sum(p.nu for p in probs)

    def batch_call(prec, chunk=64):
        """sdg_solve_viscous_batch over consecutive chunks of the requests
        (one call per chunk; within a call the shapes run their CG
        iterations in lockstep, one combined graph launch per iteration)."""
        pa, ps = PRECS[prec]
        opts = sdg.make_options(rtol=RTOL, max_it=3000, refine=1, prec_apply=pa, prec_smoother=ps)
        t0 = time.perf_counter()
        good, its, us = 0, [], [None] * nreq
        for i in range(0, nreq, chunk):
            part = probs[i:i + chunk]
            try:
                _, u, _, sts = sdg.sdg_solve_viscous_batch(ctx, [sdg.make_mesh(p.nx, p.ny, p.k) for p in part], opts,
                                                           [p.eta for p in part], [p.f for p in part])
            except sdg.SDGError as e:
                log(f"[bench] batch call failed: {e}")
                continue
            us[i:i + chunk] = u
            good += sum(ok(st) for st in sts)
            its += [st["outer_its"] for st in sts]
        return time.perf_counter() - t0, good, float(np.mean(its)) if its else None, us

    def alone(prec):
        pa, ps = PRECS[prec]
        opts = sdg.make_options(rtol=RTOL, max_it=3000, refine=1, prec_apply=pa, prec_smoother=ps)
        t0 = time.perf_counter()
        good = 0
        for p in probs:
            u = np.empty(p.nu)
            try:
                rc, st = sdg.sdg_solve_viscous(ctx, sdg.make_mesh(p.nx, p.ny, p.k), opts, p.eta,
                                               np.ascontiguousarray(p.f.reshape(-1)), None, u)
                good += ok(st)
            except sdg.SDGError:
                pass
        return time.perf_counter() - t0, good

    runs = {}
    checks = []
    for prec in ("fp32", "fp64"):
        t, good, its, us = batch_call(prec)
        runs[f"batch_call_{prec}_cycle"] = {"seconds": t, "solves_per_s": nreq / t, "dof_per_s": dofs / t,
                                            "converged": good, "mean_cg_its": its, "chunk": 64}
        log(f"[bench] batch call {prec}: {nreq} solves in {t:.2f} s, converged {good}")
        if prec == "fp32" and pool is not None:
            # oracle checks of sampled requests (smallest meshes: refined references)
            small = [i for i, p in enumerate(probs) if p.nx <= 32 and us[i] is not None][:3]
            checks = [pool.apply_async(_oracle_viscous, ((probs[i].nx, probs[i].k, probs[i].eta, probs[i].f,
                                                          us[i], np.zeros_like(us[i])),)) for i in small]
    t, good = alone("fp32")
    runs["per_request_fp32_cycle"] = {"seconds": t, "solves_per_s": nreq / t, "converged": good}
    log(f"[bench] per-request fp32: {t:.2f} s, converged {good}")
    t, good = alone("fp64")
    runs["per_request_fp64_plain"] = {"seconds": t, "solves_per_s": nreq / t, "converged": good}
    log(f"[bench] per-request fp64 (plain path): {t:.2f} s, converged {good}")
    plain = runs["per_request_fp64_plain"]["seconds"]
    return {"workload": f"{nreq}-grf-viscous-n16..128-k2..5-rtol1e-8", "runs": runs,
            "speedup_mixed_batched_vs_plain_fp64": plain / runs["batch_call_fp32_cycle"]["seconds"],
            "speedup_batching_alone_fp64": plain / runs["batch_call_fp64_cycle"]["seconds"],
            "speedup_precision_alone_per_request": plain / runs["per_request_fp32_cycle"]["seconds"],
            "oracle_sample_async": checks}


def served_runs(sdg, ctx, nreq, slots, max_batch):
    """The batched leg's requests submitted at once to the request server
    (requests of one shape share launches; each slot launches its own
    iterations), with the FP32 and with the FP64 cycle."""
    from paper_1607_03777_amd import inputs as gen
    probs = [gen.grf_problem(seed) for seed in range(nreq)]
    dofs = sum(p.nu for p in probs)
    runs = {}
    for prec in ("fp32", "fp64"):
        pa, ps = PRECS[prec]
        opts = sdg.make_options(rtol=RTOL, max_it=3000, refine=1, prec_apply=pa, prec_smoother=ps)
        srv = sdg.sdg_server_create(ctx, slots=slots, max_batch=max_batch)
        t0 = time.perf_counter()
        hs = [sdg.sdg_submit(srv, sdg.make_mesh(p.nx, p.ny, p.k), opts, sdg.VISCOUS, p.eta, p.f.reshape(-1))
              for p in probs]
        good, its, groups, failed = 0, [], [], 0
        for h, p in zip(hs, probs):
            try:
                rc, u, _, st, info = sdg.sdg_wait(h, p.nu)
                good += ok(st)
                its.append(st["outer_its"])
                groups.append(info["batch"])
            except sdg.SDGError as e:
                failed += 1
                if failed == 1:
                    log(f"[bench] served request failed: {e}")
            sdg.sdg_req_free(h)
        t = time.perf_counter() - t0
        ls = sdg.sdg_server_launch_stats(srv)
        sst = sdg.sdg_server_stats(srv)
        sdg.sdg_server_destroy(srv)
        runs[f"served_{prec}_cycle"] = {"seconds": t, "solves_per_s": nreq / t, "dof_per_s": dofs / t,
                                        "converged": good, "failed": failed,
                                        "mean_cg_its": float(np.mean(its)) if its else None,
                                        "mean_launch_group": float(np.mean(groups)) if groups else None,
                                        "slots": slots, "max_batch": max_batch, "launch_stats": ls,
                                        "peak_bytes": sst["peak_bytes"], "budget": sst["budget"]}
        log(f"[bench] served {prec}: {nreq} solves in {t:.2f} s, converged {good}, launches {ls}")
    return runs


def serving_leg(sdg, ctx, nreq, rate, prec, nmax, kmax, slots):
    """Request-server form: a Poisson trace of Stokes requests (n a multiple
    of 16 in [32, nmax], k in [2, kmax], 1-16 disks with contrast 10^U[2,6],
    rtol 1e-8 with extended refinement) replayed in real time into the server
    (mixed-precision cycle), and the same trace through the plain FP64
    per-request path (one-shot solves one after another, FP64 cycle, no
    batching).  Latency = completion - arrival.  Returns the two smallest
    requests' results for the oracle's checks."""
    from paper_1607_03777_amd import inputs as gen
    trace = gen.serving_trace(nreq=nreq, rate=rate, seed=0, nmin=32, nmax=nmax, kmin=2, kmax=kmax)
    probs = [gen.serving_problem(r) for r in trace]
    pa, ps = PRECS[prec]
    o_mix = sdg.make_options(rtol=RTOL, inner_rtol=1e-3, max_it=3000, refine=1, prec_apply=pa, prec_smoother=ps)
    o_64 = sdg.make_options(rtol=RTOL, inner_rtol=1e-3, max_it=3000, refine=1)

    def pct(x):
        return {"p50": float(np.percentile(x, 50)), "p99": float(np.percentile(x, 99))}

    srv = sdg.sdg_server_create(ctx, slots=slots, max_batch=16)
    t0 = time.perf_counter()
    hs = []
    for r, pr in zip(trace, probs):
        now = time.perf_counter() - t0
        if r["t"] > now:
            time.sleep(r["t"] - now)
        hs.append(sdg.sdg_submit(srv, sdg.make_mesh(pr.nx, pr.ny, pr.k), o_mix, sdg.STOKES, pr.eta,
                                 pr.f.reshape(-1)))
    lat, good, batches, res = [], 0, [], []
    for h, pr in zip(hs, probs):
        rc, u, p, st, info = sdg.sdg_wait(h, pr.nu, pr.np_)
        sdg.sdg_req_free(h)
        good += ok(st)
        lat.append(info["end_ms"] - info["submit_ms"])
        batches.append(info["batch"])
        res.append((pr, u, p))
    t_srv = time.perf_counter() - t0
    sst = sdg.sdg_server_stats(srv)
    ls = sdg.sdg_server_launch_stats(srv)
    sdg.sdg_server_destroy(srv)
    log(f"[bench] served {nreq} requests in {t_srv:.2f} s, p50 {np.percentile(lat, 50):.0f} ms "
        f"p99 {np.percentile(lat, 99):.0f} ms, converged {good}, launches {ls}")
    # refined references by a Stokes LU: only requests small enough for it
    small = [i for i in sorted(range(nreq), key=lambda i: probs[i].nu + probs[i].np_)
             if probs[i].nu + probs[i].np_ <= 60_000][:2]
    samples = [(res[i][0].nx, res[i][0].k, res[i][0].eta, res[i][0].f, res[i][1], res[i][2]) for i in small]
    t0 = time.perf_counter()
    lat64, good64 = [], 0
    for r, pr in zip(trace, probs):
        now = time.perf_counter() - t0
        if r["t"] > now:
            time.sleep(r["t"] - now)
        u = np.empty(pr.nu)
        p = np.empty(pr.np_)
        try:
            rc, st = sdg.sdg_solve_stokes(ctx, sdg.make_mesh(pr.nx, pr.ny, pr.k), o_64, pr.eta,
                                          np.ascontiguousarray(pr.f.reshape(-1)), None, u, p)
            good64 += ok(st)
        except sdg.SDGError:
            pass
        lat64.append((time.perf_counter() - t0 - r["t"]) * 1e3)
    t_64 = time.perf_counter() - t0
    log(f"[bench] FP64 per-request path: {t_64:.2f} s, p50 {np.percentile(lat64, 50):.0f} ms "
        f"p99 {np.percentile(lat64, 99):.0f} ms, converged {good64}")
    return {"workload": f"poisson-{rate:g}-per-s-{nreq}-stokes-requests-n32..{nmax}-k2..{kmax}-rtol1e-8",
            "server": {"requests_per_s": nreq / t_srv, "latency_ms": pct(lat), "converged": good,
                       "cycle_precision": prec, "slots": slots, "max_batch": 16,
                       "mean_launch_group": float(np.mean(batches)), "peak_bytes": sst["peak_bytes"],
                       "launch_stats": ls},
            "fp64_per_request": {"requests_per_s": nreq / t_64, "latency_ms": pct(lat64), "converged": good64},
            "speedup": t_64 / t_srv, "oracle_samples": samples}


def _child_leg(conn, which, kw):
    """Entry of the child process that runs a request-server leg on its own
    context (a failure there cannot take the benchmark line with it)."""
    try:
        import torch
        from paper_1607_03777_amd import sdg
        torch.cuda.set_device(0)
        ctx = sdg.sdg_create(0, 0)
        fn = served_runs if which == "served" else serving_leg
        res = fn(sdg, ctx, **kw)
        sdg.sdg_destroy(ctx)
        conn.send(("ok", res))
    except Exception as e:  # reported in the JSON line
        conn.send(("error", repr(e)))
    conn.close()


def isolated_leg(which, kw, timeout_s):
    """Runs a server leg in a spawned child process; returns its result, or
    {"failed": ...} when the child raised, died or ran past timeout_s."""
    mpc = mp.get_context("spawn")
    rd, wr = mpc.Pipe(duplex=False)
    proc = mpc.Process(target=_child_leg, args=(wr, which, kw))
    proc.start()
    wr.close()
    msg = None
    try:
        if rd.poll(timeout_s):
            msg = rd.recv()
    except (EOFError, OSError):
        msg = None
    proc.join(60)
    if proc.is_alive():
        proc.kill()
        proc.join()
    if msg is None:
        log(f"[bench] {which} leg: child process ended without a result (exit code {proc.exitcode})")
        return {"failed": f"child process ended without a result (exit code {proc.exitcode})"}
    if msg[0] != "ok":
        log(f"[bench] {which} leg failed: {msg[1]}")
        return {"failed": msg[1]}
    return msg[1]


def kernel_probe(sdg, ctx, torch, B, reps, phases="all"):
    """Only the kernels of the hot path, for rocprofv3 counter runs, in
    phases separated by marker copies (torch.neg over 4096 (i + 1) doubles
    before phase i > 0, so a per-dispatch counter file splits by grid size):
      0. at the headline's shape (batch B of 64 x 64, k = 4 variants, FP64):
         `reps` launches each of the SIP residual, the SIP apply and the
         block-Jacobi apply, then `reps` plain device copies of the
         residual's vector (known bytes) that calibrate the HBM counters;
      1. `reps` FP64 V-cycles at the same shape (p-transfers, h-level
         Chebyshev, restriction, prolongation, the LDS coarse tail);
      2. the FP32-factor smoother: `reps` block-Jacobi applies and V-cycles
         (FP32 apply and smoother);
      3. the same with BF16 factors;
      4. distinct blocks: B problems of 64 x 64, k = 4 with log-uniform
         random viscosity (no two elements share a block), `reps`
         block-Jacobi applies with FP64, FP32 and BF16 factors.
    `phases` = "all" or "0" (the first phase alone)."""
    from paper_1607_03777_amd import inputs as gen
    probs = [gen.c2_variant(s) for s in range(B)]
    nel, nb = N * N, 2 * (K + 1) ** 2
    eta = torch.as_tensor(np.concatenate([p.eta for p in probs]), device="cuda")
    mesh = sdg.make_mesh(N, N, K)
    h = sdg.sdg_problem_create_batch(ctx, mesh, sdg.make_options(), B, eta, sdg.current_stream())
    u = torch.randn(B * nel * nb, dtype=torch.float64, device="cuda")
    b = torch.randn_like(u)
    r = torch.empty_like(u)
    for _ in range(reps):
        sdg.sdg_residual_viscous(h, b, u, r)
    for _ in range(reps):
        sdg.sdg_apply_viscous(h, u, r)
    for _ in range(reps):
        sdg.sdg_apply_blockjacobi(h, u, r)
    for _ in range(reps):
        torch.neg(u, out=r)  # plain elementwise copy: reads and writes one vector
    torch.cuda.synchronize()
    var = sdg.sdg_get_tile(h, sdg.TILE_RESIDUAL, sdg.FP64)
    info = {"batch": B, "reps": reps, "vector_bytes": u.numel() * 8,
            "tile": sdg.sdg_tile_shape(K, var), "variant": var,
            "residual_bytes": B * nel * (3 * nb * 8 + 8),
            "apply_bytes": B * nel * (2 * nb * 8 + 8),
            "blockjacobi_bytes": B * nel * (2 * nb * 8 + 12)}

    def marker(i):
        torch.cuda.synchronize()
        m = torch.zeros(4096 * (i + 1), dtype=torch.float64, device="cuda")
        torch.neg(m, out=m)
        torch.cuda.synchronize()

    if phases == "all":
        marker(1)
        for _ in range(reps):
            sdg.sdg_vcycle(h, b, r)
        torch.cuda.synchronize()
        sdg.sdg_problem_destroy(h)
        h = None
        precs = {}
        for ph, prec in ((2, sdg.FP32), (3, sdg.BF16)):
            marker(ph)
            hp = sdg.sdg_problem_create_batch(ctx, mesh, sdg.make_options(prec_apply=sdg.FP32, prec_smoother=prec),
                                              B, eta, sdg.current_stream())
            precs[ph] = sdg.sdg_problem_smoother_precision(hp)
            for _ in range(reps):
                sdg.sdg_apply_blockjacobi(hp, u, r)
            for _ in range(reps):
                sdg.sdg_vcycle(hp, b, r)
            torch.cuda.synchronize()
            sdg.sdg_problem_destroy(hp)
        rng = np.random.default_rng(7)
        # contrast 10 (BF16 factors hold; the kernels' cost does not depend on it)
        eta_d = torch.as_tensor(10.0 ** rng.uniform(-0.5, 0.5, B * nel), device="cuda")
        marker(4)
        for prec in (sdg.FP64, sdg.FP32, sdg.BF16):
            hd = sdg.sdg_problem_create_batch(ctx, mesh, sdg.make_options(prec_apply=sdg.FP32 if prec else sdg.FP64,
                                                                          prec_smoother=prec),
                                              B, eta_d, sdg.current_stream())
            precs[f"distinct_{prec}"] = sdg.sdg_problem_smoother_precision(hd)
            for _ in range(reps):
                sdg.sdg_apply_blockjacobi(hd, u, r)
            torch.cuda.synchronize()
            sdg.sdg_problem_destroy(hd)
        info["smoother_precision"] = precs
        info["markers"] = {i: 4096 * (i + 1) for i in range(1, 5)}
    if h is not None:
        sdg.sdg_problem_destroy(h)
    print(json.dumps({"kernel_probe": info}), flush=True)


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    or None when the kernel's source changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "sip_and_smoother_k4_batch16_hbm_traffic.md")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
        k = rec["kernels"][kernel]
        src = open(os.path.join(ROOT, k["source"]), "rb").read()
    except (OSError, AttributeError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != k["source_sha256"]:
        return None
    return k["traffic_bytes"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--prec", choices=list(PRECS), default="fp64",
                    help="arithmetic of the headline's fine-level cycle (operator apply and block smoother); "
                         "Krylov, refinement residual and the coarse Q1 hierarchy stay FP64 or above")
    ap.add_argument("--latency-solves", type=int, default=5)
    ap.add_argument("--kernel-probe", type=int, default=0,
                    help="only launch the operator kernels this many times (counter runs)")
    ap.add_argument("--probe-phases", choices=["0", "all"], default="0",
                    help="kernel probe: the operator kernels alone (0) or every kernel class (all)")
    ap.add_argument("--c3", default="3,4,5,6", help="orders of the 256 x 256 leg ('' = skip)")
    ap.add_argument("--c3-prec", choices=list(PRECS), default="bf16")
    ap.add_argument("--batched", type=int, default=512, help="requests of the random-field leg (0 = skip)")
    ap.add_argument("--served", type=int, default=0,
                    help="also submit the random-field leg's requests to the request server (child process)")
    ap.add_argument("--serve-requests", type=int, default=24, help="requests of the serving leg (0 = skip)")
    ap.add_argument("--serve-nmax", type=int, default=128)
    ap.add_argument("--serve-kmax", type=int, default=6)
    ap.add_argument("--serve-prec", choices=list(PRECS), default="fp32")
    ap.add_argument("--serve-slots", type=int, default=4, help="request-server slots of the serving leg")
    ap.add_argument("--sinkers", default="64,128,256", help="mesh sizes of the six-inclusion leg ('' = skip)")
    ap.add_argument("--sweeps", choices=["default", "full", "none"], default="default",
                    help="SolCx-shaped and checkerboard sweeps (full: up to 1024^2 at every k)")
    ap.add_argument("--no-oracle", action="store_true", help="skip the oracle's accuracy checks")
    ap.add_argument("--no-trace", action="store_true",
                    help="skip the traced step after the timed region (per-kernel breakdown)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver library runs each problem on a single MI355X "
              "(sharding across GPUs is design-only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1607_03777_amd import inputs as gen
    from paper_1607_03777_amd import sdg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ctx = sdg.sdg_create(0, 0)
    if args.kernel_probe:
        kernel_probe(sdg, ctx, torch, args.batch, args.kernel_probe, args.probe_phases)
        sdg.sdg_destroy(ctx)
        return
    model, ncpu = host_cpu()
    pool_cores = max(1, min(ncpu, 16))
    pool = mp.get_context("spawn").Pool(min(4, pool_cores)) if not args.no_oracle else None

    B = args.batch
    probs = [gen.c2_variant(s) for s in range(B)]
    nel, nb = N * N, 2 * (K + 1) ** 2
    nu, npr = nel * nb, nel * K * K
    eta = torch.as_tensor(np.concatenate([p.eta for p in probs]), device="cuda")
    f = torch.as_tensor(np.concatenate([p.f.reshape(-1) for p in probs]), device="cuda")
    eta1, f1 = eta[:nel].contiguous(), f[:nu].contiguous()
    u = torch.zeros(B * nu, dtype=torch.float64, device="cuda")
    ul = torch.zeros_like(u)
    p = torch.zeros(B * npr, dtype=torch.float64, device="cuda")
    pl = torch.zeros_like(p)
    u1, ul1 = torch.zeros(nu, dtype=torch.float64, device="cuda"), torch.zeros(nu, dtype=torch.float64, device="cuda")
    p1, pl1 = torch.zeros(npr, dtype=torch.float64, device="cuda"), torch.zeros(npr, dtype=torch.float64, device="cuda")
    mesh = sdg.make_mesh(N, N, K)
    pa, ps = PRECS[args.prec]
    opts = sdg.make_options(rtol=RTOL, inner_rtol=1e-3, max_it=2000, prec_apply=pa, prec_smoother=ps, refine=1)
    stream = sdg.current_stream()

    def step():
        h = sdg.sdg_problem_create_batch(ctx, mesh, opts, B, eta, stream)
        rc, st = sdg.sdg_solve_stokes_ext_dev(h, f, None, u, ul, p, pl)
        sdg.sdg_problem_destroy(h)
        return st if isinstance(st, list) else [st]

    def solo():
        h = sdg.sdg_problem_create(ctx, mesh, opts, eta1, stream)
        rc, st = sdg.sdg_solve_stokes_ext_dev(h, f1, None, u1, ul1, p1, pl1)
        sdg.sdg_problem_destroy(h)
        return st

    tiles = {}
    h = sdg.sdg_problem_create_batch(ctx, mesh, opts, B, eta, stream)
    for kern, name in ((sdg.TILE_APPLY, "apply"), (sdg.TILE_RESIDUAL, "residual")):
        v = sdg.sdg_get_tile(h, kern, sdg.FP64)
        tiles[name] = {"variant": v, "shape": sdg.sdg_tile_shape(K, v),
                       "kernel": "sip_wave_kernel" if v == 0 else "sip_tile_kernel"}
    sdg.sdg_problem_destroy(h)
    log(f"[bench] batch {B} distinct variants, cycle {args.prec}: warmup {args.warmup} steps")
    for i in range(args.warmup):
        st = step()
        log(f"[bench] warmup step {i}: status={sorted(set(s['status'] for s in st))} outer={st[0]['outer_its']} "
            f"inner={st[0]['inner_its_total']} solve_ms={st[0]['solve_ms']:.1f}")
    torch.cuda.synchronize()
    stats = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        st = step()
        torch.cuda.synchronize()
        stats.append(st)
        log(f"[bench] step {i}: {(time.perf_counter() - ts) * 1e3:.1f} ms converged {sum(ok(s) for s in st)}/{B} "
            f"max resid {max(s['rel_residual'] for s in st):.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    converged = sum(ok(s) for st in stats for s in st)
    last = stats[-1]
    # oracle check of problem 0 (background, host CPU)
    c2_check = None
    if pool is not None:
        c2_check = pool.apply_async(_oracle_c2, ((probs[0].eta, probs[0].f, u[:nu].cpu().numpy(),
                                                  ul[:nu].cpu().numpy(), p[:npr].cpu().numpy(),
                                                  pl[:npr].cpu().numpy()),))
    traced = {}
    if not args.no_trace:
        sdg.sdg_trace_enable(ctx, 1)
        step()
        torch.cuda.synchronize()
        sdg.sdg_trace_enable(ctx, 0)
        for cls, name in sdg.TRACE_NAMES.items():
            n_, ms, by = sdg.sdg_trace_read(ctx, cls)
            traced[name] = {"launches": n_, "total_ms": ms, "us_per_launch": 1e3 * ms / max(n_, 1),
                            "bytes_per_launch": by / max(n_, 1),
                            "GB_per_s": (by / (ms * 1e-3) / 1e9) if ms > 0 and by > 0 else None}
            log(f"[bench] traced {name}: {n_} launches, {ms:.1f} ms total, {1e3 * ms / max(n_, 1):.2f} us/launch")
    lat = []
    for i in range(args.latency_solves):
        ts = time.perf_counter()
        s1 = solo()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        log(f"[bench] solo solve {i}: {lat[-1]:.1f} ms outer={s1['outer_its']} inner={s1['inner_its_total']} "
            f"status={s1['status']}")

    # roofline of the dominant kernel: the traced class with the largest
    # time in the traced step, launched back to back at the step's shape on
    # the problem's stream between two HIP events
    def kname(t, mode):
        if t["kernel"] == "sip_wave_kernel":
            return f"sip_wave_kernel<{K + 1},{mode},double>"
        return f"sip_tile_kernel<{K + 1},{mode},double,{t['shape'][0]},{t['shape'][1]}>"
    kernel_names = {"sip_apply": kname(tiles["apply"], "apply"),
                    "sip_residual": kname(tiles["residual"], "residual"),
                    "block_jacobi_smoother": f"bj_wave_kernel<{K + 1}>"}
    cand = {k: v for k, v in traced.items() if v["bytes_per_launch"] > 0}
    dom = max(cand, key=lambda k: cand[k]["total_ms"]) if cand else "sip_residual"
    o64 = sdg.make_options()
    h = sdg.sdg_problem_create_batch(ctx, mesh, o64, B, eta, stream)
    uu = torch.randn(B * nu, dtype=torch.float64, device="cuda")
    bb = torch.randn(B * nu, dtype=torch.float64, device="cuda")
    yy = torch.empty(B * nu, dtype=torch.float64, device="cuda")
    reps = max(args.kernel_reps, 20)
    t_app = kernel_time_us(torch, lambda: sdg.sdg_apply_viscous(h, uu, yy), reps)
    cases = {
        "sip_residual": ((lambda: sdg.sdg_residual_viscous(h, bb, uu, yy)), B * nel * (3 * nb * 8 + 8),
                         "r = b - A u: read b, u, eta; write r"),
        "sip_apply": ((lambda: sdg.sdg_apply_viscous(h, uu, yy)), B * nel * (2 * nb * 8 + 8),
                      "y = A u: read u, eta; write y"),
        "block_jacobi_smoother": ((lambda: sdg.sdg_apply_blockjacobi(h, uu, yy)), B * nel * (2 * nb * 8 + 12),
                                  "z = M^-1 r: read r, scale, permutation; write z (blocks cache-resident)"),
    }

    def roofline(name):
        fn, nbytes, what = cases[name]
        t = t_app if name == "sip_apply" else kernel_time_us(torch, fn, reps)
        gbs = nbytes / (t * 1e-6) / 1e9
        return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": recorded_traffic(kernel_names[name]),
                "kernel": kernel_names[name], "algorithmic_bytes": what, "bytes_per_launch": nbytes,
                "us_per_launch": t, "launches_timed": reps}
    # the FP64 kernels are the ones timed (the headline's cycle precision
    # decides which class dominates the step; the FP64 forms are the
    # reference forms of the roofline)
    dom64 = dom if dom in cases else "sip_residual"
    roof = roofline(dom64)
    other = "block_jacobi_smoother" if dom64 != "block_jacobi_smoother" else "sip_residual"
    roof_other = roofline(other)
    sdg.sdg_problem_destroy(h)
    log(f"[bench] dominant kernel {kernel_names[dom64]}: {roof['us_per_launch']:.2f} us/launch, "
        f"{roof['achieved']:.0f} GB/s; {kernel_names[other]} {roof_other['us_per_launch']:.2f} us/launch, "
        f"{roof_other['achieved']:.0f} GB/s; sip apply {t_app:.2f} us")

    st0 = last[0]
    out = {
        "metric": "SIP viscous DoF/s + Stokes solves/s at 1e-8 resid; p50/p99 solve latency",
        "value": converged / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else f"f64-krylov/{args.prec}-cycle",
        "data": "synthetic",
        "config": {"workload": "stokes-inclusion-64x64-Q4Q3-eta1e4-rtol1e-8-16-distinct-variants",
                   "nx": N, "ny": N, "k": K, "eta_contrast": ETA_IN, "rtol": RTOL, "inner_rtol": 1e-3,
                   "refinement": "extended (double-FP64 iterate and residual)", "velocity_dofs": nu,
                   "pressure_dofs": npr, "batch_per_step": B, "setup_in_step": True,
                   "cycle_precision": args.prec, "tile_shapes": tiles},
        "solves_converged": converged,
        "solves_attempted": B * args.steps,
        "latency_ms": ({"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                        "samples": len(lat), "kind": "single-problem setup+solve"} if lat else None),
        "batch_ms": ms_per_step,
        "viscous_dof_per_s": converged * nu / elapsed,
        "sip_apply_dof_per_s": B * nu / (t_app * 1e-6),
        "solver": {"outer_its": [s["outer_its"] for s in last], "inner_its_total": [s["inner_its_total"] for s in last],
                   "max_rel_residual": max(s["rel_residual"] for s in last),
                   "statuses": sorted(set(s["status"] for s in last)), "setup_ms": st0["setup_ms"],
                   "solve_ms": st0["solve_ms"]},
        "roofline": roof,
        "roofline_other_kernel": roof_other,
        "kernels_traced_step": traced,
    }
    if args.c3:
        out["c3"] = c3_leg(sdg, ctx, torch, [int(x) for x in args.c3.split(",")], args.c3_prec)
    if args.sinkers:
        out["sinkers"] = sinker_leg(sdg, ctx, torch, [int(x) for x in args.sinkers.split(",")], (1, 2, 3))
    if args.sweeps != "none":
        out["sweeps"] = sweep_leg(sdg, ctx, torch, args.sweeps == "full")
    if args.batched > 0:
        out["batched"] = batched_leg(sdg, ctx, torch, args.batched, pool)
    # the request-server legs run in child processes with contexts of their
    # own: this context's cached device memory is released first
    sdg.sdg_destroy(ctx)
    torch.cuda.empty_cache()
    if args.batched > 0 and args.served:
        out["batched"]["runs"].update(isolated_leg("served", {"nreq": args.batched, "slots": 4, "max_batch": 16}, 600))
    if args.serve_requests > 0:
        out["serving"] = isolated_leg("serving", {"nreq": args.serve_requests, "rate": 200.0, "prec": args.serve_prec,
                                                  "nmax": args.serve_nmax, "kmax": args.serve_kmax,
                                                  "slots": args.serve_slots}, 600)
        samples = out["serving"].pop("oracle_samples", [])
        out["serving"]["oracle_sample_async"] = ([pool.apply_async(_oracle_stokes, (smp,)) for smp in samples]
                                                 if pool is not None else [])
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline(pool_cores, st0["inner_its_total"], st0["outer_its"])
        log(f"[bench] cpu baseline {out['cpu_baseline']['value']:.3e} solves/s on {pool_cores} cores "
            f"({out['cpu_baseline']['one_core_solves_per_s']:.3e} on one)")
    if pool is not None:
        log("[bench] collecting oracle checks")
        out["oracle_check"] = {"headline": c2_check.get()}
        for leg in ("batched", "serving"):
            if leg in out:
                out["oracle_check"][leg] = [c.get() for c in out[leg].pop("oracle_sample_async")]
        pool.close()
        pool.join()
    else:
        for leg in ("batched", "serving"):
            if leg in out:
                out[leg].pop("oracle_sample_async", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
