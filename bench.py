"""Benchmark of the HHG P1 multigrid hot path on one MI355X.

Headline workload (N = 1): Poisson -Laplace u = f with P1 elements on the
jittered 64-face annulus r in [0.55, 1], refinement level 10 (1025 points per
macro-edge, 33,538,048 interior unknowns), constant coefficient, uniform
[-1, 1] right-hand side (seed 1), homogeneous Dirichlet boundary, FP64,
V(3,3) cycles with the staged multicolour Gauss-Seidel smoother to a relative
residual of 1e-8, exact (stored-inverse) solve on coarse level 3 (1,920
unknowns; the paper fixes no coarse level, and level 3 is the finest whose
inverse stays small).

A step is one solve from u = 0 to 1e-8 (every V-cycle level: smoothing,
residual, restriction, coarse CG, prolongation, ghost-copy refresh, norms).
value = whole-job smoother throughput: finest-level interior unknowns times
the finest-level sweeps the solve performs, divided by the solve's wall time.
The roofline entry is the finest-level face smoother, timed live with HIP
events on the launch stream.

Reported beside it (untimed by the step contract, each from its own runs):
  * the mixed-precision refinement solve of the same problem;
  * the variable-coefficient problem on the same mesh at level 10, k = exp(g)
    with g a Gaussian random field: the learned face smoother trained on the
    GPU at level 7 on 256 coefficient fields (weights kept by the convergence
    factor on 2 validation fields), its acceptance against
    Gauss-Seidel on 8 held-out fields, convergence factors, time to 1e-8 of
    plain FP64, mixed precision with Gauss-Seidel and with the network, and
    the live-timed kernels of that path;
  * plain FP64 against mixed precision on the 128-face annulus at level 11
    (268,369,920 unknowns) with the final difference of the two solutions.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "smoother GDoF/s, % HBM peak; time-to-1e-8 rel. residual plain vs MP/learned"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def host_cores():
    """Cores this process may run on (the host's share on the GPU machine)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def log(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def face_interior_dofs(F, n):
    return F * (n - 2) * (n - 3) // 2


def _oracle_solve_job(level, rtol, nu, reps):
    """One worker: build the oracle hierarchy (untimed) and time `reps` plain
    solves from u = 0.  Returns (interior unknowns, cycles, seconds)."""
    import numpy as np

    import hhg_inputs as hi
    from oracle.mesh import MacroMesh
    from oracle.mg import Hierarchy
    vxy, tri = hi.mesh_by_name("annulus64")
    H = Hierarchy(MacroMesh(vxy, tri), level, 2)
    lv = H.levels[level]
    f = hi.uniform_rhs(lv.n_all, 1)
    iters = 0
    t0 = time.perf_counter()
    for _ in range(reps):
        u, hist = H.solve(np.zeros(lv.n_all), f, rtol, nu, nu)
        iters += len(hist) - 1
    return lv.interior_count(), iters, time.perf_counter() - t0


def _pool_job(a):
    return _oracle_solve_job(*a)


def cpu_baseline(level, rtol, nu, all_level, workers):
    """The oracle's plain solve, timed on the host: (i) one process on one
    core at `level`; (ii) `workers` processes at once, one per host core,
    each solving the `all_level` problem, whole-host throughput (the oracle
    itself is single-threaded scipy; it is run as it stands)."""
    import multiprocessing as mp
    n_int, iters, dt = _oracle_solve_job(level, rtol, nu, 2)
    one = {"value": n_int * 2 * nu * iters / dt / 1e9, "unit": "GDoF/s", "cores": 1,
           "kind": "oracle",
           "sample": "2 oracle plain solves to %g on the same 64-face annulus at level %d "
                     "(%d interior unknowns, %d V(%d,%d) cycles in all, %.1f s; scipy sparse "
                     "kernels, single-threaded)" % (rtol, level, n_int, iters, nu, nu, dt)}
    ctx = mp.get_context("spawn")
    # one thread per worker process: the workers share the host's cores
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})
    try:
        with ctx.Pool(workers) as pool:
            res = pool.map(_pool_job, [(all_level, rtol, nu, 1)] * workers)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    work = sum(r[0] * 2 * nu * r[1] for r in res)
    span = max(r[2] for r in res)
    return {"value": work / span / 1e9, "unit": "GDoF/s", "cores": workers, "kind": "oracle",
            "sample": "%d concurrent oracle processes (one per host core), each one plain solve "
                      "to %g on the 64-face annulus at level %d (%d interior unknowns, %d cycles); "
                      "throughput = all smoothed unknowns / slowest process (%.1f s)"
                      % (workers, rtol, all_level, res[0][0], res[0][1], span),
            "one_core": one}


def kernel_section(P, hi, torch, g, L, reps=10):
    """Per-call GDoF/s and fraction of the HBM peak at the finest level, for
    the calls the V-cycle is made of, in FP64 and FP32.  Each figure brackets
    a whole library call with events on torch's stream (the stream the call
    launches on), so a sweep includes its edge/vertex stages.  Bytes are the
    algorithmic ones per interior unknown: every field read once and written
    once (residual + restriction: read u, f, write a quarter-size f_c;
    prolongation + add: read a quarter-size u_c, read and write u)."""
    n_int, n_all = g.n_dofs(L)
    _, n_all_c = g.n_dofs(L - 1)
    stream = torch.cuda.current_stream()

    def ms_of(fn):
        for _ in range(2):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / reps

    out = {"level": L, "interior_dofs": n_int, "reps": reps}
    lap, gs = P.HHG_OP_LAPLACE, P.HHG_SMOOTH_GS
    for dt, name, w in ((P.HHG_F64, "f64", 8), (P.HHG_F32, "f32", 4)):
        x = g.from_canonical(L, hi.uniform_vector(n_all, 21), dt)
        f = g.from_canonical(L, hi.uniform_rhs(n_all, 1), dt)
        r = g.field(L, dt)
        fc = g.field(L - 1, dt)
        uc = g.from_canonical(L - 1, hi.uniform_vector(n_all_c, 22), dt)
        norm = torch.zeros(1, dtype=torch.float64, device="cuda")
        calls = [
            ("apply", 2.0, lambda: P.hhg_apply(g.h, L, lap, dt, x, r, stream=stream)),
            # two sweeps per call: the result lands back in x, so no copy
            ("gs_sweep", 3.0, lambda: P.hhg_smooth(g.h, L, lap, gs, dt, x, f, 2, 0, stream=stream)),
            ("residual_restrict", 2.25, lambda: (P.hhg_residual(g.h, L, lap, dt, x, f, r, stream=stream),
                                                 P.hhg_restrict(g.h, L, dt, r, fc, stream=stream))),
            ("prolong_add", 2.25, lambda: P.hhg_prolong_add(g.h, L, dt, uc, x, stream=stream)),
            ("residual_norm", 2.0, lambda: P.hhg_residual(g.h, L, lap, dt, x, f, None, norm, stream=stream)),
        ]
        res = {}
        for key, words, fn in calls:
            ms = ms_of(fn) / (2 if key == "gs_sweep" else 1)
            nbytes = words * w * n_int
            res[key] = {"ms": round(ms, 4), "gdofs": round(n_int / (ms * 1e-3) / 1e9, 2),
                        "alg_bytes_per_dof": words * w,
                        "hbm_frac": round(nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
        out[name] = res
        del x, f, r, fc, uc
    # a plain device copy of the same size as one field: the practical ceiling
    src = torch.empty(n_all, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    ms = ms_of(lambda: dst.copy_(src))
    out["stream_copy"] = {"bytes": 2 * src.numel() * 8, "ms": round(ms, 4),
                          "gbs": round(2 * src.numel() * 8 / (ms * 1e-3) / 1e9, 1),
                          "hbm_frac": round(2 * src.numel() * 8 / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)}
    del src, dst
    return out


def timed_solve(P, g, u, f, mode, op, rtol, nu, max_iters=100):
    import torch
    u.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st, hist = P.hhg_solve(g.h, u, f, mode=mode, op=op, rtol=rtol, nu1=nu, nu2=nu,
                               max_iters=max_iters)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, rc, st, hist


def face_sweep_rate(P, g, L, launches_ms, bytes_per_dof):
    """GB/s and GDoF/s of the finest face smoother from hhg_timing."""
    launches, kern_ms = launches_ms
    n = 2 ** L + 1
    nface = face_interior_dofs(g.F, n)
    avg = kern_ms * 1e-3 / max(launches, 1)
    return {"launches": launches, "avg_launch_ms": round(avg * 1e3, 5),
            "gdofs": round(nface / avg / 1e9, 3),
            "gbs": round(nface * bytes_per_dof / avg / 1e9, 2),
            "hbm_frac": round(nface * bytes_per_dof / avg / 1e9 / HBM_PEAK_GBS, 4)}


def learned_section(args, P, hi, torch):
    """Variable-coefficient workload: training, acceptance, solves, kernels."""
    import numpy as np

    from paper_1805_10167_amd import train
    out = {"workload": "variable-k P1 diffusion, 64-face annulus, level %d, k = exp(g), GRF "
                       "corr. length 0.1, sigma 1, 512 Fourier features" % args.level}
    D = P.HHG_OP_DIFFUSION
    feats = P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_VARK | P.HHG_FEAT_NET
    vxy, tri = hi.mesh_by_name("annulus64")

    # the benchmark-level mesh, for validation during training and evaluation
    L = args.level
    g = P.Mesh(vxy, tri, L, args.coarse_level, feats)
    _, n_all = g.n_dofs(L)
    xy = g.coords(L)
    vseeds = list(range(20000, 20000 + args.val_fields))
    vk = [torch.exp(hi.grf_eval_device(xy, s)) for s in vseeds]
    vf = [hi.uniform_rhs(n_all, 1000 + s) for s in vseeds]

    # training at the coarser level on noise pairs, the weights chosen by the
    # convergence factor on the validation fields
    Lt = args.train_level
    t0 = time.perf_counter()
    gt = P.Mesh(vxy, tri, Lt, 2, feats)
    _, nt_all = gt.n_dofs(Lt)
    xy_t = gt.coords(Lt)
    kaps = [torch.exp(hi.grf_eval_device(xy_t, s)) for s in range(args.train_fields)]
    pairs = train.noise_pairs(gt, kaps, lambda s, j: hi.uniform_vector_device(
        nt_all, 5000 + 100 * s + j), per_field=args.pairs_per_field)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    w_init = train.jacobi_init()
    P.hhg_net_set_weights(gt.h, w_init)
    tr = train.Trainer(pairs, lr=args.lr, batch=4, seed=0)
    sub = np.random.default_rng(1).choice(len(pairs), min(256, len(pairs)), replace=False)
    loss0 = tr.mean_loss(sub)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    w_net, best_step, vhist, losses = train.train_early_stopping(
        tr, args.train_steps, args.val_every, g, vk, vf)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    loss_last = tr.mean_loss(sub)
    P.hhg_net_set_weights(gt.h, w_net)
    loss1 = tr.mean_loss(sub)
    log("trained %d steps in %.1f s (with validation), kept step %d: loss %.4f -> %.4f"
        % (args.train_steps, t_train, best_step, loss0, loss1))
    out["train"] = {"level": Lt, "fields": args.train_fields, "pairs": len(pairs),
                    "pair_kind": "noise", "steps": args.train_steps, "batch": 4, "lr": args.lr,
                    "precision": "bf16 forward (MFMA), fp32 master weights",
                    "validation": {"fields": len(vseeds), "seeds": [vseeds[0], vseeds[-1]],
                                   "every": args.val_every, "kept_step": best_step,
                                   "factor": [[s, round(r, 5)] for s, r in vhist]},
                    "loss_jacobi_init": round(loss0, 5), "loss_kept": round(loss1, 5),
                    "loss_last_step": round(loss_last, 5),
                    "data_s": round(t_data, 2), "train_s": round(t_train, 2),
                    "ms_per_step": round(t_train * 1e3 / args.train_steps, 3)}
    if args.cycle_pair_check:
        ncf = min(32, args.train_fields)
        cp = train.capture_pairs(gt, kaps[:ncf], [hi.uniform_rhs(nt_all, 1000 + s)
                                                  for s in range(ncf)], cycles=8)
        P.hhg_net_set_weights(gt.h, w_init)
        trc = train.Trainer(cp, lr=args.lr, batch=4, seed=0)
        trc.train(500)
        w_cyc = trc.weights()
        del cp, trc
    del pairs, tr, kaps, gt
    torch.cuda.empty_cache()

    # evaluation at the benchmark level
    seeds = list(range(10000, 10000 + args.eval_fields))
    ek = [torch.exp(hi.grf_eval_device(xy, s)) for s in seeds]
    ef = [hi.uniform_rhs(n_all, 1000 + s) for s in seeds]
    dec = train.accept(g, ek, ef, w_net)
    rho_init, _ = train.evaluate(g, ek, ef, w_init)
    out.update({"accepted": dec["accepted"], "guard_tripped": dec["guard_tripped"],
                "rho_gs_mean": round(dec["rho_gs_mean"], 5),
                "rho_net_mean": round(dec["rho_net_mean"], 5),
                "rho_jacobi_init_mean": round(float(rho_init.mean()), 5),
                "rho_gs": [round(x, 5) for x in dec["rho_gs"]],
                "rho_net": [round(x, 5) for x in dec["rho_net"]],
                "eval_fields": len(seeds)})
    log("acceptance: GS %.4f net %.4f init %.4f accepted %s" % (
        dec["rho_gs_mean"], dec["rho_net_mean"], rho_init.mean(), dec["accepted"]))
    if args.cycle_pair_check:
        d2 = train.accept(g, ek[:2], ef[:2], w_cyc)
        out["cycle_pair_network"] = {"fields": ncf, "steps": 500, "guard_tripped":
                                     d2["guard_tripped"], "accepted": d2["accepted"]}

    # time to 1e-8 on the first held-out field
    P.hhg_set_coefficient(g.h, ek[0])
    f = g.from_canonical(L, ef[0])
    u = g.field(L)
    t2t, its = {}, {}
    for name, mode in (("plain_fp64", P.HHG_MODE_PLAIN_FP64), ("mp_gs", P.HHG_MODE_MP_IR)):
        ms = []
        for _ in range(max(1, args.mp_runs)):
            t, rc, st, _ = timed_solve(P, g, u, f, mode, D, 1e-8, 3)
            assert rc == 0, st
            ms.append(t)
        t2t[name], its[name] = round(statistics.median(ms), 3), st["iters"]
    P.hhg_net_set_weights(g.h, w_net)
    P.hhg_net_set_options(g.h, P.HHG_BF16, 1)        # the network regardless of the decision
    ms = []
    for _ in range(max(1, args.mp_runs)):
        t, rc, st, _ = timed_solve(P, g, u, f, P.HHG_MODE_LEARNED, D, 1e-8, 3)
        ms.append(t)
    t2t["mp_net"], its["mp_net"] = round(statistics.median(ms), 3), st["iters"]
    out["mp_net_guard_fallback"] = st["fallback"]
    P.hhg_net_set_options(g.h, P.HHG_BF16, int(dec["accepted"]))
    t, rc, st, _ = timed_solve(P, g, u, f, P.HHG_MODE_LEARNED, D, 1e-8, 3)
    t2t["learned_mode"], its["learned_mode"] = round(t, 3), st["iters"]
    out["learned_mode_smoother"] = "net" if st["smoother_used"] == P.HHG_SMOOTH_NET else "gs"
    out["time_to_tol_ms"], out["iterations"] = t2t, its

    # kernels of the path, live: variable-k FP64 face smoother, FP32 net step
    P.hhg_timing_read(g.h, reset=True)
    P.hhg_timing_enable(g.h, 1)
    for _ in range(20):
        P.hhg_smooth(g.h, L, D, P.HHG_SMOOTH_GS, P.HHG_F64, u, f, 1, 0)
    P.hhg_timing_enable(g.h, 0)
    out["vark_face_smoother_fp64"] = face_sweep_rate(P, g, L, P.hhg_timing_read(g.h), 32.0)
    u32, f32 = g.field(L, P.HHG_F32), g.from_canonical(L, ef[0], P.HHG_F32)
    rho = g.field(L, P.HHG_F32)
    n_int = g.n_dofs(L)[0]
    nface = face_interior_dofs(g.F, 2 ** L + 1)

    def event_ms(fn, reps=20):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps

    sweep_ms = event_ms(lambda: P.hhg_smooth(g.h, L, D, P.HHG_SMOOTH_NET, P.HHG_F32, u32, f32, 1, 0))
    jac_ms = event_ms(lambda: P.hhg_jacobi(g.h, L, D, P.HHG_F32, u32, f32, rho))
    fwd_ms = event_ms(lambda: P.hhg_net_forward(g.h, L, rho, u32))
    flops = 448.0 * nface
    out["net_step_fp32"] = {
        "sweep_ms": round(sweep_ms, 4), "sweep_gdofs": round(n_int / sweep_ms / 1e6, 3),
        "sweep_hbm_frac_vs_16B": round(n_int * 16.0 / sweep_ms / 1e6 / HBM_PEAK_GBS, 4),
        "jacobi_ms": round(jac_ms, 4), "forward_ms": round(fwd_ms, 4),
        "forward_tflops": round(flops / fwd_ms / 1e9, 3),
        "mfma_frac_of_bf16_peak": round(flops / fwd_ms / 1e9 / BF16_PEAK_TFLOPS, 6),
        "note": "events around whole calls on torch's stream (the library's launch stream)"}
    del g, ek, u, f, u32, f32, rho
    torch.cuda.empty_cache()
    return out


def square_section(P, hi, torch, levels=(3, 4, 5, 6, 7, 8), timed_level=6, reps=5):
    """The manufactured case on the unit square: -Laplace u = f with
    f = 2 pi^2 sin(pi x) sin(pi y) and u = 0 on the boundary, so that
    u = sin(pi x) sin(pi y).  The right-hand side is b = M f_I (the library's
    mass operator on the nodal interpolant), the solve plain FP64 V(2,2) to
    1e-10 on coarse level 2.  Reports the solve time at one level and the
    discretisation error against u at the nodes on several levels (it should
    fall by 4 per level)."""
    vxy, tri = hi.unit_square()
    out = {"workload": "unit square, 2 macro-faces, manufactured sin(pi x) sin(pi y), "
                       "V(2,2) to 1e-10, coarse level 2", "levels": {}}
    prev = None
    for L in levels:
        g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64)
        n_int, _ = g.n_dofs(L)
        xy = torch.tensor(g.coords(L), dtype=torch.float64, device="cuda")
        s2 = torch.sin(math.pi * xy[:, 0]) * torch.sin(math.pi * xy[:, 1])
        fI = g.from_canonical(L, 2.0 * math.pi ** 2 * s2)
        b = g.field(L)
        P.hhg_apply(g.h, L, P.HHG_OP_MASS, P.HHG_F64, fI, b)
        u = g.field(L)
        ms = []
        for _ in range(reps if L == timed_level else 1):
            t, rc, st, _ = timed_solve(P, g, u, b, P.HHG_MODE_PLAIN_FP64, P.HHG_OP_LAPLACE, 1e-10, 2)
            assert rc == 0, st
            ms.append(t)
        err = (g.to_canonical(L, u) - s2).abs().max().item()
        h = 1.0 / 2 ** L
        rec = {"interior_dofs": n_int, "iterations": st["iters"], "max_error": err,
               "rms_error": ((g.to_canonical(L, u) - s2) ** 2).sum().item() ** 0.5 * h}
        if prev is not None:
            rec["max_error_ratio"] = round(prev / err, 3)
        if L == timed_level:
            rec["time_to_tol_ms"] = round(statistics.median(ms), 3)
        out["levels"][str(L)] = rec
        prev = err
        del g, u, b, fI, xy, s2
    return out


def large_mp_section(args, P, hi, torch):
    """Plain FP64 against mixed precision on the 128-face annulus."""
    L = args.large_level
    vxy, tri = hi.mesh_by_name("annulus128")
    t0 = time.perf_counter()
    g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP)
    n_int, n_all = g.n_dofs(L)
    f = g.from_canonical(L, hi.uniform_rhs(n_all, 1))
    log("large mesh level %d: %d unknowns, setup %.1f s" % (L, n_int, time.perf_counter() - t0))
    u, ref = g.field(L), g.field(L)
    out = {"workload": "Poisson P1, 128-face annulus, level %d, uniform RHS seed 1" % L,
           "interior_dofs": n_int}
    res = {}
    for name, mode in (("plain_fp64", P.HHG_MODE_PLAIN_FP64), ("mp_ir", P.HHG_MODE_MP_IR)):
        ms = []
        for _ in range(max(1, args.mp_runs)):
            t, rc, st, _ = timed_solve(P, g, u, f, mode, P.HHG_OP_LAPLACE, 1e-8, 3)
            assert rc == 0, st
            ms.append(t)
        res[name] = (round(statistics.median(ms), 3), st["iters"], st["rel_res"])
        if name == "plain_fp64":
            ref.copy_(u)
    out["time_to_tol_ms"] = {k: v[0] for k, v in res.items()}
    out["iterations"] = {k: v[1] for k, v in res.items()}
    out["final_rel_res"] = {k: v[2] for k, v in res.items()}
    # u (MP) against a plain solve to 1e-12
    _, rc, st, _ = timed_solve(P, g, ref, f, P.HHG_MODE_PLAIN_FP64, P.HHG_OP_LAPLACE, 1e-12, 3)
    d = torch.zeros(2, dtype=torch.float64, device="cuda")
    P.hhg_axpby(g.h, L, P.HHG_F64, 1.0, u, -1.0, ref, u)
    P.hhg_dot(g.h, L, P.HHG_F64, u, u, d[0:1])
    P.hhg_dot(g.h, L, P.HHG_F64, ref, ref, d[1:2])
    dd = d.cpu().numpy()
    out["mp_rel_err_vs_fp64_1e-12"] = float(math.sqrt(dd[0] / dd[1]))
    del u, ref, f
    torch.cuda.empty_cache()
    if not args.no_kernels:
        log("per-call kernel rates at level %d" % L)
        out["kernels"] = kernel_section(P, hi, torch, g, L, reps=5)
    del g
    torch.cuda.empty_cache()
    return out


STOKES_DELTA = 1.0 / 12.0


def stokes_section(args, P, hi, torch):
    """PSPG-stabilised P1-P1 Stokes on the 128-face annulus: viscosity 1 in
    the inner and 100 in the outer ring of faces, buoyancy forcing -T r_hat
    with T a seeded Gaussian random field (correlation length 0.1, sigma 1),
    velocity zero on both boundaries; MINRES with the block-diagonal
    preconditioner (one V(2,2) cycle per velocity component; pressure block
    the lumped 1/mu mass plus 4 diag(C)) to a relative residual of 1e-8 in the preconditioner's
    norm, FP64 and FP32 velocity cycles.  Also the Stokes operator's rate."""
    L = args.stokes_level
    vxy, tri = hi.mesh_by_name("annulus128")
    mu = hi.face_viscosity(vxy, tri)
    g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_STOKES)
    P.hhg_stokes_setup(g.h, mu, STOKES_DELTA)
    n_int, n_all = g.n_dofs(L)
    fs = P.hhg_field_elems(g.h, L)
    xy = torch.tensor(g.coords(L), dtype=torch.float64, device="cuda")
    T = hi.grf_eval_device(xy, 500)
    rr = torch.sqrt(xy[:, 0] ** 2 + xy[:, 1] ** 2)
    b = g.stokes_vector(L)
    for c in range(2):
        fc = g.from_canonical(L, -T * xy[:, c] / rr)
        P.hhg_apply(g.h, L, P.HHG_OP_MASS, P.HHG_F64, fc, b[c * fs:(c + 1) * fs])
    del xy, T, rr
    x = g.stokes_vector(L)
    out = {"workload": "P1-P1 PSPG Stokes, 128-face annulus, level %d, viscosity 1:100 jump at "
                       "r = 0.775, buoyancy -T r_hat (GRF seed 500), zero velocity on the boundary"
                       % L,
           "dofs": {"velocity": 2 * n_int, "pressure": n_all, "total": 2 * n_int + n_all},
           "solver": "MINRES, blockdiag(V(2,2) per velocity component, lumped 1/mu pressure mass + 4 diag(C)), "
                     "rtol 1e-8 in the preconditioner's norm, coarse level 2", "delta": STOKES_DELTA}
    res = {}
    for name, prec in (("plain_fp64", P.HHG_F64), ("fp32_precond", P.HHG_F32)):
        ms = []
        for rep in range(1 + args.stokes_runs):
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rc, st, hist = P.hhg_stokes_solve(g.h, x, b, precision=prec, rtol=1e-8, max_iters=2000,
                                              nu1=2, nu2=2)
            torch.cuda.synchronize()
            if rep > 0:                          # the first run warms up
                ms.append((time.perf_counter() - t0) * 1e3)
            assert rc == 0, st
        # true relative residual |b - K x| / |b| (Euclidean, owned points)
        r = g.stokes_vector(L)
        P.hhg_stokes_residual(g.h, L, x, b, r)
        d = torch.zeros(2, dtype=torch.float64, device="cuda")
        P.hhg_stokes_dot(g.h, L, r, r, d[0:1])
        P.hhg_stokes_dot(g.h, L, b, b, d[1:2])
        dd = d.cpu().numpy()
        res[name] = {"time_to_tol_ms": round(statistics.median(ms), 2), "iterations": st["iters"],
                     "ms_per_iteration": round(statistics.median(ms) / max(st["iters"], 1), 3),
                     "rel_res_precond_norm": st["rel_res"],
                     "rel_res_euclidean": float(math.sqrt(dd[0] / dd[1]))}
        log("stokes %s: %d iterations, %.1f ms" % (name, st["iters"], res[name]["time_to_tol_ms"]))
        del r
    out["solves"] = res
    # the Stokes operator alone: 3 fields read, 3 written per point
    y = g.stokes_vector(L)
    for _ in range(2):
        P.hhg_stokes_apply(g.h, L, x, y)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 10
    ev[0].record()
    for _ in range(reps):
        P.hhg_stokes_apply(g.h, L, x, y)
    ev[1].record()
    ev[1].synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    nbytes = 48.0 * n_all
    out["stokes_apply"] = {"ms": round(ms, 4), "gdofs": round(3 * n_all / ms / 1e6, 2),
                           "alg_bytes_per_point": 48, "hbm_frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4)}
    del g, x, y, b
    torch.cuda.empty_cache()
    return out


def energy_section(args, P, hi, torch):
    """The paper's energy-transport example at its own size: isoviscous
    Stokes on a 256-face annulus (64 sectors x 2 rings) at level 6 (2,145
    points per face, more than half a million unknowns), buoyancy -Ra T r_hat,
    temperature on the micro-triangles advanced by the explicit upwind
    scheme, a Stokes solve (MINRES, warm started) before every third
    transport step.  T starts from the conductive profile plus a seeded
    perturbation; dt = 0.5 h / max|u| from the first flow."""
    L = args.energy_level
    vxy, tri = hi.annulus(n_tan=64)
    g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_STOKES)
    P.hhg_stokes_setup(g.h, [1.0] * len(tri), STOKES_DELTA)
    n_int, n_all = g.n_dofs(L)
    fs = P.hhg_field_elems(g.h, L)
    n = 2 ** L + 1
    ncell = len(tri) * (n - 1) ** 2
    cen = g.cell_coords(L)
    T0 = hi.conductive_temperature(cen) + 0.05 * hi.grf_eval(cen, 600)
    T = torch.zeros(2 * fs, dtype=torch.float64, device="cuda")
    P.hhg_cells_from_canonical(g.h, L, torch.tensor(T0, dtype=torch.float64, device="cuda"), T)
    x = g.stokes_vector(L)
    Ra = args.energy_ra
    rc, st = P.hhg_energy_run(g.h, x, T, Ra=Ra, dt=0.0, steps=1, stokes_every=3)
    assert rc == 0, st
    umax = torch.sqrt(x[:fs] ** 2 + x[fs:2 * fs] ** 2).max().item()
    hmin = 0.55 * 2 * math.pi / 64 / (n - 1)
    dt = 0.5 * hmin / umax
    steps = args.energy_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, st = P.hhg_energy_run(g.h, x, T, Ra=Ra, dt=dt, steps=steps, stokes_every=3)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3
    assert rc == 0, st
    # transport step alone
    T2 = torch.empty_like(T)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    P.hhg_transport_step(g.h, L, x, T, T2, dt)
    ev[0].record()
    for _ in range(20):
        P.hhg_transport_step(g.h, L, x, T, T2, dt)
    ev[1].record()
    ev[1].synchronize()
    step_ms = ev[0].elapsed_time(ev[1]) / 20
    Tc = torch.zeros(ncell, dtype=torch.float64, device="cuda")
    P.hhg_cells_to_canonical(g.h, L, T, Tc)
    return {"workload": "isoviscous P1-P1 PSPG Stokes + upwind FV temperature, 256-face annulus, level %d "
                        "(%d faces x %d points per face), Ra %g, Stokes every 3 steps" % (L, len(tri), n * (n + 1) // 2, Ra),
            "dofs": {"stokes": 2 * n_int + n_all, "cells": ncell},
            "dt": dt, "steps": steps, "stokes_solves": st["stokes_solves"],
            "minres_iters_per_solve": round(st["minres_iters"] / max(st["stokes_solves"], 1), 1),
            "ms_per_step": round(wall / steps, 3), "transport_step_ms": round(step_ms, 4),
            "T_range": [Tc.min().item(), Tc.max().item()]}


def p2_section(args, P, hi, torch):
    """Quadratic (P2) elements on the 64-face annulus at P2 level 9 (the
    level-10 point layout: 33.5M unknowns, the headline's count), uniform
    random right-hand side, p-multigrid (3 + 3 damped Jacobi sweeps, omega
    0.7, one P1 V(2,2) cycle of the h-hierarchy on level 9 per cycle) to a
    relative residual of 1e-8; also one Jacobi sweep alone (x, f read, y
    written: 24 B per unknown)."""
    l = args.p2_level
    vxy, tri = hi.mesh_by_name("annulus64")
    g = P.Mesh(vxy, tri, l + 1, 3, P.HHG_FEAT_F64 | P.HHG_FEAT_P2)
    P.hhg_p2_setup(g.h)
    n_int, n_all = g.n_dofs(l + 1)
    f = hi.uniform_vector_device(n_all, 1)
    fd = g.from_canonical(l + 1, f)
    del f
    u = g.field(l + 1)
    ms, st = [], None
    for rep in range(1 + args.p2_runs):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc, st, hist = P.hhg_p2_solve(g.h, l, u, fd, rtol=1e-8, max_iters=100, nu1=3, nu2=3, vnu1=2,
                                      vnu2=2, omega=0.7, history=False)
        torch.cuda.synchronize()
        assert rc == 0, st
        if rep > 0:
            ms.append((time.perf_counter() - t0) * 1e3)
    y = g.field(l + 1)
    for _ in range(2):
        P.hhg_p2_jacobi(g.h, l, 0.7, u, fd, y)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    reps = 10
    ev[0].record()
    for _ in range(reps):
        P.hhg_p2_jacobi(g.h, l, 0.7, u, fd, y)
    ev[1].record()
    ev[1].synchronize()
    sweep = ev[0].elapsed_time(ev[1]) / reps
    out = {"workload": "P2 Poisson, 64-face annulus, P2 level %d (level-%d layout), uniform RHS seed 1" % (l, l + 1),
           "interior_dofs": n_int,
           "solver": "p-multigrid: 3+3 damped Jacobi (omega 0.7) on P2, one P1 V(2,2) on level %d, "
                     "coarse level 3" % l,
           "time_to_tol_ms": round(statistics.median(ms), 2), "cycles": st["iters"],
           "ms_per_cycle": round(statistics.median(ms) / max(st["iters"], 1), 3),
           "rel_res": st["rel_res"],
           "jacobi_sweep": {"ms": round(sweep, 4), "gdofs": round(n_int / sweep / 1e6, 2),
                            "alg_bytes_per_dof": 24,
                            "hbm_frac": round(24.0 * n_int / sweep / 1e6 / HBM_PEAK_GBS, 4)}}
    del g, u, y, fd
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=10)
    ap.add_argument("--coarse-level", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-level", type=int, default=9)
    ap.add_argument("--cpu-all-level", type=int, default=8)
    ap.add_argument("--cpu-workers", type=int, default=0, help="0: one per host core")
    ap.add_argument("--mp-runs", type=int, default=3)
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-level", type=int, default=7)
    ap.add_argument("--train-fields", type=int, default=256)
    ap.add_argument("--pairs-per-field", type=int, default=8)
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--val-every", type=int, default=100)
    ap.add_argument("--val-fields", type=int, default=2)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--eval-fields", type=int, default=8)
    ap.add_argument("--cycle-pair-check", type=int, default=1)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--no-kernels", action="store_true")
    ap.add_argument("--no-square", action="store_true")
    ap.add_argument("--large-level", type=int, default=11)
    ap.add_argument("--no-stokes", action="store_true")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--no-p2", action="store_true")
    ap.add_argument("--p2-level", type=int, default=9)
    ap.add_argument("--p2-runs", type=int, default=2)
    ap.add_argument("--energy-level", type=int, default=6)
    ap.add_argument("--energy-steps", type=int, default=30)
    ap.add_argument("--energy-ra", type=float, default=1e4)
    ap.add_argument("--stokes-level", type=int, default=9)
    ap.add_argument("--stokes-runs", type=int, default=2)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="bytes of a plain device copy run after the benchmark (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: sharding the macro-faces over several GPUs is "
              "designed but not implemented; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import hhg_inputs as hi
    import paper_1805_10167_amd as P

    torch.cuda.set_device(0)
    L, nu, rtol = args.level, 3, 1e-8
    vxy, tri = hi.mesh_by_name("annulus64")
    log("setting up annulus64 level %d" % L)
    lc = args.coarse_level
    g = P.Mesh(vxy, tri, L, lc, P.HHG_FEAT_F64 | P.HHG_FEAT_MP)
    n_int, n_all = g.n_dofs(L)
    n = 2 ** L + 1
    F = len(tri)
    f = g.from_canonical(L, hi.uniform_rhs(n_all, 1))
    u = g.field(L)
    stream = torch.cuda.current_stream()

    def solve(mode):
        u.zero_()
        return P.hhg_solve(g.h, u, f, mode=mode, rtol=rtol, nu1=nu, nu2=nu, history=True,
                           stream=stream)

    for _ in range(args.warmup):
        rc, st, _ = solve(P.HHG_MODE_PLAIN_FP64)
        assert rc == 0, st
    # the timed steps: no per-launch events inside them
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, st, _ = solve(P.HHG_MODE_PLAIN_FP64)
        assert rc == 0, st
        iters.append(st["iters"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the roofline kernel, live: the same solves again with an event pair
    # around every finest-level face-smoother launch on its stream
    P.hhg_timing_read(g.h, reset=True)
    P.hhg_timing_enable(g.h, 1)
    for _ in range(args.steps):
        solve(P.HHG_MODE_PLAIN_FP64)
    torch.cuda.synchronize()
    P.hhg_timing_enable(g.h, 0)
    launches, kern_ms = P.hhg_timing_read(g.h, reset=True)
    log("%d solves, iters %s, %d face-smoother launches timed" % (args.steps, iters, launches))

    ms_per_step = wall * 1e3 / args.steps
    sweeps = 2 * nu * statistics.mean(iters)
    value = n_int * sweeps / (ms_per_step * 1e-3) / 1e9
    nface = face_interior_dofs(F, n)
    avg_launch_s = kern_ms * 1e-3 / max(launches, 1)
    bytes_per_launch = nface * 24.0          # read u, f; write u (FP64)
    achieved = bytes_per_launch / avg_launch_s / 1e9

    # mixed-precision refinement on the same problem
    mp_times, mp_iters, mp_res = [], [], []
    for _ in range(args.mp_runs):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rc, st, _ = solve(P.HHG_MODE_MP_IR)
        torch.cuda.synchronize()
        mp_times.append((time.perf_counter() - t1) * 1e3)
        mp_iters.append(st["iters"])
        mp_res.append(st["rel_res"])
        assert rc == 0, st

    if args.copy_calibration:
        src = torch.empty(args.copy_calibration // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    from paper_1805_10167_amd.profiling import traffic_for
    traffic = traffic_for(os.path.join(ROOT, "profiles", "face_smoother_annulus64_l10.txt"))
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GDoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson-p1-annulus64-level%d-V33-rtol1e-8" % L,
                   "mesh": "jittered annulus, 64 macro-faces", "level": L,
                   "interior_dofs": n_int, "solver": "V(3,3) staged multicolour GS, direct "
                   "solve on coarse level %d, plain FP64" % lc},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "kernel": "finest-level face smoother (all colours, one sweep)",
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": round(avg_launch_s * 1e3, 5), "launches": launches},
        "smoother_kernel_gdofs": round(nface / avg_launch_s / 1e9, 3),
        "time_to_tol_ms": {"plain_fp64": round(ms_per_step, 3)},
        "iterations": {"plain_fp64": iters[0]},
    }
    if mp_times:
        out["time_to_tol_ms"]["mp_ir"] = round(statistics.median(mp_times), 3)
        out["iterations"]["mp_ir"] = mp_iters[0]
        out["mp_final_rel_res"] = mp_res[0]
    if not args.no_kernels:
        log("per-call kernel rates at level %d" % L)
        out["kernels"] = kernel_section(P, hi, torch, g, L)
    del g, u, f
    torch.cuda.empty_cache()
    if not args.no_learned:
        log("learned smoother: training and acceptance")
        out["learned"] = learned_section(args, P, hi, torch)
    if not args.no_large:
        log("plain vs mixed precision on the 128-face annulus")
        out["mp_large"] = large_mp_section(args, P, hi, torch)
    if not args.no_stokes:
        log("Stokes on the 128-face annulus")
        out["stokes"] = stokes_section(args, P, hi, torch)
    if not args.no_energy:
        log("energy transport on the 256-face annulus")
        out["energy"] = energy_section(args, P, hi, torch)
    if not args.no_p2:
        log("P2 elements with p-multigrid on the 64-face annulus")
        out["p2"] = p2_section(args, P, hi, torch)
    if not args.no_square:
        log("manufactured solution on the unit square")
        out["square"] = square_section(P, hi, torch)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle at level %d" % args.cpu_level)
        out["cpu_baseline"] = cpu_baseline(args.cpu_level, rtol, nu, args.cpu_all_level,
                                           args.cpu_workers or host_cores())
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
