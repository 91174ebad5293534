"""Benchmark of the HHG P1 multigrid hot path on one MI355X.

Workload (N = 1): Poisson -Laplace u = f with P1 elements on the jittered
64-face annulus r in [0.55, 1], refinement level 10 (1025 points per
macro-edge, 33,538,048 interior unknowns), constant coefficient, uniform
[-1, 1] right-hand side (seed 1), homogeneous Dirichlet boundary, FP64,
V(3,3) cycles with the staged multicolour Gauss-Seidel smoother to a relative
residual of 1e-8.

A step is one solve from u = 0 to 1e-8 (every V-cycle level: smoothing,
residual, restriction, coarse CG, prolongation, ghost-copy refresh, norms).
value = whole-job smoother throughput: finest-level interior unknowns times
the finest-level sweeps the solve performs, divided by the solve's wall time.
The roofline entry is the finest-level face smoother, timed live with HIP
events on the launch stream; the mixed-precision solve of the same problem is
reported beside it.
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


def face_interior_dofs(F, n):
    return F * (n - 2) * (n - 3) // 2


def cpu_baseline(level, rtol, nu):
    """Time the oracle's plain solve on the same mesh at a smaller level."""
    import numpy as np

    import hhg_inputs as hi
    from oracle.mesh import MacroMesh
    from oracle.mg import Hierarchy
    vxy, tri = hi.mesh_by_name("annulus64")
    H = Hierarchy(MacroMesh(vxy, tri), level, 2)
    lv = H.levels[level]
    f = hi.uniform_rhs(lv.n_all, 1)
    t0 = time.perf_counter()
    u, hist = H.solve(np.zeros(lv.n_all), f, rtol, nu, nu)
    dt = time.perf_counter() - t0
    iters = len(hist) - 1
    work = lv.interior_count() * 2 * nu * iters
    return {"value": work / dt / 1e9, "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": "oracle plain solve to %g on the same 64-face annulus at level %d "
                      "(%d interior unknowns, %d V(%d,%d) cycles, %.1f s; scipy sparse "
                      "kernels, single-threaded)" % (rtol, level, lv.interior_count(), iters,
                                                     nu, nu, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--level", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-level", type=int, default=9)
    ap.add_argument("--mp-runs", type=int, default=3)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="bytes of a plain device copy run after the benchmark (counter scale)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the method's multi-GPU sharding is not part "
              "of this build (see the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import hhg_inputs as hi
    import paper_1805_10167_amd as P

    torch.cuda.set_device(0)
    L, nu, rtol = args.level, 3, 1e-8
    vxy, tri = hi.mesh_by_name("annulus64")
    print("bench: setting up annulus64 level %d" % L, file=sys.stderr, flush=True)
    g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP)
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
    torch.cuda.synchronize()
    P.hhg_timing_read(g.h, reset=True)
    P.hhg_timing_enable(g.h, 1)
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, st, _ = solve(P.HHG_MODE_PLAIN_FP64)
        iters.append(st["iters"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    P.hhg_timing_enable(g.h, 0)
    launches, kern_ms = P.hhg_timing_read(g.h, reset=True)
    print("bench: %d solves, iters %s, %d face-smoother launches" % (args.steps, iters, launches),
          file=sys.stderr, flush=True)

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

    from paper_1805_10167_amd.profiling import traffic_for
    traffic = traffic_for(os.path.join(ROOT, "profiles", "face_smoother_annulus64_l10.txt"))
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GDoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson-p1-annulus64-level%d-V33-rtol1e-8" % L,
                   "mesh": "jittered annulus, 64 macro-faces", "level": L,
                   "interior_dofs": n_int, "solver": "V(3,3) staged multicolour GS, "
                   "Jacobi-PCG coarse level 2, plain FP64"},
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
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle at level %d" % args.cpu_level, file=sys.stderr,
              flush=True)
        out["cpu_baseline"] = cpu_baseline(args.cpu_level, rtol, nu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
