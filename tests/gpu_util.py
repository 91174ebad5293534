"""Shared helpers of the GPU parity tests: build the library mesh and the
oracle hierarchy on the same seeded inputs and compare canonical vectors."""
import functools
import sys

import numpy as np

import hhg_inputs as hi


# Bounds of the reduced-precision paths against the FP64 oracle (relative,
# max norm).  FP32 V-cycle on FP32-representable inputs: unit roundoff 6e-8
# times a growth factor of about 30 (7-term stencil sums, rounding damped by
# the smoother rather than accumulated over the sweeps).  Mixed-precision
# refinement to a relative residual of 1e-8: the final error against an
# oracle solve to 1e-12 is the algebraic error of that residual, of order
# 1e-8 times the error-to-residual ratio of a few, so 1e-7.
F32_VCYCLE_TOL = 2e-6
MP_TOL = 1e-7


def rel_err(a, b):
    """max |a - b| / max |b| (b = oracle)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=8)
def oracle_hierarchy(name, L, lc, kappa_seed=None):
    from oracle.mesh import MacroMesh
    from oracle.mg import Hierarchy
    vxy, tri = hi.mesh_by_name(name)
    kap = None
    if kappa_seed is not None:
        from oracle.mesh import Level
        lv = Level(MacroMesh(vxy, tri), L)
        kap = np.exp(hi.grf_eval(lv.xy, kappa_seed))
    return Hierarchy(MacroMesh(vxy, tri), L, lc, kap)


def gpu_mesh(name, L, lc, features):
    import paper_1805_10167_amd as P
    vxy, tri = hi.mesh_by_name(name)
    return P.Mesh(vxy, tri, L, lc, features)


def to_np(t):
    return t.detach().cpu().numpy().astype(np.float64)
