"""Shared helpers of the GPU parity tests: build the library mesh and the
oracle hierarchy on the same seeded inputs and compare canonical vectors."""
import functools
import sys

import numpy as np

import hhg_inputs as hi


# Bounds of the reduced-precision paths against the FP64 oracle (relative,
# max norm).  FP32 V-cycle on FP32-representable inputs: besides the rounding
# of every operation (unit roundoff 6e-8, 7-term stencil sums), the FP32 path
# rounds the operator's weights, a relative perturbation of the operator of
# unit-roundoff size.  A V-cycle from a random iterate takes most of its
# result from the coarse-grid correction of smooth error, and the perturbed
# operator changes that correction by the perturbation times the ratio of
# the operator's norm to its smallest eigenvalue on the coarse grid, a few
# tens: 2.6e-6 and 3.1e-6 were measured at levels 8 and 9 (about 50 unit
# roundoffs), 1e-5 is the bound.  Mixed-precision refinement to a relative
# residual of 1e-8: the final error against an oracle solve to 1e-12 is the
# algebraic error of that residual, of order 1e-8 times the error-to-residual
# ratio of a few, so 1e-7.
F32_VCYCLE_TOL = 1e-5
MP_TOL = 1e-7


def f32_vcycle_tol(level):
    return F32_VCYCLE_TOL


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
