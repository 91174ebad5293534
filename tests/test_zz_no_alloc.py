"""The allocation-free dot product (partial sums in the library's static
device scratch) against hhg_dot (partial sums in the workspace): the same
kernels and summation order, so equal bit for bit, on two calls in a row,
the second on a smaller level, in both precisions, and again after other
library calls have used the GPU."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import gpu_mesh, log

pytestmark = pytest.mark.gpu


def test_dot_noalloc_matches_dot():
    import torch

    import paper_1805_10167_amd as P
    g = gpu_mesh("annulus64", 7, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP)
    outs = torch.zeros(4, dtype=torch.float64, device="cuda")
    for level in (7, 4):
        _, n_all = g.n_dofs(level)
        for dt in (P.HHG_F64, P.HHG_F32):
            x = g.from_canonical(level, hi.uniform_vector(n_all, 3 + level), dt)
            y = g.from_canonical(level, hi.uniform_vector(n_all, 4 + level), dt)
            outs.zero_()
            P.hhg_dot_noalloc(g.h, level, dt, x, y, outs[0:1])
            P.hhg_dot(g.h, level, dt, x, y, outs[1:2])
            # the static scratch keeps the last call's partials: a call on
            # other data right after must not see them
            P.hhg_dot_noalloc(g.h, level, dt, y, y, outs[2:3])
            P.hhg_dot(g.h, level, dt, y, y, outs[3:4])
            o = outs.cpu().numpy()
            log("noalloc dot level %d dtype %d: %r" % (level, dt, o))
            assert o[0] == o[1] and o[2] == o[3]
            xc = g.to_canonical(level, x, dt).cpu().numpy().astype(np.float64)
            yc = g.to_canonical(level, y, dt).cpu().numpy().astype(np.float64)
            # against the plain definition over the owned interior points
            from gpu_util import oracle_hierarchy
            ii = oracle_hierarchy("annulus64", 7, 2).levels[level].interior
            assert abs(o[0] - xc[ii] @ yc[ii]) <= 1e-12 * np.abs(xc[ii] * yc[ii]).sum()
    with pytest.raises(P.HHGError):
        P.hhg_dot_noalloc(g.h, 0, P.HHG_F64, x, y, outs[0:1])
