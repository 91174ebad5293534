"""MI355X-native hierarchical-hybrid-grid P1 multigrid (HIP library + binding).

The computation lives in libhhg.so (HIP kernels for gfx950 behind the C ABI of
include/hhg.h).  This package only marshals arguments; torch supplies device
memory and streams.  `Mesh` bundles a mesh handle with its workspace.
"""
import numpy as np

from ._lib import *  # noqa: F401,F403
from ._lib import (lib, HHG_F32, HHG_F64, HHG_FEAT_F64, HHG_OP_LAPLACE, HHGError,  # noqa: F401
                   hhg_bind_workspace, hhg_coords, hhg_destroy_mesh, hhg_field_elems,
                   hhg_from_canonical, hhg_n_dofs, hhg_setup_mesh, hhg_to_canonical,
                   hhg_workspace_bytes)


class Mesh:
    """A macro mesh with a bound device workspace.

    vxy[V, 2], tri[F, 3]: macro mesh; max_level / coarse_level: hierarchy;
    features: HHG_FEAT_* bits of the workspace."""

    def __init__(self, vxy, tri, max_level, coarse_level=2, features=HHG_FEAT_F64,
                 device="cuda"):
        import torch
        self.h = hhg_setup_mesh(vxy, tri, max_level, coarse_level)
        self._destroy = lib().hhg_destroy_mesh   # kept alive for interpreter exit
        self.L = max_level
        self.lc = coarse_level
        self.F = len(tri)
        self.features = features
        self.device = device
        nbytes = hhg_workspace_bytes(self.h, features)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        hhg_bind_workspace(self.h, features, self.ws)

    def __del__(self):
        h = getattr(self, "h", None)
        if h and getattr(self, "_destroy", None) is not None:
            self._destroy(h)
            self.h = None

    @staticmethod
    def _tdtype(dtype):
        import torch
        return torch.float64 if dtype == HHG_F64 else torch.float32

    def field(self, level, dtype=HHG_F64):
        import torch
        return torch.zeros(hhg_field_elems(self.h, level), dtype=self._tdtype(dtype),
                           device=self.device)

    def n_dofs(self, level):
        return hhg_n_dofs(self.h, level)

    def coords(self, level):
        return hhg_coords(self.h, level)

    def from_canonical(self, level, canon, dtype=HHG_F64):
        import torch
        c = torch.as_tensor(np.asarray(canon) if not hasattr(canon, "data_ptr") else canon)
        c = c.to(device=self.device, dtype=self._tdtype(dtype)).contiguous()
        fld = self.field(level, dtype)
        hhg_from_canonical(self.h, level, dtype, c, fld)
        return fld

    def stokes_vector(self, level):
        """Zeroed Stokes vector (u_x | u_y | p) of `level` (FP64)."""
        import torch
        return torch.zeros(3 * hhg_field_elems(self.h, level), dtype=torch.float64, device=self.device)

    def stokes_from_canonical(self, level, canon3):
        """Stokes vector from canonical [u_x | u_y | p] (3 n_all values)."""
        import torch
        _, n_all = self.n_dofs(level)
        c = torch.as_tensor(np.asarray(canon3)).to(device=self.device, dtype=torch.float64)
        n = hhg_field_elems(self.h, level)
        out = self.stokes_vector(level)
        for k in range(3):
            hhg_from_canonical(self.h, level, HHG_F64, c[k * n_all:(k + 1) * n_all].contiguous(),
                               out[k * n:(k + 1) * n])
        return out

    def stokes_to_canonical(self, level, vec):
        """Canonical [u_x | u_y | p] of a Stokes vector."""
        import torch
        n = hhg_field_elems(self.h, level)
        return torch.cat([self.to_canonical(level, vec[k * n:(k + 1) * n]) for k in range(3)])

    def cell_coords(self, level):
        """Centroids of the micro-triangle cells in canonical cell order."""
        return hhg_cell_coords(self.h, level, self.F)

    def cells_from_canonical(self, level, canon):
        """Device cell field of a canonical cell array."""
        import torch
        out = torch.zeros(2 * hhg_field_elems(self.h, level), dtype=torch.float64, device=self.device)
        hhg_cells_from_canonical(self.h, level, canon, out)
        return out

    def cells_to_canonical(self, level, cells):
        """Canonical cell array of a device cell field."""
        import torch
        n = 2 ** level + 1
        out = torch.empty(self.F * (n - 1) ** 2, dtype=torch.float64, device=self.device)
        hhg_cells_to_canonical(self.h, level, cells, out)
        return out

    def to_canonical(self, level, fld, dtype=HHG_F64):
        import torch
        _, n_all = self.n_dofs(level)
        out = torch.empty(n_all, dtype=self._tdtype(dtype), device=self.device)
        hhg_to_canonical(self.h, level, dtype, fld, out)
        return out
