"""Pins of the oracle's finite-volume transport and its coupling to Stokes
(CPU only): counts and areas of the cells, flux antisymmetry, exact
conservation of the total heat, invariance of a constant field under a
discretely divergence-free flow, the discrete maximum principle below the
CFL limit, and the buoyancy load of a constant temperature against the row
sums of the independently assembled mass matrix."""
import numpy as np
import pytest

import hhg_inputs as hi
from oracle import transport as tr
from oracle.assemble import assemble
from oracle.mesh import Level, MacroMesh


def level(name, l):
    return Level(MacroMesh(*hi.mesh_by_name(name)), l)


@pytest.mark.parametrize("name,l", [("square", 3), ("annulus64", 3)])
def test_cells_tile_the_domain(name, l):
    lv = level(name, l)
    c = tr.Cells(lv)
    assert c.C == lv.mesh.F * (lv.n - 1) ** 2
    P = lv.mesh.vxy[lv.mesh.tri]
    area = 0.5 * np.abs((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                        - (P[:, 1, 1] - P[:, 0, 1]) * (P[:, 2, 0] - P[:, 0, 0]))
    assert abs(c.area.sum() - area.sum()) <= 1e-13
    # boundary micro-edges: one cell each, (n - 1) per boundary macro-edge
    nb = int(lv.mesh.edge_boundary.sum())
    assert (c.nbr < 0).sum() == nb * (lv.n - 1)
    # neighbours are mutual and share two points
    for cc in range(0, c.C, 7):
        for k in range(3):
            o = c.nbr[cc, k]
            if o >= 0:
                assert cc in c.nbr[o]
                assert len(set(c.tri[cc]) & set(c.tri[o])) == 2


def _random_velocity(lv, seed):
    rng = np.random.default_rng(seed)
    ux, uy = rng.uniform(-1, 1, lv.n_all), rng.uniform(-1, 1, lv.n_all)
    ux[lv.dirichlet] = 0.0
    uy[lv.dirichlet] = 0.0
    return ux, uy


def test_fluxes_are_antisymmetric_and_heat_is_conserved():
    lv = level("annulus64", 3)
    c = tr.Cells(lv)
    ux, uy = _random_velocity(lv, 1)
    F = tr.fluxes(c, ux, uy)
    for cc in range(c.C):
        for k in range(3):
            o = c.nbr[cc, k]
            if o >= 0:
                ko = int(np.flatnonzero(c.nbr[o] == cc)[0])
                assert abs(F[cc, k] + F[o, ko]) <= 1e-15
    T = np.random.default_rng(2).uniform(0, 1, c.C)
    T1 = tr.upwind_step(c, T, F, 0.01)
    assert abs(c.area @ T1 - c.area @ T) <= 1e-14 * (c.area @ T)
    # the step as a matrix gives the same values
    assert np.abs(tr.upwind_matrix(c, F, 0.01) @ T - T1).max() <= 1e-15


def test_constant_temperature_is_kept_by_a_divergence_free_flow():
    """u = (2x - 3y + 1, -2y + 4x) is linear with div u = 0; the flux of a
    linear field through a micro-edge is exact, so every cell's net flux is
    the integral of div u over it, zero: a constant T stays constant on the
    cells away from the boundary (where the scheme drops the flux)."""
    lv = level("annulus64", 3)
    c = tr.Cells(lv)
    x, y = lv.xy[:, 0], lv.xy[:, 1]
    F = tr.fluxes(c, 2 * x - 3 * y + 1, -2 * y + 4 * x)
    inner = (c.nbr >= 0).all(axis=1)
    assert np.abs(F[inner].sum(axis=1)).max() <= 1e-15
    dt = 0.05
    T1 = tr.upwind_step(c, np.full(c.C, 0.7), F, dt)
    # rounding of the three-term flux sum, scaled by dt / |c|
    tol = 4e-16 * np.abs(F).max() * dt / c.area.min()
    assert np.abs(T1[inner] - 0.7).max() <= tol


def test_maximum_principle_below_the_cfl_limit():
    """With a divergence-free flow and dt |outflow| <= |c|, every new value
    is a convex combination of the old values of the cell and its upwind
    neighbours."""
    lv = level("annulus64", 3)
    c = tr.Cells(lv)
    x, y = lv.xy[:, 0], lv.xy[:, 1]
    F = tr.fluxes(c, 2 * x - 3 * y + 1, -2 * y + 4 * x)
    out = np.where(F > 0, F, 0).sum(axis=1)
    dt = 0.9 * (c.area[out > 0] / out[out > 0]).min()
    T = np.random.default_rng(5).uniform(0, 1, c.C)
    T1 = tr.upwind_step(c, T, F, dt)
    inner = (c.nbr >= 0).all(axis=1)
    Tn = np.where(c.nbr >= 0, T[np.maximum(c.nbr, 0)], T[:, None])
    lo = np.minimum(T, Tn.min(axis=1))
    hi = np.maximum(T, Tn.max(axis=1))
    assert (T1[inner] >= lo[inner] - 1e-15).all() and (T1[inner] <= hi[inner] + 1e-15).all()


def test_buoyancy_of_a_constant_temperature():
    """T = 1: b_i = -Ra r_hat(x_i) int phi_i, and int phi_i is the row sum of
    the consistent mass matrix."""
    lv = level("annulus64", 3)
    c = tr.Cells(lv)
    bx, by = tr.buoyancy(lv, c, np.ones(c.C), 2.5)
    M = assemble(lv, want=("M",))["M"]
    m = np.asarray(M.sum(axis=1)).ravel()
    r = np.hypot(lv.xy[:, 0], lv.xy[:, 1])
    ii = lv.interior
    assert np.abs(bx[ii] + 2.5 * m[ii] * lv.xy[ii, 0] / r[ii]).max() <= 1e-15
    assert np.abs(by[ii] + 2.5 * m[ii] * lv.xy[ii, 1] / r[ii]).max() <= 1e-15
    assert (bx[lv.dirichlet] == 0).all()


def test_coupled_loop_solves_stokes_every_third_step():
    from oracle import stokes as S
    m = MacroMesh(*hi.mesh_by_name("annulus64"))
    st = S.Stokes(m, 3, 2, S.face_viscosity(m))
    c = tr.Cells(st.lv)
    T0 = hi.conductive_temperature(c.centroid) + 0.05 * hi.grf_eval(c.centroid, 600)
    T, x, its = tr.simulate(st, c, T0, 1e3, 1e-4, 7)
    assert len(its) == 3 and all(i > 0 for i in its)
    assert abs(c.area @ T - c.area @ T0) <= 1e-12 * (c.area @ T0)
    assert np.abs(T - T0).max() > 0


def test_heat_moves_downstream():
    """With the uniform flow u = (1, 0) a temperature bump's first moment in
    x grows: the scheme transports along the velocity (inward normals or a
    downwind choice would move it upstream)."""
    lv = level("annulus64", 4)
    c = tr.Cells(lv)
    F = tr.fluxes(c, np.ones(lv.n_all), np.zeros(lv.n_all))
    T = np.exp(-((c.centroid[:, 0] + 0.2) ** 2 + (c.centroid[:, 1] - 0.7) ** 2) / 0.01)
    dt = 0.5 * c.area.min() / np.abs(F).max()
    T1 = tr.upwind_step(c, T, F, dt)
    m0 = c.area @ (T * c.centroid[:, 0])
    m1 = c.area @ (T1 * c.centroid[:, 0])
    heat = c.area @ T
    assert m1 - m0 > 0.5 * dt * heat
