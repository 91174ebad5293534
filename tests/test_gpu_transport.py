"""GPU parity of the energy-transport coupling (finite-volume upwind step on
the cells, buoyancy load, the coupled Stokes/transport loop) against the
oracle, through the C ABI.  FP64: 1e-12 relative (max norm) for a step and
for the load; the coupled loop follows the oracle's MINRES iterates, so its
temperature after several steps agrees to 1e-10."""
import numpy as np
import pytest

import hhg_inputs as hi
from gpu_util import log, rel_err, to_np

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12
_CACHE = {}


def setup(name, L):
    import paper_1805_10167_amd as P
    from oracle import stokes as S
    from oracle import transport as tr
    from oracle.mesh import MacroMesh
    key = (name, L)
    if key not in _CACHE:
        vxy, tri = hi.mesh_by_name(name)
        m = MacroMesh(vxy, tri)
        mu = np.ones(m.F) if name == "square" else S.face_viscosity(m)
        st = S.Stokes(m, L, 2, mu)
        g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_STOKES)
        P.hhg_stokes_setup(g.h, mu, S.DELTA)
        _CACHE[key] = (g, st, tr.Cells(st.lv))
    return _CACHE[key]


def cells_to_np(g, L, T):
    import torch
    n_cells = g.F * (2 ** L) ** 2
    out = torch.zeros(n_cells, dtype=torch.float64, device="cuda")
    import paper_1805_10167_amd as P
    P.hhg_cells_to_canonical(g.h, L, T, out)
    return to_np(out)


def cells_from_np(g, L, Tc):
    import torch

    import paper_1805_10167_amd as P
    T = torch.zeros(2 * P.hhg_field_elems(g.h, L), dtype=torch.float64, device="cuda")
    P.hhg_cells_from_canonical(g.h, L, torch.tensor(Tc, dtype=torch.float64, device="cuda"), T)
    return T


CASES = [("annulus64", 4), ("annulus64", 6), ("square", 5), ("annulus128", 4)]


@pytest.mark.parametrize("name,L", CASES)
def test_cell_layout_roundtrip(name, L):
    g, st, c = setup(name, L)
    Tc = hi.uniform_vector(c.C, 3)
    assert np.array_equal(cells_to_np(g, L, cells_from_np(g, L, Tc)), Tc)


@pytest.mark.parametrize("name,L", CASES)
def test_upwind_step(name, L):
    """One step with a random velocity (zero on the boundary) and random T."""
    import paper_1805_10167_amd as P
    from oracle import transport as tr
    log("upwind step %s L=%d" % (name, L))
    g, st, c = setup(name, L)
    lv = st.lv
    rng = np.random.default_rng(7)
    ux, uy = rng.uniform(-1, 1, lv.n_all), rng.uniform(-1, 1, lv.n_all)
    ux[lv.dirichlet] = 0.0
    uy[lv.dirichlet] = 0.0
    Tc = hi.uniform_vector(c.C, 8)
    dt = 0.2 * c.area.min() / np.abs(tr.fluxes(c, ux, uy)).max()
    x = g.stokes_from_canonical(L, np.concatenate([ux, uy, np.zeros(lv.n_all)]))
    import torch
    T = cells_from_np(g, L, Tc)
    T2 = torch.zeros_like(T)
    P.hhg_transport_step(g.h, L, x, T, T2, dt)
    got = cells_to_np(g, L, T2)
    ref = tr.upwind_step(c, Tc, tr.fluxes(c, ux, uy), dt)
    err = rel_err(got, ref)
    log("  rel err %.2e; heat change %.2e" % (err, abs(c.area @ got - c.area @ Tc) / (c.area @ np.abs(Tc))))
    assert err <= F64_TOL
    assert abs(c.area @ got - c.area @ Tc) <= 1e-13 * (c.area @ np.abs(Tc))


@pytest.mark.parametrize("name,L", CASES)
def test_buoyancy_load(name, L):
    import paper_1805_10167_amd as P
    from oracle import transport as tr
    g, st, c = setup(name, L)
    lv = st.lv
    Tc = hi.uniform_vector(c.C, 9, 0.0, 1.0)
    b = g.stokes_vector(L)
    P.hhg_buoyancy(g.h, L, cells_from_np(g, L, Tc), 7.5, b)
    bx, by = tr.buoyancy(lv, c, Tc, 7.5)
    got = to_np(g.stokes_to_canonical(L, b))
    ref = np.concatenate([bx, by, np.zeros(lv.n_all)])
    assert rel_err(got, ref) <= F64_TOL
    # copies are consistent: the Stokes residual against b with x = 0 is b
    r = g.stokes_vector(L)
    P.hhg_stokes_residual(g.h, L, g.stokes_vector(L), b, r)
    assert rel_err(to_np(g.stokes_to_canonical(L, r)), ref) <= F64_TOL


@pytest.mark.parametrize("name,L", [("annulus64", 4), ("annulus128", 4)])
def test_coupled_loop(name, L):
    """Seven steps (Stokes solves before steps 0, 3 and 6) from the conductive
    profile plus a random perturbation, against the oracle's loop."""
    import paper_1805_10167_amd as P
    from oracle import transport as tr
    log("coupled loop %s L=%d" % (name, L))
    g, st, c = setup(name, L)
    T0 = hi.conductive_temperature(c.centroid) + 0.05 * hi.grf_eval(c.centroid, 600)
    Ra, dt, steps = 1e3, 2e-5, 7
    To, xo, its = tr.simulate(st, c, T0, Ra, dt, steps)
    T = cells_from_np(g, L, T0)
    x = g.stokes_vector(L)
    rc, stats = P.hhg_energy_run(g.h, x, T, Ra=Ra, dt=dt, steps=steps, stokes_every=3, rtol=1e-8)
    log("  stokes solves %d, MINRES iterations %d (oracle %s)" % (stats["stokes_solves"],
                                                                   stats["minres_iters"], its))
    assert rc == 0 and stats["steps"] == steps and stats["stokes_solves"] == 3
    assert stats["minres_iters"] == sum(its)
    eT = rel_err(cells_to_np(g, L, T), To)
    ex = rel_err(to_np(g.stokes_to_canonical(L, x)), xo)
    log("  T rel err %.2e, flow rel err %.2e" % (eT, ex))
    assert eT <= 1e-10 and ex <= 1e-8
    assert abs(c.area @ cells_to_np(g, L, T) - c.area @ T0) <= 1e-12 * (c.area @ T0)


def test_full_size_step_and_load():
    """The benchmark's configuration (256-face annulus, level 6, about a
    million cells): one upwind step with a random flow and the buoyancy load,
    element by element against the oracle."""
    import torch

    import paper_1805_10167_amd as P
    from oracle import stokes as S
    from oracle import transport as tr
    from oracle.mesh import Level, MacroMesh
    L = 6
    vxy, tri = hi.annulus(n_tan=64)
    log("full-size transport: %d faces, level %d" % (len(tri), L))
    lv = Level(MacroMesh(vxy, tri), L)
    c = tr.Cells(lv)
    g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_STOKES)
    P.hhg_stokes_setup(g.h, np.ones(len(tri)), S.DELTA)
    rng = np.random.default_rng(11)
    ux, uy = rng.uniform(-1, 1, lv.n_all), rng.uniform(-1, 1, lv.n_all)
    ux[lv.dirichlet] = 0.0
    uy[lv.dirichlet] = 0.0
    Fl = tr.fluxes(c, ux, uy)
    dt = 0.2 * c.area.min() / np.abs(Fl).max()
    Tc = hi.conductive_temperature(c.centroid) + 0.05 * hi.grf_eval(c.centroid, 600)
    x = g.stokes_from_canonical(L, np.concatenate([ux, uy, np.zeros(lv.n_all)]))
    T = cells_from_np(g, L, Tc)
    T2 = torch.zeros_like(T)
    P.hhg_transport_step(g.h, L, x, T, T2, dt)
    err = rel_err(cells_to_np(g, L, T2), tr.upwind_step(c, Tc, Fl, dt))
    log("  step rel err %.2e" % err)
    assert err <= F64_TOL
    b = g.stokes_vector(L)
    P.hhg_buoyancy(g.h, L, T, 1e4, b)
    bx, by = tr.buoyancy(lv, c, Tc, 1e4)
    err = rel_err(to_np(g.stokes_to_canonical(L, b)), np.concatenate([bx, by, np.zeros(lv.n_all)]))
    log("  load rel err %.2e" % err)
    assert err <= F64_TOL


def test_buoyancy_with_more_tiles_than_face_blocks():
    """Level 8 of the 64-face annulus (10,560 face tiles against 8,192 face
    blocks): the load of T = 1 is -Ra r_hat_i times the integral of phi_i,
    the row sum of the consistent mass matrix."""
    import torch

    import paper_1805_10167_amd as P
    from oracle import stokes as S
    from oracle.assemble import assemble
    from oracle.mesh import Level, MacroMesh
    L = 8
    vxy, tri = hi.mesh_by_name("annulus64")
    lv = Level(MacroMesh(vxy, tri), L)
    mrow = np.asarray(assemble(lv, want=("M",))["M"].sum(axis=1)).ravel()
    g = P.Mesh(vxy, tri, L, 2, P.HHG_FEAT_F64 | P.HHG_FEAT_MP | P.HHG_FEAT_STOKES)
    P.hhg_stokes_setup(g.h, np.ones(len(tri)), S.DELTA)
    T = torch.ones(2 * P.hhg_field_elems(g.h, L), dtype=torch.float64, device="cuda")
    b = g.stokes_vector(L)
    P.hhg_buoyancy(g.h, L, T, 3.0, b)
    r = np.hypot(lv.xy[:, 0], lv.xy[:, 1])
    ref = np.concatenate([-3.0 * mrow * lv.xy[:, 0] / r, -3.0 * mrow * lv.xy[:, 1] / r, np.zeros(lv.n_all)])
    ref[:lv.n_all][lv.dirichlet] = 0.0
    ref[lv.n_all:2 * lv.n_all][lv.dirichlet] = 0.0
    err = rel_err(to_np(g.stokes_to_canonical(L, b)), ref)
    log("buoyancy of T = 1 at annulus64 L=%d: rel err %.2e" % (L, err))
    assert err <= F64_TOL
