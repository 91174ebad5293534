"""Pins of oracle pieces that the other oracle tests reach only indirectly
(CPU only): injection of the coefficient to coarse levels, the consistent
mass matrix, and the tap geometry of the learned network's forward pass.

Each pin comes from outside the function it checks: point values of known
functions at known coordinates, exact integrals of polynomials, and the
physical displacement of each stencil tap."""
import numpy as np
import pytest

import hhg_inputs as hi
from oracle import net
from oracle.assemble import assemble, inject
from oracle.mesh import Level, MacroMesh


# ---------------------------------------------------------------- injection

@pytest.mark.parametrize("name", ["square", "annulus64"])
@pytest.mark.parametrize("lf", [2, 4])
def test_inject_samples_the_fine_field_at_the_coarse_points(name, lf):
    """Injection (coarse k of the variable-coefficient operator) takes the
    fine value at the fine point that coincides with each coarse point
    (nested refinement, sec. 3.1).  A field that is a non-symmetric function
    of the coordinates therefore comes out as that function at the coarse
    coordinates; a swapped (I, J), a wrong stride or a wrong edge direction
    puts a value from another place there."""
    m = MacroMesh(*hi.mesh_by_name(name))
    fine, coarse = Level(m, lf), Level(m, lf - 1)

    def field(xy):
        return 0.3 + 1.7 * xy[:, 0] - 0.6 * xy[:, 1] + np.sin(3.1 * xy[:, 0] + 0.4) * xy[:, 1] ** 2

    got = inject(fine, coarse, field(fine.xy))
    assert np.abs(got - field(coarse.xy)).max() < 1e-14


def test_inject_reproduces_a_linear_field_exactly():
    """k = a + b x + c y evaluated at the fine points and injected equals the
    same linear k at the coarse points bit for bit: the fine point 2I of an
    edge with n - 1 = 2 (nc - 1) intervals sits at 2I / (2 (nc - 1)), the
    same rounded quotient as I / (nc - 1)."""
    m = MacroMesh(*hi.annulus(16))
    fine, coarse = Level(m, 3), Level(m, 2)
    lin = lambda xy: 2.0 + 0.75 * xy[:, 0] - 1.25 * xy[:, 1]   # noqa: E731
    assert np.array_equal(inject(fine, coarse, lin(fine.xy)), lin(coarse.xy))


# ---------------------------------------------------------------- mass matrix

@pytest.mark.parametrize("level", [1, 3, 5])
def test_mass_matrix_integrates_linear_products_exactly(level):
    """x^T M y is the integral of the product of the two P1 interpolants
    (sec. 4.2: element matrices of the L2 inner product).  For linear x and
    y the interpolants are the functions themselves, so on the unit square:
    int 1 = 1, int x = 1/2, int x^2 = 1/3, int x y = 1/4, int y^2 = 1/3.
    A lumped (row-sum diagonal) mass matrix gets int x^2 wrong by O(h^2)."""
    lv = Level(MacroMesh(*hi.unit_square()), level)
    M = assemble(lv, want=("M",))["M"]
    one = np.ones(lv.n_all)
    x, y = lv.xy[:, 0], lv.xy[:, 1]
    assert abs(one @ (M @ one) - 1.0) < 1e-14
    assert abs(one @ (M @ x) - 0.5) < 1e-14
    assert abs(x @ (M @ x) - 1.0 / 3.0) < 1e-14
    assert abs(x @ (M @ y) - 0.25) < 1e-14
    assert abs(y @ (M @ y) - 1.0 / 3.0) < 1e-14
    # the lumped alternative fails this pin (the test can tell them apart)
    lumped = np.asarray(M.sum(axis=1)).ravel()
    assert abs(x @ (lumped * x) - 1.0 / 3.0) > 1e-4


def test_mass_matrix_integrates_linear_products_on_the_annulus():
    """The same on the jittered annulus, against the second moments of the
    polygonal domain, computed here over the macro-triangles with the
    three-point edge-midpoint rule (exact for quadratics on a triangle)."""
    m = MacroMesh(*hi.annulus(16))
    lv = Level(m, 3)
    M = assemble(lv, want=("M",))["M"]
    x, y = lv.xy[:, 0], lv.xy[:, 1]
    exact = {"xx": 0.0, "xy": 0.0, "yy": 0.0}
    for t in m.tri:
        P = m.vxy[t]
        area = 0.5 * abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[1, 1] - P[0, 1]) * (P[2, 0] - P[0, 0]))
        mids = 0.5 * (P + np.roll(P, -1, axis=0))
        exact["xx"] += area / 3.0 * (mids[:, 0] ** 2).sum()
        exact["xy"] += area / 3.0 * (mids[:, 0] * mids[:, 1]).sum()
        exact["yy"] += area / 3.0 * (mids[:, 1] ** 2).sum()
    assert abs(x @ (M @ x) - exact["xx"]) < 1e-13
    assert abs(x @ (M @ y) - exact["xy"]) < 1e-13
    assert abs(y @ (M @ y) - exact["yy"]) < 1e-13


def test_mass_matrix_face_interior_row():
    """A face-interior point touches six congruent micro-triangles of area
    |T| = |F| / 4^l: its row of the consistent mass matrix is |T| at the
    centre and |T| / 6 at each of the six neighbours (two triangles share
    each neighbour edge, each giving int phi_p phi_q = |T| / 12)."""
    m = MacroMesh(*hi.annulus(16))
    lv = Level(m, 4)
    M = assemble(lv, want=("M",))["M"].tocsr()
    n = lv.n
    for f in (0, 17, 40):
        P = m.vxy[m.tri[f]]
        areaF = 0.5 * abs((P[1, 0] - P[0, 0]) * (P[2, 1] - P[0, 1]) - (P[1, 1] - P[0, 1]) * (P[2, 0] - P[0, 0]))
        T = areaF / 4 ** lv.level
        loc = lv.loc[f]
        for (i, j) in ((1, 1), (5, 3), (n - 4, 2)):
            p = loc[j, i]
            row = M[p]
            assert row.nnz == 7
            assert abs(M[p, p] - T) < 1e-15
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1), (1, -1), (-1, 1)):
                assert abs(M[p, loc[j + dj, i + di]] - T / 6.0) < 1e-15


# ---------------------------------------------------------------- network taps

def _physical_step(lv, f):
    """Displacements of one micro-step along face-local i and j."""
    x0, x1, x2 = lv.mesh.vxy[lv.mesh.tri[f]]
    return (x1 - x0) / (lv.n - 1), (x2 - x0) / (lv.n - 1)


@pytest.mark.parametrize("s", range(7))
@pytest.mark.parametrize("t", range(7))
def test_forward_tap_geometry(s, t):
    """A unit impulse of rho at point q, one input tap s and one output tap t
    (both weights 1, one hidden channel) yields exactly one non-zero output,
    value 1, at the point p with x(p) = x(q) - d_s - d_t, where d_s is tap
    s's physical displacement (C = 0, E/W = +-step along face-local i, N/S =
    +-step along j, SE = i-step minus j-step, NW its negative).  A flipped
    shift, a transposed tap or a wrong tap table moves the output."""
    lv = Level(MacroMesh(*hi.annulus(16)), 4)
    f = 5
    n = lv.n
    qi, qj = 6, 5                          # at least 3 points inside the face ring
    q = lv.loc[f][qj, qi]
    rho = np.zeros(lv.n_all)
    rho[q] = 1.0
    W1 = np.zeros((net.NCH, 7))
    W2 = np.zeros((net.NCH, 7))
    W1[3, s] = 1.0
    W2[3, t] = 1.0
    out = net.forward(lv, rho, W1, W2)
    nz = np.flatnonzero(out)
    assert len(nz) == 1 and out[nz[0]] == 1.0
    ei, ej = _physical_step(lv, f)
    geo = {"C": 0 * ei, "E": ei, "W": -ei, "N": ej, "S": -ej, "SE": ei - ej, "NW": ej - ei}
    names = ["C", "E", "W", "N", "S", "SE", "NW"]
    want_xy = lv.xy[q] - geo[names[s]] - geo[names[t]]
    assert np.abs(lv.xy[nz[0]] - want_xy).max() < 1e-13
    assert lv.kind[nz[0]] == 2 and lv.prim[nz[0]] == f and n > 8


def test_forward_relu_and_hidden_mask():
    """A negative pre-activation is cut by the ReLU, and hidden values exist
    only on face-interior points: an impulse on a macro-edge point reaches
    the output only through hidden pixels next to it inside the face."""
    lv = Level(MacroMesh(*hi.annulus(16)), 3)
    f = 2
    loc = lv.loc[f]
    rho = np.zeros(lv.n_all)
    rho[loc[3, 2]] = 1.0
    W1 = np.zeros((net.NCH, 7))
    W2 = np.zeros((net.NCH, 7))
    W1[0, 0], W2[0, 0] = -1.0, 1.0
    assert not net.forward(lv, rho, W1, W2).any()
    # impulse on the side j = 0 (an edge point): with centre-only weights
    # nothing reaches the output (no hidden pixel on the edge) ...
    rho = np.zeros(lv.n_all)
    rho[loc[0, 3]] = 1.0
    W1[0, 0] = 1.0
    assert not net.forward(lv, rho, W1, W2).any()
    # ... but the S tap of the hidden pixel (3, 1) reads it (the ring holds
    # the edge values), and the centre output tap puts it at (3, 1)
    W1[0, 0], W1[0, 4] = 0.0, 1.0
    out = net.forward(lv, rho, W1, W2)
    assert np.flatnonzero(out).tolist() == [loc[1, 3]]


def test_forward_equals_pointwise_sum_with_random_weights():
    """out(p) = sum_c sum_t W2[c,t] relu(sum_s W1[c,s] rho(p + d_t + d_s))
    with the hidden value zero off the face interior, evaluated point by
    point through coordinates: each neighbour is found by its physical
    position x(p) + d, not by index arithmetic."""
    lv = Level(MacroMesh(*hi.annulus(16)), 3)
    rng = np.random.default_rng(9)
    W1 = rng.standard_normal((net.NCH, 7))
    W2 = rng.standard_normal((net.NCH, 7))
    rho = rng.uniform(-1.0, 1.0, lv.n_all)
    out = net.forward(lv, rho, W1, W2)
    names = ["C", "E", "W", "N", "S", "SE", "NW"]
    for f in range(0, lv.mesh.F, 9):
        ei, ej = _physical_step(lv, f)
        geo = {"C": 0 * ei, "E": ei, "W": -ei, "N": ej, "S": -ej, "SE": ei - ej, "NW": ej - ei}
        face_pts = np.flatnonzero(lv.loc[f] >= 0)
        ids = lv.loc[f].ravel()[face_pts]
        inter = set(np.flatnonzero((lv.kind == 2) & (lv.prim == f)).tolist())

        def at(x):
            d = np.abs(lv.xy[ids] - x).sum(1)
            k = int(np.argmin(d))
            return int(ids[k]) if d[k] < 1e-12 else None

        for p in sorted(inter)[::3]:
            acc = 0.0
            for c in range(net.NCH):
                for t in range(7):
                    hp = at(lv.xy[p] + geo[names[t]])
                    if hp is None or hp not in inter:
                        continue
                    a = 0.0
                    for s in range(7):
                        rp = at(lv.xy[hp] + geo[names[s]])
                        if rp is not None:
                            a += W1[c, s] * rho[rp]
                    acc += W2[c, t] * max(a, 0.0)
            assert abs(out[p] - acc) <= 1e-12 * (1.0 + abs(acc))
