"""Pins of the reference's triquadratic (Q2) elements.

Closed forms come from exact rational integrals of the 1D Lagrange quadratics
(written here from their definition, not from the reference's code), the
3-point Gauss rule's degree of exactness, invariants of the weak form, and
central differences.
"""
import itertools
from fractions import Fraction as Fr

import numpy as np
import pytest

from paper_2009_00706_amd import inputs as I


@pytest.fixture(scope="module")
def q2(oracle):
    from oracle import q2
    return q2


# --- exact 1D integrals of the quadratic Lagrange basis of the nodes 0, h/2, h
def _lagrange_polys():
    """Coefficients (ascending powers of t in [0, 1]) of the three Lagrange
    quadratics of the nodes 0, 1/2, 1, as Fractions."""
    nodes = [Fr(0), Fr(1, 2), Fr(1)]
    out = []
    for a in range(3):
        poly = [Fr(1)]
        for b in range(3):
            if b == a:
                continue
            # poly * (t - t_b) / (t_a - t_b)
            nxt = [Fr(0)] * (len(poly) + 1)
            for i, c in enumerate(poly):
                nxt[i + 1] += c
                nxt[i] -= nodes[b] * c
            den = nodes[a] - nodes[b]
            poly = [c / den for c in nxt]
        out.append(poly)
    return out


def _deriv(p):
    return [i * c for i, c in enumerate(p)][1:]


def _int01(p, q):
    prod = [Fr(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            prod[i + j] += a * b
    return sum(c / (k + 1) for k, c in enumerate(prod))


def one_d(h):
    """{(da, db): int_0^h D^da phi_a D^db phi_b dx} as float 3x3 arrays."""
    P = _lagrange_polys()
    D = [_deriv(p) for p in P]
    out = {}
    for da, db in itertools.product((0, 1), repeat=2):
        m = np.zeros((3, 3))
        for a, b in itertools.product(range(3), repeat=2):
            v = _int01(D[a] if da else P[a], D[b] if db else P[b])
            m[a, b] = float(v) * h * (1.0 / h) ** (da + db)
        out[(da, db)] = m
    return out


def integral(h, da, db):
    """int D^da N_a D^db N_b over a cube of side h (27 x 27), da/db an axis or None."""
    T = one_d(h)
    out = np.ones((27, 27))
    for a, b in itertools.product(range(27), range(27)):
        ia = (a % 3, (a // 3) % 3, a // 9)
        ib = (b % 3, (b // 3) % 3, b // 9)
        v = 1.0
        for d in range(3):
            v *= T[(int(da == d), int(db == d))][ia[d], ib[d]]
        out[a, b] = v
    return out


def blocks(J):
    return J.reshape(27, 4, 27, 4).transpose(1, 3, 0, 2)


def test_one_d_matrices_are_the_textbook_ones():
    # the 1D quadratic mass and stiffness matrices (nodes 0, h/2, h)
    h = 0.3
    T = one_d(h)
    np.testing.assert_allclose(T[(0, 0)], h / 30 * np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]), atol=1e-16)
    np.testing.assert_allclose(T[(1, 1)], 1 / (3 * h) * np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]),
                               atol=1e-14)


def test_three_point_gauss_exact_to_degree_five(q2):
    xi, w = q2.points()
    assert abs(w.sum() - 8.0) < 1e-15
    for a, b, c in itertools.product(range(6), repeat=3):
        exact = np.prod([(1 - (-1) ** (e + 1)) / (e + 1) for e in (a, b, c)])
        got = np.sum(w * xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c)
        assert abs(got - exact) < 1e-14, (a, b, c)
    # and not to degree 6
    assert abs(np.sum(w * xi[:, 0] ** 6) - 4 * 2 / 7) > 1e-3


def _elem(oracle, q2, h, seed=0, **kw):
    prm = oracle.params(**kw)
    rng = np.random.default_rng(seed)
    return prm, rng.normal(size=(27, 4)), rng.normal(size=(27, 3))


def test_q2_mass_term_closed_form(oracle, q2):
    h = 0.25
    prm, U, U0 = _elem(oracle, q2, h, rho=1.3, dt=0.02, term_mask=1 << 0)
    R, J = q2.element(prm, h, U, U0)
    B = blocks(J)
    M = integral(h, None, None)
    for i, j in itertools.product(range(4), range(4)):
        ref = (1.3 / 0.02) * M if (i == j and i < 3) else 0 * M
        np.testing.assert_allclose(B[i][j], ref, rtol=1e-13, atol=1e-15)
    for i in range(3):
        np.testing.assert_allclose(R.reshape(27, 4)[:, i], (1.3 / 0.02) * M @ (U[:, i] - U0[:, i]),
                                   rtol=1e-12, atol=1e-14)
    # total of the mass matrix is the element volume
    assert abs(M.sum() - h ** 3) < 1e-15


def test_q2_viscous_term_closed_form(oracle, q2):
    h = 0.3
    prm, U, U0 = _elem(oracle, q2, h, mu=0.7, theta=1.0, term_mask=1 << 2)
    R, J = q2.element(prm, h, U, U0)
    B = blocks(J)
    L = sum(integral(h, k, k) for k in range(3))
    for i, j in itertools.product(range(3), range(3)):
        ref = 0.7 * ((i == j) * L + integral(h, j, i))
        np.testing.assert_allclose(B[i][j], ref, atol=1e-13)
    u = U[:, :3]
    for i in range(3):
        np.testing.assert_allclose(R.reshape(27, 4)[:, i], sum(B[i][j] @ u[:, j] for j in range(3)), atol=1e-12)


def test_q2_pressure_and_continuity_blocks(oracle, q2):
    h = 0.25
    prm, U, U0 = _elem(oracle, q2, h, theta=0.5, term_mask=(1 << 3) | (1 << 4))
    R, J = q2.element(prm, h, U, U0)
    B = blocks(J)
    for i in range(3):
        np.testing.assert_allclose(B[i][3], -integral(h, i, None), atol=1e-15)
        np.testing.assert_allclose(B[3][i], 0.5 * integral(h, None, i), atol=1e-15)
    np.testing.assert_allclose(B[3][3], 0, atol=1e-15)


def test_q2_rest_state_jacobian_closed_form(oracle, q2):
    h, dt, rho, th = 0.2, 0.05, 1.0, 0.5
    prm = oracle.params(rho=rho, mu=0.0, dt=dt, theta=th)
    R, J = q2.element(prm, h, np.zeros((27, 4)), np.zeros((27, 3)))
    assert np.abs(R).max() == 0
    B = blocks(J)
    tauM = dt / 2
    tauC = h ** 2 / (6 * dt)
    M = integral(h, None, None)
    L = sum(integral(h, k, k) for k in range(3))
    for i, j in itertools.product(range(3), range(3)):
        ref = (rho / dt) * M * (i == j) + rho * tauC * th * integral(h, i, j)
        np.testing.assert_allclose(B[i][j], ref, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(B[i][3], -integral(h, i, None), atol=1e-14)
        np.testing.assert_allclose(B[3][j], th * integral(h, None, j) + tauM / dt * integral(h, j, None),
                                   atol=1e-14)
    np.testing.assert_allclose(B[3][3], tauM / rho * L, atol=1e-14)


def test_q2_jacobian_matches_frozen_tau_finite_differences(oracle, q2):
    h = 0.15
    prm, U, U0 = _elem(oracle, q2, h, seed=3)
    U *= 0.5
    R, J = q2.element(prm, h, U, U0)
    d = 1e-6
    rng = np.random.default_rng(4)
    for col in rng.choice(108, 24, replace=False):
        e = np.zeros(108)
        e[col] = d
        fd = (q2.element_frozen(prm, h, U.ravel(), U.ravel() + e, U0) -
              q2.element_frozen(prm, h, U.ravel(), U.ravel() - e, U0)) / (2 * d)
        np.testing.assert_allclose(J[:, col], fd, rtol=1e-6, atol=1e-6 * np.abs(J).max())


def _uniform(level):
    t = I.uniform_octree(level)
    return t


def test_q2_mesh_counts_and_pattern(q2):
    t = _uniform(2)
    m = q2.derive_q2_mesh(t)
    assert m.n_nodes == 9 ** 3 and m.el_node.shape == (64, 27)
    # node rows: a vertex node of the interior couples with 5^3 nodes, a cell
    # centre with the 27 nodes of its element
    deg = np.diff(m.row_ptr)[::4] // 4
    xyz = m.node_xyz_half
    interior = np.all((xyz > 0) & (xyz < xyz.max()), axis=1)
    s2 = 2 * int(t.side()[0])          # element side in half units
    vertex = np.all(xyz % s2 == 0, axis=1)
    centre = np.all(xyz % s2 == s2 // 2, axis=1)
    assert vertex.sum() == 5 ** 3 and centre.sum() == 64
    assert (deg[interior & vertex] == 125).all() and (deg[centre] == 27).all()
    # columns ascending within a row
    for r in range(0, 4 * m.n_nodes, 37):
        c = m.col_idx[m.row_ptr[r]:m.row_ptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    with pytest.raises(ValueError):
        c = (0.5 + I.BODY_OFFSET[0], 0.5, 0.5)
        q2.derive_q2_mesh(I.sphere_refined_octree(c, 0.3, 2, 3, 1.0))


def test_q2_constant_state_zero_residual_and_mass_total(oracle, q2):
    t = _uniform(2)
    m = q2.derive_q2_mesh(t)
    n = m.n_nodes
    const = {"ux": np.full(n, 0.3), "uy": np.full(n, -0.7), "uz": np.full(n, 0.2), "p": np.zeros(n)}
    const.update({"ux0": const["ux"].copy(), "uy0": const["uy"].copy(), "uz0": const["uz"].copy()})
    _, R = q2.assemble(t, m, const, vals=False)
    assert np.abs(R).max() < 1e-15
    # mass term with a unit jump in u_x: the x rows sum to rho/dt times the domain volume
    jump = dict(const)
    jump["ux"] = const["ux"] + 1.0
    _, R = q2.assemble(t, m, jump, prm=oracle.params(rho=1.1, dt=0.05, term_mask=1 << 0), vals=False)
    assert abs(R[0::4].sum() - 1.1 / 0.05) < 1e-12


def test_q2_patch_test_viscous_harmonic_field(oracle, q2):
    """u = (x^2 - y^2, -2xy, 0) is harmonic and divergence free: the viscous
    rows of interior nodes vanish (the weak Laplacian of a harmonic field of the
    discrete space, integrated exactly)."""
    t = _uniform(2)
    m = q2.derive_q2_mesh(t)
    x = q2.node_xyz(t, m)
    u = np.stack([x[:, 0] ** 2 - x[:, 1] ** 2, -2 * x[:, 0] * x[:, 1], 0 * x[:, 0]], 1)
    f = {"ux": u[:, 0], "uy": u[:, 1], "uz": u[:, 2], "p": np.zeros(m.n_nodes)}
    f.update({"ux0": f["ux"], "uy0": f["uy"], "uz0": f["uz"]})
    _, R = q2.assemble(t, m, f, prm=oracle.params(mu=0.9, theta=1.0, term_mask=1 << 2), vals=False)
    xyz = m.node_xyz_half
    interior = np.all((xyz > 0) & (xyz < xyz.max()), axis=1)
    Rr = R.reshape(-1, 4)
    assert np.abs(Rr[interior, :3]).max() < 1e-14
    assert np.abs(Rr[~interior, :3]).max() > 1e-3     # the boundary rows are not zero


# uniform flow u = u_prev = c, p linear: grad u = 0, u' = -tau_M grad p constant
UF = dict(h=0.2, dt=0.05, mu=0.03, rho=1.3, th=0.5, c=np.array([0.6, -0.9, 0.4]),
          g=np.array([0.7, -0.4, 1.3]))


def _uf(oracle, q2, bit):
    h, dt, mu, rho, th, c, g = (UF[k] for k in ("h", "dt", "mu", "rho", "th", "c", "g"))
    nodes = np.array([[(a % 3) / 2, ((a // 3) % 3) / 2, (a // 9) / 2] for a in range(27)]) * h
    U = np.zeros((27, 4)); U[:, :3] = c; U[:, 3] = nodes @ g + 0.2
    prm = oracle.params(rho=rho, mu=mu, dt=dt, theta=th, term_mask=1 << bit)
    R, J = q2.element(prm, h, U, np.tile(c, (27, 1)))
    nu = mu / rho
    tauM = (4 / dt ** 2 + 4 * (c @ c) / h ** 2 + 36 * nu ** 2 * 48 / h ** 4) ** -0.5
    up = -tauM * g
    return R.reshape(27, 4), blocks(J), tauM, up, h / (2 * np.linalg.norm(up))


def test_q2_supg_cross_taubar_uniform_flow(oracle, q2):
    h, dt, rho, th, c = (UF[k] for k in ("h", "dt", "rho", "th", "c"))
    # SUPG / PSPG (term 5)
    R, B, tauM, up, tb = _uf(oracle, q2, 5)
    gradN = np.stack([integral(h, k, None).sum(1) for k in range(3)], 1)
    for i in range(3):
        np.testing.assert_allclose(R[:, i], -(gradN @ c) * up[i], rtol=1e-12, atol=1e-16)
    np.testing.assert_allclose(R[:, 3], -(1 / rho) * gradN @ up, rtol=1e-12, atol=1e-16)
    cN = sum(c[k] * integral(h, k, None) for k in range(3))
    cc = sum(c[k] * c[l] * integral(h, k, l) for k in range(3) for l in range(3))
    sc = 1e-12 * max(np.abs(B[i][j]).max() for i in range(4) for j in range(4))
    for i, j in itertools.product(range(3), range(3)):
        ref = -th * up[i] * integral(h, j, None) + (i == j) * tauM * rho * (cN / dt + th * cc)
        np.testing.assert_allclose(B[i][j], ref, rtol=0, atol=sc)
    # cross stress (term 7) and tau-bar term (term 9): zero residual, closed-form Jacobian
    for bit, ref in ((7, th * sum(up[k] * integral(h, None, k) for k in range(3))),
                     (9, tb * th * sum(up[k] * up[l] * integral(h, k, l) for k in range(3) for l in range(3)))):
        R, B, *_ = _uf(oracle, q2, bit)
        assert np.abs(R).max() < 1e-16
        for i, j in itertools.product(range(4), range(4)):
            np.testing.assert_allclose(B[i][j], ref if (i == j and i < 3) else 0 * ref, rtol=0,
                                       atol=1e-12 * np.abs(ref).max())
