"""Pins of the CPU reference against what the paper and the mathematics fix.

Each test checks the reference against something other than itself: printed
values of the paper, closed forms from exact 1D integrals, invariants, exact
rational arithmetic, brute force, or analytic point sets.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_2009_00706_amd import inputs as I

# ---------------------------------------------------------------------------
# exact element integrals of trilinear basis functions (closed forms)
# ---------------------------------------------------------------------------


def _1d(h):
    s = [-1.0, 1.0]
    I00 = np.array([[h / 3, h / 6], [h / 6, h / 3]])                 # int phi_a phi_b
    I10 = np.array([[s[a] / 2 for b in range(2)] for a in range(2)])  # int phi_a' phi_b
    I01 = I10.T.copy()                                                # int phi_a phi_b'
    I11 = np.array([[s[a] * s[b] / h for b in range(2)] for a in range(2)])
    return {(0, 0): I00, (1, 0): I10, (0, 1): I01, (1, 1): I11}


def integral(h, da, db):
    """int D^da N_a D^db N_b over a cube of side h; da, db: derivative axis or None."""
    T = _1d(h)
    out = np.ones((8, 8))
    for a, b in itertools.product(range(8), range(8)):
        v = 1.0
        for d in range(3):
            ia, ib = (a >> d) & 1, (b >> d) & 1
            v *= T[(int(da == d), int(db == d))][ia, ib]
        out[a, b] = v
    return out


def blocks(J):
    """J[(a,i),(b,j)] -> B[i][j][a,b]"""
    return J.reshape(8, 4, 8, 4).transpose(1, 3, 0, 2)


def one_element(oracle, h=0.3, seed=0, **kw):
    prm = oracle.params(**kw)
    xi, w = oracle.std_points(h)
    rng = np.random.default_rng(seed)
    U = rng.normal(size=(8, 4))
    U0 = rng.normal(size=(8, 3))
    return prm, xi, w, U, U0


# ---------------------------------------------------------------------------
# Quadrature tables and scalings (Fig. GP; scale factors of Alg. 6's text)
# ---------------------------------------------------------------------------


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _sketch():
    """The printed values of the adaptive-quadrature sketch (tests/golden)."""
    vals, points = {}, []
    with open(os.path.join(GOLDEN, "adaptive_quadrature_sketch.txt")) as fh:
        for line in fh:
            f = line.split("#", 1)[0].split()
            if not f:
                continue
            if f[0] == "point":
                points.append((int(f[1]), float(f[2]), float(f[3])))
            else:
                vals[f[0]] = (float(f[1]), int(f[2]))
    return vals, points


def test_gauss_abscissae_match_paper(oracle):
    # printed [0,1] abscissae of the Gauss-point figure, to their printed digits
    vals, _ = _sketch()
    for name, g in (("g_minus", oracle.G_MINUS), ("g_plus", oracle.G_PLUS)):
        v, digits = vals[name]
        assert abs(g - v) <= 0.5 * 10.0 ** -digits
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    s3 = Decimal(3).sqrt()
    for g, true in ((oracle.G_MINUS, (1 - 1 / s3) / 2), (oracle.G_PLUS, (1 + 1 / s3) / 2),
                    (oracle.XI, 1 / s3)):
        assert abs(Decimal(g) - true) <= Decimal(float(np.spacing(g))) / 2   # correctly rounded


def test_two_point_gauss_integrates_cubics_exactly(oracle):
    h = 0.375
    xi, w = oracle.std_points(h)
    x = (xi + 1) * h / 2
    for a, b, c in itertools.product(range(4), repeat=3):
        exact = h ** (a + 1) / (a + 1) * h ** (b + 1) / (b + 1) * h ** (c + 1) / (c + 1)
        q = np.sum(w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c)
        assert abs(q - exact) <= 1e-15 * max(1.0, exact) + 1e-18


def test_laplacian_closed_form_and_scale(oracle):
    # stiffness = sum_k Op(dphi/dk) Op(dphi/dk) (App. A), scale dx/2
    h = 0.3
    L = sum(integral(h, k, k) for k in range(3))
    for a, b in itertools.product(range(8), range(8)):
        ndiff = bin(a ^ b).count("1")
        ref = {0: 4, 1: 0, 2: -1, 3: -1}[ndiff] * h / 12
        assert abs(L[a, b] - ref) < 1e-15
    prm, xi, w, U, U0 = one_element(oracle, h, mu=0.7, theta=1.0, term_mask=1 << 2)
    R, J = oracle.element(prm, h, xi, w, np.eye(8), U, U0)
    B = blocks(J)
    for i, j in itertools.product(range(3), range(3)):
        ref = 0.7 * ((i == j) * L + integral(h, j, i))
        np.testing.assert_allclose(B[i][j], ref, atol=1e-14)
    # residual of the viscous term is linear: R = J u (theta = 1)
    u = U[:, :3]
    for i in range(3):
        ri = sum(B[i][j] @ u[:, j] for j in range(3))
        np.testing.assert_allclose(R.reshape(8, 4)[:, i], ri, atol=1e-13)


def test_mass_closed_form_row_sums(oracle):
    h = 0.3
    M = integral(h, None, None)
    for a, b in itertools.product(range(8), range(8)):
        ndiff = bin(a ^ b).count("1")
        assert abs(M[a, b] - {0: 8, 1: 4, 2: 2, 3: 1}[ndiff] * h ** 3 / 216) < 1e-16
    np.testing.assert_allclose(M.sum(1), h ** 3 / 8)
    prm, xi, w, U, U0 = one_element(oracle, h, rho=1.3, dt=0.02, term_mask=1 << 0)
    R, J = oracle.element(prm, h, xi, w, np.eye(8), U, U0)
    B = blocks(J)
    for i, j in itertools.product(range(4), range(4)):
        ref = (1.3 / 0.02) * M if (i == j and i < 3) else 0 * M
        np.testing.assert_allclose(B[i][j], ref, rtol=1e-14, atol=1e-14)
    Rr = R.reshape(8, 4)
    for i in range(3):
        np.testing.assert_allclose(Rr[:, i], (1.3 / 0.02) * M @ (U[:, i] - U0[:, i]), rtol=1e-13)
    # total of the mass term = (rho/dt) * element volume for a unit jump
    assert abs(B[0][0].sum() - (1.3 / 0.02) * h ** 3) < 1e-12


def test_pressure_and_continuity_blocks(oracle):
    h = 0.25
    prm, xi, w, U, U0 = one_element(oracle, h, theta=0.5, term_mask=(1 << 3) | (1 << 4))
    R, J = oracle.element(prm, h, xi, w, np.eye(8), U, U0)
    B = blocks(J)
    for i in range(3):
        np.testing.assert_allclose(B[i][3], -integral(h, i, None), atol=1e-15)
        np.testing.assert_allclose(B[3][i], 0.5 * integral(h, None, i), atol=1e-15)
    np.testing.assert_allclose(B[3][3], 0, atol=1e-15)


def test_convection_linearisation_constant_state(oracle):
    # u = u_prev = c: residual of convection 0, Jacobian rho theta delta_ij int N_a c.grad N_b
    h, c = 0.2, np.array([0.3, -1.1, 0.7])
    prm = oracle.params(rho=1.7, theta=0.5, term_mask=1 << 1)
    xi, w = oracle.std_points(h)
    U = np.zeros((8, 4)); U[:, :3] = c
    U0 = np.tile(c, (8, 1))
    R, J = oracle.element(prm, h, xi, w, np.eye(8), U, U0)
    assert np.abs(R).max() < 1e-15
    ref = 1.7 * 0.5 * sum(c[k] * integral(h, None, k) for k in range(3))
    B = blocks(J)
    for i, j in itertools.product(range(3), range(3)):
        np.testing.assert_allclose(B[i][j], ref if i == j else 0 * ref, atol=1e-14)


def test_tau_closed_form(oracle):
    h, dt, mu, rho = 0.1, 0.01, 0.02, 1.0
    prm = oracle.params(rho=rho, mu=mu, dt=dt)
    xi, _ = oracle.std_points(h)
    t = oracle.taus(prm, h, xi, np.zeros((8, 4)), np.zeros((8, 3)))
    nu = mu / rho
    tauM = (4 / dt ** 2 + 36 * nu ** 2 * 48 / h ** 4) ** -0.5
    np.testing.assert_allclose(t[:, 0], tauM, rtol=1e-15)
    np.testing.assert_allclose(t[:, 1], 1 / (tauM * 12 / h ** 2), rtol=1e-15)
    assert np.all(t[:, 2] == 0)      # u' = 0: the tau-bar term vanishes
    # with a uniform velocity u.G.u = 4|u|^2/h^2 enters tau_M
    u = np.array([0.5, -0.25, 1.0])
    Uv = np.zeros((8, 4)); Uv[:, :3] = u
    t = oracle.taus(prm, h, xi, Uv, np.tile(u, (8, 1)))
    tauM = (4 / dt ** 2 + 4 * (u @ u) / h ** 2 + 36 * nu ** 2 * 48 / h ** 4) ** -0.5
    np.testing.assert_allclose(t[:, 0], tauM, rtol=1e-15)


def test_rest_state_jacobian_closed_form(oracle):
    # u = u_prev = 0, p = 0, mu = 0: all fine scales vanish; every block is closed form
    h, dt, rho, th = 0.2, 0.05, 1.0, 0.5
    prm = oracle.params(rho=rho, mu=0.0, dt=dt, theta=th)
    xi, w = oracle.std_points(h)
    R, J = oracle.element(prm, h, xi, w, np.eye(8), np.zeros((8, 4)), np.zeros((8, 3)))
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


def test_linear_pressure_state_residual(oracle):
    # u = u_prev = 0, p linear: u' = -tau_M grad p (constant)
    h, dt, mu, rho = 0.25, 0.01, 0.01, 1.0
    prm = oracle.params(rho=rho, mu=mu, dt=dt)
    xi, w = oracle.std_points(h)
    g = np.array([0.7, -0.4, 1.3])
    corners = np.array([[(a >> d) & 1 for d in range(3)] for a in range(8)]) * h
    U = np.zeros((8, 4)); U[:, 3] = corners @ g + 0.2
    R, _ = oracle.element(prm, h, xi, w, np.eye(8), U, np.zeros((8, 3)))
    R = R.reshape(8, 4)
    nu = mu / rho
    tauM = (4 / dt ** 2 + 36 * nu ** 2 * 48 / h ** 4) ** -0.5
    L = sum(integral(h, k, k) for k in range(3))
    np.testing.assert_allclose(R[:, 3], tauM / rho * L @ U[:, 3], rtol=1e-12, atol=1e-15)
    up = -tauM * g
    gradN = np.stack([integral(h, k, None).sum(1) for k in range(3)], 1)   # int d_k N_a
    for i in range(3):
        ref = -integral(h, i, None) @ U[:, 3] - (1 / rho) * (gradN @ up) * up[i]
        np.testing.assert_allclose(R[:, i], ref, rtol=1e-12, atol=1e-15)


def test_jacobian_matches_frozen_tau_finite_differences(oracle):
    h = 0.15
    prm, xi, w, U, U0 = one_element(oracle, h, seed=3)
    U *= 0.5
    R, J = oracle.element(prm, h, xi, w, np.eye(8), U, U0)
    d = 1e-6
    for col in range(32):
        e = np.zeros(32); e[col] = d
        Rp = oracle.element_frozen(prm, h, xi, w, np.eye(8), U.ravel(), U.ravel() + e, U0)
        Rm = oracle.element_frozen(prm, h, xi, w, np.eye(8), U.ravel(), U.ravel() - e, U0)
        fd = (Rp - Rm) / (2 * d)
        np.testing.assert_allclose(J[:, col], fd, rtol=1e-6, atol=1e-6 * np.abs(J).max())


# ---------------------------------------------------------------------------
# Mesh derivation: hanging constraints and CSR pattern (Alg. 3, node figure)
# ---------------------------------------------------------------------------


def small_adaptive_tree():
    c = (0.5 + I.BODY_OFFSET[0], 0.5, 0.5)
    return I.sphere_refined_octree(c, 0.3, 2, 4, 1.0)


def test_uniform_counts(oracle):
    t = I.uniform_octree(4)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    assert ms.n_nodes == 17 ** 3 == 4913
    assert ms.nnz == 49 ** 3 * 16 == 1882384
    assert ms.n_hanging == 0
    assert np.all(ms.nm == 8)
    # no hanging vertex: C is a permutation (master slots are sorted by node id)
    assert np.all(np.sort(ms.C, axis=2)[:, :, :7] == 0) and np.all(ms.C.sum(1) == 1)


def test_hanging_constraints_partition_of_unity_and_linear_reproduction(oracle):
    t = small_adaptive_tree()
    assert I.check_balanced(t)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    assert ms.n_hanging > 0
    np.testing.assert_allclose(ms.C.sum(2), 1.0, atol=0)
    assert ms.nm.max() <= 8
    # C reproduces linear fields: values at masters -> values at every vertex
    lin = lambda x: 0.3 * x[..., 0] - 1.7 * x[..., 1] + 2.2 * x[..., 2] + 0.1
    nx = ms.node_xyz_int.astype(np.float64)
    side = t.side()
    corners = np.stack([t.ax, t.ay, t.az], 1)[:, None, :].astype(np.int64) + \
        np.array([[(c >> d) & 1 for d in range(3)] for c in range(8)])[None] * side[:, None, None]
    mvals = np.where(ms.masters >= 0, lin(nx[np.maximum(ms.masters, 0)]), 0.0)
    vv = np.einsum("eas,es->ea", ms.C, mvals)
    np.testing.assert_allclose(vv, lin(corners.astype(np.float64)), rtol=0, atol=1e-12)
    # constraint weights are 1, 1/2 or 1/4 only
    assert set(np.unique(ms.C[ms.C > 0]).tolist()) <= {1.0, 0.5, 0.25}


def test_csr_pattern_structure(oracle):
    t = small_adaptive_tree()
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    rp, ci = ms.row_ptr, ms.col_idx
    for r in range(4 * ms.n_nodes):
        cols = ci[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cols) > 0)
        assert (cols.size % 4) == 0
        assert np.all(cols.reshape(-1, 4) % 4 == np.arange(4))
        assert r in set(cols[::4] + (r % 4))  # diagonal present
    # symmetric pattern
    rows = np.repeat(np.arange(4 * ms.n_nodes), np.diff(rp))
    a = set(zip(rows.tolist(), ci.tolist()))
    assert all((c, r) in a for (r, c) in list(a)[:20000])


def test_dense_brute_force_assembly(oracle):
    # tiny tree: global K = sum_e P_e^T K_e P_e built densely equals the CSR assembly
    c = (0.5 + I.BODY_OFFSET[0], 0.5, 0.5)
    t = I.sphere_refined_octree(c, 0.2, 1, 3, 0.6)
    assert t.n <= 120
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    nx = ms.node_xyz_int / float(1 << t.max_level)
    f = I.make_fields(nx, 7)
    prm = oracle.params()
    V, R = oracle.assemble(t, ms, f, prm)
    n = 4 * ms.n_nodes
    Kd = np.zeros((n, n)); Rd = np.zeros(n)
    h = oracle.element_h(t)
    xi, w = oracle.std_points(1.0)
    for e in range(t.n):
        nm = ms.nm[e]
        m = ms.masters[e, :nm]
        Um = np.stack([f["ux"][m], f["uy"][m], f["uz"][m], f["p"][m]], 1)
        U0 = np.stack([f["ux0"][m], f["uy0"][m], f["uz0"][m]], 1)
        Re, Je = oracle.element(prm, h[e], xi, np.full(8, (h[e] / 2) ** 3), ms.C[e, :, :nm], Um, U0)
        idx = (4 * m[:, None] + np.arange(4)).ravel()
        Kd[np.ix_(idx, idx)] += Je
        Rd[idx] += Re
    rows = np.repeat(np.arange(n), np.diff(ms.row_ptr))
    Kc = np.zeros((n, n)); Kc[rows, ms.col_idx] = V
    np.testing.assert_allclose(Kc, Kd, rtol=1e-13, atol=1e-13 * np.abs(Kd).max())
    np.testing.assert_allclose(R, Rd, rtol=1e-13, atol=1e-14)
    # the pattern holds exactly the structurally coupled blocks
    assert set(zip(*np.nonzero(Kd))) <= set(zip(rows.tolist(), ms.col_idx.tolist()))


def test_constant_state_zero_residual_on_hanging_mesh(oracle):
    t = small_adaptive_tree()
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    n = ms.n_nodes
    f = {"ux": np.full(n, 0.4), "uy": np.full(n, -0.2), "uz": np.full(n, 1.1), "p": np.zeros(n)}
    f.update({"ux0": f["ux"].copy(), "uy0": f["uy"].copy(), "uz0": f["uz"].copy()})
    _, R = oracle.assemble(t, ms, f, vals=False)
    assert np.abs(R).max() < 1e-16


def test_patch_test_viscous_on_hanging_mesh(oracle):
    # linear u: eps(u) constant, so interior rows of the viscous term vanish
    t = small_adaptive_tree()
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    x = ms.node_xyz_int / float(1 << t.max_level)
    A = np.array([[0.3, -1.0, 0.5], [2.0, 0.1, -0.7], [-0.4, 0.9, 0.2]])
    u = x @ A.T
    f = {"ux": u[:, 0], "uy": u[:, 1], "uz": u[:, 2], "p": np.zeros(len(x)),
         "ux0": u[:, 0], "uy0": u[:, 1], "uz0": u[:, 2]}
    prm = oracle.params(term_mask=1 << 2, theta=1.0)
    _, R = oracle.assemble(t, ms, f, prm, vals=False)
    interior = np.all((ms.node_xyz_int > 0) & (ms.node_xyz_int < (1 << t.max_level)), 1)
    Rr = R.reshape(-1, 4)
    assert interior.sum() > 50
    assert np.abs(Rr[interior, :3]).max() < 1e-15
    assert np.abs(Rr[~interior, :3]).max() > 1e-6


# ---------------------------------------------------------------------------
# Exact predicates and in-out labels (Alg. 4, Alg. 5 and the ray-tracing fallback)
# ---------------------------------------------------------------------------


def _orient3d_exact(a, b, c, d):
    F = [[Fraction(x) for x in p] for p in (a, b, c, d)]
    ad = [F[0][k] - F[3][k] for k in range(3)]
    bd = [F[1][k] - F[3][k] for k in range(3)]
    cd = [F[2][k] - F[3][k] for k in range(3)]
    det = (ad[0] * (bd[1] * cd[2] - bd[2] * cd[1]) + bd[0] * (cd[1] * ad[2] - cd[2] * ad[1])
           + cd[0] * (ad[1] * bd[2] - ad[2] * bd[1]))
    return (det > 0) - (det < 0)


def test_orient3d_exact_against_rationals(oracle):
    rng = np.random.default_rng(5)
    n_zero = 0
    for it in range(3000):
        a, b, c = rng.uniform(-1, 1, (3, 3))
        mode = it % 4
        if mode == 0:
            d = rng.uniform(-1, 1, 3)
        elif mode == 1:      # nearly coplanar, rounded off the plane
            s, t = rng.uniform(-1, 1, 2)
            d = a + s * (b - a) + t * (c - a)
        elif mode == 2:      # exactly coplanar on a dyadic grid
            a, b, c = (np.round(x * 64) / 64 for x in (a, b, c))
            d = a + 0.5 * (b - a) + 0.25 * (c - a)
        else:                # tiny perturbation of a coplanar point
            s, t = rng.uniform(-1, 1, 2)
            d = a + s * (b - a) + t * (c - a)
            d = d + np.array([1, -1, 1]) * np.ldexp(1.0, -52) * rng.integers(-3, 4, 3)
        ref = _orient3d_exact(a, b, c, d)
        n_zero += ref == 0
        assert oracle.orient3d(a, b, c, d) == ref
    assert n_zero > 100


def test_labels_sphere_analytic(oracle):
    c = np.array([0.5, 0.5, 0.5]) + I.BODY_OFFSET
    r = 0.1
    s = I.icosphere(3, r, c)
    assert I.is_watertight(s)
    # inradius: distance from c to the closest triangle plane
    a, b, cc = (s.verts[s.tris[:, k]] for k in range(3))
    n = np.cross(b - a, cc - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    r_in = np.abs(np.einsum("ij,ij->i", a - c, n)).min()
    rng = np.random.default_rng(11)
    p = c + rng.uniform(-0.13, 0.13, (4000, 3))
    d = np.linalg.norm(p - c, axis=1)
    lab, nd = oracle.label_points(s, p)
    assert nd == 0
    assert np.all(lab[d > r] == 0)
    assert np.all(lab[d < r_in] == 1)
    assert ((d > r_in) & (d < r)).sum() > 0
    # surface vertices are on the surface: IN
    lab_v, _ = oracle.label_points(s, s.verts[:50])
    assert np.all(lab_v == 1)


def _winding_number(surf, p):
    """Generalised winding number: the solid angles of the triangles seen from
    each point (Van Oosterom and Strackee's formula) summed over 4 pi; 1 inside
    a closed, outward-oriented surface, 0 outside."""
    w = np.zeros(p.shape[0])
    for t in surf.tris:
        A, B, C = (surf.verts[t[k]][None] - p for k in range(3))
        la, lb, lc = (np.linalg.norm(X, axis=1) for X in (A, B, C))
        num = np.einsum("ij,ij->i", A, np.cross(B, C))
        den = (la * lb * lc + np.einsum("ij,ij->i", A, B) * lc + np.einsum("ij,ij->i", A, C) * lb
               + np.einsum("ij,ij->i", B, C) * la)
        w += 2.0 * np.arctan2(num, den)
    return w / (4.0 * np.pi)


def test_labels_against_winding_number(oracle):
    # an independent definition of inside, on a convex body (including the
    # shell between the polyhedron and its sphere), a dented (non-convex) body
    # and two separate filleted boxes
    c = np.array([0.5, 0.5, 0.5]) + I.BODY_OFFSET
    ico = I.icosphere(3, 0.2, c)
    v = ico.verts.copy()
    v[0] = c + (v[0] - c) * 0.6
    dent = I.Surface(v, ico.tris.copy(), {"kind": "dented icosphere"})
    boxes = I.two_boxes(4)
    rng = np.random.default_rng(31)
    for surf in (ico, dent, boxes):
        lo, hi = surf.verts.min(0), surf.verts.max(0)
        pad = 0.1 * (hi - lo)
        p = rng.uniform(lo - pad, hi + pad, (1500, 3))
        # points near vertex 0 (the dent) and near the surface
        k = 300
        p[:k] = surf.verts[rng.integers(0, surf.verts.shape[0], k)] + rng.normal(scale=0.02 * (hi - lo).max(), size=(k, 3))
        p[k:k + 100] = surf.verts[0] + rng.normal(scale=0.05 * (hi - lo).max(), size=(100, 3))
        if surf is dent:
            # inside the dent: between the pushed vertex and its place on the
            # sphere (inside the convex hull, outside the body)
            s_ = rng.uniform(0.1, 0.9, 100)[:, None]
            p[k + 100:k + 200] = v[0] + s_ * (ico.verts[0] - v[0]) + rng.normal(scale=1e-3, size=(100, 3))
        lab, _ = oracle.label_points(surf, p)
        w = _winding_number(surf, p)
        clear = np.abs(w - np.round(w)) < 1e-6     # away from the surface
        assert clear.mean() > 0.95
        assert set(np.unique(np.round(w[clear]))) <= {0.0, 1.0}
        assert np.array_equal(lab[clear], np.round(w[clear]).astype(np.uint8))
        assert 0 < lab[clear].sum() < clear.sum()
        if surf is dent:
            assert (lab[k + 100:k + 200] == 0).sum() > 50


def test_labels_box_analytic_and_brute_force(oracle):
    lo, hi = np.array([0.21, 0.33, 0.4]), np.array([0.74, 0.61, 0.83])
    s = I.box_surface(lo, hi)
    rng = np.random.default_rng(2)
    p = rng.uniform(0, 1, (3000, 3))
    lab, nd = oracle.label_points(s, p)
    inside = np.all((p > lo) & (p < hi), 1)
    np.testing.assert_array_equal(lab, inside.astype(np.uint8))
    # all-triangle segment parity with a far point, plain Python loop
    for P in p[:40]:
        Q = np.array([2.5, P[1] + 0.01 * np.pi, P[2] + 0.01 * np.e])
        cnt = 0
        for t in s.tris:
            r = oracle.seg_tri(P, Q, *s.verts[t])
            assert r in (0, 1)
            cnt += r
        assert cnt % 2 == int(np.all((P > lo) & (P < hi)))


def test_markers_rule(oracle):
    # Alg. 4: all IN -> IN, none -> OUT, else INTERCEPTED
    lo = np.array([37, 43, 51]) / 128.0
    hi = np.array([91, 85, 77]) / 128.0
    s = I.box_surface(lo, hi)
    t = I.uniform_octree(4)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, vlab, nd = oracle.markers(t, ms, s)
    # grid rays hit the face diagonals exactly here: the fallback directions decide
    assert nd > 0
    h = 1 / 16
    a = np.stack([t.ax, t.ay, t.az], 1) * h
    b = a + h
    full_in = np.all((a > lo) & (b < hi), 1)
    none = np.any((b < lo) | (a > hi), 1)
    assert np.all(mk[full_in] == oracle.IN)
    assert np.all(mk[none] == oracle.OUT)
    assert np.all(mk[~full_in & ~none] == oracle.INTERCEPTED)


# ---------------------------------------------------------------------------
# Adaptive quadrature (Section "Adaptive Quadrature", Gauss-point figure)
# ---------------------------------------------------------------------------


def test_adaptive_quadrature_exact_box_volume(oracle):
    # box faces at odd multiples of h/8: the Gauss-point stop rule resolves the
    # box exactly from depth 2 on (0.211 and 0.789 bracket 1/4, 1/2, 3/4 of a
    # level-1 cell; at level 2 the face halves the cell and the two-point rule
    # halves the volume exactly), but not at depth 1
    lo = np.array([37, 43, 51]) / 128.0
    hi = np.array([91, 85, 77]) / 128.0
    s = I.box_surface(lo, hi)
    t = I.uniform_octree(4)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms, s)
    cut = np.nonzero(mk == oracle.INTERCEPTED)[0]
    h = oracle.element_h(t)
    vbox = np.prod(hi - lo)
    for depth, exact in ((3, True), (2, True), (1, False)):
        sq = oracle.subquad(t, s, cut, depth)
        _, w = oracle.subgp_xi(t, sq["el"], sq["key"], sq["lvl"], depth)
        vol = (h[mk == oracle.OUT] ** 3).sum() + w.sum()
        if exact:
            assert vol == 1.0 - vbox
        else:
            assert vol != 1.0 - vbox
    # per element the kept weight never exceeds the element volume
    sq = oracle.subquad(t, s, cut, 3)
    _, w = oracle.subgp_xi(t, sq["el"], sq["key"], sq["lvl"], 3)
    per = np.bincount(sq["el"], weights=w, minlength=t.n)
    assert np.all(per <= h ** 3 + 1e-18)


def test_adaptive_quadrature_stop_rule_and_order(oracle):
    # depth 0: the element's own Gauss points, OUT ones only; uniform cells not split
    lo = np.array([37, 43, 51]) / 128.0
    hi = np.array([91, 85, 77]) / 128.0
    s = I.box_surface(lo, hi)
    t = I.uniform_octree(4)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms, s)
    cut = np.nonzero(mk == oracle.INTERCEPTED)[0]
    sq0 = oracle.subquad(t, s, cut, 0)
    assert np.all(sq0["lvl"] == 0)
    assert np.all(np.bincount(sq0["el"], minlength=t.n)[cut] <= 8)
    sq = oracle.subquad(t, s, cut, 3)
    # canonical order: elements ascending, keys ascending within an element
    el, key = sq["el"], sq["key"]
    assert np.all(np.diff(el) >= 0)
    same = el[1:] == el[:-1]
    assert np.all(key[1:][same] > key[:-1][same])
    # kept points of a sub-cell come in full groups of 8 below the maximum level
    for lv in (1, 2):
        m = sq["lvl"] == lv
        cells = (el[m] << 12) | (key[m] >> (3 * (3 - lv) + 3))
        assert np.all(np.unique(cells, return_counts=True)[1] == 8)


def test_subcell_points_sit_where_the_sketch_draws_them(oracle):
    # the sketch of the adaptive quadrature prints its points: every point of
    # split level l lies at (i + g) / 2^l of its element's side (4), g one of
    # the two printed offsets and i its sub-cell index; a sub-cell of the first
    # level is kept whole (all 4 of its points in the plane), one of the last
    # level keeps the points on the fluid side only
    vals, points = _sketch()
    gm, gp = vals["g_minus"][0], vals["g_plus"][0]
    assert len(points) == 51
    cells = {}
    for lvl, x, y in points:
        key = [lvl]
        for v in (x, y):
            e = 4.0 * np.floor(v / 4.0)
            u = (v - e) / 4.0 * 2 ** lvl
            i = int(np.floor(u))
            assert min(abs(u - i - gm), abs(u - i - gp)) < 1e-9, (lvl, x, y)
            key += [e, i]
        cells.setdefault(tuple(key), set()).add((round(x, 6), round(y, 6)))
    sizes = {k: len(v) for k, v in cells.items()}
    assert all(n == 4 for k, n in sizes.items() if k[0] == 1) and any(k[0] == 1 for k in sizes)
    assert all(1 <= n <= 4 for k, n in sizes.items() if k[0] == 2)
    assert any(n < 4 for k, n in sizes.items() if k[0] == 2)
    # every kept point of the reference's adaptive quadrature (its C routine)
    # follows it at every split level, and the key decoding agrees
    c0 = np.array([0.5, 0.5, 0.5]) + I.BODY_OFFSET
    s = I.icosphere(2, 0.3, c0)
    t = I.uniform_octree(2)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms, s)
    cut = np.nonzero(mk == oracle.INTERCEPTED)[0]
    h = oracle.element_h(t)
    corner = np.asarray(t.origin, np.float64)[None] + t.root_len * np.stack(
        [t.ax, t.ay, t.az], 1).astype(np.float64) / float(1 << t.max_level)
    for depth in (2, 3):
        sq = oracle.subquad(t, s, cut, depth)
        el, lvl, xyz = sq["el"], sq["lvl"].astype(np.int64), sq["xyz"]
        assert set(np.unique(lvl)) == set(range(1, depth + 1))
        u = (xyz - corner[el]) / h[el, None] * (2.0 ** lvl)[:, None]
        i = np.floor(u)
        f = u - i
        assert np.all((i >= 0) & (i < (2 ** lvl)[:, None]))
        near = np.minimum(np.abs(f - gm), np.abs(f - gp))
        assert near.max() < 1e-9
        # both offsets occur on every axis at every level
        for lv in range(1, depth + 1):
            for ax in range(3):
                fl = f[lvl == lv, ax]
                assert np.any(np.abs(fl - gm) < 1e-9) and np.any(np.abs(fl - gp) < 1e-9)
        xi, _ = oracle.subgp_xi(t, el, sq["key"], sq["lvl"], depth)
        np.testing.assert_allclose(corner[el] + (xi + 1.0) / 2.0 * h[el, None], xyz, rtol=0, atol=1e-15)


def test_adaptive_quadrature_sphere_converges_to_polyhedron_volume(oracle):
    # joint refinement of h and the split depth: the fluid volume converges to
    # the domain minus the polyhedron volume (divergence theorem), not 4/3 pi r^3
    c = np.array([0.5, 0.5, 0.5]) + I.BODY_OFFSET
    s = I.icosphere(2, 0.3, c)
    vpoly = I.signed_volume(s)
    errs = []
    for L, depth in ((3, 0), (4, 1), (5, 2)):
        t = I.uniform_octree(L)
        ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
        mk, _, _ = oracle.markers(t, ms, s)
        cut = np.nonzero(mk == oracle.INTERCEPTED)[0]
        h = oracle.element_h(t)
        sq = oracle.subquad(t, s, cut, depth)
        _, w = oracle.subgp_xi(t, sq["el"], sq["key"], sq["lvl"], depth)
        vol = (h[mk == oracle.OUT] ** 3).sum() + w.sum()
        errs.append(abs((1.0 - vol) - vpoly))
    assert errs[0] > 5 * errs[1] > 25 * errs[2]
    assert errs[-1] < 5e-4 * vpoly
    assert abs(vpoly - 4 / 3 * np.pi * 0.3 ** 3) > 10 * errs[-1]


# ---------------------------------------------------------------------------
# Unsigned distance to a triangulated surface (training targets of the
# learned in-out filter)
# ---------------------------------------------------------------------------


def _brute_distance(verts, tris, x, n=200):
    """min over a dense barycentric grid of every triangle (an upper bound that
    is within the grid spacing of the true distance)."""
    u, v = np.meshgrid(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1))
    m = (u + v) <= 1.0
    u, v = u[m], v[m]
    best = np.full(x.shape[0], np.inf)
    for t in tris:
        a, b, c = verts[t[0]], verts[t[1]], verts[t[2]]
        P = a[None] + u[:, None] * (b - a)[None] + v[:, None] * (c - a)[None]
        d = np.sqrt(((x[:, None, :] - P[None]) ** 2).sum(-1)).min(1)
        best = np.minimum(best, d)
    return best


def test_unsigned_distance_closed_forms_and_brute_force(oracle):
    class S:
        pass
    s = S()
    s.verts = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    s.tris = np.array([[0, 1, 2]], np.int32)
    x = np.array([
        [0.2, 0.2, 0.7],     # face region: distance = height
        [-0.3, -0.4, 0.0],   # vertex region of a: |x - a|
        [0.5, -0.2, 0.1],    # edge region of ab: distance to the line
        [1.0, 1.0, 0.0],     # edge region of bc (in plane)
        [2.0, -1.0, 0.5],    # vertex region of b
    ])
    ref = np.array([0.7, 0.5, np.hypot(0.2, 0.1), np.sqrt(0.5), np.sqrt(1 + 1 + 0.25)])
    np.testing.assert_allclose(oracle.unsigned_distance(s, x), ref, rtol=1e-14, atol=1e-15)
    # a closed polyhedron: brute force within the grid spacing, never above it
    c = np.array([0.5, 0.5, 0.5])
    ico = I.icosphere(1, 0.3, c)
    rng = np.random.default_rng(4)
    q = rng.uniform(0.0, 1.0, (60, 3))
    d = oracle.unsigned_distance(ico, q)
    bf = _brute_distance(ico.verts, ico.tris, q)
    edge = max(np.linalg.norm(ico.verts[t[0]] - ico.verts[t[1]]) for t in ico.tris)
    assert np.all(d <= bf + 1e-12)
    assert np.all(bf - d <= edge / 200 * 1.5)
    # the icosphere's centre is at the inradius from every face
    nrm = [np.cross(ico.verts[t[1]] - ico.verts[t[0]], ico.verts[t[2]] - ico.verts[t[0]])
           for t in ico.tris]
    inr = min(abs(np.dot(n / np.linalg.norm(n), ico.verts[t[0]] - c)) for n, t in zip(nrm, ico.tris))
    assert abs(oracle.unsigned_distance(ico, c[None])[0] - inr) <= 1e-15


# ---------------------------------------------------------------------------
# Jacobian action (the matrix-free product): the directional derivative of the
# residual, one complex-step evaluation per element
# ---------------------------------------------------------------------------


def test_jacobian_action_equals_assembled_jacobian_times_x(oracle):
    """On a cut, hanging mesh with sub-cell points: the derivative of the
    residual along x equals the column-by-column Jacobian times x (two
    independent complex-step formulations), inactive rows included (y = x)."""
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    t = I.sphere_refined_octree(c, 0.25, 2, 4, 1.0)
    s = I.icosphere(2, 0.25, c)
    ms0 = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms0, s)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level, active=mk != oracle.IN)
    assert ms.n_hanging > 0 and (~ms.node_active).sum() > 0
    sub = oracle.subquad(t, s, np.nonzero(mk == oracle.INTERCEPTED)[0], 2)
    xyz = ms.node_xyz_int.astype(np.float64) / float(1 << t.max_level)
    f = I.make_fields(xyz, 11)
    rng = np.random.default_rng(5)
    x = rng.normal(size=4 * ms.n_nodes)
    V, _ = oracle.assemble(t, ms, f, mk=mk, sub=sub, depth=2, resid=False)
    rid = np.repeat(np.arange(4 * ms.n_nodes), np.diff(ms.row_ptr))
    y_ref = np.zeros(4 * ms.n_nodes)
    np.add.at(y_ref, rid, V * x[ms.col_idx])
    y = oracle.jacobian_apply(t, ms, f, x, mk=mk, sub=sub, depth=2)
    assert np.linalg.norm(y - y_ref) <= 1e-13 * np.linalg.norm(y_ref)
    inact = np.nonzero(~ms.node_active)[0]
    assert np.array_equal(y[4 * inact], x[4 * inact])


def test_jacobian_action_rest_state_closed_form(oracle):
    """u = u_prev = 0, p = 0 on a uniform mesh, x = a constant velocity c: the
    fine scales vanish and only the mass term survives, so interior momentum
    rows are rho h^3 / dt c exactly (the node's basis integrates to h^3) and
    interior continuity rows are 0 (the integral of grad N_a over its support)."""
    lev, rho, dt = 3, 1.3, 0.02
    t = I.uniform_octree(lev)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    n = ms.n_nodes
    z = np.zeros(n)
    f = {"ux": z, "uy": z, "uz": z, "p": z, "ux0": z, "uy0": z, "uz0": z}
    cvel = np.array([0.7, -1.1, 0.4])
    x = np.zeros(4 * n)
    for k in range(3):
        x[k::4] = cvel[k]
    prm = oracle.params(rho=rho, mu=0.05, dt=dt)
    y = oracle.jacobian_apply(t, ms, f, x, prm=prm)
    h = 1.0 / (1 << lev)
    ijk = ms.node_xyz_int // (1 << (t.max_level - lev))
    interior = np.all((ijk > 0) & (ijk < (1 << lev)), axis=1)
    assert interior.sum() == ((1 << lev) - 1) ** 3
    for k in range(3):
        np.testing.assert_allclose(y[4 * np.nonzero(interior)[0] + k], rho * h ** 3 / dt * cvel[k],
                                   rtol=1e-13)
    assert np.abs(y[4 * np.nonzero(interior)[0] + 3]).max() < 1e-15


# ---------------------------------------------------------------------------
# Weak (Nitsche) boundary terms, eq. (weakbc): surface points and terms
# ---------------------------------------------------------------------------


def _cut_setup(oracle, r=0.2, lmin=3, lmax=5, beta=1.5, sub=2):
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    t = I.sphere_refined_octree(c, r, lmin, lmax, beta)
    s = I.icosphere(sub, r, c)
    ms0 = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms0, s)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level, active=mk != oracle.IN)
    return t, s, mk, ms


def _fields_const(n, u, p=0.0):
    f = {"ux": np.full(n, u[0]), "uy": np.full(n, u[1]), "uz": np.full(n, u[2]), "p": np.full(n, p)}
    f.update({"ux0": f["ux"].copy(), "uy0": f["uy"].copy(), "uz0": f["uz"].copy()})
    return f


def test_surface_points_lie_in_their_leaves(oracle):
    t, s, mk, ms = _cut_setup(oracle)
    sp = oracle.surface_points(t, s, mk)
    assert sp["el"].size == 3 * s.tris.shape[0]   # the sphere lies inside the domain, no IN leaf holds a point
    assert np.all(np.abs(sp["xi"]) <= 1.0)
    h = oracle.element_h(t)[sp["el"]]
    lo = np.stack([t.ax, t.ay, t.az], 1)[sp["el"]] / float(1 << t.max_level)
    assert np.all((sp["xyz"] >= lo) & (sp["xyz"] < lo + h[:, None]))
    area = 0.5 * np.linalg.norm(np.cross(s.verts[s.tris[:, 1]] - s.verts[s.tris[:, 0]],
                                         s.verts[s.tris[:, 2]] - s.verts[s.tris[:, 0]]), axis=1).sum()
    assert abs(sp["w"].sum() - area) <= 1e-14 * area
    np.testing.assert_allclose(np.linalg.norm(sp["n"], axis=1), 1.0, rtol=1e-15)


def test_weak_bc_zero_for_state_equal_to_g(oracle):
    """u = g (constant), p = 0: every term of the surface integrals vanishes."""
    t, s, mk, ms = _cut_setup(oracle)
    g = (0.3, -0.2, 0.1)
    _, R, _ = oracle.weak_bc(t, ms, s, mk, _fields_const(ms.n_nodes, g), g=g, vals=False)
    assert np.abs(R).max() < 1e-17


def test_weak_bc_closed_surface_pressure_identity(oracle):
    """u = g = 0, p = 1: the momentum rows summed over all nodes give the
    integral of p n over a closed surface, which is zero (the basis is a
    partition of unity; sum of area times normal over a closed polyhedron);
    the continuity rows vanish."""
    t, s, mk, ms = _cut_setup(oracle)
    _, R, sp = oracle.weak_bc(t, ms, s, mk, _fields_const(ms.n_nodes, (0, 0, 0), 1.0), vals=False)
    area = sp["w"].sum()
    for i in range(3):
        assert abs(R[i::4].sum()) <= 1e-14 * area
        # a single term is not small: the sum is a cancellation
        assert np.abs(R[i::4]).max() > 1e-4 * area
    assert np.abs(R[3::4]).max() == 0.0


def test_weak_bc_inflow_flux_through_a_box(oracle):
    """Axis-aligned box, u = u_prev = (1, 0, 0), p = 0, mu = 0, no penalty:
    only the inflow term remains, on the face where the flow enters the fluid
    (x = hi, fluid normal -x); the x-momentum rows summed over all nodes are
    rho times that face's area, the other rows sum to zero."""
    lo = np.array([37, 43, 51]) / 128.0
    hi = np.array([91, 85, 77]) / 128.0
    s = I.box_surface(lo, hi)
    t = I.uniform_octree(4)
    ms0 = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms0, s)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level, active=mk != oracle.IN)
    rho = 1.7
    prm = oracle.params(rho=rho, mu=0.0)
    _, R, _ = oracle.weak_bc(t, ms, s, mk, _fields_const(ms.n_nodes, (1.0, 0.0, 0.0)), c_b=0.0,
                             prm=prm, vals=False)
    a_yz = (hi[1] - lo[1]) * (hi[2] - lo[2])
    assert abs(R[0::4].sum() - rho * a_yz) <= 1e-14 * rho * a_yz
    for i in (1, 2, 3):
        assert abs(R[i::4].sum()) <= 1e-15


def test_weak_bc_jacobian_against_central_differences(oracle):
    """The complex-step Jacobian of the surface terms against central
    differences of the real residual along a random direction."""
    t, s, mk, ms = _cut_setup(oracle)
    xyz = ms.node_xyz_int.astype(np.float64) / float(1 << t.max_level)
    f = I.make_fields(xyz, 21)
    V, R, _ = oracle.weak_bc(t, ms, s, mk, f, c_b=4.0, g=(0.1, 0.0, -0.2))
    rng = np.random.default_rng(2)
    d = rng.normal(size=4 * ms.n_nodes)
    rid = np.repeat(np.arange(4 * ms.n_nodes), np.diff(ms.row_ptr))
    jd = np.zeros(4 * ms.n_nodes)
    np.add.at(jd, rid, V * d[ms.col_idx])
    eps = 1e-6

    def res(sign):
        g = dict(f)
        for c, k in enumerate(("ux", "uy", "uz", "p")):
            g[k] = f[k] + sign * eps * d[c::4]
        return oracle.weak_bc(t, ms, s, mk, g, c_b=4.0, g=(0.1, 0.0, -0.2), vals=False)[1]
    fd = (res(1) - res(-1)) / (2 * eps)
    assert np.linalg.norm(fd - jd) <= 1e-7 * np.linalg.norm(jd)


def test_element_weights_reduce_to_one_and_zero(oracle):
    """eq. (Wpart) reduces to 1 for OUT and 0 for IN elements (the text after
    it); the weights of the INTERCEPTED ones add up to the point counts."""
    t, s, mk, ms = _cut_setup(oracle)
    sub = oracle.subquad(t, s, np.nonzero(mk == oracle.INTERCEPTED)[0], 3)
    sp = oracle.surface_points(t, s, mk)
    w = oracle.element_weights(t, mk, sub, sp, 2.5)
    assert np.all(w[mk == oracle.OUT] == 1.0) and np.all(w[mk == oracle.IN] == 0.0)
    cut = mk == oracle.INTERCEPTED
    assert abs(8.0 * w[cut].sum() - (sub["el"].size + 2.5 * sp["el"].size)) < 1e-9


# ---------------------------------------------------------------------------
# Newton's linear step: the exact solve that the Krylov methods approximate
# ---------------------------------------------------------------------------


def test_linear_solve_recovers_a_known_solution(oracle):
    """On a cut, hanging mesh: the CSR product equals the matrix-free Jacobian
    action (independent complex-step formulation), and solving A x = A x*
    returns x* to within the conditioning of A (dense 2-norm condition number)."""
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    t = I.sphere_refined_octree(c, 0.25, 2, 4, 1.0)
    s = I.icosphere(2, 0.25, c)
    ms0 = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms0, s)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level, active=mk != oracle.IN)
    sub = oracle.subquad(t, s, np.nonzero(mk == oracle.INTERCEPTED)[0], 2)
    f = I.make_fields(ms.node_xyz_int.astype(np.float64) / float(1 << t.max_level), 12)
    V, _ = oracle.assemble(t, ms, f, mk=mk, sub=sub, depth=2, resid=False)
    xs = np.random.default_rng(8).normal(size=4 * ms.n_nodes)
    b = oracle.csr_matvec(ms, V, xs)
    y = oracle.jacobian_apply(t, ms, f, xs, mk=mk, sub=sub, depth=2)
    assert np.linalg.norm(b - y) <= 1e-13 * np.linalg.norm(b)
    # INTERCEPTED elements whose sub-cell points are all IN leave rows of IN
    # nodes empty: only the Dirichlet rows of IN nodes make the system regular
    nodes = oracle.dirichlet_nodes(ms, mk)
    V, _ = oracle.apply_dirichlet(ms, V, None, nodes)
    b = oracle.csr_matvec(ms, V, xs)
    x = oracle.linear_solve(ms, V, b)
    A = np.zeros((b.size, b.size))
    A[np.repeat(np.arange(b.size), np.diff(ms.row_ptr)), ms.col_idx] = V
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    print(f"{b.size} unknowns, condition number {kappa:.2e}, error {err:.2e}")
    assert err <= 100 * kappa * np.finfo(float).eps
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_dirichlet_nodes_are_the_in_corners(oracle):
    """The Dirichlet nodes are exactly the independent vertices labelled IN that
    are corners of IN elements (the exact labels decide, no hanging vertex), and
    the rows they replace become identity rows while the others keep their
    values."""
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    t = I.sphere_refined_octree(c, 0.25, 2, 4, 1.0)
    s = I.icosphere(2, 0.25, c)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, vlab, _ = oracle.markers(t, ms, s)
    nodes = oracle.dirichlet_nodes(ms, mk)
    xyz = ms.node_xyz_int[nodes].astype(np.float64) / float(1 << t.max_level)
    lab, _ = oracle.label_points(s, xyz)
    assert nodes.size > 0 and lab.all()             # every Dirichlet node is IN
    # brute force: an independent vertex is a Dirichlet node iff some IN element has it as a corner
    side = (1 << (t.max_level - t.level.astype(np.int64)))
    want = set()
    for e in np.nonzero(mk == oracle.IN)[0]:
        for a in range(8):
            p = (int(t.ax[e]) + (a & 1) * side[e], int(t.ay[e]) + ((a >> 1) & 1) * side[e],
                 int(t.az[e]) + ((a >> 2) & 1) * side[e])
            want.add(p)
    got = {tuple(map(int, q)) for q in ms.node_xyz_int[nodes]}
    indep = {tuple(map(int, q)) for q in ms.node_xyz_int}
    assert got == want & indep
    V = np.random.default_rng(2).normal(size=ms.nnz)
    R = np.random.default_rng(3).normal(size=4 * ms.n_nodes)
    V2, R2 = oracle.apply_dirichlet(ms, V, R, nodes)
    rows = np.zeros(4 * ms.n_nodes, bool)
    rows[(4 * nodes[:, None] + np.arange(4)).ravel()] = True
    rid = np.repeat(np.arange(4 * ms.n_nodes), np.diff(ms.row_ptr))
    sel = rows[rid]
    assert np.array_equal(V2[~sel], V[~sel]) and np.array_equal(R2[~rows], R[~rows])
    assert np.array_equal(V2[sel], (ms.col_idx[sel] == rid[sel]).astype(float))
    assert not R2[rows].any()


# ---------------------------------------------------------------------------
# eq. (vms): the momentum SUPG, cross-stress and tau-bar terms at a state
# where every one of them is non-zero in closed form. u = u_prev = c (uniform
# flow) and p linear with gradient g: grad u = 0, a_t = 0, so r_M = g and
# u' = -tau_M g is constant; tau_M, tau_C, taubar are the same at every point.
# ---------------------------------------------------------------------------


def _uniform_flow_state(h, c, g):
    corners = np.array([[(a >> d) & 1 for d in range(3)] for a in range(8)]) * h
    U = np.zeros((8, 4)); U[:, :3] = c; U[:, 3] = corners @ g + 0.2
    return U, np.tile(c, (8, 1))


UF = dict(h=0.2, dt=0.05, mu=0.03, rho=1.3, th=0.5, c=np.array([0.6, -0.9, 0.4]),
          g=np.array([0.7, -0.4, 1.3]))


def _uf_taus():
    h, dt, mu, rho, c, g = (UF[k] for k in ("h", "dt", "mu", "rho", "c", "g"))
    nu = mu / rho
    tauM = (4 / dt ** 2 + 4 * (c @ c) / h ** 2 + 36 * nu ** 2 * 48 / h ** 4) ** -0.5
    up = -tauM * g
    taubar = h / (2 * np.linalg.norm(up))      # (u'.G.u')^(-1/2) with G = (2/h)^2 I
    return tauM, up, taubar


def test_taubar_closed_form_uniform_flow(oracle):
    h, dt, mu, rho, th, c, g = (UF[k] for k in ("h", "dt", "mu", "rho", "th", "c", "g"))
    prm = oracle.params(rho=rho, mu=mu, dt=dt, theta=th)
    xi, _ = oracle.std_points(h)
    U, U0 = _uniform_flow_state(h, c, g)
    t = oracle.taus(prm, h, xi, U, U0)
    tauM, up, taubar = _uf_taus()
    np.testing.assert_allclose(t[:, 0], tauM, rtol=1e-14)
    np.testing.assert_allclose(t[:, 1], h ** 2 / (12 * tauM), rtol=1e-14)
    np.testing.assert_allclose(t[:, 2], taubar, rtol=1e-14)


def _uf_element(oracle, bit):
    h, dt, mu, rho, th, c, g = (UF[k] for k in ("h", "dt", "mu", "rho", "th", "c", "g"))
    prm = oracle.params(rho=rho, mu=mu, dt=dt, theta=th, term_mask=1 << bit)
    xi, w = oracle.std_points(h)
    U, U0 = _uniform_flow_state(h, c, g)
    R, J = oracle.element(prm, h, xi, w, np.eye(8), U, U0)
    return R.reshape(8, 4), blocks(J)


def test_supg_term_uniform_flow_closed_form(oracle):
    """Term 5 of eq. (vms), -(u.grad w + grad q / rho) . u': residual and its
    frozen-tau Jacobian (u' varies through r_M = rho (a_t + u.grad u) + grad p)."""
    h, dt, rho, th, c = (UF[k] for k in ("h", "dt", "rho", "th", "c"))
    tauM, up, _ = _uf_taus()
    R, B = _uf_element(oracle, 5)
    gradN = np.stack([integral(h, k, None).sum(1) for k in range(3)], 1)    # int d_k N_a
    cgrad = gradN @ c                                                       # int c.grad N_a
    for i in range(3):
        np.testing.assert_allclose(R[:, i], -cgrad * up[i], rtol=1e-13, atol=1e-16)
    np.testing.assert_allclose(R[:, 3], -(1 / rho) * gradN @ up, rtol=1e-13, atol=1e-16)
    cN = sum(c[k] * integral(h, k, None) for k in range(3))                # int (c.grad N_a) N_b
    cc = sum(c[k] * c[l] * integral(h, k, l) for k in range(3) for l in range(3))
    L = sum(integral(h, k, k) for k in range(3))
    sc = 1e-12 * max(np.abs(B[i][j]).max() for i in range(4) for j in range(4))
    for i, j in itertools.product(range(3), range(3)):
        ref = -th * up[i] * integral(h, j, None) + (i == j) * tauM * rho * (cN / dt + th * cc)
        np.testing.assert_allclose(B[i][j], ref, rtol=0, atol=sc)
        np.testing.assert_allclose(B[i][3], tauM * sum(c[k] * integral(h, k, i) for k in range(3)),
                                   rtol=0, atol=sc)
        np.testing.assert_allclose(B[3][j], tauM * (integral(h, j, None) / dt
                                                    + th * sum(c[k] * integral(h, j, k) for k in range(3))),
                                   rtol=0, atol=sc)
    np.testing.assert_allclose(B[3][3], tauM / rho * L, rtol=0, atol=sc)


def test_cross_stress_term_uniform_flow_closed_form(oracle):
    """Term 7, w . (u' . grad u): zero residual at grad u = 0, Jacobian
    delta_ij theta sum_k u'_k int N_a d_k N_b (the u' derivative meets grad u = 0)."""
    h, th = UF["h"], UF["th"]
    _, up, _ = _uf_taus()
    R, B = _uf_element(oracle, 7)
    assert np.abs(R).max() < 1e-16
    ref = th * sum(up[k] * integral(h, None, k) for k in range(3))
    sc = 1e-12 * np.abs(ref).max()
    for i, j in itertools.product(range(4), range(4)):
        want = ref if (i == j and i < 3) else 0 * ref
        np.testing.assert_allclose(B[i][j], want, rtol=0, atol=sc)


def test_taubar_term_uniform_flow_closed_form(oracle):
    """Term 9, (u' . grad w) taubar (u' . grad u): zero residual at grad u = 0,
    Jacobian delta_ij taubar theta sum_kl u'_k u'_l int d_k N_a d_l N_b."""
    h, th = UF["h"], UF["th"]
    _, up, taubar = _uf_taus()
    R, B = _uf_element(oracle, 9)
    assert np.abs(R).max() < 1e-16
    ref = taubar * th * sum(up[k] * up[l] * integral(h, k, l) for k in range(3) for l in range(3))
    sc = 1e-12 * np.abs(ref).max()
    for i, j in itertools.product(range(4), range(4)):
        want = ref if (i == j and i < 3) else 0 * ref
        np.testing.assert_allclose(B[i][j], want, rtol=0, atol=sc)


# ---------------------------------------------------------------------------
# eq. (weakbc): Nitsche consistency, adjoint consistency and penalty terms on
# an axis-aligned box. Weighting the node rows by phi(x_node) for phi in the
# trilinear space turns the residual into the surface integral with test
# function phi; the divergence theorem (fluid normal = minus the box's outward
# normal) gives each integral in closed form.
# ---------------------------------------------------------------------------

BOX_LO = np.array([37, 43, 51]) / 128.0
BOX_HI = np.array([91, 85, 77]) / 128.0


def _box_moments():
    V = float(np.prod(BOX_HI - BOX_LO))
    cen = (BOX_LO + BOX_HI) / 2
    return V, cen


def _box_setup(oracle, surf):
    t = I.uniform_octree(4)
    ms0 = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms0, surf)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level, active=mk != oracle.IN)
    xyz = ms.node_xyz_int.astype(np.float64) / float(1 << t.max_level)
    return t, mk, ms, xyz


def _linear_fields(xyz, A, b, q=np.zeros(3), p0=0.0):
    u = xyz @ A.T + b
    f = {"ux": u[:, 0].copy(), "uy": u[:, 1].copy(), "uz": u[:, 2].copy(), "p": xyz @ q + p0}
    f.update({"ux0": f["ux"].copy(), "uy0": f["uy"].copy(), "uz0": f["uz"].copy()})
    return f


def test_weak_bc_consistency_and_adjoint_moments(oracle):
    """u = u_prev = A x + b, g = 0, p = 0, rho = 0 (no inflow term), no penalty:
    what remains are -w.(2 mu eps(u) n) and -(2 mu eps(w) n).(u - g), and the
    continuity row -q n.(u - g). With S = A + A^T, V the box volume and c its
    centre, for m != l:
      sum_n x_m R_(n,i)      = 2 mu V S_im
      sum_n x_m x_l R_(n,i)  = mu V [2 S_im c_l + 2 S_il c_m + d_il v_m(c) + d_im v_l(c)]
      sum_n x_m R_(n,p)      = V [v_m(c) + c_m tr A]
    (every integrand is a polynomial of degree <= 2 on the faces, which the
    three-point triangle rule integrates exactly)."""
    s = I.box_surface(BOX_LO, BOX_HI)
    t, mk, ms, xyz = _box_setup(oracle, s)
    rng = np.random.default_rng(11)
    A = rng.normal(size=(3, 3)); b = rng.normal(size=3)
    mu = 0.7
    prm = oracle.params(rho=0.0, mu=mu)
    _, R, _ = oracle.weak_bc(t, ms, s, mk, _linear_fields(xyz, A, b), c_b=0.0, prm=prm, vals=False)
    R = R.reshape(-1, 4)
    V, cen = _box_moments()
    S = A + A.T
    vc = A @ cen + b
    scale = mu * V * np.abs(S).max()
    for i in range(3):
        for m in range(3):
            got = xyz[:, m] @ R[:, i]
            assert abs(got - 2 * mu * V * S[i, m]) <= 1e-12 * scale, (i, m)
            for l in range(3):
                if l == m:
                    continue
                want = mu * V * (2 * S[i, m] * cen[l] + 2 * S[i, l] * cen[m]
                                 + (i == l) * vc[m] + (i == m) * vc[l])
                got = (xyz[:, m] * xyz[:, l]) @ R[:, i]
                assert abs(got - want) <= 1e-12 * scale, (i, m, l)
    for m in range(3):
        want = V * (vc[m] + cen[m] * np.trace(A))
        assert abs(xyz[:, m] @ R[:, 3] - want) <= 1e-12 * V * np.abs(A).max()
    # the continuity row's plain sum is the net flux of a linear field: V tr A
    assert abs(R[:, 3].sum() - V * np.trace(A)) <= 1e-12 * V * np.abs(A).max()


def test_weak_bc_pressure_moment(oracle):
    """u = g, p = q.x + p0: only w.(p n) remains;
    sum_n x_m R_(n,i) = -V (d_im p(c) + c_m q_i)."""
    s = I.box_surface(BOX_LO, BOX_HI)
    t, mk, ms, xyz = _box_setup(oracle, s)
    gv = np.array([0.3, -0.2, 0.5]); q = np.array([0.9, -1.4, 0.6]); p0 = 0.35
    _, R, _ = oracle.weak_bc(t, ms, s, mk, _linear_fields(xyz, np.zeros((3, 3)), gv, q, p0),
                             c_b=4.0, g=tuple(gv), prm=oracle.params(mu=0.5), vals=False)
    R = R.reshape(-1, 4)
    V, cen = _box_moments()
    pc = q @ cen + p0
    for i, m in itertools.product(range(3), range(3)):
        want = -V * ((i == m) * pc + cen[m] * q[i])
        assert abs(xyz[:, m] @ R[:, i] - want) <= 1e-12 * V, (i, m)
    assert np.abs(R[:, 3]).max() < 1e-16


def _grid_box_surface(h):
    """The box's faces cut into rectangles on the element grid lines (spacing h),
    two outward triangles each, so that every triangle lies in one element's
    footprint. Returns the surface and the rectangles (centre, area)."""
    verts, tris, rects = [], [], []
    for k in range(3):
        a1, a2 = [d for d in range(3) if d != k]
        cuts = []
        for d in (a1, a2):
            inner = np.arange(np.floor(BOX_LO[d] / h) + 1, np.ceil(BOX_HI[d] / h)) * h
            cuts.append(np.concatenate([[BOX_LO[d]], inner[(inner > BOX_LO[d]) & (inner < BOX_HI[d])],
                                        [BOX_HI[d]]]))
        for side, x0 in ((-1, BOX_LO[k]), (1, BOX_HI[k])):
            for i in range(len(cuts[0]) - 1):
                for j in range(len(cuts[1]) - 1):
                    quad = []
                    for (u, v) in ((i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)):
                        p = np.zeros(3); p[k] = x0; p[a1] = cuts[0][u]; p[a2] = cuts[1][v]
                        quad.append(p)
                    base = len(verts)
                    verts += quad
                    # orientation: normal along side * e_k
                    n = np.cross(quad[1] - quad[0], quad[2] - quad[0])
                    if np.sign(n[k]) == side:
                        tris += [[base, base + 1, base + 2], [base, base + 2, base + 3]]
                    else:
                        tris += [[base, base + 2, base + 1], [base, base + 3, base + 2]]
                    area = (cuts[0][i + 1] - cuts[0][i]) * (cuts[1][j + 1] - cuts[1][j])
                    rects.append((np.mean(quad, 0), area))
    return I.Surface(np.array(verts), np.array(tris, np.int32), {"kind": "grid box"}), rects


def test_weak_bc_penalty_closed_form(oracle):
    """u = u_prev = g + d (constant), p = 0, rho = 0: consistency, adjoint and
    continuity parts sum to zero over a closed surface, and the penalty
    (tau_T = tau_N = tau_B) leaves sum_n phi(x_n) R_(n,i) = d_i sum over
    surface pieces of tau_B(e) int phi, with tau_B = c_b mu / max(h_b, h/100)
    and h_b the largest distance from the element's fluid corners to the box."""
    t = I.uniform_octree(4)
    h = 1.0 / 16
    s, rects = _grid_box_surface(h)
    t, mk, ms, xyz = _box_setup(oracle, s)
    gv = np.array([0.1, 0.0, -0.2]); d = np.array([0.4, -0.7, 0.25])
    mu, c_b = 0.05, 6.0
    _, R, _ = oracle.weak_bc(t, ms, s, mk, _linear_fields(xyz, np.zeros((3, 3)), gv + d), c_b=c_b,
                             g=tuple(gv), prm=oracle.params(rho=0.0, mu=mu), vals=False)
    R = R.reshape(-1, 4)
    off = np.array([[(v >> k) & 1 for k in range(3)] for v in range(8)], np.float64)
    tot0, tot1 = 0.0, np.zeros(3)
    for cen, area in rects:
        lo = np.floor(cen / h) * h
        corners = lo + h * off
        outside = np.any((corners < BOX_LO) | (corners > BOX_HI), axis=1)
        dist = np.linalg.norm(corners - np.clip(corners, BOX_LO, BOX_HI), axis=1)
        hb = max(dist[outside].max(), 0.01 * h)
        tau = c_b * mu / hb
        tot0 += tau * area
        tot1 += tau * area * cen          # int x_m over a rectangle = area * centre
    for i in range(3):
        assert abs(R[:, i].sum() - d[i] * tot0) <= 1e-12 * abs(d[i] * tot0)
        for m in range(3):
            assert abs(xyz[:, m] @ R[:, i] - d[i] * tot1[m]) <= 1e-12 * abs(d[i]) * tot0
    assert abs(R[:, 3].sum()) <= 1e-15


# ---------------------------------------------------------------------------
# Independence of the reference and its node-numbering convention
# ---------------------------------------------------------------------------


def test_oracle_imports_nothing_from_the_product_package():
    import subprocess
    import sys
    code = ("import sys; import oracle.core, oracle.mesh, oracle.mlp, oracle.window; "
            "bad = [m for m in sys.modules if m.startswith('paper_2009_00706_amd')]; "
            "print(bad); sys.exit(1 if bad else 0)")
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr


def test_morton_key_known_values_and_round_trip(oracle):
    from oracle import mesh as M
    # x in bit 0, y in bit 1, z in bit 2, then the next bit of each
    assert M.morton_key(1, 0, 0) == 1 and M.morton_key(0, 1, 0) == 2 and M.morton_key(0, 0, 1) == 4
    assert M.morton_key(2, 0, 0) == 8 and M.morton_key(3, 3, 3) == 63 and M.morton_key(5, 0, 0) == 0b1000001
    assert M.morton_key(1 << 20, 0, 0) == 1 << 60 and M.morton_key(0, 0, 1 << 20) == 1 << 62
    # ordering: sorting by key visits the 2x2x2 children of a cube with x fastest
    pts = np.array([(x, y, z) for z in range(2) for y in range(2) for x in range(2)])
    assert list(M.morton_key(pts[:, 0], pts[:, 1], pts[:, 2])) == list(range(8))
    rng = np.random.default_rng(4)
    p = rng.integers(0, 1 << 21, size=(1000, 3))
    assert np.array_equal(M._decode(M.morton_key(p[:, 0], p[:, 1], p[:, 2])), p)
    with pytest.raises(ValueError):
        M.morton_key(1 << 21, 0, 0)


def test_windowed_rows_equal_the_full_assembly(oracle):
    """The windowed reference rows used at full size (sampled nodes, local
    leaves, global numbering from the whole tree) equal the rows of the whole
    reference assembly on a cut, hanging mesh: same columns, same values."""
    import sampled_rows as SR
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    t = I.sphere_refined_octree(c, 0.25, 2, 5, 1.5)
    s = I.icosphere(2, 0.25, c)
    ms0 = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level)
    mk, _, _ = oracle.markers(t, ms0, s)
    ms = oracle.derive_mesh(t.ax, t.ay, t.az, t.level, t.max_level, active=mk != oracle.IN)
    keys = oracle._mesh.independent_node_keys(t.ax, t.ay, t.az, t.level, t.max_level)
    assert np.array_equal(keys, ms.node_keys)
    sub = oracle.subquad(t, s, np.nonzero(mk == oracle.INTERCEPTED)[0], 2)
    f = I.make_fields(ms.node_xyz_int.astype(np.float64) / float(1 << t.max_level), 4)
    V, R = oracle.assemble(t, ms, f, mk=mk, sub=sub, depth=2)
    rng = np.random.default_rng(1)
    # nodes of INTERCEPTED elements, masters of hanging vertices, inactive nodes, random ones
    cutm = ms.masters[mk == oracle.INTERCEPTED].ravel()
    hang_el = np.nonzero((ms.C > 0).sum(2).max(1) > 1)[0]
    hm = ms.masters[hang_el].ravel()
    nodes = np.unique(np.concatenate([rng.choice(cutm[cutm >= 0], 6), rng.choice(hm[hm >= 0], 6),
                                      rng.choice(np.nonzero(~ms.node_active)[0], 2),
                                      rng.choice(ms.n_nodes, 6)]))
    ref = SR.reference_rows(oracle, t, s, f, keys, nodes, depth=2)
    for n in nodes:
        rows = ref[int(n)]
        assert rows["active"] == ms.node_active[n]
        for c in range(4):
            r = 4 * n + c
            a, b = ms.row_ptr[r], ms.row_ptr[r + 1]
            assert np.array_equal(rows["cols"][c], ms.col_idx[a:b])
            np.testing.assert_allclose(rows["vals"][c], V[a:b], rtol=0,
                                       atol=1e-14 * max(np.abs(V[a:b]).sum(), 1e-300))
            assert abs(rows["resid"][c] - R[r]) <= 1e-14 * max(np.abs(R).max(), 1e-300)
