"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every test here checks the oracle against something other than itself: the
moment identities the paper prints for its equilibria, conservation laws,
closed forms (shape functions, motion laws, rigid-body characteristics,
Gauss's theorem for the force integral), brute force, and the paper's
free-stream table.  None of them re-derives a value through the oracle's own
formula.
"""

import math

import numpy as np
import pytest

from paper_2002_04353_amd import cases, meshgen

V = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]], float)
CV = 1.0 / (1.4 - 1.0)
RNG = np.random.default_rng(1234)


def _states(n=6):
    for _ in range(n):
        yield (RNG.uniform(0.5, 1.5), RNG.uniform(-0.2, 0.2), RNG.uniform(-0.2, 0.2), RNG.uniform(0.15, 0.35))


# --------------------------------------------------------------------------
# equilibria: moments printed in Sec. IV (eqs. feq, geq_gstar, tab. Eq_Moments)
# --------------------------------------------------------------------------

def test_feq_moments_and_third_moment_deviation(oracle_mod):
    O = oracle_mod
    for rho, ux, uy, T in _states():
        f = O.feq(rho, ux, uy, T)
        u = np.array([ux, uy])
        assert abs(f.sum() - rho) < 1e-14
        np.testing.assert_allclose(V.T @ f, rho * u, atol=1e-14)
        P = np.einsum("ia,ib,i->ab", V, V, f)
        np.testing.assert_allclose(P, rho * np.outer(u, u) + rho * T * np.eye(2), atol=1e-14)
        # the lattice third moment deviates from Maxwell-Boltzmann's rho u^3 + 3 rho u T
        # by exactly Q'_aaa = rho u (1 - 3T) - rho u^3 (eq. DeviationTerms)
        for a in range(2):
            lattice = np.sum(V[:, a] ** 3 * f)
            mb = rho * u[a] ** 3 + 3.0 * rho * u[a] * T
            q_dev = rho * u[a] * (1 - 3 * T) - rho * u[a] ** 3
            assert abs((lattice - mb) - q_dev) < 1e-14


def test_geq_moments(oracle_mod):
    O = oracle_mod
    for rho, ux, uy, T in _states():
        g = O.geq(rho, ux, uy, T)
        u = np.array([ux, uy])
        E = CV * T + 0.5 * u @ u
        assert abs(g.sum() - 2 * rho * E) < 1e-13
        np.testing.assert_allclose(V.T @ g, 2 * rho * u * (E + T), atol=1e-13)
        R = np.einsum("ia,ib,i->ab", V, V, g)
        Req = 2 * rho * E * (T * np.eye(2) + np.outer(u, u)) + 2 * rho * T * (T * np.eye(2) + 2 * np.outer(u, u))
        np.testing.assert_allclose(R, Req, atol=1e-13)


def test_quasi_equilibrium(oracle_mod):
    O = oracle_mod
    for rho, ux, uy, T in _states():
        u = np.array([ux, uy])
        E = CV * T + 0.5 * u @ u
        Peq = rho * np.outer(u, u) + rho * T * np.eye(2)
        # at P = P^eq the quasi-equilibrium coincides with the equilibrium
        g0 = O.gqe(rho, ux, uy, T, [Peq[0, 0], Peq[0, 1], Peq[1, 1]])
        np.testing.assert_allclose(g0, O.geq(rho, ux, uy, T), atol=1e-14)
        # away from it, its heat flux is q^eq + 2 u.(P - P^eq) and R stays R^eq
        dP = RNG.normal(0, 0.01, (2, 2))
        dP = dP + dP.T
        P = Peq + dP
        gs = O.gqe(rho, ux, uy, T, [P[0, 0], P[0, 1], P[1, 1]])
        np.testing.assert_allclose(V.T @ gs, 2 * rho * u * (E + T) + 2 * dP @ u, atol=1e-13)
        assert abs(gs.sum() - 2 * rho * E) < 1e-13


# --------------------------------------------------------------------------
# collision (eqs. feqn, geqn, Ai)
# --------------------------------------------------------------------------

def test_collision_conservation_and_correction_moments(oracle_mod):
    O = oracle_mod
    for rho, ux, uy, T in _states():
        ft = O.feq(rho, ux, uy, T) * (1 + RNG.normal(0, 0.05, 9))
        gt = O.geq(rho, ux, uy, T) * (1 + RNG.normal(0, 0.05, 9))
        dt = 0.7
        fs, gs = O.collide(ft, gt, [0.0, 0.0], 1.4, 0.71, 0.01, dt)
        assert abs(fs.sum() - ft.sum()) < 1e-13
        np.testing.assert_allclose(V.T @ fs, V.T @ ft, atol=1e-13)
        assert abs(gs.sum() - gt.sum()) < 1e-13
        X = RNG.normal(0, 0.1, 2)
        fx, gx = O.collide(ft, gt, X, 1.4, 0.71, 0.01, dt)
        # phi_i = A_ia X_a: no mass, momentum source exactly dt X
        assert abs(fx.sum() - ft.sum()) < 1e-13
        np.testing.assert_allclose(V.T @ fx - V.T @ ft, dt * X, atol=1e-13)
        np.testing.assert_allclose(gx, gs, atol=0)


def test_collision_equilibrium_is_fixed_point(oracle_mod):
    O = oracle_mod
    for rho, ux, uy, T in _states():
        f = O.feq(rho, ux, uy, T)
        g = O.geq(rho, ux, uy, T)
        fs, gs = O.collide(f, g, [0.0, 0.0], 1.4, 0.71, 0.003, 1.0)
        np.testing.assert_allclose(fs, f, atol=1e-14)
        np.testing.assert_allclose(gs, g, atol=1e-14)


def test_collision_relaxation_rates(oracle_mod):
    """The shear stress relaxes with w, where mu = (1/w - 1/2) rho T dt."""
    O = oracle_mod
    rho, ux, uy, T, mu, dt = 1.0, 0.05, -0.02, 0.3, 0.02, 0.5
    f = O.feq(rho, ux, uy, T)
    g = O.geq(rho, ux, uy, T)
    d = np.zeros(9)
    d[5] = d[7] = 1e-3
    d[6] = d[8] = -1e-3  # pure xy-stress perturbation: no mass or momentum
    fs, _ = O.collide(f + d, g, [0.0, 0.0], 1.4, 0.71, mu, dt)
    w = 1.0 / (mu / (rho * T * dt) + 0.5)
    pxy_in = np.sum(V[:, 0] * V[:, 1] * (f + d))
    pxy_out = np.sum(V[:, 0] * V[:, 1] * fs)
    pxy_eq = rho * ux * uy
    assert abs((pxy_out - pxy_eq) - (1 - w) * (pxy_in - pxy_eq)) < 1e-14


def _w1(mu, Pr, rho, T, dt):
    # kappa = Cp (1/w1 - 1/2) rho T dt and Pr = Cp mu / kappa  =>  1/w1 = mu / (Pr rho T dt) + 1/2
    return 1.0 / (mu / (Pr * rho * T * dt) + 0.5)


def test_heat_flux_relaxation_rate(oracle_mod):
    """The energy populations relax at w1, set by the Prandtl number (Sec. IV,
    eq. geqn with kappa = Cp (1/w1 - 1/2) rho T dt and Pr = Cp mu / kappa).

    With f at equilibrium (P = P^eq) the quasi-equilibrium coincides with g^eq,
    so every moment of g that the equilibrium fixes relaxes by (1 - w1): the
    heat flux q = sum c g and the second moment R = sum c c g.  At Pr = 0.71,
    w1 differs from w, so this fails if w1 is replaced by w or the (w1 - w)
    term changes sign."""
    O = oracle_mod
    mu, dt, Pr = 0.02, 0.5, 0.71
    for rho, ux, uy, T in _states():
        u = np.array([ux, uy])
        E = CV * T + 0.5 * u @ u
        w = 1.0 / (mu / (rho * T * dt) + 0.5)
        w1 = _w1(mu, Pr, rho, T, dt)
        assert abs(w1 - w) > 1e-3
        f = O.feq(rho, ux, uy, T)
        d = np.zeros(9)
        d[1], d[3] = 2e-3, -2e-3      # heat flux along x: no energy, no second moment
        d[2], d[4] = -1e-3, 1e-3      # and along y
        d[5] = d[7] = 5e-4            # R_xy: no energy, no heat flux
        d[6] = d[8] = -5e-4
        g = O.geq(rho, ux, uy, T) + d
        fs, gs = O.collide(f, g, [0.0, 0.0], 1.4, Pr, mu, dt)
        np.testing.assert_allclose(fs, f, atol=1e-15)
        q_eq = 2 * rho * u * (E + T)                                   # tab. Eq_Moments
        Rxy_eq = 2 * rho * E * ux * uy + 2 * rho * T * 2 * ux * uy     # tab. Eq_Moments
        np.testing.assert_allclose(V.T @ gs - q_eq, (1 - w1) * (V.T @ g - q_eq), rtol=0, atol=1e-14)
        rxy_in = np.sum(V[:, 0] * V[:, 1] * g)
        rxy_out = np.sum(V[:, 0] * V[:, 1] * gs)
        assert abs((rxy_out - Rxy_eq) - (1 - w1) * (rxy_in - Rxy_eq)) < 1e-14
        assert abs(gs.sum() - g.sum()) < 1e-14


def test_heat_flux_coupling_to_stress(oracle_mod):
    """With g at equilibrium and f carrying a shear stress, the energy
    populations take the heat flux of the quasi-equilibrium: the collision
    adds (w1 - w)(g* - g^eq), whose first moment is (w1 - w) 2 u_b (P_ab -
    P^eq_ab) (Sec. IV, eq. geqn and the q* entry of tab. Eq_Moments)."""
    O = oracle_mod
    mu, dt, Pr = 0.02, 0.5, 0.71
    for rho, ux, uy, T in _states():
        u = np.array([ux, uy])
        E = CV * T + 0.5 * u @ u
        w = 1.0 / (mu / (rho * T * dt) + 0.5)
        w1 = _w1(mu, Pr, rho, T, dt)
        f = O.feq(rho, ux, uy, T)
        d = np.zeros(9)
        d[5] = d[7] = 1e-3
        d[6] = d[8] = -1e-3           # P_xy + 4e-3: no mass or momentum
        g = O.geq(rho, ux, uy, T)
        _, gs = O.collide(f + d, g, [0.0, 0.0], 1.4, Pr, mu, dt)
        dP = np.array([[0.0, 4e-3], [4e-3, 0.0]])
        q_eq = 2 * rho * u * (E + T)
        np.testing.assert_allclose(V.T @ gs - q_eq, (w1 - w) * 2 * dP @ u, rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# Grad approximation of missing populations (Sec. IV.A, tab. Neq_Moments)
# --------------------------------------------------------------------------

def test_grad_missing_moments(oracle_mod):
    O = oracle_mod
    mu, dt = 0.01, 0.5
    for rho, ux, uy, T in _states():
        gu = RNG.normal(0, 0.05, 4)
        gT = RNG.normal(0, 0.05, 2)
        fm, gm = O.grad_missing(rho, ux, uy, T, gu, gT, 1.4, 0.71, mu, dt)
        f1 = (fm - O.feq(rho, ux, uy, T)) / dt
        g1 = (gm - O.geq(rho, ux, uy, T)) / dt
        # no mass or momentum in f^(1); no energy in g^(1)
        assert abs(f1.sum()) < 1e-12
        np.testing.assert_allclose(V.T @ f1, 0.0, atol=1e-12)
        assert abs(g1.sum()) < 1e-12
        # shear stress of f^(1): the Newtonian stress tau = mu S_xy follows from
        # the pre-collision non-equilibrium as tau = -(1 - w/2) dt P^(1)_xy
        w = 1.0 / (mu / (rho * T * dt) + 0.5)
        Sxy = gu[1] + gu[2]
        Pxy = np.sum(V[:, 0] * V[:, 1] * f1)
        assert abs(-(1 - w / 2) * dt * Pxy - mu * Sxy) < 1e-12
        # heat flux of g^(1) with the velocity gradients switched off: the
        # non-equilibrium energy flux (1 - w1/2) dt q^(1) / 2 is Fourier's -kappa grad T
        # with kappa = Cp mu / Pr (the first moment of g carries twice the energy flux)
        fm0, gm0 = O.grad_missing(rho, ux, uy, T, np.zeros(4), gT, 1.4, 0.71, mu, dt)
        q1 = V.T @ ((gm0 - O.geq(rho, ux, uy, T)) / dt)
        w1 = 1.0 / (mu / (0.71 * rho * T * dt) + 0.5)
        kappa = (CV + 1) * mu / 0.71
        np.testing.assert_allclose((1 - w1 / 2) * dt * q1 / 2, -kappa * gT, atol=1e-12)
    # zero gradients: the missing populations are the equilibrium
    fm, gm = O.grad_missing(1.0, 0.0, 0.0, 0.3, np.zeros(4), np.zeros(2), 1.4, 0.71, mu, dt)
    np.testing.assert_allclose(fm, O.feq(1.0, 0, 0, 0.3), atol=1e-15)
    np.testing.assert_allclose(gm, O.geq(1.0, 0, 0, 0.3), atol=1e-15)


# --------------------------------------------------------------------------
# P2 shape functions (Sec. III, eq. Propagation; GCL, Sec. III.A)
# --------------------------------------------------------------------------

def test_p2_shape_functions(oracle_mod):
    O = oracle_mod
    nodes = [np.array(v, float) for v in ([1, 0, 0], [0, 1, 0], [0, 0, 1], [0, .5, .5], [.5, 0, .5], [.5, .5, 0])]
    for s, lam in enumerate(nodes):
        N = O.p2_shape(lam)
        e = np.zeros(6)
        e[s] = 1.0
        np.testing.assert_allclose(N, e, atol=1e-15)
    # partition of unity and exact reproduction of quadratics on a reference triangle
    P = np.array([[0.0, 0.0], [1.0, 0.2], [0.3, 0.9]])
    nodes_xy = [P[0], P[1], P[2], 0.5 * (P[1] + P[2]), 0.5 * (P[2] + P[0]), 0.5 * (P[0] + P[1])]
    q = lambda x: 0.3 + 1.1 * x[0] - 0.7 * x[1] + 0.9 * x[0] ** 2 - 1.3 * x[0] * x[1] + 0.4 * x[1] ** 2
    qn = np.array([q(x) for x in nodes_xy])
    for _ in range(50):
        lam = RNG.dirichlet([1, 1, 1]) * 1.4 - 0.1  # inside and slightly outside
        lam[0] = 1 - lam[1] - lam[2]
        N = O.p2_shape(lam)
        assert abs(N.sum() - 1.0) < 1e-14
        x = lam[0] * P[0] + lam[1] * P[1] + lam[2] * P[2]
        assert abs(N @ qn - q(x)) < 1e-13


# --------------------------------------------------------------------------
# mesh motion: metrics against finite differences and closed forms (Sec. II)
# --------------------------------------------------------------------------

MOTIONS = [
    dict(motion="sine", motion_p=[0.05, 1.0, 1.0, 3.0]),
    dict(motion="plunge", motion_p=[0.3, 1.7, 0.2]),
    dict(motion="pitch_plunge", motion_p=[0.3, 1.3, 0.25, 0.05, 0.1, 0.2, 0.4, 0.0, 0.0]),
    dict(motion="pitch_plunge", motion_p=[0.3, 1.3, 0.25, 0.05, 0.1, 0.2, 0.4, 0.6, 2.0]),
]


@pytest.mark.parametrize("mo", MOTIONS, ids=["sine", "plunge", "pitch_rigid", "pitch_blend"])
def test_motion_metrics_finite_differences(oracle_mod, mo):
    O = oracle_mod
    p = dict(dt=1.0, mu=0.0, **mo)
    h = 1e-6
    for _ in range(20):
        X, Y, t = RNG.uniform(-1.5, 1.5), RNG.uniform(-1.5, 1.5), RNG.uniform(0, 3)
        x, J, v = O.motion(p, X, Y, t)
        xpX = O.motion(p, X + h, Y, t)[0]
        xmX = O.motion(p, X - h, Y, t)[0]
        xpY = O.motion(p, X, Y + h, t)[0]
        xmY = O.motion(p, X, Y - h, t)[0]
        xpt = O.motion(p, X, Y, t + h)[0]
        xmt = O.motion(p, X, Y, t - h)[0]
        Jfd = np.stack([(xpX - xmX) / (2 * h), (xpY - xmY) / (2 * h)], axis=1)
        np.testing.assert_allclose(J, Jfd, atol=1e-8)
        np.testing.assert_allclose(v, (xpt - xmt) / (2 * h), atol=1e-8)
        if mo["motion"] in ("plunge",) or (mo["motion"] == "pitch_plunge" and mo["motion_p"][8] <= 0):
            assert abs(np.linalg.det(J) - 1.0) < 1e-14


def test_sine_motion_determinant_closed_form(oracle_mod):
    O = oracle_mod
    a, Tp = 0.05, 3.0
    p = dict(dt=1.0, mu=0.0, motion="sine", motion_p=[a, 1.0, 1.0, Tp])
    for _ in range(20):
        X, Y, t = RNG.uniform(0, 1, 3)
        _, J, _ = O.motion(p, X, Y, t)
        # x = X + d, y = Y + d  =>  det J = 1 + d_X + d_Y = 1 + 2 pi a s(t) sin(2 pi (X + Y))
        det = 1 + 2 * math.pi * a * math.sin(2 * math.pi * t / Tp) * math.sin(2 * math.pi * (X + Y))
        assert abs(np.linalg.det(J) - det) < 1e-14


# --------------------------------------------------------------------------
# locate and interpolate (Sec. III, eqs. NonLinear_Eq, Propagation)
# --------------------------------------------------------------------------

def test_walk_matches_brute_force(oracle_mod):
    O = oracle_mod
    m = meshgen.periodic_square(12, 10, 1.0, 1.0, jitter=0.25, seed=7)
    o = O.Oracle(m.arrays(), dict(dt=0.01, mu=0.001))
    K = np.sin(2 * np.pi * m.X[:, 0]) * np.cos(2 * np.pi * m.X[:, 1]) + m.X[:, 0] * 0
    for _ in range(200):
        P = RNG.uniform(0, 1, 2)
        e0 = int(RNG.integers(0, m.n_elems))
        # start the walk from a random element: the point is expressed in that element's frame
        v0 = m.X[m.elem[e0, 0]]
        Pf = P + np.round((v0 - P) / 1.0)
        st, e, lam, steps = o.locate(e0, Pf)
        assert st == 0
        assert lam.min() >= -1e-12
        stb, eb, lamb = o.brute_locate(P)
        assert stb == 0
        st2, val = o.interpolate(e0, Pf, K)
        st3, valb = o.interpolate(eb, P + np.round((m.X[m.elem[eb, 0]] - P) / 1.0), K)
        assert st2 == 0 and st3 == 0
        assert abs(val - valb) < 1e-13


def test_propagation_reproduces_quadratics(oracle_mod):
    """With the collision switched off, one step moves a quadratic field exactly
    along c^_i = c_i - v_g (plunge: J = I, uniform grid velocity)."""
    O = oracle_mod
    m = meshgen.structured_square(12, 12, 1.0, 1.0, jitter=0.2, seed=3)
    dt = 0.02
    p = dict(dt=dt, mu=0.001, motion="plunge", motion_p=[0.05, 2.0, 0.3], T_inf=0.3)
    o = O.Oracle(m.arrays(), p, flags=O.F_NO_COLLIDE)
    X = m.X
    coef = RNG.normal(0, 1, (18, 6))
    q = lambda c, x, y: c[0] + c[1] * x + c[2] * y + c[3] * x * x + c[4] * x * y + c[5] * y * y
    pops = np.stack([q(coef[k], X[:, 0], X[:, 1]) for k in range(18)])
    mac = np.zeros((4, m.n_nodes))
    mac[0] = 1.0
    mac[3] = 0.3
    t0 = 0.4
    o.set_state(pops, mac, t0, 0)
    o.step(1)
    pt, mw, mf = o.streamed()
    vy = -0.05 * 2.0 * math.cos(2.0 * (t0 + 0.5 * dt) + 0.3)
    inside = (mf == 0) & (mw == 0)
    assert inside.sum() > 0.6 * m.n_nodes
    for k in range(18):
        i = k % 9
        xd = X[:, 0] - dt * V[i, 0]
        yd = X[:, 1] - dt * (V[i, 1] - vy)
        exact = q(coef[k], xd, yd)
        ok = (mf & (1 << i)) == 0
        np.testing.assert_allclose(pt[k][ok], exact[ok], atol=1e-12)


def _pitch_G(p, X, t):
    A, w, Xc, Yc, php, h, phh = p[:7]
    th = A * math.sin(w * t + php)
    R = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    return R, np.array([Xc, Yc]), np.array([0.0, -h * math.sin(w * t + phh)])


def test_departure_point_follows_the_characteristic(oracle_mod):
    """Rigid pitch + plunge: the exact departure point in computational
    coordinates is G^-1(G(X, t+dt) - c dt, t).  The traced departure point (read
    back through a linear field, which P2 reproduces exactly) must approach it
    at third order per step."""
    O = oracle_mod
    m = meshgen.structured_square(10, 10, 2.0, 2.0, jitter=0.1, seed=5)
    mp = [0.6, 2.0, 1.0, 1.0, 0.3, 0.1, 0.7, 0.0, 0.0]
    X = m.X
    a_x, a_y = 0.37, -0.81
    errs = []
    for dt in (0.02, 0.01, 0.005):
        p = dict(dt=dt, mu=0.001, motion="pitch_plunge", motion_p=mp, T_inf=0.3)
        o = O.Oracle(m.arrays(), p, flags=O.F_NO_COLLIDE)
        pops = np.tile(a_x * X[:, 0] + a_y * X[:, 1], (18, 1))
        mac = np.zeros((4, m.n_nodes))
        mac[0] = 1.0
        mac[3] = 0.3
        t0 = 0.3
        o.set_state(pops, mac, t0, 0)
        o.step(1)
        pt, mw, mf = o.streamed()
        err = 0.0
        sel = np.nonzero((mf == 0) & (np.hypot(X[:, 0] - 1, X[:, 1] - 1) < 0.6))[0]
        for i in range(1, 9):
            R1, c1, s1 = _pitch_G(mp, None, t0 + dt)
            R0, c0, s0 = _pitch_G(mp, None, t0)
            for a in sel[:40]:
                x1 = c1 + R1 @ (X[a] - c1) + s1
                xd = x1 - dt * V[i]
                Xd = c0 + R0.T @ (xd - s0 - c0)
                err = max(err, abs(pt[i][a] - (a_x * Xd[0] + a_y * Xd[1])))
        errs.append(err)
    r1 = math.log2(errs[0] / errs[1])
    r2 = math.log2(errs[1] / errs[2])
    assert r1 > 2.6 and r2 > 2.6, errs


# --------------------------------------------------------------------------
# FE derivatives (eqs. Ph_Derivative, FE_Derivative)
# --------------------------------------------------------------------------

def test_node_gradient_exact_for_quadratics_under_rigid_motion(oracle_mod):
    O = oracle_mod
    m = meshgen.structured_square(8, 8, 2.0, 2.0, jitter=0.2, seed=11)
    mp = [0.5, 1.0, 1.0, 1.0, 0.2, 0.3, 0.1, 0.0, 0.0]
    p = dict(dt=0.1, mu=0.001, motion="pitch_plunge", motion_p=mp)
    o = O.Oracle(m.arrays(), p)
    t = 0.9
    R, c, s = _pitch_G(mp, None, t)
    x = (c + (m.X - c) @ R.T) + s
    q = lambda x, y: 0.2 + 0.5 * x - 0.3 * y + 0.7 * x * x - 0.4 * x * y + 0.9 * y * y
    K = q(x[:, 0], x[:, 1])
    g = o.node_gradient(K, t)
    gx = 0.5 + 1.4 * x[:, 0] - 0.4 * x[:, 1]
    gy = -0.3 - 0.4 * x[:, 0] + 1.8 * x[:, 1]
    np.testing.assert_allclose(g[:, 0], gx, atol=1e-12)
    np.testing.assert_allclose(g[:, 1], gy, atol=1e-12)


def test_owner_is_largest_containing_element(oracle_mod):
    O = oracle_mod
    m = meshgen.periodic_square(9, 7, 1.0, 1.0, jitter=0.25, seed=13)
    o = O.Oracle(m.arrays(), dict(dt=0.01, mu=0.001))
    own = o.owner()
    P = m.X[m.elem[:, :3]]
    P = P.copy()
    for k in (1, 2):
        P[:, k] = P[:, k] + np.round((P[:, 0] - P[:, k]) / 1.0)
    area = 0.5 * ((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))
    for a in range(m.n_nodes):
        es = np.nonzero((m.elem == a).any(axis=1))[0]
        assert own[a] == es[np.argmax(area[es])]


# --------------------------------------------------------------------------
# whole step: free-stream preservation (Sec. III.A; Sec. V.A, tab. GCL_Error)
# --------------------------------------------------------------------------

def test_free_stream_preservation_paper_values(oracle_mod):
    """The paper's free-stream test: T=0.2, Ma=0.2, deformation amplitude
    500/8000 of the box, t0 = 1.5 L/u, run to t* = 1.  The paper reports
    relative velocity errors of 1.1e-15 .. 3.9e-16."""
    O = oracle_mod
    c = cases.uniform(nx=25, ny=20, paper=True)
    o = O.Oracle(c["mesh"].arrays(), c["params"])
    o.init_fields(**c["init"])
    o.step(c["steps"])
    mac = o.fields()
    u = c["params"]["u_inf"][0]
    eps = np.sum(np.hypot(mac[1] - u, mac[2])) / np.sum(np.full(mac.shape[1], u))
    assert eps < 1e-13
    assert np.abs(mac[0] - 1.0).max() < 1e-13


def test_rest_state_with_moving_walls_is_preserved(oracle_mod):
    """A fluid at rest around a wall at rest stays at rest (the Grad missing
    populations reduce to the equilibrium)."""
    O = oracle_mod
    c = cases.small("plunge", n_nodes=8000)
    p = dict(c["params"])
    p["u_inf"] = (0.0, 0.0)
    p["motion"] = "none"
    o = O.Oracle(c["mesh"].arrays(), p)
    N = c["mesh"].n_nodes
    o.init_fields(np.ones(N), np.zeros(N), np.zeros(N), np.full(N, 0.3))
    o.step(20)
    mac = o.fields()
    assert np.abs(mac[0] - 1).max() < 1e-12
    assert np.abs(mac[1:3]).max() < 1e-12


def test_vortex_convergence_order(oracle_mod):
    """Isentropic vortex on a deforming periodic mesh at fixed CFL: the density
    error against the translated analytic vortex falls at about second order
    (the paper's second-order finite-element reconstruction, Sec. II/III)."""
    O = oracle_mod
    L = 32.0
    ns, errs = [12, 16, 24, 32], []
    for n in ns:
        c = cases.vortex(n=n, L=L, beta=1.0, Re_R=3e3, amp_frac=0.05,
                         period_steps=int(round(4 * L / (0.25 * L / n))))
        p = c["params"]
        o = O.Oracle(c["mesh"].arrays(), p)
        o.init_fields(**c["init"])
        o.step(int(round(8.0 / p["dt"])))
        pops, mac, t, _ = o.state()
        _, x, _, _, _ = o.move_mesh(t)
        v = c["vortex"]
        rho = cases.vortex_fields(x[:, 0], x[:, 1], t, L, v["U"], v["R"], v["beta"], v["T_inf"])[0]
        errs.append(np.sqrt(np.mean((mac[0] - rho) ** 2)))
    slope = -np.polyfit(np.log(ns), np.log(errs), 1)[0]
    assert 1.8 < slope < 3.5, (errs, slope)


# --------------------------------------------------------------------------
# forces (Sec. V.B / V.C coefficient definitions): Gauss's theorem
# --------------------------------------------------------------------------

def _wall_polygon(m):
    """Area and centroid of the body bounded by the wall edges (straight P2
    edges: the mid-edge nodes lie on the chords), by the shoelace formulas over
    the directed edges, each oriented with the fluid on its left."""
    s = cx = cy = 0.0
    for e, k in m.wall_edges:
        a = m.X[m.elem[e, (k + 1) % 3]]
        b = m.X[m.elem[e, (k + 2) % 3]]
        cr = a[0] * b[1] - b[0] * a[1]
        s += 0.5 * cr
        cx += (a[0] + b[0]) * cr
        cy += (a[1] + b[1]) * cr
    # fluid on the left => the body is traversed clockwise (negative signed area)
    return -s, cx / (6.0 * s), cy / (6.0 * s)


def test_force_closed_forms(oracle_mod):
    """Gauss's theorem over the body B (normal n out of the body), for the
    force F = -int p n + int tau n and the moment about the reference point
    r0, nose-up positive: M = -int ((x - r0) x traction)_z (Sec. V.B/V.C
    coefficient definitions).  Every traction below is at most quadratic along
    a straight edge, where Simpson's rule is exact."""
    O = oracle_mod
    c = cases.small("plunge", n_nodes=8000)
    m = c["mesh"]
    p = dict(c["params"])
    p["motion"] = "none"
    o = O.Oracle(m.arrays(), p)
    N = m.n_nodes
    pops = np.zeros((18, N))
    X = m.X
    area, xc, yc = _wall_polygon(m)
    x0, y0 = p["ref_point"]
    assert area > 0 and 0.3 * 200 < xc < 0.5 * 200 and abs(yc) < 1.0
    mu = p["mu"]
    qc = 0.5 * p["rho_inf"] * (p["u_inf"][0] ** 2 + p["u_inf"][1] ** 2) * p["chord"]
    # uniform pressure on a closed body: no force, no moment
    mac = np.stack([np.full(N, 1.3), np.zeros(N), np.zeros(N), np.full(N, 0.3)])
    o.set_state(pops, mac, 0.0, 0)
    F = o.forces()
    assert np.abs(F["F_p"]).max() < 1e-10 * 0.39 * 400
    assert abs(F["M_p"]) < 1e-10 * 0.39 * 400 * 200
    # linear pressure p = a + b.x:  F_p = -b Area,
    # M_p = int_B (b_y (x - x0) - b_x (y - y0)) = Area (b_y (xc - x0) - b_x (yc - y0))
    bx, by = 0.002, -0.003
    rho = (1.0 + bx * X[:, 0] + by * X[:, 1]) / 0.3
    mac = np.stack([rho, np.zeros(N), np.zeros(N), np.full(N, 0.3)])
    o.set_state(pops, mac, 0.0, 0)
    F = o.forces()
    np.testing.assert_allclose(F["F_p"], [-bx * area, -by * area], rtol=1e-10)
    Mp = area * (by * (xc - x0) - bx * (yc - y0))
    assert abs(F["M_p"] - Mp) < 1e-10 * abs(Mp), (F["M_p"], Mp)
    assert abs(F["cm"] - (F["M_p"] + F["M_v"]) / (qc * p["chord"])) < 1e-14 * abs(F["cm"]) + 1e-300
    # a downward force behind the reference point pitches the nose up
    assert (by * (xc - x0) > 0) == (F["M_p"] > 0)
    # rigid rotation u = W x r has no strain: no viscous force or moment
    Wz = 0.01
    mac = np.stack([np.ones(N), -Wz * X[:, 1], Wz * X[:, 0], np.full(N, 0.3)])
    o.set_state(pops, mac, 0.0, 0)
    F = o.forces()
    assert np.abs(F["F_v"]).max() < 1e-14
    assert abs(F["M_v"]) < 1e-12
    # simple shear u = (s y, 0) on a closed body: viscous force mu s (n_y, n_x)
    # integrated over the closed surface vanishes
    mac = np.stack([np.ones(N), 0.01 * X[:, 1], np.zeros(N), np.full(N, 0.3)])
    o.set_state(pops, mac, 0.0, 0)
    F = o.forces()
    assert np.abs(F["F_v"]).max() < 1e-14
    # u = (0, s x^2 / 2): tau = mu s x (e_x e_y + e_y e_x), traction mu s x (n_y, n_x);
    # F_v = (0, mu s Area), M_v = -mu s int_B (x - x0) = -mu s Area (xc - x0).
    # P2 holds the quadratic exactly, so the nodal gradients are exact.
    s = 1e-4
    mac = np.stack([np.ones(N), np.zeros(N), 0.5 * s * X[:, 0] ** 2, np.full(N, 0.3)])
    o.set_state(pops, mac, 0.0, 0)
    F = o.forces()
    np.testing.assert_allclose(F["F_v"], [0.0, mu * s * area], rtol=0, atol=1e-10 * mu * s * area)
    Mv = -mu * s * area * (xc - x0)
    assert abs(F["M_v"] - Mv) < 1e-9 * abs(Mv), (F["M_v"], Mv)


# --------------------------------------------------------------------------
# meshes (input generator invariants)
# --------------------------------------------------------------------------

def test_mesh_invariants():
    m = meshgen.periodic_square(20, 16, 1.0, 1.0, seed=1)
    V_ = m.n_vertices
    assert m.n_nodes == 4 * V_ and m.n_elems == 2 * V_
    for e in range(m.n_elems):
        for k in range(3):
            n = m.nbr[e, k]
            assert n >= 0 and e in m.nbr[n]
    a = meshgen.naca_omesh(6000, seed=3)
    assert len(a.wall_edges) == a.meta["n_surface"]
    assert set(np.unique(a.nbr[a.nbr < 0])) == {-1, -2}


def test_energy_equilibrium_rest_weight(oracle_mod):
    """Linearised about rest, the energy equilibrium distributes an increment of
    sum g over the directions with weights v_i = d g^eq_i / d(2 rho E).  From the
    G form (eq. geq_gstar) with its temperature-dependent W_i, v_0 = W_0(T) +
    (2 rho E) dW_0/dT / (2 rho Cv) + ... changes sign between T = 0.2 and 0.3:
    the rest weight is negative at the airfoil temperature 0.3.  This is the
    property behind the step-size reading (CFL 0.25) of the workloads.  It
    differentiates the oracle's own g^eq, so it documents a property and is
    not a pin of the oracle."""
    O = oracle_mod
    Cv = 2.5
    for T, sign in ((0.2, 1.0), (0.3, -1.0), (1.0 / 3.0, -1.0)):
        eps = 1e-7
        g0 = O.geq(1.0, 0.0, 0.0, T)
        g1 = O.geq(1.0, 0.0, 0.0, T + eps / (2 * Cv))
        v = (g1 - g0) / eps
        assert abs(v.sum() - 1.0) < 1e-6
        assert np.sign(v[0]) == sign
