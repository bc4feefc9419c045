"""Pins of the oracle's splitting steps and monitors (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import mumode as om
from oracle import operators as op
from oracle import schemes as sc


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def _gpe_setup(n=16, a=-8.0, b=8.0, tau=0.05, beta=100.0):
    E = op.ho_exponential(n, a, b, tau)
    psi = synth.thomas_fermi_initial(n, a, b, 3, beta, cfg_id=4)
    return psi, [E, E, E]


def test_gpe_beta_zero_reduces_to_integrator():
    psi, E = _gpe_setup()
    out = sc.gpe_strang(psi, E, 0.05, 0.0, 3)
    assert _rel(out, om.expstep(psi, E, 3)) < 1e-14


def test_gpe_nonlinear_flow_solves_its_ode():
    g = synth.rng(201, 0)
    psi = synth.random_tensor((5, 6, 7), True, g)
    beta, s, ds = 100.0, 0.013, 1e-6
    out = sc.gpe_nonlinear(psi, s, beta)
    assert np.max(np.abs(np.abs(out) - np.abs(psi))) < 1e-14
    # d/ds N(s) psi = -i beta |N(s) psi|^2 N(s) psi   (central difference in s)
    dNds = (sc.gpe_nonlinear(psi, s + ds, beta) - sc.gpe_nonlinear(psi, s - ds, beta)) / (2 * ds)
    rhs = -1j * beta * np.abs(out) ** 2 * out
    assert _rel(dNds, rhs) < 1e-6
    # flows compose: N(a) N(b) = N(a + b)
    assert _rel(sc.gpe_nonlinear(sc.gpe_nonlinear(psi, 0.01, beta), 0.003, beta),
                sc.gpe_nonlinear(psi, 0.013, beta)) < 1e-13


def test_gpe_merged_equals_unmerged():
    psi, E = _gpe_setup()
    a = sc.gpe_strang(psi, E, 0.05, 100.0, 4)
    b = sc.gpe_strang_merged(psi, E, 0.05, 100.0, 4)
    assert _rel(b, a) < 1e-13


def test_gpe_mass_conserved():
    n, a, b = 16, -8.0, 8.0
    psi, E = _gpe_setup(n, a, b)
    h = (b - a) / (n + 1)
    m0 = sc.norm2(psi, h ** 3)
    m1 = sc.norm2(sc.gpe_strang(psi, E, 0.05, 100.0, 5), h ** 3)
    assert abs(m0 - 1.0) < 1e-13 and abs(m1 - m0) < 1e-13


def test_gpe_strang_second_order():
    n, a, b, beta, T = 12, -6.0, 6.0, 100.0, 0.2
    psi0 = synth.thomas_fermi_initial(n, a, b, 3, beta, cfg_id=4)

    def run(k):
        tau = T / k
        E = op.ho_exponential(n, a, b, tau)
        return sc.gpe_strang(psi0, [E, E, E], tau, beta, k)

    ref = run(256)
    e1 = np.linalg.norm((run(8) - ref).ravel())
    e2 = np.linalg.norm((run(16) - ref).ravel())
    e3 = np.linalg.norm((run(32) - ref).ravel())
    assert 3.5 < e1 / e2 < 4.5 and 3.5 < e2 / e3 < 4.5


# ------------------------------------------------ harmonic oscillator ------

def _ho_mats(m):
    return op.hermite_forward(m), op.hermite_backward(m), op.hermite_nodes(m)


def test_ho_eigenstate_gets_exact_phase():
    m, tau = 16, 0.37
    Phi, Psi, X = _ho_mats(m)
    f = op.hermite_functions(m, X)
    k = (2, 0, 5)
    psi = f[k[0]][:, None, None] * f[k[1]][None, :, None] * f[k[2]][None, None, :]
    out = sc.ho_strang(psi, [Phi] * 3, [Psi] * 3, [X] * 3, 0.0, tau, 0.0, nsteps=3)
    lam = sum(k) + 1.5
    assert _rel(out, np.exp(-1j * 3 * tau * lam) * psi) < 1e-12


def test_ho_unitary_in_discrete_inner_product():
    m = 16
    Phi, Psi, X = _ho_mats(m)
    w = op.hermite_weights(m, X)
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    c = synth.hermite_coefficients(m, 6, 3, cfg_id=3)
    psi = om.tucker(c, [Psi] * 3)
    out = sc.ho_strang(psi, [Phi] * 3, [Psi] * 3, [X] * 3, 0.3, 0.02, 0.1, nsteps=4)
    n0 = np.sum(np.abs(psi) ** 2 * W)
    n1 = np.sum(np.abs(out) ** 2 * W)
    assert abs(n1 / n0 - 1.0) < 1e-12
    # the weighted nodal norm equals the coefficient norm (discrete Parseval)
    assert abs(n0 / np.sum(np.abs(c) ** 2) - 1.0) < 1e-12


def test_ho_strang_second_order():
    m, T, eps = 12, 1.0, 0.1
    Phi, Psi, X = _ho_mats(m)
    c = synth.hermite_coefficients(m, 5, 3, cfg_id=3)
    psi0 = om.tucker(c, [Psi] * 3)

    def run(k):
        return sc.ho_strang(psi0, [Phi] * 3, [Psi] * 3, [X] * 3, 0.0, T / k, eps, nsteps=k)

    ref = run(512)
    e1 = np.linalg.norm((run(8) - ref).ravel())
    e2 = np.linalg.norm((run(16) - ref).ravel())
    assert 3.5 < e1 / e2 < 4.5


def test_ho_potential_flow_composes():
    g = synth.rng(202, 0)
    X = [np.linspace(-3, 3, 4), np.linspace(-2, 2, 5), np.linspace(-1, 1, 3)]
    psi = synth.random_tensor((4, 5, 3), True, g)
    one = sc.ho_potential_flow(psi, X, 0.1, 0.9, 0.1)
    two = sc.ho_potential_flow(sc.ho_potential_flow(psi, X, 0.1, 0.4, 0.1), X, 0.4, 0.9, 0.1)
    assert _rel(two, one) < 1e-14
    # solves i psi_t = (eps/2) sin(t) |x|^2 psi at t = b (difference in b)
    db = 1e-6
    d = (sc.ho_potential_flow(psi, X, 0.1, 0.9 + db, 0.1) - sc.ho_potential_flow(psi, X, 0.1, 0.9 - db, 0.1)) / (2 * db)
    r2 = X[0][:, None, None] ** 2 + X[1][None, :, None] ** 2 + X[2][None, None, :] ** 2
    assert _rel(1j * d, 0.05 * np.sin(0.9) * r2 * one) < 1e-6


# ----------------------------------------------------------- monitors ------

def test_energy_of_fd_eigenvectors():
    n, a, b = 20, -5.0, 5.0
    h = (b - a) / (n + 1)
    H = op.ho_hamiltonian(n, a, b)
    lam, V = np.linalg.eigh(H)
    vs = [V[:, k] / np.sqrt(h) for k in (0, 1, 3)]        # h sum v^2 = 1
    psi = vs[0][:, None, None] * vs[1][None, :, None] * vs[2][None, None, :]
    assert abs(sc.norm2(psi, h ** 3) - 1.0) < 1e-13
    e0 = sc.energy_gpe(psi, [H, H, H], 0.0, h ** 3)
    assert abs(e0 - (lam[0] + lam[1] + lam[3])) < 1e-11
    beta = 7.0
    e1 = sc.energy_gpe(psi, [H, H, H], beta, h ** 3)
    quartic = np.prod([np.sum(v ** 4) for v in vs]) * h ** 3
    assert abs(e1 - e0 - 0.5 * beta * quartic) < 1e-11


# ------------------------------------------- exponential midpoint rule ----

def test_magnus_without_time_dependence_is_exact_ho():
    m, tau = 10, 0.3
    Phi, Psi, X = _ho_mats(m)
    B = [op.hermite_ho_generator(m)] * 3
    g = synth.rng(211, 0)
    psi = synth.random_tensor((m, m, m), True, g)
    got = sc.magnus_midpoint(psi, B, [None] * 3, lambda mu, t: 0.0, tau, 2)
    ref = sc.ho_linear(sc.ho_linear(psi, [Phi] * 3, [Psi] * 3, tau), [Phi] * 3, [Psi] * 3, tau)
    assert _rel(got, ref) < 1e-12


def test_magnus_constant_generator_exact_in_time():
    m, tau = 8, 0.4
    B, d, _ = op.hkmp_problem(m)
    g = synth.rng(212, 0)
    psi = synth.random_tensor((m, m, m), True, g)
    const = lambda mu, t: (-0.3j if mu == 2 else 0.0)
    one = sc.magnus_midpoint(psi, B, d, const, tau, 1)
    five = sc.magnus_midpoint(psi, B, d, const, tau / 5, 5)
    assert _rel(five, one) < 1e-12


def test_magnus_second_order_against_ode_solution():
    # 1-D mode-3 problem u' = (B + g(t) diag(x)) u, solved to high accuracy
    # by an adaptive Runge-Kutta method, against the exponential midpoint rule
    from scipy.integrate import solve_ivp
    m, T = 10, 1.0
    B, d, gf = op.hkmp_problem(m)
    A0, X = B[2], d[2]
    g = synth.rng(213, 0)
    u0 = g.standard_normal(m) + 1j * g.standard_normal(m)
    sol = solve_ivp(lambda t, u: (A0 + gf(2, t) * np.diag(X)) @ u, (0.0, T), u0, method="DOP853",
                    rtol=1e-13, atol=1e-13)
    exact = sol.y[:, -1]

    def run(k):
        u = u0.reshape(m, 1, 1)
        out = sc.magnus_midpoint(u, [A0, None, None], [X, None, None],
                                 lambda mu, t: gf(2, t) if mu == 0 else 0.0, T / k, k)
        return out.reshape(m)

    e1 = np.linalg.norm(run(16) - exact)
    e2 = np.linalg.norm(run(32) - exact)
    assert e2 < 1e-3 * np.linalg.norm(exact)
    assert 3.5 < e1 / e2 < 4.5


def test_magnus_product_state_is_product_of_mode_steps():
    m, tau = 7, 0.2
    B, d, gf = op.hkmp_problem(m)
    g = synth.rng(214, 0)
    v = [g.standard_normal(m) + 1j * g.standard_normal(m) for _ in range(3)]
    psi = np.einsum("i,j,k->ijk", *v)
    got = sc.magnus_midpoint(psi, B, d, gf, tau, 3, t0=0.1)
    w = []
    for mu in range(3):
        u = v[mu].reshape(m, 1, 1)
        Bs = [B[mu], None, None]
        ds = [d[mu], None, None]
        w.append(sc.magnus_midpoint(u, Bs, ds, lambda nu, t, mu=mu: gf(mu, t) if nu == 0 else 0.0,
                                    tau, 3, t0=0.1).reshape(m))
    assert _rel(got, np.einsum("i,j,k->ijk", *w)) < 1e-12


# ------------------------------------------ vortex problem (Section 4.5) ----

def _vortex_setup(dims=(14, 12, 10), alpha=1.5):
    xs = [synth.graded_nodes(n, -20.0, 20.0, alpha) for n in dims]
    Ms, ws = zip(*[op.nonuniform_neumann_d2(x) for x in xs])
    winv = 1.0 / (ws[0][:, None, None] * ws[1][None, :, None] * ws[2][None, None, :])
    return xs, Ms, ws, winv


def test_vortex_nonlinear_flow_solves_its_ode():
    xs, _, ws, winv = _vortex_setup()
    W = 1.0 / winv
    v = np.sqrt(W) * synth.vortex_pair_initial(xs)
    s, dt = 0.3, 1e-4
    vs = sc.vortex_nonlinear(v, s, winv)
    assert np.allclose(np.abs(vs), np.abs(v), rtol=1e-14, atol=0)
    deriv = (sc.vortex_nonlinear(v, s + dt, winv) - sc.vortex_nonlinear(v, s - dt, winv)) / (2 * dt)
    rhs = 0.5j * (1.0 - winv * np.abs(vs) ** 2) * vs
    assert np.max(np.abs(deriv - rhs)) < 1e-7 * np.max(np.abs(rhs))


def test_vortex_background_is_a_steady_state():
    # u = 1 everywhere: the Neumann Laplacian annihilates constants and the
    # nonlinearity (1 - |u|^2) vanishes, so the whole step leaves it unchanged
    xs, Ms, ws, winv = _vortex_setup()
    E = [op.exp_symmetric(M, 0.5j * 0.1) for M in Ms]
    v = np.sqrt(ws[0][:, None, None] * ws[1][None, :, None] * ws[2][None, None, :]).astype(np.complex128)
    out = sc.vortex_strang(v, E, winv, 0.1, 5)
    assert np.max(np.abs(out - v)) < 1e-12 * np.max(np.abs(v))


def test_vortex_step_keeps_weighted_mass_and_is_second_order():
    xs, Ms, ws, winv = _vortex_setup()
    v0 = np.sqrt(1.0 / winv) * synth.vortex_pair_initial(xs)
    T = 0.4

    def run(k):
        tau = T / k
        E = [op.exp_symmetric(M, 0.5j * tau) for M in Ms]
        return sc.vortex_strang(v0, E, winv, tau, k)

    r1, r2, r4 = run(4), run(8), run(16)
    assert abs(np.sum(np.abs(r4) ** 2) / np.sum(np.abs(v0) ** 2) - 1.0) < 1e-12
    e1 = np.linalg.norm(r1 - r2)
    e2 = np.linalg.norm(r2 - r4)
    assert 3.5 < e1 / e2 < 4.5
