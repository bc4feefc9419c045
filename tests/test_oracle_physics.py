"""Pins of the oracle's Schroedinger generators and exponentials against the
mathematics of the equations they discretise (closed-form discrete spectra,
the continuum harmonic oscillator, the free-particle Gaussian, and the
time-dependent Hamiltonian of Section 4.4 evaluated on closed-form
functions).  None of these re-types the oracle's own formula: each expected
value comes from the PDE or from a textbook closed form."""
import numpy as np

import synth
from oracle import operators as op


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


# ----------------------------------------------- free Schroedinger --------

def test_free_schrodinger_sine_mode_gets_exact_phase():
    # i psi_t = -1/2 psi_xx; the k-th discrete sine mode is an eigenvector of
    # the Dirichlet second difference with eigenvalue
    # lambda_k = -(4/h^2) sin^2(k pi / (2(n+1))), so one step multiplies it
    # by exp(i tau lambda_k / 2) exactly
    n, a, b, tau = 64, -10.0, 10.0, 0.01
    h = (b - a) / (n + 1)
    E = op.free_schrodinger_exponential(n, a, b, tau)
    j = np.arange(1, n + 1)
    for k in (1, 2, 9, 40, n):
        v = np.sqrt(2.0 / (n + 1)) * np.sin(j * k * np.pi / (n + 1))
        lam = -(4.0 / h ** 2) * np.sin(k * np.pi / (2 * (n + 1))) ** 2
        assert np.max(np.abs(E @ v - np.exp(0.5j * tau * lam) * v)) < 1e-13


def test_free_schrodinger_gaussian_spreads_as_closed_form():
    # exp(-x^2/2) under i psi_t = -1/2 psi_xx becomes
    # (1 + i t)^(-1/2) exp(-x^2 / (2 (1 + i t))); on a fine grid the discrete
    # flow matches to O(h^2) (the domain edge is ~e^-40 away)
    a, b, t = -12.0, 12.0, 0.5
    errs = []
    for n in (255, 511):
        x = synth.dirichlet_nodes(n, a, b)
        E = op.free_schrodinger_exponential(n, a, b, t)
        exact = (1.0 + 1j * t) ** -0.5 * np.exp(-x ** 2 / (2.0 * (1.0 + 1j * t)))
        errs.append(_rel(E @ np.exp(-0.5 * x ** 2), exact))
    assert errs[1] < 2e-4
    assert 3.5 < errs[0] / errs[1] < 4.5


# ----------------------------------------------- harmonic oscillator ------

def test_ho_hamiltonian_spectrum_converges_to_k_plus_half():
    # the continuum oscillator -1/2 d^2/dx^2 + x^2/2 has eigenvalues k + 1/2;
    # the second-order discretisation converges to them at order two
    a, b = -8.0, 8.0
    ks = np.arange(5)
    errs = []
    for n in (96, 192):
        lam = np.linalg.eigvalsh(op.ho_hamiltonian(n, a, b))[:5]
        errs.append(np.abs(lam - (ks + 0.5)))
    assert np.all(errs[1] < 1e-2)
    ratio = errs[0] / errs[1]
    assert np.all((3.6 < ratio) & (ratio < 4.4))


def test_ho_exponential_eigenvector_gets_exact_phase():
    # i psi_t = H psi: an eigenvector v of H with eigenvalue lambda evolves
    # as exp(-i tau lambda) v
    n, a, b, tau = 80, -8.0, 8.0, 0.07
    H = op.ho_hamiltonian(n, a, b)
    lam, V = np.linalg.eigh(H)
    E = op.ho_exponential(n, a, b, tau)
    for k in (0, 1, 5, 30):
        v = V[:, k]
        assert np.max(np.abs(E @ v - np.exp(-1j * tau * lam[k]) * v)) < 1e-13


def _hermite_function(k, x):
    # phi_k(x) = (2^k k! sqrt(pi))^(-1/2) H_k(x) exp(-x^2/2) with the physicists'
    # Hermite polynomial from numpy (independent of the oracle's recurrence)
    from math import factorial
    c = np.zeros(k + 1)
    c[k] = 1.0
    Hk = np.polynomial.hermite.hermval(x, c)
    return Hk * np.exp(-0.5 * x ** 2) / np.sqrt(2.0 ** k * factorial(k) * np.sqrt(np.pi))


def test_ho_exponential_matches_continuum_oscillator():
    # a combination of the first Hermite functions sampled on the grid: the
    # exact oscillator flow multiplies phi_k by exp(-i tau (k + 1/2)); the
    # finite-difference propagator reproduces it to O(h^2)
    a, b, tau = -8.0, 8.0, 0.3
    g = synth.rng(301, 0)
    c = g.standard_normal(6) + 1j * g.standard_normal(6)
    errs = []
    for n in (128, 256):
        x = synth.dirichlet_nodes(n, a, b)
        psi0 = sum(c[k] * _hermite_function(k, x) for k in range(6))
        exact = sum(c[k] * np.exp(-1j * tau * (k + 0.5)) * _hermite_function(k, x) for k in range(6))
        errs.append(_rel(op.ho_exponential(n, a, b, tau) @ psi0, exact))
    assert errs[1] < 5e-3
    assert 3.5 < errs[0] / errs[1] < 4.5


# ------------------------------------ time-dependent problem (Sec. 4.4) ---

def test_hkmp_generators_are_the_papers_hamiltonian():
    # psi_t = (i/2)(Laplace - |x|^2 - 2 x_3 sin^2 t) psi.  In nodal Hermite
    # space mode mu's generator A_mu(t) = B_mu + g(mu, t) diag(d_mu) must act
    # on a function in the span of the first m Hermite functions as
    # (i/2)(f'' - x^2 f) (modes 1, 2) and (i/2)(f'' - x^2 f - 2 x sin^2(t) f)
    # (mode 3) at the nodes.  f = p(x) exp(-x^2/2), p = 1 + x + x^2:
    # f'' = (p'' - 2 x p' + (x^2 - 1) p) exp(-x^2/2).
    m = 24
    B, d, gfun = op.hkmp_problem(m)
    X = op.hermite_nodes(m)
    p = 1.0 + X + X ** 2
    dp = 1.0 + 2.0 * X
    ddp = 2.0 * np.ones_like(X)
    gauss = np.exp(-0.5 * X ** 2)
    f = p * gauss
    fxx = (ddp - 2.0 * X * dp + (X ** 2 - 1.0) * p) * gauss
    for t in (0.3, 1.1, 2.0):
        for mu in range(3):
            A = B[mu] + (gfun(mu, t) * np.diag(d[mu]) if d[mu] is not None else 0.0)
            want = 0.5j * (fxx - X ** 2 * f)
            if mu == 2:
                want = want + 0.5j * (-2.0 * X * np.sin(t) ** 2 * f)
            assert np.max(np.abs(A @ f - want)) < 1e-11 * np.max(np.abs(want)), (t, mu)


# ------------------------------------- non-uniform Neumann (Section 4.5) ---

def test_nonuniform_neumann_uniform_grid_is_symmetrised_ghost_point_matrix():
    # on a uniform grid the textbook ghost-point Neumann matrix is
    # h^-2 [-2 2; 1 -2 1; ...; 2 -2]; with T = diag(1/2, 1, ..., 1, 1/2) the
    # similarity T^(1/2) D T^(-1/2) is symmetric and must be M_W
    n, a, b = 17, -3.0, 5.0
    x = np.linspace(a, b, n)
    h = x[1] - x[0]
    D = (np.diag(-2.0 * np.ones(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)) / h ** 2
    D[0, 1] = D[n - 1, n - 2] = 2.0 / h ** 2
    t = np.ones(n)
    t[0] = t[-1] = 0.5
    M, w = op.nonuniform_neumann_d2(x)
    assert np.allclose(w, h * t, rtol=1e-14, atol=0)
    ref = np.sqrt(t)[:, None] * D / np.sqrt(t)[None, :]
    assert np.max(np.abs(M - ref)) < 1e-12 * np.max(np.abs(ref))


def test_nonuniform_neumann_uniform_spectrum_closed_form():
    # Neumann cosine modes cos(k pi j/(n-1)): lambda_k = -(4/h^2) sin^2(k pi/(2(n-1)))
    n = 40
    x = np.linspace(0.0, 2.0, n)
    h = x[1] - x[0]
    lam = np.sort(np.linalg.eigvalsh(op.nonuniform_neumann_d2(x)[0]))
    k = np.arange(n)
    ref = np.sort(-(4.0 / h ** 2) * np.sin(k * np.pi / (2 * (n - 1))) ** 2)
    assert np.max(np.abs(lam - ref)) < 1e-10 * np.max(np.abs(ref))


def test_nonuniform_neumann_constants_in_kernel():
    # homogeneous Neumann: constants are harmonic, so W^(1/2) 1 is a null
    # vector of M_W on any grid (a wrong end weight or flux breaks this)
    g = np.random.default_rng(7)
    x = np.sort(g.uniform(-20.0, 20.0, 37))
    M, w = op.nonuniform_neumann_d2(x)
    v = np.sqrt(w)
    assert np.linalg.norm(M @ v) < 1e-12 * np.linalg.norm(M) * np.linalg.norm(v)
    assert np.max(np.abs(M - M.T)) < 1e-15 * np.max(np.abs(M))


def test_nonuniform_neumann_second_order_on_graded_grid():
    # u = cos(pi (x - a)/(b - a)) has u' = 0 and u''' = 0 at both ends; the
    # unsymmetrised operator W^(-1/2) M W^(1/2) approximates u'' at second
    # order on a smoothly graded grid, boundary rows included
    a, b = -20.0, 20.0
    errs = []
    for n in (81, 161, 321):
        x = synth.graded_nodes(n, a, b, 2.0)
        M, w = op.nonuniform_neumann_d2(x)
        u = np.cos(np.pi * (x - a) / (b - a))
        D = (M * np.sqrt(w)[None, :]) / np.sqrt(w)[:, None]
        exact = -(np.pi / (b - a)) ** 2 * u
        errs.append(np.max(np.abs(D @ u - exact)) / np.max(np.abs(exact)))
    assert errs[-1] < 1e-3
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.6 < e0 / e1 < 4.4


def test_nonuniform_neumann_flow_keeps_weighted_mass():
    # i psi_t = -1/2 D psi in the variable v = W^(1/2) psi: exp(i tau/2 M_W)
    # is unitary, so sum_j w_j |psi_j|^2 is conserved
    g = np.random.default_rng(8)
    x = synth.graded_nodes(50, -20.0, 20.0, 1.5)
    M, w = op.nonuniform_neumann_d2(x)
    E = op.exp_symmetric(M, 0.5j * 0.1)
    psi = g.standard_normal(50) + 1j * g.standard_normal(50)
    v = np.sqrt(w) * psi
    psi1 = (E @ v) / np.sqrt(w)
    assert abs(np.sum(w * np.abs(psi1) ** 2) / np.sum(w * np.abs(psi) ** 2) - 1.0) < 1e-13
