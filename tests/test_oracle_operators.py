"""Pins of the oracle's 1-D operators, exponentials and Hermite quadrature."""
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import mumode as om
from oracle import operators as op

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def test_fd2_dirichlet_closed_form_eigenpairs():
    n, a, b = 37, -2.0, 3.0
    D = op.fd2(n, a, b, "dirichlet")
    h = (b - a) / (n + 1)
    j = np.arange(1, n + 1)
    for k in (1, 2, 17, n):
        lam = -(4.0 / h ** 2) * np.sin(k * np.pi / (2 * (n + 1))) ** 2
        v = np.sqrt(2.0 / (n + 1)) * np.sin(j * k * np.pi / (n + 1))
        assert np.max(np.abs(D @ v - lam * v)) < 1e-12 * abs(lam) + 1e-12


@pytest.mark.parametrize("c", [-1e-3, -0.37, 0.5j * 0.01, -1j * 0.1])
def test_exp_symmetric_matches_scipy_expm(c):
    A = op.ho_hamiltonian(48, -8.0, 8.0)
    E = op.exp_symmetric(A, c)
    assert _rel(E, scipy.linalg.expm(c * A)) < 1e-13


def test_heat_exponential_sine_mode_decay_exact():
    # E = exp(tau D2) maps the k-th discrete sine mode to exp(tau lambda_k) times itself
    n, tau = 64, 1e-3
    h = 1.0 / (n + 1)
    E = op.heat_exponential(n, 0.0, 1.0, "dirichlet", tau)
    j = np.arange(1, n + 1)
    for k in (1, 3, 10):
        v = np.sin(j * k * np.pi / (n + 1))
        lam = -(4.0 / h ** 2) * np.sin(k * np.pi / (2 * (n + 1))) ** 2
        assert np.max(np.abs(E @ v - np.exp(tau * lam) * v)) < 1e-13
        # continuum decay exp(-k^2 pi^2 tau) is matched to O(h^2)
        assert abs(tau * lam + (k * np.pi) ** 2 * tau) < (k * np.pi) ** 4 * h ** 2 * tau / 12 * 1.01


def test_heat_exponential_positive_and_contractive():
    E = op.heat_exponential(40, 0.0, 1.0, "dirichlet", 1e-2)
    assert np.min(E) >= -1e-15          # exp(tau D2) is entrywise non-negative
    assert np.max(np.sum(E, axis=1)) <= 1.0 + 1e-14   # maximum principle


def test_unitary_exponentials():
    E = op.free_schrodinger_exponential(64, -10.0, 10.0, 0.01)
    assert np.max(np.abs(E.conj().T @ E - np.eye(64))) < 1e-13
    G = op.ho_exponential(64, -8.0, 8.0, 0.1)
    assert np.max(np.abs(G.conj().T @ G - np.eye(64))) < 1e-13


def _golden_heat():
    rows = []
    with open(os.path.join(GOLDEN, "heat_periodic_fd2_errors.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, err, _sec, usable = line.split()
            rows.append((int(n), float(err), usable == "1"))
    return rows


def _heat_error(n):
    a, b = 0.0, 2.0 * np.pi
    x, _ = op.grid(n, a, b, "periodic")
    c = np.cos(x)
    U0 = c[:, None, None] + c[None, :, None] + c[None, None, :]
    E = op.heat_exponential(n, a, b, "periodic", 1.0)
    U = om.expstep(U0, [E, E, E], 1)
    ref = np.exp(-1.0) * U0
    return _rel(U, ref)


@pytest.mark.parametrize("n,printed,usable", [r for r in _golden_heat() if r[0] <= 100])
def test_paper_heat_errors_section_4_1(n, printed, usable):
    err = _heat_error(n)
    # printed with three significant digits: agree to half a unit in the last digit
    unit = 10.0 ** (np.floor(np.log10(printed)) - 2)
    assert abs(err - printed) <= 0.5 * unit + 1e-18


@pytest.mark.slow
@pytest.mark.parametrize("n,printed,usable", [r for r in _golden_heat() if 100 < r[0] <= 400])
def test_paper_heat_errors_section_5_1(n, printed, usable):
    err = _heat_error(n)
    unit = 10.0 ** (np.floor(np.log10(printed)) - 2)
    assert usable and abs(err - printed) <= 0.5 * unit


def test_paper_heat_error_n500_reading():
    # the printed 1.47e-05 is inconsistent with the exact one-step error of
    # the cosine eigenvector, exp((lambda+1)T) - 1 with lambda = -(2-2cos h)/h^2
    row = [r for r in _golden_heat() if r[0] == 500][0]
    assert not row[2]
    h = 2 * np.pi / 500
    lam = -(2 - 2 * np.cos(h)) / h ** 2
    closed = np.expm1(lam + 1.0)
    assert abs(closed - 1.316e-5) < 1e-8 and abs(closed - row[1]) > 1e-6
    # and the oracle's 1-D periodic operator reproduces that closed form
    x, _ = op.grid(500, 0.0, 2 * np.pi, "periodic")
    E = op.heat_exponential(500, 0.0, 2 * np.pi, "periodic", 1.0)
    v = np.cos(x)
    # eigh backward error ~ eps * ||D2|| = 2.2e-16 * 4/h^2 ~ 6e-12 sets the tolerance
    assert abs(np.linalg.norm(E @ v) / np.linalg.norm(v) - np.exp(lam)) < 2e-11


# ------------------------------------------------------------- Hermite -----

@pytest.mark.parametrize("m", [8, 32, 128])
def test_hermite_nodes_and_weights_vs_numpy_hermgauss(m):
    X = op.hermite_nodes(m)
    Xr, Wr = np.polynomial.hermite.hermgauss(m)
    assert np.max(np.abs(X - Xr)) < 1e-11 * max(1.0, np.max(np.abs(Xr)))
    w = op.hermite_weights(m, X)
    # weights for Hermite functions = Gauss-Hermite weights times exp(x^2)
    wr = Wr * np.exp(Xr ** 2)
    assert np.max(np.abs(w - wr) / wr) < 1e-9


def test_hermite_weight_formulas_agree_and_max_node():
    m = 128
    w1 = op.hermite_weights(m)
    w2 = op.hermite_weights_christoffel(m)
    assert np.max(np.abs(w1 - w2) / w2) < 1e-11
    assert abs(np.max(op.hermite_nodes(m)) - 15.2918) < 1e-3


@pytest.mark.parametrize("m", [16, 128])
def test_hermite_discrete_orthonormality(m):
    Phi = op.hermite_forward(m)
    Psi = op.hermite_backward(m)
    assert np.max(np.abs(Phi @ Psi - np.eye(m))) < 1e-12


def test_hermite_functions_continuum_orthonormal_and_eigen():
    x = np.linspace(-14.0, 14.0, 28001)
    h = x[1] - x[0]
    phi = op.hermite_functions(12, x)
    G = (phi * h) @ phi.T
    assert np.max(np.abs(G - np.eye(12))) < 1e-9
    # (-1/2 d^2 + 1/2 x^2) phi_k = (k + 1/2) phi_k  (Section 3, d = 1)
    for k in (0, 1, 5, 11):
        f = phi[k]
        d2 = (f[2:] - 2 * f[1:-1] + f[:-2]) / h ** 2
        lhs = -0.5 * d2 + 0.5 * x[1:-1] ** 2 * f[1:-1]
        assert np.max(np.abs(lhs - (k + 0.5) * f[1:-1])) < 1e-4


def test_exp_symmetric_complex_hermitian_matches_scipy_expm():
    import synth
    g = synth.rng(301, 0)
    B = synth.random_matrix(20, 20, True, g)
    Hm = 0.5 * (B + B.conj().T)
    E = op.exp_symmetric(Hm, -0.8j)
    assert _rel(E, scipy.linalg.expm(-0.8j * Hm)) < 1e-13


# ------------------------------------------------ operator front-ends ----

def test_central_weights_known_orders():
    # order 2: (1, -2, 1); order 4: (-1/12, 4/3, -5/2, 4/3, -1/12)
    assert np.allclose(op.central_d2_weights(2), [-2.0, 1.0], atol=1e-14)
    assert np.allclose(op.central_d2_weights(4), [-2.5, 4.0 / 3, -1.0 / 12], atol=1e-13)


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_fd2_periodic_order_converges_at_its_order(order):
    errs = []
    for n in (32, 64):
        D = op.fd2_periodic_order(n, 0.0, 2 * np.pi, order)
        x = 2 * np.pi * np.arange(n) / n
        u = np.exp(np.sin(x))
        exact = (np.cos(x) ** 2 - np.sin(x)) * u
        errs.append(np.abs(D @ u - exact).max())
    assert order - 0.5 < np.log2(errs[0] / errs[1]) < order + 0.7


def test_fd2_periodic_order2_is_fd2():
    assert np.allclose(op.fd2_periodic_order(17, 0.0, 3.0, 2), op.fd2(17, 0.0, 3.0, "periodic"), atol=1e-12)


def test_fourier_d2_exact_on_trigonometric_polynomials():
    n, a, b = 24, -1.0, 3.0
    L = b - a
    D = op.fourier_d2(n, a, b)
    x = a + L * np.arange(n) / n
    for k in range(0, n // 2 + 1):
        w = 2 * np.pi * k / L
        u = np.cos(w * (x - a))
        assert np.abs(D @ u + w ** 2 * u).max() < 1e-9 * max(1.0, w ** 2)
    assert np.allclose(D, D.T, atol=1e-10)


def test_pipe_flow_operators_second_order_and_boundary_conditions():
    rmin, rmax, zmax, alpha = 0.1, 5.0, 8.0, 1.0 / 90
    er, ez = [], []
    for n in (100, 200):
        A_r, A_z, r, z = op.pipe_flow_operators(n, n, rmin, rmax, zmax, alpha)
        k = np.pi / (rmax - rmin)
        c = np.cos(k * (r - rmin))                       # Neumann at both ends
        exact = alpha * (-k ** 2 * c - k * np.sin(k * (r - rmin)) / r)
        er.append(np.abs(A_r @ c - exact).max())
        q = np.pi / (2 * zmax)
        cz = np.sin(q * z)                               # c(0) = 0, c'(z_max) = 0
        s = 2 + np.tanh(4 * (z - 2.5)) - np.tanh(4 * (z - 5))
        exact_z = -alpha * q ** 2 * cz - s * q * np.cos(q * z)
        ez.append(np.abs(A_z @ cz - exact_z).max())
    assert 3.5 < er[0] / er[1] < 4.5
    assert 3.5 < ez[0] / ez[1] < 4.5
