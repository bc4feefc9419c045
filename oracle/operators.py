"""1-D generators, their exponentials, Hermite quadrature (oracle; tests only).

Pins (tests/test_oracle_operators.py):
  fd2 / exp_symmetric -- closed-form Dirichlet eigenpairs
                         lambda_k = -(4/h^2) sin^2(k pi / (2(n+1))),
                         v_k(j) = sqrt(2/(n+1)) sin(j k pi/(n+1));
                         scipy.linalg.expm (scaling-and-squaring Pade, the
                         method the paper used for its small exponentials,
                         Section 4); periodic cosine eigenvector whose
                         one-step error reproduces the errors printed in
                         Section 4.1 and Section 5.1 (tests/golden).
  hermite_*           -- discrete orthonormality Phi_tilde Psi = I
                         (Section 3, m = k Gauss-Hermite case); the two weight
                         formulas agree; Hermite eigen-relation
                         (-1/2 sum (d^2 - x^2)) H_i = lambda_i H_i checked on
                         the continuum by finite differences of the functions.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- grids ----

def grid(n: int, a: float, b: float, bc: str):
    """Nodes and spacing.  Dirichlet: n interior nodes, h = (b-a)/(n+1),
    x_j = a + j h (j = 1..n).  Periodic: h = (b-a)/n, x_j = a + (j-1) h."""
    if bc == "dirichlet":
        h = (b - a) / (n + 1)
        return a + h * np.arange(1, n + 1, dtype=np.float64), h
    if bc == "periodic":
        h = (b - a) / n
        return a + h * np.arange(n, dtype=np.float64), h
    raise ValueError(bc)


# ------------------------------------------------------ FD generators ------

def fd2(n: int, a: float, b: float, bc: str) -> np.ndarray:
    """Second-order centred second difference h^-2 (1, -2, 1) (Section 4.1)."""
    _, h = grid(n, a, b, bc)
    D = np.zeros((n, n))
    for j in range(n):
        D[j, j] = -2.0
        if j > 0:
            D[j, j - 1] = 1.0
        if j < n - 1:
            D[j, j + 1] = 1.0
    if bc == "periodic":
        D[0, n - 1] += 1.0
        D[n - 1, 0] += 1.0
    return D / h ** 2


def ho_hamiltonian(n: int, a: float, b: float) -> np.ndarray:
    """1-D harmonic-oscillator Hamiltonian -1/2 D2 + 1/2 diag(x^2), Dirichlet."""
    x, _ = grid(n, a, b, "dirichlet")
    return -0.5 * fd2(n, a, b, "dirichlet") + np.diag(0.5 * x ** 2)


# ------------------------------------------------------- exponentials ------

def exp_symmetric(A: np.ndarray, c: complex) -> np.ndarray:
    """exp(c A) for a real symmetric (or complex Hermitian) A through its
    eigendecomposition A = V diag(lambda) V^H."""
    lam, V = np.linalg.eigh(A)
    return (V * np.exp(c * lam)) @ V.conj().T


def heat_exponential(n: int, a: float, b: float, bc: str, tau: float) -> np.ndarray:
    """E = exp(tau A) for the heat generator A = D2 (equation dd-tensor)."""
    return exp_symmetric(fd2(n, a, b, bc), tau)


def free_schrodinger_exponential(n: int, a: float, b: float, tau: float) -> np.ndarray:
    """E = exp(i tau/2 D2) for i psi_t = -1/2 Laplace psi (Dirichlet)."""
    return exp_symmetric(fd2(n, a, b, "dirichlet"), 0.5j * tau)


def ho_exponential(n: int, a: float, b: float, tau: float) -> np.ndarray:
    """E = exp(-i tau H) with H = -1/2 D2 + 1/2 x^2 (Dirichlet)."""
    return exp_symmetric(ho_hamiltonian(n, a, b), -1j * tau)


# ------------------------------------------------------------ Hermite ------

def hermite_nodes(m: int) -> np.ndarray:
    """Gauss-Hermite nodes: eigenvalues of the Jacobi matrix of the
    orthonormal Hermite polynomials (zero diagonal, off-diagonal sqrt(k/2))."""
    off = np.sqrt(np.arange(1, m) / 2.0)
    J = np.diag(off, 1) + np.diag(off, -1)
    return np.sort(np.linalg.eigvalsh(J))


def hermite_functions(kmax: int, x: np.ndarray) -> np.ndarray:
    """phi[k, l] = H_k(x_l) exp(-x_l^2/2), H_k orthonormal w.r.t. exp(-x^2)
    (Section 3), by the normalised three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    phi = np.zeros((kmax, x.size))
    phi[0] = np.pi ** -0.25 * np.exp(-0.5 * x ** 2)
    if kmax > 1:
        phi[1] = np.sqrt(2.0) * x * phi[0]
    for k in range(1, kmax - 1):
        phi[k + 1] = np.sqrt(2.0 / (k + 1)) * x * phi[k] - np.sqrt(k / (k + 1.0)) * phi[k - 1]
    return phi


def hermite_weights(m: int, X: np.ndarray | None = None) -> np.ndarray:
    """Quadrature weights for Hermite *functions* at the m Gauss-Hermite
    nodes: w_l = 1 / (m phi_{m-1}(X_l)^2)."""
    X = hermite_nodes(m) if X is None else X
    phi = hermite_functions(m, X)
    return 1.0 / (m * phi[m - 1] ** 2)


def hermite_weights_christoffel(m: int, X: np.ndarray | None = None) -> np.ndarray:
    """Same weights by the Christoffel sum w_l = 1 / sum_{k<m} phi_k(X_l)^2."""
    X = hermite_nodes(m) if X is None else X
    phi = hermite_functions(m, X)
    return 1.0 / np.sum(phi ** 2, axis=0)


def hermite_forward(m: int) -> np.ndarray:
    """Forward transform matrix with the quadrature weights folded in:
    Phi_tilde[k, l] = conj(phi_k(X_l)) w_l  (equation real2spec with F_W
    = f(x_l) w_l; phi_k is real)."""
    X = hermite_nodes(m)
    return hermite_functions(m, X) * hermite_weights(m, X)[None, :]


def hermite_backward(m: int) -> np.ndarray:
    """Backward (evaluation) matrix Psi[l, k] = phi_k(X_l) (equation
    spec2real, evaluation points = quadrature nodes)."""
    X = hermite_nodes(m)
    return hermite_functions(m, X).T.copy()


def hermite_ho_generator(m: int) -> np.ndarray:
    """(i/2)(d^2/dx^2 - x^2) in nodal Hermite space: Psi diag(-i (k + 1/2)) Phi
    (phi_k is an eigenfunction of d^2/dx^2 - x^2 with eigenvalue -(2k+1),
    Section 3)."""
    Phi, Psi = hermite_forward(m), hermite_backward(m)
    return Psi @ np.diag(-1j * (np.arange(m) + 0.5)) @ Phi


def hkmp_problem(m: int):
    """Mode generators of the time-dependent Schroedinger problem of Section
    4.3 in nodal Hermite space: psi_t = (i/2)(Laplace - |x|^2 - 2 x_3 sin^2 t) psi,
    i.e. A_mu = hermite_ho_generator for every mode plus, on mode 3,
    -i sin^2(t) diag(x_3).  Returns (B, d, g) for schemes.magnus_midpoint."""
    X = hermite_nodes(m)
    Bm = hermite_ho_generator(m)
    B = [Bm, Bm, Bm]
    d = [None, None, X]
    return B, d, (lambda mu, t: -1j * np.sin(t) ** 2 if mu == 2 else 0.0)
