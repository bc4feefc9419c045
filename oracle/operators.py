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
  central_d2_weights /  -- the textbook orders 2 and 4; convergence at the
  fd2_periodic_order       stencil's order on a smooth periodic function
                           (error ratio 2^p when n doubles); order 2 = fd2.
  fourier_d2            -- exact (to rounding) on every trigonometric mode
                           the grid carries, symmetric.
  pipe_flow_operators   -- second-order consistency, boundary rows included,
                           on functions that satisfy the boundary conditions
                           (Neumann / Dirichlet-Neumann), against the
                           analytic operator including the 1/r and s(z) terms.
  nonuniform_neumann_d2 -- on a uniform grid, the similarity transform of the
                           textbook ghost-point Neumann matrix and its closed-
                           form cosine spectrum; constants in the kernel
                           (W^(1/2) 1 is a null vector); second-order
                           consistency of W^(-1/2) M W^(1/2) on a smoothly
                           graded grid; the W-weighted mass is conserved by
                           the exponential of i M.
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
    4.4 in nodal Hermite space: psi_t = (i/2)(Laplace - |x|^2 - 2 x_3 sin^2 t) psi,
    i.e. A_mu = hermite_ho_generator for every mode plus, on mode 3,
    -i sin^2(t) diag(x_3).  Returns (B, d, g) for schemes.magnus_midpoint."""
    X = hermite_nodes(m)
    Bm = hermite_ho_generator(m)
    B = [Bm, Bm, Bm]
    d = [None, None, X]
    return B, d, (lambda mu, t: -1j * np.sin(t) ** 2 if mu == 2 else 0.0)


# ------------------------------------------------ operator front-ends ----

def central_d2_weights(order: int) -> np.ndarray:
    """Weights w_0..w_m (m = order/2) of the centred second difference of the
    given even order, from the Taylor conditions: sum_k w_|k| k^(2q) = 2 [q == 1]
    for q = 0..m (symmetric stencil, h = 1)."""
    m = order // 2
    ks = np.arange(0, m + 1)
    # unknowns w_0..w_m; row q: w_0 [q==0] + 2 sum_{k>=1} w_k k^(2q)
    M = np.zeros((m + 1, m + 1))
    rhs = np.zeros(m + 1)
    for q in range(m + 1):
        M[q, 0] = 1.0 if q == 0 else 0.0
        M[q, 1:] = 2.0 * ks[1:].astype(float) ** (2 * q)
    rhs[1] = 2.0
    return np.linalg.solve(M, rhs)


def fd2_periodic_order(n: int, a: float, b: float, order: int) -> np.ndarray:
    """Centred second difference of even `order` on n periodic nodes of
    [a, b) (h = (b - a)/n): a symmetric circulant (Section 4.1, Test 2)."""
    h = (b - a) / n
    w = central_d2_weights(order)
    D = np.zeros((n, n))
    for i in range(n):
        D[i, i] += w[0]
        for k in range(1, len(w)):
            D[i, (i + k) % n] += w[k]
            D[i, (i - k) % n] += w[k]
    return D / h ** 2


def fourier_d2(n: int, a: float, b: float) -> np.ndarray:
    """Fourier spectral second derivative on n periodic nodes of [a, b): the
    matrix of u -> ifft(-(2 pi k / L)^2 fft(u)), k the FFT wavenumbers (the
    Nyquist mode of even n multiplied by -(pi n / L)^2), applied to the unit
    vectors."""
    L = b - a
    k = np.fft.fftfreq(n, d=1.0 / n)
    if n % 2 == 0:
        k[n // 2] = n // 2
    sym = -(2.0 * np.pi * k / L) ** 2
    return np.real(np.fft.ifft(sym[:, None] * np.fft.fft(np.eye(n), axis=0), axis=0))


def pipe_flow_operators(n_rho: int, n_z: int, rho_min: float, rho_max: float, z_max: float, alpha: float):
    """1-D operators of the pipe-flow problem of Section 4.2,
    c_t = alpha (c_rr + c_r / r + c_zz) - s(z) c_z, s(z) = 2 + tanh(4(z - 5/2))
    - tanh(4(z - 5)), by second-order centred differences:
      r: n_rho nodes r_i = r_min + i h, i = 0..n-1, h = (r_max - r_min)/(n - 1),
         homogeneous Neumann at both ends by mirrored ghost values;
      z: n_z nodes z_j = j h, j = 1..n, h = z_max / n, c = 0 at z = 0
         (Dirichlet, eliminated), homogeneous Neumann at z_max by a mirrored
         ghost value.
    Returns (A_r, A_z, r, z)."""
    def d1_d2(n, h, left, right):
        D1 = np.zeros((n, n))
        D2 = np.zeros((n, n))
        for i in range(n):
            for j, c1, c2 in ((i - 1, -0.5 / h, 1.0 / h ** 2), (i, 0.0, -2.0 / h ** 2), (i + 1, 0.5 / h, 1.0 / h ** 2)):
                if j < 0:
                    if left == "dirichlet":
                        continue
                    j = 1            # mirrored ghost value c_{-1} = c_1
                if j >= n:
                    if right == "dirichlet":
                        continue
                    j = n - 2        # mirrored ghost value c_n = c_{n-2}
                D1[i, j] += c1
                D2[i, j] += c2
        return D1, D2

    hr = (rho_max - rho_min) / (n_rho - 1)
    r = rho_min + hr * np.arange(n_rho)
    D1r, D2r = d1_d2(n_rho, hr, "neumann", "neumann")
    A_r = alpha * (D2r + np.diag(1.0 / r) @ D1r)
    hz = z_max / n_z
    z = hz * np.arange(1, n_z + 1)
    D1z, D2z = d1_d2(n_z, hz, "dirichlet", "neumann")
    s = 2.0 + np.tanh(4.0 * (z - 2.5)) - np.tanh(4.0 * (z - 5.0))
    A_z = alpha * D2z - np.diag(s) @ D1z
    return A_r, A_z, r, z


def nonuniform_neumann_d2(x: np.ndarray):
    """Second derivative on the non-uniform nodes x_0 < ... < x_{n-1} of
    [x_0, x_{n-1}] with homogeneous Neumann conditions at both ends, in the
    symmetrised form of Section 4.5 (reading: the conservative three-point
    scheme with dual cells, then the variable change that makes it
    symmetric).

    Cells h_j = x_{j+1} - x_j; dual cells w_0 = h_0 / 2, w_j = (h_{j-1} +
    h_j) / 2, w_{n-1} = h_{n-2} / 2.  The scheme is
        (D u)_j = (1/w_j) [(u_{j+1} - u_j)/h_j - (u_j - u_{j-1})/h_{j-1}],
    with the flux through each end set to zero (homogeneous Neumann), i.e.
    D = W^-1 S with S symmetric tridiagonal and W = diag(w).  The variable
    v = W^(1/2) u turns it into the symmetric M_W = W^(-1/2) S W^(-1/2), and
    sum_j w_j |u_j|^2 = |v|^2.  Returns (M_W, w)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    h = np.diff(x)
    w = np.empty(n)
    w[0] = 0.5 * h[0]
    w[-1] = 0.5 * h[-1]
    w[1:-1] = 0.5 * (h[:-1] + h[1:])
    S = np.zeros((n, n))
    for j in range(n - 1):
        c = 1.0 / h[j]          # flux between nodes j and j + 1
        S[j, j] -= c
        S[j + 1, j + 1] -= c
        S[j, j + 1] += c
        S[j + 1, j] += c
    r = 1.0 / np.sqrt(w)
    return S * r[:, None] * r[None, :], w
