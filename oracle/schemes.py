"""Splitting steps and monitors built on the mu-mode integrator (oracle).

Pins (tests/test_oracle_schemes.py):
  gpe_strang     -- beta = 0 reduces to the plain integrator with E(tau);
                    the nonlinear subflow against its closed form (|psi|
                    constant, phase -s beta |psi|^2); mass conservation
                    (Section 2, advantages list); second order in tau (error
                    ratio ~4 when tau halves, self-convergence).
  ho_strang      -- eps = 0: a product of Hermite functions sampled at the
                    nodes acquires exactly exp(-i tau lambda_i) per step,
                    lambda_i = sum (1/2 + i_mu) (Section 3); unitarity;
                    second order in tau for eps != 0.
  merged loops   -- gpe_strang_merged equals gpe_strang (phase flows of the
                    nonlinear part compose: N(a) N(b) = N(a + b) because N
                    keeps |psi|).
  monitors       -- mass of a normalised state is 1; energy of a 1-D HO
                    eigenvector of the FD Hamiltonian equals its eigenvalue.
  vortex_strang  -- the nonlinear subflow of the Section 4.5 vortex problem
                    against its ODE (central differences in time) and |v|
                    constant; the background u = 1 (v = W^(1/2) 1) is an
                    exact steady state of the whole step; the W-weighted mass
                    is conserved; second order in tau.
  magnus_midpoint -- g = 0 equals the exact harmonic-oscillator propagation
                    in Hermite space; a constant g is exact in time (one step
                    of tau equals k steps of tau/k); second order against a
                    high-accuracy ODE solution of the 1-D time-dependent mode
                    problem; a product state evolves as the product of the
                    1-D steps (Kronecker structure).
"""
from __future__ import annotations

import numpy as np

from .mumode import mode_product, tucker


# ------------------------------------------------- Gross-Pitaevskii --------

def gpe_nonlinear(psi: np.ndarray, s: float, beta: float) -> np.ndarray:
    """Exact flow over time s of i psi_t = beta |psi|^2 psi:
    psi <- exp(-i s beta |psi|^2) psi (|psi| is constant along it)."""
    return np.exp(-1j * s * beta * np.abs(psi) ** 2) * psi


def gpe_strang(psi: np.ndarray, E, tau: float, beta: float, nsteps: int = 1) -> np.ndarray:
    """Strang splitting N(tau/2) L(tau) N(tau/2) per step, where L(tau) is the
    mu-mode integrator with E_mu = exp(-i tau H_mu) and N the exact nonlinear
    flow (Section 4.5: linear part by the integrator, nonlinear part exact)."""
    for _ in range(nsteps):
        psi = gpe_nonlinear(psi, 0.5 * tau, beta)
        psi = tucker(psi, E)
        psi = gpe_nonlinear(psi, 0.5 * tau, beta)
    return psi


def gpe_strang_merged(psi: np.ndarray, E, tau: float, beta: float, nsteps: int = 1) -> np.ndarray:
    """Same scheme with adjacent half-steps of N merged:
    N(tau/2) [L N(tau)]^(nsteps-1) L N(tau/2)."""
    psi = gpe_nonlinear(psi, 0.5 * tau, beta)
    for k in range(nsteps):
        psi = tucker(psi, E)
        psi = gpe_nonlinear(psi, tau if k < nsteps - 1 else 0.5 * tau, beta)
    return psi


# --------------------------------------- harmonic oscillator (Hermite) -----

def vortex_nonlinear(v: np.ndarray, s: float, winv: np.ndarray) -> np.ndarray:
    """Exact flow over time s of the nonlinear part of the Section 4.5
    vortex problem in the symmetrised variable v = W^(1/2) u,
    v_t = (i/2)(1 - W^-1 |v|^2) v: |v| is constant along it, so
    v <- exp((i s / 2)(1 - W^-1 |v|^2)) v.  winv: the tensor of W^-1 (the
    product over the modes of the inverse dual-cell widths)."""
    return np.exp(0.5j * s * (1.0 - winv * np.abs(v) ** 2)) * v


def vortex_strang(v: np.ndarray, E, winv: np.ndarray, tau: float, nsteps: int = 1) -> np.ndarray:
    """Strang splitting of v_t = (i/2) M_W v + (i/2)(1 - W^-1 |v|^2) v
    (Section 4.5): N(tau/2) L(tau) N(tau/2) per step, L the mu-mode integrator
    with E_mu = exp(i tau/2 M_mu) (M_W is the Kronecker sum of the modes'
    M_mu), N the exact nonlinear flow."""
    for _ in range(nsteps):
        v = vortex_nonlinear(v, 0.5 * tau, winv)
        v = tucker(v, E)
        v = vortex_nonlinear(v, 0.5 * tau, winv)
    return v


def ho_potential_flow(psi: np.ndarray, nodes, a: float, b: float, eps: float) -> np.ndarray:
    """Exact flow from time a to b of i psi_t = (eps/2) sin(t) |x|^2 psi:
    psi <- exp(-i (eps/2) |x|^2 (cos a - cos b)) psi (pointwise)."""
    d = psi.ndim
    r2 = np.zeros((1,) * d)
    for mu in range(d):
        shape = [1] * d
        shape[mu] = len(nodes[mu])
        r2 = r2 + (np.asarray(nodes[mu]) ** 2).reshape(shape)
    return np.exp(-1j * 0.5 * eps * r2 * (np.cos(a) - np.cos(b))) * psi


def ho_linear(psi: np.ndarray, Phi, Psi, tau: float) -> np.ndarray:
    """Exact flow of i psi_t = -1/2 sum (d^2 - x^2) psi in Hermite space:
    forward transform (equation real2spec), multiply coefficient i by
    exp(-i tau lambda_i) with lambda_i = sum_mu (1/2 + i_mu) (Section 3),
    backward transform (equation spec2real)."""
    d = psi.ndim
    c = tucker(psi, Phi)
    lam = np.zeros((1,) * d)
    for mu in range(d):
        shape = [1] * d
        shape[mu] = c.shape[mu]
        lam = lam + (0.5 + np.arange(c.shape[mu], dtype=np.float64)).reshape(shape)
    c = np.exp(-1j * tau * lam) * c
    return tucker(c, Psi)


def ho_strang(psi: np.ndarray, Phi, Psi, nodes, t0: float, tau: float, eps: float,
              nsteps: int = 1) -> np.ndarray:
    """Strang step for V(x,t) = |x|^2/2 (1 + eps sin t): the harmonic part is
    exact in Hermite space, the time-dependent remainder is integrated
    exactly over each half step:
    P(t+tau/2, t+tau) L_H(tau) P(t, t+tau/2)."""
    t = t0
    for _ in range(nsteps):
        psi = ho_potential_flow(psi, nodes, t, t + 0.5 * tau, eps)
        psi = ho_linear(psi, Phi, Psi, tau)
        psi = ho_potential_flow(psi, nodes, t + 0.5 * tau, t + tau, eps)
        t = t + tau
    return psi


# ------------------------------------------- exponential midpoint rule ----

def magnus_generators(B, d, coef):
    """Mode generators A_mu = B_mu + coef_mu diag(d_mu) (B_mu None: mode
    left unchanged; d_mu None: no time-dependent part)."""
    out = []
    for mu, Bm in enumerate(B):
        if Bm is None:
            out.append(None)
            continue
        A = np.array(Bm, dtype=np.complex128)
        if d[mu] is not None:
            A = A + coef[mu] * np.diag(np.asarray(d[mu], dtype=np.float64))
        out.append(A)
    return out


def magnus_midpoint(psi: np.ndarray, B, d, g, tau: float, nsteps: int = 1, t0: float = 0.0) -> np.ndarray:
    """Exponential midpoint rule (second-order Magnus integrator, equation
    mag2 of Section 4.4) for u' = A(t) u with A(t) in Kronecker-sum form,
    A(t) = sum_mu I x A_mu(t) x I, A_mu(t) = B_mu + g(mu, t) diag(d_mu):
    u_{n+1} = exp(tau A(t_n + tau/2)) u_n.  The exponential of a Kronecker
    sum is the Kronecker product of the mode exponentials (Section 2), so a
    step is the mu-mode integrator with E_mu = exp(tau A_mu(t_n + tau/2)).
    g: callable (mu, t) -> complex coefficient."""
    from scipy.linalg import expm
    for n in range(nsteps):
        tm = t0 + (n + 0.5) * tau
        A = magnus_generators(B, d, [g(mu, tm) for mu in range(len(B))])
        E = [expm(tau * a) if a is not None else None for a in A]
        psi = tucker(psi, E)
    return psi


# ----------------------------------------------------------- monitors ------

def norm2(psi: np.ndarray, cell: float) -> float:
    """Discrete mass h^d sum |psi|^2 (conserved by unitary steps)."""
    return float(cell * np.sum(np.abs(psi) ** 2))


def energy_gpe(psi: np.ndarray, H, beta: float, cell: float) -> float:
    """Discrete GPE energy h^d [Re sum conj(psi) (sum_mu psi x_mu H_mu)
    + (beta/2) sum |psi|^4]."""
    Hpsi = np.zeros_like(psi)
    for mu, Hm in enumerate(H, start=1):
        Hpsi = Hpsi + mode_product(psi, Hm, mu)
    kin = np.real(np.vdot(psi.reshape(-1), Hpsi.reshape(-1)))
    return float(cell * (kin + 0.5 * beta * np.sum(np.abs(psi) ** 4)))
