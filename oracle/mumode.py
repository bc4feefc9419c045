"""mu-mode product and mu-mode integrator (oracle; test infrastructure only).

Pins (tests/test_oracle_mumode.py):
  mode_product    -- pure-Python loops over Definition 2.1; Kronecker matrix
                     I (x) .. (x) L (x) .. (x) I acting on vec(U) (Section 2,
                     equation tensor-structure); rectangular, non-symmetric L.
  tucker/expstep  -- expm of the full Kronecker-sum matrix applied to vec(U)
                     (Section 2: u(t) = exp(tM) u0 with M the Kronecker sum);
                     commutation of products along different modes.
"""
from __future__ import annotations

import itertools

import numpy as np


def mode_product(U: np.ndarray, L: np.ndarray, mu: int) -> np.ndarray:
    """S = U x_mu L (Definition 2.1): S(.., i, ..) = sum_j L[i, j] U(.., j, ..).

    ``mu`` is 1-based as in the paper.  L may be rectangular (m x n_mu)."""
    d = U.ndim
    if not 1 <= mu <= d:
        raise ValueError("mu out of range")
    if L.shape[1] != U.shape[mu - 1]:
        raise ValueError("L.cols must equal n_mu")
    return np.moveaxis(np.tensordot(L, U, axes=(1, mu - 1)), 0, mu - 1)


def mode_product_loops(U: np.ndarray, L: np.ndarray, mu: int) -> np.ndarray:
    """Definition 2.1 written as explicit loops (tiny tensors only)."""
    d = U.ndim
    m = L.shape[0]
    out_shape = list(U.shape)
    out_shape[mu - 1] = m
    dt = np.result_type(U.dtype, L.dtype)
    S = np.zeros(out_shape, dtype=dt)
    for idx in itertools.product(*[range(s) for s in out_shape]):
        i = idx[mu - 1]
        acc = 0
        for j in range(U.shape[mu - 1]):
            src = list(idx)
            src[mu - 1] = j
            acc = acc + L[i, j] * U[tuple(src)]
        S[idx] = acc
    return S


def vec(U: np.ndarray) -> np.ndarray:
    """Column-major stacking, index i_1 + n_1 (i_2 - 1) + ... (Section 4.1)."""
    return U.reshape(-1, order="F")


def unvec(u: np.ndarray, dims) -> np.ndarray:
    return u.reshape(tuple(dims), order="F")


def kron_factor(dims, L: np.ndarray, mu: int) -> np.ndarray:
    """I_d (x) ... (x) I_{mu+1} (x) L (x) I_{mu-1} (x) ... (x) I_1
    (equation tensor-structure); for rectangular L the identity factors keep
    their sizes and L maps n_mu -> m."""
    d = len(dims)
    K = np.ones((1, 1))
    # Kronecker product is built from the highest mode down to mode 1, so
    # that mode 1 is the fastest index of the result.
    for nu in range(d, 0, -1):
        F = L if nu == mu else np.eye(dims[nu - 1])
        K = np.kron(K, F)
    return K


def kron_sum(mats) -> np.ndarray:
    """M = A_d (+) ... (+) A_1 = sum_mu A_{(x) mu} (Section 2)."""
    dims = [A.shape[0] for A in mats]
    M = None
    for mu, A in enumerate(mats, start=1):
        F = kron_factor(dims, A, mu)
        M = F if M is None else M + F
    return M


def tucker(U: np.ndarray, mats) -> np.ndarray:
    """U x_1 L_1 x_2 L_2 ... x_d L_d, modes in the order 1..d (Section 2, the
    Tucker operator).  An entry ``None`` leaves that mode unchanged."""
    S = U
    for mu, L in enumerate(mats, start=1):
        if L is not None:
            S = mode_product(S, L, mu)
    return S


def expstep(U: np.ndarray, E, nsteps: int = 1) -> np.ndarray:
    """``nsteps`` applications of the mu-mode integrator (equation dd-tensor):
    U <- U x_1 E_1 x_2 ... x_d E_d with E_mu = exp(tau A_mu)."""
    S = U
    for _ in range(nsteps):
        S = tucker(S, E)
    return S
