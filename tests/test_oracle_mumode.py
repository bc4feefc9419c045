"""Pins of the oracle's mu-mode product and integrator (CPU only)."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import mumode as om


def _rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("mu", [1, 2, 3])
def test_mode_product_vs_loops_rectangular_complex(mu):
    g = synth.rng(101, mu)
    dims = (3, 4, 5)
    U = synth.random_tensor(dims, True, g)
    L = synth.random_matrix(6, dims[mu - 1], True, g)   # rectangular, non-symmetric
    S = om.mode_product(U, L, mu)
    S_loop = om.mode_product_loops(U, L, mu)
    assert S.shape[mu - 1] == 6
    assert _rel(S, S_loop) < 1e-14


@pytest.mark.parametrize("mu", [1, 2, 3])
def test_mode_product_vs_kronecker_matrix(mu):
    g = synth.rng(102, mu)
    dims = (3, 4, 5)
    U = synth.random_tensor(dims, True, g)
    L = synth.random_matrix(7, dims[mu - 1], True, g)
    K = om.kron_factor(dims, L, mu)
    out_dims = list(dims)
    out_dims[mu - 1] = 7
    S_k = om.unvec(K @ om.vec(U), out_dims)
    assert _rel(om.mode_product(U, L, mu), S_k) < 1e-14


def test_transposed_operator_is_detected():
    # a plausible bug (using L^T) must change the result for non-symmetric L
    g = synth.rng(103, 0)
    U = synth.random_tensor((4, 4), False, g)
    L = synth.random_matrix(4, 4, False, g)
    assert _rel(om.mode_product(U, L.T, 1), om.mode_product(U, L, 1)) > 1e-2


def test_modes_commute():
    # products along different modes commute (Section 2)
    g = synth.rng(104, 0)
    U = synth.random_tensor((4, 5, 6), True, g)
    A = synth.random_matrix(4, 4, True, g)
    B = synth.random_matrix(5, 5, True, g)
    lhs = om.mode_product(om.mode_product(U, A, 1), B, 2)
    rhs = om.mode_product(om.mode_product(U, B, 2), A, 1)
    assert _rel(lhs, rhs) < 1e-14


def test_expstep_equals_expm_of_kronecker_sum():
    # u(t) = exp(tM) u0 with M the Kronecker sum of arbitrary A_mu (Section 2)
    g = synth.rng(105, 0)
    dims = (4, 5, 6)
    A = [synth.random_matrix(n, n, True, g) for n in dims]
    t = 0.7
    M = om.kron_sum(A)
    U = synth.random_tensor(dims, True, g)
    ref = om.unvec(scipy.linalg.expm(t * M) @ om.vec(U), dims)
    E = [scipy.linalg.expm(t * a) for a in A]
    assert _rel(om.expstep(U, E, 1), ref) < 1e-13
    # two steps of t/2 equal one step of t (exact in time)
    Eh = [scipy.linalg.expm(0.5 * t * a) for a in A]
    assert _rel(om.expstep(U, Eh, 2), ref) < 1e-13


def test_kron_sum_structure_2d():
    # M = I_2 (x) A_1 + A_2 (x) I_1 (Section 2, equation heat2D-fd)
    g = synth.rng(106, 0)
    A1 = synth.random_matrix(3, 3, False, g)
    A2 = synth.random_matrix(4, 4, False, g)
    M = om.kron_sum([A1, A2])
    ref = np.kron(np.eye(4), A1) + np.kron(A2, np.eye(3))
    assert np.max(np.abs(M - ref)) == 0.0


def test_tucker_none_is_identity():
    g = synth.rng(107, 0)
    U = synth.random_tensor((3, 4), True, g)
    L = synth.random_matrix(4, 4, True, g)
    assert _rel(om.tucker(U, [None, L]), om.mode_product(U, L, 2)) == 0.0
