"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol the header declares, reports the missing device cleanly, and its FP64
host-side operator formation agrees with the oracle."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import operators as op

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2103_01691_amd import _lib
    return _lib


def _header_functions():
    src = open(os.path.join(ROOT, "include", "mumode.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_binding_exports():
    assert sorted(_lib().EXPORTS) == _header_functions()


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_lib().LIB_PATH)
    for name in _header_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = _lib().lib
    for s in range(10):
        assert lib.mm_status_string(s)
    assert lib.mm_status_string(99) == b"unknown status"


def test_create_without_gpu_reports_nodevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib().lib
    h = C.c_void_p()
    assert lib.mm_create(C.byref(h), 0, None) == _lib().MM_ERR_NODEVICE
    assert h.value is None
    assert b"device" in lib.mm_last_error(None)
    assert lib.mm_destroy(None) == 0


def test_null_context_rejected():
    lib = _lib().lib
    t = _lib().MMTensor()
    assert lib.mumode_apply(None, C.byref(t), C.byref(t), None, 1, None) == _lib().MM_ERR_ARG
    assert lib.mumode_expstep(None, C.byref(t), None, 1, None) == _lib().MM_ERR_ARG


# ---------------------------------------------- host operator formation ----

def test_fd2_matrix_matches_oracle():
    import paper_2103_01691_amd as mm
    for bc in ("dirichlet", "periodic"):
        for n in (5, 64, 257):
            assert np.max(np.abs(mm.fd2_matrix(n, -8.0, 8.0, bc) - op.fd2(n, -8.0, 8.0, bc))) < 1e-9


@pytest.mark.parametrize("kind", ["heat", "schrodinger", "ho"])
def test_library_expm_matches_oracle(kind):
    import paper_2103_01691_amd as mm
    n = 96
    if kind == "heat":
        A, c = op.fd2(n, 0.0, 1.0, "dirichlet"), 1e-3
        ref = op.heat_exponential(n, 0.0, 1.0, "dirichlet", 1e-3)
    elif kind == "schrodinger":
        A, c = op.fd2(n, -10.0, 10.0, "dirichlet"), 0.5j * 0.01
        ref = op.free_schrodinger_exponential(n, -10.0, 10.0, 0.01)
    else:
        A, c = op.ho_hamiltonian(n, -8.0, 8.0), -1j * 0.1
        ref = op.ho_exponential(n, -8.0, 8.0, 0.1)
    E = mm.expm(A, c)
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-13


def test_library_expm_general_nonnormal():
    import paper_2103_01691_amd as mm
    g = synth.rng(401, 0)
    A = synth.random_matrix(30, 30, True, g, scale=1.0)
    E = mm.expm(A, 0.7)
    ref = scipy.linalg.expm(0.7 * A)
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("m", [16, 128])
def test_library_hermite_matches_oracle(m):
    import paper_2103_01691_amd as mm
    X, w = mm.hermite_nodes(m)
    assert np.max(np.abs(X - op.hermite_nodes(m))) < 1e-12 * 16
    assert np.max(np.abs(w / op.hermite_weights(m) - 1)) < 1e-11
    Phi, Psi = mm.hermite_matrices(m)
    assert np.max(np.abs(Phi - op.hermite_forward(m))) < 1e-12
    assert np.max(np.abs(Psi - op.hermite_backward(m))) < 1e-12


def test_host_builders_validate():
    lib = _lib().lib
    buf = (C.c_double * 4)()
    assert lib.mm_fd2_matrix(0, 0.0, 1.0, 0, buf) == _lib().MM_ERR_SHAPE
    assert lib.mm_fd2_matrix(2, 1.0, 0.0, 0, buf) == _lib().MM_ERR_SHAPE
    assert lib.mm_fd2_matrix(2, 0.0, 1.0, 7, buf) == _lib().MM_ERR_ARG
    assert lib.mm_fd2_matrix(2, 0.0, 1.0, 0, None) == _lib().MM_ERR_ARG
    assert lib.mm_expm(0, buf, 1.0, 0.0, buf) == _lib().MM_ERR_SHAPE
    nan = (C.c_double * 2)(float("nan"), 0.0)
    assert lib.mm_expm(1, nan, 1.0, 0.0, buf) == _lib().MM_ERR_NONFINITE


@pytest.mark.parametrize("order", [2, 4, 6, 10, 16])
def test_library_fd2_periodic_order_matches_oracle(order):
    import paper_2103_01691_amd as mm
    for n in (order + 1, 40, 101):
        L = mm.fd2_periodic_order(n, 0.0, 2 * np.pi, order)
        O = op.fd2_periodic_order(n, 0.0, 2 * np.pi, order)
        assert np.max(np.abs(L - O)) <= 1e-9 * np.max(np.abs(O))


@pytest.mark.parametrize("n", [2, 7, 24, 65, 128])
def test_library_fourier_d2_matches_oracle(n):
    import paper_2103_01691_amd as mm
    L = mm.fourier_d2(n, -1.0, 3.0)
    O = op.fourier_d2(n, -1.0, 3.0)
    assert np.max(np.abs(L - O)) <= 1e-10 * np.max(np.abs(O))


def test_library_pipe_flow_operators_match_oracle():
    import paper_2103_01691_amd as mm
    for nr, nz in ((3, 3), (50, 70), (200, 200)):
        Lr, Lz = mm.pipe_flow_operators(nr, nz, 0.1, 5.0, 8.0, 1.0 / 90)
        Or, Oz, _, _ = op.pipe_flow_operators(nr, nz, 0.1, 5.0, 8.0, 1.0 / 90)
        assert np.max(np.abs(Lr - Or)) <= 1e-12 * np.max(np.abs(Or))
        assert np.max(np.abs(Lz - Oz)) <= 1e-12 * np.max(np.abs(Oz))


def test_front_end_builders_validate():
    import paper_2103_01691_amd as mm
    with pytest.raises(mm.MumodeError):
        mm.fd2_periodic_order(10, 0.0, 1.0, 3)          # odd order
    with pytest.raises(mm.MumodeError):
        mm.fd2_periodic_order(4, 0.0, 1.0, 8)           # stencil wider than the grid
    with pytest.raises(mm.MumodeError):
        mm.fourier_d2(8, 1.0, 1.0)
    with pytest.raises(mm.MumodeError):
        mm.pipe_flow_operators(10, 10, 0.0, 5.0, 8.0)   # r_min must be > 0


@pytest.mark.parametrize("n", [8, 96, 256])
def test_library_schrodinger_builders_match_oracle(n):
    # the library's Hamiltonian and exponentials against the oracle's, whose
    # constants are pinned to the continuum physics (tests/test_oracle_physics.py)
    import paper_2103_01691_amd as mm
    H = mm.schrodinger_fd_hamiltonian(n, -8.0, 8.0, 1.0)
    assert np.max(np.abs(H - op.ho_hamiltonian(n, -8.0, 8.0))) <= 1e-12 * np.max(np.abs(H))
    E = mm.schrodinger_fd_exponential(n, -8.0, 8.0, 1.0, 0.1)
    ref = op.ho_exponential(n, -8.0, 8.0, 0.1)
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-12
    F = mm.schrodinger_fd_exponential(n, -10.0, 10.0, 0.0, 0.01)
    ref = op.free_schrodinger_exponential(n, -10.0, 10.0, 0.01)
    assert np.linalg.norm(F - ref) / np.linalg.norm(ref) < 1e-12


def test_library_hermite_generator_matches_oracle():
    import paper_2103_01691_amd as mm
    for m in (4, 40):
        G = mm.hermite_ho_generator(m)
        ref = op.hermite_ho_generator(m)
        assert np.max(np.abs(G - ref)) <= 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("alpha", [0.0, 2.0])
def test_library_nonuniform_neumann_matches_oracle(alpha):
    import paper_2103_01691_amd as mm
    for n in (2, 5, 64):
        x = synth.graded_nodes(n, -20.0, 20.0, alpha)
        M, w = mm.nonuniform_neumann_d2(x)
        Mo, wo = op.nonuniform_neumann_d2(x)
        assert np.max(np.abs(M - Mo)) <= 1e-14 * np.max(np.abs(Mo))
        assert np.max(np.abs(w - wo)) <= 1e-14 * np.max(wo)


def test_library_nonuniform_neumann_validates():
    import paper_2103_01691_amd as mm
    with pytest.raises(mm.MumodeError):
        mm.nonuniform_neumann_d2(np.array([0.0, 1.0, 1.0, 2.0]))     # not strictly increasing
    with pytest.raises(mm.MumodeError):
        mm.nonuniform_neumann_d2(np.array([0.0]))
