"""GPU parity of the splitting steps and monitors against the oracle:
harmonic-oscillator Hermite Strang step (time-dependent potential) and the
GPE energy monitor."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, from_gpu, note, rel, to_gpu
from oracle import mumode as om
from oracle import operators as op
from oracle import schemes as sc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
@pytest.mark.parametrize("nsteps", [1, 4])
def test_ho_strang_matches_oracle(ctx, prec, nsteps):
    import paper_2103_01691_amd as mm
    m, kmax, t0, tau, eps = 48, 8, 0.3, 0.02, 0.1
    Phi, Psi, X = op.hermite_forward(m), op.hermite_backward(m), op.hermite_nodes(m)
    c = synth.hermite_coefficients(m, kmax, 3, cfg_id=3)
    psi0 = cast(om.tucker(c, [Psi] * 3), prec, True)
    ref = sc.ho_strang(psi0, [Phi] * 3, [Psi] * 3, [X] * 3, t0, tau, eps, nsteps)
    Xl, _ = mm.hermite_nodes(m)
    Fl, Bl = mm.hermite_matrices(m)
    F, B = ctx.mm_op_prepare(Fl, prec), ctx.mm_op_prepare(Bl, prec)
    psi = to_gpu(psi0, prec, True)
    ctx.ho_strang_step(psi, [F] * 3, [B] * 3, [Xl] * 3, t0, tau, eps, nsteps)
    err = rel(from_gpu(psi), ref)
    note(f"ho prec={prec} nsteps={nsteps} rel err {err:.3e}")
    assert err < REL_TOL[prec] * nsteps


@pytest.mark.parametrize("nsteps", [1, 3])
def test_ho_strang_mixed_precision_operators(ctx, nsteps):
    # one operator precision per mode: the step's operators are then prepared
    # one launch per mode (the same-precision case prepares all in one), and
    # the FP16x2 product starts its own running bound after the others
    import paper_2103_01691_amd as mm
    m, kmax, t0, tau, eps = 40, 8, 0.1, 0.02, 0.1
    Phi, Psi, X = op.hermite_forward(m), op.hermite_backward(m), op.hermite_nodes(m)
    c = synth.hermite_coefficients(m, kmax, 3, cfg_id=3)
    psi0 = cast(om.tucker(c, [Psi] * 3), "fp32", True)
    ref = sc.ho_strang(psi0, [Phi] * 3, [Psi] * 3, [X] * 3, t0, tau, eps, nsteps)
    Xl, _ = mm.hermite_nodes(m)
    Fl, Bl = mm.hermite_matrices(m)
    F = [ctx.mm_op_prepare(Fl, p) for p in ("fp32", "bf16x3", "fp16x2")]
    B = [ctx.mm_op_prepare(Bl, p) for p in ("fp32", "bf16x3", "fp16x2")]
    psi = to_gpu(psi0, "fp32", True)
    ctx.ho_strang_step(psi, F, B, [Xl] * 3, t0, tau, eps, nsteps)
    err = rel(from_gpu(psi), ref)
    note(f"ho mixed precisions nsteps={nsteps} rel err {err:.3e}")
    assert err < REL_TOL["fp32"] * nsteps


def test_ho_eigenstate_phase_on_gpu(ctx):
    import paper_2103_01691_amd as mm
    m, tau = 32, 0.37
    X, _ = mm.hermite_nodes(m)
    f = op.hermite_functions(m, op.hermite_nodes(m))
    k = (3, 1, 6)
    psi0 = f[k[0]][:, None, None] * f[k[1]][None, :, None] * f[k[2]][None, None, :]
    Fl, Bl = mm.hermite_matrices(m)
    F, B = ctx.mm_op_prepare(Fl, "fp64"), ctx.mm_op_prepare(Bl, "fp64")
    psi = to_gpu(psi0.astype(np.complex128), "fp64", True)
    ctx.ho_strang_step(psi, [F] * 3, [B] * 3, [X] * 3, 0.0, tau, 0.0, 2)
    assert rel(from_gpu(psi), np.exp(-2j * tau * (sum(k) + 1.5)) * psi0) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_energy_gpe_matches_oracle(ctx, prec):
    import paper_2103_01691_amd as mm
    n, a, b, beta = 40, -8.0, 8.0, 100.0
    h = (b - a) / (n + 1)
    psi0 = cast(synth.thomas_fermi_initial(n, a, b, 3, beta, cfg_id=4), prec, True)
    Ho = op.ho_hamiltonian(n, a, b)
    ref = sc.energy_gpe(psi0, [Ho] * 3, beta, h ** 3)
    Hl = mm.schrodinger_fd_hamiltonian(n, a, b, 1.0)
    Hop = ctx.mm_op_prepare(Hl, prec)
    e = ctx.mm_energy_gpe(to_gpu(psi0, prec, True), [Hop] * 3, beta, h ** 3)
    note(f"energy prec={prec} gpu={e:.12g} oracle={ref:.12g}")
    assert abs(e - ref) / abs(ref) < (1e-12 if prec == "fp64" else 1e-5)
