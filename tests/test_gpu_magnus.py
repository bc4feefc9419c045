"""GPU parity of the device matrix exponential and of the exponential
midpoint (second-order Magnus) integrator against the oracle, on the
time-dependent Schroedinger problem of Section 4.4 in nodal Hermite space."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, from_gpu, note, rel, to_gpu
from oracle import operators as op
from oracle import schemes as sc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("n,scale,c", [(5, 1.0, 1.0), (37, 3.0, -0.7j), (64, 20.0, 0.05 - 1j), (200, 8.0, 1j)])
def test_expm_device_matches_scipy(ctx, n, scale, c):
    import torch
    from scipy.linalg import expm
    g = synth.rng(1201, n)
    A = (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))) * scale / np.sqrt(n)
    ref = expm(c * A)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda()          # column-major storage of A
    out = torch.empty_like(Ad)
    ctx.mm_expm_device(Ad, c, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().T
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    note(f"device expm n={n} |cA|~{scale * abs(c):.2f} rel err {err:.3e}")
    assert err < 1e-12


def _lib_problem(mm, m):
    Phi, Psi = mm.hermite_matrices(m)
    X, _ = mm.hermite_nodes(m)
    Bm = Psi @ np.diag(-1j * (np.arange(m) + 0.5)) @ Phi
    return [Bm, Bm, Bm], [None, None, X]


def _coeffs(nsteps, tau, t0=0.0):
    g = np.zeros((nsteps, 3), dtype=np.complex128)
    for k in range(nsteps):
        g[k, 2] = -1j * np.sin(t0 + (k + 0.5) * tau) ** 2
    return g


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_magnus_step_matches_oracle(ctx, prec):
    import paper_2103_01691_amd as mm
    m, tau, nsteps = 24, 0.02, 3
    c = synth.hermite_coefficients(m, 8, 3, cfg_id=3)
    from oracle import mumode as om
    psi0 = cast(om.tucker(c, [op.hermite_backward(m)] * 3), prec, True)
    B, d, gf = op.hkmp_problem(m)
    ref = sc.magnus_midpoint(psi0, B, d, gf, tau, nsteps)
    Bl, dl = _lib_problem(mm, m)
    psi = to_gpu(psi0, prec, True)
    ctx.mumode_magnus_step(psi, Bl, dl, _coeffs(nsteps, tau), tau, nsteps, prec)
    err = rel(from_gpu(psi), ref)
    note(f"magnus m={m} {nsteps} steps {prec} rel err {err:.3e}")
    assert err < (1e-12 if prec == "fp64" else REL_TOL[prec]) * nsteps


@pytest.mark.parametrize("prec", ["fp64", "fp16x2"])
def test_magnus_step_hermite_128(ctx, prec):
    import paper_2103_01691_amd as mm
    from oracle import mumode as om
    m, tau = 128, 0.02
    c = synth.hermite_coefficients(m, 16, 3, cfg_id=3)
    psi0 = cast(om.tucker(c, [op.hermite_backward(m)] * 3), prec, True)
    B, d, gf = op.hkmp_problem(m)
    ref = sc.magnus_midpoint(psi0, B, d, gf, tau, 1, t0=0.3)
    Bl, dl = _lib_problem(mm, m)
    psi = to_gpu(psi0, prec, True)
    ctx.mumode_magnus_step(psi, Bl, dl, _coeffs(1, tau, 0.3), tau, 1, prec)
    err = rel(from_gpu(psi), ref)
    note(f"magnus m=128 one step {prec} rel err {err:.3e}")
    assert err < (1e-12 if prec == "fp64" else REL_TOL[prec])


def test_magnus_rejects_missing_coefficients(ctx):
    import paper_2103_01691_amd as mm
    m = 8
    Bl, dl = _lib_problem(mm, m)
    psi = to_gpu(np.zeros((m, m, m), np.complex128), "fp64", True)
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_magnus_step(psi, Bl, dl, None, 0.1, 1, "fp64")
    assert e.value.status == 1
