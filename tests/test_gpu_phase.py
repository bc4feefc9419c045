"""The fused nonlinear phase of the GPE step at small and large phase angles.

The split FP16x2 path compiles its prologue sincos without range reduction
when the running state bound proves every angle |s| |psi|^2 is within pi/4,
and with it otherwise; beta = 100 (angles below 0.01) takes the first form,
beta = 1e5 (angles up to ~3.4 rad at tau = 1e-3) the second.  Both are held
to the oracle's unmerged Strang steps.  Tolerance per step: the product
bound of the precision plus the FP32 rounding of the angle itself
(8 theta_max 2^-24, FP32 state paths only)."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, from_gpu, note, rel, to_gpu
from oracle import operators as op
from oracle import schemes as sc

pytestmark = pytest.mark.gpu

N, A, B, TAU, STEPS = 40, -8.0, 8.0, 1e-3, 3


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("beta", [100.0, 1e5])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_gpe_phase_angles(ctx, prec, beta):
    psi0 = cast(synth.thomas_fermi_initial(N, A, B, 3, 100.0, cfg_id=4), prec, True)
    E = op.ho_exponential(N, A, B, TAU)
    ref = sc.gpe_strang(psi0, [E] * 3, TAU, beta, STEPS)
    psi = to_gpu(psi0, prec, True)
    ctx.gpe_strang_step(psi, [ctx.mm_op_prepare(E, prec)] * 3, TAU, beta, STEPS)
    err = rel(from_gpu(psi), ref)
    theta = TAU * beta * float(np.max(np.abs(psi0) ** 2))
    tol = STEPS * (REL_TOL[prec] + (0.0 if prec == "fp64" else 8 * theta * 2.0 ** -24))
    note(f"gpe phase beta={beta:g} (max angle {theta:.3g}) {prec}: rel err {err:.3e} (tol {tol:.2e})")
    assert err < tol
