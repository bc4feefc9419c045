"""Per-launch profiling (mm_profile_begin / mm_profile_end): recording the
launch events must not change results, and the records must describe the
launches that ran."""
import numpy as np
import pytest

import synth
from gpu_util import from_gpu, note, to_gpu
from oracle import operators as op

pytestmark = pytest.mark.gpu

N, A, B, BETA, TAU, STEPS = 48, -8.0, 8.0, 100.0, 1e-3, 4


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16x2"])
def test_profiled_run_is_bit_identical_and_recorded(ctx, prec):
    import torch
    psi0 = synth.thomas_fermi_initial(N, A, B, 3, BETA, cfg_id=4)
    E = ctx.mm_op_prepare(op.ho_exponential(N, A, B, TAU), prec)
    plain = to_gpu(psi0, prec, True)
    ctx.gpe_strang_step(plain, [E] * 3, TAU, BETA, STEPS)
    prof = to_gpu(psi0, prec, True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ctx.mm_profile_begin()
    ev0.record()
    ctx.gpe_strang_step(prof, [E] * 3, TAU, BETA, STEPS)
    ev1.record()
    recs = ctx.mm_profile_end()
    torch.cuda.synchronize()
    span = ev0.elapsed_time(ev1)
    assert np.array_equal(from_gpu(plain), from_gpu(prof))
    assert len(recs) == 3 * STEPS
    kinds = [k for k, _ in recs]
    # kind = prec*1000 + complex*100 + load*10 + prologue*2 + epilogue:
    # the first product of every step carries the phase before it, the
    # last product of the call the closing half phase
    assert all((k // 100) % 10 == 1 for k in kinds)
    assert (kinds[0] % 10) & 2 and kinds[-1] % 2 == 1
    assert all(k % 2 == 0 for k in kinds[:-1])
    ms = np.array([t for _, t in recs])
    note(f"profile {prec}: {len(recs)} launches, sum {ms.sum():.4f} ms, span {span:.4f} ms")
    assert np.all(ms > 0) and ms.sum() <= span * 1.05
