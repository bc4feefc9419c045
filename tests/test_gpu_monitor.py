"""In-call monitor (norm every K steps, non-finite flag) of mumode_expstep and
gpe_strang_step against the FP64 oracle's sum |T|^2 after the same number of
steps (the discrete mass of §2 without the cell volume).

Tolerance: a state within relative L2 error e of the reference has a mass
within 2e + e^2 of the reference mass, and the flows here do not amplify
errors, so a record taken after k steps is held to 2 k tol (tol the one-step
bound of the precision)."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, from_gpu, note, to_gpu
from oracle import mumode as om
from oracle import operators as op
from oracle import schemes as sc

pytestmark = pytest.mark.gpu

N, A, B, BETA, TAU = 40, -8.0, 8.0, 100.0, 1e-3


@pytest.fixture(scope="module")
def mm():
    import paper_2103_01691_amd as m
    return m


@pytest.fixture()
def ctx(mm):
    c = mm.Context(0)
    yield c
    c.close()


def _mass(U):
    return float(np.sum(np.abs(U) ** 2))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x2"])
def test_gpe_monitor_log(ctx, mm, prec):
    psi0 = cast(synth.thomas_fermi_initial(N, A, B, 3, BETA, cfg_id=4), prec, True)
    E = op.ho_exponential(N, A, B, TAU)
    steps, every = 10, 3
    ctx.mm_set_option(mm.MM_OPT_MONITOR_EVERY, every)
    psi = to_gpu(psi0, prec, True)
    Eop = ctx.mm_op_prepare(E, prec)
    ctx.gpe_strang_step(psi, [Eop] * 3, TAU, BETA, steps)
    log = ctx.mm_monitor_log()
    assert [s for s, _ in log] == [3, 6, 9, 10]
    ref, p, done = [], psi0, 0
    for s, _ in log:
        p = sc.gpe_strang(p, [E] * 3, TAU, BETA, s - done)
        done = s
        ref.append(_mass(p))
    got = np.array([v for _, v in log])
    err = np.abs(got - ref) / np.array(ref)
    note(f"gpe monitor {prec}: rel mass errors {err}")
    assert np.all(err < 2 * np.array([s for s, _ in log]) * REL_TOL[prec])
    # the log is the mass of the state the call returned
    assert abs(got[-1] - _mass(from_gpu(psi))) <= 1e-6 * got[-1]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_expstep_monitor_log(ctx, mm, prec):
    # heat flow: the mass decays, so every record differs
    dims = (33, 20, 7)
    rng = np.random.default_rng(11)
    U0 = cast(rng.standard_normal(dims), prec, False)
    Es = [op.heat_exponential(n, 0.0, 1.0, "dirichlet", 1e-3) for n in dims]
    ctx.mm_set_option(mm.MM_OPT_MONITOR_EVERY, 2)
    T = to_gpu(U0, prec, False)
    ctx.mumode_expstep(T, [ctx.mm_op_prepare(E, prec) for E in Es], 5)
    log = ctx.mm_monitor_log()
    assert [s for s, _ in log] == [2, 4, 5]
    ref = [_mass(om.expstep(U0, Es, s)) for s, _ in log]
    got = np.array([v for _, v in log])
    assert np.all(np.diff(got) < 0)
    assert np.all(np.abs(got - ref) / np.array(ref) < 2 * np.array([s for s, _ in log]) * REL_TOL[prec])
    # switching the monitor off leaves the log of the next call empty
    ctx.mm_set_option(mm.MM_OPT_MONITOR_EVERY, 0)
    ctx.mumode_expstep(T, [ctx.mm_op_prepare(E, prec) for E in Es], 2)
    assert ctx.mm_monitor_log() == []


def test_monitor_flags_nonfinite(ctx, mm):
    psi0 = synth.thomas_fermi_initial(N, A, B, 3, BETA, cfg_id=4)
    psi0[3, 5, 7] = np.nan
    E = op.ho_exponential(N, A, B, TAU)
    ctx.mm_set_option(mm.MM_OPT_MONITOR_EVERY, 4)
    psi = to_gpu(psi0, "fp32", True)
    with pytest.raises(mm.MumodeError) as e:
        ctx.gpe_strang_step(psi, [ctx.mm_op_prepare(E, "fp32")] * 3, TAU, BETA, 5)
    assert e.value.status == 8  # MM_ERR_NONFINITE
    log = ctx.mm_monitor_log()
    assert [s for s, _ in log] == [4, 5] and not np.isfinite(log[0][1])


def test_monitor_rejects_negative_interval(ctx, mm):
    with pytest.raises(mm.MumodeError) as e:
        ctx.mm_set_option(mm.MM_OPT_MONITOR_EVERY, -1)
    assert e.value.status == 1  # MM_ERR_ARG
