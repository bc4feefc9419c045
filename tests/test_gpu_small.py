"""GPU parity of the whole-run single-workgroup paths for small expsteps
(every step and mode in one launch) against the oracle and against the
one-launch-per-product path: the general one (state in global memory / L2
between products) and, for 2-D real FP64 states with both modes at most 64
long, the one holding the state and both operators in LDS."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, from_gpu, note, rel, to_gpu
from oracle import mumode as om
from oracle import operators as op

pytestmark = pytest.mark.gpu

SMALL_KIND = 90
LDS_KIND = 91


def _expect(prec, cplx, dims):
    return LDS_KIND if (prec == "fp64" and not cplx and len(dims) == 2 and max(dims) <= 64) else SMALL_KIND


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


def _run(ctx, U, ops, nsteps, prec, cplx, small):
    import paper_2103_01691_amd as mm
    ctx.mm_set_option(mm.MM_OPT_SMALL_RUN, 1 if small else 0)
    T = to_gpu(U, prec, cplx)
    ctx.mm_profile_begin()
    ctx.mumode_expstep(T, ops, nsteps)
    kinds = [k % 100 for k, _ in ctx.mm_profile_end()]
    ctx.mm_set_option(mm.MM_OPT_SMALL_RUN, 1)
    return from_gpu(T), kinds


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("cplx,dims", [(False, (64, 64)), (True, (16, 20, 12)), (False, (37, 30, 21)),
                                       (True, (64, 40)), (False, (6, 5, 4, 3))])
def test_small_run_matches_oracle(ctx, prec, cplx, dims):
    g = synth.rng(1301, len(dims) + int(cplx))
    U = cast(synth.random_tensor(dims, cplx, g), prec, cplx)
    E = [synth.random_matrix(n, n, cplx, g) for n in dims]
    ops = [ctx.mm_op_prepare(e, prec) for e in E]
    nsteps = 5
    ref = om.expstep(U, E, nsteps)
    got, kinds = _run(ctx, U, ops, nsteps, prec, cplx, True)
    off, kinds_off = _run(ctx, U, ops, nsteps, prec, cplx, False)
    err, err_off = rel(got, ref), rel(off, ref)
    note(f"small run {prec} cplx={cplx} dims={dims}: rel err {err:.3e} (per-product path {err_off:.3e}), "
         f"launches {len(kinds)} vs {len(kinds_off)}")
    assert kinds == [_expect(prec, cplx, dims)]
    assert len(kinds_off) == nsteps * len(dims)
    assert err < REL_TOL[prec] * nsteps
    assert err_off < REL_TOL[prec] * nsteps


def test_small_run_heat_config(ctx):
    import paper_2103_01691_amd as mm
    n, tau = 64, 1e-3
    u0 = synth.heat_initial(n, 2, cfg_id=1)
    E = mm.expm(mm.fd2_matrix(n, 0.0, 1.0), tau).real.copy()
    Eo = op.heat_exponential(n, 0.0, 1.0, "dirichlet", tau)
    got, kinds = _run(ctx, u0, [ctx.mm_op_prepare(E, "fp64")] * 2, 20, "fp64", False, True)
    assert kinds == [LDS_KIND]
    assert rel(got, om.expstep(u0, [Eo] * 2, 20)) < 1e-12


def test_small_run_not_taken_for_large_or_split(ctx):
    g = synth.rng(1302, 0)
    U = cast(synth.random_tensor((16, 16, 8), True, g), "bf16x3", True)
    E = [synth.random_matrix(n, n, True, g) for n in (16, 16, 8)]
    got, kinds = _run(ctx, U, [ctx.mm_op_prepare(e, "bf16x3") for e in E], 2, "bf16x3", True, True)
    assert SMALL_KIND not in kinds and LDS_KIND not in kinds
    U = cast(synth.random_tensor((256, 24, 4), True, g), "fp32", True)   # 256 complex rows > one small tile
    E = [synth.random_matrix(n, n, True, g) for n in (256, 24, 4)]
    got, kinds = _run(ctx, U, [ctx.mm_op_prepare(e, "fp32") for e in E], 2, "fp32", True, True)
    assert SMALL_KIND not in kinds
    assert rel(got, om.expstep(U, E, 2)) < REL_TOL["fp32"] * 2


@pytest.mark.parametrize("dims,modes", [((37, 50), (1, 1)), ((64, 16), (0, 1)), ((1, 64), (1, 0)), ((17, 3), (1, 1))])
def test_lds_run_ragged_and_identity_modes(ctx, dims, modes):
    # ragged sizes (padding to whole 16-row tiles), a NULL operator leaving
    # its mode unchanged, unit-length modes
    g = synth.rng(1303, dims[0] + dims[1])
    U = cast(synth.random_tensor(dims, False, g), "fp64", False)
    E = [synth.random_matrix(n, n, False, g) if m else None for n, m in zip(dims, modes)]
    ops = [ctx.mm_op_prepare(e, "fp64") if e is not None else None for e in E]
    nsteps = 7
    ref = U
    for _ in range(nsteps):
        for mu, e in enumerate(E, start=1):
            if e is not None:
                ref = om.mode_product(ref, e, mu)
    got, kinds = _run(ctx, U, ops, nsteps, "fp64", False, True)
    err = rel(got, ref)
    note(f"LDS run dims={dims} modes={modes}: rel err {err:.3e}")
    assert kinds == [LDS_KIND]
    assert err < 1e-12 * nsteps
