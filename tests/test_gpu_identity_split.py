"""GPU parity of operators prepared with the identity split
(MM_OP_IDENTITY_SPLIT: the pieces hold L - I, each product adds its input
back in FP32): every epilogue form (full-tile LDS-staged, full-tile direct,
bounds-checked), every load path, real and complex, with and without the
fused phases, the batched step, and the argument checks."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, empty_gpu, from_gpu, note, rel, to_gpu
from oracle import mumode as om
from oracle import operators as op
from oracle import schemes as sc

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32", "bf16x3", "fp16x2"]


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


def _near_identity(n, cplx, g, eps=0.05):
    # I + eps R: the case the split is for (small-step exponentials)
    return np.eye(n) + eps * synth.random_matrix(n, n, cplx, g)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("dims", [(48, 40, 36), (37, 30, 21), (64, 32, 16)])
@pytest.mark.parametrize("mu", [1, 2, 3])
def test_apply_identity_split(ctx, prec, cplx, dims, mu):
    g = synth.rng(1501, mu)
    U = cast(synth.random_tensor(dims, cplx, g), prec, cplx)
    n = dims[mu - 1]
    L = _near_identity(n, cplx, g)
    ref = om.mode_product(U, L, mu)
    Lop = ctx.mm_op_prepare(L, prec, identity_split=True)
    out = empty_gpu(dims, prec, cplx)
    ctx.mumode_apply(out, to_gpu(U, prec, cplx), Lop, mu)
    err = rel(from_gpu(out), ref)
    Lop.destroy()
    note(f"identity split apply {prec} cplx={cplx} dims={dims} mu={mu}: rel err {err:.3e}")
    assert err < REL_TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("mu", [1, 2])
def test_apply_identity_split_real_operator_on_complex_state(ctx, prec, mu):
    dims = (64, 40, 12)
    g = synth.rng(1502, mu)
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    L = _near_identity(dims[mu - 1], False, g)
    Lop = ctx.mm_op_prepare(L, prec, identity_split=True)
    out = empty_gpu(dims, prec, True)
    ctx.mumode_apply(out, to_gpu(U, prec, True), Lop, mu)
    err = rel(from_gpu(out), om.mode_product(U, L, mu))
    Lop.destroy()
    assert err < REL_TOL[prec]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,nsteps", [(48, 3), (256, 2)])
def test_gpe_identity_split(ctx, prec, n, nsteps):
    # n = 256: full tiles (LDS-staged epilogue on mode 1, direct stores on
    # modes 2, 3) with the fused prologue and epilogue phases
    import paper_2103_01691_amd as mm
    a, b, beta, tau = -8.0, 8.0, 100.0, 1e-3
    psi0 = cast(synth.thomas_fermi_initial(n, a, b, 3, beta, cfg_id=4), prec, True)
    E = ctx.mm_op_prepare(mm.schrodinger_fd_exponential(n, a, b, 1.0, tau), prec, identity_split=True)
    psi = to_gpu(psi0, prec, True)
    note(f"identity split gpe n={n} {prec} {nsteps} steps")
    ctx.gpe_strang_step(psi, [E] * 3, tau, beta, nsteps)
    got = from_gpu(psi)
    del psi
    E.destroy()
    ref = sc.gpe_strang(psi0, [op.ho_exponential(n, a, b, tau)] * 3, tau, beta, nsteps)
    err = rel(got, ref)
    note(f"  rel err {err:.3e}")
    assert err < nsteps * REL_TOL[prec]


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x2"])
@pytest.mark.parametrize("cls", [8, 9])
def test_identity_split_ignores_three_product_class(ctx, tmp_path, prec, cls):
    # the three-product kernels have no identity-add form: a tune entry that
    # names one for the shape of an identity-split product must give way to
    # a four-product class (same result as untuned)
    import paper_2103_01691_amd as mm
    code = {"bf16x3": 2, "fp16x2": 3}[prec]
    n, a, b, beta, tau = 64, -8.0, 8.0, 100.0, 1e-3
    psi0 = cast(synth.thomas_fermi_initial(n, a, b, 3, beta, cfg_id=4), prec, True)
    lines = [f"{code} 1 {ld} {2 * n} {2 * n} {n * n} {cls} 0.0\n" for ld in (0, 1, 8, 9)]
    f = tmp_path / "t.txt"
    f.write_text("mumode-tune 1\n" + "".join(lines))
    E = ctx.mm_op_prepare(mm.schrodinger_fd_exponential(n, a, b, 1.0, tau), prec, identity_split=True)
    ref = sc.gpe_strang(psi0, [op.ho_exponential(n, a, b, tau)] * 3, tau, beta, 2)
    outs = []
    for tuned in (False, True):
        ctx.mm_tune_clear()
        if tuned:
            ctx.mm_tune_load(f)
        psi = to_gpu(psi0, prec, True)
        ctx.gpe_strang_step(psi, [E] * 3, tau, beta, 2)
        outs.append(from_gpu(psi))
    ctx.mm_tune_clear()
    E.destroy()
    note(f"identity split, class {cls} in the tune table, {prec}: rel err {rel(outs[1], ref):.3e}")
    assert np.array_equal(outs[0], outs[1])
    assert rel(outs[1], ref) < 2 * REL_TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batched_identity_split(ctx, prec):
    g = synth.rng(1503, 0)
    dims = [(32, 48, 40), (64, 32), (96, 64)]
    cplx = [True, False, True]
    U = [cast(synth.random_tensor(d, c, g), prec, c) for d, c in zip(dims, cplx)]
    E = [[_near_identity(n, c, g) for n in d] for d, c in zip(dims, cplx)]
    ops = [[ctx.mm_op_prepare(e, prec, identity_split=True) for e in el] for el in E]
    T = [to_gpu(u, prec, c) for u, c in zip(U, cplx)]
    ctx.mumode_expstep_batched(T, ops, 2)
    for t, u, el in zip(T, U, E):
        assert rel(from_gpu(t), om.expstep(u, el, 2)) < 2 * REL_TOL[prec]
    for ol in ops:
        for o in ol:
            o.destroy()


def test_identity_split_checks(ctx):
    import paper_2103_01691_amd as mm
    with pytest.raises(mm.MumodeError) as e:
        ctx.mm_op_prepare(np.ones((4, 5)), "fp32", identity_split=True)
    assert e.value.status == 2
    Lop = ctx.mm_op_prepare(np.eye(6), "fp32", identity_split=True)
    flags = mm._lib.C.c_uint()
    assert mm._lib.lib.mm_op_flags(Lop.handle, mm._lib.C.byref(flags)) == 0 and flags.value == 1
    Lop.destroy()
