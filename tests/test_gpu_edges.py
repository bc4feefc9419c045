"""Edge and degenerate cases of the mu-mode path on the GPU, against the
oracle: tensors of order 1 and 6, modes of length 1, a 1 x 1 operator,
modes longer than one workgroup's rows (products through the workspace),
the largest operator the library accepts, zero steps, invalid shapes."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, empty_gpu, from_gpu, note, rel, to_gpu
from oracle import mumode as om

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
@pytest.mark.parametrize("dims", [(300,), (5, 1, 7), (1, 33), (3, 4, 2, 5, 3, 4), (1, 1, 1)])
def test_expstep_degenerate_shapes(ctx, prec, dims):
    g = synth.rng(1401, len(dims) * 7 + sum(dims))
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    E = [synth.random_matrix(n, n, True, g) for n in dims]
    T = to_gpu(U, prec, True)
    ctx.mumode_expstep(T, [ctx.mm_op_prepare(e, prec) for e in E], 2)
    err = rel(from_gpu(T), om.expstep(U, E, 2))
    note(f"degenerate {dims} {prec}: rel err {err:.3e}")
    assert err < 2 * REL_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x2"])
def test_long_mode_goes_through_workspace(ctx, prec):
    # 600 complex rows per mode: more than one workgroup's rows, so products
    # cannot run in place
    dims = (600, 6, 4)
    g = synth.rng(1402, 0)
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    E = [synth.random_matrix(n, n, True, g) for n in dims]
    T = to_gpu(U, prec, True)
    ctx.mumode_expstep(T, [ctx.mm_op_prepare(e, prec) for e in E], 1)
    err = rel(from_gpu(T), om.expstep(U, E, 1))
    note(f"long mode {dims} {prec}: rel err {err:.3e}")
    assert err < REL_TOL[prec]


def test_largest_operator(ctx):
    # 4096 x 4096 real operator (the maximum) on a thin tensor, FP32
    n, q = 4096, 8
    g = synth.rng(1403, 0)
    U = cast(synth.random_tensor((n, q), False, g), "fp32", False)
    L = synth.random_matrix(n, n, False, g)
    out = empty_gpu((n, q), "fp32", False)
    ctx.mumode_apply(out, to_gpu(U, "fp32", False), ctx.mm_op_prepare(L, "fp32"), 1)
    err = rel(from_gpu(out), om.mode_product(U, L, 1))
    note(f"largest operator 4096 x 4096 fp32: rel err {err:.3e}")
    assert err < REL_TOL["fp32"]


def test_one_by_one_operator_scales(ctx):
    U = synth.random_tensor((1, 40), True, synth.rng(1404, 0))
    L = np.array([[0.5 - 2.0j]])
    out = empty_gpu((1, 40), "fp64", True)
    ctx.mumode_apply(out, to_gpu(U, "fp64", True), ctx.mm_op_prepare(L, "fp64"), 1)
    assert rel(from_gpu(out), L[0, 0] * U) < 1e-15


def test_zero_steps_is_identity(ctx):
    g = synth.rng(1405, 0)
    U = synth.random_tensor((16, 12), True, g)
    T = to_gpu(U, "fp64", True)
    ops = [ctx.mm_op_prepare(synth.random_matrix(n, n, True, g), "fp64") for n in (16, 12)]
    ctx.mumode_expstep(T, ops, 0)
    ctx.gpe_strang_step(T, ops, 0.1, 10.0, 0)
    assert rel(from_gpu(T), U) == 0.0


def test_invalid_shapes_rejected(ctx):
    import torch
    import paper_2103_01691_amd as mm
    with pytest.raises(mm.MumodeError):
        ctx.mm_op_prepare(np.zeros((4097, 4)), "fp64")                 # rows > 4096
    L = ctx.mm_op_prepare(np.eye(5), "fp64")
    T = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_expstep(T, [L, None], 1)                            # n_1 = 4 != 5
    assert e.value.status == 2
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_apply(torch.zeros((3, 5), dtype=torch.float64, device="cuda"), T, L, 3)   # mu > d
    assert e.value.status == 2
