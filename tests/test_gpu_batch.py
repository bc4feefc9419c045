"""GPU parity of the batched integrator (many independent instances of
uneven order, sizes and dtype in one captured graph per step)."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, from_gpu, note, rel, to_gpu
from oracle import mumode as om
from oracle import operators as op

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


def _lib_exponential(mm, kind, n, tau):
    if kind == "heat":
        return mm.expm(mm.fd2_matrix(n, 0.0, 1.0), tau).real.copy()
    return mm.schrodinger_fd_exponential(n, -10.0, 10.0, 0.0, tau)


def _oracle_exponential(kind, n, tau):
    if kind == "heat":
        return op.heat_exponential(n, 0.0, 1.0, "dirichlet", tau)
    return op.free_schrodinger_exponential(n, -10.0, 10.0, tau)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batched_expstep_matches_oracle(ctx, prec):
    import paper_2103_01691_amd as mm
    mix = synth.batch_mix(24, cfg_id=5, sizes=(32, 48, 64))
    tensors, ops, refs = [], [], []
    opcache = {}
    for inst in mix:
        cplx = inst["kind"] == "schrodinger"
        g = synth.rng(5, 1000 + inst["index"])
        U = cast(synth.random_tensor(inst["dims"], cplx, g), prec, cplx)
        Eo = [_oracle_exponential(inst["kind"], n, inst["tau"]) for n in inst["dims"]]
        refs.append(om.expstep(U, Eo, 2))
        ol = []
        for n in inst["dims"]:
            key = (inst["kind"], n, inst["tau"])
            if key not in opcache:
                opcache[key] = ctx.mm_op_prepare(_lib_exponential(mm, inst["kind"], n, inst["tau"]), prec)
            ol.append(opcache[key])
        ops.append(ol)
        tensors.append(to_gpu(U, prec, cplx))
    ctx.mumode_expstep_batched(tensors, ops, 1)       # captures the graph, one replay
    ctx.mumode_expstep_batched(tensors, ops, 1)       # replays the cached graph
    worst = 0.0
    for inst, t, ref in zip(mix, tensors, refs):
        err = rel(from_gpu(t), ref)
        worst = max(worst, err)
        assert err < 2 * REL_TOL[prec], (inst, err)
    note(f"batch prec={prec} instances={len(mix)} worst rel err {worst:.3e}")


def test_batched_rejects_unsupported(ctx):
    import torch
    import paper_2103_01691_amd as mm
    L = ctx.mm_op_prepare(np.eye(6), "fp32")
    t = torch.zeros((5, 6), dtype=torch.float32, device="cuda")   # P = 6 on mode 2 is not 4-aligned
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_expstep_batched([t], [[L, None]], 1)
    assert e.value.status in (2, 7)


def test_batched_rejects_fp16x2(ctx):
    import torch
    import paper_2103_01691_amd as mm
    L = ctx.mm_op_prepare(np.eye(8), "fp16x2")
    t = torch.zeros((8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_expstep_batched([t], [[L, L]], 1)
    assert e.value.status == 7


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batch_autotuner_then_parity(ctx, prec):
    # the batch autotuner times whole batched steps per (mode, real/complex)
    # tile class; the step with the chosen classes must still match the oracle
    import paper_2103_01691_amd as mm
    mix = synth.batch_mix(40, cfg_id=5, sizes=(32, 48, 64, 96))
    tensors, ops, inputs, refs = [], [], [], []
    opcache = {}
    for inst in mix:
        cplx = inst["kind"] == "schrodinger"
        g = synth.rng(5, 2000 + inst["index"])
        U = cast(synth.random_tensor(inst["dims"], cplx, g), prec, cplx)
        Eo = [_oracle_exponential(inst["kind"], n, inst["tau"]) for n in inst["dims"]]
        refs.append(om.expstep(U, Eo, 1))
        inputs.append((U, cplx))
        ol = []
        for n in inst["dims"]:
            key = (inst["kind"], n, inst["tau"])
            if key not in opcache:
                opcache[key] = ctx.mm_op_prepare(_lib_exponential(mm, inst["kind"], n, inst["tau"]), prec)
            ol.append(opcache[key])
        ops.append(ol)
        tensors.append(to_gpu(U, prec, cplx))
    chosen = ctx.mm_autotune_batched(tensors, ops, 20)
    note(f"batch autotuner {prec}: {chosen}")
    assert all(0 <= c <= 2 for c in chosen.values())
    for t, (U, cplx) in zip(tensors, inputs):
        t.copy_(to_gpu(U, prec, cplx))
    ctx.mumode_expstep_batched(tensors, ops, 1)
    for inst, t, ref in zip(mix, tensors, refs):
        assert rel(from_gpu(t), ref) < REL_TOL[prec], inst
    ctx.mm_tune_clear()
