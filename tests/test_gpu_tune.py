"""GPU tests of the autotuner, the tune cache and the caller-owned workspace.

Every tile class of the split kernels is forced in turn through a tune file
and checked against the FP64 oracle, so each class the autotuner may pick is
parity-tested."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, empty_gpu, from_gpu, note, rel, to_gpu
from oracle import mumode as om

pytestmark = pytest.mark.gpu

DIMS = (256, 48, 40)          # mode 1: contiguous fibres, 512 real rows; modes 2, 3: strided
PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x2": 3, "bf16": 4}


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


def _keys(prec, dims, cplx=True):
    c = 2 if cplx else 1
    keys = []
    for k, n in enumerate(dims):
        P = int(np.prod(dims[:k]))
        F = int(np.prod(dims)) // n
        load = 0 if (P == 1 and (c * n) % 8 == 0) else (1 if P % 4 == 0 else 2)
        keys.append((PREC_CODE[prec], int(cplx), load, c * n, c * n, F))
    return keys


def _problem(prec):
    g = synth.rng(1101, PREC_CODE[prec])
    U = cast(synth.random_tensor(DIMS, True, g), prec, True)
    E = [synth.random_matrix(n, n, True, g) for n in DIMS]
    return U, E


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x2"])
@pytest.mark.parametrize("cls", list(range(11)))
def test_every_split_class_matches_oracle(ctx, tmp_path, prec, cls):
    U, E = _problem(prec)
    f = tmp_path / "t.txt"
    f.write_text("mumode-tune 1\n" + "".join(" ".join(map(str, k)) + f" {cls} 0.0\n" for k in _keys(prec, DIMS)))
    ctx.mm_tune_clear()
    ctx.mm_tune_load(f)
    ops = [ctx.mm_op_prepare(e, prec) for e in E]
    T = to_gpu(U, prec, True)
    ctx.mumode_expstep(T, ops, 1)
    err = rel(from_gpu(T), om.expstep(U, E, 1))
    ctx.mm_tune_clear()
    note(f"forced class {cls} {prec} rel err {err:.3e}")
    assert err < REL_TOL[prec]


@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("cls", [0, 1, 2, 3])
def test_every_fp64_class_matches_oracle(ctx, tmp_path, cplx, cls):
    # FP64 classes, including the one-wave class 3 that the device
    # exponential uses for its few-fibre matrix products (rows split over
    # workgroups, so every product here runs out of place)
    g = synth.rng(1103, int(cplx) * 10 + cls)
    U = synth.random_tensor(DIMS, cplx, g)
    E = [synth.random_matrix(n, n, cplx, g) for n in DIMS]
    f = tmp_path / "t.txt"
    f.write_text("mumode-tune 1\n" + "".join(" ".join(map(str, k)) + f" {cls} 0.0\n"
                                             for k in _keys("fp64", DIMS, cplx)))
    ctx.mm_tune_clear()
    ctx.mm_tune_load(f)
    ops = [ctx.mm_op_prepare(e, "fp64") for e in E]
    T = to_gpu(U, "fp64", cplx)
    ctx.mumode_expstep(T, ops, 1)
    err = rel(from_gpu(T), om.expstep(U, E, 1))
    ctx.mm_tune_clear()
    note(f"forced FP64 class {cls} complex={cplx}: rel err {err:.3e}")
    assert err < REL_TOL["fp64"]


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x2"])
@pytest.mark.parametrize("cls", [8, 9])
@pytest.mark.parametrize("dims", [(200, 136), (40, 48, 24), (8, 16)])
def test_three_product_classes_ragged(ctx, tmp_path, prec, cls, dims):
    # the three-product (Gauss) classes on fibre counts that leave a partial
    # fibre tile, row counts below / not a multiple of the 256-row tile, and
    # mode lengths that end inside an LDS chunk; each product once with the
    # fused phases (prologue on mode 1, epilogue on the last mode) through
    # one GPE step, once without through an expstep
    from oracle import schemes as sc
    g = synth.rng(1102, PREC_CODE[prec] * 10 + cls)
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    E = [synth.random_matrix(n, n, True, g) for n in dims]
    f = tmp_path / "t.txt"
    f.write_text("mumode-tune 1\n" + "".join(" ".join(map(str, k)) + f" {cls} 0.0\n" for k in _keys(prec, dims)))
    ctx.mm_tune_clear()
    ctx.mm_tune_load(f)
    ops = [ctx.mm_op_prepare(e, prec) for e in E]
    T = to_gpu(U, prec, True)
    ctx.mumode_expstep(T, ops, 1)
    err = rel(from_gpu(T), om.expstep(U, E, 1))
    T = to_gpu(U, prec, True)
    ctx.mm_profile_begin()
    ctx.gpe_strang_step(T, ops, 0.01, 3.0, 1)
    kinds = [k for k, _ in ctx.mm_profile_end()]
    err_ph = rel(from_gpu(T), sc.gpe_strang(U, E, 0.01, 3.0, 1))
    ctx.mm_tune_clear()
    note(f"three-product class {cls} {prec} dims {dims}: rel err {err:.3e}, with phases {err_ph:.3e}, kinds {kinds}")
    assert err < REL_TOL[prec]
    assert err_ph < REL_TOL[prec]
    # first product with the prologue phase, last with the epilogue
    assert kinds[0] % 10 == 2 and kinds[-1] % 10 == 1


@pytest.mark.parametrize("prec", ["fp32", "fp16x2"])
def test_autotune_records_and_round_trips(ctx, tmp_path, prec):
    U, E = _problem(prec)
    ops = [ctx.mm_op_prepare(e, prec) for e in E]
    T = to_gpu(U, prec, True)
    ctx.mm_tune_clear()
    ctx.mm_autotune(T, ops, 300)
    assert rel(from_gpu(T), U) == 0.0                      # the tuner does not touch T
    ent = ctx.mm_tune_entries()
    note(f"autotune {prec}: {[(k, c, round(us, 1)) for k, c, us in ent]}")
    # complex products with complex operators also get a key with the
    # prologue phase (load path + 8)
    want = _keys(prec, DIMS) + [(k[0], k[1], k[2] + 8) + k[3:] for k in _keys(prec, DIMS)]
    assert sorted(k for k, _, _ in ent) == sorted(want)
    assert all(0 <= c < 11 and us > 0 for _, c, us in ent)
    ctx.mumode_expstep(T, ops, 1)                          # runs with the tuned classes
    assert rel(from_gpu(T), om.expstep(U, E, 1)) < REL_TOL[prec]
    f = tmp_path / "tune.txt"
    ctx.mm_tune_save(f)
    ctx.mm_tune_clear()
    assert ctx.mm_tune_entries() == []
    ctx.mm_tune_load(f)
    back = ctx.mm_tune_entries()
    assert [(k, c) for k, c, _ in back] == [(k, c) for k, c, _ in ent]
    ctx.mm_tune_clear()


def test_tune_load_rejects_malformed(ctx, tmp_path):
    import paper_2103_01691_amd as mm
    ctx.mm_tune_clear()
    f = tmp_path / "bad.txt"
    f.write_text("mumode-tune 1\n2 1 0 512 512\n")
    with pytest.raises(mm.MumodeError) as e:
        ctx.mm_tune_load(f)
    assert e.value.status == 1
    f.write_text("something else\n")
    with pytest.raises(mm.MumodeError):
        ctx.mm_tune_load(f)
    f.write_text("mumode-tune 1\n2 1 0 512 512 100 99 1.0\n")   # class out of range
    with pytest.raises(mm.MumodeError):
        ctx.mm_tune_load(f)
    assert ctx.mm_tune_entries() == []


def test_caller_workspace(ctx):
    import torch
    import paper_2103_01691_amd as mm
    dims, outd = (40, 28, 20), (24, 36, 20)
    g = synth.rng(1102, 0)
    U = synth.random_tensor(dims, True, g)
    Phi = [synth.random_matrix(outd[k], dims[k], False, g) for k in range(2)] + [None]
    ops = [ctx.mm_op_prepare(p, "fp64") if p is not None else None for p in Phi]
    need = 2 * 16 * max(24 * 28 * 20, 24 * 36 * 20)
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    ctx.mm_set_workspace(small)
    out = empty_gpu(outd, "fp64", True)
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_transform(out, to_gpu(U, "fp64", True), ops)
    assert e.value.status == 5          # MM_ERR_NOMEM
    big = torch.empty(need + 4096, dtype=torch.uint8, device="cuda")
    ctx.mm_set_workspace(big)
    ctx.mumode_transform(out, to_gpu(U, "fp64", True), ops)
    assert rel(from_gpu(out), om.tucker(U, Phi)) < 1e-12
    ctx.mm_set_workspace(None)
    ctx.mumode_transform(out, to_gpu(U, "fp64", True), ops)
    assert rel(from_gpu(out), om.tucker(U, Phi)) < 1e-12
    del small, big


def test_tune_cache_path_persists_across_contexts(tmp_path):
    # mm_create's tune cache: read at creation when present, written by every
    # autotuner run; a malformed file refuses the context
    import paper_2103_01691_amd as mm
    path = tmp_path / "cache.txt"
    U, E = _problem("fp32")
    with mm.Context(0, tune_cache_path=path) as c1:
        assert c1.mm_tune_entries() == []
        ops = [c1.mm_op_prepare(e, "fp32") for e in E]
        c1.mm_autotune(to_gpu(U, "fp32", True), ops, 100)
        ent = [(k, c) for k, c, _ in c1.mm_tune_entries()]
    assert path.exists() and len(ent) == 2 * len(DIMS)   # plain and prologue-phase keys
    with mm.Context(0, tune_cache_path=path) as c2:
        assert [(k, c) for k, c, _ in c2.mm_tune_entries()] == ent
    bad = tmp_path / "bad.txt"
    bad.write_text("not a tune file\n")
    with pytest.raises(mm.MumodeError) as e:
        mm.Context(0, tune_cache_path=bad)
    assert e.value.status == 1


@pytest.mark.parametrize("cls", [8, 9])
@pytest.mark.parametrize("state,op,growth", [(1e-9, 1.0, 1.0), (1e7, 1.0, 1.0), (1.0, 1e-6, 1.0), (1.0, 1e4, 1.0),
                                             (1.0, 1.0, 40.0), (1.0, 1.0, 1.0 / 40.0)])
def test_three_product_fp16x2_range(ctx, tmp_path, cls, state, op, growth):
    # the three-product FP16x2 form keeps one more bit of headroom for x + y
    # and Re L + Im L: its error must not depend on the magnitudes of the
    # state or the operator, nor on a bound that moves by growth^9 over a
    # chain of nine products
    dims = (64, 40, 24)
    g = synth.rng(1104, cls)
    U = cast(synth.random_tensor(dims, True, g) * state, "fp16x2", True)
    E = [synth.random_matrix(n, n, True, g) * op * growth for n in dims]
    steps = 3 if growth != 1.0 else 1
    ref = om.expstep(U, E, steps)
    f = tmp_path / "t.txt"
    f.write_text("mumode-tune 1\n" + "".join(" ".join(map(str, k)) + f" {cls} 0.0\n" for k in _keys("fp16x2", dims)))
    ctx.mm_tune_clear()
    ctx.mm_tune_load(f)
    ops = [ctx.mm_op_prepare(e, "fp16x2") for e in E]
    T = to_gpu(U, "fp16x2", True)
    ctx.mumode_expstep(T, ops, steps)
    err = rel(from_gpu(T), ref)
    ctx.mm_tune_clear()
    note(f"three-product class {cls} state x{state:g} operator x{op:g} growth {growth:g}: rel err {err:.3e}")
    assert err < steps * REL_TOL["fp16x2"]


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x2"])
@pytest.mark.parametrize("cls", [8, 9])
@pytest.mark.parametrize("mu,m", [(1, 40), (2, 72), (3, 24)])
def test_three_product_rectangular_apply(ctx, tmp_path, prec, cls, mu, m):
    # a rectangular complex operator (m x n_mu, m != n_mu) through
    # mumode_apply on the three-product kernels: rows and columns of the
    # prepared Re L, Im L, Re L + Im L blocks differ
    dims = (48, 56, 32)
    g = synth.rng(1105, mu * 10 + cls)
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    n = dims[mu - 1]
    L = synth.random_matrix(m, n, True, g)
    ref = om.mode_product(U, L, mu)
    P = int(np.prod(dims[:mu - 1]))
    F = int(np.prod(dims)) // n
    load = 0 if P == 1 else 1
    f = tmp_path / "t.txt"
    f.write_text(f"mumode-tune 1\n{PREC_CODE[prec]} 1 {load} {2 * m} {2 * n} {F} {cls} 0.0\n")
    ctx.mm_tune_clear()
    ctx.mm_tune_load(f)
    odims = list(dims)
    odims[mu - 1] = m
    out = empty_gpu(odims, prec, True)
    Lop = ctx.mm_op_prepare(L, prec)
    ctx.mm_profile_begin()
    ctx.mumode_apply(out, to_gpu(U, prec, True), Lop, mu)
    rec = ctx.mm_profile_end()
    got = from_gpu(out)
    ctx.mm_tune_clear()
    # the four-product kernel of the built-in choice rounds differently: the
    # forced class really ran
    ctx.mumode_apply(out, to_gpu(U, prec, True), Lop, mu)
    assert not np.array_equal(got, from_gpu(out))
    err = rel(got, ref)
    note(f"three-product class {cls} {prec} mode {mu} {m}x{n}: rel err {err:.3e}")
    assert len(rec) == 1
    assert err < REL_TOL[prec]
