"""Full-size parity of the five synthetic workloads, in the launch
configuration the benchmark uses, against the FP64 oracle.

  gpe     3-D GPE Strang step, n = 256 on [-8, 8]^3, beta = 100, split BF16x3
  free    3-D free Schroedinger step, n = 256 on [-10, 10]^3, FP64 / FP32 / BF16x3
  ho      3-D harmonic oscillator, Hermite n = 128, eps = 0.1, tau = 0.02, complex64
  heat    2-D heat, n = 64 on [0, 1]^2, tau = 1e-3, 20 steps, FP64
  batch   512 instances (d in {2,3}, n_mu in {32..192}, heat / Schroedinger),
          one step each; every instance compared with the oracle
"""
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


def _lib_ho_exp(mm, n, a, b, tau):
    return mm.schrodinger_fd_exponential(n, a, b, 1.0, tau)


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x2"])
@pytest.mark.parametrize("tau", [1e-3, 0.1])
def test_gpe_256_split_one_step(ctx, tau, prec):
    import paper_2103_01691_amd as mm
    n, a, b, beta = 256, -8.0, 8.0, 100.0
    note(f"gpe 256 tau={tau} {prec}: building inputs")
    psi0 = cast(synth.thomas_fermi_initial(n, a, b, 3, beta, cfg_id=4), prec, True)
    Eop = ctx.mm_op_prepare(_lib_ho_exp(mm, n, a, b, tau), prec)
    psi = to_gpu(psi0, prec, True)
    ctx.gpe_strang_step(psi, [Eop] * 3, tau, beta, 1)
    got = from_gpu(psi)
    del psi
    note("gpe 256: oracle step")
    Eo = op.ho_exponential(n, a, b, tau)
    ref = sc.gpe_strang(psi0, [Eo] * 3, tau, beta, 1)
    err = rel(got, ref)
    note(f"gpe 256 tau={tau} split {prec} one step rel L2 {err:.3e}")
    assert err < REL_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_free_schrodinger_256_one_step(ctx, prec):
    import paper_2103_01691_amd as mm
    n, a, b, tau = 256, -10.0, 10.0, 0.01
    psi0 = cast(synth.wavepacket_initial(n, a, b, 3, cfg_id=2), prec, True)
    E = mm.schrodinger_fd_exponential(n, a, b, 0.0, tau)
    Eop = ctx.mm_op_prepare(E, prec)
    psi = to_gpu(psi0, prec, True)
    ctx.mumode_expstep(psi, [Eop] * 3, 1)
    got = from_gpu(psi)
    del psi
    Eo = op.free_schrodinger_exponential(n, a, b, tau)
    ref = om.expstep(psi0, [Eo] * 3, 1)
    err = rel(got, ref)
    note(f"free 256 prec={prec} rel L2 {err:.3e}")
    assert err < REL_TOL[prec]


@pytest.mark.parametrize("prec", ["bf16x3", "fp16x2"])
def test_ho_hermite_128_one_step(ctx, prec):
    import paper_2103_01691_amd as mm
    m, kmax, tau, eps, t0 = 128, 16, 0.02, 0.1, 0.0
    Phi, Psi, X = op.hermite_forward(m), op.hermite_backward(m), op.hermite_nodes(m)
    c = synth.hermite_coefficients(m, kmax, 3, cfg_id=3)
    psi0 = cast(om.tucker(c, [Psi] * 3), prec, True)
    ref = sc.ho_strang(psi0, [Phi] * 3, [Psi] * 3, [X] * 3, t0, tau, eps, 2)
    Xl, _ = mm.hermite_nodes(m)
    Fl, Bl = mm.hermite_matrices(m)
    F, B = ctx.mm_op_prepare(Fl, prec), ctx.mm_op_prepare(Bl, prec)
    psi = to_gpu(psi0, prec, True)
    ctx.ho_strang_step(psi, [F] * 3, [B] * 3, [Xl] * 3, t0, tau, eps, 2)
    err = rel(from_gpu(psi), ref)
    note(f"ho 128 {prec} two steps rel L2 {err:.3e}")
    assert err < 2 * REL_TOL[prec]


def test_heat_2d_64_twenty_steps_fp64(ctx):
    import paper_2103_01691_amd as mm
    n, tau = 64, 1e-3
    u0 = synth.heat_initial(n, 2, cfg_id=1)
    E = mm.expm(mm.fd2_matrix(n, 0.0, 1.0), tau).real.copy()
    Eop = ctx.mm_op_prepare(E, "fp64")
    u = to_gpu(u0, "fp64", False)
    ctx.mumode_expstep(u, [Eop] * 2, 20)
    Eo = op.heat_exponential(n, 0.0, 1.0, "dirichlet", tau)
    ref = om.expstep(u0, [Eo] * 2, 20)
    err = rel(from_gpu(u), ref)
    note(f"heat 64^2 20 steps fp64 rel L2 {err:.3e}")
    assert err < REL_TOL["fp64"]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batch_512_all_instances(ctx, prec):
    # every one of the 512 instances is compared with the oracle; the inputs
    # are drawn again from their seeds after the run, so only one FP64 copy
    # is held at a time
    import paper_2103_01691_amd as mm
    mix = synth.batch_mix(512, cfg_id=5)
    tensors, ops = [], []
    cache = {}

    def lib_op(kind, n, tau):
        key = (kind, n, tau)
        if key not in cache:
            if kind == "heat":
                E = mm.expm(mm.fd2_matrix(n, 0.0, 1.0), tau).real.copy()
            else:
                E = mm.schrodinger_fd_exponential(n, -10.0, 10.0, 0.0, tau)
            cache[key] = ctx.mm_op_prepare(E, prec)
        return cache[key]

    def draw(inst):
        cplx = inst["kind"] == "schrodinger"
        g = synth.rng(5, 1000 + inst["index"])
        return cast(synth.random_tensor(inst["dims"], cplx, g), prec, cplx), cplx

    note(f"batch 512 {prec}: building inputs")
    for inst in mix:
        U, cplx = draw(inst)
        tensors.append(to_gpu(U, prec, cplx))
        ops.append([lib_op(inst["kind"], n, inst["tau"]) for n in inst["dims"]])
    note(f"batch 512 {prec}: one batched step")
    ctx.mumode_expstep_batched(tensors, ops, 1)
    note(f"batch 512 {prec}: oracle for every instance")
    worst = 0.0
    for inst in mix:
        U, _ = draw(inst)
        if inst["kind"] == "heat":
            Eo = [op.heat_exponential(n, 0.0, 1.0, "dirichlet", inst["tau"]) for n in inst["dims"]]
        else:
            Eo = [op.free_schrodinger_exponential(n, -10.0, 10.0, inst["tau"]) for n in inst["dims"]]
        err = rel(from_gpu(tensors[inst["index"]]), om.expstep(U, Eo, 1))
        worst = max(worst, err)
        assert err < REL_TOL[prec], (inst, err)
    note(f"batch 512 {prec}: worst rel err over all instances {worst:.3e}")
