"""GPU parity of the HIP mu-mode kernels against the FP64 oracle.

Every case calls the library through the C ABI (Python ctypes binding) and
compares element-wise (relative L2) with the oracle run on the identically
cast input.  Shapes span several workgroup tiles with ragged tails and
exercise the three load paths of the kernel (contiguous fibres, strided
fibres, generic gather)."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, empty_gpu, from_gpu, note, rel, to_gpu
from oracle import mumode as om
from oracle import operators as op
from oracle import schemes as sc

pytestmark = pytest.mark.gpu

PRECS = ["fp64", "fp32", "bf16x3", "fp16x2", "bf16"]


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


# dims chosen so that: mu=1 is the contiguous-fibre path, mu>=2 the strided
# path (P % 4 == 0); the second set forces the generic gather everywhere.
SHAPES = [(48, 40, 36), (37, 30, 21)]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("cplx", [True, False])
@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("mu", [1, 2, 3])
def test_apply_rectangular(ctx, prec, cplx, dims, mu):
    note(f"apply prec={prec} cplx={cplx} dims={dims} mu={mu}")
    g = synth.rng(1001, mu)
    U = cast(synth.random_tensor(dims, cplx, g), prec, cplx)
    m = dims[mu - 1] + 5                       # rectangular, non-symmetric
    L = synth.random_matrix(m, dims[mu - 1], cplx, g)
    ref = om.mode_product(U, L, mu)
    Lop = ctx.mm_op_prepare(L, prec)
    out_dims = list(dims)
    out_dims[mu - 1] = m
    out = empty_gpu(out_dims, prec, cplx)
    ctx.mumode_apply(out, to_gpu(U, prec, cplx), Lop, mu)
    err = rel(from_gpu(out), ref)
    note(f"  rel err {err:.3e}")
    assert err < REL_TOL[prec]
    Lop.destroy()


PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x2": 3, "bf16": 4}


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", [(48, 40, 36), (37, 30, 21), (64, 6, 10)])
@pytest.mark.parametrize("mu", [1, 2, 3])
def test_apply_real_operator_on_complex_state(ctx, prec, dims, mu):
    # a real (rectangular, non-symmetric) operator on a complex state runs
    # the real kernels on the (re, im) planes as two real fibres per complex
    # one: mode 1 with n_1 % 8 == 0 through the paired-fibre load, the other
    # modes through the strided load (2P % 4 == 0) or the gather
    note(f"real op on complex prec={prec} dims={dims} mu={mu}")
    g = synth.rng(1002, mu)
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    m = dims[mu - 1] + 3
    L = synth.random_matrix(m, dims[mu - 1], False, g)
    ref = om.mode_product(U, L, mu)
    Lop = ctx.mm_op_prepare(L, prec)
    out_dims = list(dims)
    out_dims[mu - 1] = m
    out = empty_gpu(out_dims, prec, True)
    ctx.mm_profile_begin()
    ctx.mumode_apply(out, to_gpu(U, prec, True), Lop, mu)
    rec = ctx.mm_profile_end()
    err = rel(from_gpu(out), ref)
    Lop.destroy()
    note(f"  rel err {err:.3e}, kernels {[k for k, _ in rec]}")
    assert err < REL_TOL[prec]
    # one launch of the real kernel (complex digit 0); mode 1 with whole
    # 8-row runs uses the paired-fibre load (load digit 3)
    assert len(rec) == 1 and (rec[0][0] // 100) % 10 == 0 and rec[0][0] // 1000 == PREC_CODE[prec]
    P2 = 2 * int(np.prod(dims[:mu - 1]))
    want = 3 if (P2 == 2 and dims[0] % 8 == 0) else (1 if P2 % 4 == 0 else 2)
    assert (rec[0][0] // 10) % 10 == want


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_expstep_real_operators_on_complex_state(ctx, prec):
    # in place over all modes, twice (the FP16x2 bound follows the chain)
    dims = (64, 40, 24)
    g = synth.rng(1007, 0)
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    E = [synth.random_matrix(n, n, False, g) for n in dims]
    ref = om.expstep(U, E, 2)
    ops = [ctx.mm_op_prepare(e, prec) for e in E]
    T = to_gpu(U, prec, True)
    ctx.mumode_expstep(T, ops, 2)
    err = rel(from_gpu(T), ref)
    note(f"expstep real ops on complex prec={prec} rel err {err:.3e}")
    assert err < 2 * REL_TOL[prec]
    for o in ops:
        o.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_hermite_transform_real_on_complex_128(ctx, prec):
    # the forward / backward Hermite transforms of Section 3 (real Phi, Psi)
    # on a complex state, n = 128 per mode: spec = psi x_1 Phi x_2 Phi x_3 Phi
    # and back
    import paper_2103_01691_amd as mm
    m = 128
    Phi, Psi = op.hermite_forward(m), op.hermite_backward(m)
    c = synth.hermite_coefficients(m, 16, 3, cfg_id=3)
    psi0 = cast(om.tucker(c, [Psi] * 3), prec, True)
    Fl, Bl = mm.hermite_matrices(m)
    F, B = ctx.mm_op_prepare(Fl, prec), ctx.mm_op_prepare(Bl, prec)
    spec = empty_gpu((m, m, m), prec, True)
    back = empty_gpu((m, m, m), prec, True)
    ctx.mm_profile_begin()
    ctx.mumode_transform(spec, to_gpu(psi0, prec, True), [F] * 3)
    ctx.mumode_transform(back, spec, [B] * 3)
    rec = ctx.mm_profile_end()
    ref_spec = om.tucker(psi0, [Phi] * 3)
    e1 = rel(from_gpu(spec), ref_spec)
    e2 = rel(from_gpu(back), om.tucker(ref_spec, [Psi] * 3))
    note(f"hermite transform 128 {prec}: forward {e1:.3e}, back {e2:.3e}")
    assert e1 < REL_TOL[prec] and e2 < 2 * REL_TOL[prec]
    assert len(rec) == 6 and all((k // 100) % 10 == 0 for k, _ in rec)
    F.destroy()
    B.destroy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_apply_large_fibres_and_rows(ctx, prec):
    # 256-long complex mode (the main workload's operator size), many tiles
    dims = (256, 24, 20)
    g = synth.rng(1003, 0)
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    for mu, perm in ((1, None), (2, None)):
        n = dims[mu - 1]
        L = synth.random_matrix(n, n, True, g)
        ref = om.mode_product(U, L, mu)
        Lop = ctx.mm_op_prepare(L, prec)
        out = empty_gpu(dims, prec, True)
        ctx.mumode_apply(out, to_gpu(U, prec, True), Lop, mu)
        err = rel(from_gpu(out), ref)
        note(f"large prec={prec} mu={mu} rel err {err:.3e}")
        assert err < REL_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
@pytest.mark.parametrize("cplx", [True, False])
def test_expstep_in_place(ctx, prec, cplx):
    dims = (32, 48, 24)
    g = synth.rng(1004, int(cplx))
    U = cast(synth.random_tensor(dims, cplx, g), prec, cplx)
    E = [synth.random_matrix(n, n, cplx, g) for n in dims]
    ref = om.expstep(U, E, 2)
    ops = [ctx.mm_op_prepare(e, prec) for e in E]
    T = to_gpu(U, prec, cplx)
    ctx.mumode_expstep(T, ops, 2)
    err = rel(from_gpu(T), ref)
    note(f"expstep prec={prec} cplx={cplx} rel err {err:.3e}")
    assert err < REL_TOL[prec]


def test_expstep_identity_modes(ctx):
    dims = (16, 20, 12)
    g = synth.rng(1005, 0)
    U = synth.random_tensor(dims, True, g)
    E2 = synth.random_matrix(20, 20, True, g)
    op2 = ctx.mm_op_prepare(E2, "fp64")
    T = to_gpu(U, "fp64", True)
    ctx.mumode_expstep(T, [None, op2, None], 1)
    assert rel(from_gpu(T), om.mode_product(U, E2, 2)) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "fp16x2"])
def test_transform_rectangular(ctx, prec):
    dims = (40, 28, 20)
    outd = (24, 36, 20)
    g = synth.rng(1006, 0)
    U = cast(synth.random_tensor(dims, True, g), prec, True)
    Phi = [synth.random_matrix(outd[k], dims[k], False, g) for k in range(2)] + [None]
    ref = om.tucker(U, Phi)
    ops = [ctx.mm_op_prepare(p, prec) if p is not None else None for p in Phi]
    out = empty_gpu(outd, prec, True)
    ctx.mumode_transform(out, to_gpu(U, prec, True), ops)
    assert rel(from_gpu(out), ref) < REL_TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
@pytest.mark.parametrize("tau", [1e-3, 0.1])
@pytest.mark.parametrize("nsteps", [1, 3])
def test_gpe_strang_small(ctx, prec, tau, nsteps):
    n, a, b, beta = 40, -8.0, 8.0, 100.0
    import paper_2103_01691_amd as mm
    psi0 = cast(synth.thomas_fermi_initial(n, a, b, 3, beta, cfg_id=4), prec, True)
    Eo = op.ho_exponential(n, a, b, tau)
    ref = sc.gpe_strang(psi0, [Eo] * 3, tau, beta, nsteps)
    # the library forms its own operator (host FP64 expm of its own FD Hamiltonian)
    El = mm.schrodinger_fd_exponential(n, a, b, 1.0, tau)
    Eop = ctx.mm_op_prepare(El, prec)
    psi = to_gpu(psi0, prec, True)
    ctx.gpe_strang_step(psi, [Eop] * 3, tau, beta, nsteps)
    err = rel(from_gpu(psi), ref)
    note(f"gpe small prec={prec} tau={tau} nsteps={nsteps} rel err {err:.3e}")
    assert err < REL_TOL[prec] * nsteps


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_norm2(ctx, prec):
    g = synth.rng(1007, 0)
    U = cast(synth.random_tensor((33, 17, 9), True, g), prec, True)
    v = ctx.mm_norm2(to_gpu(U, prec, True), 0.25)
    ref = 0.25 * np.sum(np.abs(U) ** 2)
    assert abs(v - ref) / ref < 1e-12


def test_errors_are_reported(ctx):
    import torch
    import paper_2103_01691_amd as mm
    L = ctx.mm_op_prepare(np.eye(8), "fp64")
    T = torch.zeros((4, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_apply(T, T, L, 1)                  # aliasing
    assert e.value.status == 1
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_apply(torch.zeros((8, 4), dtype=torch.float64, device="cuda"), T, L, 2)  # cols != n_2
    assert e.value.status == 2
    T32 = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_apply(torch.zeros_like(T32), T32, L, 1)   # fp64 op on fp32 tensor
    assert e.value.status == 3
    Lc = ctx.mm_op_prepare(np.eye(8) * (1 + 1j), "fp64")
    with pytest.raises(mm.MumodeError) as e:
        ctx.mumode_apply(torch.zeros_like(T), T, Lc, 1)      # complex op on real tensor
    assert e.value.status == 3


def test_deterministic(ctx):
    dims = (64, 32, 16)
    g = synth.rng(1008, 0)
    U = synth.random_tensor(dims, True, g)
    E = [synth.random_matrix(n, n, True, g) for n in dims]
    ops = [ctx.mm_op_prepare(e, "bf16x3") for e in E]
    a = to_gpu(U, "bf16x3", True)
    b = a.clone()
    ctx.mumode_expstep(a, ops, 1)
    ctx.mumode_expstep(b, ops, 1)
    import torch
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("scale", [1e-9, 1e7])
def test_fp16x2_state_range(ctx, scale):
    # half precision spans 2^-24 .. 65504: the state is rescaled by a power
    # of two from its largest component, so the relative error must not
    # depend on the magnitude
    dims = (64, 40, 24)
    g = synth.rng(1009, int(scale > 1))
    U = cast(synth.random_tensor(dims, True, g) * scale, "fp16x2", True)
    E = [synth.random_matrix(n, n, True, g) for n in dims]
    ref = om.expstep(U, E, 1)
    ops = [ctx.mm_op_prepare(e, "fp16x2") for e in E]
    T = to_gpu(U, "fp16x2", True)
    ctx.mumode_expstep(T, ops, 1)
    err = rel(from_gpu(T), ref)
    note(f"fp16x2 state scale {scale:g} rel err {err:.3e}")
    assert err < REL_TOL["fp16x2"]


@pytest.mark.parametrize("scale", [1e-6, 1e4])
def test_fp16x2_operator_range(ctx, scale):
    dims = (48, 40, 36)
    g = synth.rng(1010, int(scale > 1))
    U = cast(synth.random_tensor(dims, False, g), "fp16x2", False)
    L = synth.random_matrix(40, 40, False, g) * scale
    ref = om.mode_product(U, L, 2)
    out = empty_gpu(dims, "fp16x2", False)
    ctx.mumode_apply(out, to_gpu(U, "fp16x2", False), ctx.mm_op_prepare(L, "fp16x2"), 2)
    err = rel(from_gpu(out), ref)
    note(f"fp16x2 operator scale {scale:g} rel err {err:.3e}")
    assert err < REL_TOL["fp16x2"]


@pytest.mark.parametrize("growth", [40.0, 1.0 / 40.0])
def test_fp16x2_bound_follows_chain(ctx, growth):
    # every product scales the state by ~growth: over 3 steps x 3 modes the
    # magnitude moves by growth^9 (~2.6e14 or its inverse), far outside half
    # precision, so each launch must pass the bound of its output on
    dims = (32, 48, 24)
    g = synth.rng(1011, int(growth > 1))
    U = cast(synth.random_tensor(dims, True, g), "fp16x2", True)
    E = [synth.random_matrix(n, n, True, g) * growth for n in dims]
    ref = om.expstep(U, E, 3)
    ops = [ctx.mm_op_prepare(e, "fp16x2") for e in E]
    T = to_gpu(U, "fp16x2", True)
    ctx.mumode_expstep(T, ops, 3)
    err = rel(from_gpu(T), ref)
    note(f"fp16x2 chain growth {growth:g} rel err {err:.3e}")
    assert err < 3 * REL_TOL["fp16x2"]


def test_fp16x2_state_changed_between_calls(ctx):
    # a new call re-derives the bound from the data, so writes by the caller
    # between calls are seen
    import torch
    dims = (32, 32, 16)
    g = synth.rng(1012, 0)
    U = synth.random_tensor(dims, True, g)
    E = [synth.random_matrix(n, n, True, g) for n in dims]
    ops = [ctx.mm_op_prepare(e, "fp16x2") for e in E]
    T = to_gpu(cast(U, "fp16x2", True), "fp16x2", True)
    ctx.mumode_expstep(T, ops, 1)
    with torch.no_grad():
        T.mul_(3.0e5)
    mid = from_gpu(T)
    ctx.mumode_expstep(T, ops, 1)
    err = rel(from_gpu(T), om.expstep(mid, E, 1))
    note(f"fp16x2 rescaled between calls rel err {err:.3e}")
    assert err < REL_TOL["fp16x2"]


def test_fp16x2_chain_across_calls(ctx):
    # MM_OPT_FP16X2_CHAIN: consecutive GPE calls on one tensor continue the
    # running bound the previous call's last product wrote (the exact maximum
    # of its output), so the results equal those of calls that each start
    # with a max-abs pass, bit for bit; a call on another tensor starts a
    # chain of its own
    import paper_2103_01691_amd as mm
    n, a, b, beta, tau = 48, -8.0, 8.0, 100.0, 1e-3
    psi0 = cast(synth.thomas_fermi_initial(n, a, b, 3, beta, cfg_id=4), "fp16x2", True)
    E = ctx.mm_op_prepare(mm.schrodinger_fd_exponential(n, a, b, 1.0, tau), "fp16x2")
    other0 = cast(synth.wavepacket_initial(n, -10.0, 10.0, 3, cfg_id=2), "fp16x2", True)
    runs = {}
    for chain in (0, 1):
        ctx.mm_set_option(mm.MM_OPT_FP16X2_CHAIN, chain)
        psi = to_gpu(psi0, "fp16x2", True)
        other = to_gpu(other0, "fp16x2", True)
        for it in range(4):
            ctx.gpe_strang_step(psi, [E] * 3, tau, beta, 1)
            if it == 1:
                ctx.gpe_strang_step(other, [E] * 3, tau, beta, 1)
        runs[chain] = (from_gpu(psi), from_gpu(other))
    ctx.mm_set_option(mm.MM_OPT_FP16X2_CHAIN, 0)
    E.destroy()
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    Eo = op.ho_exponential(n, a, b, tau)
    assert rel(runs[1][0], sc.gpe_strang(psi0, [Eo] * 3, tau, beta, 4)) < 4 * REL_TOL["fp16x2"]
    assert rel(runs[1][1], sc.gpe_strang(other0, [Eo] * 3, tau, beta, 1)) < REL_TOL["fp16x2"]
