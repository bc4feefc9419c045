"""GPU parity of the kernel instances the benchmark times.

The 3-D GPE Strang step at n = 256 runs every split tile class the
autotuner may choose (0, 3, 4, 5, 6, 7 and the three-product classes 8, 9;
classes 1 and 2 have no fused-phase instances; class 7 covers half the rows,
so its products run out of place)
with the nonlinear phase fused into the prologue of each step's
first product and the epilogue of the last, and with the full-tile epilogue
(every tile complete at n = 256).  Two steps, so that the prologue runs with
both coefficients (tau/2 on the first step, tau on the merged second) and
the final epilogue with tau/2.  Each class is forced through a tune file
whose keys are the three products' shapes."""
import numpy as np
import pytest

import synth
from gpu_util import REL_TOL, cast, from_gpu, note, rel, to_gpu
from oracle import operators as op
from oracle import schemes as sc

pytestmark = pytest.mark.gpu

N, A, B, BETA, TAU, STEPS = 256, -8.0, 8.0, 100.0, 1e-3, 2
PREC_CODE = {"fp64": 0, "fp32": 1, "bf16x3": 2, "fp16x2": 3, "bf16": 4}


@pytest.fixture(scope="module")
def ctx():
    import paper_2103_01691_amd as mm
    c = mm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def problem():
    # the two split precisions share the complex64 input, hence the oracle
    note("gpe 256 classes: oracle, two steps")
    psi0 = cast(synth.thomas_fermi_initial(N, A, B, 3, BETA, cfg_id=4), "fp16x2", True)
    Eo = op.ho_exponential(N, A, B, TAU)
    ref = sc.gpe_strang(psi0, [Eo] * 3, TAU, BETA, STEPS)
    return psi0, ref


def _tune_file(path, prec, cls):
    dims = (N, N, N)
    lines = []
    for k, n in enumerate(dims):
        P = int(np.prod(dims[:k]))
        F = int(np.prod(dims)) // n
        load = 0 if P == 1 else 1
        lines.append(f"{PREC_CODE[prec]} 1 {load} {2 * n} {2 * n} {F} {cls} 0.0\n")
    path.write_text("mumode-tune 1\n" + "".join(lines))


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x3"])
@pytest.mark.parametrize("cls", [0, 3, 4, 5, 6, 7, 8, 9, 10])
def test_gpe_256_every_phase_class(ctx, problem, tmp_path, prec, cls):
    import paper_2103_01691_amd as mm
    psi0, ref = problem
    f = tmp_path / "tune.txt"
    _tune_file(f, prec, cls)
    ctx.mm_tune_clear()
    ctx.mm_tune_load(f)
    Eop = ctx.mm_op_prepare(mm.schrodinger_fd_exponential(N, A, B, 1.0, TAU), prec)
    psi = to_gpu(psi0, prec, True)
    note(f"gpe 256 {prec} forced class {cls}: {STEPS} steps")
    ctx.mm_profile_begin()
    ctx.gpe_strang_step(psi, [Eop] * 3, TAU, BETA, STEPS)
    rec = ctx.mm_profile_end()
    got = from_gpu(psi)
    ctx.mm_tune_clear()
    Eop.destroy()
    del psi
    # kind code prec*1000 + complex*100 + load*10 + prologue*2 + epilogue:
    # the first product of each step carries the prologue phase, the last
    # product of the call the epilogue
    kinds = [k for k, _ in rec]
    p = PREC_CODE[prec] * 1000 + 100
    assert kinds == [p + 2, p + 10, p + 10, p + 2, p + 10, p + 11], kinds
    err = rel(got, ref)
    note(f"gpe 256 {prec} class {cls}: rel L2 {err:.3e}")
    assert err < STEPS * REL_TOL[prec]


@pytest.mark.parametrize("prec", ["fp16x2"])
@pytest.mark.parametrize("tau", [0.05, 0.1])
def test_magnus_fp16x2_hermite_256_large_steps(ctx, prec, tau):
    # the FP16x2 operator scale comes from a bound of the entries of the
    # per-step exponential; for this skew-Hermitian generator the bound is
    # 1, so the operator keeps its full split accuracy at large steps
    import paper_2103_01691_amd as mm
    from oracle import mumode as om
    m = 256
    c = synth.hermite_coefficients(m, 16, 3, cfg_id=3)
    psi0 = cast(om.tucker(c, [op.hermite_backward(m)] * 3), prec, True)
    Bo, do, gf = op.hkmp_problem(m)
    note(f"magnus m=256 tau={tau}: oracle step")
    ref = sc.magnus_midpoint(psi0, Bo, do, gf, tau, 1, t0=0.3)
    Phi, Psi = mm.hermite_matrices(m)
    X, _ = mm.hermite_nodes(m)
    Bm = Psi @ np.diag(-1j * (np.arange(m) + 0.5)) @ Phi
    g = np.zeros((1, 3), dtype=np.complex128)
    g[0, 2] = -1j * np.sin(0.3 + 0.5 * tau) ** 2
    psi = to_gpu(psi0, prec, True)
    ctx.mumode_magnus_step(psi, [Bm] * 3, [None, None, X], g, tau, 1, prec)
    err = rel(from_gpu(psi), ref)
    note(f"magnus m=256 tau={tau} {prec}: rel L2 {err:.3e}")
    assert err < REL_TOL[prec]


def test_batch_graph_rebuilt_after_operators_change(ctx):
    # a captured batch step holds prepared-operator addresses and tile codes:
    # destroying the operators and preparing others (here in another
    # precision, often at the same host address) must rebuild it
    import paper_2103_01691_amd as mm
    from oracle import mumode as om
    g = synth.rng(1301, 0)
    dims = [(32, 48, 40), (64, 32)]
    U = [cast(synth.random_tensor(d, True, g), "fp32", True) for d in dims]
    E = [[synth.random_matrix(n, n, True, g) for n in d] for d in dims]
    tensors = [to_gpu(u, "fp32", True) for u in U]
    for prec in ("fp32", "bf16x3", "fp32"):
        ops = [[ctx.mm_op_prepare(e, prec) for e in el] for el in E]
        for t, u in zip(tensors, U):
            t.copy_(to_gpu(u, "fp32", True))
        ctx.mumode_expstep_batched(tensors, ops, 1)
        for t, u, el in zip(tensors, U, E):
            err = rel(from_gpu(t), om.expstep(u, el, 1))
            note(f"batch rebuilt {prec}: rel err {err:.3e}")
            assert err < REL_TOL[prec]
        for ol in ops:
            for o in ol:
                o.destroy()
    # a tune change also rebuilds the graph (same operators, other tiles)
    ops = [[ctx.mm_op_prepare(e, "fp32") for e in el] for el in E]
    ctx.mumode_expstep_batched(tensors, ops, 1)
    ctx.mm_autotune(tensors[0], ops[0], 50)
    for t, u in zip(tensors, U):
        t.copy_(to_gpu(u, "fp32", True))
    ctx.mumode_expstep_batched(tensors, ops, 1)
    for t, u, el in zip(tensors, U, E):
        assert rel(from_gpu(t), om.expstep(u, el, 1)) < REL_TOL["fp32"]
    ctx.mm_tune_clear()


def test_ho_step_reforms_propagator_when_tau_or_nodes_change(ctx):
    # the collapsed propagator is cached per (operators, tau, precision) and
    # the node squares per node values: changing tau, then the nodes'
    # operators and nodes (another m), must give the oracle's result each time
    import paper_2103_01691_amd as mm
    from oracle import mumode as om
    t0, eps = 0.2, 0.1
    for m, tau in ((24, 0.02), (24, 0.05), (32, 0.05), (24, 0.05)):
        Phi, Psi, X = op.hermite_forward(m), op.hermite_backward(m), op.hermite_nodes(m)
        c = synth.hermite_coefficients(m, 8, 3, cfg_id=3)
        psi0 = cast(om.tucker(c, [Psi] * 3), "fp64", True)
        ref = sc.ho_strang(psi0, [Phi] * 3, [Psi] * 3, [X] * 3, t0, tau, eps, 2)
        Fl, Bl = mm.hermite_matrices(m)
        Xl, _ = mm.hermite_nodes(m)
        F, Bo = ctx.mm_op_prepare(Fl, "fp64"), ctx.mm_op_prepare(Bl, "fp64")
        psi = to_gpu(psi0, "fp64", True)
        ctx.ho_strang_step(psi, [F] * 3, [Bo] * 3, [Xl] * 3, t0, tau, eps, 2)
        err = rel(from_gpu(psi), ref)
        note(f"ho cache m={m} tau={tau}: rel err {err:.3e}")
        assert err < 2e-12
        F.destroy()
        Bo.destroy()


def test_ho_step_truncated_hermite_basis(ctx):
    # K < m Hermite functions (rectangular Phi K x m, Psi m x K): the
    # collapsed propagator is Psi diag Phi of rank K
    import paper_2103_01691_amd as mm
    from oracle import mumode as om
    m, K, tau, t0, eps = 32, 20, 0.03, 0.0, 0.0
    Phi, Psi = op.hermite_forward(m), op.hermite_backward(m)
    c = synth.hermite_coefficients(m, 8, 3, cfg_id=3)
    psi0 = cast(om.tucker(c, [Psi] * 3), "fp64", True)
    Lh = Psi[:, :K] @ np.diag(np.exp(-1j * tau * (np.arange(K) + 0.5))) @ Phi[:K, :]
    ref = om.expstep(psi0, [Lh] * 3, 1)
    Fl, Bl = mm.hermite_matrices(m)
    Xl, _ = mm.hermite_nodes(m)
    F = ctx.mm_op_prepare(np.ascontiguousarray(Fl[:K, :]), "fp64")
    Bo = ctx.mm_op_prepare(np.ascontiguousarray(Bl[:, :K]), "fp64")
    psi = to_gpu(psi0, "fp64", True)
    ctx.ho_strang_step(psi, [F] * 3, [Bo] * 3, [Xl] * 3, t0, tau, eps, 1)
    assert rel(from_gpu(psi), ref) < 1e-12
