"""GPU parity of the integrator with the operator front-ends: centred
differences of higher order and the Fourier spectral second derivative on
the periodic heat problem of Section 4.1 (Test 2), and the non-constant-
coefficient pipe-flow operators of Section 4.2."""
import numpy as np
import pytest

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


def _heat_u0(n):
    x = 2 * np.pi * np.arange(n) / n
    c = np.cos(x)
    return c[:, None, None] + c[None, :, None] + c[None, None, :]


@pytest.mark.parametrize("order", [4, 8, "spectral"])
def test_periodic_heat_higher_order(ctx, order):
    import paper_2103_01691_amd as mm
    n, T = 40, 1.0
    if order == "spectral":
        Al, Ao = mm.fourier_d2(n, 0.0, 2 * np.pi), op.fourier_d2(n, 0.0, 2 * np.pi)
    else:
        Al, Ao = mm.fd2_periodic_order(n, 0.0, 2 * np.pi, order), op.fd2_periodic_order(n, 0.0, 2 * np.pi, order)
    El = mm.expm(Al, T).real.copy()
    Eo = op.exp_symmetric(Ao, T).real
    u0 = _heat_u0(n)
    ref = om.expstep(u0, [Eo] * 3, 1)
    u = to_gpu(u0, "fp64", False)
    ctx.mumode_expstep(u, [ctx.mm_op_prepare(El, "fp64")] * 3, 1)
    got = from_gpu(u)
    err = rel(got, ref)
    # closed form: cos(x) is an eigenvector of every periodic stencil, with
    # eigenvalue (w_0 + 2 sum_k w_k cos(k h)) / h^2 (-1 for the spectral
    # matrix), so u(T) = exp(lambda T) u0
    h = 2 * np.pi / n
    if order == "spectral":
        lam = -1.0
    else:
        w = op.central_d2_weights(order)
        lam = (w[0] + 2 * sum(w[k] * np.cos(k * h) for k in range(1, len(w)))) / h ** 2
    cf = rel(got, np.exp(lam * T) * u0)
    note(f"periodic heat order={order}: rel err vs oracle {err:.3e}, vs closed form {cf:.3e}, "
         f"vs continuum exp(-T) u0 {rel(got, np.exp(-T) * u0):.3e}")
    assert err < 1e-12
    assert cf < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pipe_flow_step(ctx, prec):
    import paper_2103_01691_amd as mm
    from scipy.linalg import expm
    n, T = 200, 1.0
    rmin, rmax, zmax, alpha = 0.1, 5.0, 8.0, 1.0 / 90
    Ar, Az, r, z = op.pipe_flow_operators(n, n, rmin, rmax, zmax, alpha)
    c0 = np.exp(-8 * (r[:, None] - 0.5 * (rmin + rmax)) ** 2 - 8 * (z[None, :] - 1.5) ** 2)
    c0 = cast(c0, prec, False)
    ref = om.expstep(c0, [expm(T * Ar), expm(T * Az)], 1)
    Lr, Lz = mm.pipe_flow_operators(n, n, rmin, rmax, zmax, alpha)
    ops = [ctx.mm_op_prepare(mm.expm(L, T).real.copy(), prec) for L in (Lr, Lz)]
    c = to_gpu(c0, prec, False)
    ctx.mumode_expstep(c, ops, 1)
    err = rel(from_gpu(c), ref)
    note(f"pipe flow n={n} {prec} rel err {err:.3e}")
    assert err < REL_TOL[prec] * (10 if prec == "fp64" else 1)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_nonuniform_neumann_schroedinger_flow(ctx, prec):
    # the linear part of the Section 4.5 vortex problem, i psi_t = -1/2 Laplace
    # psi on [-20, 20]^3 with homogeneous Neumann ends, discretised on graded
    # non-uniform nodes (a different count per mode) and symmetrised: in
    # v = W^(1/2) psi the flow is the mu-mode integrator with
    # E_mu = exp(i tau/2 M_mu), and the W-weighted mass sum W |psi|^2 = |v|^2
    # is conserved
    import synth
    import paper_2103_01691_amd as mm
    dims, tau, steps = (48, 40, 32), 0.1, 3
    xs = [synth.graded_nodes(n, -20.0, 20.0, 2.0) for n in dims]
    El, Eo, ws = [], [], []
    for x in xs:
        Ml, wl = mm.nonuniform_neumann_d2(x)
        Mo, wo = op.nonuniform_neumann_d2(x)
        El.append(mm.expm(Ml, 0.5j * tau))
        Eo.append(op.exp_symmetric(Mo, 0.5j * tau))
        ws.append(wo)
    g = synth.rng(1401, 0)
    W = ws[0][:, None, None] * ws[1][None, :, None] * ws[2][None, None, :]
    # two displaced Gaussian blobs with opposite momenta plus noise
    psi = (np.exp(-((xs[0][:, None, None] - 3) ** 2 + xs[1][None, :, None] ** 2 + xs[2][None, None, :] ** 2) / 8
                  + 1j * xs[0][:, None, None])
           + np.exp(-((xs[0][:, None, None] + 3) ** 2 + xs[1][None, :, None] ** 2 + xs[2][None, None, :] ** 2) / 8
                    - 1j * xs[0][:, None, None]))
    psi = psi + 1e-3 * synth.random_tensor(dims, True, g)
    v0 = cast(np.sqrt(W) * psi, prec, True)
    ref = om.expstep(v0, Eo, steps)
    ops = [ctx.mm_op_prepare(e, prec) for e in El]
    v = to_gpu(v0, prec, True)
    ctx.mumode_expstep(v, ops, steps)
    got = from_gpu(v)
    err = rel(got, ref)
    mass0 = float(np.sum(np.abs(v0) ** 2))
    mass = ctx.mm_norm2(v, 1.0)
    note(f"non-uniform Neumann {prec}: rel L2 {err:.3e}, weighted mass drift {abs(mass / mass0 - 1):.2e}")
    assert err < steps * REL_TOL[prec]
    assert abs(mass / mass0 - 1.0) < (1e-12 if prec == "fp64" else 1e-5)
    for o in ops:
        o.destroy()


def _vortex_problem(dims, alpha=2.0):
    import synth
    import paper_2103_01691_amd as mm
    xs = [synth.graded_nodes(n, -20.0, 20.0, alpha) for n in dims]
    Ml, Mo, ws = [], [], []
    for x in xs:
        m, _ = mm.nonuniform_neumann_d2(x)
        mo, wo = op.nonuniform_neumann_d2(x)
        Ml.append(m)
        Mo.append(mo)
        ws.append(wo)
    W = ws[0][:, None, None] * ws[1][None, :, None] * ws[2][None, None, :]
    return xs, Ml, Mo, ws, W


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x2"])
def test_vortex_strang_step(ctx, prec):
    # the Section 4.5 vortex pair on graded non-uniform nodes (a different
    # count per mode, none a multiple of the tile edge), symmetrised variable
    # v = W^(1/2) u: three Strang steps, nonlinear half steps merged
    import synth
    import paper_2103_01691_amd as mm
    from oracle import schemes as sc
    dims, tau, steps = (40, 36, 30), 0.1, 3
    xs, Ml, Mo, ws, W = _vortex_problem(dims)
    Eo = [op.exp_symmetric(m, 0.5j * tau) for m in Mo]
    v0 = cast(np.sqrt(W) * synth.vortex_pair_initial(xs), prec, True)
    note(f"vortex {prec}: oracle, {steps} steps")
    ref = sc.vortex_strang(v0, Eo, 1.0 / W, tau, steps)
    ops = [ctx.mm_op_prepare(mm.expm(m, 0.5j * tau), prec) for m in Ml]
    v = to_gpu(v0, prec, True)
    ctx.vortex_strang_step(v, ops, ws, tau, steps)
    got = from_gpu(v)
    err = rel(got, ref)
    mass0 = float(np.sum(np.abs(v0) ** 2))
    mass = ctx.mm_norm2(v, 1.0)
    note(f"vortex {prec}: rel L2 {err:.3e}, weighted mass drift {abs(mass / mass0 - 1):.2e}")
    assert err < 2 * steps * REL_TOL[prec]
    # both parts of the splitting are unitary in v
    assert abs(mass / mass0 - 1.0) < (1e-12 if prec == "fp64" else 1e-5)
    for o in ops:
        o.destroy()


def test_vortex_background_steady_and_weights_reuploaded(ctx):
    # u = 1: the Neumann Laplacian annihilates constants and the nonlinearity
    # vanishes at |u| = 1, so steps leave v = W^(1/2) unchanged; then the same
    # context with other nodes (other weights, same sizes) must use the new
    # weights
    import synth
    import paper_2103_01691_amd as mm
    from oracle import schemes as sc
    dims, tau = (24, 20, 16), 0.1
    for alpha in (2.0, 1.0):
        xs, Ml, Mo, ws, W = _vortex_problem(dims, alpha)
        ops = [ctx.mm_op_prepare(mm.expm(m, 0.5j * tau), "fp64") for m in Ml]
        v0 = np.sqrt(W).astype(np.complex128)
        v = to_gpu(v0, "fp64", True)
        ctx.vortex_strang_step(v, ops, ws, tau, 4)
        dev = np.max(np.abs(from_gpu(v) - v0)) / np.max(np.abs(v0))
        u1 = np.sqrt(W) * synth.vortex_pair_initial(xs)
        ref = sc.vortex_strang(u1, [op.exp_symmetric(m, 0.5j * tau) for m in Mo], 1.0 / W, tau, 2)
        v = to_gpu(u1, "fp64", True)
        ctx.vortex_strang_step(v, ops, ws, tau, 2)
        err = rel(from_gpu(v), ref)
        note(f"vortex alpha={alpha}: background deviation {dev:.2e}, vortex pair rel err {err:.3e}")
        assert dev < 1e-12
        assert err < 1e-12
        for o in ops:
            o.destroy()


def test_vortex_step_checks(ctx):
    # zero steps leave the state alone; a real state, a non-positive width,
    # a wrong operator size or a missing weight array are refused before any
    # launch
    import paper_2103_01691_amd as mm
    dims, tau = (24, 16, 8), 0.1
    xs, Ml, Mo, ws, W = _vortex_problem(dims)
    ops = [ctx.mm_op_prepare(mm.expm(m, 0.5j * tau), "fp64") for m in Ml]
    v0 = np.sqrt(W).astype(np.complex128) * (1.0 + 0.1j)
    v = to_gpu(v0, "fp64", True)
    ctx.vortex_strang_step(v, ops, ws, tau, 0)
    assert np.array_equal(from_gpu(v), v0)
    with pytest.raises(mm.MumodeError) as e:
        ctx.vortex_strang_step(to_gpu(np.abs(v0), "fp64", False), ops, ws, tau, 1)
    assert e.value.status == 3       # MM_ERR_DTYPE
    bad = [w.copy() for w in ws]
    bad[1][3] = 0.0
    with pytest.raises(mm.MumodeError) as e:
        ctx.vortex_strang_step(v, ops, bad, tau, 1)
    assert e.value.status == 1       # MM_ERR_ARG
    with pytest.raises(mm.MumodeError) as e:
        ctx.vortex_strang_step(v, [ops[1], ops[0], ops[2]], ws, tau, 1)
    assert e.value.status == 2       # MM_ERR_SHAPE
    assert np.array_equal(from_gpu(v), v0)
    for o in ops:
        o.destroy()
