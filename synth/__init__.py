"""Seeded synthetic inputs shared by the oracle side and the library side.

This module draws random numbers and samples initial data on a grid.  It
holds none of the integrator's arithmetic: no operators, no exponentials, no
mode products.  Both the CPU oracle (``oracle/``) and the HIP library path
receive the arrays produced here, so that a parity comparison starts from
identical inputs.

Tensors are returned as numpy arrays indexed ``U[i_1, ..., i_d]`` in the
paper's index order (Section 2: the grid tensor collects u at
(x_1^{i_1}, ..., x_d^{i_d})).  ``to_device_layout`` turns such an array into
the C-ordered array of shape (n_d, ..., n_1) whose memory is the column-major
(i_1 fastest) layout the library uses (Section 4.1, the vec index
i_1 + n_1 (i_2 - 1) + n_1 n_2 (i_3 - 1)).

Seeds follow one rule: ``rng(cfg_id, instance_id)`` is
``default_rng(SeedSequence([cfg_id, instance_id, 20210302]))``.
"""
from __future__ import annotations

import numpy as np

SEED_TAG = 20210302


def rng(cfg_id: int, instance_id: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(cfg_id), int(instance_id), SEED_TAG]))


# --------------------------------------------------------------------------
# layout helpers (pure index bookkeeping)
# --------------------------------------------------------------------------

def to_device_layout(U: np.ndarray) -> np.ndarray:
    """U[i_1..i_d] -> C-contiguous array of shape (n_d..n_1) with i_1 fastest."""
    return np.ascontiguousarray(np.transpose(U, tuple(range(U.ndim - 1, -1, -1))))


def from_device_layout(A: np.ndarray) -> np.ndarray:
    """Inverse of ``to_device_layout``."""
    return np.transpose(A, tuple(range(A.ndim - 1, -1, -1)))


# --------------------------------------------------------------------------
# grids on which initial data are sampled (problem set-up, not the method)
# --------------------------------------------------------------------------

def dirichlet_nodes(n: int, a: float, b: float) -> np.ndarray:
    """n interior nodes of [a, b], spacing (b - a)/(n + 1)."""
    h = (b - a) / (n + 1)
    return a + h * np.arange(1, n + 1, dtype=np.float64)


def periodic_nodes(n: int, a: float, b: float) -> np.ndarray:
    """n nodes of [a, b), spacing (b - a)/n, first node at a."""
    h = (b - a) / n
    return a + h * np.arange(n, dtype=np.float64)


# --------------------------------------------------------------------------
# random tensors and matrices
# --------------------------------------------------------------------------

def graded_nodes(n: int, a: float, b: float, alpha: float = 2.0) -> np.ndarray:
    """n nodes from a to b (both included), denser near the centre:
    x = c + r sinh(alpha xi) / sinh(alpha), xi uniform on [-1, 1] (c the
    centre, r the half-width); alpha -> 0 gives the uniform grid.  A smooth
    grading, so three-point differences on it stay second order."""
    xi = np.linspace(-1.0, 1.0, n)
    c, r = 0.5 * (a + b), 0.5 * (b - a)
    if alpha == 0.0:
        return c + r * xi
    return c + r * np.sinh(alpha * xi) / np.sinh(alpha)


def vortex_pair_initial(nodes, d: float = 2.0, cfg_id: int = 6, instance_id: int = 0) -> np.ndarray:
    """A vortex and an anti-vortex, straight lines along x_3 through
    (x_1, x_2) = (+d, 0) and (-d, 0), in a background of density 1:
    u = prod_s ((x_1 - s d) + i s x_2) / sqrt((x_1 - s d)^2 + x_2^2 + 1),
    s = +1, -1, plus 1e-3 seeded complex noise (3-D; nodes: three 1-D node
    arrays).  |u| -> 1 away from the lines."""
    x1, x2 = nodes[0][:, None, None], nodes[1][None, :, None]
    u = np.ones((nodes[0].size, nodes[1].size, nodes[2].size), dtype=np.complex128)
    for sgn in (1.0, -1.0):
        z = (x1 - sgn * d) + 1j * sgn * x2
        u = u * (z / np.sqrt(np.abs(z) ** 2 + 1.0))
    g = rng(cfg_id, instance_id)
    return u + 1e-3 * complex_noise(u.shape, g)


def random_tensor(dims, complex_: bool, g: np.random.Generator, dist: str = "normal") -> np.ndarray:
    dims = tuple(int(x) for x in dims)
    if dist == "uniform":
        draw = lambda: g.random(dims)
    else:
        draw = lambda: g.standard_normal(dims)
    if complex_:
        return (draw() + 1j * draw()) / np.sqrt(2.0)
    return draw().astype(np.float64)


def random_matrix(rows: int, cols: int, complex_: bool, g: np.random.Generator,
                  scale: float | None = None) -> np.ndarray:
    """Dense, non-symmetric matrix with entries ~ N(0,1)/sqrt(cols) (or ``scale``)."""
    s = (1.0 / np.sqrt(cols)) if scale is None else scale
    if complex_:
        M = (g.standard_normal((rows, cols)) + 1j * g.standard_normal((rows, cols))) / np.sqrt(2.0)
    else:
        M = g.standard_normal((rows, cols))
    return M * s


def complex_noise(dims, g: np.random.Generator) -> np.ndarray:
    return (g.standard_normal(dims) + 1j * g.standard_normal(dims)) / np.sqrt(2.0)


# --------------------------------------------------------------------------
# initial data of the synthetic workloads
# --------------------------------------------------------------------------

def heat_initial(n: int = 64, d: int = 2, cfg_id: int = 1, instance_id: int = 0) -> np.ndarray:
    """d-dim heat state, entries uniform in [0, 1)."""
    return rng(cfg_id, instance_id).random((n,) * d)


def _normalise(psi: np.ndarray, cell: float) -> np.ndarray:
    return psi / np.sqrt(cell * np.sum(np.abs(psi) ** 2))


def wavepacket_initial(n: int = 256, a: float = -10.0, b: float = 10.0, d: int = 3,
                       cfg_id: int = 2, instance_id: int = 0, noise: float = 1e-3) -> np.ndarray:
    """Gaussian packet of width 1 centred at 0 with momentum k0 ~ U[-2,2]^d,
    plus ``noise`` * complex normal noise (peak amplitude 1), normalised so
    that h^d sum |psi|^2 = 1 on the Dirichlet interior grid."""
    g = rng(cfg_id, instance_id)
    k0 = g.uniform(-2.0, 2.0, size=d)
    x = dirichlet_nodes(n, a, b)
    h = (b - a) / (n + 1)
    psi = np.ones((1,) * d, dtype=np.complex128)
    for mu in range(d):
        shape = [1] * d
        shape[mu] = n
        f = np.exp(-0.5 * x ** 2 + 1j * k0[mu] * x).reshape(shape)
        psi = psi * f
    psi = psi + noise * complex_noise((n,) * d, g)
    return _normalise(psi, h ** d)


def thomas_fermi_initial(n: int = 256, a: float = -8.0, b: float = 8.0, d: int = 3,
                         beta: float = 100.0, cfg_id: int = 4, instance_id: int = 0,
                         noise: float = 1e-3) -> np.ndarray:
    """Thomas-Fermi-like profile sqrt(max(mu_TF - |x|^2/2, 0)/beta) with
    mu_TF = (1/2)(15 beta / (4 pi))^(2/5) (3-d harmonic trap), plus ``noise``
    complex normal noise, normalised on the Dirichlet interior grid."""
    g = rng(cfg_id, instance_id)
    x = dirichlet_nodes(n, a, b)
    h = (b - a) / (n + 1)
    mu_tf = 0.5 * (15.0 * beta / (4.0 * np.pi)) ** 0.4
    r2 = np.zeros((1,) * d)
    for mu in range(d):
        shape = [1] * d
        shape[mu] = n
        r2 = r2 + (x ** 2).reshape(shape)
    psi = np.sqrt(np.maximum(mu_tf - 0.5 * r2, 0.0) / beta).astype(np.complex128)
    psi = psi + noise * complex_noise((n,) * d, g)
    return _normalise(psi, h ** d)


def hermite_coefficients(m: int = 128, kmax: int = 16, d: int = 3, cfg_id: int = 3,
                         instance_id: int = 0) -> np.ndarray:
    """Coefficient tensor with c_k ~ complex normal for all k_mu < kmax, else 0."""
    g = rng(cfg_id, instance_id)
    c = np.zeros((m,) * d, dtype=np.complex128)
    c[(slice(0, kmax),) * d] = complex_noise((kmax,) * d, g)
    return c


def batch_mix(count: int = 512, cfg_id: int = 5, sizes=(32, 48, 64, 96, 128, 192)):
    """Instance descriptors of the batched workload: d in {2,3} and the
    problem kind (heat: real, Schroedinger: complex) drawn with probability
    1/2 each, every n_mu uniform from ``sizes``, tau log-uniform in
    [1e-4, 1e-2]."""
    g = rng(cfg_id, 0)
    out = []
    for i in range(count):
        d = int(g.integers(2, 4))
        kind = "heat" if g.random() < 0.5 else "schrodinger"
        dims = tuple(int(sizes[j]) for j in g.integers(0, len(sizes), size=d))
        tau = float(10.0 ** g.uniform(-4.0, -2.0))
        out.append({"index": i, "d": d, "kind": kind, "dims": dims, "tau": tau})
    return out
