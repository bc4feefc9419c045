"""Python binding of the MI355X mu-mode product library (include/mumode.h).

Argument marshalling only: every tensor operation runs in the HIP kernels of
``libmumode.so``.  Tensors are torch tensors on the GPU with shape
(n_d, ..., n_1), C-contiguous, so that their memory is the column-major
(i_1 fastest) layout of the library; dtypes float32, float64, complex64,
complex128.  Matrices are numpy arrays indexed L[i, j]; they are handed to
the library as column-major FP64 masters.  Work is enqueued on torch's
current stream.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (MM_C64, MM_C128, MM_PREC_BF16, MM_PREC_FP32, MM_PREC_FP64,  # noqa: F401
                   MM_PREC_SPLIT_BF16X3, MM_PREC_SPLIT_FP16X2, MM_R32, MM_R64)

MM_OPT_SMALL_RUN = 1
MM_OPT_MONITOR_EVERY = 2
MM_OPT_FP16X2_CHAIN = 3
MM_OP_IDENTITY_SPLIT = 1

PRECISIONS = {"fp64": MM_PREC_FP64, "fp32": MM_PREC_FP32, "bf16x3": MM_PREC_SPLIT_BF16X3,
              "fp16x2": MM_PREC_SPLIT_FP16X2, "bf16": MM_PREC_BF16}


def _mode_arrays(xs, t, name):
    """Per-mode host arrays of the tensor's mode lengths (the library reads
    n_k values of array k), as FP64 and as the pointer array the ABI takes."""
    keep = [np.ascontiguousarray(np.asarray(x, dtype=np.float64)).reshape(-1) for x in xs]
    if len(keep) < t.d or any(keep[k].size != t.dims[k] for k in range(t.d)):
        raise ValueError(f"{name}: one array per mode with n_k entries each, "
                         f"modes {[int(t.dims[k]) for k in range(t.d)]}")
    arr = (C.POINTER(C.c_double) * len(keep))(*[k.ctypes.data_as(C.POINTER(C.c_double)) for k in keep])
    return keep, arr


class MumodeError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        name = _lib.lib.mm_status_string(status).decode()
        super().__init__(f"{where}: {name} ({status}): {detail}")


def _check(status: int, where: str, ctx=None):
    if status != 0:
        detail = _lib.lib.mm_last_error(ctx).decode() if ctx is not None or where == "mm_create" else ""
        raise MumodeError(status, where, detail)


def version() -> str:
    return _lib.lib.mm_version().decode()


# ------------------------------------------------------------ host FP64 ----

def fd2_matrix(n: int, a: float, b: float, bc: str = "dirichlet") -> np.ndarray:
    out = np.zeros((n, n), dtype=np.float64, order="F")
    _check(_lib.lib.mm_fd2_matrix(n, a, b, 0 if bc == "dirichlet" else 1,
                                  out.ctypes.data_as(C.POINTER(C.c_double))), "mm_fd2_matrix")
    return np.asarray(out)


def expm(A: np.ndarray, c: complex = 1.0) -> np.ndarray:
    """exp(c A) of a small square matrix (FP64 on the host)."""
    A = np.asfortranarray(np.asarray(A, dtype=np.complex128))
    n = A.shape[0]
    out = np.zeros((n, n), dtype=np.complex128, order="F")
    _check(_lib.lib.mm_expm(n, A.ctypes.data_as(C.POINTER(C.c_double)), float(np.real(c)), float(np.imag(c)),
                            out.ctypes.data_as(C.POINTER(C.c_double))), "mm_expm")
    return np.asarray(out)


def hermite_nodes(m: int):
    X = np.zeros(m)
    w = np.zeros(m)
    _check(_lib.lib.mm_hermite_nodes(m, X.ctypes.data_as(C.POINTER(C.c_double)),
                                     w.ctypes.data_as(C.POINTER(C.c_double))), "mm_hermite_nodes")
    return X, w


def hermite_matrices(m: int):
    Phi = np.zeros((m, m), order="F")
    Psi = np.zeros((m, m), order="F")
    _check(_lib.lib.mm_hermite_matrices(m, Phi.ctypes.data_as(C.POINTER(C.c_double)),
                                        Psi.ctypes.data_as(C.POINTER(C.c_double))), "mm_hermite_matrices")
    return np.asarray(Phi), np.asarray(Psi)


def hermite_ho_exponential(m: int, tau: float) -> np.ndarray:
    """Psi diag(exp(-i tau (k + 1/2))) Phi (exact HO propagator, nodal space)."""
    out = np.zeros((m, m), dtype=np.complex128, order="F")
    _check(_lib.lib.mm_hermite_ho_exponential(m, float(tau), out.ctypes.data_as(C.POINTER(C.c_double))),
           "mm_hermite_ho_exponential")
    return np.asarray(out)


def schrodinger_fd_hamiltonian(n: int, a: float, b: float, omega2: float = 1.0) -> np.ndarray:
    """-1/2 D2 + (omega2/2) diag(x^2) on n interior Dirichlet nodes of [a, b]."""
    out = np.zeros((n, n), dtype=np.float64, order="F")
    _check(_lib.lib.mm_schrodinger_fd_hamiltonian(n, float(a), float(b), float(omega2),
                                                  out.ctypes.data_as(C.POINTER(C.c_double))),
           "mm_schrodinger_fd_hamiltonian")
    return np.asarray(out)


def schrodinger_fd_exponential(n: int, a: float, b: float, omega2: float, tau: float) -> np.ndarray:
    """exp(-i tau H), H = schrodinger_fd_hamiltonian(n, a, b, omega2)."""
    out = np.zeros((n, n), dtype=np.complex128, order="F")
    _check(_lib.lib.mm_schrodinger_fd_exponential(n, float(a), float(b), float(omega2), float(tau),
                                                  out.ctypes.data_as(C.POINTER(C.c_double))),
           "mm_schrodinger_fd_exponential")
    return np.asarray(out)


def hermite_ho_generator(m: int) -> np.ndarray:
    """(i/2)(d^2/dx^2 - x^2) in nodal Hermite space, Psi diag(-i (k + 1/2)) Phi."""
    out = np.zeros((m, m), dtype=np.complex128, order="F")
    _check(_lib.lib.mm_hermite_ho_generator(m, out.ctypes.data_as(C.POINTER(C.c_double))),
           "mm_hermite_ho_generator")
    return np.asarray(out)


def fd2_periodic_order(n: int, a: float, b: float, order: int) -> np.ndarray:
    """Centred second difference of even `order` on n periodic nodes of [a, b)."""
    out = np.zeros((n, n), dtype=np.float64, order="F")
    _check(_lib.lib.mm_fd2_periodic_order(n, float(a), float(b), int(order), out.ctypes.data_as(C.POINTER(C.c_double))),
           "mm_fd2_periodic_order")
    return np.asarray(out)


def fourier_d2(n: int, a: float, b: float) -> np.ndarray:
    """Fourier spectral second derivative on n periodic nodes of [a, b)."""
    out = np.zeros((n, n), dtype=np.float64, order="F")
    _check(_lib.lib.mm_fourier_d2(n, float(a), float(b), out.ctypes.data_as(C.POINTER(C.c_double))), "mm_fourier_d2")
    return np.asarray(out)


def pipe_flow_operators(n_r: int, n_z: int, r_min: float = 0.1, r_max: float = 5.0, z_max: float = 8.0,
                        alpha: float = 1.0 / 90):
    """(A_r, A_z) of the pipe-flow problem (Section 4.2)."""
    A_r = np.zeros((n_r, n_r), dtype=np.float64, order="F")
    A_z = np.zeros((n_z, n_z), dtype=np.float64, order="F")
    _check(_lib.lib.mm_pipe_flow_operators(n_r, n_z, float(r_min), float(r_max), float(z_max), float(alpha),
                                           A_r.ctypes.data_as(C.POINTER(C.c_double)),
                                           A_z.ctypes.data_as(C.POINTER(C.c_double))), "mm_pipe_flow_operators")
    return np.asarray(A_r), np.asarray(A_z)


def nonuniform_neumann_d2(x):
    """(M_W, w): symmetrised second derivative on the non-uniform nodes x with
    homogeneous Neumann ends, and the dual-cell weights (Section 4.5)."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    n = x.size
    M = np.zeros((n, n), dtype=np.float64, order="F")
    w = np.zeros(n)
    _check(_lib.lib.mm_nonuniform_neumann_d2(n, x.ctypes.data_as(C.POINTER(C.c_double)),
                                             M.ctypes.data_as(C.POINTER(C.c_double)),
                                             w.ctypes.data_as(C.POINTER(C.c_double))), "mm_nonuniform_neumann_d2")
    return np.asarray(M), w


# -------------------------------------------------------------- tensors ----

def _dtype_code(t) -> int:
    import torch
    m = {torch.float32: MM_R32, torch.float64: MM_R64, torch.complex64: MM_C64, torch.complex128: MM_C128}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def as_mm_tensor(t) -> _lib.MMTensor:
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    d = t.dim()
    if not 1 <= d <= _lib.MM_MAXD:
        raise ValueError("tensor order out of range")
    mt = _lib.MMTensor()
    mt.d = d
    for k in range(d):
        mt.dims[k] = int(t.shape[d - 1 - k])      # n_1 is the last torch dim
    mt.dtype = _dtype_code(t)
    mt.data = t.data_ptr()
    return mt


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Op:
    """A prepared operator owned by a Context."""

    def __init__(self, ctx: "Context", handle: C.c_void_p, rows: int, cols: int, cplx: bool, prec: int):
        self.ctx = ctx
        self.handle = handle
        self.rows, self.cols, self.cplx, self.prec = rows, cols, cplx, prec

    def destroy(self):
        if self.handle:
            _check(_lib.lib.mm_op_destroy(self.ctx.handle, self.handle), "mm_op_destroy", self.ctx.handle)
            self.handle = None


def _op_array(ops):
    arr = (C.c_void_p * len(ops))()
    for k, o in enumerate(ops):
        arr[k] = None if o is None else o.handle
    return arr


class Context:
    """mm_create / mm_destroy around one device."""

    def __init__(self, device: int = 0, tune_cache_path=None):
        h = C.c_void_p()
        st = _lib.lib.mm_create(C.byref(h), device, None if tune_cache_path is None else str(tune_cache_path).encode())
        if st != 0:
            raise MumodeError(st, "mm_create", _lib.lib.mm_last_error(None).decode())
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _lib.lib.mm_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st, where):
        _check(st, where, self.handle)

    # ------------------------------------------------------------ ops ----
    def mm_op_prepare(self, L: np.ndarray, prec="fp64", identity_split: bool = False) -> Op:
        """identity_split: prepare L - I and add the input back in each product
        (MM_OP_IDENTITY_SPLIT; square L)."""
        prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        L = np.asarray(L)
        cplx = np.iscomplexobj(L)
        F = np.asfortranarray(L.astype(np.complex128 if cplx else np.float64))
        m = _lib.MMMatrix()
        m.rows, m.cols = F.shape
        m.ld = F.shape[0]
        m.dtype = MM_C128 if cplx else MM_R64
        m.data = F.ctypes.data
        m.on_device = 0
        h = C.c_void_p()
        self._chk(_lib.lib.mm_op_prepare_ex(self.handle, C.byref(m), prec, MM_OP_IDENTITY_SPLIT if identity_split else 0,
                                            C.byref(h)), "mm_op_prepare_ex")
        return Op(self, h, F.shape[0], F.shape[1], cplx, prec)

    # -------------------------------------------------------- products ----
    def mumode_apply(self, out, T, L: Op, mu: int, stream=None):
        o, t = as_mm_tensor(out), as_mm_tensor(T)
        self._chk(_lib.lib.mumode_apply(self.handle, C.byref(o), C.byref(t), L.handle, mu, _stream(stream)),
                  "mumode_apply")
        return out

    def mumode_expstep(self, T, E, nsteps: int = 1, stream=None):
        t = as_mm_tensor(T)
        self._chk(_lib.lib.mumode_expstep(self.handle, C.byref(t), _op_array(E), nsteps, _stream(stream)),
                  "mumode_expstep")
        return T

    def mumode_transform(self, out, T, Phi, stream=None):
        o, t = as_mm_tensor(out), as_mm_tensor(T)
        self._chk(_lib.lib.mumode_transform(self.handle, C.byref(o), C.byref(t), _op_array(Phi),
                                            _stream(stream)), "mumode_transform")
        return out

    def gpe_strang_step(self, psi, E, tau: float, beta: float, nsteps: int = 1, stream=None):
        t = as_mm_tensor(psi)
        self._chk(_lib.lib.gpe_strang_step(self.handle, C.byref(t), _op_array(E), float(tau), float(beta),
                                           nsteps, _stream(stream)), "gpe_strang_step")
        return psi

    def gpe_strang_step_noalloc(self, psi, E, tau: float, beta: float, nsteps: int = 1, stream=None):
        t = as_mm_tensor(psi)
        self._chk(_lib.lib.gpe_strang_step_noalloc(self.handle, C.byref(t), _op_array(E), float(tau), float(beta),
                                                   nsteps, _stream(stream)), "gpe_strang_step_noalloc")
        return psi

    def mumode_expstep_batched(self, tensors, ops, nsteps: int = 1, stream=None):
        """tensors: list of torch tensors; ops: list of per-instance op lists."""
        n = len(tensors)
        mts = [as_mm_tensor(t) for t in tensors]
        tarr = (C.POINTER(_lib.MMTensor) * n)(*[C.pointer(m) for m in mts])
        oarrs = [_op_array(o) for o in ops]
        earr = (C.POINTER(C.c_void_p) * n)(*[C.cast(o, C.POINTER(C.c_void_p)) for o in oarrs])
        self._chk(_lib.lib.mumode_expstep_batched(self.handle, n, tarr, earr, nsteps, _stream(stream)),
                  "mumode_expstep_batched")
        return tensors

    def ho_strang_step(self, psi, Phi_fwd, Psi_bwd, nodes, t0: float, tau: float, eps: float, nsteps: int = 1,
                       stream=None):
        """Phi_fwd / Psi_bwd: per-mode prepared real forward / backward Hermite
        transforms (Op); nodes: per-mode arrays of the quadrature nodes."""
        t = as_mm_tensor(psi)
        keep, arr = _mode_arrays(nodes, t, "nodes")
        self._chk(_lib.lib.ho_strang_step(self.handle, C.byref(t), _op_array(Phi_fwd), _op_array(Psi_bwd), arr,
                                          float(t0), float(tau), float(eps), nsteps, _stream(stream)),
                  "ho_strang_step")
        return psi

    def vortex_strang_step(self, v, E, w, tau: float, nsteps: int = 1, stream=None):
        """E: per-mode exp(i tau/2 M_k) operators; w: per-mode dual-cell widths."""
        t = as_mm_tensor(v)
        keep, arr = _mode_arrays(w, t, "w")
        self._chk(_lib.lib.vortex_strang_step(self.handle, C.byref(t), _op_array(E), arr, float(tau), nsteps,
                                              _stream(stream)), "vortex_strang_step")
        return v

    def mm_energy_gpe(self, psi, H, beta: float, cell: float, stream=None) -> float:
        t = as_mm_tensor(psi)
        out = C.c_double()
        self._chk(_lib.lib.mm_energy_gpe(self.handle, C.byref(t), _op_array(H), float(beta), float(cell),
                                         C.byref(out), _stream(stream)), "mm_energy_gpe")
        return out.value

    def mm_norm2(self, T, cell: float = 1.0, stream=None) -> float:
        t = as_mm_tensor(T)
        out = C.c_double()
        self._chk(_lib.lib.mm_norm2(self.handle, C.byref(t), float(cell), C.byref(out), _stream(stream)),
                  "mm_norm2")
        return out.value

    def mumode_magnus_step(self, T, B, d, g, tau: float, nsteps: int = 1, prec="fp64", stream=None):
        """B: list of n_k x n_k numpy matrices (None: mode unchanged); d: list of
        real node arrays or None; g: array (nsteps, T.d) of complex coefficients
        at the step midpoints (or None)."""
        prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        t = as_mm_tensor(T)
        k = len(B)
        mats = (_lib.MMMatrix * k)()
        keep = []
        for i, Bm in enumerate(B):
            if Bm is None:
                mats[i].data = None
                continue
            F = np.asfortranarray(np.asarray(Bm, dtype=np.complex128))
            keep.append(F)
            mats[i].rows, mats[i].cols = F.shape
            mats[i].ld = F.shape[0]
            mats[i].dtype = MM_C128
            mats[i].data = F.ctypes.data
            mats[i].on_device = 0
        darr = None
        if d is not None:
            dk = [np.ascontiguousarray(np.asarray(x, dtype=np.float64)) if x is not None else None for x in d]
            keep.extend(x for x in dk if x is not None)
            darr = (C.POINTER(C.c_double) * k)(*[x.ctypes.data_as(C.POINTER(C.c_double)) if x is not None else None
                                                 for x in dk])
        garr = None
        if g is not None:
            G = np.ascontiguousarray(np.asarray(g, dtype=np.complex128).reshape(nsteps, k))
            keep.append(G)
            garr = G.ctypes.data_as(C.POINTER(C.c_double))
        self._chk(_lib.lib.mumode_magnus_step(self.handle, C.byref(t), mats, darr, garr, float(tau), nsteps, prec,
                                              _stream(stream)), "mumode_magnus_step")
        return T

    def mm_expm_device(self, A, c: complex, out, stream=None):
        """A, out: torch complex128 CUDA tensors holding column-major n x n
        matrices (e.g. the transpose view .T of a row-major matrix's storage)."""
        n = A.shape[0]
        c = complex(c)
        self._chk(_lib.lib.mm_expm_device(self.handle, n, C.c_void_p(A.data_ptr()), c.real, c.imag,
                                          C.c_void_p(out.data_ptr()), _stream(stream)), "mm_expm_device")
        return out

    # ------------------------------------------------- tuning, memory ----
    def mm_set_option(self, option: int, value: int):
        self._chk(_lib.lib.mm_set_option(self.handle, int(option), int(value)), "mm_set_option")

    def mm_monitor_log(self, max_records: int = 1 << 16):
        """List of (steps, sum |T|^2) recorded by the last monitored call."""
        n = C.c_int()
        st = (C.c_int * max_records)()
        v = (C.c_double * max_records)()
        self._chk(_lib.lib.mm_monitor_log(self.handle, max_records, C.byref(n), st, v), "mm_monitor_log")
        return [(st[i], v[i]) for i in range(min(n.value, max_records))]

    def mm_autotune(self, T, E, budget_ms: int = 1000, stream=None):
        t = as_mm_tensor(T)
        self._chk(_lib.lib.mm_autotune(self.handle, C.byref(t), _op_array(E), int(budget_ms), _stream(stream)),
                  "mm_autotune")

    def mm_autotune_batched(self, tensors, ops, budget_ms: int = 200, stream=None):
        """Choose the batched step's tile class per (mode, real / complex) by
        timing the batch itself (runs steps in place on the tensors)."""
        n = len(tensors)
        mts = [as_mm_tensor(t) for t in tensors]
        tarr = (C.POINTER(_lib.MMTensor) * n)(*[C.pointer(m) for m in mts])
        oarrs = [_op_array(o) for o in ops]
        earr = (C.POINTER(C.c_void_p) * n)(*[C.cast(o, C.POINTER(C.c_void_p)) for o in oarrs])
        self._chk(_lib.lib.mm_autotune_batched(self.handle, n, tarr, earr, int(budget_ms), _stream(stream)),
                  "mm_autotune_batched")
        out = {}
        for mode in range(1, _lib.MM_MAXD + 1):
            for cplx in (0, 1):
                c = C.c_int()
                self._chk(_lib.lib.mm_autotune_batched_get(self.handle, mode, cplx, C.byref(c)),
                          "mm_autotune_batched_get")
                if c.value >= 0:
                    out[(mode, bool(cplx))] = c.value
        return out

    def mm_tune_entries(self):
        """List of (key6 tuple, tile class, microseconds) of the recorded entries."""
        n = C.c_int()
        self._chk(_lib.lib.mm_tune_count(self.handle, C.byref(n)), "mm_tune_count")
        out = []
        for i in range(n.value):
            key = (C.c_int64 * 6)()
            cls = C.c_int()
            us = C.c_double()
            self._chk(_lib.lib.mm_tune_get(self.handle, i, key, C.byref(cls), C.byref(us)), "mm_tune_get")
            out.append((tuple(key), cls.value, us.value))
        return out

    def mm_tune_clear(self):
        self._chk(_lib.lib.mm_tune_clear(self.handle), "mm_tune_clear")

    def mm_tune_save(self, path: str):
        self._chk(_lib.lib.mm_tune_save(self.handle, str(path).encode()), "mm_tune_save")

    def mm_tune_load(self, path: str):
        self._chk(_lib.lib.mm_tune_load(self.handle, str(path).encode()), "mm_tune_load")

    def mm_set_workspace(self, buf=None):
        """buf: a torch CUDA tensor the caller keeps alive, or None."""
        if buf is None:
            self._chk(_lib.lib.mm_set_workspace(self.handle, None, 0), "mm_set_workspace")
        else:
            self._chk(_lib.lib.mm_set_workspace(self.handle, C.c_void_p(buf.data_ptr()),
                                                buf.numel() * buf.element_size()), "mm_set_workspace")

    # --------------------------------------------------------- timing ----
    def mm_profile_begin(self):
        self._chk(_lib.lib.mm_profile_begin(self.handle), "mm_profile_begin")

    def mm_profile_end(self, max_records: int = 1 << 16):
        """Returns a list of (kind_code, ms) per recorded launch."""
        n = C.c_int()
        kinds = (C.c_int * max_records)()
        ms = (C.c_double * max_records)()
        self._chk(_lib.lib.mm_profile_end(self.handle, max_records, C.byref(n), kinds, ms), "mm_profile_end")
        k = min(n.value, max_records)
        return [(kinds[i], ms[i]) for i in range(k)]
