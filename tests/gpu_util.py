"""Helpers shared by the GPU parity tests (no test functions here)."""
import sys

import numpy as np

import synth

# Tolerances on relative L2 error against the FP64 oracle (relative L2 over
# all real components, reference computed from the identically cast input).
#   fp64   1e-12  (FP64 MFMA; rounding ~ 1e-16 sqrt(n) per product)
#   fp32   1e-5   (FP32 MFMA)
#   bf16x3 1e-6   (three-piece split, six products, FP32 accumulation)
#   fp16x2 1e-6   (two-piece half-precision split, three products, FP32
#                  accumulation)
#   bf16   1e-2   (one piece; reported only)
REL_TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-6, "fp16x2": 1e-6, "bf16": 1e-2}


def rel(a, b):
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / np.linalg.norm(np.asarray(b).ravel()))


def state_dtype(prec, cplx):
    import torch
    if prec == "fp64":
        return (np.complex128, torch.complex128) if cplx else (np.float64, torch.float64)
    return (np.complex64, torch.complex64) if cplx else (np.float32, torch.float32)


def cast(U, prec, cplx):
    """Round an FP64 tensor to the state dtype of `prec` (returns FP64 copy)."""
    npdt, _ = state_dtype(prec, cplx)
    return U.astype(npdt).astype(np.complex128 if cplx else np.float64)


def to_gpu(U, prec, cplx):
    import torch
    npdt, _ = state_dtype(prec, cplx)
    return torch.from_numpy(synth.to_device_layout(U.astype(npdt))).cuda()


def from_gpu(t):
    import torch
    torch.cuda.synchronize()
    return synth.from_device_layout(t.cpu().numpy()).astype(np.complex128 if t.is_complex() else np.float64)


def empty_gpu(dims, prec, cplx):
    import torch
    _, tdt = state_dtype(prec, cplx)
    return torch.zeros(tuple(reversed(dims)), dtype=tdt, device="cuda")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()
