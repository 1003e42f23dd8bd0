"""Shared helpers of the GPU parity tests (compare the HIP path with the CPU oracle)."""
import numpy as np

# Normwise relative tolerance for FP32 results against the FP64 oracle (complex64 state).
TOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def t2n(t):
    return t.detach().cpu().numpy().astype(np.float64)


def report(name, **errs):
    print(name, " ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
