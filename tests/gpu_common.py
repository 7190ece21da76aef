"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import sys

import numpy as np


def announce(*parts):
    """Names the case before any device work, so a failure that ends the run is attributable."""
    print("CASE", *parts, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(x):
    return x.detach().cpu().numpy()


def rel_fro(x, ref):
    den = np.linalg.norm(np.ravel(ref))
    return float(np.linalg.norm(np.ravel(x - ref)) / (den if den > 0 else 1.0))


# Relative Frobenius tolerances of each arithmetic form against the float64 oracle.
TOL = {0: 1e-12, 1: 1e-6, 2: 1e-9}
# split-bf16 at S digit slices (default product sets: S = 2, 3 the triangle, S = 4
# one more anti-diagonal).  Each operand keeps 8S bits below its row maximum;
# 16 * 2^(-8S) bounds the relative error on unstructured inputs (four rounded
# operands, rows whose maximum exceeds their rms several times).  The MP2-like
# workloads are held to the precision form's 1e-9 target at S = 4.
TOL_SPLIT = {2: 16 * 2.0 ** -16, 3: 16 * 2.0 ** -24, 4: 2e-9}
TOL_SPLIT_WORKLOAD = {2: 16 * 2.0 ** -16, 3: 16 * 2.0 ** -24, 4: 1e-9}
