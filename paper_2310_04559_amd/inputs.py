"""Seeded synthetic inputs for the Cholesky-vector particle-particle ladder.

This module draws the arrays both sides consume: the Cholesky vectors of the
virtual-virtual block, MP2-like doubles amplitudes and, for the adjoint, an
upstream gradient.  It holds none of the ladder's arithmetic; the oracle and
the HIP library both take its arrays as plain inputs.

Recipe (the paper's workloads are random arrays, Sec. "Numerical results";
its molecular case is not reproducible without the molecule, so these draws
stand in for it):

1. ``rng = numpy.random.default_rng(seed)`` (PCG64).
2. ``X = rng.standard_normal((P, n, n))`` with ``n = o + v``; every Cholesky
   vector is made symmetric in its two orbital indices by mirroring the upper
   triangle (diagonal included), because real orbitals give one symmetric
   factor for both pair indices (Sec. "The CC ansatz", eq. cholesky).  Vector
   ``x`` (0-based) is then scaled by ``exp(-x/25)/sqrt(n)``: a decaying
   spectrum like a converged decomposition.
3. ``e_occ = sort(U[-2, -0.3]^o)``, ``e_vir = sort(U[0.1, 3]^v)``.
4. ``(ia|jb) = sum_x L[x,i,o+a] L[x,j,o+b]`` and
   ``t[i,j,a,b] = (ia|jb) / (e_i + e_j - e_a - e_b)`` (MP2-like amplitudes;
   the denominator lies in [-10, -0.8], never zero).
5. ``L_vv = L[:, o:, o:]`` (contiguous ``[P][v][v]``),
   ``L_ov = L[:, :o, o:]`` (contiguous ``[P][o][v]``, occupied first) and
   ``L_oo = L[:, :o, :o]`` (contiguous ``[P][o][o]``).
6. With ``with_lambda``: ``G = 1e-2 * rng.standard_normal((o, o, v, v))`` and
   ``lam = (G + G.transpose(1, 0, 3, 2)) / 2`` (pair-symmetric), drawn after
   everything above.

All arrays are float64, C-contiguous, laid out as ``L[x][p][q]`` and
``t[i][j][a][b]``.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

__all__ = ["LadderInputs", "make_inputs", "paper_shape", "CONFIGS", "seed_for", "random_general",
           "integer_inputs", "random_ov", "integer_ov"]


@dataclass
class LadderInputs:
    o: int
    v: int
    P: int
    seed: int
    L_vv: np.ndarray          # [P][v][v]
    t: np.ndarray             # [o][o][v][v]
    e_occ: np.ndarray         # [o]
    e_vir: np.ndarray         # [v]
    ovov: np.ndarray          # (ia|jb) stored as [i][j][a][b]
    lam: Optional[np.ndarray] = None  # [o][o][v][v]
    L_ov: Optional[np.ndarray] = None  # [P][o][v]
    L_oo: Optional[np.ndarray] = None  # [P][o][o]


# Workload shapes: (o, v, P), named by their sizes: the brute-force tier
# (5/20/75), the first GPU parity tier (20/180/600), the throughput workload
# (40/360/1200), the adjoint workload (30/300/900) and the large single-GPU case
# (60/600/1800).
CONFIGS = {
    "o5_v20_P75": (5, 20, 75),
    "o20_v180_P600": (20, 180, 600),
    "o40_v360_P1200": (40, 360, 1200),
    "o30_v300_P900": (30, 300, 900),
    "o60_v600_P1800": (60, 600, 1800),
}


# One seed per workload, in the order above.
SEEDS = {name: 1001 + k for k, name in enumerate(CONFIGS)}


def seed_for(name: str) -> int:
    """The workload's seed (1001 ... 1005 in the order of CONFIGS)."""
    return SEEDS[name]


def paper_shape(K: int):
    """Orbital split of the paper's isolated-contraction benchmarks.

    v = int(3K/4), o = K - v and x = 5K Cholesky vectors (Sec. "Numerical
    results", setup of the contraction timings).
    """
    v = int(3 * K / 4)
    o = K - v
    return o, v, 5 * K


def _ovov(L_ov: np.ndarray, device=None) -> np.ndarray:
    """(ia|jb) = sum_x L[x,i,a] L[x,j,b], returned as [i][j][a][b]."""
    P, o, v = L_ov.shape
    if device is not None:
        import torch  # optional: only for large draws

        X = torch.from_numpy(np.ascontiguousarray(L_ov.reshape(P, o * v))).to(device)
        g = (X.T @ X).reshape(o, v, o, v).permute(0, 2, 1, 3).contiguous()
        return g.cpu().numpy()
    g = np.tensordot(L_ov, L_ov, axes=([0], [0]))  # [i][a][j][b]
    return np.ascontiguousarray(g.transpose(0, 2, 1, 3))


def make_inputs(o: int, v: int, P: int, seed: int, with_lambda: bool = False,
                device=None) -> LadderInputs:
    """Draw one workload.  ``device`` (a torch device) only speeds up the
    (ia|jb) product for large shapes; the arrays returned are host float64."""
    if min(o, v, P) <= 0:
        raise ValueError("o, v and P must be positive")
    rng = np.random.default_rng(seed)
    n = o + v
    L = rng.standard_normal((P, n, n))
    upper = np.triu(L)
    L = upper + np.transpose(np.triu(L, 1), (0, 2, 1))
    del upper
    L *= (np.exp(-np.arange(P, dtype=np.float64) / 25.0) / np.sqrt(n))[:, None, None]
    e_occ = np.sort(rng.uniform(-2.0, -0.3, o))
    e_vir = np.sort(rng.uniform(0.1, 3.0, v))
    L_ov = np.ascontiguousarray(L[:, :o, o:])
    ovov = _ovov(L_ov, device)
    D = (e_occ[:, None, None, None] + e_occ[None, :, None, None]
         - e_vir[None, None, :, None] - e_vir[None, None, None, :])
    t = ovov / D
    del D
    L_vv = np.ascontiguousarray(L[:, o:, o:])
    L_oo = np.ascontiguousarray(L[:, :o, :o])
    del L
    lam = None
    if with_lambda:
        G = 1e-2 * rng.standard_normal((o, o, v, v))
        lam = 0.5 * (G + G.transpose(1, 0, 3, 2))
        lam = np.ascontiguousarray(lam)
    return LadderInputs(o=o, v=v, P=P, seed=seed, L_vv=L_vv, t=np.ascontiguousarray(t),
                        e_occ=e_occ, e_vir=e_vir, ovov=ovov, lam=lam, L_ov=L_ov, L_oo=L_oo)


def integer_inputs(o: int, v: int, P: int, seed: int, lo: int = -2, hi: int = 2):
    """Small-integer L (not symmetrised) and t, exactly representable in every
    dtype the library computes in; sums stay exact while they are < 2**24."""
    rng = np.random.default_rng(seed)
    L = rng.integers(lo, hi + 1, size=(P, v, v)).astype(np.float64)
    t = rng.integers(lo, hi + 1, size=(o, o, v, v)).astype(np.float64)
    return L, t


def random_general(o: int, v: int, P: int, seed: int):
    """Unstructured N(0,1) L (not symmetric) and t (not pair-symmetric), and an
    unsymmetrised lambda: exercises every index role independently."""
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((P, v, v)) / np.sqrt(v)
    t = rng.standard_normal((o, o, v, v)) / v
    lam = rng.standard_normal((o, o, v, v)) / v
    return L, t, lam


def random_ov(o: int, v: int, P: int, seed: int):
    """Unstructured N(0,1)/sqrt(v) occupied-virtual Cholesky vectors [P][o][v]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((P, o, v)) / np.sqrt(v)


def integer_ov(o: int, v: int, P: int, seed: int, lo: int = -2, hi: int = 2):
    """Small-integer occupied-virtual Cholesky vectors [P][o][v]."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(P, o, v)).astype(np.float64)
