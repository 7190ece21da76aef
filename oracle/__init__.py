"""FP64 CPU oracle for the Cholesky-vector particle-particle ladder.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package: only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
call it.  It shares no code with the HIP path.

What it computes (arXiv 2310.04559):

* eq. (cholesky): the four-index integral is factorised through one set of
  Cholesky vectors, ``V[a,c,b,d] = (ac|bd) = sum_x L[x,a,c] L[x,b,d]``.
* eq. (vfunction): the ladder term of the doubles vector function,
  ``R[i,j,a,b] += sum_{c,d} V[a,c,b,d] t[i,j,c,d]``.
* The adjoint of that term for ``Loss = sum_{ijab} lam[i,j,a,b] R[i,j,a,b]``:
  ``dt[i,j,c,d] = sum_{a,b} lam[i,j,a,b] V[a,c,b,d]``;
  with ``W[a,b,c,d] = sum_{i,j} lam[i,j,a,b] t[i,j,c,d]``,
  ``dL[x,p,q] = sum_{b,d} W[p,b,q,d] L[x,b,d] + sum_{a,c} W[a,p,c,q] L[x,a,c]``
  (entrywise gradient: each array entry of L is an independent variable).
* eq. (vfunction2): the exchange partner ``R[i,j,a,b] += sum_{c,d} (ad|bc) t[i,j,c,d]``
  and its adjoint.
* eq. (vfunction3): ``X[i,j,k,l] += sum_{c,d} (kc|ld) t[i,j,c,d]`` and
  eq. (vfunction4): ``Y[i,j,b,k] += sum_{c,d} (bd|kc) t[i,j,c,d]``, with the
  occupied-virtual vectors ``L_ov[x][k][c]`` in ``(kc|ld) = sum_x L_ov[x,k,c] L_ov[x,l,d]``
  and ``(bd|kc) = sum_x L[x,b,d] L_ov[x,k,c]``.
* the hole-hole ladder that the paper's pCCD-LCCSD vector function also
  offloads (Sec. "Comparison between CPU and GPU-accelerated
  implementations", the contraction of order o^4 v^2):
  ``R[i,j,a,b] += sum_{k,l} (ik|jl) t[k,l,a,b]`` with
  ``(ik|jl) = sum_x L_oo[x,i,k] L_oo[x,j,l]``.  The paper gives only its
  einsum subscript; reading its first operand the way the paper translates a
  Cholesky operand ``abcd`` into ``xac,xbd`` gives this sum.

Algorithm: the definitions written out as sums, one library matrix product
per step, in float64.  The forward terms sum over the first contracted
virtual index ``c`` in an explicit loop: for each ``c`` the integrals
``(ac|bd)`` (or ``(ad|bc)``) for every ``a, b, d`` come from the Cholesky
vectors (eq. cholesky), and their product with ``t[:, :, c, :]`` over ``d`` is
added to the whole of ``R``.  The accumulation runs in place through BLAS
``dgemm`` with ``beta = 1`` (``_acc_product_nt``), so no temporary of R's size
is made.  The adjoint and the occupied-index terms loop over their first
output index instead, building that index's slice of the integral, which is
the same definition summed in another order.  There is no further blocking
or fusion.

Layouts: ``L[x][p][q]`` (the virtual-virtual block), ``L_ov[x][k][c]``,
``L_oo[x][i][k]``, ``t, R, lam[i][j][a][b]``, ``X[i][j][k][l]``,
``Y[i][j][b][k]``, all float64 C-contiguous.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg.blas import dgemm

__all__ = ["ladder_forward", "ladder_backward", "ladder_pairs", "ladder_row", "ladder_loss",
           "exchange_forward", "exchange_backward", "intermediate_ijkl", "intermediate_ijbk",
           "hole_ladder",
           "reduce_dot", "eri_slice", "nominal_flops_forward", "nominal_flops_backward",
           "nominal_flops_ijkl", "nominal_flops_ijbk", "nominal_flops_hole"]


def _check(L, t):
    L = np.asarray(L, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    if L.ndim != 3 or L.shape[1] != L.shape[2]:
        raise ValueError("L must be [P][v][v]")
    if t.ndim != 4 or t.shape[0] != t.shape[1] or t.shape[2] != t.shape[3]:
        raise ValueError("t must be [o][o][v][v]")
    if t.shape[2] != L.shape[1]:
        raise ValueError("L and t disagree on v")
    return L, t


def eri_slice(L: np.ndarray, a: int) -> np.ndarray:
    """``V[a, c, b, d]`` for one fixed ``a``, returned as ``[b][c][d]``
    (eq. cholesky restricted to one virtual index)."""
    P, v, _ = L.shape
    # [c][(b,d)] = sum_x L[x,a,c] * L[x,b,d]
    Vc_bd = L[:, a, :].T @ L.reshape(P, v * v)
    return Vc_bd.reshape(v, v, v).transpose(1, 0, 2)


def _acc_product_nt(C, A, Bt):
    """``C += A @ Bt.T`` in place for C-contiguous float64 ``C[m][n]``,
    ``A[m][k]``, ``Bt[n][k]``: BLAS ``dgemm`` with ``beta = 1`` on the
    column-major views (``C^T += Bt @ A^T``)."""
    out = dgemm(1.0, Bt.T, A.T, beta=1.0, c=C.T, trans_a=1, overwrite_c=1)
    if not np.shares_memory(out, C):
        raise RuntimeError("dgemm did not accumulate in place")


def ladder_forward(L, t, R=None, c_begin: int = 0, c_end=None) -> np.ndarray:
    """``R[i,j,a,b] += sum_{c,d} (ac|bd) t[i,j,c,d]`` (eq. vfunction) with
    ``(ac|bd) = sum_x L[x,a,c] L[x,b,d]`` (eq. cholesky).

    The sum over ``c`` is the explicit loop: per ``c``,
    ``Vc[(a,b), d] = (ac|bd)`` and ``R[(i,j),(a,b)] += sum_d t[i,j,c,d] Vc[(a,b),d]``.
    ``R`` is accumulated in place when given, else a zero array is made.
    ``[c_begin, c_end)`` restricts the sum over ``c`` (a bounded sample of the work)."""
    L, t = _check(L, t)
    P, v, _ = L.shape
    o = t.shape[0]
    if R is None:
        R = np.zeros((o, o, v, v))
    c_end = v if c_end is None else c_end
    R2 = R.reshape(o * o, v * v)
    if not np.shares_memory(R2, R):
        raise ValueError("R must be C-contiguous")
    Lf = L.reshape(P, v * v)                              # [x][(b,d)]
    for c in range(c_begin, c_end):
        Lc = np.ascontiguousarray(L[:, :, c])            # [x][a] = L[x,a,c]
        Vc = (Lc.T @ Lf).reshape(v * v, v)               # [(a,b)][d] = (ac|bd)
        Tc = np.ascontiguousarray(t[:, :, c, :]).reshape(o * o, v)   # [(i,j)][d]
        _acc_product_nt(R2, Tc, Vc)
    return R


def exchange_forward(L, t, R=None) -> np.ndarray:
    """Exchange partner of the ladder (eq. vfunction2):
    ``R[i,j,a,b] += sum_{c,d} (ad|bc) t[i,j,c,d]`` with
    ``(ad|bc) = sum_x L[x,a,d] L[x,b,c]``; the same explicit sum over ``c``:
    per ``c``, ``Xc[(a,b), d] = (ad|bc)``."""
    L, t = _check(L, t)
    P, v, _ = L.shape
    o = t.shape[0]
    if R is None:
        R = np.zeros((o, o, v, v))
    R2 = R.reshape(o * o, v * v)
    if not np.shares_memory(R2, R):
        raise ValueError("R must be C-contiguous")
    Lf = L.reshape(P, v * v)                              # [x][(a,d)]
    for c in range(v):
        Lc = np.ascontiguousarray(L[:, :, c])            # [x][b] = L[x,b,c]
        X = (Lc.T @ Lf).reshape(v, v, v)                 # [b][a][d] = (ad|bc)
        Xc = np.ascontiguousarray(X.transpose(1, 0, 2)).reshape(v * v, v)   # [(a,b)][d]
        Tc = np.ascontiguousarray(t[:, :, c, :]).reshape(o * o, v)
        _acc_product_nt(R2, Tc, Xc)
    return R


def exchange_backward(L, t, lam):
    """Entrywise ``(dL, dt)`` of ``sum lam * R`` with R the exchange term, from
    the definitions: with ``Y[a,b,c,d] = sum_{i,j} lam[i,j,a,b] t[i,j,c,d]``,
    ``dt[i,j,c,d] = sum_{a,b} lam[i,j,a,b] (ad|bc)``,
    ``dL[x,p,q] = sum_{b,c} Y[p,b,c,q] L[x,b,c] + sum_{a,d} Y[a,p,q,d] L[x,a,d]``."""
    L, t = _check(L, t)
    lam = np.asarray(lam, dtype=np.float64)
    P, v, _ = L.shape
    o = t.shape[0]
    T = t.reshape(o * o, v * v)
    Lf = L.reshape(P, v * v)
    dt = np.zeros((o * o, v * v))
    dL = np.zeros((P, v, v))
    for a in range(v):
        X = (L[:, a, :].T @ Lf).reshape(v, v, v)      # [d][b][c] = (ad|bc)
        lam_a = lam[:, :, a, :].reshape(o * o, v)     # [(i,j)][b]
        # dt[(i,j),(c,d)] += sum_b lam[i,j,a,b] (ad|bc)
        dt += lam_a @ X.transpose(1, 2, 0).reshape(v, v * v)
        Ya = (lam_a.T @ T).reshape(v, v, v)          # [b][c][d] = Y[a,b,c,d]
        # dL[x,a,d] += sum_{b,c} L[x,b,c] Y[a,b,c,d]
        dL[:, a, :] += Lf @ Ya.reshape(v * v, v)
        # dL[x,b,c] += sum_d L[x,a,d] Y[a,b,c,d]
        dL += np.einsum("xd,bcd->xbc", L[:, a, :], Ya)
    return dL, dt.reshape(o, o, v, v)


def _check_ov(L_ov, t):
    L_ov = np.asarray(L_ov, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    if L_ov.ndim != 3 or t.ndim != 4 or t.shape[0] != t.shape[1] or t.shape[2] != t.shape[3]:
        raise ValueError("L_ov must be [P][o][v] and t [o][o][v][v]")
    if L_ov.shape[1] != t.shape[0] or L_ov.shape[2] != t.shape[2]:
        raise ValueError("L_ov and t disagree on o or v")
    return L_ov, t


def intermediate_ijkl(L_ov, t, X=None, k_begin: int = 0, k_end=None) -> np.ndarray:
    """``X[i,j,k,l] += sum_{c,d} (kc|ld) t[i,j,c,d]`` (eq. vfunction3), with
    ``(kc|ld) = sum_x L_ov[x,k,c] L_ov[x,l,d]``; loop over the occupied ``k``,
    building ``(kc|ld)`` for one ``k`` at a time.  ``[k_begin, k_end)``
    restricts the loop (a bounded sample)."""
    L_ov, t = _check_ov(L_ov, t)
    P, o, v = L_ov.shape
    if X is None:
        X = np.zeros((o, o, o, o))
    k_end = o if k_end is None else k_end
    T = t.reshape(o * o, v * v)                       # [(i,j)][(c,d)]
    Lf = L_ov.reshape(P, o * v)
    for k in range(k_begin, k_end):
        G = (L_ov[:, k, :].T @ Lf).reshape(v, o, v)   # [c][l][d] = (kc|ld)
        Gk = G.transpose(1, 0, 2).reshape(o, v * v)   # [l][(c,d)]
        X[:, :, k, :] += (T @ Gk.T).reshape(o, o, o)
    return X


def intermediate_ijbk(L, L_ov, t, Y=None, b_begin: int = 0, b_end=None) -> np.ndarray:
    """``Y[i,j,b,k] += sum_{c,d} (bd|kc) t[i,j,c,d]`` (eq. vfunction4), with
    ``(bd|kc) = sum_x L[x,b,d] L_ov[x,k,c]``; loop over the virtual ``b``.
    ``[b_begin, b_end)`` restricts the loop (a bounded sample)."""
    L, t = _check(L, t)
    L_ov, _ = _check_ov(L_ov, t)
    P, o, v = L_ov.shape
    if L.shape[0] != P:
        raise ValueError("L and L_ov disagree on P")
    if Y is None:
        Y = np.zeros((o, o, v, o))
    b_end = v if b_end is None else b_end
    T = t.reshape(o * o, v * v)
    Lf = L_ov.reshape(P, o * v)
    for b in range(b_begin, b_end):
        G = (L[:, b, :].T @ Lf).reshape(v, o, v)      # [d][k][c] = (bd|kc)
        Gb = G.transpose(1, 2, 0).reshape(o, v * v)   # [k][(c,d)]
        Y[:, :, b, :] += (T @ Gb.T).reshape(o, o, o)
    return Y


def hole_ladder(L_oo, t, R=None, i_begin: int = 0, i_end=None) -> np.ndarray:
    """``R[i,j,a,b] += sum_{k,l} (ik|jl) t[k,l,a,b]`` with
    ``(ik|jl) = sum_x L_oo[x,i,k] L_oo[x,j,l]``; loop over the occupied ``i``,
    building ``(ik|jl)`` for one ``i`` at a time.  ``[i_begin, i_end)``
    restricts the loop (a bounded sample)."""
    L_oo = np.asarray(L_oo, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    if L_oo.ndim != 3 or L_oo.shape[1] != L_oo.shape[2]:
        raise ValueError("L_oo must be [P][o][o]")
    if t.ndim != 4 or t.shape[0] != t.shape[1] or t.shape[2] != t.shape[3]:
        raise ValueError("t must be [o][o][v][v]")
    if t.shape[0] != L_oo.shape[1]:
        raise ValueError("L_oo and t disagree on o")
    P, o, _ = L_oo.shape
    v = t.shape[2]
    if R is None:
        R = np.zeros((o, o, v, v))
    i_end = o if i_end is None else i_end
    T = t.reshape(o * o, v * v)                       # [(k,l)][(a,b)]
    Lf = L_oo.reshape(P, o * o)
    for i in range(i_begin, i_end):
        G = (L_oo[:, i, :].T @ Lf).reshape(o, o, o)   # [k][j][l] = (ik|jl)
        Gi = G.transpose(1, 0, 2).reshape(o, o * o)   # [j][(k,l)]
        R[i] += (Gi @ T).reshape(o, v, v)
    return R


def ladder_backward(L, t, lam):
    """Entrywise gradients ``(dL, dt)`` of ``sum lam * R`` with R the ladder
    term; one pass over ``a`` as in the forward, V[a] rebuilt, not stored."""
    L, t = _check(L, t)
    lam = np.asarray(lam, dtype=np.float64)
    P, v, _ = L.shape
    o = t.shape[0]
    if lam.shape != t.shape:
        raise ValueError("lam must match t")
    T = t.reshape(o * o, v * v)
    Lf = L.reshape(P, v * v)
    dt = np.zeros((o * o, v * v))
    dL = np.zeros((P, v, v))
    for a in range(v):
        Va = eri_slice(L, a)                          # [b][c][d]
        lam_a = lam[:, :, a, :].reshape(o * o, v)     # [(i,j)][b]
        # dt[(i,j),(c,d)] += sum_b lam[i,j,a,b] V[a,c,b,d]
        dt += lam_a @ Va.reshape(v, v * v)
        # W[a,b,(c,d)] = sum_{(i,j)} lam[i,j,a,b] t[i,j,c,d]
        Wa = (lam_a.T @ T).reshape(v, v, v)          # [b][c][d]
        Wa_cbd = Wa.transpose(1, 0, 2).reshape(v, v * v)   # [c][(b,d)]
        # first term: dL[x,a,c] += sum_{b,d} L[x,b,d] W[a,b,c,d]
        dL[:, a, :] += Lf @ Wa_cbd.T
        # second term: dL[x,b,d] += sum_c L[x,a,c] W[a,b,c,d]
        dL += (L[:, a, :] @ Wa_cbd).reshape(P, v, v)
    return dL, dt.reshape(o, o, v, v)


def ladder_pairs(L, t, pairs) -> np.ndarray:
    """``R[:, :, a, b]`` of the ladder term for each ``(a, b)`` in ``pairs``,
    one at a time from the definition: ``V[a,:,b,:]`` from eq. cholesky, then
    the (c,d) sum of eq. vfunction.  Returns ``[len(pairs)][o][o]``."""
    L, t = _check(L, t)
    P, v, _ = L.shape
    o = t.shape[0]
    T = t.reshape(o * o, v * v)
    out = np.empty((len(pairs), o, o))
    for k, (a, b) in enumerate(pairs):
        Vab = L[:, a, :].T @ L[:, b, :]               # [c][d]
        out[k] = (T @ Vab.reshape(v * v)).reshape(o, o)
    return out


def ladder_row(L, t, i: int, j: int) -> np.ndarray:
    """``R[i, j, :, :]`` of the ladder term for one occupied pair, from eq.
    cholesky and eq. vfunction regrouped per Cholesky vector:
    ``R[i,j,a,b] = sum_x sum_c L[x,a,c] sum_d t[i,j,c,d] L[x,b,d]``, i.e.
    ``sum_x L_x t_ij L_x^T``.  Returns ``[v][v]``."""
    L, t = _check(L, t)
    T = t[i, j]
    out = np.zeros((L.shape[1], L.shape[1]))
    for x in range(L.shape[0]):
        out += L[x] @ T @ L[x].T
    return out


def ladder_loss(lam, R) -> float:
    """``sum_{ijab} lam[i,j,a,b] R[i,j,a,b]``."""
    return float(np.dot(np.ravel(lam), np.ravel(R)))


def reduce_dot(x, y):
    """``(sum x*y, sum y*y)`` in float64."""
    xf = np.ravel(np.asarray(x, dtype=np.float64))
    yf = np.ravel(np.asarray(y, dtype=np.float64))
    return float(np.dot(xf, yf)), float(np.dot(yf, yf))


def nominal_flops_forward(o: int, v: int, P: int) -> float:
    """Factorised cost of one forward: 2 P v^4 (integral slices) + 2 o^2 v^4
    (amplitude contraction)."""
    return 2.0 * (P + o * o) * float(v) ** 4


def nominal_flops_ijkl(o: int, v: int, P: int) -> float:
    """Integrals (kc|ld) for all k, l (2 P o^2 v^2) + contraction (2 o^4 v^2)."""
    return 2.0 * (P + o * o) * float(o * v) ** 2


def nominal_flops_ijbk(o: int, v: int, P: int) -> float:
    """Integrals (bd|kc) (2 P o v^3) + contraction (2 o^3 v^3)."""
    return 2.0 * (P + o * o) * o * float(v) ** 3


def nominal_flops_hole(o: int, v: int, P: int) -> float:
    """Integrals (ik|jl) (2 P o^4) + contraction (2 o^4 v^2)."""
    return 2.0 * (P + v * v) * float(o) ** 4


def nominal_flops_backward(o: int, v: int, P: int) -> float:
    """Rebuild (2Pv^4) + dt (2o^2v^4) + W (2o^2v^4) + two dL terms (2Pv^4 each)."""
    return (6.0 * P + 4.0 * o * o) * float(v) ** 4
