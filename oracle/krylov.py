"""Arnoldi with incomplete orthogonalisation (Alg 1).  Test infrastructure only.

Alg 1 builds v_1 = v / ||v|| and, for m = 1, 2, ..., forms w = Q~ v_m and
orthogonalises it by modified Gram-Schmidt against the two newest basis
vectors (v_{m-1} then v_m), storing the coefficients in column m of the upper
Hessenberg H; h_{m+1,m} = ||w||, the loop stops when that falls below tol,
otherwise v_{m+1} = w / h_{m+1,m}.

Here the window length is a parameter k >= 1 (the paper's method is k = 2;
k >= m_max is full single-pass MGS, i.e. Lanczos with full
re-orthogonalisation for symmetric Q): column t is orthogonalised against
v_j for j = max(1, t-k+1), ..., t, oldest first, each coefficient taken from
the already-updated w.

Reading of the exit (the algorithm's final "H(1:m,1:m)" is one row/column
past the loop when no breakdown happens): the effective dimension m_eff is
the number of mat-vecs performed, m_eff = min(m_exit, m_max); a breakdown at
step t (h_{t+1,t} < tol) gives m_eff = t and keeps column t.
"""
from __future__ import annotations

import numpy as np


def windowed_arnoldi(apply_op, v, m_max: int, window: int, tol: float):
    """Run the recurrence from start vector v.

    Returns (H, beta0, V, m_eff, broke):
      H      (m_eff x m_eff) float64 upper-Hessenberg projection,
      beta0  ||v||_2,
      V      list of the m_eff basis vectors v_1..v_{m_eff},
      m_eff  number of mat-vecs performed,
      broke  True when the run stopped on h_{t+1,t} < tol.
    """
    v = np.asarray(v, dtype=np.float64)
    beta0 = float(np.linalg.norm(v))
    basis = [v / beta0]
    hfull = np.zeros((m_max + 1, m_max), dtype=np.float64)
    for t in range(m_max):  # 0-based column index; the paper's m = t + 1
        w = apply_op(basis[t])
        for j in range(max(0, t - window + 1), t + 1):
            hjt = float(basis[j] @ w)
            hfull[j, t] = hjt
            w = w - hjt * basis[j]
        h = float(np.linalg.norm(w))
        hfull[t + 1, t] = h
        if h < tol:
            m_eff = t + 1
            return hfull[:m_eff, :m_eff].copy(), beta0, basis[:m_eff], m_eff, True
        basis.append(w / h)
    return hfull[:m_max, :m_max].copy(), beta0, basis[:m_max], m_max, False
