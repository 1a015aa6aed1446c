"""Tensor algebra of the Kronecker-sum structure (oracle; test infrastructure only).

Tensors are numpy arrays in natural index order V[i_1, ..., i_d]; mode mu is
numpy axis mu-1.  vec() stacks columns: first index fastest (section 1, the
text after eq. tuckerexp), which is numpy's Fortran order.
"""

from __future__ import annotations

import itertools
from typing import Sequence

import numpy as np


def vec(V: np.ndarray) -> np.ndarray:
    """vec(V): column stacking, first index fastest."""
    return np.asarray(V).ravel(order="F")


def unvec(v: np.ndarray, n: Sequence[int]) -> np.ndarray:
    return np.asarray(v).reshape(tuple(n), order="F")


def mode_product(V: np.ndarray, M: np.ndarray, mu: int) -> np.ndarray:
    """mu-mode product V x_mu M (mu is 1-based).

    (V x_mu M)[i_1..i_mu..i_d] = sum_j M[i_mu, j] V[i_1..j..i_d], the
    contraction that eq. forloop spells out element by element."""
    out = np.tensordot(M, V, axes=([1], [mu - 1]))  # axis 0 is i_mu, the rest keep V's order
    return np.moveaxis(out, 0, mu - 1)


def tucker(V: np.ndarray, Ms: Sequence[np.ndarray]) -> np.ndarray:
    """Tucker operator V x_1 M_1 x_2 M_2 ... x_d M_d (eq. tuckerexp)."""
    out = V
    for mu, M in enumerate(Ms, start=1):
        out = mode_product(out, M, mu)
    return out


def kron_sum_action(U: np.ndarray, As: Sequence[np.ndarray]) -> np.ndarray:
    """K u in tensor form, sum_mu U x_mu A_mu, without assembling K (section 3.2)."""
    out = np.zeros(np.shape(U), dtype=np.result_type(U, *As))
    for mu, A in enumerate(As, start=1):
        out = out + mode_product(U, A, mu)
    return out


def dense_kron_sum(As: Sequence[np.ndarray]) -> np.ndarray:
    """K = A_d (+) ... (+) A_1 = sum_mu I_d (x) .. (x) A_mu (x) .. (x) I_1 (eq. kronsum).

    Brute force for tiny sizes only."""
    d = len(As)
    ns = [A.shape[0] for A in As]
    N = int(np.prod(ns))
    K = np.zeros((N, N), dtype=np.result_type(*As))
    for mu in range(d):
        # factors are listed from direction d down to direction 1
        factors = [As[nu] if nu == mu else np.eye(ns[nu]) for nu in reversed(range(d))]
        term = factors[0]
        for f in factors[1:]:
            term = np.kron(term, f)
        K = K + term
    return K


def dense_kron_product(Ms: Sequence[np.ndarray]) -> np.ndarray:
    """M_d (x) ... (x) M_1 (the right-hand side of eq. vecexp); tiny sizes only."""
    out = Ms[-1]
    for M in reversed(Ms[:-1]):
        out = np.kron(out, M)
    return out


def forloop_tucker(V: np.ndarray, Ms: Sequence[np.ndarray]) -> np.ndarray:
    """Element-by-element evaluation of eq. forloop (pure Python; tiny sizes only)."""
    n = V.shape
    out = np.zeros(n, dtype=np.result_type(V, *Ms))
    for i in itertools.product(*[range(k) for k in n]):
        acc = 0.0
        for j in itertools.product(*[range(k) for k in n]):
            w = V[j]
            for mu in range(len(n)):
                w = w * Ms[mu][i[mu], j[mu]]
            acc += w
        out[i] = acc
    return out


def tucker_entry(V: np.ndarray, Ms: Sequence[np.ndarray], i: Sequence[int]):
    """One entry of the Tucker operator by eq. forloop:
    sum_j M_1[i_1, j_1] ... M_d[i_d, j_d] V[j_1, ..., j_d], contracting mode 1
    first (each step a library matrix-vector product over one index; the
    column-stacked layout of the tensors makes every step a view).  Also returns
    the same sum over absolute values, which bounds its rounding error."""
    w, a = np.asarray(V), np.abs(V)
    for mu in range(len(Ms)):
        rest = w.shape[1:]
        w = (Ms[mu][i[mu], :] @ w.reshape(w.shape[0], -1, order="F")).reshape(rest, order="F")
        a = (np.abs(Ms[mu][i[mu], :]) @ a.reshape(a.shape[0], -1, order="F")).reshape(rest, order="F")
    return w[()], a[()]
