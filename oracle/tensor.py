"""mu-mode products, Tucker operators and Kronecker-sum actions (oracle, FP64).

Sec. 2: for an order-d tensor W of size n_1 x ... x n_d, the mu-mode product
W x_mu M multiplies the n_mu x n_mu matrix M onto every mu-fibre of W:

    (W x_mu M)[i_1, .., i_mu, .., i_d] = sum_k M[i_mu, k] W[i_1, .., k, .., i_d].

The Tucker operator (eq. (5)) is the chain W x_1 M_1 x_2 ... x_d M_d, and the
action of a Kronecker sum on vec(W) is sum_mu W x_mu A_mu (eq. (6) and the
identity that follows it).  vec stacks the first index fastest, i.e. Fortran
order.  Direction mu of the paper is axis mu-1 here.

Parity: pinned by tests/test_oracle_tensor.py (pure-Python loops on tiny
tensors, vec(W x_1 M_1 ... x_d M_d) = (M_d x ... x M_1) vec(W) with numpy.kron,
the 2D form M_1 W M_2^T).
"""
from __future__ import annotations

import numpy as np


def vec(W: np.ndarray) -> np.ndarray:
    """Stack the entries of W with the first index fastest."""
    return np.asarray(W).reshape(-1, order="F")


def unvec(w: np.ndarray, shape) -> np.ndarray:
    return np.asfortranarray(np.asarray(w).reshape(tuple(shape), order="F"))


def mode_product(W: np.ndarray, M: np.ndarray, mu: int) -> np.ndarray:
    """W x_mu M  (axis ``mu`` is 0-based: paper direction mu+1)."""
    if M.shape != (W.shape[mu], W.shape[mu]):
        raise ValueError("matrix size must match the mu-th tensor dimension")
    # tensordot contracts M's column index with W's axis mu and puts the
    # new index first; move it back into position mu
    out = np.tensordot(M, W, axes=([1], [mu]))
    return np.moveaxis(out, 0, mu)


def tucker(W: np.ndarray, Ms, order=None) -> np.ndarray:
    """W x_1 M_1 x_2 M_2 ... x_d M_d  (eq. (5)), applied in the order mu = 1..d.

    ``order`` (a permutation of the 0-based directions) applies the same
    products in another order.  Mode products along different directions
    commute (each acts on its own index), so every order gives the same
    operator; only the rounding differs.  Used to measure how far rounding
    alone moves a long run."""
    out = W
    for mu in (range(len(Ms)) if order is None else order):
        out = mode_product(out, Ms[mu], mu)
    return np.asfortranarray(out)


def kron_sum_action(W: np.ndarray, As) -> np.ndarray:
    """sum_mu W x_mu A_mu = unvec(K vec(W)) with K = A_d (+) ... (+) A_1 (eq. (6))."""
    acc = np.zeros(W.shape)
    for mu, A in enumerate(As):
        acc = acc + mode_product(W, A, mu)
    return np.asfortranarray(acc)
