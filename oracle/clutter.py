"""Oracle: eigen-based SVD clutter filter of a Casorati matrix (FP64, CPU).

TEST INFRASTRUCTURE ONLY.

Section II-A2: the spatiotemporal (Casorati) matrix I in C^{n x n_t} stacks
each frame as a column.  The eigen-based filter computes the covariance
C = I^H I (n_t x n_t), takes its eigendecomposition, and removes the
projection onto the clutter subspace spanned by the eigenvectors of the
largest eigenvalues: I_f = I - (I V_c) V_c^H.  The cutoff is a fixed count c
of removed modes (a reading: the paper gives no cutoff rule).

The projection stack layout is [F][n_pix] (frame-major), i.e. the transpose
of the Casorati matrix; every function below builds the Casorati matrix
explicitly so the arithmetic reads as in the paper.
"""
from __future__ import annotations

import numpy as np


def casorati(stack) -> np.ndarray:
    """[F][n_pix] stack -> Casorati matrix I (n_pix x F), complex128."""
    s = np.asarray(stack)
    return np.ascontiguousarray(s.reshape(s.shape[0], -1).T.astype(np.complex128))


def covariance(stack) -> np.ndarray:
    """C = I^H I (F x F, Hermitian)."""
    I = casorati(stack)
    return I.conj().T @ I


def clutter_subspace(C, cutoff: int):
    """Eigenvalues sorted descending and the top-`cutoff` eigenvectors V_c (F x c)."""
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    V = V[:, order]
    return lam, V[:, :cutoff]


def clutter_filter(stack, cutoff: int):
    """Eigen route.  Returns (filtered stack [F][...] complex128, eigenvalues desc)."""
    s = np.asarray(stack)
    I = casorati(s)
    lam, Vc = clutter_subspace(I.conj().T @ I, cutoff)
    If = I - (I @ Vc) @ Vc.conj().T
    return If.T.reshape(s.shape), lam


def clutter_filter_svd(stack, cutoff: int):
    """Direct SVD route (reference for the eigen route): I - U_c S_c V_c^H."""
    s = np.asarray(stack)
    I = casorati(s)
    U, sv, Vh = np.linalg.svd(I, full_matrices=False)
    If = I - (U[:, :cutoff] * sv[:cutoff]) @ Vh[:cutoff]
    return If.T.reshape(s.shape), sv


def filter_planes(proj, cutoff: int):
    """Apply the filter to every plane of P[o][b][f][z][u]; returns (filtered, eig[o][b][F])."""
    P = np.asarray(proj)
    out = np.empty(P.shape, dtype=np.complex128)
    eig = np.empty(P.shape[:3], dtype=np.float64)
    for o in range(P.shape[0]):
        for b in range(P.shape[1]):
            out[o, b], eig[o, b] = clutter_filter(P[o, b], cutoff)
    return out, eig
