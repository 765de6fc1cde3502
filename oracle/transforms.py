"""Eigenfunction expansions along the homogeneous direction (Table 1, Sec. 2).

For n cells on a uniform staggered grid the 1D second difference with
homogeneous conditions at the two ends has eigenvalues

    lambda_q = 2 (cos(kappa_q dl) - 1),  q = 0..n-1,

with kappa_q dl = 2 pi k_q / n and k_q = q (periodic), q/2 (Neumann-Neumann),
(q+1)/2 (Dirichlet-Dirichlet), (2q+1)/4 (Neumann-Dirichlet) per Table 1.  The
Dirichlet-Neumann pair, not printed in Table 1 but covered by the paper's claim
that every valid combination is supported, has the same eigenvalues as
Neumann-Dirichlet with the sine counterpart of the DCT-IV basis.

The eigenvectors are written out by their closed-form definitions, scaled to
be orthonormal (the paper's FFTW forms are unnormalised; ``table1_unnormalised``
builds those and the tests check the theta factors of Table 1 separately).
For the periodic pair the real orthonormal basis used is the discrete Hartley
one, cas(2 pi q j / n) / sqrt(n); it carries the eigenvalue of index q in
position q exactly like the DFT.
"""
from __future__ import annotations

import numpy as np

KINDS = ("PP", "NN", "DD", "ND", "DN")


def _k(kind: str, n: int) -> np.ndarray:
    q = np.arange(n, dtype=np.float64)
    if kind == "PP":
        return q
    if kind == "NN":
        return q / 2.0
    if kind == "DD":
        return (q + 1.0) / 2.0
    if kind in ("ND", "DN"):
        return (2.0 * q + 1.0) / 4.0
    raise ValueError(kind)


def eigenvalues(kind: str, n: int) -> np.ndarray:
    """lambda_q of Table 1 (dimensionless: multiply by 1/dz^2 for the shift)."""
    return 2.0 * (np.cos(2.0 * np.pi * _k(kind, n) / n) - 1.0)


def basis(kind: str, n: int) -> np.ndarray:
    """Orthonormal eigenvector matrix T with T[j, q] = phi_q(j).

    Forward transform: fhat = T.T @ f (along the cell index j); inverse:
    f = T @ fhat.
    """
    j = np.arange(n, dtype=np.float64)[:, None] + 0.5  # cell centres in units of dl
    q = np.arange(n, dtype=np.float64)[None, :]
    if kind == "PP":
        jj = np.arange(n, dtype=np.float64)[:, None]
        th = 2.0 * np.pi * q * jj / n
        return (np.cos(th) + np.sin(th)) / np.sqrt(n)
    if kind == "NN":
        T = np.cos(np.pi * q * j / n) * np.sqrt(2.0 / n)
        T[:, 0] = 1.0 / np.sqrt(n)
        return T
    if kind == "DD":
        T = np.sin(np.pi * (q + 1.0) * j / n) * np.sqrt(2.0 / n)
        T[:, n - 1] /= np.sqrt(2.0)
        return T
    if kind == "ND":
        return np.cos(np.pi * (q + 0.5) * j / n) * np.sqrt(2.0 / n)
    if kind == "DN":
        return np.sin(np.pi * (q + 0.5) * j / n) * np.sqrt(2.0 / n)
    raise ValueError(kind)


def table1_unnormalised(kind: str, n: int):
    """(F, B, theta): unnormalised forward and backward transform matrices.

    These are the standard unnormalised DFT / DCT / DST definitions named in
    Table 1 (forward F maps values to coefficients, backward B maps back), so
    that B @ F = theta * I with theta = n (periodic) or 2n (the others).
    """
    jj = np.arange(n, dtype=np.float64)
    qq = np.arange(n, dtype=np.float64)
    if kind == "PP":
        F = np.exp(-2j * np.pi * np.outer(qq, jj) / n)
        B = np.exp(2j * np.pi * np.outer(jj, qq) / n)
        return F, B, n
    if kind == "NN":  # DCT-II forward, DCT-III backward
        F = 2.0 * np.cos(np.pi * np.outer(qq, jj + 0.5) / n)
        B = 2.0 * np.cos(np.pi * np.outer(jj + 0.5, qq) / n)
        B[:, 0] = 1.0
        return F, B, 2 * n
    if kind == "DD":  # DST-II forward, DST-III backward
        F = 2.0 * np.sin(np.pi * np.outer(qq + 1.0, jj + 0.5) / n)
        B = 2.0 * np.sin(np.pi * np.outer(jj + 0.5, qq + 1.0) / n)
        B[:, n - 1] = (-1.0) ** jj
        return F, B, 2 * n
    if kind == "ND":  # DCT-IV both ways
        F = 2.0 * np.cos(np.pi * np.outer(qq + 0.5, jj + 0.5) / n)
        return F, F.T.copy(), 2 * n
    if kind == "DN":  # DST-IV both ways
        F = 2.0 * np.sin(np.pi * np.outer(qq + 0.5, jj + 0.5) / n)
        return F, F.T.copy(), 2 * n
    raise ValueError(kind)
