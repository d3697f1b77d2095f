"""Brute-force matrix form of the whole recurrence for tiny grids.

An independent construction used to pin the oracle's loop code: the 3-D
operators are assembled from Kronecker products of 1-D band matrices
(zero values beyond the faces = the bands are simply truncated), and a time
step is a dense matrix-vector product on the state (u^n, u^{n-1}, phi^n).
It shares nothing with the oracle's C loops except the readings they both
follow (Eq. 2-3 of the paper plus the layer update stated in the oracle's
header).  Stencil weights are derived here from the Taylor conditions
(exactness on even monomials up to degree 8), not copied from the oracle.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def second_difference_weights(r: int = 4):
    """Weights C_0..C_r of the symmetric 2r+1 point second difference that is
    exact for polynomials of degree <= 2r+1: solve
    sum_{m=-r..r} C_|m| m^(2q) = 2 [q == 1], q = 0..r, in exact rationals."""
    n = r + 1
    A = [[Fraction(0)] * n for _ in range(n)]
    b = [Fraction(0)] * n
    for q in range(n):
        for m in range(n):
            A[q][m] = Fraction(1) if (m == 0 and q == 0) else (
                Fraction(0) if m == 0 else Fraction(2) * Fraction(m) ** (2 * q))
        b[q] = Fraction(2) if q == 1 else Fraction(0)
    # Gaussian elimination in rationals
    for i in range(n):
        piv = next(r_ for r_ in range(i, n) if A[r_][i] != 0)
        A[i], A[piv] = A[piv], A[i]
        b[i], b[piv] = b[piv], b[i]
        for r_ in range(n):
            if r_ != i and A[r_][i] != 0:
                f = A[r_][i] / A[i][i]
                A[r_] = [x - f * y for x, y in zip(A[r_], A[i])]
                b[r_] = b[r_] - f * b[i]
    return [b[i] / A[i][i] for i in range(n)]


def d2_matrix(n: int, h: float, C) -> np.ndarray:
    M = np.zeros((n, n))
    for i in range(n):
        for m in range(-4, 5):
            j = i + m
            if 0 <= j < n:
                M[i, j] = float(C[abs(m)]) / (h * h)
    return M


def d1_matrix(n: int) -> np.ndarray:
    """u(i+1) - u(i-1) with zero beyond the ends."""
    M = np.zeros((n, n))
    for i in range(n):
        if i + 1 < n:
            M[i, i + 1] = 1.0
        if i - 1 >= 0:
            M[i, i - 1] = -1.0
    return M


def operators(nx, ny, nz, dx, dy, dz):
    """3-D Laplacian and the three first-difference operators on the
    x-fastest ordering p = (k ny + j) nx + i."""
    C = second_difference_weights(4)
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    Lx = np.kron(Iz, np.kron(Iy, d2_matrix(nx, dx, C)))
    Ly = np.kron(Iz, np.kron(d2_matrix(ny, dy, C), Ix))
    Lz = np.kron(d2_matrix(nz, dz, C), np.kron(Iy, Ix))
    Gx = np.kron(Iz, np.kron(Iy, d1_matrix(nx)))
    Gy = np.kron(Iz, np.kron(d1_matrix(ny), Ix))
    Gz = np.kron(d1_matrix(nz), np.kron(Iy, Ix))
    return Lx + Ly + Lz, (Gx, Gy, Gz)


def run(nx, ny, nz, w, dx, dy, dz, vp, eta, src, wavelet, steps, inner_mask):
    """Advance `steps` steps from zero with the dense matrix form.
    vp, eta: flat float64 arrays (x fastest); inner_mask: bool flat array.
    Returns (u^T, u^{T-1}, phi^T) flat."""
    L, G = operators(nx, ny, nz, dx, dy, dz)
    h2 = (dx * dx, dy * dy, dz * dz)
    N = nx * ny * nz
    layer = ~inner_mask
    # gradient coefficients of eta per axis (a fixed vector: eta is static)
    ge = [G[a] @ eta / (4.0 * h2[a]) for a in range(3)]
    u = np.zeros(N)
    up = np.zeros(N)
    ph = np.zeros(N)
    a_coef = 2.0 + 2.0 * eta - eta * eta
    den = 1.0 + 2.0 * eta
    for n in range(steps):
        Lu = L @ u
        un_inner = 2.0 * u - up + vp * Lu
        un_layer = (a_coef * u - up + vp * (Lu + ph)) / den
        un = np.where(layer, un_layer, un_inner)
        gsum = sum(ge[a] * (G[a] @ u) for a in range(3))
        phn = np.where(layer, (ph - gsum) / (1.0 + eta), ph)
        for s, (i, j, k) in enumerate(src):
            p = (k * ny + j) * nx + i
            wv = wavelet[s][n] if n < len(wavelet[s]) else 0.0
            un[p] += vp[p] * wv
        up, u, ph = u, un, phn
    return u, up, ph
