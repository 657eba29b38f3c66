"""Independent dense references used to pin the oracle (test support only).

Nothing here imports the oracle or the GPU library.  The routines rebuild the
objects of the method from their mathematical definitions with different
machinery (exact rationals, dense matrices, LAPACK eigensolvers, Bloch
Hamiltonians) so that a mistake in the oracle shows up as a disagreement:

* FD weights as exact rationals from the Taylor conditions (not from the
  closed form of Sec. 3.1);
* the nodal Hamiltonian as an explicit dense matrix (Sec. 3.1, region of
  influence; zero Dirichlet outside the cube);
* moments e^T T_j(Hhat) e from a full eigendecomposition (Sec. 3.2);
* the periodic Bloch Hamiltonian H(k) for Brillouin-zone integrated densities,
  the infinite-crystal limit the infinite-cell method approaches.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def fd_weights_taylor(no: int) -> list[Fraction]:
    """Central second-derivative weights of order 2 no from the moment
    conditions sum_d d^{2p} c_d = delta_{p,1} (p = 0..no), solved exactly.

    Returns [w_0, w_1, ..., w_no] for unit spacing, with the convention of
    Sec. 3.1: the 1D second derivative is w_0 f_0 + sum_d w_d (f_d + f_-d)
    where the *per-axis* centre weight is 2 w_0 (so that 3 axes give 6 w_0)."""
    # unknowns: c_0 (full centre weight of the 1D stencil), c_1..c_no (pair weights)
    n = no + 1
    A = [[Fraction(0)] * n for _ in range(n)]
    b = [Fraction(0)] * n
    for p in range(n):
        A[p][0] = Fraction(1) if p == 0 else Fraction(0)
        for d in range(1, n):
            A[p][d] = Fraction(2 * d ** (2 * p))
        b[p] = Fraction(2) if p == 1 else Fraction(0)   # second derivative of x^2/... -> 2 / 2!
    # Gaussian elimination over the rationals
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                b[r] -= f * b[col]
    c = [b[i] / A[i][i] for i in range(n)]
    # the conditions above give f''(0) * 1 for f = x^2 (sum d^2 c_d * 2 = 2)
    return [c[0] / 2] + c[1:]


def grid_n(cell: float, h: float) -> int:
    return int(math.floor(cell / h + 0.5))


def projector_tables(atoms, kb, h):
    """Per atom: integer grid coordinates (infinite grid) and normalised values."""
    out = []
    for R, (sig, rc, gam) in zip(np.asarray(atoms, float), np.asarray(kb, float)):
        lo = np.floor((R - rc) / h).astype(int) - 2
        hi = np.ceil((R + rc) / h).astype(int) + 2
        ii, jj, kk = np.meshgrid(*[np.arange(lo[a], hi[a] + 1) for a in range(3)], indexing="ij")
        ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)
        d = ijk * h - R
        r2 = (d ** 2).sum(1)
        keep = r2 <= rc * rc
        ijk = ijk[keep]
        chi = np.exp(-r2[keep] / (2 * sig * sig))
        p = chi / math.sqrt(h ** 3 * (chi ** 2).sum())
        out.append((ijk, p, gam))
    return out


def kinetic_1d(C: int, w) -> np.ndarray:
    """(C x C) Dirichlet-truncated 1D block of -1/2 d^2/dx^2 (diag -w0, the
    3D diagonal being the sum of three such blocks)."""
    K = np.zeros((C, C))
    no = len(w) - 1
    for a in range(C):
        K[a, a] = -0.5 * 2 * float(w[0])
        for d in range(1, no + 1):
            for b in (a - d, a + d):
                if 0 <= b < C:
                    K[a, b] = -0.5 * float(w[d])
    return K


def dense_hq(n, h, m, w, veff, tables, q):
    """Explicit nodal Hamiltonian of node q (infinite-cell, Sec. 3.1)."""
    C = 2 * m + 1
    qi, qj, qk = q % n, (q // n) % n, q // (n * n)
    K1 = kinetic_1d(C, w)
    I = np.eye(C)
    # local index a + C (b + C c): x fastest -> kron(z, y, x)
    H = (np.kron(np.kron(I, I), K1) + np.kron(np.kron(I, K1), I) + np.kron(np.kron(K1, I), I))
    a = np.arange(C)
    gx = (qi - m + a) % n
    gy = (qj - m + a) % n
    gz = (qk - m + a) % n
    vwin = veff.reshape(n, n, n)[np.ix_(gz, gy, gx)].ravel()
    H[np.diag_indices_from(H)] += vwin
    lo = np.array([qi - m, qj - m, qk - m])
    for ijk, p, gam in tables:
        # every lattice translation t whose sphere meets the cube
        tr = []
        for ax in range(3):
            tmin = math.floor((lo[ax] - ijk[:, ax].max()) / n) - 1
            tmax = math.ceil((lo[ax] + C - 1 - ijk[:, ax].min()) / n) + 1
            tr.append(range(tmin, tmax + 1))
        for tz in tr[2]:
            for ty in tr[1]:
                for tx in tr[0]:
                    loc = ijk + np.array([tx, ty, tz]) * n - lo
                    inside = np.all((loc >= 0) & (loc < C), axis=1)
                    if not inside.any():
                        continue
                    li = loc[inside]
                    idx = li[:, 0] + C * (li[:, 1] + C * li[:, 2])
                    v = np.zeros(C ** 3)
                    v[idx] = p[inside]
                    H += gam * h ** 3 * np.outer(v, v)
    return H


def cheb_moments_eig(H, chi, zeta, centre, npl):
    """e^T T_j((H - chi)/zeta) e for j = 0..npl from eigh."""
    lam, U = np.linalg.eigh(H)
    x = np.clip((lam - chi) / zeta, -1.0, 1.0)
    wgt = U[centre, :] ** 2
    j = np.arange(npl + 1)
    return (wgt[None, :] * np.cos(j[:, None] * np.arccos(x)[None, :])).sum(1), lam, U


def bloch_hamiltonian(n, h, w, veff, tables, k):
    """Periodic FD Hamiltonian with Bloch phases exp(i k . T) for a cubic
    cell of edge n h (complex Hermitian, n^3 x n^3)."""
    L = n * h
    N = n ** 3
    H = np.zeros((N, N), dtype=complex)
    idx = np.arange(N)
    i, j, kk = idx % n, (idx // n) % n, idx // (n * n)
    no = len(w) - 1
    H[idx, idx] += -0.5 * 6 * float(w[0]) + veff
    coords = [i, j, kk]
    for ax in range(3):
        for d in range(1, no + 1):
            for s in (+1, -1):
                c = [x.copy() for x in coords]
                raw = c[ax] + s * d
                wrap = np.floor_divide(raw, n)
                c[ax] = raw - wrap * n
                tgt = c[0] + n * (c[1] + n * c[2])
                phase = np.exp(1j * k[ax] * wrap * L)
                np.add.at(H, (idx, tgt), -0.5 * float(w[d]) * phase)
    for ijk, p, gam in tables:
        wrap = np.floor_divide(ijk, n)
        loc = ijk - wrap * n
        tgt = loc[:, 0] + n * (loc[:, 1] + n * loc[:, 2])
        phase = np.exp(1j * (wrap * L) @ k)
        v = np.zeros(N, dtype=complex)
        np.add.at(v, tgt, p * np.conj(phase))
        H += gam * h ** 3 * np.outer(v, np.conj(v))
    return H


def fermi(x):
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def fd_gradient_weights_taylor(no: int) -> list[Fraction]:
    """Central first-derivative weights of order 2 no for unit spacing, from
    the moment conditions on an antisymmetric stencil:
    f'(0) ~ sum_d g_d (f_d - f_-d) with sum_d 2 d^(2p+1) g_d = delta_{p,0},
    p = 0 .. no - 1, solved exactly.  Returns [0, g_1, ..., g_no]."""
    A = [[Fraction(2 * d ** (2 * p + 1)) for d in range(1, no + 1)] for p in range(no)]
    b = [Fraction(1) if p == 0 else Fraction(0) for p in range(no)]
    for col in range(no):
        piv = next(r for r in range(col, no) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for r in range(no):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                b[r] -= f * b[col]
    return [Fraction(0)] + [b[i] / A[i][i] for i in range(no)]


def periodic_gradient(n, h, g, ax):
    """Dense periodic FD derivative along axis ax (0 = x, fastest index) of an
    n^3 grid, weights g = [0, g_1, ..] for unit spacing."""
    N = n ** 3
    G = np.zeros((N, N))
    idx = np.arange(N)
    coords = [idx % n, (idx // n) % n, idx // (n * n)]
    for d in range(1, len(g)):
        for s in (+1, -1):
            c = [x.copy() for x in coords]
            c[ax] = (c[ax] + s * d) % n
            tgt = c[0] + n * (c[1] + n * c[2])
            np.add.at(G, (idx, tgt), s * float(g[d]) / h)
    return G


def projector_vectors(n, tables):
    """Each atom's projector as a periodic grid vector (sphere wrapped into the cell)."""
    out = []
    for ijk, p, gam in tables:
        loc = np.mod(ijk, n)
        v = np.zeros(n ** 3)
        np.add.at(v, loc[:, 0] + n * (loc[:, 1] + n * loc[:, 2]), p)
        out.append((v, gam))
    return out
