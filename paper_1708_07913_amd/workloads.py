"""Seeded synthetic inputs for the spectral-quadrature density step.

This module builds the *inputs* of the method and nothing else: atomic
positions of displaced FCC aluminium-like crystals, the effective potential
V_eff sampled on the periodic finite-difference grid, and the per-atom
Kleinman-Bylander projector parameters.  It holds none of the method's
arithmetic (no stencil, no Hamiltonian, no quadrature), so both the CPU
oracle and the HIP path can take their inputs from it.

The paper's Al workloads (FCC, lattice constant 7.78 Bohr, randomly displaced
atoms, mesh 0.4-0.78 Bohr, R_cut 6-7 Bohr, n_pl 28-64; Sec. 4.1-4.3) use
Troullier-Martins pseudopotentials and an LDA self-consistent potential that
are not available here.  They are replaced by a fixed Gaussian-well V_eff and
one s-type projector per atom:

* V_eff(x) = sum over atoms of -1.5 exp(-|d|^2 / (2 * 0.8^2)) Ha, with d the
  minimum-image displacement (each component reduced by L * rint(d / L)),
  terms with |d| > 8 Bohr dropped (they are below 1e-21 Ha).
* projector chi(r) = exp(-r^2 / (2 * 0.7^2)), cut at 2.5 Bohr, energy
  gamma = +0.5 Ha, 3 valence electrons per atom.

All lengths are in Bohr, energies in Hartree.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

HARTREE_EV = 27.211386245988

FCC_BASIS = np.array([[0.0, 0.0, 0.0],
                      [0.0, 0.5, 0.5],
                      [0.5, 0.0, 0.5],
                      [0.5, 0.5, 0.0]])

WELL_DEPTH = 1.5      # Ha
WELL_WIDTH = 0.8      # Bohr
WELL_CUTOFF = 8.0     # Bohr
KB_SIGMA = 0.7        # Bohr
KB_RCUT = 2.5         # Bohr
KB_GAMMA = 0.5        # Ha
ELECTRONS_PER_ATOM = 3


@dataclass
class Workload:
    """One snapshot: geometry, grid and SQ parameters."""
    name: str
    cell: float                 # cubic cell edge L (Bohr)
    h: float                    # requested mesh size (Bohr)
    fd_order: int               # 2 n_o
    rcut: float                 # R_cut (Bohr)
    npl: int                    # quadrature order n_pl
    kT_eV: float                # smearing sigma in eV
    atoms: np.ndarray           # (natom, 3) positions in [0, L)
    kb: np.ndarray              # (natom, 3): projector sigma, cut radius, gamma
    n_electrons: float
    seed: int
    amplitude: float
    precision: str = "fp64"
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return grid_points_per_axis(self.cell, self.h)

    @property
    def h_eff(self) -> float:
        return self.cell / self.n

    @property
    def kT(self) -> float:
        return self.kT_eV / HARTREE_EV

    @property
    def natom(self) -> int:
        return int(self.atoms.shape[0])

    def veff(self) -> np.ndarray:
        """V_eff on the n^3 grid, x fastest (flat index i + n (j + n k))."""
        return gaussian_well_potential(self.cell, self.n, self.atoms)


def grid_points_per_axis(cell: float, h: float) -> int:
    """n = round(L / h); the mesh is then refitted to h_eff = L / n."""
    n = int(math.floor(cell / h + 0.5))
    if n < 1:
        raise ValueError("cell smaller than one mesh interval")
    return n


def fcc_positions(cells: int, a: float, amplitude: float, seed: int) -> np.ndarray:
    """FCC supercell of cells^3 conventional cells (ix fastest, then iy, iz;
    the 4 basis atoms innermost), each coordinate displaced by an independent
    uniform draw in [-amplitude, amplitude], then wrapped into [0, L)."""
    idx = np.arange(cells)
    iz, iy, ix = np.meshgrid(idx, idx, idx, indexing="ij")
    corners = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    pos = (corners[:, None, :] + FCC_BASIS[None, :, :]).reshape(-1, 3) * a
    rng = np.random.default_rng(seed)
    pos = pos + rng.uniform(-amplitude, amplitude, pos.shape)
    L = cells * a
    return np.mod(pos, L)


def gaussian_well_potential(cell: float, n: int, atoms: np.ndarray,
                            depth: float = WELL_DEPTH, width: float = WELL_WIDTH,
                            cutoff: float = WELL_CUTOFF) -> np.ndarray:
    """Sum of minimum-image Gaussian wells sampled at x = h (i, j, k)."""
    h = cell / n
    V = np.zeros((n, n, n))           # indexed [k, j, i]
    inv2w2 = 1.0 / (2.0 * width * width)
    rc2 = cutoff * cutoff
    half = int(math.ceil(cutoff / h))
    use_box = (2 * cutoff < cell) and (2 * half + 1 < n)
    full = np.arange(n) * h
    for R in atoms:
        axes = []
        for ax in range(3):
            if use_box:
                c = int(math.floor(R[ax] / h))
                i = np.arange(c - half, c + half + 2)
                d = i * h - R[ax]
                axes.append((np.mod(i, n), d))
            else:
                d = full - R[ax]
                d = d - cell * np.rint(d / cell)
                axes.append((np.arange(n), d))
        (ix, dx), (iy, dy), (iz, dz) = axes
        r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        val = np.where(r2 <= rc2, -depth * np.exp(-r2 * inv2w2), 0.0)
        V[np.ix_(iz, iy, ix)] += val
    return V.reshape(-1)


def _kb(natom: int) -> np.ndarray:
    kb = np.empty((natom, 3))
    kb[:, 0] = KB_SIGMA
    kb[:, 1] = KB_RCUT
    kb[:, 2] = KB_GAMMA
    return kb


def fcc_workload(name: str, cells: int, a: float, amplitude: float, seed: int,
                 h: float, rcut: float, npl: int, kT_eV: float,
                 fd_order: int = 12, precision: str = "fp64") -> Workload:
    atoms = fcc_positions(cells, a, amplitude, seed)
    return Workload(name=name, cell=cells * a, h=h, fd_order=fd_order, rcut=rcut,
                    npl=npl, kT_eV=kT_eV, atoms=atoms, kb=_kb(atoms.shape[0]),
                    n_electrons=float(ELECTRONS_PER_ATOM * atoms.shape[0]),
                    seed=seed, amplitude=amplitude, precision=precision)


def tiny_cell(precision: str = "fp64", npl: int = 24, kT_eV: float = 1.0) -> Workload:
    """8 Bohr cubic cell, 4 atoms, h = 0.5 (16^3 grid), R_cut 2.5 (11^3 cube)."""
    return fcc_workload("al4_h0.5_rc2.5", 1, 8.0, 0.1, 1, 0.5, 2.5, npl, kT_eV,
                        precision=precision)


def paper_size_cell() -> Workload:
    """4x4x4 FCC (256 atoms, 31.12 Bohr), h 0.4 (78^3 grid), R_cut 6 (31^3), n_pl 48."""
    return fcc_workload("al256_h0.4_rc6", 4, 7.78, 0.15, 2, 0.4, 6.0, 48, 1.0)


def paper_cell_small() -> Workload:
    """2x2x2 FCC version of the paper-size cell (32 atoms, 39^3 grid, same 31^3 regions)."""
    return fcc_workload("al32_h0.4_rc6", 2, 7.78, 0.15, 2, 0.4, 6.0, 48, 1.0)


def large_cell(precision: str = "fp64") -> Workload:
    """7x7x7 FCC (1372 atoms, 54.46 Bohr), h 0.5 (109^3), R_cut 7 (29^3), n_pl 64."""
    return fcc_workload("al1372_h0.5_rc7", 7, 7.78, 0.2, 5, 0.5, 7.0, 64, 1.0,
                        precision=precision)


def mixed_sweep():
    """Tiny-cell geometry with kT in {0.5, 1, 2, 5} eV and n_pl in {24, 32, 48, 96}."""
    out = []
    for kT in (0.5, 1.0, 2.0, 5.0):
        for npl in (24, 32, 48, 96):
            out.append(tiny_cell("mixed", npl=npl, kT_eV=kT))
    return out


def qmd_ensemble():
    """Twelve snapshots of uneven size: FCC edges 2..5 cells (32..500 atoms),
    three displacement sets each (0.1/0.2/0.3 Bohr, R_cut 5/6/7, n_pl 32/48/64)."""
    sizes = {2: (0.40, 1.0), 3: (0.45, 3.0), 4: (0.50, 1.0), 5: (0.50, 3.0)}
    sets = [(0.1, 5.0, 32), (0.2, 6.0, 48), (0.3, 7.0, 64)]
    out = []
    for M, (h, kT) in sizes.items():
        for b, (A, rc, npl) in enumerate(sets):
            s = 3 * (M - 2) + b
            out.append(fcc_workload(f"qmd{s:02d}_al{4 * M ** 3}", M, 7.78, A, 400 + s,
                                    h, rc, npl, kT, precision="mixed"))
    return out
