"""Seeded synthetic molecules shaped like the paper's workloads.

This module only draws inputs: Kohn-Sham eigenvalues and eigenvectors, a
block-sparse product vertex, product centres, the Coulomb metric and the
frequency grid description.  It holds none of the screened-interaction
arithmetic (no pair vectors, no histogram, no response function, no solve), so
both the CPU oracle and the GPU path can consume the same bytes without sharing
any of the method's code.

The paper's own inputs (SIESTA Hamiltonians and dominant-product vertices for
benzene, naphthalene and anthracene, Sections 6 and 10) are not available;
these generators stand in for them with the same kinds of structure:

* eigenvalues measured from the Fermi level, E < 0 occupied, E > 0 empty
  (Section 3, text after eq. local_propagator);
* eigenvectors X_a^E as columns of an orthogonal matrix (S = 1);
* a product vertex V_mu^ab that is nonzero only when a, b and mu sit on one
  atom or one bonded atom pair, and symmetric in ab (Section 3, text after
  eq. VertexDefinition);
* a symmetric positive Coulomb metric v^{mu nu} (Section 3, after
  eq. tensorform-dyson), here the softened 1/sqrt(d^2 + 2 bohr^2) between
  product centres.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

__all__ = [
    "Molecule",
    "Grid",
    "chain_molecule",
    "cluster_molecule",
    "make_config",
    "config_grid",
    "batch_molecules",
    "serving_stream",
    "truncate_products",
    "two_window_grids",
]


@dataclasses.dataclass
class Grid:
    """Uniform frequency grid omega_j = omega_min + j*domega, j = 0..n_omega-1.

    domega = (omega_max - omega_min) / n_omega, so omega_max itself is not a
    grid point.  eps is the Lorentzian broadening.  All energies in Hartree.
    """

    n_omega: int
    omega_min: float
    omega_max: float
    eps: float
    frac_bits: int = -1  # < 0: the library / oracle picks it from the data

    @property
    def domega(self) -> float:
        return (self.omega_max - self.omega_min) / self.n_omega

    def omegas(self) -> np.ndarray:
        return self.omega_min + self.domega * np.arange(self.n_omega, dtype=np.float64)


@dataclasses.dataclass
class Molecule:
    """One synthetic molecule in the flat block layout the C ABI takes.

    Products are grouped in blocks; every product of block b lives on the same
    ascending orbital set orb_idx[blk_orb[b]:blk_orb[b+1]] and stores an
    |O| x |O| symmetric row-major matrix at vals[blk_val[b] + i*|O|*|O|] for its
    i-th product in the block.
    """

    n_orb: int
    n_occ: int
    eig: np.ndarray  # [n_orb] float64, ascending
    X: np.ndarray  # [n_orb, n_orb] float64, X[a, E] = X_a^E
    blk_prod: np.ndarray  # [n_blk+1] int32
    blk_orb: np.ndarray  # [n_blk+1] int32
    orb_idx: np.ndarray  # int32
    blk_val: np.ndarray  # [n_blk+1] int64
    vals: np.ndarray  # float64
    centres: np.ndarray  # [n_prod, 3]
    atoms: np.ndarray  # [n_atoms, 3]
    v: np.ndarray  # [n_prod, n_prod] float64

    @property
    def n_prod(self) -> int:
        return int(self.blk_prod[-1])

    @property
    def n_blk(self) -> int:
        return len(self.blk_prod) - 1

    @property
    def n_virt(self) -> int:
        return self.n_orb - self.n_occ

    @property
    def n_pairs(self) -> int:
        return self.n_occ * self.n_virt

    def block_of(self, b: int):
        """(first product, n products, orbital list, list of |O|x|O| matrices)."""
        o = self.orb_idx[self.blk_orb[b] : self.blk_orb[b + 1]]
        n = len(o)
        p0, p1 = int(self.blk_prod[b]), int(self.blk_prod[b + 1])
        base = int(self.blk_val[b])
        mats = [
            self.vals[base + i * n * n : base + (i + 1) * n * n].reshape(n, n)
            for i in range(p1 - p0)
        ]
        return p0, p1 - p0, o, mats

    def scaled_vertex(self, t: float) -> "Molecule":
        """Same molecule with V -> t*V (used for the V -> 0 limit)."""
        return dataclasses.replace(self, vals=self.vals * t)


def _coulomb(centres: np.ndarray) -> np.ndarray:
    d2 = ((centres[:, None, :] - centres[None, :, :]) ** 2).sum(-1)
    return 1.0 / np.sqrt(d2 + 2.0)


def _assemble(
    rng: np.random.Generator,
    atoms: np.ndarray,
    orb_per_atom: int,
    occ_per_atom: int,
    prod_per_atom: int,
    prod_per_bond: int,
    bonds: List[tuple],
) -> Molecule:
    n_atoms = len(atoms)
    n_orb = n_atoms * orb_per_atom
    n_occ = n_atoms * occ_per_atom
    occ = rng.uniform(-1.0, -0.2, size=n_occ)
    virt = rng.uniform(0.0, 2.0, size=n_orb - n_occ)
    eig = np.sort(np.concatenate([occ, virt]))
    q, _ = np.linalg.qr(rng.standard_normal((n_orb, n_orb)))
    X = np.ascontiguousarray(q)

    blk_prod = [0]
    blk_orb = [0]
    blk_val = [0]
    orb_idx: List[int] = []
    vals: List[np.ndarray] = []
    centres: List[np.ndarray] = []

    def add_block(atom_list, n_products, centre):
        orbs = []
        owner = []
        for at in atom_list:
            orbs.extend(range(at * orb_per_atom, (at + 1) * orb_per_atom))
            owner.extend([at] * orb_per_atom)
        n = len(orbs)
        pos = atoms[owner]
        r = np.sqrt(((pos[:, None, :] - pos[None, :, :]) ** 2).sum(-1))
        damp = np.exp(-r)
        iu = np.triu_indices(n)
        for _ in range(n_products):
            m = np.zeros((n, n))
            m[iu] = rng.standard_normal(len(iu[0]))
            m = np.triu(m) + np.triu(m, 1).T
            vals.append((m * damp).ravel())
            centres.append(centre)
        orb_idx.extend(orbs)
        blk_orb.append(len(orb_idx))
        blk_prod.append(blk_prod[-1] + n_products)
        blk_val.append(blk_val[-1] + n_products * n * n)

    for a in range(n_atoms):
        add_block([a], prod_per_atom, atoms[a])
    for (a, b) in bonds:
        add_block([a, b], prod_per_bond, 0.5 * (atoms[a] + atoms[b]))

    centres_a = np.array(centres, dtype=np.float64)
    return Molecule(
        n_orb=n_orb,
        n_occ=n_occ,
        eig=eig,
        X=X,
        blk_prod=np.array(blk_prod, dtype=np.int32),
        blk_orb=np.array(blk_orb, dtype=np.int32),
        orb_idx=np.array(orb_idx, dtype=np.int32),
        blk_val=np.array(blk_val, dtype=np.int64),
        vals=np.concatenate(vals).astype(np.float64),
        centres=centres_a,
        atoms=atoms,
        v=_coulomb(centres_a),
    )


def chain_molecule(
    n_atoms: int,
    seed: int,
    orb_per_atom: int = 13,
    occ_per_atom: int = 4,
    prod_per_atom: int = 40,
    prod_per_bond: int = 16,
    bond_cutoff: Optional[float] = 5.0,
    spacing: float = 2.6,
    jitter: float = 0.1,
) -> Molecule:
    """Linear chain on the x axis, spacing 2.6 bohr, N(0, jitter) jitter in x.

    bond_cutoff=None bonds consecutive atoms only; otherwise every atom pair
    closer than the cutoff carries bond products.
    """
    rng = np.random.default_rng(seed)
    x = spacing * np.arange(n_atoms) + rng.normal(0.0, jitter, size=n_atoms)
    atoms = np.zeros((n_atoms, 3))
    atoms[:, 0] = x
    if bond_cutoff is None:
        bonds = [(i, i + 1) for i in range(n_atoms - 1)]
    else:
        bonds = [
            (i, j)
            for i in range(n_atoms)
            for j in range(i + 1, n_atoms)
            if abs(x[j] - x[i]) < bond_cutoff
        ]
    return _assemble(rng, atoms, orb_per_atom, occ_per_atom, prod_per_atom, prod_per_bond, bonds)


def cluster_molecule(
    n_atoms: int,
    seed: int,
    radius: float = 20.0,
    d_min: float = 2.4,
    orb_per_atom: int = 13,
    occ_per_atom: int = 4,
    prod_per_atom: int = 40,
    prod_per_bond: int = 16,
    bond_cutoff: float = 6.0,
) -> Molecule:
    """Atoms uniform in a sphere of the given radius, rejection-sampled so that
    no two are closer than d_min bohr; pairs within bond_cutoff are bonded."""
    rng = np.random.default_rng(seed)
    pts: List[np.ndarray] = []
    tries = 0
    while len(pts) < n_atoms:
        tries += 1
        if tries > 1000000:
            raise RuntimeError("cannot place atoms; sphere too small")
        p = rng.uniform(-radius, radius, size=3)
        if p @ p > radius * radius:
            continue
        if pts and np.min(np.sum((np.array(pts) - p) ** 2, axis=1)) < d_min * d_min:
            continue
        pts.append(p)
    atoms = np.array(pts)
    bonds = [
        (i, j)
        for i in range(n_atoms)
        for j in range(i + 1, n_atoms)
        if np.sum((atoms[i] - atoms[j]) ** 2) < bond_cutoff * bond_cutoff
    ]
    return _assemble(rng, atoms, orb_per_atom, occ_per_atom, prod_per_atom, prod_per_bond, bonds)


def truncate_products(mol: Molecule, n_keep: int) -> Molecule:
    """Keep the first n_keep products (whole blocks plus a partial last block)."""
    if n_keep >= mol.n_prod:
        return mol
    nb = int(np.searchsorted(mol.blk_prod, n_keep, side="left"))
    # blocks 0..nb-1 kept whole or partially; block nb-1 may be cut
    blk_prod = list(mol.blk_prod[: nb + 1])
    blk_orb = list(mol.blk_orb[: nb + 1])
    blk_val = list(mol.blk_val[: nb + 1])
    last = nb - 1
    n_last = n_keep - int(mol.blk_prod[last])
    o = int(mol.blk_orb[last + 1] - mol.blk_orb[last])
    blk_prod[-1] = n_keep
    blk_val[-1] = int(mol.blk_val[last]) + n_last * o * o
    vals = mol.vals[: blk_val[-1]].copy()
    orb_idx = mol.orb_idx[: blk_orb[-1]].copy()
    centres = mol.centres[:n_keep].copy()
    return dataclasses.replace(
        mol,
        blk_prod=np.array(blk_prod, dtype=np.int32),
        blk_orb=np.array(blk_orb, dtype=np.int32),
        blk_val=np.array(blk_val, dtype=np.int64),
        orb_idx=orb_idx,
        vals=vals,
        centres=centres,
        v=_coulomb(centres),
    )


def config_grid(i: int) -> Grid:
    """Frequency grids of the five workloads (Hartree)."""
    if i == 0:
        return Grid(256, -4.0, 4.0, 0.05)
    if i == 1:
        return Grid(1024, -8.0, 8.0, 0.02)
    if i == 2:
        return Grid(2048, -8.0, 8.0, 0.01)
    if i == 3:
        g = Grid(512, -8.0, 8.0, 0.0)
        g.eps = 1.5 * g.domega  # the paper's automatic broadening
        return g
    if i == 4:
        return Grid(1024, -8.0, 8.0, 0.02)
    raise ValueError(i)


def two_window_grids() -> Tuple[Grid, Grid]:
    """The two-window meshes of the 2000-product workload (Hartree): a fine
    256-point mesh over |omega| < 0.5 (spacing 2^-8, about 0.11 eV) and a
    coarse 256-point mesh over |omega| < 4 (spacing 2^-5, about 0.85 eV), each
    broadened by 1.5 times its own spacing (the paper's automatic choice).
    Returns (small, large)."""
    small = Grid(256, -0.5, 0.5, 0.0)
    large = Grid(256, -4.0, 4.0, 0.0)
    small.eps = 1.5 * small.domega
    large.eps = 1.5 * large.domega
    return small, large


def make_config(i: int, seed: Optional[int] = None) -> Molecule:
    """Single-molecule workloads: 0 tiny chain, 1 40-atom chain, 2 120-atom cluster."""
    if i == 0:
        return chain_molecule(
            4, 0 if seed is None else seed, orb_per_atom=4, occ_per_atom=2,
            prod_per_atom=10, prod_per_bond=8, bond_cutoff=None,
        )
    if i == 1:
        return chain_molecule(40, 1 if seed is None else seed)
    if i == 2:
        return cluster_molecule(120, 2 if seed is None else seed)
    raise ValueError(i)


def batch_molecules(n: int = 64, base_seed: int = 1000, lo: int = 8, hi: int = 80) -> List[Molecule]:
    """Batched workload: chain molecules with atom counts uniform in [lo, hi]."""
    rng = np.random.default_rng(base_seed)
    counts = rng.integers(lo, hi + 1, size=n)
    return [chain_molecule(int(c), base_seed + i) for i, c in enumerate(counts)]


def serving_stream(rate: float = 20.0, duration: float = 60.0, seed: int = 4,
                   lo: int = 10, hi: int = 200):
    """Poisson arrivals (times, atom counts); molecules are drawn lazily with
    cluster_molecule(n, 4000 + i, radius=20*(n/120)**(1/3))."""
    rng = np.random.default_rng(seed)
    times = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        times.append(t)
    counts = np.exp(rng.uniform(math.log(lo), math.log(hi), size=len(times)))
    counts = np.maximum(lo, np.round(counts)).astype(int)
    return np.array(times), counts


def serving_molecule(i: int, n_atoms: int) -> Molecule:
    return cluster_molecule(n_atoms, 4000 + i, radius=20.0 * (n_atoms / 120.0) ** (1.0 / 3.0))


def lowrank_w_factors(n_prod: int, n_omega: int, rank: int = 4, k_max: int = 300, seed: int = 7):
    """Seeded factors of a synthetic interaction W(k domega) = v + U diag(c[k]) U^T
    on the positive half of a symmetric n_omega-point mesh (k = 0 .. n_omega/2 - 1):
    U [n_prod][rank] real, c [n_omega/2][rank] complex with Im c <= 0, a Gaussian
    bump per rank inside 0 < k < k_max and exactly zero elsewhere (so a
    convolution with it stays inside a mesh whose bins reach n_omega/2)."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((n_prod, rank)) / math.sqrt(n_prod)
    k = np.arange(n_omega // 2, dtype=float)
    centre = rng.uniform(0.2, 0.8, rank) * k_max
    width = rng.uniform(0.05, 0.2, rank) * k_max
    amp = rng.uniform(0.5, 2.0, rank)
    im = -amp[None, :] * np.exp(-0.5 * ((k[:, None] - centre[None, :]) / width[None, :]) ** 2)
    im[0] = 0.0
    im[k_max:] = 0.0
    re = rng.standard_normal((n_omega // 2, rank))
    return U, re + 1j * im


def lowrank_sigma_factors(n_orb: int, n_omega: int, rank: int = 4, seed: int = 11):
    """Seeded factors of a synthetic correlation self-energy
    Sigma_c(omega_j) = Y diag(s[j]) Y^T: Y [n_orb][rank] real, s [n_omega][rank]
    complex with Im s <= 0 (so Im Sigma_c is negative semidefinite), and a
    static pair (Sigma_x, V_xc) of small symmetric matrices."""
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((n_orb, rank)) / math.sqrt(n_orb)
    s = 0.3 * rng.standard_normal((n_omega, rank)) - 0.2j * rng.uniform(0.1, 1.0, (n_omega, rank))
    A = 0.02 * rng.standard_normal((n_orb, n_orb))
    B = 0.02 * rng.standard_normal((n_orb, n_orb))
    return Y, s, A + A.T, B + B.T
