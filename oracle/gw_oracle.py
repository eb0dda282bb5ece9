"""FP64 reference implementation of a0 -> chi0 -> W (test infrastructure only).

What the method computes, in the paper's notation (energies in Hartree):

* Pair vertex, Section 7.A (closed form of chi0 below eq. subsetof_vef's
  preamble): V_mu^{EF} = X_a^E V_mu^{ab} X_b^F for an occupied state E and an
  empty state F (Section 3: E < 0 occupied, E > 0 empty).
* Spectral function of the free response, Section 5.A eq. chi_by_spectra: for
  s > 0 it is the density of electron-hole pair weights; a(-s) = -a(s); chi0 is
  its Cauchy transform.  With the closed form of Section 7.A this is
  a_{mu nu}(s) = 2 sum_p V_mu^p V_nu^p delta(s - Delta_p), Delta_p = F - E,
  the 2 being the spin sum (Section 2, eq. more_screening).
* Discretisation on a uniform mesh, Section 5 (mesh spacing somewhat smaller
  than the broadening) and Section 5.B (eps = 1.5 domega by default).
* Screening, Section 2 eq. Coulombscreening / Section 3 eq.
  tensorform-scr-inter: W = (1 - v chi0)^{-1} v, frequency by frequency.
* Two spectral windows, Section 5.B eq. win2-for-response.
* The paper's own route to a0: the electronic density matrix rho_ab(s) of
  Section 5 split into its empty (rho^+) and occupied (rho^-) parts on the
  mesh, and a0 as their convolution contracted with the vertex (Section 5.A
  eq. chi_by_spectra), which Section 8.A eq. sf-of-response-time evaluates
  time by time.
* Downstream of W: the spectral function gamma of the dynamical part
  W - v, the spectral functions sigma+- of the GW self-energy as convolutions
  of rho+- with gamma contracted with the vertex (Section 5.A eq. spectral_3,
  evaluated time by time in Section 8.B), the self-energy as their Cauchy
  transform (eq. Cauchy1), and the instantaneous exchange part (Section 4
  eq. instantaneous); Dyson's equation and the density of states (Section 2
  eqs. Dyson and the DOS definition, Section 3 eq. tensorform-dyson, with
  V_xc subtracted from Sigma as Section 2 prescribes).
* Compression, Section 7.B eqs. subspace_chi0 and chi_RPA; the paper's own
  subspace, Section 7.A eqs. subsetof_vef, projector0, subspace and
  global-basis-orthogonality.

Readings where the paper is silent (each also listed in the design notes):

1. Grid: omega_j = omega_min + j*domega, domega = (omega_max-omega_min)/N
   (omega_max excluded).  This is what reproduces the 0.234375 eV the paper
   prints for N = 1024 on [-80, 80] eV with eps = 1.5 domega (Section 6).
   domega must be a power of two so that Delta/domega is exact.
2. Deposition: linear (two-bin) split of each pole onto the mesh, in int64
   fixed point with 2^-s resolution so the sum is exact and order-free.
3. Retarded response at every omega: chi0(-omega) = conj chi0(omega).
4. Spectral bins are m = 0 .. nhb-1 (s = m*domega >= 0); bin 0 is stored but,
   by a(-s) = -a(s), contributes nothing to chi0.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Iterable, Optional, Sequence

import numpy as np

__all__ = [
    "grid_spacing",
    "grid_omegas",
    "grid_shift_bits",
    "pair_vectors",
    "pair_bins",
    "hist_bins",
    "frac_bits",
    "histogram",
    "histogram_c",
    "packed_index",
    "unpack_upper",
    "chi0_from_hist",
    "chi0_apply",
    "chi0_poles",
    "screened_W",
    "compress_basis",
    "screened_W_compressed",
    "project_pairs",
    "pair_subset",
    "pair_basis",
    "pair_projector",
    "screened_W_pair_basis",
    "two_window_split",
    "chi0_two_window",
    "level_bins",
    "spectral_densities",
    "level_hist_bins",
    "a0_by_convolution",
    "a0_by_pairs",
    "chi0_from_spectrum",
    "w_spectral",
    "self_energy_spectra",
    "self_energy_spectra_by_levels",
    "self_energy_from_spectra",
    "exchange_self_energy",
    "dyson_dos",
]


# ----------------------------------------------------------------------------
# grid (Section 5, Section 5.B, Section 6)


def grid_spacing(n_omega: int, omega_min: float, omega_max: float) -> float:
    """domega = (omega_max - omega_min) / N (reading 1)."""
    return (omega_max - omega_min) / n_omega


def grid_omegas(n_omega: int, omega_min: float, omega_max: float) -> np.ndarray:
    d = grid_spacing(n_omega, omega_min, omega_max)
    return omega_min + d * np.arange(n_omega, dtype=np.float64)


def grid_shift_bits(domega: float) -> int:
    """k with domega = 2^-k; raises unless domega is an exact power of two."""
    m, e = math.frexp(domega)
    if m != 0.5:
        raise ValueError("domega must be a power of two")
    return 1 - e


# ----------------------------------------------------------------------------
# pair vertex (Section 7.A closed form; Section 3 eq. VertexDefinition sparsity)


def pair_vectors(mol) -> np.ndarray:
    """P[mu, p] = V_mu^{EF} = sum_a X_a^E sum_b V_mu^{ab} X_b^F, p = E*N_virt + (F - N_occ).

    The contraction runs over the atom-local orbital set O of mu only (the
    vertex vanishes elsewhere).  The order is fixed: first T[a, F] = sum over b
    ascending of V^{ab} X_b^F, then sum over a ascending of X_a^E T[a, F],
    every product and every addition rounded separately.
    """
    n_occ, n_orb = mol.n_occ, mol.n_orb
    n_virt = n_orb - n_occ
    X = mol.X
    P = np.zeros((mol.n_prod, n_occ * n_virt))
    for b in range(mol.n_blk):
        p0, nprod, orbs, mats = mol.block_of(b)
        Xv = X[orbs][:, n_occ:]  # [|O|, N_virt]
        Xo = X[orbs][:, :n_occ]  # [|O|, N_occ]
        for i, V in enumerate(mats):
            n = len(orbs)
            T = np.zeros((n, n_virt))
            for bb in range(n):
                T = T + V[:, bb][:, None] * Xv[bb][None, :]
            acc = np.zeros((n_occ, n_virt))
            for aa in range(n):
                acc = acc + Xo[aa][:, None] * T[aa][None, :]
            P[p0 + i] = acc.ravel()
    return P


# ----------------------------------------------------------------------------
# binning (Section 5 mesh; Section 5.A spectral function of the response)


def pair_bins(eig: np.ndarray, n_occ: int, domega: float):
    """Delta_p = E_F - E_E; x = Delta_p / domega (exact: domega = 2^-k);
    m_p = floor(x); frac_p = x - m_p in [0, 1)."""
    k = grid_shift_bits(domega)
    e_occ = eig[:n_occ]
    e_vir = eig[n_occ:]
    delta = (e_vir[None, :] - e_occ[:, None]).ravel()
    x = np.ldexp(delta, k)
    m = np.floor(x)
    frac = x - m
    return m.astype(np.int64), frac


def hist_bins(eig: np.ndarray, n_omega: int, domega: float) -> int:
    """Number of stored spectral bins: enough for the largest pair energy plus
    its upper neighbour, at most n_omega/2 (s < omega_max)."""
    k = grid_shift_bits(domega)
    dmax = float(eig[-1] - eig[0])
    mmax = int(math.floor(math.ldexp(dmax, k)))
    return int(min(n_omega // 2, mmax + 2))


def frac_bits(P: np.ndarray, n_pairs: int) -> int:
    """Fixed-point exponent s (weights are integers times 2^-s).

    With vmax = max |V_mu^p| < 2^e and 2*n_pairs < 2^c, every rounded weight
    stays below 2^(61-c) and below 2^50, so every histogram entry fits in
    int64 with a bit to spare.  s = min(61 - c - 2e, 50 - 2e), clamped to
    [-200, 960].
    """
    vmax = float(np.max(np.abs(P))) if P.size else 0.0
    _, e = math.frexp(vmax)
    c = int(2 * n_pairs).bit_length()
    s = min(61 - c - 2 * e, 50 - 2 * e)
    return int(max(-200, min(960, s)))


def packed_index(mu: np.ndarray, nu: np.ndarray, n: int) -> np.ndarray:
    """Row-major index of (mu, nu), mu <= nu, in the packed upper triangle."""
    mu = np.asarray(mu, dtype=np.int64)
    nu = np.asarray(nu, dtype=np.int64)
    return mu * n - (mu * (mu - 1)) // 2 + (nu - mu)


def histogram(P: np.ndarray, m: np.ndarray, frac: np.ndarray, s: int, nhb: int) -> np.ndarray:
    """Exact int64 spectral histogram H[bin, packed (mu<=nu)].

    For each pair p and mu <= nu (Section 5.A eq. chi_by_spectra with the
    closed form of Section 7.A):
      t    = RNE(2^s * fl(V_mu^p * V_nu^p))
      t_hi = RNE(fl(fl(V_mu^p * 2^s frac_p) * V_nu^p))
      bin m_p   += 2 (t - t_hi)   (the 2 is the spin sum)
      bin m_p+1 += 2 t_hi
    Pairs whose upper bin m_p + 1 >= nhb are dropped.  Plain loop over pairs;
    for tiny inputs only.
    """
    n_prod, n_pairs = P.shape
    iu, ju = np.triu_indices(n_prod)
    H = np.zeros((nhb, len(iu)), dtype=np.int64)
    for p in range(n_pairs):
        mp = int(m[p])
        if mp + 1 >= nhb:
            continue
        vm = P[iu, p]
        vn = P[ju, p]
        t = np.rint(np.ldexp(vm * vn, s)).astype(np.int64)
        w = math.ldexp(float(frac[p]), s)
        th = np.rint((vm * w) * vn).astype(np.int64)
        H[mp] += 2 * (t - th)
        H[mp + 1] += 2 * th
    return H


_CLIB = None


def _clib():
    global _CLIB
    if _CLIB is None:
        here = os.path.dirname(os.path.abspath(__file__))
        path = os.path.join(here, "libhist_ref.so")
        if not os.path.exists(path):
            build_c()
        lib = ctypes.CDLL(path)
        lib.hist_ref_entries.restype = ctypes.c_int
        lib.hist_ref_entries.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
        ]
        _CLIB = lib
    return _CLIB


def build_c() -> str:
    """Compile the plain C histogram (no FMA contraction, OpenMP over entries)."""
    import subprocess

    here = os.path.dirname(os.path.abspath(__file__))
    src = os.path.join(here, "hist_ref.c")
    out = os.path.join(here, "libhist_ref.so")
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(
        ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", "-fno-math-errno", "-std=c99", src, "-o", tmp, "-lm"]
    )
    os.replace(tmp, out)
    return out


def histogram_c(P: np.ndarray, m: np.ndarray, frac: np.ndarray, s: int, nhb: int,
                mu: Optional[np.ndarray] = None, nu: Optional[np.ndarray] = None):
    """Same definition as histogram(), in plain C, for chosen (mu, nu) entries
    (all of mu <= nu by default).  Returns (H[nhb, n_entries], n_dropped)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    n_prod, n_pairs = P.shape
    if mu is None:
        mu, nu = np.triu_indices(n_prod)
    mu = np.ascontiguousarray(mu, dtype=np.int64)
    nu = np.ascontiguousarray(nu, dtype=np.int64)
    if np.any(mu > nu):
        raise ValueError("entries must have mu <= nu")
    m = np.ascontiguousarray(m, dtype=np.int64)
    frac = np.ascontiguousarray(frac, dtype=np.float64)
    H = np.zeros((nhb, len(mu)), dtype=np.int64)
    dropped = np.zeros(1, dtype=np.int64)
    rc = _clib().hist_ref_entries(
        P.ctypes.data, n_prod, n_pairs, m.ctypes.data, frac.ctypes.data, int(s),
        mu.ctypes.data, nu.ctypes.data, len(mu), nhb, H.ctypes.data, dropped.ctypes.data,
    )
    if rc != 0:
        raise RuntimeError("hist_ref_entries failed: %d" % rc)
    return H, int(dropped[0])


def unpack_upper(packed: np.ndarray, n: int) -> np.ndarray:
    """[..., n(n+1)/2] packed upper triangle -> [..., n, n] symmetric."""
    iu, ju = np.triu_indices(n)
    out = np.zeros(packed.shape[:-1] + (n, n), dtype=packed.dtype)
    out[..., iu, ju] = packed
    out[..., ju, iu] = packed
    return out


# ----------------------------------------------------------------------------
# chi0 (Section 5.A eq. chi_by_spectra: Cauchy transform of the odd-extended a)


def chi0_apply(mol, y: np.ndarray, omega: float, eps: float, domega: float, n_hbins: int) -> np.ndarray:
    """chi0(omega + i eps) y for y [n_prod] or [n_prod][r], without forming chi0
    or the pair vectors:
        chi0 = sum_p 2 V^p (V^p)^T [(1 - frac_p) K(m_p) + frac_p K(m_p + 1)],
        K(m) = 1/(omega - m domega + i eps) - 1/(omega + m domega + i eps),
    the same binned spectral function as the histogram (Section 5.A eq.
    chi_by_spectra, spin factor 2), unquantised, pairs with m_p + 1 >= n_hbins
    dropped.  The closed form of the pair vertex (Section 7.A) is summed the
    other way round: V^p . y = X_E^T (sum_mu y_mu V_mu) X_F for every pair
    p = (E, F) at once, and (chi0 y)_mu = sum_{ab} V_mu^{ab} (X_occ b X_virt^T)_{ab}
    with b_p = (V^p . y) times the pair's weight."""
    n_occ, n_orb = mol.n_occ, mol.n_orb
    Y = np.asarray(y).reshape(mol.n_prod, -1)
    m, fr = pair_bins(mol.eig, n_occ, domega)

    def K(mm):
        return 1.0 / (omega - mm * domega + 1j * eps) - 1.0 / (omega + mm * domega + 1j * eps)

    wgt = 2.0 * ((1.0 - fr) * K(m) + fr * K(m + 1))
    wgt[m + 1 >= n_hbins] = 0.0
    wgt = wgt.reshape(n_occ, n_orb - n_occ)
    Xo, Xv = mol.X[:, :n_occ], mol.X[:, n_occ:]
    blocks = [mol.block_of(b) for b in range(mol.n_blk)]
    out = np.zeros(Y.shape, dtype=np.complex128)
    for col in range(Y.shape[1]):
        Vy = np.zeros((n_orb, n_orb), dtype=np.complex128)
        for p0, _, orbs, mats in blocks:
            ix = np.ix_(orbs, orbs)
            for i, M in enumerate(mats):
                Vy[ix] += Y[p0 + i, col] * M
        a = Xo.T @ Vy @ Xv  # V^p . y, p = (E, F)
        B = Xo @ (a * wgt) @ Xv.T
        for p0, _, orbs, mats in blocks:
            Bo = B[np.ix_(orbs, orbs)]
            for i, M in enumerate(mats):
                out[p0 + i, col] = np.sum(M * Bo)
    return out.reshape(np.shape(y))


def chi0_from_hist(H: np.ndarray, s: int, n_omega: int, omega_min: float, omega_max: float,
                   eps: float, js: Optional[Sequence[int]] = None,
                   omegas: Optional[np.ndarray] = None) -> np.ndarray:
    """chi0[j, entry] = sum_{m>=1} 2^-s H[m, entry] *
        (1/(omega_j - m domega + i eps) - 1/(omega_j + m domega + i eps)).

    Direct summation over bins (no FFT).  The second term is the a(-s) = -a(s)
    half of the spectral function.  By default omega_j are grid points j (all,
    or the listed js); explicit omegas may be given instead."""
    d = grid_spacing(n_omega, omega_min, omega_max)
    if omegas is None:
        om = grid_omegas(n_omega, omega_min, omega_max)
        if js is None:
            js = range(n_omega)
        js = np.asarray(list(js), dtype=np.int64)
        om = om[js]
    else:
        om = np.asarray(omegas, dtype=np.float64)
    nhb = H.shape[0]
    mvals = np.arange(1, nhb, dtype=np.float64) * d
    w = om[:, None]
    K = 1.0 / (w - mvals[None, :] + 1j * eps) - 1.0 / (w + mvals[None, :] + 1j * eps)
    h = np.ldexp(H[1:].astype(np.float64), -s)
    return K @ h


def chi0_poles(P: np.ndarray, eig: np.ndarray, n_occ: int, omegas: np.ndarray, eps: float) -> np.ndarray:
    """Closed form of Section 7.A with the poles where they really are:
    chi0_{mu nu}(w) = 2 sum_p V_mu^p V_nu^p (1/(w - Delta_p + i eps) - 1/(w + Delta_p + i eps)).
    Full [n_omega, n_prod, n_prod]; for convergence checks on small inputs."""
    delta = (eig[n_occ:][None, :] - eig[:n_occ][:, None]).ravel()
    out = np.empty((len(omegas), P.shape[0], P.shape[0]), dtype=np.complex128)
    for i, w in enumerate(omegas):
        g = 1.0 / (w - delta + 1j * eps) - 1.0 / (w + delta + 1j * eps)
        out[i] = 2.0 * (P * g[None, :]) @ P.T
    return out


# ----------------------------------------------------------------------------
# screening (Section 2 eq. Coulombscreening, Section 3 eq. tensorform-scr-inter)


def screened_W(v: np.ndarray, chi0: np.ndarray) -> np.ndarray:
    """W = (1 - v chi0)^{-1} v by dense LU (LAPACK gesv)."""
    n = v.shape[0]
    A = np.eye(n, dtype=np.complex128) - v.astype(np.complex128) @ chi0
    return np.linalg.solve(A, v.astype(np.complex128))


def compress_basis(v: np.ndarray, k: int):
    """Top-k eigenpairs of the Coulomb metric, eigenvalues descending."""
    lam, U = np.linalg.eigh(v)
    order = np.argsort(lam)[::-1][:k]
    return U[:, order], lam[order]


def project_pairs(P: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Pair vectors in the compressed basis: U^T V^p (so that the histogram of
    the projected vectors is U^T chi0 U, Section 7.B eq. subspace_chi0)."""
    return U.T @ P


def screened_W_compressed(v: np.ndarray, chi0: np.ndarray, k: int) -> np.ndarray:
    """Section 7.B with the subspace spanned by the top-k eigenvectors of v:
    with v_k = U_k L_k U_k^T, chi_hat = U_k^T chi0 U_k,
      W = U_k (1 - L_k chi_hat)^{-1} L_k U_k^T  ( = (1 - v_k chi0)^{-1} v_k ).
    No square root of L_k is needed, so zero or slightly negative kept
    eigenvalues are harmless."""
    U, lam = compress_basis(v, k)
    chat = U.T @ chi0 @ U
    A = np.eye(k, dtype=np.complex128) - lam[:, None] * chat
    Xk = np.linalg.solve(A, np.diag(lam).astype(np.complex128))
    return U @ Xk @ U.T


# ----------------------------------------------------------------------------
# the paper's compression subspace (Section 7.A), and W in it (Section 7.B)


def pair_subset(eig: np.ndarray, n_occ: int, e_threshold: float) -> np.ndarray:
    """Indices p = E*N_virt + (F - N_occ) of the electron-hole pairs with
    F - E < e_threshold (Section 7.A eq. subsetof_vef), ascending."""
    e_occ = eig[:n_occ]
    e_vir = eig[n_occ:]
    delta = (e_vir[None, :] - e_occ[:, None]).ravel()
    return np.nonzero(delta < e_threshold)[0]


def pair_basis(X: np.ndarray, v: np.ndarray, k: int):
    """Section 7.A: Gram matrix of the generators in the Coulomb metric,
    g^{mn} = X_mu^m v^{mu nu} X_nu^n (eq. projector0), its eigenpairs
    g xi = lambda xi, and Z^lambda = X xi^lambda / sqrt(lambda) for the k
    largest lambda (eq. subspace).  The Z are orthonormal in the Coulomb
    metric, Z^T v Z = 1 (eq. global-basis-orthogonality).  Returns Z [n][k]
    and the kept eigenvalues, descending."""
    g = X.T @ v @ X
    lam, xi = np.linalg.eigh(g)
    order = np.argsort(lam)[::-1][:k]
    lam, xi = lam[order], xi[:, order]
    Z = X @ xi / np.sqrt(lam)[None, :]
    return Z, lam


def pair_projector(Z: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Section 7.A: the projector onto the subspace, P^mu_nu = v^{mu mu'}
    P_{mu' nu} with P_{mu nu} = Z_mu Z_nu (the generators with g inverted on
    the kept space), so P^2 = P."""
    return v @ Z @ Z.T


def screened_W_pair_basis(v: np.ndarray, chi0: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """Section 7.B: chi0_mn = Z_m^mu chi0_{mu nu} Z_n^nu with Z^mu = v Z
    (eq. subspace_chi0), chi_RPA = (1 - chi0_mn)^{-1} chi0_mn, and
    W = v + Z^mu chi_RPA Z^nu (eq. chi_RPA)."""
    U = v @ Z
    c = U.T @ chi0 @ U
    k = c.shape[0]
    rpa = np.linalg.solve(np.eye(k, dtype=np.complex128) - c, c)
    return v.astype(np.complex128) + U @ rpa @ U.T


# ----------------------------------------------------------------------------
# two spectral windows (Section 5.B eq. win2-for-response)


def two_window_split(domega_small: float, omega_max_small: float, domega_large: float) -> float:
    """Energy lambda_s that separates the pairs of the two windows: the
    largest edge of the large mesh's bins with lambda_s <= lambda - domega_small
    (lambda = omega_max_small, the half-width of the small window), so that a
    pair below it deposits its split weight inside the small mesh and a pair at
    or above it starts a large-mesh bin."""
    m = math.floor((omega_max_small - domega_small) / domega_large)
    return m * domega_large


def chi0_two_window(P: np.ndarray, eig: np.ndarray, n_occ: int, s: int,
                    small: tuple, large: tuple, js: Optional[Sequence[int]] = None,
                    entries: Optional[tuple] = None) -> np.ndarray:
    """chi0 on the small window's mesh (Section 5.B eq. win2-for-response):
    the Cauchy transform with eps_small of the spectral function of the pairs
    with Delta < lambda_s (histogrammed on the small mesh), plus the Cauchy
    transform with eps_large of the spectral function of the pairs with
    Delta >= lambda_s (histogrammed on the large mesh) evaluated at the small
    mesh's frequencies.  small/large: (n_omega, omega_min, omega_max, eps).
    Every pair is counted once: the split is by pair, at a bin edge of the
    large mesh.  Returns packed upper [len(js)][n(n+1)/2], or with
    entries = (mu, nu) (mu <= nu) those entries only, [len(js)][len(mu)]."""
    ns, a_s, b_s, e_s = small
    nl, a_l, b_l, e_l = large
    ds = grid_spacing(ns, a_s, b_s)
    dl = grid_spacing(nl, a_l, b_l)
    lam_s = two_window_split(ds, b_s, dl)
    delta = (eig[n_occ:][None, :] - eig[:n_occ][:, None]).ravel()
    low = delta < lam_s
    # small window, fine mesh
    m_s, f_s = pair_bins(eig, n_occ, ds)
    nhb_s = hist_bins(eig, ns, ds)
    def hist(sel, m, f, nhb):
        if entries is None:
            return histogram(P[:, sel], m[sel], f[sel], s, nhb)
        return histogram_c(P[:, sel], m[sel], f[sel], s, nhb, entries[0], entries[1])[0]

    H_s = hist(low, m_s, f_s, nhb_s)
    chi = chi0_from_hist(H_s, s, ns, a_s, b_s, e_s, js=js)
    # the rest, coarse mesh, evaluated at the fine mesh's frequencies
    m_l, f_l = pair_bins(eig, n_occ, dl)
    nhb_l = hist_bins(eig, nl, dl)
    H_l = hist(~low, m_l, f_l, nhb_l)
    om = grid_omegas(ns, a_s, b_s)
    om = om if js is None else om[np.asarray(list(js), dtype=np.int64)]
    return chi + chi0_from_hist(H_l, s, nl, a_l, b_l, e_l, omegas=om)


# ----------------------------------------------------------------------------
# the paper's own route to a0 (Section 5 density matrix; Section 5.A
# eq. chi_by_spectra; Section 8.A eq. sf-of-response-time)


def level_bins(e: np.ndarray, domega: float):
    """One-particle poles on the mesh: x = |e| / domega (exact for a power of
    two), k = floor(x), phi = x - k; the pole's weight is split linearly,
    1 - phi into bin k and phi into bin k + 1 (the same deposition rule as for
    the pair poles)."""
    kb = grid_shift_bits(domega)
    x = np.ldexp(np.abs(np.asarray(e, dtype=np.float64)), kb)
    k = np.floor(x)
    return k.astype(np.int64), x - k


def spectral_densities(mol, domega: float):
    """rho^+_ab[k] = sum over empty F of X_a^F X_b^F w_F[k] (poles at E_F >= 0)
    and rhobar^-_ab[k] = rho^-_ab(-s) = sum over occupied E of X_a^E X_b^E
    wbar_E[k] (poles at -E_E > 0), where w is the two-bin split of the pole
    (level_bins).  Section 5: rho_ab(s) = sum_E X_a^E X_b^E delta(s - E),
    positive and negative parts as in eq. spectral_1.
    Returns (rho_p [K+][n_orb][n_orb], rho_m [K-][n_orb][n_orb])."""
    X, eig, n_occ = mol.X, mol.eig, mol.n_occ
    if not (eig[n_occ - 1] < 0.0 <= eig[n_occ]):
        raise ValueError("energies must be measured from the Fermi level")
    k_p, f_p = level_bins(eig[n_occ:], domega)
    k_m, f_m = level_bins(eig[:n_occ], domega)
    n = mol.n_orb
    rho_p = np.zeros((int(k_p.max()) + 2, n, n))
    rho_m = np.zeros((int(k_m.max()) + 2, n, n))
    for F in range(n_occ, mol.n_orb):
        xx = np.outer(X[:, F], X[:, F])
        i = F - n_occ
        rho_p[k_p[i]] += (1.0 - f_p[i]) * xx
        rho_p[k_p[i] + 1] += f_p[i] * xx
    for E in range(n_occ):
        xx = np.outer(X[:, E], X[:, E])
        rho_m[k_m[E]] += (1.0 - f_m[E]) * xx
        rho_m[k_m[E] + 1] += f_m[E] * xx
    return rho_p, rho_m


def level_hist_bins(eig: np.ndarray, n_occ: int, n_omega: int, domega: float) -> int:
    """Bins of a0 on this route: the convolution of rho^+ (bins up to
    k_max^+ + 1) with rhobar^- (up to k_max^- + 1) reaches k_max^+ + k_max^- + 2,
    so k_max^+ + k_max^- + 3 bins, at most n_omega/2."""
    k_p, _ = level_bins(eig[-1:], domega)
    k_m, _ = level_bins(eig[:1], domega)
    return int(min(n_omega // 2, int(k_p[0]) + int(k_m[0]) + 3))


def _dense_vertex(mol) -> np.ndarray:
    """V[mu][a][b] with the block matrices placed at their orbital sets."""
    V = np.zeros((mol.n_prod, mol.n_orb, mol.n_orb))
    for b in range(mol.n_blk):
        p0, nprod, orbs, mats = mol.block_of(b)
        for i, M in enumerate(mats):
            V[p0 + i][np.ix_(orbs, orbs)] = M
    return V


def a0_by_convolution(mol, rho_p: np.ndarray, rho_m: np.ndarray, nhb: int) -> np.ndarray:
    """a_{mu nu}[m] = 2 sum_{k1 + k2 = m} V_mu^{ab} rho^+_{bc}[k1] V_nu^{cd}
    rhobar^-_{da}[k2], m < nhb: eq. chi_by_spectra on the mesh (the s1, s2
    integrals become sums over bins, the delta function the condition
    k1 + k2 = m), with the spin factor 2 of the pair route.  Bins m >= nhb
    are dropped.  Packed upper triangle [nhb][n(n+1)/2]."""
    V = _dense_vertex(mol)
    n = mol.n_prod
    iu, ju = np.triu_indices(n)
    out = np.zeros((nhb, len(iu)))
    Z = {}
    for k2 in range(rho_m.shape[0]):
        if np.any(rho_m[k2]):
            Z[k2] = (V @ rho_m[k2]).reshape(n, -1)  # (V_nu rhobar^-)[c][a]
    for k1 in range(rho_p.shape[0]):
        if not np.any(rho_p[k1]):
            continue
        Y = V @ rho_p[k1]  # (V_mu rho^+)[a][c]
        Yt = np.transpose(Y, (0, 2, 1)).reshape(n, -1)  # [mu][(c, a)]
        for k2, Zk in Z.items():
            m = k1 + k2
            if m >= nhb:
                continue
            A = Yt @ Zk.T  # sum_{a,c} (V_mu rho^+)[a][c] (V_nu rhobar^-)[c][a]
            out[m] += 2.0 * A[iu, ju]
    return out


def a0_by_pairs(P: np.ndarray, eig: np.ndarray, n_occ: int, domega: float, nhb: int,
                entries: Optional[tuple] = None) -> np.ndarray:
    """The same discrete a0 from the pair vectors (Section 7.A closed form):
    each pair (E, F) carries 2 V_mu^p V_nu^p with the convolution of the two
    one-particle splits as its weight, (1-phi_F)(1-phi_E) at k_F + k_E,
    (1-phi_F) phi_E + phi_F (1-phi_E) one bin up and phi_F phi_E two bins up.
    Packed upper [nhb][n(n+1)/2], or [nhb][len(mu)] for entries = (mu, nu)."""
    k_p, f_p = level_bins(eig[n_occ:], domega)
    k_m, f_m = level_bins(eig[:n_occ], domega)
    base = (k_m[:, None] + k_p[None, :]).ravel()
    fm = np.repeat(f_m, len(k_p))
    fp = np.tile(f_p, len(k_m))
    w = [(1.0 - fp) * (1.0 - fm), (1.0 - fp) * fm + fp * (1.0 - fm), fp * fm]
    if entries is None:
        mu, nu = np.triu_indices(P.shape[0])
    else:
        mu, nu = entries
    out = np.zeros((nhb, len(mu)))
    for d in range(3):
        bins = base + d
        for m in np.unique(bins):
            if m >= nhb:
                continue
            sel = bins == m
            Pw = P[:, sel] * w[d][sel][None, :]
            out[m] += 2.0 * np.einsum("ip,ip->i", Pw[mu], P[nu][:, sel])
    return out


def chi0_from_spectrum(a: np.ndarray, n_omega: int, omega_min: float, omega_max: float, eps: float,
                       js: Optional[Sequence[int]] = None, omegas: Optional[np.ndarray] = None) -> np.ndarray:
    """chi0[j, entry] = sum_{m>=1} a[m, entry] (1/(omega_j - m domega + i eps)
    - 1/(omega_j + m domega + i eps)) for a spectral array a in floating
    point (the Cauchy transform of Section 5.A with a(-s) = -a(s))."""
    d = grid_spacing(n_omega, omega_min, omega_max)
    if omegas is None:
        om = grid_omegas(n_omega, omega_min, omega_max)
        if js is not None:
            om = om[np.asarray(list(js), dtype=np.int64)]
    else:
        om = np.asarray(omegas, dtype=np.float64)
    mvals = np.arange(1, a.shape[0], dtype=np.float64) * d
    w = om[:, None]
    K = 1.0 / (w - mvals[None, :] + 1j * eps) - 1.0 / (w + mvals[None, :] + 1j * eps)
    return K @ a[1:]


# ----------------------------------------------------------------------------
# the GW self-energy from W (Section 5.A eqs. spectral_3 and Cauchy1; Section
# 8.B; Section 4 eq. instantaneous)


def w_spectral(W: np.ndarray, n_omega: int, omega_min: float, omega_max: float) -> np.ndarray:
    """Spectral weight of the dynamical interaction W - v on the mesh bins
    s = k domega, k = 0 .. n_omega/2 - 1:
        gamma[k] = -(domega / pi) Im W(omega = k domega),
    (v is real, so Im(W - v) = Im W; the factor domega turns the density into
    the weight of the bin, as for the histograms).  gamma(-s) = -gamma(s), so
    gamma[0] = 0.  W: [n_omega][n][n] on the whole mesh.  Returns
    [n_omega/2][n][n]."""
    d = grid_spacing(n_omega, omega_min, omega_max)
    j0 = int(round(-omega_min / d))
    g = -(d / math.pi) * np.imag(W[j0:j0 + n_omega // 2])
    g = np.array(g, dtype=np.float64)
    g[0] = 0.0
    return g


def self_energy_spectra(mol, rho_p: np.ndarray, rho_m: np.ndarray, gamma: np.ndarray, n_sbins: int):
    """sigma+^{ab}[m] = sum_{k1 + k2 = m} V_mu^{aa'} rho+_{a'b'}[k1] V_nu^{b'b} gamma^{mu nu}[k2]
    and, at s = -m domega,
    sigma-^{ab}[m] = sum_{k1 + k2 = m} V_mu^{aa'} rhobar-_{a'b'}[k1] V_nu^{b'b} gamma^{mu nu}[k2]:
    eq. spectral_3 on the mesh (sigma-'s explicit minus sign meets
    gamma(-s) = -gamma(s)).  m < n_sbins; weight beyond is dropped.
    Returns (sigma_p, sigma_m), each [n_sbins][n_orb][n_orb]."""
    V = _dense_vertex(mol)
    no = mol.n_orb
    out = []
    for rho in (rho_p, rho_m):
        sig = np.zeros((n_sbins, no, no))
        G = {}
        for k2 in range(gamma.shape[0]):
            if np.any(gamma[k2]):
                G[k2] = np.einsum("mn,ncd->mcd", gamma[k2], V)  # sum_nu gamma^{mu nu} V_nu
        for k1 in range(rho.shape[0]):
            if not np.any(rho[k1]):
                continue
            A = V @ rho[k1]  # (V_mu rho)[a][b']
            for k2, Gk in G.items():
                m = k1 + k2
                if m >= n_sbins:
                    continue
                sig[m] += np.einsum("mab,mbc->ac", A, Gk)
        out.append(sig)
    return out[0], out[1]


def self_energy_spectra_by_levels(mol, gamma: np.ndarray, domega: float, n_sbins: int):
    """The same spectra from the levels: with u^E_{mu a} = sum_{a'} V_mu^{aa'} X_{a'}^E,
    sigma+[m] = sum over empty F of sum_k w_F[m - k] (u^F)^T gamma[k] u^F and
    sigma-[m] likewise over the occupied E at -E (w: the two-bin split of the
    level).  An independent contraction order, for checking."""
    V = _dense_vertex(mol)
    U = np.einsum("mab,bE->Ema", V, mol.X)  # [state][mu][a]
    kk, ph = level_bins(mol.eig, domega)
    no = mol.n_orb
    sp = np.zeros((n_sbins, no, no))
    sm = np.zeros((n_sbins, no, no))
    for E in range(mol.n_orb):
        tgt = sp if E >= mol.n_occ else sm
        for k in range(gamma.shape[0]):
            if not np.any(gamma[k]):
                continue
            blk = U[E].T @ gamma[k] @ U[E]
            for dm, w in ((0, 1.0 - ph[E]), (1, ph[E])):
                m = kk[E] + k + dm
                if m < n_sbins and w != 0.0:
                    tgt[m] += w * blk
    return sp, sm


def self_energy_from_spectra(sp: np.ndarray, sm: np.ndarray, n_omega: int, omega_min: float, omega_max: float,
                             eps: float, js: Optional[Sequence[int]] = None) -> np.ndarray:
    """Sigma(omega_j + i eps) = sum_m sigma+[m] / (omega_j - m domega + i eps)
                              + sum_m sigma-[m] / (omega_j + m domega + i eps)
    (eq. Cauchy1 on the mesh, the sigma+ weights at s = m domega and the
    sigma- weights at s = -m domega).  Returns [len(js)][n][n]."""
    d = grid_spacing(n_omega, omega_min, omega_max)
    om = grid_omegas(n_omega, omega_min, omega_max)
    if js is not None:
        om = om[np.asarray(list(js), dtype=np.int64)]
    mv = np.arange(sp.shape[0], dtype=np.float64) * d
    w = om[:, None]
    Kp = 1.0 / (w - mv[None, :] + 1j * eps)
    Km = 1.0 / (w + mv[None, :] + 1j * eps)
    n = sp.shape[1]
    return (Kp @ sp.reshape(sp.shape[0], -1) + Km @ sm.reshape(sm.shape[0], -1)).reshape(len(om), n, n)


def exchange_self_energy(mol) -> np.ndarray:
    """Sigma_x^{ab} = -V_mu^{aa'} (sum over occupied E of X_{a'}^E X_{b'}^E) V_nu^{b'b} v^{mu nu}
    (Section 4 eq. instantaneous; the minus sign of exchange, i G(0-) v with
    G(0-) = i times the density matrix, is written out here)."""
    V = _dense_vertex(mol)
    Xo = mol.X[:, :mol.n_occ]
    D = Xo @ Xo.T
    A = V @ D  # (V_mu D)[a][b']
    G = np.einsum("mn,ncd->mcd", mol.v, V)
    return -np.einsum("mab,mbc->ac", A, G)


def dyson_dos(mol, n_omega: int, omega_min: float, omega_max: float, eps: float,
              Sigma_c: Optional[np.ndarray] = None, Sigma_x: Optional[np.ndarray] = None,
              Vxc: Optional[np.ndarray] = None, js: Optional[Sequence[int]] = None):
    """G(omega_j + i eps) = [(omega_j + i eps) - H_KS - (Sigma_x + Sigma_c(omega_j) - V_xc)]^{-1}
    with H_KS = X diag(E) X^T in the (orthonormal, S = 1) orbital basis, and
    rho(omega_j) = -(1/pi) Im tr G (Section 2 eq. Dyson with the V_xc
    replacement, Section 3 eq. tensorform-dyson, the DOS definition of
    Section 2).  Sigma_c: [n_omega][n_orb][n_orb] or None (zero).  Returns
    (dos [len(js)], G [len(js)][n_orb][n_orb])."""
    om = grid_omegas(n_omega, omega_min, omega_max)
    jj = np.arange(n_omega) if js is None else np.asarray(list(js), dtype=np.int64)
    H = (mol.X * mol.eig[None, :]) @ mol.X.T
    static = H.copy()
    if Sigma_x is not None:
        static = static + Sigma_x
    if Vxc is not None:
        static = static - Vxc
    n = mol.n_orb
    G = np.empty((len(jj), n, n), dtype=np.complex128)
    for i, j in enumerate(jj):
        A = (om[j] + 1j * eps) * np.eye(n) - static
        if Sigma_c is not None:
            A = A - Sigma_c[j]
        G[i] = np.linalg.inv(A)
    dos = -np.imag(np.trace(G, axis1=1, axis2=2)) / math.pi
    return dos, G
