"""Pins of the CPU oracle to facts fixed by the paper or by mathematics.

None of these re-types an oracle formula and compares it with itself: each
checks a printed number, a closed form, a conservation law, a brute-force
contraction, a symmetry or a limit that a plausible mistake (wrong sign, lost
factor 2, swapped bins, transposed operand, off-by-one grid) would break.
"""
import dataclasses
import math
import os

import numpy as np
import pytest

import gw_synth as gs
import oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = [x.strip() for x in line.split("=")]
                out[k] = float(v)
    return out


def _pipeline(mol, grid):
    P = o.pair_vectors(mol)
    d = grid.domega
    m, fr = o.pair_bins(mol.eig, mol.n_occ, d)
    nhb = o.hist_bins(mol.eig, grid.n_omega, d)
    s = o.frac_bits(P, mol.n_pairs)
    H = o.histogram(P, m, fr, s, nhb)
    return P, m, fr, nhb, s, H


def _tiny(eig, n_occ, V, X=None):
    """Hand-built molecule with one product block spanning all orbitals."""
    n = len(eig)
    if X is None:
        X = np.eye(n)
    if V.ndim == 2:
        V = V[None]
    nprod = V.shape[0]
    centres = np.zeros((nprod, 3))
    centres[:, 0] = np.arange(nprod)
    d2 = (centres[:, None, 0] - centres[None, :, 0]) ** 2
    return gs.Molecule(
        n_orb=n, n_occ=n_occ, eig=np.asarray(eig, float), X=np.asarray(X, float),
        blk_prod=np.array([0, nprod], np.int32), blk_orb=np.array([0, n], np.int32),
        orb_idx=np.arange(n, dtype=np.int32), blk_val=np.array([0, nprod * n * n], np.int64),
        vals=np.ascontiguousarray(V, float).ravel(), centres=centres, atoms=np.zeros((1, 3)),
        v=1.0 / np.sqrt(d2 + 2.0),
    )


# --------------------------------------------------------------------------- grid


def test_grid_reproduces_printed_benzene_broadening():
    """Section 6 prints eps = 1.5*domega = 0.234375 eV for 1024 points on
    [-80, 80] eV; only domega = range/N (omega_max excluded) gives it."""
    g = _read_golden("benzene_grid.txt")
    d = o.grid_spacing(int(g["n_omega"]), g["omega_min_eV"], g["omega_max_eV"])
    assert g["eps_factor"] * d == g["eps_eV"]
    d_alt = (g["omega_max_eV"] - g["omega_min_eV"]) / (g["n_omega"] - 1)
    assert abs(g["eps_factor"] * d_alt - g["eps_eV"]) > 1e-4
    om = o.grid_omegas(int(g["n_omega"]), g["omega_min_eV"], g["omega_max_eV"])
    assert om[0] == g["omega_min_eV"] and om[-1] < g["omega_max_eV"]
    assert om[int(g["n_omega"]) // 2] == 0.0


def test_grid_requires_power_of_two_spacing():
    assert o.grid_shift_bits(2.0 ** -6) == 6
    with pytest.raises(ValueError):
        o.grid_shift_bits(0.03)


# --------------------------------------------------------------------------- pair vertex


@pytest.mark.parametrize("which", ["c0", "chain8"])
def test_pair_vectors_match_dense_bruteforce(which):
    """V^{EF} = X^T V_mu X restricted to occupied x empty, built from the dense
    (assembled) vertex: pins the block indexing and the E/F roles."""
    if which == "c0":
        mol = gs.make_config(0)
    else:
        mol = gs.chain_molecule(8, 7, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10,
                                prod_per_bond=8, bond_cutoff=None)
    P = o.pair_vectors(mol)
    n = mol.n_orb
    dense = np.zeros((mol.n_prod, n, n))
    for b in range(mol.n_blk):
        p0, npr, orbs, mats = mol.block_of(b)
        for i, M in enumerate(mats):
            dense[p0 + i][np.ix_(orbs, orbs)] = M
    full = np.einsum("aE,mab,bF->mEF", mol.X, dense, mol.X)
    ref = full[:, : mol.n_occ, mol.n_occ :].reshape(mol.n_prod, -1)
    assert np.abs(P - ref).max() < 1e-13 * max(1.0, np.abs(ref).max())
    # orthogonal X: sum over ALL (E, F) of (V^EF)^2 equals ||V_mu||_F^2; the
    # occupied-empty block is part of it and never exceeds it
    fro = (dense ** 2).sum(axis=(1, 2))
    assert np.allclose((full ** 2).sum(axis=(1, 2)), fro, rtol=1e-12)
    assert np.all((P ** 2).sum(axis=1) <= fro * (1 + 1e-12))


def test_pair_vectors_identity_eigenvectors():
    """X = 1: V^{EF} is the vertex entry V^{EF} itself."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((4, 4))
    A = A + A.T
    mol = _tiny([-0.5, -0.25, 0.25, 0.5], 2, A)
    P = o.pair_vectors(mol)
    assert np.array_equal(P[0], A[:2, 2:].ravel())


# --------------------------------------------------------------------------- bins


def test_pair_bins_on_and_between_grid_points():
    d = 2.0 ** -5
    eig = np.array([-10 * d, -3 * d, 4 * d, 6.5 * d])
    m, fr = o.pair_bins(eig, 2, d)
    # pairs (E,F): (0,2) 14, (0,3) 16.5, (1,2) 7, (1,3) 9.5
    assert list(m) == [14, 16, 7, 9]
    assert list(fr) == [0.0, 0.5, 0.0, 0.5]
    assert o.hist_bins(eig, 64, d) == 16 + 2
    assert o.hist_bins(eig, 32, d) == 16  # capped at n_omega / 2


def test_frac_bits_rule_bounds():
    for vmax, npairs in [(1.4737, 64), (0.28, 57600), (2.0 ** -3, 518400), (3.0, 1)]:
        P = np.array([[vmax, -vmax / 3]])
        s = o.frac_bits(P, npairs)
        x = math.ldexp(vmax * vmax, s)
        assert x <= 2.0 ** 50
        assert 2 * npairs * 2 * x < 2.0 ** 63
        # the rule bounds vmax by the next power of two, so it is within three
        # bits of the largest safe exponent
        x3 = 8 * x
        assert x3 > 2.0 ** 50 or 2 * npairs * 2 * x3 >= 2.0 ** 61


# --------------------------------------------------------------------------- histogram


def test_histogram_sum_rule_and_first_moment():
    """Zeroth moment: integral of a0_{mu nu} = 2 sum_p V_mu^p V_nu^p (the sum
    rule; on the diagonal it is 2 sum_p |V_mu^p|^2).  First moment: linear
    deposition keeps the pole position, sum_m m domega H_m = 2 sum_p Delta_p
    V_mu V_nu.  A lost spin factor, swapped lo/hi bins, nearest-bin deposition
    or an off-by-one bin all fail one of the two."""
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    iu, ju = np.triu_indices(mol.n_prod)
    lsb = 2.0 ** -s
    pair = P[iu] * P[ju]
    zeroth = np.ldexp(H.sum(axis=0).astype(float), -s)
    ref0 = 2.0 * pair.sum(axis=1)
    assert np.abs(zeroth - ref0).max() <= mol.n_pairs * (2 * lsb + 1e-15 * np.abs(pair).max())
    diag = [o.packed_index(i, i, mol.n_prod) for i in range(mol.n_prod)]
    assert np.allclose(zeroth[diag], 2.0 * (P ** 2).sum(axis=1), rtol=1e-12)
    d = grid.domega
    delta = (mol.eig[mol.n_occ:][None, :] - mol.eig[: mol.n_occ][:, None]).ravel()
    first = d * np.ldexp((np.arange(nhb)[:, None] * H).sum(axis=0).astype(float), -s)
    ref1 = 2.0 * (pair * delta[None, :]).sum(axis=1)
    tol1 = mol.n_pairs * nhb * d * 4 * lsb + 1e-13 * np.abs(ref1).max()
    assert np.abs(first - ref1).max() <= tol1
    # the first moment is far more sensitive than the tolerance: nearest-bin
    # deposition would miss it by ~ domega * |V V| per pair
    assert np.abs(pair).sum(axis=1).max() * d * 0.05 > tol1


def test_histogram_order_free_and_c_matches():
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    perm = np.random.default_rng(5).permutation(mol.n_pairs)
    H2 = o.histogram(P[:, perm], m[perm], fr[perm], s, nhb)
    assert np.array_equal(H, H2)
    Hc, dropped = o.histogram_c(P, m, fr, s, nhb)
    assert dropped == 0 and np.array_equal(H, Hc)
    sel = np.array([3, 17, 40]), np.array([3, 50, 63])
    Hs, _ = o.histogram_c(P, m, fr, s, nhb, sel[0], sel[1])
    assert np.array_equal(Hs, H[:, o.packed_index(sel[0], sel[1], mol.n_prod)])


def test_histogram_drops_pairs_beyond_grid():
    d = 2.0 ** -3
    eig = np.array([-1.0, 0.25, 2.0])  # pair energies 1.25 (m=10), 3.0 (m=24)
    V = np.array([[0.0, 0.3, 0.2], [0.3, 0.0, 0.0], [0.2, 0.0, 0.0]])
    mol = _tiny(eig, 1, V)
    P = o.pair_vectors(mol)
    m, fr = o.pair_bins(eig, 1, d)
    nhb = o.hist_bins(eig, 32, d)  # 16 bins: m=24 does not fit
    assert nhb == 16
    s = o.frac_bits(P, 2)
    H = o.histogram(P, m, fr, s, nhb)
    _, dropped = o.histogram_c(P, m, fr, s, nhb)
    assert dropped == 1
    assert H[10, 0] == 2 * int(np.rint(math.ldexp(0.09, s)))


# --------------------------------------------------------------------------- chi0


def test_chi0_single_pole_closed_form():
    """One product, one pair: chi0 = 2 V^2 [1/(w - D + i eps) - 1/(w + D + i eps)]
    when D sits on a grid point, and the average of the two neighbouring poles
    when it sits half way (linear deposition)."""
    grid = gs.config_grid(0)
    d = grid.domega
    om = grid.omegas()
    for D, parts in [(24 * d, [(24, 1.0)]), (24.5 * d, [(24, 0.5), (25, 0.5)])]:
        eig = np.array([-D / 2, D / 2])
        V = np.array([[0.0, 0.7], [0.7, 0.0]])
        mol = _tiny(eig, 1, V)
        P, m, fr, nhb, s, H = _pipeline(mol, grid)
        chi = o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps)[:, 0]
        ref = sum(w * 2 * 0.49 * (1 / (om - k * d + 1j * grid.eps) - 1 / (om + k * d + 1j * grid.eps))
                  for k, w in parts)
        assert np.abs(chi - ref).max() < 1e-12 * np.abs(ref).max()


def test_chi0_symmetries():
    """chi0 is complex-symmetric in (mu, nu) (Section 5: real basis),
    chi0(-w) = conj chi0(w) (retarded reading), -Im chi0(w>0) is PSD."""
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min,
                                          grid.omega_max, grid.eps), mol.n_prod)
    N = grid.n_omega
    for j in [1, 37, 100, 127]:
        a, b = chi[N - j], chi[j]
        assert np.abs(a - np.conj(b)).max() <= 1e-13 * np.abs(b).max()
    for j in [N // 2 + 5, N // 2 + 40, N // 2 + 100]:
        ev = np.linalg.eigvalsh(-chi[j].imag)
        assert ev.min() > -1e-10 * ev.max()
    assert np.abs(chi[N // 2].imag).max() < 1e-12 * np.abs(chi).max()


def test_chi0_converges_to_true_poles_second_order():
    """Refining the mesh at fixed eps, the binned chi0 approaches the closed
    form with the poles at their true energies (Section 7.A) as domega^2."""
    mol = gs.make_config(0)
    P = o.pair_vectors(mol)
    eps = 0.05
    errs = []
    test_w = np.array([0.45, 0.8, 1.3, 2.1])
    ref = o.chi0_poles(P, mol.eig, mol.n_occ, test_w, eps)
    iu, ju = np.triu_indices(mol.n_prod)
    for n in [256, 512, 1024]:
        d = 8.0 / n
        m, fr = o.pair_bins(mol.eig, mol.n_occ, d)
        nhb = o.hist_bins(mol.eig, n, d)
        s = o.frac_bits(P, mol.n_pairs)
        H = o.histogram(P, m, fr, s, nhb)
        chi = o.chi0_from_hist(H, s, n, -4.0, 4.0, eps, omegas=test_w)
        errs.append(np.linalg.norm(chi - ref[:, iu, ju]) / np.linalg.norm(ref[:, iu, ju]))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


def test_chi0_kramers_kronig():
    """Re chi0 is the Hilbert transform of Im chi0 (analytic in the upper half
    plane): checks signs, the factor pi and the odd extension a(-s) = -a(s)."""
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    e = o.packed_index(5, 5, mol.n_prod)
    h = grid.eps / 10
    L = 60.0
    w = np.arange(-L, L, h)
    chi = o.chi0_from_hist(H[:, [e]], s, grid.n_omega, grid.omega_min, grid.omega_max,
                           grid.eps, omegas=w)[:, 0]
    im = chi.imag
    for w0_idx in [len(w) // 2 + 40, len(w) // 2 + 400, len(w) // 2 - 700]:
        k = np.arange(len(w)) - w0_idx
        odd = (k % 2) != 0
        # Maclaurin rule for the principal value: sum over odd offsets, weight 2h
        re_kk = (2 * h / np.pi) * np.sum(im[odd] / (w[odd] - w[w0_idx]))
        assert abs(re_kk - chi.real[w0_idx]) < 2e-3 * np.abs(chi).max()


# --------------------------------------------------------------------------- W


def test_W_reduces_to_v_without_vertex():
    """V -> 0 removes all screening: W = v exactly; and W - v scales as t^2
    under V -> tV (chi0 is quadratic in V)."""
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    z = mol.scaled_vertex(0.0)
    P, m, fr, nhb, s, H = _pipeline(z, grid)
    assert not H.any()
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max,
                                          grid.eps, js=[140]), mol.n_prod)[0]
    W = o.screened_W(mol.v, chi)
    assert np.array_equal(W, mol.v.astype(complex))
    dev = []
    for t in [1e-3, 2e-3]:
        P, m, fr, nhb, s, H = _pipeline(mol.scaled_vertex(t), grid)
        chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min,
                                              grid.omega_max, grid.eps, js=[140]), mol.n_prod)[0]
        dev.append(np.linalg.norm(o.screened_W(mol.v, chi) - mol.v))
    assert abs(dev[1] / dev[0] - 4.0) < 0.01


def test_W_one_by_one_closed_form():
    grid = gs.config_grid(0)
    d = grid.domega
    eig = np.array([-10 * d, 14.25 * d])
    mol = _tiny(eig, 1, np.array([[0.1, 0.9], [0.9, -0.2]]))
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    chi = o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps)
    v = mol.v[0, 0]
    for j in [128, 150, 151, 200, 20]:
        W = o.screened_W(mol.v, chi[j].reshape(1, 1))[0, 0]
        assert abs(W - v / (1 - v * chi[j, 0])) < 1e-14 * abs(W)


def test_W_symmetric_and_series():
    """W^T = W in a real basis (Section 5); for weak response W matches the
    series v + v chi0 v + v chi0 v chi0 v of Section 7.B eq. W-series."""
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max,
                                          grid.eps, js=[150]), mol.n_prod)[0]
    W = o.screened_W(mol.v, chi)
    assert np.abs(W - W.T).max() < 1e-10 * np.abs(W).max()
    weak = mol.scaled_vertex(0.01)
    P, m, fr, nhb, s, H = _pipeline(weak, grid)
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max,
                                          grid.eps, js=[150]), mol.n_prod)[0]
    v = mol.v
    W = o.screened_W(v, chi)
    vc = v @ chi
    series = v + vc @ v + vc @ vc @ v
    nxt = np.linalg.norm(vc @ vc @ vc @ v)
    assert np.linalg.norm(W - series) < 3 * nxt
    assert np.linalg.norm(W - v - vc @ v) > 0.3 * np.linalg.norm(vc @ vc @ v)


def test_compressed_W_equals_full_when_rank_fits():
    """Section 7.B: if chi0 acts inside the kept subspace nothing is lost.  The
    synthetic v has rank = number of distinct centres (7 for the tiny chain),
    so k = 16 reproduces the full W, k = 4 does not, and the compressed form
    equals (1 - v_k chi0)^{-1} v_k with v_k the rank-k truncation of v."""
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max,
                                          grid.eps, js=[150]), mol.n_prod)[0]
    Wf = o.screened_W(mol.v, chi)
    Wk = o.screened_W_compressed(mol.v, chi, 16)
    assert np.linalg.norm(Wk - Wf) < 1e-9 * np.linalg.norm(Wf)
    W4 = o.screened_W_compressed(mol.v, chi, 4)
    U, lam = o.compress_basis(mol.v, 4)
    vk = (U * lam) @ U.T
    alt = np.linalg.solve(np.eye(mol.n_prod) - vk @ chi, vk.astype(complex))
    assert np.linalg.norm(W4 - alt) < 1e-10 * np.linalg.norm(alt)
    assert np.linalg.norm(W4 - Wf) > 1e-3 * np.linalg.norm(Wf)


def test_projected_histogram_is_projected_chi0():
    """Histogram of U^T V^p equals U^T chi0 U up to fixed-point rounding
    (Section 8.A: compress the response as soon as it is formed)."""
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    U, lam = o.compress_basis(mol.v, 10)
    Pt = o.project_pairs(P, U)
    st = o.frac_bits(Pt, mol.n_pairs)
    Ht = o.histogram(Pt, m, fr, st, nhb)
    js = [150, 170]
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max,
                                          grid.eps, js=js), mol.n_prod)
    chit = o.unpack_upper(o.chi0_from_hist(Ht, st, grid.n_omega, grid.omega_min,
                                           grid.omega_max, grid.eps, js=js), 10)
    for i in range(len(js)):
        ref = U.T @ chi[i] @ U
        assert np.abs(chit[i] - ref).max() < 1e-9 * np.abs(ref).max()


def _chi_of_pairs(P, mol, sel, omega, eps):
    """Retarded chi0 of the listed electron-hole pairs at one frequency
    directly from Section 7.A's double sum (no mesh)."""
    e_occ, e_vir = mol.eig[:mol.n_occ], mol.eig[mol.n_occ:]
    delta = (e_vir[None, :] - e_occ[:, None]).ravel()[sel]
    g = 1.0 / (omega - delta + 1j * eps) - 1.0 / (omega + delta + 1j * eps)
    return 2.0 * (P[:, sel] * g[None, :]) @ P[:, sel].T


def test_pair_subset_threshold():
    """Section 7.A eq. subsetof_vef: exactly the pairs with F - E below the
    threshold, for hand-placed levels."""
    eig = np.array([-0.5, -0.3, 0.1, 0.4, 0.9])
    sel = o.pair_subset(eig, 2, 0.75)
    # pairs (E, F): (-0.5, 0.1)=0.6 (-0.5,0.4)=0.9 (-0.5,0.9)=1.4 (-0.3,0.1)=0.4 (-0.3,0.4)=0.7 (-0.3,0.9)=1.2
    assert list(sel) == [0, 3, 4]


def test_pair_basis_orthonormal_and_projector():
    """Section 7.A: Z is orthonormal in the Coulomb metric
    (eq. global-basis-orthogonality), spans the generators' visible part, and
    P = v Z Z^T is a projector (P^2 = P) that reproduces v X."""
    mol = gs.chain_molecule(3, 5)
    P = o.pair_vectors(mol)
    sel = o.pair_subset(mol.eig, mol.n_occ, 1.0)
    X = P[:, sel]
    lam_all = np.linalg.eigvalsh(X.T @ mol.v @ X)[::-1]
    k = int(np.sum(lam_all > 1e-10 * lam_all[0]))
    Z, lam = o.pair_basis(X, mol.v, k)
    assert np.allclose(lam, lam_all[:k], rtol=1e-10, atol=0)
    G = Z.T @ mol.v @ Z
    assert np.abs(G - np.eye(k)).max() < 1e-9
    Pr = o.pair_projector(Z, mol.v)
    assert np.abs(Pr @ Pr - Pr).max() < 1e-9 * np.abs(Pr).max()
    # every generator's Coulomb image lies in the subspace: P (v X) = v X
    VX = mol.v @ X
    assert np.abs(Pr @ VX - VX).max() < 1e-9 * np.abs(VX).max()


def test_pair_basis_W_exact_when_chi0_in_subspace():
    """Section 7.B eq. chi_RPA: when chi0 is built from the generating pairs
    only, it acts inside the subspace and W = v + Z^mu chi_RPA Z^nu equals the
    full (1 - v chi0)^{-1} v; keeping fewer eigenvectors loses accuracy."""
    mol = gs.make_config(0)
    P = o.pair_vectors(mol)
    for thr in (10.0, 1.2):
        sel = o.pair_subset(mol.eig, mol.n_occ, thr)
        assert 0 < len(sel) <= mol.n_pairs
        X = P[:, sel]
        lam_all = np.linalg.eigvalsh(X.T @ mol.v @ X)[::-1]
        k = int(np.sum(lam_all > 1e-10 * lam_all[0]))
        Z, _ = o.pair_basis(X, mol.v, k)
        for w in (0.3, 1.1, -0.7):
            chi = _chi_of_pairs(P, mol, sel, w, 0.05)
            Wf = o.screened_W(mol.v, chi)
            Wp = o.screened_W_pair_basis(mol.v, chi, Z)
            assert np.linalg.norm(Wp - Wf) < 1e-9 * np.linalg.norm(Wf)
        Z2, _ = o.pair_basis(X, mol.v, max(1, k - 3))
        chi = _chi_of_pairs(P, mol, sel, 0.3, 0.05)
        Wf = o.screened_W(mol.v, chi)
        assert np.linalg.norm(o.screened_W_pair_basis(mol.v, chi, Z2) - Wf) > 1e-4 * np.linalg.norm(Wf)


def test_two_window_same_mesh_is_single_window():
    """Section 5.B eq. win2-for-response: the two windows partition the pairs,
    so with the same mesh and broadening in both windows the result is the
    single-window chi0; the split sits on a bin edge below lambda."""
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    lam = o.two_window_split(grid.domega, grid.omega_max, grid.domega)
    assert lam == grid.omega_max - grid.domega
    g = (grid.n_omega, grid.omega_min, grid.omega_max, grid.eps)
    js = [grid.n_omega // 2 + 3, 150, 60, 250]
    two = o.chi0_two_window(P, mol.eig, mol.n_occ, s, g, g, js=js)
    one = o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps, js=js)
    assert np.abs(two - one).max() < 1e-12 * np.abs(one).max()


def test_two_window_partition_and_sum_rule():
    """Every pair lands in exactly one window: the small-window histogram
    (fine mesh) and the large-window one (coarse mesh) carry the integer sum
    rule 2 sum_p V_mu V_nu together, and the split agrees with the bins."""
    mol = gs.chain_molecule(3, 5)
    P = o.pair_vectors(mol)
    ds, dl = 2.0 ** -6, 2.0 ** -3
    lam = o.two_window_split(ds, 0.5, dl)
    assert lam == 0.375 and lam <= 0.5 - ds
    delta = (mol.eig[mol.n_occ:][None, :] - mol.eig[:mol.n_occ][:, None]).ravel()
    low = delta < lam
    assert 0 < low.sum() < mol.n_pairs
    s = o.frac_bits(P, mol.n_pairs)
    ms, fs = o.pair_bins(mol.eig, mol.n_occ, ds)
    ml, fl = o.pair_bins(mol.eig, mol.n_occ, dl)
    assert ms[low].max() + 1 < 0.5 / ds  # small-window pairs stay inside the small mesh
    assert np.all(ml[~low] >= lam / dl)  # large-window pairs start at or above the split bin
    Hs = o.histogram(P[:, low], ms[low], fs[low], s, o.hist_bins(mol.eig, 64, ds))
    Hl = o.histogram(P[:, ~low], ml[~low], fl[~low], s, o.hist_bins(mol.eig, 64, dl))
    iu, ju = np.triu_indices(mol.n_prod)
    t = np.rint(np.ldexp(P[iu] * P[ju], s)).astype(np.int64)
    assert np.array_equal(Hs.sum(axis=0) + Hl.sum(axis=0), 2 * t.sum(axis=1))


def test_two_window_sampled_entries_equal_full():
    """The sampled-entry form of the two-window chi0 (the C histogram on
    chosen entries) returns exactly the full form's values at those entries."""
    mol = gs.chain_molecule(3, 5)
    P = o.pair_vectors(mol)
    s = o.frac_bits(P, mol.n_pairs)
    small, large = gs.two_window_grids()
    sm = (small.n_omega, small.omega_min, small.omega_max, small.eps)
    lg = (large.n_omega, large.omega_min, large.omega_max, large.eps)
    js = [small.n_omega // 2 + 5, 40]
    full = o.chi0_two_window(P, mol.eig, mol.n_occ, s, sm, lg, js=js)
    iu, ju = np.triu_indices(mol.n_prod)
    pick = np.array([0, 7, len(iu) // 2, len(iu) - 1])
    part = o.chi0_two_window(P, mol.eig, mol.n_occ, s, sm, lg, js=js, entries=(iu[pick], ju[pick]))
    assert np.array_equal(part, full[:, pick])


# ---------------------------------------------------------------- the paper's own a0 route


def _time_route(mol, domega, n_omega=256):
    rho_p, rho_m = o.spectral_densities(mol, domega)
    nhb = o.level_hist_bins(mol.eig, mol.n_occ, n_omega, domega)
    return rho_p, rho_m, nhb, o.a0_by_convolution(mol, rho_p, rho_m, nhb)


def test_spectral_densities_completeness():
    """Section 5 density matrix on the mesh: summed over bins, rho^+ is the
    projector onto the empty states and rhobar^- the one onto the occupied
    states (X orthogonal), so together they give the identity; each pole
    keeps its position (first moment)."""
    mol = gs.make_config(0)
    d = gs.config_grid(0).domega
    rho_p, rho_m = o.spectral_densities(mol, d)
    Xv, Xo = mol.X[:, mol.n_occ:], mol.X[:, :mol.n_occ]
    assert np.abs(rho_p.sum(0) - Xv @ Xv.T).max() < 1e-14
    assert np.abs(rho_m.sum(0) - Xo @ Xo.T).max() < 1e-14
    assert np.abs(rho_p.sum(0) + rho_m.sum(0) - np.eye(mol.n_orb)).max() < 1e-13
    kk = np.arange(rho_p.shape[0])[:, None, None] * d
    assert np.abs((kk * rho_p).sum(0) - (Xv * mol.eig[mol.n_occ:]) @ Xv.T).max() < 1e-14
    kk = np.arange(rho_m.shape[0])[:, None, None] * d
    assert np.abs((kk * rho_m).sum(0) + (Xo * mol.eig[:mol.n_occ]) @ Xo.T).max() < 1e-14


@pytest.mark.parametrize("which", ["tiny", "chain3"])
def test_time_route_equals_pair_form(which):
    """The convolution of the two densities contracted with the vertex equals
    the pair form: each pair (E, F) with weight 2 V_mu^p V_nu^p spread by the
    convolution of its two one-particle splits.  The pair vectors come from an
    independent contraction (pair_vectors), so a misplaced index or density
    in the convolution breaks this."""
    mol = gs.make_config(0) if which == "tiny" else gs.chain_molecule(3, 5)
    d = 2.0 ** -5
    _, _, nhb, a = _time_route(mol, d)
    P = o.pair_vectors(mol)
    b = o.a0_by_pairs(P, mol.eig, mol.n_occ, d, nhb)
    assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()


def test_time_route_sum_rule_and_first_moment():
    """Zeroth moment: the integer-free sum rule 2 sum_p V_mu V_nu; first
    moment: 2 sum_p Delta_p V_mu V_nu (linear splits keep each pole's
    position, and the convolution adds the two positions)."""
    mol = gs.chain_molecule(3, 5)
    d = 2.0 ** -5
    _, _, nhb, a = _time_route(mol, d)
    P = o.pair_vectors(mol)
    iu, ju = np.triu_indices(mol.n_prod)
    pp = P[iu] * P[ju]
    delta = (mol.eig[mol.n_occ:][None, :] - mol.eig[:mol.n_occ][:, None]).ravel()
    s0 = 2.0 * pp.sum(1)
    s1 = 2.0 * (pp * delta[None, :]).sum(1)
    assert np.abs(a.sum(0) - s0).max() <= 1e-13 * np.abs(s0).max()
    m1 = (np.arange(nhb)[:, None] * d * a).sum(0)
    assert np.abs(m1 - s1).max() <= 1e-13 * np.abs(s1).max()


def test_time_route_on_mesh_equals_pair_histogram():
    """With every level on a mesh point no pole is split, and the two routes
    (convolution of densities, int64 pair histogram) put the same weight in
    the same bins, up to the histogram's 2^-s quantisation."""
    d = 2.0 ** -5
    mol = gs.make_config(0)
    eig = np.round(mol.eig / d) * d
    assert np.all(np.diff(eig) >= 0) and eig[mol.n_occ - 1] < 0 <= eig[mol.n_occ]
    mol = dataclasses.replace(mol, eig=eig)
    _, _, nhb, a = _time_route(mol, d)
    P = o.pair_vectors(mol)
    m, fr = o.pair_bins(mol.eig, mol.n_occ, d)
    assert not fr.any()
    s = o.frac_bits(P, mol.n_pairs)
    H = o.histogram(P, m, fr, s, o.hist_bins(mol.eig, 256, d))
    h = np.ldexp(H.astype(np.float64), -s)
    k = min(len(h), nhb)
    assert np.abs(a[:k] - h[:k]).max() <= 2.0 * mol.n_pairs * 2.0 ** -s
    assert not a[k:].any() and not h[k:].any()


def test_chi0_from_spectrum_is_the_histogram_transform():
    mol = gs.make_config(0)
    grid = gs.config_grid(0)
    P, m, fr, nhb, s, H = _pipeline(mol, grid)
    js = [grid.n_omega // 2 + 3, 7, 200]
    a = o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps, js=js)
    b = o.chi0_from_spectrum(np.ldexp(H.astype(np.float64), -s), grid.n_omega, grid.omega_min, grid.omega_max,
                             grid.eps, js=js)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- the self-energy downstream of W


def _w_on_mesh(mol, n_omega=64, wmax=4.0):
    g = gs.Grid(n_omega, -wmax, wmax, 0.0)
    g.eps = 1.5 * g.domega
    d = g.domega
    P = o.pair_vectors(mol)
    m, fr = o.pair_bins(mol.eig, mol.n_occ, d)
    s = o.frac_bits(P, mol.n_pairs)
    H = o.histogram(P, m, fr, s, o.hist_bins(mol.eig, n_omega, d))
    chi = o.unpack_upper(o.chi0_from_hist(H, s, n_omega, g.omega_min, g.omega_max, g.eps), mol.n_prod)
    W = np.array([o.screened_W(mol.v, c) for c in chi])
    return g, W


def test_w_spectral_is_positive_and_odd():
    """-Im W(omega > 0) is positive semidefinite (Im chi0 <= 0 and v >= 0 give
    Im W <= 0), W(-omega) = W(omega)* makes it odd, and bin 0 is empty."""
    mol = gs.make_config(0)
    g, W = _w_on_mesh(mol)
    gam = o.w_spectral(W, g.n_omega, g.omega_min, g.omega_max)
    assert gam.shape == (g.n_omega // 2, mol.n_prod, mol.n_prod)
    assert not gam[0].any()
    scale = np.abs(gam).max()
    for k in range(1, len(gam)):
        assert np.linalg.eigvalsh(gam[k]).min() >= -1e-12 * scale


def test_w_spectral_rebuilds_w_by_the_cauchy_integral():
    """The weights gamma[k] are the spectral function of W - v on the mesh
    (Section 5.A: a retarded correlator is the Cauchy integral of minus its
    imaginary part over pi).  With F(z) = W(z + i eps) - v, analytic above the
    real axis, F(omega + i eta) = int rho(s) / (omega + i eta - s) ds with
    rho(s) = -(1/pi) Im W(s + i eps); the trapezoid sum of that integral over
    the mesh, with the odd extension gamma(-s) = -gamma(s), is
        sum_k gamma[k] [1/(z - k domega) - 1/(z + k domega)],  z = omega + i eta,
    and it must equal W(omega + i(eps + eta)) - v solved directly at off-mesh
    omega (chi0 summed at the larger broadening).  The sum converges
    exponentially in eps/domega and eta/domega; the vertex is weakened
    (V -> 0.3 V) so that the weight of W - v stays well inside the window.
    The same check fails for a lost domega (1/pi), a doubled weight
    (2 domega/pi) and a zero-frequency bin moved by one mesh point."""
    mol = gs.make_config(0).scaled_vertex(0.3)
    n_omega, wmax = 1024, 16.0
    g = gs.Grid(n_omega, -wmax, wmax, 0.0)
    d = g.domega
    g.eps = 1.5 * d
    eta = 1.5 * d
    P, m, fr, nhb, s, H = _pipeline(mol, g)
    chi = o.unpack_upper(o.chi0_from_hist(H, s, n_omega, g.omega_min, g.omega_max, g.eps), mol.n_prod)
    W = np.array([o.screened_W(mol.v, c) for c in chi])
    gam = o.w_spectral(W, n_omega, g.omega_min, g.omega_max)
    oms = np.array([0.0, 0.37, 0.91, 1.53, 2.2, 3.1, -0.8])  # off the mesh except 0
    chiz = o.unpack_upper(o.chi0_from_hist(H, s, n_omega, g.omega_min, g.omega_max, g.eps + eta, omegas=oms),
                          mol.n_prod)
    F = np.array([o.screened_W(mol.v, c) for c in chiz]) - mol.v[None]

    def mismatch(gm):
        k = np.arange(gm.shape[0]) * d
        z = oms[:, None] + 1j * eta
        K = 1.0 / (z - k[None, :]) - 1.0 / (z + k[None, :])
        R = np.einsum("jk,kab->jab", K, gm)
        return np.linalg.norm(R - F) / np.linalg.norm(F)

    assert mismatch(gam) <= 2e-3
    # planted mistakes, each built from W on the CPU: they must all fail
    j0 = n_omega // 2

    def from_bin(jz):
        gg = -(d / math.pi) * np.imag(W[jz:jz + n_omega // 2])
        gg[0] = 0.0
        return gg

    for bad in (gam / d, 2.0 * gam, from_bin(j0 + 1), from_bin(j0 - 1)):
        assert mismatch(bad) >= 1e-2


@pytest.mark.parametrize("which", ["tiny", "chain3"])
def test_self_energy_convolution_equals_levels(which):
    """eq. spectral_3 on the mesh, summed as a convolution of the densities
    with gamma, equals the sum over levels of (u^E)^T gamma u^E with
    u^E = V X^E (an independent contraction order)."""
    mol = gs.make_config(0) if which == "tiny" else gs.chain_molecule(3, 5)
    g, W = _w_on_mesh(mol)
    gam = o.w_spectral(W, g.n_omega, g.omega_min, g.omega_max)
    rho_p, rho_m = o.spectral_densities(mol, g.domega)
    sp, sm = o.self_energy_spectra(mol, rho_p, rho_m, gam, g.n_omega // 2)
    lp, lm = o.self_energy_spectra_by_levels(mol, gam, g.domega, g.n_omega // 2)
    assert np.abs(sp - lp).max() <= 1e-13 * np.abs(lp).max()
    assert np.abs(sm - lm).max() <= 1e-13 * np.abs(lm).max()


def test_self_energy_zeroth_moment_factorises():
    """The sum over bins of a convolution is the product of the sums: with no
    weight dropped, sum_m sigma+[m] = V_mu D+ V_nu Gamma^{mu nu}, D+ the
    projector on the empty states and Gamma = sum_k gamma[k] (and likewise
    for sigma- with the occupied projector)."""
    mol = gs.make_config(0)
    g, W = _w_on_mesh(mol, n_omega=256)
    gam = o.w_spectral(W, g.n_omega, g.omega_min, g.omega_max)
    gam[g.n_omega // 4:] = 0.0  # keep every convolution inside the bins
    rho_p, rho_m = o.spectral_densities(mol, g.domega)
    sp, sm = o.self_energy_spectra(mol, rho_p, rho_m, gam, g.n_omega // 2)
    V = np.zeros((mol.n_prod, mol.n_orb, mol.n_orb))
    for b in range(mol.n_blk):
        p0, _, orbs, mats = mol.block_of(b)
        for i, M in enumerate(mats):
            V[p0 + i][np.ix_(orbs, orbs)] = M
    Gam = gam.sum(0)
    for sig, X in ((sp, mol.X[:, mol.n_occ:]), (sm, mol.X[:, :mol.n_occ])):
        D = X @ X.T
        ref = sum(Gam[i, j] * V[i] @ D @ V[j] for i in range(mol.n_prod) for j in range(mol.n_prod))
        assert np.abs(sig.sum(0) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_self_energy_cauchy_single_pole_and_sign():
    """eq. Cauchy1 on the mesh: one unit weight of sigma+ at m0 gives
    1/(omega - m0 domega + i eps), one of sigma- at m0 gives
    1/(omega + m0 domega + i eps); from W of a molecule, Sigma is complex
    symmetric with Im Sigma negative semidefinite at every mesh point."""
    n_omega, wmax, eps = 64, 4.0, 0.1
    d = 2 * wmax / n_omega
    om = -wmax + d * np.arange(n_omega)
    sp = np.zeros((32, 2, 2))
    sm = np.zeros((32, 2, 2))
    sp[5, 0, 1] = sp[5, 1, 0] = 1.0
    sm[9, 1, 1] = 1.0
    S = o.self_energy_from_spectra(sp, sm, n_omega, -wmax, wmax, eps)
    assert np.abs(S[:, 0, 1] - 1.0 / (om - 5 * d + 1j * eps)).max() < 1e-15
    assert np.abs(S[:, 1, 1] - 1.0 / (om + 9 * d + 1j * eps)).max() < 1e-15
    assert not S[:, 0, 0].any()
    mol = gs.make_config(0)
    g, W = _w_on_mesh(mol)
    gam = o.w_spectral(W, g.n_omega, g.omega_min, g.omega_max)
    rho_p, rho_m = o.spectral_densities(mol, g.domega)
    sp, sm = o.self_energy_spectra(mol, rho_p, rho_m, gam, g.n_omega // 2)
    S = o.self_energy_from_spectra(sp, sm, g.n_omega, g.omega_min, g.omega_max, g.eps)
    assert np.abs(S - np.transpose(S, (0, 2, 1))).max() <= 1e-13 * np.abs(S).max()
    for x in S:
        assert np.linalg.eigvalsh(x.imag).max() <= 1e-13 * np.abs(S).max()


def test_exchange_self_energy_by_levels():
    """Section 4 eq. instantaneous: -sum over occupied E of (u^E)^T v u^E,
    u^E = V X^E; symmetric and negative semidefinite (v >= 0)."""
    mol = gs.chain_molecule(3, 5)
    Sx = o.exchange_self_energy(mol)
    V = np.zeros((mol.n_prod, mol.n_orb, mol.n_orb))
    for b in range(mol.n_blk):
        p0, _, orbs, mats = mol.block_of(b)
        for i, M in enumerate(mats):
            V[p0 + i][np.ix_(orbs, orbs)] = M
    ref = np.zeros_like(Sx)
    for E in range(mol.n_occ):
        u = V @ mol.X[:, E]  # [mu][a]
        ref -= u.T @ mol.v @ u
    assert np.abs(Sx - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(Sx - Sx.T).max() <= 1e-12 * np.abs(Sx).max()
    assert np.linalg.eigvalsh(Sx).max() <= 1e-10 * np.abs(Sx).max()


def test_dyson_dos_closed_forms():
    """No self-energy: G = G0 and the DOS is a sum of Lorentzians of width eps
    at the levels; a constant real shift of the self-energy moves every
    level; Sigma = V_xc cancels exactly."""
    mol = gs.make_config(0)
    n_omega, wmax, eps = 128, 4.0, 0.05
    om = -wmax + (2 * wmax / n_omega) * np.arange(n_omega)
    lor = lambda E: (eps / math.pi) / ((om[:, None] - E[None, :]) ** 2 + eps ** 2)
    dos, G = o.dyson_dos(mol, n_omega, -wmax, wmax, eps)
    assert np.abs(dos - lor(mol.eig).sum(1)).max() < 1e-10 * dos.max()
    d = 0.3
    dos2, _ = o.dyson_dos(mol, n_omega, -wmax, wmax, eps, Sigma_x=d * np.eye(mol.n_orb))
    assert np.abs(dos2 - lor(mol.eig + d).sum(1)).max() < 1e-10 * dos2.max()
    rng = np.random.default_rng(3)
    M = rng.standard_normal((mol.n_orb, mol.n_orb))
    M = M + M.T
    dos3, G3 = o.dyson_dos(mol, n_omega, -wmax, wmax, eps, Sigma_x=M, Vxc=M)
    assert np.abs(G3 - G).max() <= 1e-12 * np.abs(G).max()
    # G0 in the orbital basis is X diag(1/(w - E + i eps)) X^T
    j = 77
    ref = (mol.X / (om[j] + 1j * eps - mol.eig)[None, :]) @ mol.X.T
    assert np.abs(G[j] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_dyson_dos_diagonal_self_energy():
    """A self-energy diagonal in the Kohn-Sham eigenbasis, Sigma_c(w) =
    X diag(s(w)) X^T, gives G = X diag(1/(w + i eps - E - s(w))) X^T level by
    level (fixes the frequency index and the sign of Sigma_c), and V_xc = c 1
    moves every level by -c (fixes the sign of V_xc)."""
    mol = gs.make_config(0)
    n_omega, wmax, eps = 64, 4.0, 0.05
    om = -wmax + (2 * wmax / n_omega) * np.arange(n_omega)
    rng = np.random.default_rng(5)
    # a causal single-pole self-energy per level: s_a(w) = g_a / (w - p_a + i eta)
    g = rng.uniform(0.01, 0.1, mol.n_orb)
    p = rng.uniform(-2.0, 2.0, mol.n_orb)
    s = g[None, :] / (om[:, None] - p[None, :] + 0.2j)
    Sc = np.einsum("ia,wa,ja->wij", mol.X, s, mol.X)
    dos, G = o.dyson_dos(mol, n_omega, -wmax, wmax, eps, Sigma_c=Sc)
    for j in (0, 13, 40, n_omega - 1):
        ref = (mol.X / (om[j] + 1j * eps - mol.eig - s[j])[None, :]) @ mol.X.T
        assert np.abs(G[j] - ref).max() <= 1e-12 * np.abs(ref).max()
    lev = -(1.0 / math.pi) * (1.0 / (om[:, None] + 1j * eps - mol.eig[None, :] - s)).imag.sum(1)
    assert np.abs(dos - lev).max() <= 1e-12 * np.abs(lev).max()
    c = 0.25
    lor = lambda E: (eps / math.pi) / ((om[:, None] - E[None, :]) ** 2 + eps ** 2)
    dos2, _ = o.dyson_dos(mol, n_omega, -wmax, wmax, eps, Vxc=c * np.eye(mol.n_orb))
    assert np.abs(dos2 - lor(mol.eig - c).sum(1)).max() < 1e-10 * dos2.max()


@pytest.mark.parametrize("which", ["config0", "chain3", "narrow_mesh"])
def test_chi0_apply_equals_histogram_route(which):
    """chi0 applied to vectors through the pair-vertex closed form summed in
    orbital space equals chi0 from the integer histogram times the vectors,
    up to the histogram's 2^-s quantisation (and with the same pairs dropped
    on a mesh narrower than the spectrum)."""
    mol = gs.make_config(0) if which != "chain3" else gs.chain_molecule(3, 5)
    g = gs.Grid(64, -1.0, 1.0, 0.05) if which == "narrow_mesh" else gs.config_grid(0)
    d = g.domega
    P = o.pair_vectors(mol)
    m, fr = o.pair_bins(mol.eig, mol.n_occ, d)
    nhb = o.hist_bins(mol.eig, g.n_omega, d)
    s = o.frac_bits(P, mol.n_pairs)
    H = o.histogram(P, m, fr, s, nhb)
    js = [g.n_omega // 2, g.n_omega // 2 + 5, g.n_omega - 1, 3]
    chi = o.unpack_upper(o.chi0_from_hist(H, s, g.n_omega, g.omega_min, g.omega_max, g.eps, js=js), mol.n_prod)
    rng = np.random.default_rng(9)
    y = rng.standard_normal((mol.n_prod, 3)) + 1j * rng.standard_normal((mol.n_prod, 3))
    om = g.omegas()
    for i, j in enumerate(js):
        got = o.chi0_apply(mol, y, om[j], g.eps, d, nhb)
        ref = chi[i] @ y
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
