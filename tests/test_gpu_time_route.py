"""The paper's own a0 route on the GPU (Section 8.A eq. sf-of-response-time)
against the oracle: a0 on the mesh (the convolution of the two electronic
densities contracted with the vertex) and chi0 from it, plus the argument
checks.

Bar: a0 and chi0 within 1e-12 relative Frobenius of the oracle (FP64 on
both sides; the GPU goes through discrete Fourier transforms, the oracle sums
the convolution directly or, pinned equal to it, over the pair vectors)."""
import dataclasses
import sys

import numpy as np
import pytest

import gw_synth as gs
import oracle as o

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_2065_amd.gw as gw

    ctx = gw.Context(0)
    yield gw, ctx, torch
    ctx.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _g(gw, g):
    return gw.make_grid(g.n_omega, g.omega_min, g.omega_max, g.eps, g.frac_bits)


def _run(gw, ctx, torch, mol, grid):
    dm = gw.DeviceMolecule(mol)
    n = mol.n_prod
    nhb = o.level_hist_bins(mol.eig, mol.n_occ, grid.n_omega, grid.domega)
    a = torch.full((nhb, n * (n + 1) // 2), float("nan"), dtype=torch.float64, device="cuda")
    chi = torch.full((grid.n_omega, n, n), float("nan"), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0_time(dm.struct, _g(gw, grid), chi, a_out=a)
    torch.cuda.synchronize()
    assert rep.n_hbins == nhb
    return rep, a.cpu().numpy(), chi.cpu().numpy()


_CASES = {
    # 64 products, 16 orbitals (sets of 4 and 8); 256 points (L = 512 FFT)
    "tiny": (lambda: gs.make_config(0), gs.config_grid(0), "convolution"),
    # 136 products: two 64-tiles and a ragged tail
    "chain8_ragged": (lambda: gs.chain_molecule(8, 7, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10,
                                                prod_per_bond=8, bond_cutoff=None), gs.config_grid(0), "pairs"),
    # the workload's atoms: 13 orbitals per atom, 26 per bonded pair; 1024 points
    "chain3_workload_mesh": (lambda: gs.chain_molecule(3, 5), gs.config_grid(1), "pairs"),
}


@pytest.mark.parametrize("case", sorted(_CASES))
def test_time_route_matches_oracle(gpu, case):
    gw, ctx, torch = gpu
    mk, grid, form = _CASES[case]
    mol = mk()
    d = grid.domega
    _say("time route", case, "n_prod", mol.n_prod, "n_orb", mol.n_orb, "n_omega", grid.n_omega)
    rep, a, chi = _run(gw, ctx, torch, mol, grid)
    nhb = a.shape[0]
    if form == "convolution":
        rho_p, rho_m = o.spectral_densities(mol, d)
        ref = o.a0_by_convolution(mol, rho_p, rho_m, nhb)
    else:  # pinned equal to the convolution form on the CPU
        ref = o.a0_by_pairs(o.pair_vectors(mol), mol.eig, mol.n_occ, d, nhb)
    assert rep.n_dropped_pairs == 0
    e = _rel(a, ref)
    _say("a0 rel", e)
    assert e < 1e-12
    chi_ref = o.unpack_upper(o.chi0_from_spectrum(ref, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps),
                             mol.n_prod)
    e = _rel(chi, chi_ref)
    _say("chi0 rel", e)
    assert e < 1e-12
    assert np.abs(chi - np.transpose(chi, (0, 2, 1))).max() == 0.0


def test_time_route_without_a_out_and_repeat(gpu):
    """a_out is optional; a second call on the same context gives the same
    bits (workspace reuse, fixed summation order)."""
    gw, ctx, torch = gpu
    mol, grid = gs.make_config(0), gs.config_grid(0)
    dm = gw.DeviceMolecule(mol)
    n = mol.n_prod
    c1 = torch.empty((grid.n_omega, n, n), dtype=torch.complex128, device="cuda")
    c2 = torch.empty_like(c1)
    ctx.build_chi0_time(dm.struct, _g(gw, grid), c1)
    ctx.build_chi0_time(dm.struct, _g(gw, grid), c2)
    torch.cuda.synchronize()
    assert torch.equal(c1, c2)


def test_time_route_errors(gpu):
    gw, ctx, torch = gpu
    mol, grid = gs.make_config(0), gs.config_grid(0)
    n = mol.n_prod
    chi = torch.empty((grid.n_omega, n, n), dtype=torch.complex128, device="cuda")
    # energies not measured from the Fermi level
    shifted = dataclasses.replace(mol, eig=mol.eig + 2.0)
    with pytest.raises(gw.GwError) as e:
        ctx.build_chi0_time(gw.DeviceMolecule(shifted).struct, _g(gw, grid), chi)
    assert e.value.status == gw.GW_E_INVALID
    # orbital sets beyond 32
    big = gs.chain_molecule(2, 3, orb_per_atom=20, occ_per_atom=6, prod_per_atom=6, prod_per_bond=4,
                            bond_cutoff=None)
    cb = torch.empty((grid.n_omega, big.n_prod, big.n_prod), dtype=torch.complex128, device="cuda")
    with pytest.raises(gw.GwError) as e:
        ctx.build_chi0_time(gw.DeviceMolecule(big).struct, _g(gw, grid), cb)
    assert e.value.status == gw.GW_E_INVALID
    # a mesh that is not a power of two
    with pytest.raises(gw.GwError) as e:
        ctx.build_chi0_time(gw.DeviceMolecule(mol).struct, _g(gw, gs.Grid(48, -1.0, 1.0, 0.1)), chi)
    assert e.value.status == gw.GW_E_INVALID


@pytest.mark.parametrize("case", ["tiny", "chain8_ragged"])
def test_time_route_A_matches_oracle(gpu, case):
    """gw_build_A_time: the same a0, then A = 1 - v chi0 formed from v a0 and
    W = A^{-1} v, against the oracle's a0, chi0 from it, and LAPACK."""
    gw, ctx, torch = gpu
    mk, grid, form = _CASES[case]
    mol = mk()
    d = grid.domega
    dm = gw.DeviceMolecule(mol)
    n = mol.n_prod
    nhb = o.level_hist_bins(mol.eig, mol.n_occ, grid.n_omega, d)
    a = torch.full((nhb, n * (n + 1) // 2), float("nan"), dtype=torch.float64, device="cuda")
    A = torch.full((grid.n_omega, n, n), float("nan"), dtype=torch.complex128, device="cuda")
    rep = ctx.build_A_time(dm.struct, dm.v, _g(gw, grid), A, a_out=a)
    torch.cuda.synchronize()
    assert rep.n_hbins == nhb
    if form == "convolution":
        rho_p, rho_m = o.spectral_densities(mol, d)
        ref = o.a0_by_convolution(mol, rho_p, rho_m, nhb)
    else:
        ref = o.a0_by_pairs(o.pair_vectors(mol), mol.eig, mol.n_occ, d, nhb)
    assert _rel(a.cpu().numpy(), ref) < 1e-12
    chi_ref = o.unpack_upper(o.chi0_from_spectrum(ref, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps), n)
    A_ref = np.eye(n)[None] - np.matmul(mol.v[None], chi_ref)
    e = _rel(A.cpu().numpy(), A_ref)
    _say("time route A rel", e)
    assert e < 1e-12
    W = torch.empty_like(A)
    ctx.solve_W_A(dm.v, n, A, grid.n_omega, W)
    Wg = W.cpu().numpy()
    worst = max(_rel(Wg[j], o.screened_W(mol.v, chi_ref[j])) for j in range(grid.n_omega))
    _say("time route W from A, worst rel", worst)
    assert worst < 1e-10


@pytest.mark.parametrize("n_omega", [64, 2048])
def test_time_route_A_other_meshes(gpu, n_omega):
    """The Cauchy transform as a matrix product takes any mesh: A from the
    time route on 64 and 2048 points against the oracle's a0 and chi0."""
    gw, ctx, torch = gpu
    g0 = gs.config_grid(0)
    grid = gs.Grid(n_omega, g0.omega_min, g0.omega_max, g0.eps)
    mol = gs.make_config(0)
    n = mol.n_prod
    _say("time route A on", n_omega, "points")
    dm = gw.DeviceMolecule(mol)
    A = torch.full((n_omega, n, n), float("nan"), dtype=torch.complex128, device="cuda")
    ctx.build_A_time(dm.struct, dm.v, _g(gw, grid), A)
    torch.cuda.synchronize()
    nhb = o.level_hist_bins(mol.eig, mol.n_occ, n_omega, grid.domega)
    rho_p, rho_m = o.spectral_densities(mol, grid.domega)
    ref = o.a0_by_convolution(mol, rho_p, rho_m, nhb)
    chi_ref = o.unpack_upper(o.chi0_from_spectrum(ref, n_omega, grid.omega_min, grid.omega_max, grid.eps), n)
    A_ref = np.eye(n)[None] - np.matmul(mol.v[None], chi_ref)
    e = _rel(A.cpu().numpy(), A_ref)
    _say("time route A rel", e)
    assert e < 1e-12


def test_time_route_A_fft_transform_rejects_meshes_out_of_range(gpu, monkeypatch):
    """The FFT form of the transform (GW_A_TRANSFORM=fft) keeps 128..1024
    points and rejects other meshes before anything is launched.  The output
    is sized for the full mesh all the same."""
    gw, ctx, torch = gpu
    monkeypatch.setenv("GW_A_TRANSFORM", "fft")
    mol = gs.make_config(0)
    n = mol.n_prod
    g0 = gs.config_grid(0)
    dm = gw.DeviceMolecule(mol)
    for n_omega in (64, 2048):
        A = torch.empty((n_omega, n, n), dtype=torch.complex128, device="cuda")
        with pytest.raises(gw.GwError) as ei:
            ctx.build_A_time(dm.struct, dm.v, gw.make_grid(n_omega, g0.omega_min, g0.omega_max, g0.eps, -1), A)
        assert ei.value.status == gw.GW_E_INVALID
