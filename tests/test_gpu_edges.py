"""Edge cases of the chi0 build and the solve on the GPU, against the oracle:
pairs beyond the mesh (dropped and counted), every pair dropped (chi0 = 0,
W = v exactly), poles exactly on mesh points (no split), and every mesh size
the library takes (each FFT length, both FFT kernels)."""
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


def _build(gw, ctx, torch, mol, grid):
    dm = gw.DeviceMolecule(mol)
    g = gw.make_grid(grid.n_omega, grid.omega_min, grid.omega_max, grid.eps, grid.frac_bits)
    sz = gw.query_sizes(mol.n_orb, mol.n_occ, mol.n_prod, np.ascontiguousarray(mol.eig), g)
    H = torch.empty((sz.n_hbins, sz.n_upper), dtype=torch.int64, device="cuda")
    chi = torch.full((grid.n_omega, mol.n_prod, mol.n_prod), float("nan"), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0(dm.struct, g, chi, hist_out=H)
    torch.cuda.synchronize()
    return dm, rep, H.cpu().numpy(), chi


def _oracle(mol, grid):
    P = o.pair_vectors(mol)
    d = grid.domega
    m, fr = o.pair_bins(mol.eig, mol.n_occ, d)
    nhb = o.hist_bins(mol.eig, grid.n_omega, d)
    s = o.frac_bits(P, mol.n_pairs)
    H, dropped = o.histogram_c(P, m, fr, s, nhb)
    return H, s, dropped


def test_pairs_beyond_the_mesh_are_dropped(gpu):
    gw, ctx, torch = gpu
    mol = gs.make_config(0)
    grid = gs.Grid(64, -1.0, 1.0, 0.05)
    H, s, dropped = _oracle(mol, grid)
    assert 0 < dropped < mol.n_pairs
    dm, rep, Hg, chi = _build(gw, ctx, torch, mol, grid)
    _say("narrow mesh: dropped", rep.n_dropped_pairs, "of", mol.n_pairs)
    assert rep.n_dropped_pairs == dropped
    assert np.array_equal(Hg, H)
    ref = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps),
                         mol.n_prod)
    assert _rel(chi.cpu().numpy(), ref) < 1e-12
    W = torch.empty_like(chi)
    ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W)
    torch.cuda.synchronize()
    for j in (0, grid.n_omega // 2, grid.n_omega // 2 + 7, grid.n_omega - 1):
        assert _rel(W[j].cpu().numpy(), o.screened_W(mol.v, ref[j])) < 1e-10


def test_every_pair_dropped(gpu):
    """A window narrower than the gap: nothing lands on the mesh, so chi0 is
    zero and W = v exactly."""
    gw, ctx, torch = gpu
    mol = gs.make_config(0)
    grid = gs.Grid(16, -0.125, 0.125, 0.02)
    H, s, dropped = _oracle(mol, grid)
    assert dropped == mol.n_pairs and not H.any()
    dm, rep, Hg, chi = _build(gw, ctx, torch, mol, grid)
    assert rep.n_dropped_pairs == mol.n_pairs
    assert not Hg.any()
    assert not torch.any(chi)
    W = torch.empty_like(chi)
    ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W)
    torch.cuda.synchronize()
    v = torch.from_numpy(mol.v).to("cuda").to(torch.complex128)
    assert torch.equal(W, v.unsqueeze(0).expand_as(W))


def test_levels_on_mesh_points(gpu):
    """Every level on a mesh point: no pole is split (fraction 0), each pair
    deposits into one bin; the histogram stays bit-exact."""
    gw, ctx, torch = gpu
    grid = gs.config_grid(0)
    mol = gs.make_config(0)
    d = grid.domega
    mol = dataclasses.replace(mol, eig=np.round(mol.eig / d) * d)
    m, fr = o.pair_bins(mol.eig, mol.n_occ, d)
    assert not fr.any()
    H, s, dropped = _oracle(mol, grid)
    dm, rep, Hg, chi = _build(gw, ctx, torch, mol, grid)
    assert rep.n_dropped_pairs == dropped
    assert np.array_equal(Hg, H)
    ref = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps),
                         mol.n_prod)
    assert _rel(chi.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("n_omega", [16, 32, 64, 128, 256, 512, 1024, 2048])
def test_every_mesh_size(gpu, n_omega):
    """Every mesh the library takes (FFT lengths 32 .. 4096: the LDS kernel
    for 32, 64, 128 and 4096, the wave kernel for 256 .. 2048), the window
    fixed at |omega| < 4 Ha so the spacing 8/N is a power of two."""
    gw, ctx, torch = gpu
    mol = gs.make_config(0)
    grid = gs.Grid(n_omega, -4.0, 4.0, 0.0)
    grid.eps = 1.5 * grid.domega
    H, s, dropped = _oracle(mol, grid)
    dm, rep, Hg, chi = _build(gw, ctx, torch, mol, grid)
    assert np.array_equal(Hg, H)
    ref = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps),
                         mol.n_prod)
    got = chi.cpu().numpy()
    e = _rel(got, ref)
    _say("n_omega", n_omega, "chi0 rel", e)
    assert e < 1e-12
    assert np.abs(got - np.transpose(got, (0, 2, 1))).max() == 0.0
