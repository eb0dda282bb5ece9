"""GPU parity of the route that forms A = 1 - v chi0 from v a0 (gw_build_A)
and solves W = A^{-1} v from it (gw_solve_W_A), against the oracle's
definition: chi0 by direct summation of the exact histogram's Cauchy
transform (Section 5.A), then A = 1 - v chi0 and W = A^{-1} v (Section 2 eq.
Coulombscreening) by LAPACK.

Bars as for the chi0 route: A within 1e-12 relative Frobenius, W in FP64
within 1e-10, the mixed forms within 1e-6 after refinement."""
import sys

import numpy as np
import pytest

import gw_synth as gs
import oracle as o

pytestmark = pytest.mark.gpu

_PREC = {"fp64": 0, "fp32_ir": 1, "bf16x_ir": 2}  # gw_precision values


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


def _grid(gw, g):
    return gw.make_grid(g.n_omega, g.omega_min, g.omega_max, g.eps, g.frac_bits)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _oracle_chi(mol, grid, js=None):
    P = o.pair_vectors(mol)
    m, fr = o.pair_bins(mol.eig, mol.n_occ, grid.domega)
    nhb = o.hist_bins(mol.eig, grid.n_omega, grid.domega)
    s = o.frac_bits(P, mol.n_pairs)
    H, _ = o.histogram_c(P, m, fr, s, nhb)
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps, js=js),
                         mol.n_prod)
    return chi, nhb, s


def _gpu_A(gw, ctx, torch, mol, grid):
    dm = gw.DeviceMolecule(mol)
    n = mol.n_prod
    A = torch.empty((grid.n_omega, n, n), dtype=torch.complex128, device="cuda")
    rep = ctx.build_A(dm.struct, dm.v, _grid(gw, grid), A)
    torch.cuda.synchronize()
    return dm, A, rep


def _ragged_chain():
    # 136 products: two full 64-tiles and a ragged 8-wide tail
    return gs.chain_molecule(8, 7, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10, prod_per_bond=8,
                             bond_cutoff=None)


@pytest.mark.parametrize("transform", ["product", "fft"])
@pytest.mark.parametrize("case", ["tiny_chain", "chain8_ragged"])
def test_A_matches_oracle(gpu, case, transform, monkeypatch):
    """A at every mesh point against the oracle, with the Cauchy transform of
    v a0 as one matrix product over the solved half (the lone point j = 0 on
    its own, the other half written as the conjugate mirror) or as the FFT
    convolution (GW_A_TRANSFORM=fft)."""
    gw, ctx, torch = gpu
    if transform == "fft":
        monkeypatch.setenv("GW_A_TRANSFORM", "fft")
    else:
        monkeypatch.delenv("GW_A_TRANSFORM", raising=False)
    mol = gs.make_config(0) if case == "tiny_chain" else _ragged_chain()
    grid = gs.config_grid(0)
    _say("A route", case, transform, "n_prod", mol.n_prod, "n_omega", grid.n_omega)
    chi, nhb, s = _oracle_chi(mol, grid)
    dm, A, rep = _gpu_A(gw, ctx, torch, mol, grid)
    assert rep.n_hbins == nhb and rep.frac_bits_used == s
    ref = np.eye(mol.n_prod)[None] - np.matmul(mol.v[None], chi)
    got = A.cpu().numpy()
    e = _rel(got, ref)
    _say("A rel", e)
    assert e < 1e-12
    assert np.isfinite(got).all()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32_ir", 1e-6), ("bf16x_ir", 1e-6)])
def test_W_from_A_matches_oracle(gpu, prec, tol):
    gw, ctx, torch = gpu
    mol, grid = _ragged_chain(), gs.config_grid(0)
    _say("W from A", prec, "n_prod", mol.n_prod)
    chi, _, _ = _oracle_chi(mol, grid)
    dm, A, _ = _gpu_A(gw, ctx, torch, mol, grid)
    W = torch.empty_like(A)
    rep = ctx.solve_W_A(dm.v, mol.n_prod, A, grid.n_omega, W, prec=_PREC[prec], tol=1e-8)
    torch.cuda.synchronize()
    assert rep.n_solved == grid.n_omega // 2 + 1 and rep.n_fallback == 0
    Wg = W.cpu().numpy()
    worst = max(_rel(Wg[j], o.screened_W(mol.v, chi[j])) for j in range(grid.n_omega))
    _say("worst rel", worst, "iters", rep.max_iter)
    assert worst < tol


@pytest.mark.parametrize("prec", ["fp64", "bf16x_ir"])
def test_W_from_A_in_place_equals_out_of_place(gpu, prec):
    """W_out == A (each batch copied to the workspace first) gives bit for bit
    the out-of-place W (factorised in the caller's A)."""
    gw, ctx, torch = gpu
    mol, grid = gs.chain_molecule(3, 5), gs.config_grid(0)
    dm, A, _ = _gpu_A(gw, ctx, torch, mol, grid)
    buf = A.clone()
    W = torch.empty_like(A)
    r1 = ctx.solve_W_A(dm.v, mol.n_prod, A, grid.n_omega, W, prec=_PREC[prec], tol=1e-8)
    r2 = ctx.solve_W_A(dm.v, mol.n_prod, buf, grid.n_omega, buf, prec=_PREC[prec], tol=1e-8)
    torch.cuda.synchronize()
    assert r1.n_fallback == r2.n_fallback == 0
    assert torch.equal(buf, W)


def test_A_route_without_vertex(gpu):
    """V = 0: an empty histogram, A = 1 and W = v exactly."""
    gw, ctx, torch = gpu
    mol, grid = gs.make_config(0).scaled_vertex(0.0), gs.config_grid(0)
    dm, A, _ = _gpu_A(gw, ctx, torch, mol, grid)
    eye = torch.eye(mol.n_prod, dtype=torch.complex128, device="cuda")
    assert torch.equal(A, eye.unsqueeze(0).expand_as(A))
    W = torch.empty_like(A)
    ctx.solve_W_A(dm.v, mol.n_prod, A, grid.n_omega, W)
    torch.cuda.synchronize()
    v = torch.from_numpy(mol.v).to("cuda").to(torch.complex128)
    assert torch.equal(W, v.unsqueeze(0).expand_as(W))


def test_A_route_single_product_closed_form(gpu):
    """n_prod = 1: A = 1 - v chi0 and W = v / (1 - v chi0), chi0 from the
    oracle's direct sum."""
    gw, ctx, torch = gpu
    grid = gs.config_grid(0)
    d = grid.domega
    eig = np.array([-10 * d, 14.25 * d, 30.5 * d])
    V = np.array([[0.1, 0.9, -0.3], [0.9, -0.2, 0.4], [-0.3, 0.4, 0.05]])
    mol = gs.Molecule(
        n_orb=3, n_occ=1, eig=eig, X=np.eye(3), blk_prod=np.array([0, 1], np.int32),
        blk_orb=np.array([0, 3], np.int32), orb_idx=np.arange(3, dtype=np.int32),
        blk_val=np.array([0, 9], np.int64), vals=V.ravel(), centres=np.zeros((1, 3)),
        atoms=np.zeros((1, 3)), v=np.array([[0.7]]))
    chi, _, _ = _oracle_chi(mol, grid)
    c = chi[:, 0, 0]
    dm, A, _ = _gpu_A(gw, ctx, torch, mol, grid)
    a = A.cpu().numpy()[:, 0, 0]
    assert np.abs(a - (1 - 0.7 * c)).max() < 1e-13
    W = torch.empty_like(A)
    ctx.solve_W_A(dm.v, 1, A, grid.n_omega, W)
    ref = 0.7 / (1 - 0.7 * c)
    assert np.abs(W.cpu().numpy()[:, 0, 0] - ref).max() < 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("n_omega", [64, 2048])
def test_A_route_other_meshes(gpu, n_omega, monkeypatch):
    """The matrix-product transform takes any mesh: A at every point of the
    64- and 2048-point meshes against the oracle on the 64-product chain; the
    FFT form (periods 256 to 2048) refuses them."""
    gw, ctx, torch = gpu
    mol = gs.make_config(0)
    g0 = gs.config_grid(0)
    grid = gs.Grid(n_omega, g0.omega_min, g0.omega_max, g0.eps)
    monkeypatch.delenv("GW_A_TRANSFORM", raising=False)
    chi, nhb, s = _oracle_chi(mol, grid)
    dm, A, rep = _gpu_A(gw, ctx, torch, mol, grid)
    assert rep.n_hbins == nhb and rep.frac_bits_used == s
    ref = np.eye(mol.n_prod)[None] - np.matmul(mol.v[None], chi)
    e = _rel(A.cpu().numpy(), ref)
    _say("A route, n_omega", n_omega, "A rel", e)
    assert e < 1e-12
    monkeypatch.setenv("GW_A_TRANSFORM", "fft")
    with pytest.raises(gw.GwError) as ei:
        ctx.build_A(dm.struct, dm.v, _grid(gw, grid), A)
    assert ei.value.status == gw.GW_E_INVALID


@pytest.mark.slow
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x_ir", 1e-6)])
def test_A_route_multi_tile_medium(gpu, prec, tol):
    """16-atom chain (~900 products, ragged last panel) on the 1024-point mesh:
    A and W at sampled frequencies against the oracle, and W equal to the
    chi0 route's within rounding."""
    gw, ctx, torch = gpu
    mol, grid = gs.chain_molecule(16, 11), gs.config_grid(1)
    N = grid.n_omega
    js = [N // 2, N // 2 + 20, N // 2 + 64, N // 2 + 150, N // 2 + 400, N - 1, 300, 0]
    _say("A route medium n_prod", mol.n_prod, prec)
    chi, _, _ = _oracle_chi(mol, grid, js=js)
    dm, A, _ = _gpu_A(gw, ctx, torch, mol, grid)
    for i, j in enumerate(js):
        e = _rel(A[j].cpu().numpy(), np.eye(mol.n_prod) - mol.v @ chi[i])
        assert e < 1e-12, (j, e)
    W = torch.empty_like(A)
    rep = ctx.solve_W_A(dm.v, mol.n_prod, A, N, W, prec=_PREC[prec], tol=1e-8)
    assert rep.n_fallback == 0
    for i, j in enumerate(js):
        e = _rel(W[j].cpu().numpy(), o.screened_W(mol.v, chi[i]))
        _say("j", j, "rel", e)
        assert e < tol
    del A
    chi_g = torch.empty_like(W)
    ctx.build_chi0(dm.struct, _grid(gw, grid), chi_g)
    W2 = torch.empty_like(W)
    ctx.solve_W(dm.v, mol.n_prod, chi_g, N, W2, prec=_PREC[prec], tol=1e-8)
    torch.cuda.synchronize()
    e = float(torch.linalg.norm(W - W2) / torch.linalg.norm(W2))
    _say("A route vs chi0 route", e)
    assert e < (1e-12 if prec == "fp64" else 1e-6)


@pytest.mark.parametrize("transform", ["product", "fft"])
@pytest.mark.parametrize("n_omega", [128, 512])
def test_A_route_other_fft_lengths(gpu, n_omega, transform, monkeypatch):
    """The 128- and 512-point meshes over the same window (FFT lengths 256
    and 1024; the cases above take 512 and 2048): A and the FP64 W at every
    frequency against the oracle, on the ragged 136-product chain, with
    either form of the Cauchy transform."""
    gw, ctx, torch = gpu
    if transform == "fft":
        monkeypatch.setenv("GW_A_TRANSFORM", "fft")
    else:
        monkeypatch.delenv("GW_A_TRANSFORM", raising=False)
    mol = _ragged_chain()
    grid = gs.Grid(n_omega, -4.0, 4.0, 0.05)
    _say("A route, n_omega", n_omega, transform)
    chi, nhb, s = _oracle_chi(mol, grid)
    dm, A, rep = _gpu_A(gw, ctx, torch, mol, grid)
    assert rep.n_hbins == nhb and rep.frac_bits_used == s
    ref = np.eye(mol.n_prod)[None] - np.matmul(mol.v[None], chi)
    e = _rel(A.cpu().numpy(), ref)
    _say("A rel", e)
    assert e < 1e-12
    W = torch.empty_like(A)
    ctx.solve_W_A(dm.v, mol.n_prod, A, grid.n_omega, W)
    Wg = W.cpu().numpy()
    worst = max(_rel(Wg[j], o.screened_W(mol.v, chi[j])) for j in range(grid.n_omega))
    _say("W worst rel", worst)
    assert worst < 1e-10


def test_A_route_histogram_ranges_bit_identical(gpu, monkeypatch):
    """The A route histograms its pairs in bin ranges on a second stream
    (GW_HIST_CHUNKS ranges, default 4) and multiplies each range's bins by v
    as soon as they are final.  The int64 sums do not depend on the order or
    the grouping of the pairs, so A is the same bit for bit for one range,
    three, the default and 64 (45 ranges of two bins for the 91 bins here);
    and it matches the oracle."""
    gw, ctx, torch = gpu
    mol = _ragged_chain()
    grid = gs.config_grid(0)
    monkeypatch.delenv("GW_A_TRANSFORM", raising=False)
    got = {}
    for chunks in ("1", "3", None, "64"):
        if chunks is None:
            monkeypatch.delenv("GW_HIST_CHUNKS", raising=False)
        else:
            monkeypatch.setenv("GW_HIST_CHUNKS", chunks)
        _say("A route, histogram ranges", chunks or "default")
        _, A, rep = _gpu_A(gw, ctx, torch, mol, grid)
        got[chunks] = A.cpu().numpy()
    nhb = rep.n_hbins
    assert nhb > 64  # "64" gives ranges of two bins
    for c, a in got.items():
        assert np.array_equal(a, got["1"]), c
    chi, _, _ = _oracle_chi(mol, grid, js=[0, grid.n_omega // 2 + 5, grid.n_omega - 1])
    ref = np.eye(mol.n_prod)[None] - np.matmul(mol.v[None], chi)
    e = _rel(got[None][[0, grid.n_omega // 2 + 5, grid.n_omega - 1]], ref)
    _say("A rel vs oracle", e)
    assert e < 1e-12
