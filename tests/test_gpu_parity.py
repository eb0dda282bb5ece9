"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: the int64 histogram bit-exact; chi0 within 1e-12 relative Frobenius
(FFT vs direct sum, both FP64); W in FP64 within 1e-10 and the mixed forms
within the 1e-6 target after refinement.
"""
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


def _oracle(mol, grid):
    P = o.pair_vectors(mol)
    d = grid.domega
    m, fr = o.pair_bins(mol.eig, mol.n_occ, d)
    nhb = o.hist_bins(mol.eig, grid.n_omega, d)
    s = o.frac_bits(P, mol.n_pairs)
    H, dropped = o.histogram_c(P, m, fr, s, nhb)
    return P, m, fr, nhb, s, H, dropped


def _gpu_chi0(gw, ctx, torch, mol, grid, want_hist=True):
    dm = gw.DeviceMolecule(mol)
    n = mol.n_prod
    sz = gw.query_sizes(mol.n_orb, mol.n_occ, n, np.ascontiguousarray(mol.eig), _grid(gw, grid))
    chi = torch.empty((grid.n_omega, n, n), dtype=torch.complex128, device="cuda")
    H = torch.empty((sz.n_hbins, sz.n_upper), dtype=torch.int64, device="cuda") if want_hist else None
    rep = ctx.build_chi0(dm.struct, _grid(gw, grid), chi, hist_out=H)
    torch.cuda.synchronize()
    return dm, chi, H, rep


def _grid(gw, g):
    return gw.make_grid(g.n_omega, g.omega_min, g.omega_max, g.eps, g.frac_bits)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("case", ["tiny_chain", "chain8_ragged"])
def test_histogram_and_chi0_match_oracle(gpu, case):
    gw, ctx, torch = gpu
    if case == "tiny_chain":
        mol, grid = gs.make_config(0), gs.config_grid(0)
    else:  # 136 products: two full 64-tiles and a ragged 8-wide tail
        mol = gs.chain_molecule(8, 7, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10,
                                prod_per_bond=8, bond_cutoff=None)
        grid = gs.config_grid(0)
    _say("case", case, "n_prod", mol.n_prod, "pairs", mol.n_pairs, "n_omega", grid.n_omega)
    P, m, fr, nhb, s, H, dropped = _oracle(mol, grid)
    dm, chi, Hg, rep = _gpu_chi0(gw, ctx, torch, mol, grid)
    assert rep.n_hbins == nhb
    assert rep.frac_bits_used == s
    assert rep.n_dropped_pairs == dropped
    assert np.array_equal(Hg.cpu().numpy(), H), "int64 histogram differs from the oracle"
    ref = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps),
                         mol.n_prod)
    got = chi.cpu().numpy()
    assert _rel(got, ref) < 1e-12
    # both triangles written
    assert np.abs(got - np.transpose(got, (0, 2, 1))).max() == 0.0


def test_histogram_independent_of_launch_and_repeat(gpu):
    """Same bits on a second run (integer sums: order and launch shape cannot matter)."""
    gw, ctx, torch = gpu
    mol, grid = gs.make_config(0), gs.config_grid(0)
    _, _, H1, _ = _gpu_chi0(gw, ctx, torch, mol, grid)
    _, _, H2, _ = _gpu_chi0(gw, ctx, torch, mol, grid)
    assert torch.equal(H1, H2)


_PREC = {"fp64": 0, "fp32_ir": 1, "bf16x_ir": 2}  # gw_precision values


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32_ir", 1e-6), ("bf16x_ir", 1e-6)])
def test_W_matches_oracle_tiny(gpu, prec, tol):
    gw, ctx, torch = gpu
    mol, grid = gs.make_config(0), gs.config_grid(0)
    _say("W tiny", prec)
    P, m, fr, nhb, s, H, _ = _oracle(mol, grid)
    chi_ref = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps),
                             mol.n_prod)
    dm, chi, _, _ = _gpu_chi0(gw, ctx, torch, mol, grid, want_hist=False)
    W = torch.empty_like(chi)
    p = _PREC[prec]
    rep = ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W, prec=p, tol=1e-8)
    torch.cuda.synchronize()
    Wg = W.cpu().numpy()
    assert rep.n_solved == grid.n_omega // 2 + 1
    # the mixed forms must reach the tolerance themselves, not via the FP64 fallback
    assert rep.n_fallback == 0
    worst = 0.0
    for j in range(grid.n_omega):
        Wr = o.screened_W(mol.v, chi_ref[j])
        worst = max(worst, _rel(Wg[j], Wr))
    _say("worst rel err", worst, "report iters", rep.max_iter, "fallback", rep.n_fallback)
    assert worst < tol


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "bf16x_ir"])
def test_W_in_place_equals_out_of_place(gpu, prec):
    """W_out == chi0: the in-place solve gives bit-for-bit the out-of-place W
    (same kernels on the same inputs), for a ragged multi-panel size."""
    gw, ctx, torch = gpu
    mol = gs.chain_molecule(3, 5)
    grid = gs.config_grid(0)
    _say("in place", prec, "n_prod", mol.n_prod)
    dm, chi, _, _ = _gpu_chi0(gw, ctx, torch, mol, grid, want_hist=False)
    W = torch.empty_like(chi)
    p = _PREC[prec]
    r1 = ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W, prec=p, tol=1e-8)
    buf = chi.clone()
    r2 = ctx.solve_W(dm.v, mol.n_prod, buf, grid.n_omega, buf, prec=p, tol=1e-8)
    torch.cuda.synchronize()
    assert r1.n_fallback == r2.n_fallback == 0
    assert torch.equal(buf, W)


def test_W_two_solve_streams_equal_one(gpu, monkeypatch):
    """GW_SOLVE_STREAMS=2 (frequency batches alternating between two streams,
    batched differently) gives bit for bit the one-stream W: every frequency
    is factorised by the same arithmetic whatever batch it is in."""
    gw, ctx, torch = gpu
    mol = gs.chain_molecule(3, 5)
    grid = gs.config_grid(0)
    dm, chi, _, _ = _gpu_chi0(gw, ctx, torch, mol, grid, want_hist=False)
    W1 = torch.empty_like(chi)
    W2 = torch.full_like(chi, float("nan"))
    monkeypatch.setenv("GW_SOLVE_STREAMS", "1")
    ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W1)
    monkeypatch.setenv("GW_SOLVE_STREAMS", "2")
    rep = ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W2)
    torch.cuda.synchronize()
    _say("two streams: solved", rep.n_solved)
    assert torch.equal(W1, W2)


def test_W_is_v_without_vertex(gpu):
    """V = 0: chi0 = 0 and W = v exactly (identity LU, no rounding)."""
    gw, ctx, torch = gpu
    mol = gs.make_config(0).scaled_vertex(0.0)
    grid = gs.config_grid(0)
    dm, chi, H, rep = _gpu_chi0(gw, ctx, torch, mol, grid)
    assert not torch.any(H)
    assert not torch.any(chi)
    W = torch.empty_like(chi)
    ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W)
    torch.cuda.synchronize()
    v = torch.from_numpy(mol.v).to("cuda").to(torch.complex128)
    assert torch.equal(W, v.unsqueeze(0).expand_as(W))


def test_single_product_closed_form(gpu):
    """n_prod = 1: W = v / (1 - v chi0) at every frequency."""
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
    dm, chi, H, rep = _gpu_chi0(gw, ctx, torch, mol, grid)
    W = torch.empty_like(chi)
    ctx.solve_W(dm.v, 1, chi, grid.n_omega, W)
    c = chi.cpu().numpy()[:, 0, 0]
    ref = 0.7 / (1 - 0.7 * c)
    assert np.abs(W.cpu().numpy()[:, 0, 0] - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.slow
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32_ir", 1e-6), ("bf16x_ir", 1e-6)])
def test_W_multi_tile_medium(gpu, prec, tol):
    """16-atom chain with the 1024-point mesh of the 40-atom workload: ~900
    products (14 LU panels, ragged last panel), W checked at sampled
    frequencies (zero, inside the pair band, above it, negative)."""
    gw, ctx, torch = gpu
    mol = gs.chain_molecule(16, 11)
    grid = gs.config_grid(1)
    _say("medium chain n_prod", mol.n_prod, "pairs", mol.n_pairs, prec)
    P, m, fr, nhb, s, H, _ = _oracle(mol, grid)
    dm, chi, Hg, rep = _gpu_chi0(gw, ctx, torch, mol, grid)
    assert np.array_equal(Hg.cpu().numpy(), H)
    W = torch.empty_like(chi)
    p = _PREC[prec]
    rep = ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W, prec=p, tol=1e-8)
    _say("report iters", rep.max_iter, "fallback", rep.n_fallback)
    assert rep.n_fallback == 0
    N = grid.n_omega
    js = [N // 2, N // 2 + 20, N // 2 + 64, N // 2 + 150, N // 2 + 400, N - 1, 300, 0]
    chi_ref = o.unpack_upper(o.chi0_from_hist(H, s, N, grid.omega_min, grid.omega_max, grid.eps, js=js),
                             mol.n_prod)
    for i, j in enumerate(js):
        got_chi = chi[j].cpu().numpy()
        assert _rel(got_chi, chi_ref[i]) < 1e-12
        Wr = o.screened_W(mol.v, chi_ref[i])
        e = _rel(W[j].cpu().numpy(), Wr)
        _say("j", j, "rel", e)
        assert e < tol


def test_kernel_timing_counts_the_work(gpu):
    """gw_profile_*: the form-A product of every solved frequency is timed and
    its algorithmic flops are exactly 4 n^3 per frequency."""
    gw, ctx, torch = gpu
    mol = gs.chain_molecule(3, 5)
    grid = gs.config_grid(0)
    dm, chi, _, _ = _gpu_chi0(gw, ctx, torch, mol, grid, want_hist=False)
    W = torch.empty_like(chi)
    ctx.profile_begin()
    rep = ctx.solve_W(dm.v, mol.n_prod, chi, grid.n_omega, W)
    st = {s["name"]: s for s in ctx.profile_read()}
    ctx.profile_end()
    _say({k: (v["launches"], round(v["ms"], 3)) for k, v in st.items()})
    n = mol.n_prod
    assert st["formA"]["flops"] == 4.0 * n ** 3 * rep.n_solved
    assert all(v["ms"] > 0 and v["launches"] > 0 for v in st.values())
    assert any(k.startswith("zgemm") for k in st) and "lu_panel" in st


@pytest.mark.slow
@pytest.mark.parametrize("n", [2600, 3500, 4200])
def test_W_tall_panels(gpu, n):
    """Panels taller than 2048 rows (six and eight rows per thread, and the
    generic panel kernel above 4096), on a dense random A = 1 - v chi0 far
    from diagonal dominance, so that rows are exchanged: W at two frequencies
    against LAPACK."""
    gw, ctx, torch = gpu
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n)) / np.sqrt(n)
    v = M + M.T
    chi = np.empty((2, n, n), complex)
    for j in range(2):
        X = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
        chi[j] = X + X.T
    _say("tall panels n", n)
    dv = torch.from_numpy(v).to("cuda")
    dchi = torch.from_numpy(chi).to("cuda")
    W = torch.empty_like(dchi)
    rep = ctx.solve_W(dv, n, dchi, 2, W)
    torch.cuda.synchronize()
    assert rep.n_solved == 2
    for j in range(2):
        e = _rel(W[j].cpu().numpy(), o.screened_W(v, chi[j]))
        _say("j", j, "rel", e)
        assert e < 1e-9
