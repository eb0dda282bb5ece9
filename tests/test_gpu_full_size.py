"""Parity at the full size of the 2000-product workload (the 40-atom chain
truncated to 2000 products, 57600 pairs, 1024-point mesh), in the launch
configuration the benchmark times: every precision form of the solve on all
mesh points with the default streams, on both routes to A = 1 - v chi0 (from
chi0, and from v a0 at the FFT).

The oracle cannot hold the whole 2000 x 2000 x 192-bin histogram in seconds,
so it checks what it can compute one by one: sampled histogram entries bit for
bit (its C histogram), chi0 at those entries and several frequencies (its
direct sums), and W through its defining equation (1 - v chi0) W = v on
sampled columns at sampled frequencies, a property that holds at any size,
plus the symmetry of W and the conjugate mirror.  The two-window chi0 of the
same molecule (the benchmark's two-window meshes) is checked the same way."""
import sys

import numpy as np
import pytest

import gw_synth as gs
import oracle as o

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_PROD = 2000


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_2065_amd.gw as gw

    torch.cuda.empty_cache()  # cached blocks of earlier tests: back to the device
    ctx = gw.Context(0)
    mol = gs.truncate_products(gs.make_config(1), N_PROD)
    _say("full size: n_prod", mol.n_prod, "pairs", mol.n_pairs)
    P = o.pair_vectors(mol)
    s = o.frac_bits(P, mol.n_pairs)
    n = mol.n_prod
    rng = np.random.default_rng(2065)
    a = rng.integers(0, n, 256)
    b = rng.integers(0, n, 256)
    special = np.array([[0, 0], [0, n - 1], [n - 1, n - 1], [63, 64], [64, 127], [127, 128], [1000, 1000],
                        [1023, 1024], [1919, 1984]])
    mu = np.concatenate([np.minimum(a, b), special[:, 0]])
    nu = np.concatenate([np.maximum(a, b), special[:, 1]])
    dm = gw.DeviceMolecule(mol)
    yield gw, ctx, torch, mol, dm, P, s, (mu, nu)
    ctx.close()
    torch.cuda.empty_cache()


def _g(gw, g):
    return gw.make_grid(g.n_omega, g.omega_min, g.omega_max, g.eps, g.frac_bits)


def _entries(torch, t, mu, nu):
    """t[:, mu, nu] as numpy, gathered on the device."""
    i = torch.as_tensor(mu, device=t.device)
    j = torch.as_tensor(nu, device=t.device)
    return t[:, i, j].cpu().numpy()


def test_full_size_chi0_and_W(setup):
    gw, ctx, torch, mol, dm, P, s, (mu, nu) = setup
    grid = gs.config_grid(1)
    N, n = grid.n_omega, mol.n_prod
    sz = gw.query_sizes(mol.n_orb, mol.n_occ, n, np.ascontiguousarray(mol.eig), _g(gw, grid))
    H = torch.empty((sz.n_hbins, sz.n_upper), dtype=torch.int64, device="cuda")
    chi = torch.empty((N, n, n), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0(dm.struct, _g(gw, grid), chi, hist_out=H)
    torch.cuda.synchronize()
    m, fr = o.pair_bins(mol.eig, mol.n_occ, grid.domega)
    nhb = o.hist_bins(mol.eig, N, grid.domega)
    assert rep.n_hbins == nhb and rep.frac_bits_used == s
    Href, dropped = o.histogram_c(P, m, fr, s, nhb, mu, nu)
    assert rep.n_dropped_pairs == dropped
    t = mu * n - mu * (mu - 1) // 2 + (nu - mu)
    Hg = H[:, torch.as_tensor(t, device="cuda")].cpu().numpy()
    assert np.array_equal(Hg, Href), "sampled int64 histogram entries differ from the oracle"
    _say("histogram: %d sampled entries bit-exact" % len(mu))
    del H
    js = [0, 100, N // 2, N // 2 + 40, N // 2 + 300, N - 1]
    ref = o.chi0_from_hist(Href, s, N, grid.omega_min, grid.omega_max, grid.eps, js=js)
    got = _entries(torch, chi[js], mu, nu)
    got_t = _entries(torch, chi[js], nu, mu)
    assert np.array_equal(got, got_t)
    for i, j in enumerate(js):
        e = np.abs(got[i] - ref[i]).max() / np.abs(ref[i]).max()
        _say("chi0 j", j, "max rel", e)
        assert e < 1e-12
    # W: the benchmark's forms, the defining equation on sampled columns
    W = torch.empty_like(chi)
    cols = np.array([0, 1, 63, 64, 777, 1500, n - 1])
    wj = [N // 2, N // 2 + 40, N // 2 + 300, N - 1]
    chis = {j: chi[j].cpu().numpy() for j in wj}
    for prec, bound in [(gw.GW_FP64, 1e-10), (gw.GW_FP32_IR, 1e-6), (gw.GW_BF16X_IR, 1e-6)]:
        W.fill_(float("nan"))
        r = ctx.solve_W(dm.v, n, chi, N, W, prec=prec, tol=1e-7)
        torch.cuda.synchronize()
        assert r.n_solved == N // 2 + 1
        assert r.n_fallback == 0
        for j in wj:
            Wc = W[j][:, torch.as_tensor(cols, device="cuda")].cpu().numpy()
            lhs = Wc - mol.v @ (chis[j] @ Wc)
            e = np.linalg.norm(lhs - mol.v[:, cols]) / np.linalg.norm(mol.v[:, cols])
            _say("prec", prec, "j", j, "residual of (1 - v chi0) W = v on sampled columns", e)
            assert e < bound
        # W symmetric (FP64: the upper triangle is the mirrored lower one; the
        # refined forms add unsymmetrised corrections); mesh points below N/2
        # are the conjugate mirror
        Wr = W[N // 2 + 40][torch.as_tensor(cols, device="cuda")].cpu().numpy()
        Wcol = W[N // 2 + 40][:, torch.as_tensor(cols, device="cuda")].cpu().numpy()
        asym = np.abs(Wr - Wcol.T).max() / np.abs(Wr).max()
        _say("prec", prec, "asymmetry", asym)
        assert asym == 0.0 if prec == gw.GW_FP64 else asym < 1e-9
        assert torch.equal(W[N - (N // 2 + 40)], W[N // 2 + 40].conj())


def test_full_size_A_route(setup):
    """The headline form: A = 1 - v chi0 formed from v a0 (gw_build_A) and W
    from A (gw_solve_W_A) in FP64, in the benchmark's launch configuration.
    A on sampled rows against 1 - v chi0 of the chi0 route (whose sampled
    entries the test above pins to the oracle), W through the defining
    equation on sampled columns, its symmetry and the conjugate mirror."""
    gw, ctx, torch, mol, dm, P, s, _ = setup
    torch.cuda.empty_cache()
    grid = gs.config_grid(1)
    N, n = grid.n_omega, mol.n_prod
    wj = [N // 2, N // 2 + 40, N // 2 + 300, N - 1]
    buf = torch.empty((N, n, n), dtype=torch.complex128, device="cuda")
    ctx.build_chi0(dm.struct, _g(gw, grid), buf)
    chis = {j: buf[j].cpu().numpy() for j in wj}
    rep = ctx.build_A(dm.struct, dm.v, _g(gw, grid), buf)
    torch.cuda.synchronize()
    assert rep.frac_bits_used == s
    idx = np.array([0, 1, 63, 64, 777, 1500, n - 1])
    it = torch.as_tensor(idx, device="cuda")
    for j in wj:
        Ar = buf[j][it].cpu().numpy()
        ref = np.eye(n)[idx] - mol.v[idx] @ chis[j]
        e = np.linalg.norm(Ar - ref) / np.linalg.norm(ref)
        _say("A j", j, "rel on sampled rows", e)
        assert e < 1e-12
    W = torch.full_like(buf, float("nan"))
    r = ctx.solve_W_A(dm.v, n, buf, N, W, prec=gw.GW_FP64)
    torch.cuda.synchronize()
    assert r.n_solved == N // 2 + 1 and r.n_fallback == 0
    del buf
    for j in wj:
        Wc = W[j][:, it].cpu().numpy()
        lhs = Wc - mol.v @ (chis[j] @ Wc)
        e = np.linalg.norm(lhs - mol.v[:, idx]) / np.linalg.norm(mol.v[:, idx])
        _say("A route j", j, "residual of (1 - v chi0) W = v on sampled columns", e)
        assert e < 1e-10
    Wr = W[N // 2 + 40][it].cpu().numpy()
    Wcol = W[N // 2 + 40][:, it].cpu().numpy()
    assert np.abs(Wr - Wcol.T).max() == 0.0
    assert torch.equal(W[N - (N // 2 + 40)], W[N // 2 + 40].conj())
    del W
    torch.cuda.empty_cache()


def test_full_size_two_windows(setup):
    gw, ctx, torch, mol, dm, P, s, (mu, nu) = setup
    small, large = gs.two_window_grids()
    n = mol.n_prod
    cs = torch.empty((small.n_omega, n, n), dtype=torch.complex128, device="cuda")
    cl = torch.empty((large.n_omega, n, n), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0_2w(dm.struct, _g(gw, small), _g(gw, large), cs, cl)
    torch.cuda.synchronize()
    assert rep.frac_bits_used == s
    sm = (small.n_omega, small.omega_min, small.omega_max, small.eps)
    lg = (large.n_omega, large.omega_min, large.omega_max, large.eps)
    ref = o.chi0_two_window(P, mol.eig, mol.n_occ, s, sm, lg, entries=(mu, nu))
    got = _entries(torch, cs, mu, nu)
    assert np.array_equal(got, _entries(torch, cs, nu, mu))
    e = np.abs(got - ref).max() / np.abs(ref).max()
    _say("two windows, fine mesh: max rel over %d entries x %d frequencies" % (len(mu), small.n_omega), e)
    assert e < 1e-12
    m, fr = o.pair_bins(mol.eig, mol.n_occ, large.domega)
    Hl, _ = o.histogram_c(P, m, fr, s, o.hist_bins(mol.eig, large.n_omega, large.domega), mu, nu)
    refl = o.chi0_from_hist(Hl, s, large.n_omega, large.omega_min, large.omega_max, large.eps)
    e = np.abs(_entries(torch, cl, mu, nu) - refl).max() / np.abs(refl).max()
    _say("two windows, coarse mesh: max rel", e)
    assert e < 1e-12
    # W on both meshes in place, as the benchmark's two-window step does
    j = small.n_omega // 2 + 20
    c0 = cs[j].cpu().numpy()
    ctx.solve_W(dm.v, n, cs, small.n_omega, cs)
    torch.cuda.synchronize()
    cols = np.array([0, 64, 1999])
    Wc = cs[j][:, torch.as_tensor(cols, device="cuda")].cpu().numpy()
    e = np.linalg.norm(Wc - mol.v @ (c0 @ Wc) - mol.v[:, cols]) / np.linalg.norm(mol.v[:, cols])
    _say("two windows: residual of W on the fine mesh", e)
    assert e < 1e-10


def test_full_size_time_route(setup):
    """The paper's own a0 route at the full size on the 1024-point mesh: a0
    and chi0 at the sampled entries against the pair form of the oracle
    (pinned equal to its convolution form)."""
    gw, ctx, torch, mol, dm, P, s, (mu, nu) = setup
    grid = gs.config_grid(1)
    N, n = grid.n_omega, mol.n_prod
    nhb = o.level_hist_bins(mol.eig, mol.n_occ, N, grid.domega)
    a = torch.empty((nhb, n * (n + 1) // 2), dtype=torch.float64, device="cuda")
    chi = torch.empty((N, n, n), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0_time(dm.struct, _g(gw, grid), chi, a_out=a)
    torch.cuda.synchronize()
    assert rep.n_hbins == nhb and rep.n_dropped_pairs == 0
    ref = o.a0_by_pairs(P, mol.eig, mol.n_occ, grid.domega, nhb, entries=(mu, nu))
    t = mu * n - mu * (mu - 1) // 2 + (nu - mu)
    got = a[:, torch.as_tensor(t, device="cuda")].cpu().numpy()
    e = np.abs(got - ref).max() / np.abs(ref).max()
    _say("time route a0: max rel over %d sampled entries" % len(mu), e)
    assert e < 1e-12
    del a
    js = [0, 100, N // 2, N // 2 + 40, N // 2 + 300, N - 1]
    cref = o.chi0_from_spectrum(ref, N, grid.omega_min, grid.omega_max, grid.eps, js=js)
    cg = _entries(torch, chi[js], mu, nu)
    e = np.abs(cg - cref).max() / np.abs(cref).max()
    _say("time route chi0: max rel", e)
    assert e < 1e-12
