"""Parity at the full size of the 2000-product workload (the 40-atom chain
truncated to 2000 products, 57600 pairs, 1024-point mesh), in the launch
configuration the benchmark times: every precision form of the solve on all
mesh points with the default streams, on both routes to A = 1 - v chi0 (from
chi0, and from v a0 at the FFT).

The oracle builds its own chi0 of the whole molecule: the exact int64
histogram of every entry mu <= nu (its plain C code on the host cores), the
direct Cauchy sums at nine sampled frequencies (the lone point omega_min,
omega = 0, three inside the pair band, two above it, two negative ones), and
W there by LAPACK.  The GPU's histogram must equal it bit for bit, chi0 and
A = 1 - v chi0 entry by entry within 1e-12, W entry by entry within 1e-10 in
FP64 and 1e-6 for the refined forms.  The two-window chi0 and the time-route
a0 of the same molecule are checked on sampled entries."""
import sys

import numpy as np
import pytest

import gw_synth as gs
import oracle as o
from _oracle_full import OracleFull, compare

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
    orc = OracleFull(mol, gs.config_grid(1))
    n = mol.n_prod
    rng = np.random.default_rng(2065)
    a = rng.integers(0, n, 256)
    b = rng.integers(0, n, 256)
    special = np.array([[0, 0], [0, n - 1], [n - 1, n - 1], [63, 64], [64, 127], [127, 128], [1000, 1000],
                        [1023, 1024], [1919, 1984]])
    mu = np.concatenate([np.minimum(a, b), special[:, 0]])
    nu = np.concatenate([np.maximum(a, b), special[:, 1]])
    dm = gw.DeviceMolecule(mol)
    yield gw, ctx, torch, mol, dm, orc, (mu, nu)
    ctx.close()
    torch.cuda.empty_cache()


def _g(gw, g):
    return gw.make_grid(g.n_omega, g.omega_min, g.omega_max, g.eps, g.frac_bits)


def _entries(torch, t, mu, nu):
    """t[:, mu, nu] as numpy, gathered on the device."""
    i = torch.as_tensor(mu, device=t.device)
    j = torch.as_tensor(nu, device=t.device)
    return t[:, i, j].cpu().numpy()


FORMS = [("fp64", 0, 1e-10), ("fp32_ir", 1, 1e-6), ("bf16x_ir", 2, 1e-6)]


def _check_W(gw, torch, W, orc, N, name, prec):
    j = N // 2 + 40
    Wj = W[j].cpu().numpy()
    asym = np.abs(Wj - Wj.T).max() / np.abs(Wj).max()
    _say("%s: asymmetry %.2e" % (name, asym))
    # FP64: the upper triangle is the mirrored lower one; the refined forms
    # add unsymmetrised corrections
    assert asym == 0.0 if prec == gw.GW_FP64 else asym < 1e-9
    assert torch.equal(W[N - j], W[j].conj())
    compare(name + " W vs LAPACK on the oracle's chi0", W[orc.js].cpu().numpy(), orc.W,
            1e-10 if prec == gw.GW_FP64 else 1e-6)


def test_full_size_chi0_and_W(setup):
    gw, ctx, torch, mol, dm, orc, _ = setup
    grid = gs.config_grid(1)
    N, n = grid.n_omega, mol.n_prod
    sz = gw.query_sizes(mol.n_orb, mol.n_occ, n, np.ascontiguousarray(mol.eig), _g(gw, grid))
    H = torch.empty((sz.n_hbins, sz.n_upper), dtype=torch.int64, device="cuda")
    chi = torch.empty((N, n, n), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0(dm.struct, _g(gw, grid), chi, hist_out=H)
    torch.cuda.synchronize()
    assert rep.n_hbins == orc.nhb and rep.frac_bits_used == orc.s and rep.n_dropped_pairs == orc.dropped
    Ho = torch.from_numpy(orc.H).to("cuda")
    assert torch.equal(H, Ho), "int64 histogram differs from the oracle's"
    _say("histogram: all %d x %d entries bit-exact" % tuple(orc.H.shape))
    del H, Ho
    got = chi[orc.js].cpu().numpy()
    assert all(np.array_equal(c, c.T) for c in got)
    compare("chi0 vs the oracle's direct sums", got, orc.chi, 1e-12)
    del got
    W = torch.empty_like(chi)
    for name, prec, _ in FORMS:
        W.fill_(float("nan"))
        r = ctx.solve_W(dm.v, n, chi, N, W, prec=prec, tol=1e-7)
        torch.cuda.synchronize()
        _say("chi0 route %s: refinement steps %d, fallbacks %d" % (name, r.max_iter, r.n_fallback))
        assert r.n_solved == N // 2 + 1 and r.n_fallback == 0
        _check_W(gw, torch, W, orc, N, "chi0 route " + name, prec)
    del chi, W
    torch.cuda.empty_cache()


def test_full_size_A_route(setup):
    """The headline form: A = 1 - v chi0 formed from v a0 (gw_build_A) and W
    from A (gw_solve_W_A), every precision, in the benchmark's launch
    configuration.  The mixed forms leave A unchanged; FP64 (last) factorises
    it in place."""
    gw, ctx, torch, mol, dm, orc, _ = setup
    torch.cuda.empty_cache()
    grid = gs.config_grid(1)
    N, n = grid.n_omega, mol.n_prod
    A = torch.empty((N, n, n), dtype=torch.complex128, device="cuda")
    rep = ctx.build_A(dm.struct, dm.v, _g(gw, grid), A)
    torch.cuda.synchronize()
    assert rep.frac_bits_used == orc.s
    Aref = np.array([np.eye(n) - mol.v @ c for c in orc.chi])
    compare("A vs 1 - v chi0 of the oracle", A[orc.js].cpu().numpy(), Aref, 1e-12)
    del Aref
    W = torch.empty_like(A)
    for name, prec, _ in FORMS[1:] + FORMS[:1]:
        W.fill_(float("nan"))
        r = ctx.solve_W_A(dm.v, n, A, N, W, prec=prec, tol=1e-7)
        torch.cuda.synchronize()
        _say("A route %s: refinement steps %d, fallbacks %d" % (name, r.max_iter, r.n_fallback))
        assert r.n_solved == N // 2 + 1 and r.n_fallback == 0
        if prec != gw.GW_FP64:
            assert r.max_iter <= 2, "the refined form needed %d steps" % r.max_iter
        _check_W(gw, torch, W, orc, N, "A route " + name, prec)
    del A, W
    torch.cuda.empty_cache()


def test_full_size_two_windows(setup):
    gw, ctx, torch, mol, dm, orc, (mu, nu) = setup
    P, s = orc.P, orc.s
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
    gw, ctx, torch, mol, dm, orc, (mu, nu) = setup
    P = orc.P
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
