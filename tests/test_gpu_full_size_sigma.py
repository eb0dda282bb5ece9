"""The self-energy and Dyson's equation at the full size of the 2000-product
workload (520 orbitals, the 1024-point mesh, the benchmark's launch
configuration), where the oracle cannot hold W (65 GB).  Inputs are built on
the device from seeded low-rank factors (gw_synth), never from the library:

* sigma+- (Section 5.A eq. spectral_3) from W(k domega) = v + U diag(c[k]) U^T
  whose imaginary part is zero beyond bin 300, so that no convolution term
  leaves the mesh: then the zeroth moment sum_m sigma+-[m] equals
  sum_p G_p Ut_p D+- Ut_p, with Ut_p = sum_mu U[mu, p] V_mu, G_p the summed
  spectral weight of rank p and D+- the projector on the empty / occupied
  states (the identity pinned on the CPU), checked at every orbital pair;
  and every bin of sigma+- at 200 sampled pairs, from the oracle's level
  binning (rho+-[k] is a sum of level projectors split over two bins, so
  with a low-rank gamma each bin is a short sum over levels and ranks);
* Sigma (eq. Cauchy1) at sampled frequencies and orbital pairs equals the
  retarded Cauchy sum of the library's own sigma+- (a property at any size);
* G and the DOS (Section 2 eq. Dyson, the DOS definition) at sampled
  frequencies against the oracle, with a seeded low-rank Sigma_c and
  static Sigma_x, V_xc.

Bars: 1e-10 relative (FP64 throughout; the moments sum about 10^5 terms)."""
import math
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
    grid = gs.config_grid(1)
    dm = gw.DeviceMolecule(mol)
    yield gw, ctx, torch, mol, grid, dm
    ctx.close()
    torch.cuda.empty_cache()


def _g(gw, g):
    return gw.make_grid(g.n_omega, g.omega_min, g.omega_max, g.eps, g.frac_bits)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_full_size_self_energy_moments_and_cauchy(setup):
    gw, ctx, torch, mol, grid, dm = setup
    n, no, N = mol.n_prod, mol.n_orb, grid.n_omega
    U, c = gs.lowrank_w_factors(n, N)
    dev = "cuda"
    _say("full-size self-energy: n_prod", n, "n_orb", no, "n_omega", N, "rank", U.shape[1])
    # W on the mesh: the positive half from the factors, the negative half its
    # conjugate mirror, W(omega_0) = v
    W = torch.empty((N, n, n), dtype=torch.complex128, device=dev)
    Ud = torch.from_numpy(U).to(dev).to(torch.complex128)
    Ut = Ud.transpose(0, 1).contiguous()
    cd = torch.from_numpy(c).to(dev)
    v = dm.v.to(torch.complex128)
    for k0 in range(0, N // 2, 32):
        k1 = min(k0 + 32, N // 2)
        blk = torch.matmul((Ud.unsqueeze(0) * cd[k0:k1].unsqueeze(1)).contiguous(), Ut.unsqueeze(0))
        W[N // 2 + k0:N // 2 + k1] = blk + v
    W[1:N // 2] = torch.flip(W[N // 2 + 1:], [0]).conj()
    W[0] = v
    del blk
    S = torch.empty((N, no, no), dtype=torch.complex128, device=dev)
    sig = torch.empty((2, N // 2, no, no), dtype=torch.float64, device=dev)
    rep = ctx.self_energy(dm.struct, _g(gw, grid), W, S, sigma_out=sig)
    torch.cuda.synchronize()
    assert rep.n_hbins == N // 2
    del W
    torch.cuda.empty_cache()

    # zeroth moments against the factorised identity
    d = grid.domega
    gam = -(d / math.pi) * c.imag  # spectral weight per bin and rank
    gam[0] = 0.0
    Gp = gam.sum(0)
    Ut_h = np.zeros((U.shape[1], no, no))
    for b in range(mol.n_blk):
        p0, _, orbs, mats = mol.block_of(b)
        ix = np.ix_(orbs, orbs)
        for i, M in enumerate(mats):
            for p in range(U.shape[1]):
                Ut_h[p][ix] += U[p0 + i, p] * M
    moments = sig.sum(1).cpu().numpy()
    for which, X in ((0, mol.X[:, mol.n_occ:]), (1, mol.X[:, :mol.n_occ])):
        D = X @ X.T
        ref = sum(Gp[p] * Ut_h[p] @ D @ Ut_h[p] for p in range(U.shape[1]))
        e = _rel(moments[which], ref)
        _say("zeroth moment of sigma%s: rel %.2e" % ("+-"[which], e))
        assert e < 1e-10

    # every bin of sigma+- at sampled pairs: rho+-[k] is a sum of level
    # projectors split over two bins, so with Z_p = X^T Ut_p
    #   sigma^{ab}[m] = sum_{p, E} h_{p,E}[m] Z_p[E, a] Z_p[E, b],
    #   h_{p,E}[m] = (1 - phi_E) gamma_p[m - k_E] + phi_E gamma_p[m - k_E - 1]
    rng = np.random.default_rng(5)
    a = rng.integers(0, no, 200)
    bb = rng.integers(0, no, 200)
    ia, ib = torch.as_tensor(a, device=dev), torch.as_tensor(bb, device=dev)
    sp = sig[0][:, ia, ib].cpu().numpy()
    sm = sig[1][:, ia, ib].cpu().numpy()
    ref_pm = _sigma_by_levels(mol, Ut_h, gam, d, N // 2, a, bb)
    for which, got_s in ((0, sp), (1, sm)):
        e = _rel(got_s, ref_pm[which])
        _say("sigma%s at every bin, %d pairs: rel %.2e" % ("+-"[which], len(a), e))
        assert e < 1e-10

    # Sigma = the retarded Cauchy sum of sigma+- at sampled frequencies and pairs
    js = [0, 200, N // 2 - 1, N // 2, N // 2 + 77, N - 1]
    got = S[js][:, ia, ib].cpu().numpy()
    om = grid.omegas()
    m = np.arange(N // 2) * d
    worst = 0.0
    for i, j in enumerate(js):
        kp = 1.0 / (om[j] - m + 1j * grid.eps)
        km = 1.0 / (om[j] + m + 1j * grid.eps)
        ref = kp @ sp + km @ sm
        worst = max(worst, _rel(got[i], ref))
    _say("Sigma against the Cauchy sum of sigma+-: rel %.2e" % worst)
    assert worst < 1e-12
    assert np.abs(S[js].cpu().numpy() - np.transpose(S[js].cpu().numpy(), (0, 2, 1))).max() <= \
        1e-13 * np.abs(got).max()


def _sigma_by_levels(mol, Ut, gam, d, n_sbins, a, b):
    """sigma+- [n_sbins][len(a)] at pairs (a, b) for gamma^{mu nu}[k] =
    sum_p gam[k, p] U[mu, p] U[nu, p] (Ut_p = sum_mu U[mu, p] V_mu), with
    the oracle's level binning."""
    out = []
    for levels in (np.arange(mol.n_occ, mol.n_orb), np.arange(mol.n_occ)):
        k, phi = o.level_bins(mol.eig[levels], d)
        X = mol.X[:, levels]
        acc = np.zeros((n_sbins, len(a)))
        m = np.arange(n_sbins)
        for p in range(Ut.shape[0]):
            Z = X.T @ Ut[p]  # Z[E, a]
            g = np.concatenate([gam[:, p], np.zeros(2)])
            i0 = m[:, None] - k[None, :]
            h = np.where(i0 >= 0, (1.0 - phi)[None, :] * g[np.clip(i0, 0, len(g) - 1)], 0.0)
            h += np.where(i0 - 1 >= 0, phi[None, :] * g[np.clip(i0 - 1, 0, len(g) - 1)], 0.0)
            acc += h @ (Z[:, a] * Z[:, b])
        out.append(acc)
    return out


class _LowRankSigma:
    """Sigma_c(omega_j) = Y diag(s[j]) Y^T, formed on demand."""

    def __init__(self, Y, s):
        self.Y, self.s = Y, s

    def __getitem__(self, j):
        return (self.Y * self.s[j][None, :]) @ self.Y.T


def test_full_size_dyson_dos(setup):
    gw, ctx, torch, mol, grid, dm = setup
    no, N = mol.n_orb, grid.n_omega
    Y, s, Sx, Vxc = gs.lowrank_sigma_factors(no, N)
    dev = "cuda"
    Yd = torch.from_numpy(Y).to(dev).to(torch.complex128)
    Yt = Yd.transpose(0, 1).contiguous()
    sd = torch.from_numpy(s).to(dev)
    Sc = torch.empty((N, no, no), dtype=torch.complex128, device=dev)
    for j0 in range(0, N, 64):
        j1 = min(j0 + 64, N)
        Sc[j0:j1] = torch.matmul((Yd.unsqueeze(0) * sd[j0:j1].unsqueeze(1)).contiguous(), Yt.unsqueeze(0))
    dos = torch.empty((N,), dtype=torch.float64, device=dev)
    G = torch.empty((N, no, no), dtype=torch.complex128, device=dev)
    rep = ctx.dyson_dos(dm.struct, _g(gw, grid), dos, Sigma_c=Sc, Sigma_x=torch.from_numpy(Sx).to(dev),
                        Vxc=torch.from_numpy(Vxc).to(dev), G_out=G)
    torch.cuda.synchronize()
    assert rep.n_solved == N
    js = [0, 300, N // 2 - 1, N // 2, N // 2 + 45, N - 1]
    dref, Gref = o.dyson_dos(mol, N, grid.omega_min, grid.omega_max, grid.eps, Sigma_c=_LowRankSigma(Y, s),
                             Sigma_x=Sx, Vxc=Vxc, js=js)
    d = dos.cpu().numpy()
    e_dos = np.abs(d[js] - dref).max() / np.abs(dref).max()
    e_G = max(_rel(G[j].cpu().numpy(), Gref[i]) for i, j in enumerate(js))
    _say("full-size Dyson: DOS rel %.2e, G rel %.2e" % (e_dos, e_G))
    assert e_dos < 1e-10 and e_G < 1e-10
    assert np.isfinite(d).all()
