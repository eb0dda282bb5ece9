"""Two spectral windows on the GPU (Section 5.B eq. win2-for-response) against
the oracle: the fine window's chi0 (small-window pairs on the fine mesh plus
the rest through the coarse mesh, each with its own broadening), the coarse
window's ordinary chi0, the same-mesh identity and the argument checks.

Bar: chi0 within 1e-12 relative Frobenius of the oracle's direct sums (both
FP64; the integer histograms they start from are exact)."""
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


def _auto(n, wmax):
    g = gs.Grid(n, -wmax, wmax, 0.0)
    g.eps = 1.5 * g.domega  # the paper's automatic broadening, per window
    return g


def _run(gw, ctx, torch, mol, small, large):
    dm = gw.DeviceMolecule(mol)
    n = mol.n_prod
    cs = torch.full((small.n_omega, n, n), float("nan"), dtype=torch.complex128, device="cuda")
    cl = torch.full((large.n_omega, n, n), float("nan"), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0_2w(dm.struct, _g(gw, small), _g(gw, large), cs, cl)
    torch.cuda.synchronize()
    return rep, cs.cpu().numpy(), cl.cpu().numpy()


_CASES = {
    # 64 products; L = 128 (LDS kernel) on the fine mesh, 64 on the coarse one
    "tiny": (lambda: gs.make_config(0), (64, 1.0), (32, 4.0)),
    # 136 products (two 64-tiles and a ragged tail); wave kernels on both meshes
    "chain8_ragged": (lambda: gs.chain_molecule(8, 7, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10,
                                                prod_per_bond=8, bond_cutoff=None),
                      (256, 0.5), (256, 4.0)),
}


@pytest.mark.parametrize("case", sorted(_CASES))
def test_two_window_matches_oracle(gpu, case):
    gw, ctx, torch = gpu
    mk, (ns, ws), (nl, wl) = _CASES[case]
    mol = mk()
    small, large = _auto(ns, ws), _auto(nl, wl)
    lam = o.two_window_split(small.domega, small.omega_max, large.domega)
    delta = (mol.eig[mol.n_occ:][None, :] - mol.eig[:mol.n_occ][:, None]).ravel()
    n_low = int((delta < lam).sum())
    _say("two windows", case, "n_prod", mol.n_prod, "lambda_s", lam, "pairs below", n_low, "of", mol.n_pairs)
    assert 0 < n_low < mol.n_pairs
    rep, cs, cl = _run(gw, ctx, torch, mol, small, large)
    P = o.pair_vectors(mol)
    s = o.frac_bits(P, mol.n_pairs)
    assert rep.frac_bits_used == s
    assert rep.n_hbins == o.hist_bins(mol.eig, large.n_omega, large.domega)
    # fine window: every frequency
    ref = o.unpack_upper(o.chi0_two_window(P, mol.eig, mol.n_occ, s,
                                           (small.n_omega, small.omega_min, small.omega_max, small.eps),
                                           (large.n_omega, large.omega_min, large.omega_max, large.eps)),
                         mol.n_prod)
    e = _rel(cs, ref)
    _say("fine window rel", e)
    assert e < 1e-12
    assert np.abs(cs - np.transpose(cs, (0, 2, 1))).max() == 0.0
    # coarse window: the one-window chi0 of every pair
    m, fr = o.pair_bins(mol.eig, mol.n_occ, large.domega)
    H = o.histogram(P, m, fr, s, o.hist_bins(mol.eig, large.n_omega, large.domega))
    refl = o.unpack_upper(o.chi0_from_hist(H, s, large.n_omega, large.omega_min, large.omega_max, large.eps),
                          mol.n_prod)
    e = _rel(cl, refl)
    _say("coarse window rel", e)
    assert e < 1e-12


def test_two_window_same_mesh_is_one_window(gpu):
    """Equal meshes and broadenings: the windows partition the pairs, so the
    fine window's chi0 is the ordinary one (the coarse output)."""
    gw, ctx, torch = gpu
    mol = gs.chain_molecule(8, 7, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10, prod_per_bond=8,
                            bond_cutoff=None)
    g = _auto(256, 4.0)
    rep, cs, cl = _run(gw, ctx, torch, mol, g, g)
    e = _rel(cs, cl)
    _say("same mesh rel", e)
    assert e < 1e-12


def test_two_window_repeat_and_after_one_window(gpu):
    """A second call, after an ordinary build on another mesh (shared
    workspace and cached kernel spectrum), gives the same bits."""
    gw, ctx, torch = gpu
    mol = gs.make_config(0)
    small, large = _auto(64, 1.0), _auto(32, 4.0)
    _, cs1, cl1 = _run(gw, ctx, torch, mol, small, large)
    dm = gw.DeviceMolecule(mol)
    g1 = gs.config_grid(0)
    c = torch.empty((g1.n_omega, mol.n_prod, mol.n_prod), dtype=torch.complex128, device="cuda")
    ctx.build_chi0(dm.struct, _g(gw, g1), c)
    _, cs2, cl2 = _run(gw, ctx, torch, mol, small, large)
    assert np.array_equal(cs1, cs2)
    assert np.array_equal(cl1, cl2)


def test_two_window_errors(gpu):
    gw, ctx, torch = gpu
    mol = gs.make_config(0)
    dm = gw.DeviceMolecule(mol)
    n = mol.n_prod
    c1 = torch.empty((64, n, n), dtype=torch.complex128, device="cuda")
    c2 = torch.empty((64, n, n), dtype=torch.complex128, device="cuda")
    fine, coarse = _auto(64, 1.0), _auto(64, 4.0)
    bad = [
        (_g(gw, coarse), _g(gw, fine), c1, c2),       # small window coarser than the large one
        (_g(gw, _auto(64, 8.0)), _g(gw, _auto(32, 4.0)), c1, c2),  # small window reaching beyond
        (_g(gw, fine), _g(gw, coarse), c1, c1),       # aliased outputs
        (_g(gw, gs.Grid(48, -1.0, 1.0, 0.1)), _g(gw, coarse), c1, c2),  # not a power of two
    ]
    for gsml, glrg, a, b in bad:
        with pytest.raises(gw.GwError) as e:
            ctx.build_chi0_2w(dm.struct, gsml, glrg, a, b)
        assert e.value.status == gw.GW_E_INVALID


def test_two_window_in_a_basis(gpu):
    """Both windows built from pair vectors projected onto a basis (the
    compressed path): the k x k fine-window chi0 equals the oracle's two-window
    chi0 of the projected pair vectors."""
    gw, ctx, torch = gpu
    mol = gs.chain_molecule(8, 7, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10, prod_per_bond=8,
                            bond_cutoff=None)
    k = 40
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((mol.n_prod, k)))
    small, large = _auto(256, 0.5), _auto(256, 4.0)
    dm = gw.DeviceMolecule(mol)
    Qd = torch.from_numpy(np.ascontiguousarray(Q)).to("cuda")
    cs = torch.full((small.n_omega, k, k), float("nan"), dtype=torch.complex128, device="cuda")
    cl = torch.full((large.n_omega, k, k), float("nan"), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0_2w(dm.struct, _g(gw, small), _g(gw, large), cs, cl, basis=Qd, k=k)
    torch.cuda.synchronize()
    Ph = o.project_pairs(o.pair_vectors(mol), Q)
    s = o.frac_bits(Ph, mol.n_pairs)
    assert rep.frac_bits_used == s
    ref = o.unpack_upper(o.chi0_two_window(Ph, mol.eig, mol.n_occ, s,
                                           (small.n_omega, small.omega_min, small.omega_max, small.eps),
                                           (large.n_omega, large.omega_min, large.omega_max, large.eps)), k)
    e = _rel(cs.cpu().numpy(), ref)
    _say("two windows in a basis of", k, "rel", e)
    assert e < 1e-10
