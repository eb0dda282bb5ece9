"""Parity at the full size of the 120-atom cluster workload (7200 products,
518400 pairs, k = 1500, 2048 points), in the benchmark's launch
configuration: the compression basis, chi-hat from the projected pair
vectors and the compressed solve, FP64 and split-BF16 with FP64 refinement.

The oracle cannot form chi0 (7200^2 entries x 518400 pairs), so it checks:
the basis is orthonormal and holds the range of v (v Q = Q S, S = Q^T v Q;
the rank of v is far below k, so the compressed W is the full W); and the
decompressed W = Q X Q^T satisfies its defining equation (1 - v chi0) W = v
on sampled columns at sampled frequencies, chi0 applied to each column by
the oracle's pair-vertex route (unquantised, so the bar is the 1e-6 of the
refined forms rather than the FP64 round-off)."""
import sys

import numpy as np
import pytest

import gw_synth as gs
import oracle as o

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

K = 1500


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_full_size_compressed_c2():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_2065_amd.gw as gw

    # earlier tests' freed tensors stay in torch's cache, which the library's
    # own workspace allocations cannot use: give them back first
    torch.cuda.empty_cache()
    ctx = gw.Context(0)
    try:
        _run_c2(gw, ctx, torch)
    finally:
        ctx.close()
        torch.cuda.empty_cache()


def _run_c2(gw, ctx, torch):
    mol = gs.make_config(2)
    grid = gs.config_grid(2)
    n, N = mol.n_prod, grid.n_omega
    _say("C2 full size: n_prod", n, "pairs", mol.n_pairs, "k", K, "n_omega", N)
    dm = gw.DeviceMolecule(mol)
    g = gw.make_grid(N, grid.omega_min, grid.omega_max, grid.eps, grid.frac_bits)
    Q = torch.empty((n, K), dtype=torch.float64, device="cuda")
    S = torch.empty((K, K), dtype=torch.float64, device="cuda")
    ctx.compress_basis(dm.v, n, K, Q, S)
    chat = torch.empty((N, K, K), dtype=torch.complex128, device="cuda")
    rep = ctx.build_chi0(dm.struct, g, chat, basis=Q, k=K)
    assert rep.n_dropped_pairs == 0
    X = torch.empty_like(chat)
    torch.cuda.synchronize()
    Qh, Sh = Q.cpu().numpy(), S.cpu().numpy()

    # the basis: orthonormal, and v Q = Q S (the range of v inside span Q)
    assert np.abs(Qh.T @ Qh - np.eye(K)).max() < 1e-12
    vQ = mol.v @ Qh
    e = np.linalg.norm(vQ - Qh @ Sh) / np.linalg.norm(vQ)
    _say("basis: ||vQ - QS|| / ||vQ|| = %.2e" % e)
    assert e < 1e-9  # measured 5e-11 (four shifted subspace-iteration steps)

    rng = np.random.default_rng(77)
    cols = rng.integers(0, n, 3)
    js = [N // 2, N // 2 + 300, 700]
    om = grid.omegas()
    nhb = o.hist_bins(mol.eig, N, grid.domega)
    for form, prec in (("fp64", gw.GW_FP64), ("bf16x_ir", gw.GW_BF16X_IR)):
        r = ctx.solve_W(S, K, chat, N, X, prec=prec, tol=1e-7)
        torch.cuda.synchronize()
        assert r.n_fallback == 0
        worst = 0.0
        for j in js:
            Xj = X[j].cpu().numpy()
            for c in cols:
                w = Qh @ (Xj @ Qh[c])  # column c of W = Q X Q^T
                res = w - mol.v @ o.chi0_apply(mol, w, om[j], grid.eps, grid.domega, nhb) - mol.v[:, c]
                worst = max(worst, np.linalg.norm(res) / np.linalg.norm(mol.v[:, c]))
        _say("%s: max residual of (1 - v chi0) W = v over %d columns x %d frequencies: %.2e"
             % (form, len(cols), len(js), worst))
        assert worst < 1e-6
