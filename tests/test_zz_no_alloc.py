"""gw_solve_W_A_noalloc against gw_solve_W_A (FP64) through the C ABI: two
calls in a row, the second on a smaller input, each equal to the allocating
entry point's W (FP64 bar 1e-10; the two run the same kernels on the same
frequencies, so they agree to the last bit in practice), the small case also
against the oracle's LAPACK W; free device memory is the same before and after
both calls; a size whose single-frequency workspace exceeds the fixed array
is rejected before anything runs."""
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


def _case(gw, ctx, torch, mol, grid):
    """A from the molecule, then the allocating and the fixed-workspace solve
    on two copies of it; every device buffer is made before the timed calls."""
    dm = gw.DeviceMolecule(mol)
    n = mol.n_prod
    A = torch.empty((grid.n_omega, n, n), dtype=torch.complex128, device="cuda")
    ctx.build_A(dm.struct, dm.v, gw.make_grid(grid.n_omega, grid.omega_min, grid.omega_max, grid.eps), A)
    A1 = A.clone()
    A2 = A.clone()
    W1 = torch.empty_like(A)
    W2 = torch.full_like(A, float("nan"))
    torch.cuda.synchronize()
    return dm, A, A1, A2, W1, W2


def test_noalloc_matches_allocating_solve_twice(gpu):
    gw, ctx, torch = gpu
    big = gs.chain_molecule(16, 3, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10, prod_per_bond=8,
                            bond_cutoff=None)
    gbig = gs.config_grid(0)  # 256 points: two frequency batches of 64 at 280 products
    small = gs.make_config(0)
    gsmall = gs.config_grid(0)
    cases = [(big, gbig), (small, gsmall)]
    bufs = [_case(gw, ctx, torch, m, g) for m, g in cases]
    # reference: the allocating FP64 solve
    for (mol, grid), (dm, A, A1, A2, W1, W2) in zip(cases, bufs):
        ctx.solve_W_A(dm.v, mol.n_prod, A1, grid.n_omega, W1, prec=gw.GW_FP64)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    # the fixed-workspace solve: the larger input first, then the smaller one
    reps = []
    for (mol, grid), (dm, A, A1, A2, W1, W2) in zip(cases, bufs):
        _say("noalloc n_prod", mol.n_prod, "n_omega", grid.n_omega)
        reps.append(ctx.solve_W_A_noalloc(dm.v, mol.n_prod, A2, grid.n_omega, W2))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, "device memory changed during the calls: %d -> %d" % (free0, free1)
    for (mol, grid), (dm, A, A1, A2, W1, W2), rep in zip(cases, bufs, reps):
        assert rep.n_solved == grid.n_omega // 2 + 1
        w1 = W1.cpu().numpy()
        w2 = W2.cpu().numpy()
        assert np.isfinite(w2).all()
        worst = max(_rel(w2[j], w1[j]) for j in range(grid.n_omega))
        _say("  n_prod", mol.n_prod, "worst rel vs allocating solve", worst,
             "bit-identical", bool(np.array_equal(w1, w2)))
        assert worst <= 1e-10
        # both leave the same LU factors in A
        assert _rel(A2.cpu().numpy(), A1.cpu().numpy()) <= 1e-12
    # the smaller case against the oracle's LAPACK W at three frequencies
    mol, grid = cases[1]
    W2 = bufs[1][5].cpu().numpy()
    P = o.pair_vectors(mol)
    m, fr = o.pair_bins(mol.eig, mol.n_occ, grid.domega)
    nhb = o.hist_bins(mol.eig, grid.n_omega, grid.domega)
    s = o.frac_bits(P, mol.n_pairs)
    H = o.histogram(P, m, fr, s, nhb)
    js = [0, grid.n_omega // 2, grid.n_omega // 2 + 9, grid.n_omega // 2 - 9]
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps, js=js),
                         mol.n_prod)
    for i, j in enumerate(js):
        e = _rel(W2[j], o.screened_W(mol.v, chi[i]))
        _say("  oracle j", j, "rel", e)
        assert e <= 1e-10


def test_noalloc_rejects_oversized_and_aliased(gpu):
    gw, ctx, torch = gpu
    t = torch.zeros((2, 8, 8), dtype=torch.complex128, device="cuda")
    v = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    # n = 30000 needs ~92 MB of workspace per frequency: rejected before any launch
    st = gw.lib.gw_solve_W_A_noalloc(ctx.h, v.data_ptr(), 0, 30000, t.data_ptr(), 2, None,
                                     torch.empty_like(t).data_ptr(), None)
    assert st == gw.GW_E_INVALID
    assert b"fixed array" in gw.lib.gw_last_error(ctx.h)
    st = gw.lib.gw_solve_W_A_noalloc(ctx.h, v.data_ptr(), 0, 8, t.data_ptr(), 2, None, t.data_ptr(), None)
    assert st == gw.GW_E_INVALID
    assert gw.lib.gw_solve_W_A_noalloc(None, None, 0, 8, None, 2, None, None, None) == gw.GW_E_INVALID
