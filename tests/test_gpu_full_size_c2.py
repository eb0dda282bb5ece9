"""Parity at the full size of the compressed workloads, in the benchmark's
launch configuration: the 120-atom cluster (7200 products, 518400 pairs,
k = 1500, 2048 points; the compression basis, chi-hat from the projected pair
vectors and the compressed solve, FP64 and split-BF16 with FP64 refinement),
and one served request on a 150-atom cluster (k = 1500, 1024 points, the
refined split-BF16 form, through gw_submit / gw_poll).

The oracle cannot form chi0 (7200^2 entries x 518400 pairs), so it checks:
the basis is orthonormal and holds the range of v (v Q = Q S, S = Q^T v Q;
the rank of v is far below k, so the compressed W is the full W); and the
forward error of W = Q X Q^T on sampled columns at the nine sampled
frequencies: the oracle's residual r = v e_c - (1 - v chi0) w with chi0
applied by its pair-vertex route, then the error A^-1 r = r + W chi0 r
(exact with the true W; here the computed one, which changes it only at
second order).  Bar 1e-6 for every form: the pair-vertex route is unquantised,
so it also carries the 2^-s fixed-point difference of the histogram."""
import sys
import time

import numpy as np
import pytest

import gw_synth as gs
import oracle as o
from _oracle_full import forward_errors, sampled_js

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
    js = sampled_js(grid)
    for form, prec in (("fp64", gw.GW_FP64), ("bf16x_ir", gw.GW_BF16X_IR)):
        r = ctx.solve_W(S, K, chat, N, X, prec=prec, tol=1e-7)
        torch.cuda.synchronize()
        assert r.n_fallback == 0
        Xs = {j: X[j].cpu().numpy() for j in js}
        fwd, res = forward_errors(mol, grid, js, cols, lambda j, x: Qh @ (Xs[j] @ (Qh.T @ x)))
        _say("C2 %s: forward error %.2e, residual %.2e" % (form, fwd, res))
        assert fwd < 1e-6


def test_served_compressed_request_c4_size():
    """One request of the serving workload's size range (150 atoms, 3D
    cluster, k = 1500, 1024 points) in the refined split-BF16 form, through
    gw_submit / gw_poll; its result X [n_omega][k][k] and basis Q [n][k] read
    back at the sampled frequencies."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import ctypes

    import paper_1101_2065_amd.gw as gw

    torch.cuda.empty_cache()
    mol = gs.serving_molecule(150, 150)
    grid = gs.config_grid(4)
    n, N = mol.n_prod, grid.n_omega
    _say("served C4-size request: n_prod", n, "k", K, "n_omega", N)
    dm = gw.DeviceMolecule(mol)
    g = gw.make_grid(N, grid.omega_min, grid.omega_max, grid.eps, grid.frac_bits)
    ctx = gw.Context(0)
    try:
        t = ctx.submit(dm.struct, dm.v, g, k_compress=K, prec=gw.GW_BF16X_IR, tol=1e-7)
        t0 = time.time()
        while True:
            got = ctx.poll(t)
            if got is not None:
                break
            assert time.time() - t0 < 400
            time.sleep(0.01)
        ptr, rep = got
        _say("served: refinement steps %d, fallbacks %d" % (rep.max_iter, rep.n_fallback))
        assert rep.n_fallback == 0
        hip = ctypes.CDLL("libamdhip64.so")
        hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        hip.hipMemcpy.restype = ctypes.c_int
        js = sampled_js(grid)
        Xs = {}
        for j in js:
            a = np.empty((K, K), dtype=np.complex128)
            assert hip.hipMemcpy(a.ctypes.data, ptr + j * K * K * 16, a.nbytes, 2) == 0
            Xs[j] = a
        Qh = np.empty((n, K), dtype=np.float64)
        assert hip.hipMemcpy(Qh.ctypes.data, ptr + N * K * K * 16, Qh.nbytes, 2) == 0
        assert np.abs(Qh.T @ Qh - np.eye(K)).max() < 1e-12
        cols = np.random.default_rng(78).integers(0, n, 2)
        fwd, res = forward_errors(mol, grid, js, cols, lambda j, x: Qh @ (Xs[j] @ (Qh.T @ x)))
        _say("served bf16x_ir: forward error %.2e, residual %.2e" % (fwd, res))
        assert fwd < 1e-6
        ctx.release(t)
    finally:
        ctx.close()
        torch.cuda.empty_cache()
