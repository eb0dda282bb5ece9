"""Serving (continuous batching): every result is the same whether the request
ran alone or together with others, results stay on the device until released,
and the error paths report the documented status codes."""
import ctypes
import sys
import time

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

    yield gw, torch


def _wait(ctx, ticket, timeout=300.0):
    t0 = time.time()
    while True:
        r = ctx.poll(ticket)
        if r is not None:
            return r
        if time.time() - t0 > timeout:
            raise TimeoutError("request %d not done after %.0fs" % (ticket, timeout))
        time.sleep(0.002)


_HIP = None


def _fetch(gw, torch, ptr, n_omega, kk):
    """Copy a library-owned device result (complex128 [n_omega][kk][kk]) to the host."""
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _HIP.hipMemcpy.restype = ctypes.c_int
    out = np.empty((n_omega, kk, kk), dtype=np.complex128)
    rc = _HIP.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # hipMemcpyDeviceToHost
    assert rc == 0
    return out


def _workload():
    grid = gs.config_grid(0)
    mols = [
        (gs.make_config(0), 0),
        (gs.chain_molecule(8, 7, orb_per_atom=4, occ_per_atom=2, prod_per_atom=10, prod_per_bond=8,
                           bond_cutoff=None), 0),
        (gs.chain_molecule(6, 21), 0),
        (gs.cluster_molecule(12, 9, radius=9.0), 60),
    ]
    return grid, mols


@pytest.mark.parametrize("route", ["A", "chi0"])
def test_results_same_alone_and_in_the_mix(gpu, route, monkeypatch):
    """Served results (A formed in W's buffer and solved in place, or with
    GW_SERVE_CHI0=1 through chi0 in a buffer of its own) are the same alone
    and in a mix, match the oracle on the tiny molecule and the eager
    chi0-route solve on every molecule."""
    gw, torch = gpu
    if route == "chi0":
        monkeypatch.setenv("GW_SERVE_CHI0", "1")
    else:
        monkeypatch.delenv("GW_SERVE_CHI0", raising=False)
    grid, mols = _workload()
    g = gw.make_grid(grid.n_omega, grid.omega_min, grid.omega_max, grid.eps)
    dms = [gw.DeviceMolecule(m) for m, _ in mols]
    ctx = gw.Context(0)
    # alone: one request at a time
    alone = []
    for (m, k), dm in zip(mols, dms):
        _say("alone n_prod", m.n_prod, "k", k)
        t = ctx.submit(dm.struct, dm.v, g, k_compress=k)
        ptr, rep = _wait(ctx, t)
        alone.append(_fetch(gw, torch, ptr, grid.n_omega, k or m.n_prod))
        ctx.release(t)
    # in the mix: all submitted at once, twice over
    tickets = []
    for rep_i in range(2):
        for (m, k), dm in zip(mols, dms):
            tickets.append((ctx.submit(dm.struct, dm.v, g, k_compress=k), len(tickets) % len(mols)))
    _say("submitted", len(tickets))
    for t, i in tickets:
        ptr, rep = _wait(ctx, t)
        m, k = mols[i]
        got = _fetch(gw, torch, ptr, grid.n_omega, k or m.n_prod)
        e = np.linalg.norm(got - alone[i]) / np.linalg.norm(alone[i])
        _say("ticket", t, "molecule", i, "rel diff vs alone", e)
        assert e <= 1e-12
        ctx.release(t)
    # and the tiny molecule against the oracle
    m = mols[0][0]
    P = o.pair_vectors(m)
    mm, fr = o.pair_bins(m.eig, m.n_occ, grid.domega)
    nhb = o.hist_bins(m.eig, grid.n_omega, grid.domega)
    s = o.frac_bits(P, m.n_pairs)
    H = o.histogram(P, mm, fr, s, nhb)
    js = [grid.n_omega // 2 + 9, 40]
    chi = o.unpack_upper(o.chi0_from_hist(H, s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps, js=js),
                         m.n_prod)
    for i, j in enumerate(js):
        Wr = o.screened_W(m.v, chi[i])
        assert np.linalg.norm(alone[0][j] - Wr) <= 1e-10 * np.linalg.norm(Wr)
    # every served result equals the eager solve (compressed: X of the same
    # basis) within the FP64 parity bar
    for ((m, k), dm, got) in zip(mols, dms, alone):
        kk = k or m.n_prod
        chi_e = torch.empty((grid.n_omega, kk, kk), dtype=torch.complex128, device="cuda")
        W_e = torch.empty_like(chi_e)
        if k:
            Q = torch.empty((m.n_prod, k), dtype=torch.float64, device="cuda")
            S = torch.empty((k, k), dtype=torch.float64, device="cuda")
            ctx.compress_basis(dm.v, m.n_prod, k, Q, S)
            ctx.build_chi0(dm.struct, g, chi_e, basis=Q, k=k)
            ctx.solve_W(S, k, chi_e, grid.n_omega, W_e)
        else:
            ctx.build_chi0(dm.struct, g, chi_e)
            ctx.solve_W(dm.v, m.n_prod, chi_e, grid.n_omega, W_e)
        ref = W_e.cpu().numpy()
        e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        _say("served n_prod", m.n_prod, "k", k, "rel vs eager", e)
        assert e < 1e-10
    ctx.close()


def test_serving_error_paths(gpu):
    gw, torch = gpu
    grid, mols = _workload()
    g = gw.make_grid(grid.n_omega, grid.omega_min, grid.omega_max, grid.eps)
    ctx = gw.Context(0, budget_bytes=64 << 20)  # 64 MiB: too small for the larger molecules
    dm = gw.DeviceMolecule(mols[2][0])
    with pytest.raises(gw.GwError) as e:
        ctx.submit(dm.struct, dm.v, g)
    assert e.value.status == gw.GW_E_OOM
    with pytest.raises(gw.GwError) as e:
        ctx.poll(12345)
    assert e.value.status == gw.GW_E_STATE
    with pytest.raises(gw.GwError) as e:
        ctx.release(12345)
    assert e.value.status == gw.GW_E_STATE
    with pytest.raises(gw.GwError) as e:
        ctx.submit(dm.struct, dm.v, g, k_compress=dm.n_prod + 1)
    assert e.value.status == gw.GW_E_INVALID
    ctx.close()


def test_release_cancels_a_queued_request(gpu):
    """A request that cannot be admitted waits in the queue; gw_release
    cancels it, its ticket becomes unknown, and the queue keeps moving."""
    gw, torch = gpu
    grid = gs.config_grid(0)
    g = gw.make_grid(grid.n_omega, grid.omega_min, grid.omega_max, grid.eps)
    m = gs.chain_molecule(3, 5)  # 152 products
    # One request keeps 16 * 152^2 * 256 B = 95 MB of results (W; A is formed
    # in its buffer) until released, and the library estimates 145 MB of
    # workspace for it: 240 MB at its peak, so under a 280 MiB (294 MB)
    # budget it is admitted, while a second one (95 + 95 + 145 = 335 MB) is
    # not as long as the first one's results are held.
    ctx = gw.Context(0, budget_bytes=280 << 20)
    dm = gw.DeviceMolecule(m)
    t1 = ctx.submit(dm.struct, dm.v, g)
    ptr1, _ = _wait(ctx, t1)
    t2 = ctx.submit(dm.struct, dm.v, g)
    time.sleep(0.2)
    assert ctx.poll(t2) is None  # still waiting for admission
    ctx.release(t2)
    with pytest.raises(gw.GwError) as e:
        ctx.poll(t2)
    assert e.value.status == gw.GW_E_STATE
    first = _fetch(gw, torch, ptr1, grid.n_omega, m.n_prod)
    ctx.release(t1)
    t3 = ctx.submit(dm.struct, dm.v, g)
    ptr3, _ = _wait(ctx, t3)
    again = _fetch(gw, torch, ptr3, grid.n_omega, m.n_prod)
    assert np.array_equal(first, again)
    ctx.release(t3)
    ctx.close()
