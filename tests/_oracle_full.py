"""The oracle's own chi0 and W of a whole molecule at sampled frequencies, for
the full-size GPU parity tests: the exact int64 histogram over every entry
mu <= nu (the oracle's plain C code on the host cores), chi0 by direct
summation of its Cauchy transform (Section 5.A), and W = (1 - v chi0)^{-1} v
by LAPACK (Section 2 eq. Coulombscreening).  Nothing here reads GPU output."""
import sys
import time

import numpy as np

import oracle as o


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sampled_js(grid):
    """The lone point j = 0 (omega_min), omega = 0, three frequencies inside
    the pair band (0.2 .. 3 Ha), two above it and two negative ones."""
    N, d = grid.n_omega, grid.domega
    j0 = N // 2
    pick = [0.5, 1.2, 2.5, 4.0, 7.0, -1.0, -3.0]
    js = [0, j0] + [j0 + int(round(w / d)) for w in pick]
    assert all(0 <= j < N for j in js) and len(set(js)) == len(js)
    return js


class OracleFull:
    def __init__(self, mol, grid, js=None):
        self.js = list(js) if js is not None else sampled_js(grid)
        t0 = time.time()
        self.P = o.pair_vectors(mol)
        _say("oracle: pair vectors %.1fs" % (time.time() - t0))
        d = grid.domega
        self.m, self.fr = o.pair_bins(mol.eig, mol.n_occ, d)
        self.nhb = o.hist_bins(mol.eig, grid.n_omega, d)
        self.s = o.frac_bits(self.P, mol.n_pairs)
        t0 = time.time()
        self.H, self.dropped = o.histogram_c(self.P, self.m, self.fr, self.s, self.nhb)
        _say("oracle: int64 histogram of all %d entries %.1fs" % (self.H.shape[1], time.time() - t0))
        t0 = time.time()
        c = o.chi0_from_hist(self.H, self.s, grid.n_omega, grid.omega_min, grid.omega_max, grid.eps, js=self.js)
        self.chi = o.unpack_upper(c, mol.n_prod)
        del c
        _say("oracle: chi0 at %d frequencies %.1fs" % (len(self.js), time.time() - t0))
        t0 = time.time()
        self.W = np.array([o.screened_W(mol.v, self.chi[i]) for i in range(len(self.js))])
        _say("oracle: LAPACK W at %d frequencies %.1fs" % (len(self.js), time.time() - t0))


def compare(name, got, ref, bound):
    """Relative Frobenius error and the largest entry error relative to the
    largest entry, per frequency; both must be within `bound`."""
    worst = 0.0
    for i in range(len(ref)):
        fro = float(np.linalg.norm(got[i] - ref[i]) / np.linalg.norm(ref[i]))
        ent = float(np.abs(got[i] - ref[i]).max() / np.abs(ref[i]).max())
        worst = max(worst, fro, ent)
    _say("%s: worst relative error over %d frequencies %.2e (bar %.0e)" % (name, len(ref), worst, bound))
    assert worst <= bound, "%s: %.3e > %.0e" % (name, worst, bound)
    return worst


def forward_errors(mol, grid, js, cols, W_apply):
    """Forward error of computed W(omega_j) columns where the oracle cannot
    form chi0.  For column c the oracle's residual is
        r = v e_c - (1 - v chi0) w,   w = W e_c,
    with chi0 applied by its pair-vertex route, and the error of w is
    A^-1 r with A = 1 - v chi0.  Since W_true = A^-1 v, A^-1 = 1 + W_true chi0
    exactly ((1 - v chi0)(1 + W_true chi0) = 1 - v chi0 + v chi0), so the error
    is estimated by
        delta = r + W (chi0 r)
    with the computed W in place of W_true, off only by the (small) relative
    error of W itself (second order in it).
      W_apply(j, x): W(omega_j) x for a vector x (W e_c gives the column).
    Returns (largest ||delta|| / ||w||, largest ||r|| / ||v e_c||)."""
    om = grid.omegas()
    nhb = o.hist_bins(mol.eig, grid.n_omega, grid.domega)
    n = mol.n_prod
    worst_fwd = worst_res = 0.0
    for j in js:
        for c in cols:
            e = np.zeros(n)
            e[c] = 1.0
            w = W_apply(j, e)
            r = mol.v[:, c] - (w - mol.v @ o.chi0_apply(mol, w, om[j], grid.eps, grid.domega, nhb))
            d = r + W_apply(j, o.chi0_apply(mol, r, om[j], grid.eps, grid.domega, nhb))
            worst_fwd = max(worst_fwd, float(np.linalg.norm(d) / np.linalg.norm(w)))
            worst_res = max(worst_res, float(np.linalg.norm(r) / np.linalg.norm(mol.v[:, c])))
    _say("forward error over %d columns x %d frequencies: %.2e (residual %.2e)"
         % (len(cols), len(js), worst_fwd, worst_res))
    return worst_fwd, worst_res
