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
