"""Pins of the oracle's Swendsen-Wang chain against exact results.

The SW chain leaves the Potts measure invariant (Sec. II) and its bond
configurations are distributed by the random-cluster measure
(Eq. random_cluster).  Long-run averages of the oracle's per-sweep records must
therefore match:

* exact Boltzmann averages by full enumeration of tiny periodic lattices
  (4x4 Ising at beta_c, 3x4 Potts q=3 at its critical coupling, 3x3 q=4);
* exact random-cluster expectations by enumerating all 2^18 bond sets of the
  3x3 torus.

A dropped bond, a wrong neighbour index, a biased state draw or a wrong
threshold direction each moves one of these averages by many standard errors.
"""
import math

import numpy as np
import pytest

import oracle
from tests import exact

SEED = 0x1105580400000001


def _k_of_T(T):
    """Coupling that the integer threshold T realises exactly: p = T / 2^32."""
    return -math.log1p(-T / 2.0**32)


def _run(W, H, q, T, n, burn=500, seed=SEED, sid=0):
    st = oracle.init_states(W, H, q, seed, sid)
    st, _ = oracle.sw_run(W, H, q, T, seed, sid, 0, burn, st)
    st, rec = oracle.sw_run(W, H, q, T, seed, sid, burn, n, st)
    return st, rec


def _close(series, want, nsig=5.0):
    mean = float(np.mean(series))
    err = exact.binned_error(series)
    assert abs(mean - want) < nsig * err + 1e-12, (mean, want, err)


def test_ising_4x4_exact():
    W = H = 4
    N = W * H
    T = oracle.threshold(math.log1p(math.sqrt(2.0)))
    ref = exact.potts_exact(W, H, 2, _k_of_T(T))
    _, rec = _run(W, H, 2, T, 200_000)
    nsat = rec[:, oracle.REC_NSAT]
    m = (2.0 * rec[:, oracle.REC_COUNTS + 1] - N) / N
    _close(nsat / N, ref["nsat"] / N)
    _close(np.abs(m), ref["absm"])
    _close(m ** 2, ref["m2"])
    _close(m ** 4, ref["m4"])
    # the energy per site e = -(2 n_sat - 2N)/N is the paper's observable
    assert abs(np.mean(-(2 * nsat - 2 * N) / N) - (-(2 * ref["nsat"] - 2 * N) / N)) < 0.01


def test_potts3_3x4_exact():
    W, H, q = 3, 4, 3
    N = W * H
    T = oracle.threshold(math.log1p(math.sqrt(3.0)))
    ref = exact.potts_exact(W, H, q, _k_of_T(T))
    _, rec = _run(W, H, q, T, 150_000)
    _close(rec[:, oracle.REC_NSAT] / N, ref["nsat"] / N)
    cmax = rec[:, oracle.REC_COUNTS:oracle.REC_COUNTS + q].max(axis=1) / N
    _close(cmax, ref["maxfrac"])


def test_potts4_3x3_exact():
    W, H, q = 3, 3, 4
    T = oracle.threshold(1.0)
    ref = exact.potts_exact(W, H, q, _k_of_T(T))
    _, rec = _run(W, H, q, T, 150_000)
    _close(rec[:, oracle.REC_NSAT] / 9.0, ref["nsat"] / 9.0)


@pytest.mark.parametrize("q,K", [(2, math.log1p(math.sqrt(2.0))), (3, math.log1p(math.sqrt(3.0)))])
def test_fk_3x3_exact(q, K):
    T = oracle.threshold(K)
    ref = exact.fk_exact(3, 3, q, T / 2.0**32)
    _, rec = _run(3, 3, q, T, 150_000)
    _close(rec[:, oracle.REC_NCLUST], ref["nclust"])
    _close(rec[:, oracle.REC_ACTIVE], ref["active"])
    _close(rec[:, oracle.REC_MAXCL], ref["maxcl"])


def test_special_thresholds():
    W, H, q = 9, 6, 3
    N = W * H
    st0 = oracle.init_states(W, H, q, SEED)
    # T = 0: no bond is ever active, every site is its own cluster
    st, bonds, labels, rec = oracle.sw_sweep(W, H, q, 0, SEED, 0, 0, st0)
    assert not bonds.any() and np.array_equal(labels, np.arange(N))
    assert rec[oracle.REC_NCLUST] == N and rec[oracle.REC_MAXCL] == 1
    # T = 2^32 from a uniform state: one cluster, labelled 0, stays uniform
    uni = np.full(N, 2, np.uint8)
    st, bonds, labels, rec = oracle.sw_sweep(W, H, q, 2**32, SEED, 0, 5, uni)
    assert np.all(bonds == 3) and np.all(labels == 0) and rec[oracle.REC_NCLUST] == 1
    assert np.all(st == st[0])
    # T = 2^32 from a checkerboard Ising state: all bonds unsatisfied, N singletons
    cb = ((np.arange(N) % W + np.arange(N) // W) % 2).astype(np.uint8)
    W2 = 8
    cb = ((np.arange(W2 * H) % W2 + np.arange(W2 * H) // W2) % 2).astype(np.uint8)
    st, bonds, labels, rec = oracle.sw_sweep(W2, H, 2, 2**32, SEED, 0, 0, cb)
    assert not bonds.any() and rec[oracle.REC_NCLUST] == W2 * H


def test_sweep_consistency():
    """Bonds join only equal spins, clusters are uniform after the flip, labels canonical."""
    W, H, q = 23, 17, 3
    T = oracle.threshold(math.log1p(math.sqrt(3.0)))
    st = oracle.init_states(W, H, q, SEED)
    for t in range(5):
        new, bonds, labels, rec = oracle.sw_sweep(W, H, q, T, SEED, 0, t, st)
        x = np.arange(W * H) % W
        y = np.arange(W * H) // W
        right = y * W + (x + 1) % W
        down = ((y + 1) % H) * W + x
        assert np.all(st[(bonds & 1) != 0] == st[right[(bonds & 1) != 0]])
        assert np.all(st[(bonds & 2) != 0] == st[down[(bonds & 2) != 0]])
        assert np.array_equal(labels, exact.bfs_labels(W, H, bonds, True))
        assert np.all(new == new[labels])
        assert rec[oracle.REC_ACTIVE] == int((bonds & 1).astype(bool).sum() + (bonds & 2).astype(bool).sum())
        st = new


def test_checkpoint_resume():
    W, H, q = 12, 10, 2
    T = oracle.threshold(math.log1p(math.sqrt(2.0)))
    st = oracle.init_states(W, H, q, SEED, 5)
    a, rec_a = oracle.sw_run(W, H, q, T, SEED, 5, 0, 30, st)
    b, rec_b1 = oracle.sw_run(W, H, q, T, SEED, 5, 0, 13, st)
    b, rec_b2 = oracle.sw_run(W, H, q, T, SEED, 5, 13, 17, b)
    assert np.array_equal(a, b)
    assert np.array_equal(rec_a, np.concatenate([rec_b1, rec_b2]))


def test_init_uniform():
    W, H = 256, 256
    for q in (2, 3, 5):
        st = oracle.init_states(W, H, q, SEED)
        c = np.bincount(st, minlength=q)
        assert c.size == q
        e = W * H / q
        chi2 = float(((c - e) ** 2 / e).sum())
        assert chi2 < q * 10, (q, c)


@pytest.mark.slow
def test_binder_crossing_brackets_beta_c():
    """U_L = 1 - <m^4>/(3<m^2>^2) grows with L above beta_c and shrinks below."""
    bc = 0.5 * math.log1p(math.sqrt(2.0))

    def binder(L, beta, n):
        T = oracle.threshold(2.0 * beta)
        _, rec = _run(L, L, 2, T, n, burn=300)
        m = (2.0 * rec[:, oracle.REC_COUNTS + 1] - L * L) / (L * L)
        return 1.0 - np.mean(m ** 4) / (3.0 * np.mean(m ** 2) ** 2)

    lo = [binder(L, 0.85 * bc, 6000) for L in (8, 16)]
    hi = [binder(L, 1.15 * bc, 6000) for L in (8, 16)]
    assert lo[1] < lo[0]
    assert hi[1] > hi[0]
