"""Statistical checks of the coins and thresholds the hash produces, seen
through the oracle's own simulation (the device hash equals the oracle's bit
for bit, so these carry over):

* IC coins (Section 2, "Diffusion Models": each arc fires with probability
  p): on an out-star the live arcs over 10^8 coins match the encoded rate
  within 5 sigma; per-leaf counts pass a chi-square test against the
  binomial; per-trial counts have the binomial variance (arcs of one trial
  independent) and no lag-1 correlation (trials that share a hash block
  independent); adjacent arc ids are pairwise independent.
* LT thresholds (uniform on [0, 1]): a node whose only active in-neighbour
  has weight w joins with probability w; with w = j/16 for j = 1..15 the join
  rates follow the uniform CDF at those points (each within 5 sigma, and a
  chi-square over the 15 independent counts).
"""
import numpy as np
from scipy import stats

import oracle
from tests import pins


def _out_star(m):
    src = np.zeros(m, dtype=np.int64)
    dst = np.arange(1, m + 1)
    off, idx = pins.csr_from_arcs(m + 1, src, dst)
    return m + 1, off, idx


def test_ic_coins_rate_spread_and_independence():
    m, T, p = 1000, 100_000, 0.1
    n, off, idx = _out_star(m)
    thr = oracle.encode_p(np.full(m, p))
    p_eff = int(thr[0]) / 2**32
    r = oracle.simulate("ic", n, off, idx, thr, [0], T, 77, threads=8, want_bits=True)
    live = r["total"] - T  # the seed counts once per trial
    N = m * T
    assert abs(live - N * p_eff) < 5 * np.sqrt(N * p_eff * (1 - p_eff))
    # per-leaf counts: chi-square against Binomial(T, p)
    c = r["node_counts"][1:].astype(np.float64)
    chi = float((((c - T * p_eff) ** 2) / (T * p_eff * (1 - p_eff))).sum())
    pv = stats.chi2.sf(chi, m)
    assert 1e-6 < pv < 1 - 1e-6, pv
    # per-trial counts: binomial variance and no lag-1 correlation
    k = r["trial_counts"].astype(np.float64) - 1
    var = k.var()
    exp_var = m * p_eff * (1 - p_eff)
    assert abs(var / exp_var - 1) < 5 * np.sqrt(2 / T)
    r1 = np.corrcoef(k[:-1], k[1:])[0, 1]
    assert abs(r1) < 5 / np.sqrt(T)
    # adjacent arc ids: joint firing of leaves i and i + 1 (4,000 trials)
    bits = r["active_bits"][:63]  # 63 words = 4,032 trials
    tt = bits.shape[0] * 64
    both = 0
    for w in range(bits.shape[0]):
        a = bits[w, 1:m]
        b = bits[w, 2:m + 1]
        both += int(sum(bin(int(x)).count("1") for x in (a & b)))
    pairs = (m - 1) * tt
    exp = pairs * p_eff * p_eff
    assert abs(both - exp) < 5 * np.sqrt(exp * (1 - p_eff * p_eff))


def test_lt_thresholds_uniform():
    # 15 in-stars of one arc each: seed s_j -> centre c_j with weight j/16
    J, T = 15, 200_000
    src = np.arange(J)
    dst = np.arange(J, 2 * J)
    w = np.arange(1, J + 1) / 16.0
    off, idx, wp = pins.csr_from_arcs(2 * J, src, dst, w)
    enc = oracle.encode_w(wp)
    r = oracle.simulate("lt", 2 * J, off, idx, enc, np.arange(J), T, 91, threads=8, want_bits=False)
    joins = r["node_counts"][J:].astype(np.float64)
    rate = joins / T
    w_eff = enc.astype(np.float64) / 2**32
    sd = np.sqrt(w_eff * (1 - w_eff) / T)
    assert (np.abs(rate - w_eff) < 5 * sd).all(), (rate, w_eff)
    # each centre draws its own thresholds, so the 15 counts are independent
    # binomials: chi-square with 15 degrees of freedom
    chi = float((((joins - T * w_eff) ** 2) / (T * w_eff * (1 - w_eff))).sum())
    pv = stats.chi2.sf(chi, J)
    assert 1e-6 < pv < 1 - 1e-6, (chi, pv)
