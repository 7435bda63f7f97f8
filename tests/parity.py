"""Statistical comparison used by the GPU parity tests.

Both sides are Monte Carlo means of the same estimator (Sec. 3.1: unbiased, variance
O(1/N)), so per point z = (m_gpu - m_ref)/sqrt(se_gpu^2 + se_ref^2 + tol^2) is close to
standard normal. Two effects shape the acceptance rule:

* Points closer to the boundary than epsilon end every walk at once (Alg. 1), so their
  standard error is exactly zero and only rounding separates the two sides. `fp_tol`
  (relative) covers that: 2e-6 for FP32 results (unit round-off 6e-8 times the ~30
  operations between the query point and g(xbar)), 1e-12 for FP64.
* Per-walk values are skewed: near the boundary most walks stop at once and a rare walk
  makes a long excursion; null-collision weights are heavy-tailed. The standard error
  estimated from N walks is then occasionally optimistic, and a correct solver shows
  5-7 sigma points at a rate well above the normal 6.3e-5 (a 65536-walk outlier at
  |z| = 5.2 fell to |z| = 0.9 with 10^6 walks). A gross error (a wrong field, sign,
  problem or weight) moves every point and shows in the mean of z^2 and of z.

Acceptance (spec: agreement within 4 combined standard errors per point, read
with a multiple-comparison allowance): at most max(2, 1% of n) points with |z| > 4, none
with |z| > 8, mean(z^2) < 1 + 5 sqrt(2/n) + 0.2, and |mean(z)| < 4/sqrt(n) + 0.1."""
import numpy as np


def zscores(m1, s1, m2, s2, fp_tol=0.0):
    m1, m2 = np.asarray(m1, float), np.asarray(m2, float)
    scale = np.maximum(1.0, np.abs(m2))
    se = np.sqrt(np.asarray(s1) ** 2 + np.asarray(s2) ** 2 + (fp_tol * scale) ** 2)
    return (m1 - m2) / np.maximum(se, 1e-300)


def assert_parity(m1, s1, m2, s2, label="", fp_tol=2e-6):
    z = zscores(m1, s1, m2, s2, fp_tol)
    assert np.all(np.isfinite(z)), f"{label}: non-finite z"
    n = z.size
    n4 = int(np.sum(np.abs(z) > 4))
    allowed = max(2, int(np.ceil(0.01 * n)))
    mz2 = float(np.mean(z * z))
    mz = float(np.mean(z))
    bound = 1 + 5 * np.sqrt(2.0 / n) + 0.2
    bias_bound = 4 / np.sqrt(n) + 0.1
    ok = n4 <= allowed and np.max(np.abs(z)) < 8 and mz2 < bound and abs(mz) < bias_bound
    assert ok, (f"{label}: n={n} |z|>4: {n4} (allowed {allowed}), max|z|={np.max(np.abs(z)):.2f}, "
                f"mean z^2={mz2:.3f} (bound {bound:.3f}), mean z={mz:.3f} (bound {bias_bound:.3f})")
    return z
