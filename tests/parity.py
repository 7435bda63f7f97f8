"""Statistical comparison used by the GPU parity tests.

Both sides are Monte Carlo means of the same estimator (Sec. 3.1: unbiased, variance
O(1/N)), so per point z = (m_gpu - m_ref)/sqrt(se_gpu^2 + se_ref^2) is approximately
standard normal. With many points a per-point 4-SE rule fails by chance (P(|Z| > 4) =
6.3e-5), so the acceptance is: at most max(1, 2 * 6.3e-5 * n) points with |z| > 4, none
with |z| > 6, and mean(z^2) below 1 + 5 sqrt(2/n) + 0.15 (the 0.15 absorbs the
underestimated standard errors of heavy-tailed weights at small walk counts)."""
import numpy as np


def zscores(m1, s1, m2, s2):
    se = np.sqrt(np.asarray(s1) ** 2 + np.asarray(s2) ** 2)
    return (np.asarray(m1) - np.asarray(m2)) / np.maximum(se, 1e-12)


def assert_parity(m1, s1, m2, s2, label=""):
    z = zscores(m1, s1, m2, s2)
    assert np.all(np.isfinite(z)), f"{label}: non-finite z"
    n = z.size
    n4 = int(np.sum(np.abs(z) > 4))
    allowed = max(1, int(np.ceil(2 * 6.3e-5 * n)))
    mz2 = float(np.mean(z * z))
    bound = 1 + 5 * np.sqrt(2.0 / n) + 0.15
    assert n4 <= allowed and np.max(np.abs(z)) < 6 and mz2 < bound, (
        f"{label}: n={n} |z|>4: {n4} (allowed {allowed}), max|z|={np.max(np.abs(z)):.2f}, "
        f"mean z^2={mz2:.3f} (bound {bound:.3f})")
    return z
