"""Statistical comparison of two Monte Carlo estimates of the same quantity.

Both sides are means of the same estimator (Sec. 3.1, eqs. 17-18: unbiased, variance
O(1/N)), so per point

    z = (m_1 - m_2) / sqrt(se_1^2 + se_2^2 + (fp_tol max(1, |m_2|))^2)

is close to a standard score. The standard errors come either

* from the sample variance of many walks (`assert_parity`; reference distribution: the
  standard normal), or
* from batch means (`assert_parity_batches`): each side gives B independent batch means
  per point, se = their standard deviation / sqrt(B). z then follows Student's t with the
  Welch-Satterthwaite degrees of freedom of the point and is mapped to a normal score
  through that distribution. Batch means of many walks are close to normal even where
  single walks are heavy-tailed (null-collision weights, rare long excursions), and the
  degrees of freedom account for the uncertainty of the standard error itself.

`fp_tol` (relative) covers points whose walks all end at once in the epsilon shell
(zero variance), where only rounding separates the sides: 2e-6 for FP32 results (unit
round-off times the ~30 operations between the query point and g(xbar)), 1e-12 for FP64.

Acceptance: a false-alarm budget ALPHA = 1e-3 per comparison, split evenly over four
checks of the n normal scores against the standard normal:
  (1) points with |z| > 4: at most the (1 - ALPHA/4) quantile of Binomial(n, P(|Z| > 4));
  (2) max |z| below the two-sided normal quantile at ALPHA / (4 n);
  (3) |mean z| below C_MEAN / sqrt(n), C_MEAN the two-sided quantile at ALPHA/4;
  (4) mean z^2 below the (1 - ALPHA/4) quantile of chi^2_n / n.
Check (3) catches a bias shared by the points: a shift of b combined standard errors at
every point is rejected with probability 1/2 at b = C_MEAN / sqrt(n) and 0.9 at
b = (C_MEAN + 1.28) / sqrt(n) (`detectable_bias`)."""
import math

import numpy as np
from scipy import stats

ALPHA = 1e-3
C_MEAN = float(stats.norm.isf(ALPHA / 8))       # two-sided at ALPHA/4
P_BEYOND_4 = float(2 * stats.norm.sf(4.0))


def thresholds(n):
    return {"beyond_4": int(stats.binom.ppf(1 - ALPHA / 4, n, P_BEYOND_4)),
            "max_abs": float(stats.norm.isf(ALPHA / (8 * n))),
            "mean": C_MEAN / math.sqrt(n),
            "mean_sq": float(stats.chi2.isf(ALPHA / 4, n)) / n}


def detectable_bias(n, power=0.5):
    """Uniform shift, in combined standard errors, that check (3) rejects with the given
    probability at n points."""
    return (C_MEAN + float(stats.norm.isf(1 - power))) / math.sqrt(n)


def zscores(m1, s1, m2, s2, fp_tol=0.0):
    m1, m2 = np.asarray(m1, float), np.asarray(m2, float)
    scale = np.maximum(1.0, np.abs(m2))
    se = np.sqrt(np.asarray(s1) ** 2 + np.asarray(s2) ** 2 + (fp_tol * scale) ** 2)
    return (m1 - m2) / np.maximum(se, 1e-300)


def normal_scores(z, dof):
    """Maps t-distributed scores with per-point degrees of freedom to standard normal
    scores (probability-preserving); dof = inf leaves them unchanged."""
    z = np.asarray(z, float)
    dof = np.broadcast_to(np.asarray(dof, float), z.shape)
    out = z.copy()
    fin = np.isfinite(dof)
    if np.any(fin):
        p = stats.t.sf(np.abs(z[fin]), dof[fin])
        out[fin] = np.sign(z[fin]) * stats.norm.isf(np.maximum(p, 1e-300))
    return out


def statistics(z):
    n = z.size
    t = thresholds(n)
    return {"n": n, "beyond_4": int(np.sum(np.abs(z) > 4)), "max_abs": float(np.max(np.abs(z))),
            "mean": float(np.mean(z)), "mean_sq": float(np.mean(z * z)), "thresholds": t}


def accepts(z):
    s = statistics(z)
    t = s["thresholds"]
    ok = (np.all(np.isfinite(z)) and s["beyond_4"] <= t["beyond_4"] and s["max_abs"] < t["max_abs"]
          and abs(s["mean"]) < t["mean"] and s["mean_sq"] < t["mean_sq"])
    return bool(ok), s


def _check(z, label):
    assert np.all(np.isfinite(z)), f"{label}: non-finite z"
    ok, s = accepts(z)
    t = s["thresholds"]
    assert ok, (f"{label}: n={s['n']} |z|>4: {s['beyond_4']} (allowed {t['beyond_4']}), max|z|={s['max_abs']:.2f} "
                f"(bound {t['max_abs']:.2f}), mean z={s['mean']:.3f} (bound {t['mean']:.3f}), mean z^2="
                f"{s['mean_sq']:.3f} (bound {t['mean_sq']:.3f})")
    return s


def assert_parity(m1, s1, m2, s2, label="", fp_tol=2e-6):
    """Means and standard errors from the sample variance of each side's walks (or an
    exact reference with s2 = 0)."""
    z = zscores(m1, s1, m2, s2, fp_tol)
    _check(z, label)
    return z


def batch_mean_se(batches):
    """Per point: mean of the B batch means ([B][n]) and its standard error."""
    b = np.asarray(batches, float)
    B = b.shape[0]
    return b.mean(0), b.std(0, ddof=1) / math.sqrt(B), B


def batch_scores(b1, b2, fp_tol=0.0):
    """Normal scores of two sets of batch means ([B1][n], [B2][n]) of the same points."""
    m1, s1, B1 = batch_mean_se(b1)
    m2, s2, B2 = batch_mean_se(b2)
    z = zscores(m1, s1, m2, s2, fp_tol)
    v1, v2 = s1 ** 2, s2 ** 2
    den = v1 ** 2 / (B1 - 1) + v2 ** 2 / (B2 - 1)
    dof = np.where(den > 0, (v1 + v2) ** 2 / np.maximum(den, 1e-300), np.inf)
    return normal_scores(z, dof)


def batch_scores_vs_exact(b, exact, fp_tol=0.0):
    """Normal scores of batch means ([B][n]) against exact values (Student's t, B - 1
    degrees of freedom)."""
    m, s, B = batch_mean_se(b)
    z = zscores(m, s, exact, 0.0, fp_tol)
    return normal_scores(z, np.where(s > 0, B - 1.0, np.inf))


def assert_parity_batches_exact(b, exact, label="", fp_tol=2e-6):
    """Batch means against an exact solution. Per-walk estimates can be strongly skewed
    (null-collision weights above one where sigma' < 0), so that the mean of a few thousand
    walks typically falls below the expectation; comparisons against exact values use
    many walks."""
    z = batch_scores_vs_exact(b, exact, fp_tol)
    return _check(z, label)


def assert_parity_batches(b1, b2, label="", fp_tol=2e-6):
    z = batch_scores(b1, b2, fp_tol)
    return _check(z, label)


def permutation_null(ba, bb, reps, rng, fp_tol=0.0):
    """False-alarm rate of the rule on two runs of the same estimator (batch means [B][n]
    each): the 2B batches of every point are shuffled into two halves `reps` times and
    each split is judged. Returns (rejections, reps)."""
    pool = np.concatenate([np.asarray(ba, float), np.asarray(bb, float)])
    B = pool.shape[0] // 2
    rejected = 0
    for _ in range(reps):
        perm = rng.permuted(np.tile(np.arange(2 * B)[:, None], (1, pool.shape[1])), axis=0)
        sh = np.take_along_axis(pool, perm, axis=0)
        ok, _ = accepts(batch_scores(sh[:B], sh[B:], fp_tol))
        rejected += 0 if ok else 1
    return rejected, reps
