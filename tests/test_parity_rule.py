"""Calibration of the parity rule of tests/parity.py on the CPU.

* Null: two independent oracle runs of the same estimator (runs A and B of
  tests/golden/parity_*.npz, written by tests/golden/make_parity_refs.py) must be accepted
  on every full-size workload, and the rule's false-alarm rate, measured by shuffling the
  pooled batch means of each point into two halves, must stay near its budget
  (ALPHA = 1e-3 per comparison) despite the heavy-tailed walks.
* Power: a bias planted in one oracle run (every estimate scaled, as a 1-3% error in f
  and g would do by linearity of eq. 1; or shifted by a multiple of the combined standard
  error) must be rejected."""
import glob
import os

import numpy as np
import pytest
from scipy import stats

from tests import parity as P

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FILES = sorted(glob.glob(os.path.join(GOLDEN, "parity_*.npz")))
NAMES = [os.path.basename(f)[len("parity_"):-4] for f in FILES]


def load(name):
    return np.load(os.path.join(GOLDEN, f"parity_{name}.npz"), allow_pickle=False)


def test_reference_files_exist():
    assert set(NAMES) >= {"star256", "ico20480", "batch64", "square_rr"}


def test_rule_on_normal_samples():
    """The four checks hold their budget on exact normal scores and on batch means of
    normal data with unequal batch counts and spreads (Welch degrees of freedom)."""
    rng = np.random.default_rng(0)
    rej = sum(not P.accepts(rng.standard_normal(256))[0] for _ in range(4000))
    assert rej <= 12                     # Binomial(4000, 1e-3): P(> 12) < 1e-4
    rej = sum(not P.accepts(P.batch_scores(rng.standard_normal((32, 128)),
                                           3.0 * rng.standard_normal((16, 128))))[0] for _ in range(1000))
    assert rej <= 6                      # Binomial(1000, 1e-3): P(> 6) < 1e-4


def test_rule_rejects_planted_shifts():
    """A uniform shift of twice the detectable bias is rejected; a single point moved by
    8 standard errors is rejected by the per-point checks."""
    rng = np.random.default_rng(1)
    n = 256
    z = rng.standard_normal(n) + 2 * P.detectable_bias(n)
    assert not P.accepts(z)[0]
    z = rng.standard_normal(n)
    z[7] = 8.0
    assert not P.accepts(z)[0]


@pytest.mark.parametrize("name", NAMES)
def test_oracle_against_oracle_is_accepted(name):
    d = load(name)
    P.assert_parity_batches(d["run_a"], d["run_b"], f"oracle A vs B {name}", fp_tol=1e-12)


@pytest.mark.parametrize("name", NAMES)
def test_false_alarm_rate_by_permutation(name):
    """200 random splits of the 64 pooled batch means per point: the rule rejects at most
    3 (it would reject 0.2 on average at its budget; P(Binomial(200, 1e-3) > 3) < 1e-4)."""
    d = load(name)
    rej, reps = P.permutation_null(d["run_a"], d["run_b"], 200, np.random.default_rng(2), fp_tol=1e-12)
    assert rej <= 3, f"{name}: {rej} of {reps} null splits rejected"


@pytest.mark.parametrize("name", NAMES)
def test_planted_bias_is_rejected(name):
    """Run B scaled by 1 + delta, delta set to put the average shift at twice the bias
    the rule detects with probability 1/2, is rejected; so is run B shifted at every
    point by that many combined standard errors."""
    d = load(name)
    a, b = d["run_a"], d["run_b"]
    n = a.shape[1]
    ma, sa, _ = P.batch_mean_se(a)
    mb, sb, _ = P.batch_mean_se(b)
    comb = np.sqrt(sa ** 2 + sb ** 2)
    target = 2 * P.detectable_bias(n)
    delta = target * np.mean(comb) / max(np.mean(np.abs(ma)), 1e-12)
    scaled = b * (1 + np.sign(np.mean(ma)) * delta)
    assert not P.accepts(P.batch_scores(scaled, a, 1e-12))[0], f"{name}: scale 1 + {delta:.4f} accepted"
    shifted = b + target * comb[None, :]
    assert not P.accepts(P.batch_scores(shifted, a, 1e-12))[0], f"{name}: shift accepted"


def test_detectable_bias_matches_the_mean_check():
    """The detectable bias is where check (3) rejects with probability 1/2 (and 0.9)."""
    for n in (64, 256):
        b50, b90 = P.detectable_bias(n), P.detectable_bias(n, 0.9)
        thr = P.thresholds(n)["mean"]
        sd = 1 / np.sqrt(n)
        assert abs(stats.norm.sf((thr - b50) / sd) - 0.5) < 1e-9
        assert abs(stats.norm.sf((thr - b90) / sd) - 0.9) < 1e-6
