"""The generated device tables are what their generators write: the Chebyshev tables of
the Bessel functions (csrc/gen_bessel_tables.py, mpmath at 40 digits) and the envelope
constants of the radius proposals (csrc/gen_proposal_bound.py, which also asserts that
its series bounds the supremum of the acceptance ratio on a fine grid of s). The power
series forms that the FP32 walker evaluates by Horner's rule are pinned against scipy's
Bessel functions and against their Chebyshev forms."""
import os
import subprocess
import sys

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2201_13240_amd", "csrc")


@pytest.mark.parametrize("gen,header", [("gen_bessel_tables.py", "bessel_tables.h"),
                                        ("gen_proposal_bound.py", "proposal_bound.h")])
def test_header_regenerates_identically(gen, header):
    out = subprocess.run([sys.executable, gen], cwd=CSRC, capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    with open(os.path.join(CSRC, header)) as f:
        assert out.stdout == f.read()


def _table(text, name):
    import re
    body = re.search(r"WOS_%s\[\d+\] = \{(.*?)\};" % name, text, re.S).group(1)
    return [float(v) for v in body.replace("\n", " ").split(",")]


def test_fp32_power_series_fits_match_scipy():
    """The power series that the FP32 walker evaluates by Horner's rule for x >= 2,
    sqrt(x) e^-x I0(x) and sqrt(x) e^x K0(x) in t = 4/x - 1, evaluated in FP32 with one
    rounding per step, against scipy's scaled Bessel functions: within 2e-7 relative on
    x in [2, 1e6]."""
    import numpy as np
    from scipy import special
    with open(os.path.join(CSRC, "bessel_tables.h")) as f:
        text = f.read()
    x = np.concatenate([np.linspace(2.0, 40.0, 4001), np.geomspace(40.0, 1e6, 801)])
    t = (np.float32(4.0) / x.astype(np.float32) - np.float32(1.0)).astype(np.float32)
    for name, ref in (("I0E_WIDE_TAIL", np.sqrt(x) * special.i0e(x)), ("K0E_WIDE_TAIL", np.sqrt(x) * special.k0e(x))):
        p = np.array(_table(text, name + "_POW32"), dtype=np.float32)
        acc = np.full(t.shape, p[-1], dtype=np.float32)
        for c in p[-2::-1]:
            acc = (acc.astype(np.float64) * t + np.float64(c)).astype(np.float32)
        err = np.abs(acc.astype(np.float64) - ref) / ref
        assert err.max() < 2e-7, (name, err.max())


def test_envelope_power_series_equal_chebyshev_series():
    """Each envelope polynomial is written twice, as Chebyshev coefficients (FP64 walker)
    and as a power series (FP32 walker): the two agree to rounding on [-1, 1]."""
    import numpy as np
    with open(os.path.join(CSRC, "proposal_bound.h")) as f:
        text = f.read()
    u = np.linspace(-1.0, 1.0, 2001)
    for tag in ("PROP", "PROP3"):
        c = np.array(_table(text, tag + "_C"))
        p = np.array(_table(text, tag + "_P"))
        assert np.max(np.abs(np.polynomial.chebyshev.chebval(u, c) - np.polynomial.polynomial.polyval(u, p))) < 1e-12
