"""The generated device tables are what their generators write: the Chebyshev tables of
the Bessel functions (csrc/gen_bessel_tables.py, mpmath at 40 digits) and the envelope
constants of the radius proposals (csrc/gen_proposal_bound.py, which also asserts that
its series bounds the supremum of the acceptance ratio on a fine grid of s)."""
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
