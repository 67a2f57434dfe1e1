"""The normal-tail constants of the BlackScholes kernel against scipy's erfc.

The kernel's polynomial (TAIL_P, TAIL_C in lift_blackscholes.hip) is read
from the source and evaluated in binary64: Q(z) = phi(z) sum_k c_k t^k,
t = 1 / (1 + p z), must match erfc(z / sqrt 2) / 2 within 3e-8 absolute on
[0, 40], and the fitting script must reproduce the committed constants.
"""
import math
import os
import re
import runpy

import numpy as np
from scipy.special import erfc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1502_02389_amd", "csrc", "lift_blackscholes.hip")
FIT = os.path.join(ROOT, "paper_1502_02389_amd", "csrc", "fit_normal_tail.py")


def constants():
    text = open(SRC).read()
    p = float(re.search(r"TAIL_P = ([0-9.eE+-]+)f;", text).group(1))
    body = re.search(r"TAIL_C\[7\] = \{(.*?)\};", text, re.S).group(1)
    c = [float(v.strip().rstrip("f")) for v in body.split(",")]
    return np.float32(p), np.array(c, dtype=np.float32)


def test_committed_tail_constants_match_erfc():
    p, c = constants()
    assert len(c) == 7
    z = np.linspace(0.0, 40.0, 400001)
    t = 1 / (1 + float(p) * z)
    r = sum(float(ck) * t ** (k + 1) for k, ck in enumerate(c))
    q = np.exp(-z * z / 2) / math.sqrt(2 * math.pi) * r
    assert float(np.max(np.abs(q - 0.5 * erfc(z / math.sqrt(2))))) <= 3e-8


def test_fitting_script_reproduces_the_constants():
    mod = runpy.run_path(FIT)
    p, c = constants()
    c_fit = mod["fit"](float(p))
    assert np.allclose(c_fit, c.astype(np.float64), rtol=2e-7, atol=0)   # printed to 10 digits, then binary32
