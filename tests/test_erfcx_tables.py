"""The fitted erfcx tables of the pair kernels (erfcx_f32.h, erfcx_f64.h)
against independent references: mpmath at 30 digits (FP64 table) and
scipy.special.erfcx (FP32 table), each evaluated the way its kernel does
(Horner in float32; Clenshaw in float64 with fused multiply-adds)."""
import os
import re

import mpmath
import numpy as np
import pytest
from scipy.special import erfcx

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2606_27134_amd", "csrc")


def _header(name):
    txt = open(os.path.join(CSRC, name)).read()
    defs = dict(re.findall(r"#define (\w+) ([-+0-9.eE]+)f?", txt))
    coef = [float(v.rstrip("f")) for v in re.findall(r"^\s+([-+0-9.eE]+f?),\s*$", txt, re.M)]
    return defs, coef


def _fma(a, b, c):
    # exact product and sum, one rounding (via mpmath), for the FP64 recurrence
    return float(mpmath.fsum([mpmath.mpf(a) * mpmath.mpf(b), mpmath.mpf(c)]))


def test_erfcx_f64_table():
    d, c = _header("erfcx_f64.h")
    deg, A, B, S = int(d["ERFCX_F64_DEG"]), float(d["ERFCX_F64_A"]), float(d["ERFCX_F64_B"]), float(d["ERFCX_F64_SHIFT"])
    assert len(c) == deg + 1
    mpmath.mp.dps = 30
    worst = 0.0
    for t in np.concatenate([np.linspace(0.0, 1.0, 41), np.linspace(1.0, 8.0, 141), [5.04203, 5.427695, 5.807081]]):
        u = 1.0 / (1.0 + S * t)
        x = _fma(A, u, B)
        b1 = b2 = 0.0
        for k in range(deg, 0, -1):
            b0 = _fma(2.0 * x, b1, c[k] - b2)
            b2, b1 = b1, b0
        got = u * _fma(x, b1, c[0] - b2)
        ref = mpmath.exp(mpmath.mpf(t) ** 2) * mpmath.erfc(mpmath.mpf(t))
        worst = max(worst, abs(float(got / ref) - 1.0))
    assert worst < 2e-14, worst
    # beyond the fitted range the series is extrapolated; exp(-t^2) times it
    # stays far below anything a sum at 1e-12 could see
    for t in (9.0, 12.0, 20.0, 30.0):
        u = 1.0 / (1.0 + S * t)
        x = A * u + B
        b1 = b2 = 0.0
        for k in range(deg, 0, -1):
            b1, b2 = 2.0 * x * b1 + (c[k] - b2), b1
        erfc_apx = np.exp(-t * t) * u * (x * b1 + (c[0] - b2))
        assert abs(erfc_apx - float(mpmath.erfc(t))) < 1e-30


def test_erfcx_f32_table():
    d, c = _header("erfcx_f32.h")
    deg, S = int(d["ERFCX_F32_DEG"]), np.float32(float(d["ERFCX_F32_SHIFT"]))
    assert len(c) == deg + 1
    t = np.linspace(0.0, 9.3, 200001).astype(np.float32)
    u = np.float32(1.0) / (np.float32(1.0) + S * t)
    acc = np.float32(c[-1])
    for ck in c[-2::-1]:
        acc = acc * u + np.float32(ck)
    rel = np.abs((u * acc).astype(np.float64) / erfcx(t.astype(np.float64)) - 1.0)
    assert rel.max() < 5e-7, rel.max()
