"""The FP32 polynomial behind the mixed-precision real-space kernel:
erfc(x) exp(x^2) ~= t P(t), t = 1 / (1 + x / 2), with the coefficients the
kernel compiles in (read from its header).  Checked against SciPy's erfcx, in
exact arithmetic and with the kernel's FP32 Horner evaluation emulated."""
import pathlib
import re

import numpy as np
import pytest
from scipy.special import erfc, erfcx

HDR = pathlib.Path(__file__).resolve().parents[1] / "paper_1708_01135_amd" / "csrc" / "erfcx_fit.h"


def _coeffs():
    txt = HDR.read_text()
    t_scale = float(re.search(r"kErfcxT\s*=\s*([0-9.eE+-]+)f", txt).group(1))
    deg = int(re.search(r"kErfcxDegree\s*=\s*(\d+)", txt).group(1))
    body = txt[txt.index("kErfcxP[kErfcxDegree + 1] = {"):]
    body = body[body.index("{") + 1:body.index("};")]
    vals = [float.fromhex(m) for m in re.findall(r"(-?0x[0-9a-fA-Fp.+-]+)f", body)]
    assert len(vals) == deg + 1
    return t_scale, np.array(vals, dtype=np.float32)


def _fma32(a, b, c):
    # a*b of two FP32 values is exact in FP64; one rounding to FP32 after the add
    return np.float32(np.float64(a) * np.float64(b) + np.float64(c))


def _eval_fp32(x):
    p, c = _coeffs()
    x = np.asarray(x, dtype=np.float32)
    t = np.float32(1.0) / (np.float32(1.0) + np.float32(p) * x)
    acc = np.full_like(x, c[-1])
    for ci in c[-2::-1]:
        acc = _fma32(acc, t, ci)
    return (acc * t).astype(np.float32)


def test_coefficients_are_fp32_and_lead_term_matches_asymptote():
    p, c = _coeffs()
    assert c.dtype == np.float32
    # x -> infinity: erfcx(x) ~ 1 / (sqrt(pi) x) and t ~ 1 / (p x), so P(0) -> p / sqrt(pi)
    assert abs(float(c[0]) - p / np.sqrt(np.pi)) < 2e-6


def test_fit_relative_error_exact_arithmetic():
    p, c = _coeffs()
    x = np.concatenate([np.linspace(0.0, 12.0, 240001), np.geomspace(12.0, 1e7, 20001)])
    t = 1.0 / (1.0 + p * x)
    approx = np.polyval(np.float64(c)[::-1], t) * t
    assert np.max(np.abs(approx / erfcx(x) - 1.0)) < 1e-7


@pytest.mark.parametrize("lo,hi", [(0.0, 1.0), (1.0, 4.0), (4.0, 8.0)])
def test_fp32_evaluation_error(lo, hi):
    x = np.linspace(lo, hi, 100001)
    rel = np.abs(_eval_fp32(x).astype(np.float64) / erfcx(x) - 1.0)
    assert np.max(rel) < 5e-7


def test_erfc_reconstruction_over_ewald_range():
    # erfc(x) = exp(-x^2) erfcx(x): the product the kernel forms, for the
    # real-space arguments sqrt(alpha) r of typical plans (x up to ~4.5)
    x = np.linspace(0.05, 4.5, 20001)
    rec = np.exp(-x * x) * _eval_fp32(x).astype(np.float64)
    assert np.max(np.abs(rec / erfc(x) - 1.0)) < 5e-7


def _coeffs64():
    txt = HDR.read_text()
    def const(name):
        return float.fromhex(re.search(name + r"\s*=\s*(-?0x[0-9a-fA-Fp.+-]+);", txt).group(1))
    xmax = float(re.search(r"kErfcx64XMax\s*=\s*([0-9.eE+-]+);", txt).group(1))
    deg = int(re.search(r"kErfcx64Degree\s*=\s*(\d+)", txt).group(1))
    body = txt[txt.index("kErfcx64Q[kErfcx64Degree + 1] = {"):]
    body = body[body.index("{") + 1:body.index("};")]
    vals = [float.fromhex(m) for m in re.findall(r"(-?0x[0-9a-fA-Fp.+-]+),", body)]
    assert len(vals) == deg + 1
    return xmax, const("kErfcx64C"), const("kErfcx64InvH"), np.array(vals)


def _eval_fp64(x):
    _, c, inv_h, q = _coeffs64()
    t = 1.0 / (1.0 + 0.5 * x)
    u = (t - c) * inv_h
    acc = np.full_like(x, q[-1])
    for v in q[-2::-1]:
        acc = acc * u + v
    return acc * t


def test_fp64_fit_covers_its_range_to_near_double_precision():
    xmax, c, inv_h, q = _coeffs64()
    # the centred variable spans [-1, 1] over x in [0, xmax]
    assert abs((1.0 - c) * inv_h - 1.0) < 1e-12
    assert abs((1.0 / (1.0 + 0.5 * xmax) - c) * inv_h + 1.0) < 1e-12
    x = np.linspace(0.0, xmax, 400001)
    assert np.max(np.abs(_eval_fp64(x) / erfcx(x) - 1.0)) < 2e-14


def test_fp64_erfc_reconstruction():
    x = np.linspace(0.05, 6.0, 100001)
    rec = np.exp(-x * x) * _eval_fp64(x)
    assert np.max(np.abs(rec / erfc(x) - 1.0)) < 1e-13


def _gauss_fp64_split(r2, alpha, degree=13):
    """exp(-alpha r^2) as the FP64 pair loop forms it: a = -alpha log2(e) r^2,
    n = rint(a), f = a - n, 2^f by its Taylor series in f ln 2 to `degree`
    (coefficients (ln 2)^k / k! built by repeated multiplication)."""
    a = (-alpha * 1.44269504088896340735992468100189214) * r2
    n = np.rint(a)
    f = a - n
    c = [1.0]
    for k in range(1, degree + 1):
        c.append(c[-1] * 0.69314718055994530941723212145817657 / k)
    acc = np.full_like(f, c[degree])
    for k in range(degree - 1, -1, -1):
        acc = acc * f + c[k]
    return np.ldexp(acc, n.astype(np.int64))


def test_fp64_gaussian_split_matches_exp():
    # alpha r^2 over the range the FP64 fit serves (sqrt(alpha) r <= 8)
    for alpha in (0.5, 0.7, 4.0):
        r2 = np.linspace(0.0, 64.0 / alpha, 200001)
        got = _gauss_fp64_split(r2, alpha)
        ref = np.exp(-alpha * r2)
        assert np.max(np.abs(got / ref - 1.0)) < 2e-14
    # degree 13 is what the truncation bound asks for; one term fewer is visibly worse
    f = np.linspace(-0.5, 0.5, 10001)
    r2 = -f / (0.7 * 1.44269504088896340735992468100189214)
    assert np.max(np.abs(_gauss_fp64_split(r2, 0.7) / 2.0 ** f - 1.0)) < 1e-15
    assert np.max(np.abs(_gauss_fp64_split(r2, 0.7, degree=11) / 2.0 ** f - 1.0)) > 1e-15
