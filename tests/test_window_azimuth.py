"""The build window's azimuth polynomial (atan2_poly in kf_build.hip): its coefficients, read from the source and
evaluated in single precision as the kernel does (fused multiply-adds, reciprocal within one ulp), stay within
the widening the window's phi interval gets, against atan2 in double precision (the binning's definition of a
hit's azimuth for the directionally projective bins of Sec. 3)."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1705_02876_amd", "csrc", "kf_build.hip")


def _poly_source():
    src = open(SRC).read()
    body = src[src.index("float atan2_poly(float y, float x)"):]
    return body[:body.index("\n}\n")]


def _coefficients(body):
    first = float(re.search(r"float r = ([-0-9.e]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"r = fmaf\(r, q, ([-0-9.e]+)f\);", body)]
    return [first] + rest


def _widening():
    src = open(SRC).read()
    m = re.search(r"fmaf\(sphi \* __builtin_amdgcn_rsqf\(fmaf\(-sphi, sphi, 1\.f\)\), ([0-9.]+)f, ([0-9.e-]+)f\)", src)
    return float(m.group(1)) - 1.0, float(m.group(2))


def _atan2_poly(y, x, coef, rcp_ulps):
    f32 = np.float32
    ax, ay = np.abs(x), np.abs(y)
    mx, mn = np.maximum(ax, ay), np.minimum(ax, ay)
    rc = (f32(1) / mx).astype(f32)
    for _ in range(abs(rcp_ulps)):
        rc = np.nextafter(rc, f32(np.inf) if rcp_ulps > 0 else f32(-np.inf))
    a = (mn * rc).astype(f32)
    q = (a * a).astype(f32)
    r = np.full(x.shape, f32(coef[0]))
    for c in coef[1:]:
        r = (r.astype(np.float64) * q.astype(np.float64) + np.float64(f32(c))).astype(f32)  # one rounding: fma
    r = (r * a).astype(f32)
    r = np.where(ay > ax, (f32(1.57079633) - r).astype(f32), r)
    r = np.where(x < 0, (f32(3.14159265) - r).astype(f32), r)
    return np.copysign(r, y)


def test_atan2_poly_error_within_the_window_widening():
    body = _poly_source()
    coef = _coefficients(body)
    assert len(coef) == 7
    rng = np.random.default_rng(7)
    n = 400_000
    ang = np.concatenate([rng.uniform(-np.pi, np.pi, n),
                          np.arange(-8, 9) * (np.pi / 4)])  # the axes and the diagonals
    rad = np.concatenate([rng.uniform(1.0, 120.0, n), np.full(17, 30.0)])
    x = (rad * np.cos(ang)).astype(np.float32)
    y = (rad * np.sin(ang)).astype(np.float32)
    exact = np.arctan2(y.astype(np.float64), x.astype(np.float64))
    worst = 0.0
    for ulps in (-1, 0, 1):
        got = _atan2_poly(y, x, coef, ulps).astype(np.float64)
        d = np.abs(got - exact)
        d = np.minimum(d, 2 * np.pi - d)  # -pi and pi are the same azimuth
        worst = max(worst, float(d.max()))
    assert worst < 1e-6
    rel, absolute = _widening()
    assert rel >= 1e-6
    # the absolute widening covers the polynomial's error with room for the single-precision bin arithmetic
    assert absolute >= 4 * worst


def test_tangent_bounds_asin_from_above():
    s = np.linspace(0.0, 0.9, 100_001)
    assert np.all(s / np.sqrt(1 - s * s) >= np.arcsin(s))
