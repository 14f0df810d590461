"""The FP32 sinc polynomial of the HIP kernels (the sinc PSF, paper Sec. II,
the PSF paragraph) against numpy's sinc: the constants are read from the
kernel header and evaluated in FP32 exactly as the kernels do (y = (pi t)^2,
Horner with fused multiply-adds), over the main lobe |t| <= 1."""
import pathlib
import re

import numpy as np

HDR = pathlib.Path(__file__).resolve().parents[1] / "paper_1611_07289_amd" / "csrc" / "pvr_internal.h"


def _float_poly():
    src = HDR.read_text()
    body = src[src.index("sinc_poly<float>(float t) {"):]
    body = body[:body.index("\n}\n")]
    pi = float(re.search(r"const float y = \(([0-9.]+)f \* t\)", body).group(1))
    first = float(re.search(r"float s = ([-+0-9.eE]+)f;", body).group(1))
    rest = [float(v) for v in re.findall(r"fmaf\(s, y, ([-+0-9.eE]+)f\)", body)]
    return pi, [first] + rest  # highest degree first


def _fma32(a, b, c):
    # the hardware FMA rounds once; here the FP64 product of two FP32 values
    # is exact and the FP64 sum rounds to FP32 (the double rounding differs
    # from one rounding only in rare ties, by one FP32 unit at most)
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def test_fp32_sinc_polynomial_matches_numpy():
    pi, coefs = _float_poly()
    assert len(coefs) >= 6
    t = np.linspace(-1.0, 1.0, 400_001).astype(np.float32)
    p32 = np.float32(pi)
    y = (p32 * t) * (p32 * t)
    s = np.full_like(y, np.float32(coefs[0]))
    for c in coefs[1:]:
        s = _fma32(s, y, np.full_like(y, np.float32(c)))
    err = np.abs(s.astype(np.float64) - np.sinc(t.astype(np.float64)))
    # FP32 rounding of values up to 1 over a dozen operations
    assert err.max() < 3e-7, err.max()
    # exact at the centre, and the lobe edge within the same bound of 0
    assert s[len(s) // 2] == np.float32(1.0)
    assert abs(float(s[0])) < 3e-7 and abs(float(s[-1])) < 3e-7
