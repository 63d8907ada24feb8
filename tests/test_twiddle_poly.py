"""Accuracy of the FP32 twiddle used by the FP32 DFT kernels (cisphase in
k_dft.hip): the FP64 phase 4 a m in quarter turns splits into the quadrant
j = rint(u) and the exact remainder r in [-1/2, 1/2]; cos and sin of (pi/2) r
come from two polynomials in r^2 whose float coefficients are read here from
the kernel source, evaluated with single roundings per fused multiply-add,
then rotated by j quarter turns.

Checked in units in the last place of the float32 value over random (a, m)
pairs: against FP64 cos and sin of the float32 remainder (either output may
come from either polynomial; within 1.05 ulp, measured 1.01), and against
FP64 cos and sin of the FP64 phase, where rounding the remainder to float32
adds up to half an ulp (within 1.35 ulp, measured 1.32); and the phases k/8
turn, whose remainders are 0 and +-1/2, in every quadrant."""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1703_02920_amd", "csrc", "k_dft.hip")


def _coefficients():
    src = open(SRC).read()
    body = src[src.index("void cisphase(double a, int m, float &c, float &s)"):]
    body = body[:body.index("\n}\n")]
    lits = re.findall(r"(-?0x1\.[0-9a-f]+p[+-]\d+)f", body)
    assert len(lits) == 9, lits
    return [np.float32(float.fromhex(x)) for x in lits]


def _fma(a, b, c):
    """float32 fused multiply-add: the product is exact in extended
    precision, then one sum and the rounding to float32."""
    a, b, c = (np.asarray(x, np.float32).astype(np.longdouble) for x in (a, b, c))
    return (a * b + c).astype(np.float32)


def _cisphase(a, m):
    s7, s5, s3, s1lo, s1, c8, c6, c4, c2 = _coefficients()
    u = a * (4.0 * m)
    jd = np.rint(u)
    r = (u - jd).astype(np.float32)
    j = jd.astype(np.int64)
    z = (r * r).astype(np.float32)
    q = _fma(z, s7, s5)
    q = _fma(z, q, s3)
    q = _fma(z, q, s1lo)
    sn = _fma(r, s1, (r * q).astype(np.float32))
    p = _fma(z, c8, c6)
    p = _fma(z, p, c4)
    p = _fma(z, p, c2)
    cs = _fma(z, p, np.float32(1.0))
    odd = (j & 1) != 0
    cc = np.where(odd, sn, cs)
    ss = np.where(odd, cs, sn)
    c = np.where(((j + 1) & 2) != 0, -cc, cc)
    s = np.where((j & 2) != 0, -ss, ss)
    return c, s, u


def _reference(u, r=None):
    # FP64 cos, sin of the phase u quarter turns (remainder exact), or of the
    # quadrant of u with the given remainder r
    jd = np.rint(u)
    th = (np.pi / 2) * ((u - jd) if r is None else r.astype(np.float64))
    j = jd.astype(np.int64) & 3
    c0, s0 = np.cos(th), np.sin(th)
    c = np.select([j == 0, j == 1, j == 2, j == 3], [c0, -s0, -c0, s0])
    s = np.select([j == 0, j == 1, j == 2, j == 3], [s0, c0, -s0, -c0])
    return c, s


def _ulps(x, ref):
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    return np.abs(x.astype(np.float64) - ref) / ulp


def test_cisphase_within_one_ulp_of_fp64():
    rng = np.random.default_rng(1)
    a = rng.uniform(-0.75, 0.75, 400_000)
    m = rng.integers(-2048, 2049, 400_000)
    c, s, u = _cisphase(a, m)
    r = (u - np.rint(u)).astype(np.float32)
    for ref_r, bs, bc in ((r, 1.05, 1.05), (None, 1.35, 1.35)):
        rc, rs = _reference(u, ref_r)
        ok = np.abs(rs) > 1e-30
        es, ec = _ulps(s[ok], rs[ok]), _ulps(c, rc)
        assert es.max() < bs and ec.max() < bc, (ref_r is None, es.max(), ec.max())
        assert es.mean() < 0.35 and ec.mean() < 0.35


def test_cisphase_quadrants_and_special_remainders():
    # phases of exactly k/8 turns: remainder 0 or +-1/2, every quadrant and sign
    for k in range(-16, 17):
        a = np.array([k / 8.0])
        c, s, _ = _cisphase(a, np.array([1]))
        th = 2 * np.pi * k / 8.0
        assert abs(float(c[0]) - np.cos(th)) < 1e-7 and abs(float(s[0]) - np.sin(th)) < 1e-7, k
    # a m = 0: exactly (1, 0)
    c, s, _ = _cisphase(np.array([0.3]), np.array([0]))
    assert float(c[0]) == 1.0 and float(s[0]) == 0.0
