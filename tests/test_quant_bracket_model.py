"""CPU model of the e4m3 quantiser's reciprocal path
(paper_1304_7053_amd/csrc/quant.hip): the kernel multiplies by a reciprocal
of the scale s that is within 1 ulp of 1/s, brackets the product qa by
lo, hi = qa -+ |qa| 2^-20 (one rounding each) and keeps the code of lo when
lo and hi encode alike; otherwise the wave divides.  The claim checked here:
whenever the codes of lo and hi agree they equal the code of the correctly
rounded quotient fl(v / s), for every reciprocal within 1 ulp of 1/s, on
random values and on values built to put v / s on, and a few ulps either
side of, every e4m3 rounding boundary (normal and subnormal range, both
signs).  The encoder is the oracle's (round to nearest even, saturating)."""
import numpy as np

import oracle

F32 = np.float32


def _code(x):
    return oracle.encode_e4m3(float(x))


def _bracket(qa):
    q = np.float64(qa)
    d = abs(q) * 2.0 ** -20
    return F32(q - d), F32(q + d)          # exact in binary64, one rounding to binary32


def _recips(s):
    r0 = F32(1.0) / s
    return (r0, np.nextafter(r0, F32(np.inf)), np.nextafter(r0, F32(0)))


def _boundaries():
    """Rounding boundaries of e4m3: midpoints between neighbouring codes."""
    vals = sorted({oracle.decode(c, "e4m3") for c in range(0x7F)} - {float("nan")})
    vals = [v for v in vals if v == v]
    return [(a + b) / 2 for a, b in zip(vals, vals[1:])]


def test_bracket_keeps_exact_codes():
    g = np.random.default_rng(13047053)
    mids = _boundaries()
    assert len(mids) == 126 and mids[0] == 2.0 ** -10 and mids[-1] == 432.0
    scales = [F32(1.0), F32(3.0), F32(448.0) / F32(448.0) * F32(0.7), F32(2.0 ** -90), F32(2.0 ** 90)]
    scales += [F32(x) for x in g.uniform(0.5, 2.0, size=6) * 2.0 ** g.integers(-60, 60, size=6)]
    agreed = straddled = 0
    for s in scales:
        vs = []
        for m in mids:
            for sign in (1.0, -1.0):
                v = F32(sign * m * float(s))
                for k in range(-3, 4):             # a few ulps either side of the boundary
                    vs.append(v)
                    v = np.nextafter(v, F32(np.inf))
        vs += [F32(x) for x in g.standard_normal(400) * float(s) * 100]
        for v in vs:
            exact = _code(F32(v) / s)
            for r in _recips(s):
                lo, hi = _bracket(F32(v) * r)
                cl = _code(lo)
                if cl == _code(hi):
                    agreed += 1
                    assert cl == exact, (float(s), float(v), float(r))
                else:
                    straddled += 1
    assert agreed > 10000 and straddled > 1000      # both branches of the kernel are modelled


def test_random_values_rarely_take_the_division():
    """Normal inputs scaled by their absmax: the bracket straddles a boundary
    for about one element in 65,000 (width 2^-19 against an e4m3 spacing of 2^-3
    relative), so a wave of up to 1,024 elements rarely divides."""
    g = np.random.default_rng(7)
    n = 20000
    x = g.standard_normal(n).astype(F32)
    s = F32(np.max(np.abs(x))) / F32(448.0)
    r = F32(1.0) / s
    slow = 0
    for v in x:
        lo, hi = _bracket(v * r)
        slow += _code(lo) != _code(hi)
    assert slow <= 5, slow
