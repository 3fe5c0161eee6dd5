"""The generated constant tables the kernels read (host checks, no GPU).

* the (sin, cos) table: entry j is (sin, cos)(j pi/512) correctly rounded (within 1e-60 at the
  exact zeros), and the two parts of pi/512 used by the argument reduction sum to pi/512
  within 2e-34;
* the arc tangent table: entry 0 is (0, 0); entry j >= 1 is the midpoint c of bucket j (16 per
  octave of |u| from 2^-10 to 2^10, exactly representable) and atan c correctly rounded; the
  kernels' index (bits 16-30 of the high word of |u|, minus the base, clamped) selects the bucket
  that holds |u|, so the reduced argument t = (|u| - c)/(1 + |u| c) stays within 1/64; and the
  table construction, emulated in FP64 on the host with the 3-term polynomial, is within 1.5 ulp
  of a 40-digit arc tangent (the GPU's own bound, 2 ulp, is tested by test_gpu_elementary).
"""
import os
import re

import mpmath as mp
import numpy as np

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2302_05329_amd", "csrc")
mp.mp.dps = 40


def _header(name):
    with open(os.path.join(CSRC, name)) as f:
        return f.read()


def _pairs(text):
    vals = re.findall(r"^\s+([-+0-9.e]+), ([-+0-9.e]+),\s*$", text, re.M)
    return np.array([[float(a), float(b)] for a, b in vals])


def _const(text, name):
    return float(re.search(rf"constexpr (?:double|int) {name} = ([-+0-9.e]+);", text).group(1))


def test_sincos_table_is_correctly_rounded():
    t = _header("pd_sincos_table.h")
    tab = _pairs(t)
    n = int(_const(t, "kSinCosN"))
    assert tab.shape == (n, 2) and n == 1024
    with mp.workdps(60):
        for j in range(n):
            a = mp.mpf(j) * 2 * mp.pi / n
            for got, exact in ((tab[j, 0], mp.sin(a)), (tab[j, 1], mp.cos(a))):
                # correctly rounded (half an ulp), or within 1e-60 where the value is an exact zero
                # (a 60-digit pi leaves a residue of that size there)
                err = abs(mp.mpf(got) - exact)
                assert err <= mp.mpf(np.spacing(abs(float(exact)))) / 2 or err < mp.mpf("1e-60"), j
    step = 2 * mp.pi / n
    p1, p2 = _const(t, "kPiStep_1"), _const(t, "kPiStep_2")
    assert p1 == float(step)
    assert abs(mp.mpf(p1) + mp.mpf(p2) - step) < mp.mpf("2e-34")


def _atan_index(u, base, shift, n):
    hw = (np.abs(u).view(np.uint64) >> np.uint64(32)).astype(np.int64)
    return np.clip((hw >> shift) - base, 0, n - 1)


def test_atan_table_centres_and_values():
    t = _header("pd_atan_table.h")
    tab = _pairs(t)
    n = int(_const(t, "kAtanN"))
    assert tab.shape == (n, 2) and n == 1 + 20 * 16
    assert tab[0, 0] == 0.0 and tab[0, 1] == 0.0
    j = 1
    for e in range(-10, 10):
        for m in range(16):
            c = mp.ldexp(1 + (mp.mpf(m) + mp.mpf(1) / 2) / 16, e)
            assert mp.mpf(tab[j, 0]) == c, j
            assert tab[j, 1] == float(mp.atan(c)), j
            j += 1


def test_atan_index_selects_the_bucket_and_bounds_the_reduced_argument():
    t = _header("pd_atan_table.h")
    tab = _pairs(t)
    n, base, shift = int(_const(t, "kAtanN")), int(_const(t, "kAtanBase")), int(_const(t, "kAtanShift"))
    rng = np.random.default_rng(3)
    edges = np.array([2.0 ** k * (1 + m / 16) for k in range(-11, 11) for m in range(16)])
    u = np.concatenate([rng.uniform(0, 3, 200000), 10 ** rng.uniform(-9, 9, 200000), edges,
                        np.nextafter(edges, 0), np.nextafter(edges, np.inf)])
    i = _atan_index(u, base, shift, n)
    c = tab[i, 0]
    inside = (u >= 2.0 ** -10) & (u < 2.0 ** 10)
    # inside the table's range the bucket [c (1 - 1/33), c (1 + 1/33)) holds u
    assert np.all(np.abs(u[inside] - c[inside]) <= c[inside] / 32 * (1 + 1e-15))
    assert np.all(c[u < 2.0 ** -10] == 0.0)
    red = (u - c) / (1 + u * c)
    assert np.max(np.abs(red)) <= 1 / 64


def test_atan_table_construction_within_1p5_ulp():
    t = _header("pd_atan_table.h")
    tab = _pairs(t)
    n, base, shift = int(_const(t, "kAtanN")), int(_const(t, "kAtanBase")), int(_const(t, "kAtanShift"))
    rng = np.random.default_rng(4)
    u = np.concatenate([rng.uniform(0, 1, 1500), rng.uniform(0, 50, 1500), 10 ** rng.uniform(-8, 8, 1500)])
    i = _atan_index(u, base, shift, n)
    c, atc = tab[i, 0], tab[i, 1]
    tq = (u - c) / (u * c + 1.0)
    z = tq * tq
    q = (-1.0 / 7.0 * z + 1.0 / 5.0) * z - 1.0 / 3.0
    r = atc + (tq * z * q + tq)
    exact = [mp.atan(mp.mpf(float(v))) for v in u]
    err = np.array([float(abs(mp.mpf(float(a)) - e)) for a, e in zip(r, exact)])
    ulp = np.spacing(np.array([float(e) for e in exact]))
    assert np.max(err / ulp) <= 1.5
