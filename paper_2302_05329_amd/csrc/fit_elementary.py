"""Fit the polynomial coefficients of the FP64 elementary functions used by the kernels.

Method: Chebyshev interpolation (near-minimax) of the reduced function in 60-digit
arithmetic with mpmath, coefficients rounded to double, then the worst error of the
double-precision Horner evaluation measured against mpmath on a dense grid.

  sin(r) = r + r^3 S(r^2),         |r| <= pi/4 (+ margin)
  cos(r) = 1 - r^2/2 + r^4 C(r^2), |r| <= pi/4 (+ margin)
  atan(t) = t + t^3 A(t^2),        0 <= t <= tan(pi/12) (+ margin)
  exp(r) = 1 + r + r^2 E(r),       |r| <= ln(2)/2 (+ margin)

Run: python paper_2302_05329_amd/csrc/fit_elementary.py  (prints a C++ header fragment)
"""
import mpmath as mp
import numpy as np

mp.mp.dps = 60


def cheb_fit(g, a, b, deg):
    """Chebyshev interpolant of g on [a, b] of degree deg, returned as monomial coefficients
    (in the variable itself), computed exactly in mpmath."""
    n = deg + 1
    nodes = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n) for k in range(n)]
    xs = [(a + b) / 2 + (b - a) / 2 * t for t in nodes]
    ys = [g(x) for x in xs]
    # solve the Vandermonde system exactly in mpmath
    A = mp.matrix([[x**j for j in range(n)] for x in xs])
    c = mp.lu_solve(A, mp.matrix(ys))
    return [c[j] for j in range(n)]


def horner(cs, z):
    acc = np.float64(cs[-1])
    for c in reversed(cs[:-1]):
        acc = np.float64(acc) * z + np.float64(c)
    return acc


def fit_all():
    out = {}
    pi4 = mp.pi / 4 * (1 + mp.mpf("1e-6"))
    # sin: S(z) = (sin(sqrt z) - sqrt z) / z^(3/2)
    gS = lambda z: (mp.sin(mp.sqrt(z)) - mp.sqrt(z)) / z ** mp.mpf(1.5) if abs(z) > mp.mpf("1e-40") else mp.mpf(-1) / 6
    out["sin"] = cheb_fit(gS, mp.mpf(0), pi4**2, 6)
    gC = lambda z: (mp.cos(mp.sqrt(z)) - 1 + z / 2) / z**2 if abs(z) > mp.mpf("1e-40") else mp.mpf(1) / 24
    out["cos"] = cheb_fit(gC, mp.mpf(0), pi4**2, 6)
    t12 = mp.tan(mp.pi / 12) * (1 + mp.mpf("1e-6"))
    gA = lambda z: (mp.atan(mp.sqrt(z)) - mp.sqrt(z)) / z ** mp.mpf(1.5) if abs(z) > mp.mpf("1e-40") else mp.mpf(-1) / 3
    out["atan"] = cheb_fit(gA, mp.mpf(0), t12**2, 10)
    l2 = mp.log(2) / 2 * (1 + mp.mpf("1e-6"))
    gE = lambda r: (mp.exp(r) - 1 - r) / r**2 if abs(r) > mp.mpf("1e-25") else mp.mpf(1) / 2 + r / 6
    out["exp"] = cheb_fit(gE, -l2, l2, 10)
    return out


def check(out):
    rng = np.random.default_rng(1)
    res = {}
    # sin / cos on the reduced interval
    r = np.linspace(-np.pi / 4, np.pi / 4, 20001)
    z = r * r
    s = r + r * z * horner([float(c) for c in out["sin"]], z)
    c = 1 - z / 2 + z * z * horner([float(c) for c in out["cos"]], z)
    es = max(abs(float(mp.sin(mp.mpf(x))) - y) for x, y in zip(r[::7], s[::7]))
    ec = max(abs(float(mp.cos(mp.mpf(x))) - y) for x, y in zip(r[::7], c[::7]))
    res["sin_abs"], res["cos_abs"] = es, ec
    t = np.linspace(0, np.tan(np.pi / 12), 20001)
    a = t + t * t * t * horner([float(c) for c in out["atan"]], t * t)
    res["atan_rel"] = max(abs(float(mp.atan(mp.mpf(x))) - y) / max(float(mp.atan(mp.mpf(x))), 1e-300)
                          for x, y in zip(t[1::7], a[1::7]))
    x = np.linspace(-np.log(2) / 2, np.log(2) / 2, 20001)
    e = 1 + x + x * x * horner([float(c) for c in out["exp"]], x)
    res["exp_rel"] = max(abs(float(mp.exp(mp.mpf(v))) - y) / float(mp.exp(mp.mpf(v))) for v, y in zip(x[::7], e[::7]))
    return res


if __name__ == "__main__":
    out = fit_all()
    for k, cs in out.items():
        print(f"// {k}: {len(cs)} coefficients, lowest order first")
        print("{" + ", ".join(mp.nstr(c, 20, min_fixed=-1, max_fixed=-1) for c in cs) + "}")
    print("// max errors:", check(out))
