"""Generates the polynomial coefficients of the light elementary functions
(kgrt_device.hpp: sincos_bounded, fm::expm1_reduced, fm::log).

Each function, after its argument reduction, is written as the first terms of
its Taylor series plus a remainder polynomial R fitted by Chebyshev
interpolation (mpmath.chebyfit, near-minimax, 50 digits):
  sin x = x + x^3 S(x^2),        |x| <= pi/4,         S degree 5;
  cos x = 1 - x^2/2 + x^4 C(x^2), |x| <= pi/4,        C degree 5;
  e^r - 1 = r + r^2/2 + r^3 E(r), |r| <= ln(2)/2,     E degree 9;
  atanh f = f + f^3 A(f^2),      |f| <= 3 - 2 sqrt(2), A degree 6
(the log's reduced argument f = (m - 1)/(m + 1), m in [sqrt(1/2), sqrt(2))).
The truncated Taylor series of the same accuracy need 2, 2, 2 and 4 more
terms. Prints the C++ constants (highest power first) and, for each function,
the largest relative error with the coefficients rounded to double, in exact
arithmetic, in units of 2^-53: about 0.18, 0.011, 0.022 and 0.041.
Run: python gen_poly.py   (needs mpmath)
"""
import mpmath as mp

mp.mp.dps = 50
PIO4 = mp.pi / 4
RLN = mp.log(2) / 2
FMAX = 3 - 2 * mp.sqrt(2)


def remainder(exact, head, power):
    def g(u, exact=exact, head=head, power=power):
        return (exact(u) - head(u)) / u ** power
    return g


def fit(g, lo, hi, deg, at_zero):
    def safe(u):
        return at_zero if u == 0 else g(u)
    return [float(c) for c in mp.chebyfit(safe, [lo, hi], deg + 1)]


def horner(coeffs, u):
    p = mp.mpf(0)
    for c in coeffs:
        p = p * u + mp.mpf(c)
    return p


S = fit(lambda z: (mp.sin(mp.sqrt(z)) - mp.sqrt(z)) / mp.sqrt(z) ** 3, 0, PIO4 ** 2, 5, mp.mpf(-1) / 6)
C = fit(lambda z: (mp.cos(mp.sqrt(z)) - 1 + z / 2) / z ** 2, 0, PIO4 ** 2, 5, mp.mpf(1) / 24)
E = fit(lambda r: (mp.expm1(r) - r - r * r / 2) / r ** 3, -RLN, RLN, 9, mp.mpf(1) / 6)
A = fit(lambda s: (mp.atanh(mp.sqrt(s)) - mp.sqrt(s)) / mp.sqrt(s) ** 3, 0, FMAX ** 2, 6, mp.mpf(1) / 3)

err = {"sin": 0, "cos": 0, "expm1": 0, "atanh": 0}
for i in range(1, 4001):
    x = PIO4 * i / 4000
    z = x * x
    err["sin"] = max(err["sin"], abs((x + x ** 3 * horner(S, z)) / mp.sin(x) - 1))
    err["cos"] = max(err["cos"], abs((1 - z / 2 + z * z * horner(C, z)) / mp.cos(x) - 1))
    f = FMAX * i / 4000
    err["atanh"] = max(err["atanh"], abs((f + f ** 3 * horner(A, f * f)) / mp.atanh(f) - 1))
for i in range(-4000, 4001):
    r = RLN * i / 4000
    if r != 0:
        err["expm1"] = max(err["expm1"], abs((r + r * r / 2 + r ** 3 * horner(E, r)) / mp.expm1(r) - 1))
print("// max relative error in units of 2^-53: " +
      ", ".join(f"{k} {mp.nstr(v / mp.mpf(2) ** -53, 3)}" for k, v in err.items()))
for name, c in (("kSinPoly", S), ("kCosPoly", C), ("kExpm1Poly", E), ("kAtanhPoly", A)):
    print(f"constexpr double {name}[{len(c)}] = {{" + ", ".join(repr(v) for v in c) + "};")
