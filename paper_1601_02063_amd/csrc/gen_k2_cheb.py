"""Generates the Chebyshev coefficients used by bessel_k2() for x > 2.

f(t) = sqrt(x) e^x K_2(x) with t = 2/x in (0, 1] is smooth, f(0) = sqrt(pi/2)
(the leading term of the large-x expansion of K_2). It is interpolated at the
23 Chebyshev points of s = 2t - 1 with mpmath at 40 digits; the coefficients
c_j of f = sum_j c_j T_j(s) decay to ~1e-17 at j = 22. Prints the C++ array.
Run: python gen_k2_cheb.py   (needs mpmath)
"""
import mpmath as mp

mp.mp.dps = 40
N = 22


def f(t):
    x = 2 / t
    return mp.sqrt(x) * mp.e ** x * mp.besselk(2, x)


theta = [mp.pi * (k + mp.mpf(1) / 2) / (N + 1) for k in range(N + 1)]
vals = [f((1 + mp.cos(th)) / 2) for th in theta]
coef = [2 * sum(v * mp.cos(j * th) for v, th in zip(vals, theta)) / (N + 1) for j in range(N + 1)]
coef[0] /= 2
worst = 0
for i in range(1, 2001):
    t = mp.mpf(i) / 2000
    s = 2 * t - 1
    approx = sum(c * mp.chebyt(j, s) for j, c in enumerate(coef))
    worst = max(worst, abs(approx / f(t) - 1))
print(f"// max relative error of the expansion on t in (0, 1]: {mp.nstr(worst, 3)}")
print("constexpr double kK2Cheb[%d] = {" % (N + 1))
for j, c in enumerate(coef):
    print(f"    {mp.nstr(c, 17, min_fixed=1, max_fixed=0)},")
print("};")
