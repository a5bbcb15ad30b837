"""Generates the 32-point Gauss-Legendre rule on [0, 1] used by the surrogate's
crossing-radius polish (kgrt_mino.hpp): nodes t_k and weights w_k with
sum_k w_k f(t_k) = int_0^1 f(t) dt exactly for polynomials of degree <= 63.
Nodes are the roots of the Legendre polynomial P_32 mapped from [-1, 1],
found by mpmath at 40 digits. Prints the C++ arrays (the 16 nodes in
(0, 1/2) and their weights; the others are 1 - t_k with the same weights).
Run: python gen_gauss_legendre.py   (needs mpmath)
"""
import mpmath as mp

mp.mp.dps = 40
N = 32


def main():
    nodes = []
    for k in range(1, N // 2 + 1):
        x0 = mp.cos(mp.pi * (k - mp.mpf(1) / 4) / (N + mp.mpf(1) / 2))  # Tricomi's first guess
        x = mp.findroot(lambda z: mp.legendre(N, z), x0)
        dp = mp.diff(lambda z: mp.legendre(N, z), x)
        w = 2 / ((1 - x * x) * dp * dp)
        nodes.append(((1 - x) / 2, w / 2))  # map to [0, 1]: t = (1 - x)/2 in (0, 1/2)
    nodes.sort()
    print("constexpr double kGlT[16] = {" + ", ".join(mp.nstr(t, 17) for t, _ in nodes) + "};")
    print("constexpr double kGlW[16] = {" + ", ".join(mp.nstr(w, 17) for _, w in nodes) + "};")


if __name__ == "__main__":
    main()
