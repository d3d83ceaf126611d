"""Minimax polynomial for e^r on the reduced range of the leapfrog's exponential.

The trajectory kernel evaluates e^{-h} as 2^n * P(r) with n = rint(x / ln 2) and
r = x - n ln 2 (|r| <= ln2/2).  This script computes P by the Remez exchange
algorithm (relative error, 40-digit arithmetic), rounds the coefficients to
FP64, and reports the worst relative error of the rounded polynomial on a
dense grid.  Its output is pasted into rsv_exp.h; rerun to check or change
the degree:  python paper_1603_08114_amd/csrc/gen_exp_poly.py [degree]
"""
import sys

import mpmath as mp

mp.mp.dps = 40


def remez(deg, a, iters=30):
    n = deg + 2
    # Chebyshev extrema as the starting reference
    xs = [a * mp.cos(mp.pi * (n - 1 - i) / (n - 1)) for i in range(n)]
    coef = None
    for _ in range(iters):
        # solve sum_j c_j x_i^j + (-1)^i E e^{x_i} = e^{x_i}
        A = mp.matrix(n, n)
        b = mp.matrix(n, 1)
        for i, x in enumerate(xs):
            for j in range(deg + 1):
                A[i, j] = x ** j
            A[i, deg + 1] = (-1) ** i * mp.e ** x
            b[i] = mp.e ** x
        sol = mp.lu_solve(A, b)
        coef = [sol[j] for j in range(deg + 1)]
        err = lambda x: (mp.polyval(coef[::-1], x) - mp.e ** x) / mp.e ** x
        # new reference: extrema of the error between sign changes
        grid = [-a + 2 * a * k / 4000 for k in range(4001)]
        vals = [err(x) for x in grid]
        ext = [grid[0]]
        for k in range(1, len(grid) - 1):
            if (vals[k] - vals[k - 1]) * (vals[k + 1] - vals[k]) <= 0:
                ext.append(mp.findroot(lambda x: mp.diff(err, x), grid[k]))
        ext.append(grid[-1])
        ext = sorted(ext, key=lambda x: float(x))
        if len(ext) >= n:
            # keep n points with alternating sign and largest magnitude
            picked = [ext[0]]
            for x in ext[1:]:
                if mp.sign(err(x)) == mp.sign(err(picked[-1])):
                    if abs(err(x)) > abs(err(picked[-1])):
                        picked[-1] = x
                else:
                    picked.append(x)
            if len(picked) >= n:
                xs = picked[:n] if abs(err(picked[0])) >= abs(err(picked[-1])) else picked[-n:]
    return coef


def main():
    deg = int(sys.argv[1]) if len(sys.argv) > 1 else 10
    a = mp.log(2) / 2 * mp.mpf("1.0001")
    coef = remez(deg, a)
    c64 = [float(c) for c in coef]
    worst = mp.mpf(0)
    for k in range(20001):
        x = -a + 2 * a * k / 20000
        p = mp.mpf(0)
        for c in reversed(c64):  # Horner in the rounded coefficients
            p = p * x + mp.mpf(c)
        worst = max(worst, abs((p - mp.e ** x) / mp.e ** x))
    print(f"degree {deg}: worst relative error of rounded polynomial {mp.nstr(worst, 5)} "
          f"({mp.nstr(worst / mp.mpf(2) ** -53, 4)} half-ulps)")
    for j, c in enumerate(c64):
        print(f"    {c!r},  // r^{j}")


if __name__ == "__main__":
    main()
