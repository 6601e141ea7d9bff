"""Coefficients of the FP64 base-2 exponential in model.h (kExp2Coef).

The degree-11 polynomial p minimising max |p(f) - 2^f| / 2^f over
f in [-1/2, 1/2] (Remez exchange in 50-digit arithmetic, started from the
Chebyshev interpolant), printed as C99 hex doubles with the relative error of
the coefficients as rounded to double (exact arithmetic, 20,001-point grid).
Run with `python gen_exp2_coef.py`; needs mpmath.
"""
import mpmath as mp

mp.mp.dps = 50
DEG = 11
LO, HI = mp.mpf(-0.5), mp.mpf(0.5)


def rel_err(c, x):
    return (mp.polyval(c[::-1], x) - mp.power(2, x)) / mp.power(2, x)


def remez(n, iters=10):
    # reference points: Chebyshev extrema of degree n + 1
    xs = [(LO + HI) / 2 - (HI - LO) / 2 * mp.cos(mp.pi * k / (n + 1)) for k in range(n + 2)]
    grid = [LO + (HI - LO) * k / 4000 for k in range(4001)]
    c = None
    for _ in range(iters):
        # p(x_i) - 2^x_i = (-1)^i E 2^x_i, i = 0..n+1: linear in (c, E)
        M = mp.matrix(n + 2, n + 2)
        rhs = mp.matrix(n + 2, 1)
        for i, x in enumerate(xs):
            for j in range(n + 1):
                M[i, j] = x ** j
            M[i, n + 1] = (-1) ** i * mp.power(2, x)
            rhs[i] = mp.power(2, x)
        sol = mp.lu_solve(M, rhs)
        c = [sol[j] for j in range(n + 1)]
        vals = [rel_err(c, x) for x in grid]
        ext = [grid[0]]
        ext += [grid[k] for k in range(1, len(grid) - 1)
                if (vals[k] - vals[k - 1]) * (vals[k + 1] - vals[k]) <= 0]
        ext.append(grid[-1])
        if len(ext) != n + 2:
            break
        xs = ext
    return c


def main():
    c = remez(DEG)
    cd = [float(x) for x in c]
    worst = max(abs(rel_err([mp.mpf(x) for x in cd], LO + (HI - LO) * k / 20000))
                for k in range(20001))
    print(f"// degree {DEG}, relative error {mp.nstr(worst, 3)} with double coefficients")
    for x in cd:
        print(f"  {x.hex()},")


if __name__ == "__main__":
    main()
