"""Coefficients of the float64 arctangent in mu3e_math.hpp (atan2_q1).

On |u| <= tan(pi/8), atan(u) = u + u^3 P(u^2) with P a polynomial of degree
9 in s = u^2.  P is the weighted least-squares fit (weights making the
residual the relative error of atan) of (atan(sqrt s) - sqrt s) / s^(3/2) on
Chebyshev nodes of [0, tan(pi/8)^2], in 60-digit arithmetic (mpmath).  The
fit's relative error of atan is below 4e-17 on the interval.

The float32 version (atan2f_full) uses the same fit with five terms
(fit(n=5), relative error below 1e-9).

Run: python atan_coeffs.py  (prints the coefficients and the error bound)
"""
import mpmath as mp

N_COEF = 10


def fit(n=N_COEF, dps=60):
    mp.mp.dps = dps
    a = mp.tan(mp.pi / 8)
    smax = a * a

    def target(s):
        u = mp.sqrt(s)
        return (mp.atan(u) - u) / (s * u)

    m = 4 * n + 40
    nodes = [smax / 2 * (1 - mp.cos(mp.pi * (k + 0.5) / m)) for k in range(m)]
    A = mp.matrix(m, n)
    b = mp.matrix(m, 1)
    for i, s in enumerate(nodes):
        u = mp.sqrt(s)
        w = u * s / mp.atan(u)
        for j in range(n):
            A[i, j] = w * s ** j
        b[i] = w * target(s)
    c = mp.lu_solve(A.T * A, A.T * b)
    err = mp.mpf(0)
    for k in range(1, 4001):
        s = smax * k / 4000
        u = mp.sqrt(s)
        p = sum(c[j] * s ** j for j in range(n))
        at = mp.atan(u)
        err = max(err, abs((u + u ** 3 * p - at) / at))
    return [c[j] for j in range(n)], err


if __name__ == "__main__":
    coef, err = fit()
    for c in coef:
        print(mp.nstr(c, 20, min_fixed=-30, max_fixed=30))
    print("max relative error of atan:", mp.nstr(err, 4))
