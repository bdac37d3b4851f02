"""Coefficients of the sin/cos polynomials in kt_device.h (sincos_shift and
sincos_theta): weighted minimax fits by the Remez exchange algorithm in
50-digit arithmetic (mpmath), printed as the doubles the kernel uses.

With x = d^2 (or u^2) the kernel evaluates
    sin d     = d - d x S(x),  S(x) = sum_k (-1)^k x^k / (2k+3)!   (series)
    cos d - 1 =   - x C(x),    C(x) = sum_k (-1)^k x^k / (2k+2)!
and replaces S and C by polynomials of lower degree that minimise the
largest error of the result over the range the kernel needs:
    staged shift, |d| <= 1/2:  S degree 4, weight x (relative error of sin d)
                               C degree 5, weight x (absolute error of cos d)
    full, |u| <= pi/2:         C degree 7, weight x (absolute error of cos u),
                               constant term held at 1/2 so that its
                               rounding adds no error
                               S degree 7, weight x^(3/2) (absolute error of sin u)
Taylor's series needs one (staged) or two (full) more terms for the same
accuracy.

It also fits the polynomials of exp_fast and log_fast (the q-metric's
powers f^q and D^(q(2+q))):
    e^t = 1 + t + t^2 G(t), |t| <= (ln 2)/2: G degree 9, weight t^2 / e^t
        (relative error of e^t); Taylor's series needs through t^13
    ln m = 2 s + 2 s x L(x), x = s^2, s = (m - 1)/(m + 1) for m in
        [1/sqrt 2, sqrt 2), L(x) = sum_k x^k / (2k + 3): L degree 6, weight x
        (relative error of ln m); the atanh series needs through s^21

    python paper_2202_00086_amd/csrc/minimax_coefs.py
"""
import mpmath as mp

mp.mp.dps = 50

FITS = (
    # name, function, weight, x range end, degree, fixed constant term
    ("shift_sin", "S", lambda x: x, mp.mpf(1) / 4, 4, None),
    ("shift_cos", "C", lambda x: x, mp.mpf(1) / 4, 5, None),
    ("theta_cos", "C", lambda x: x, (mp.pi / 2) ** 2, 7, mp.mpf(1) / 2),
    ("theta_sin", "S", lambda x: x * mp.sqrt(x), (mp.pi / 2) ** 2, 7, None),
)


def S(x):
    return mp.fsum((-1) ** k * x ** k / mp.factorial(2 * k + 3) for k in range(40))


def C(x):
    return mp.fsum((-1) ** k * x ** k / mp.factorial(2 * k + 2) for k in range(40))


def remez(f, w, b, n, grid=2000, iters=40):
    """Degree-n polynomial p minimising max |w(x) (p(x) - f(x))| on [0, b].
    Returns (coefficients low to high, the largest weighted error)."""
    m = n + 2
    xs = [b * (1 - mp.cos(mp.pi * i / (m - 1))) / 2 for i in range(m)]
    xs[0] = b * mp.mpf("1e-6")  # the weight vanishes at 0
    pts = [b * mp.mpf(k) / grid for k in range(1, grid + 1)]
    for _ in range(iters):
        A = mp.matrix(m, m)
        rhs = mp.matrix(m, 1)
        for i, x in enumerate(xs):
            for j in range(n + 1):
                A[i, j] = x ** j
            A[i, n + 1] = (-1) ** i / w(x)
            rhs[i] = f(x)
        sol = mp.lu_solve(A, rhs)
        c = [sol[j] for j in range(n + 1)]
        level = abs(sol[n + 1])
        err = [w(x) * (mp.polyval(c[::-1], x) - f(x)) for x in pts]
        # the largest error of each run of one sign
        ext, run = [], [0]
        for k in range(1, grid):
            if mp.sign(err[k]) == mp.sign(err[run[-1]]):
                run.append(k)
            else:
                ext.append(max(run, key=lambda i: abs(err[i])))
                run = [k]
        ext.append(max(run, key=lambda i: abs(err[i])))
        worst = max(abs(e) for e in err)
        if len(ext) < m:
            break
        while len(ext) > m:
            ext.pop(0 if abs(err[ext[0]]) < abs(err[ext[-1]]) else -1)
        xs = [pts[i] for i in ext]
        if worst - level < level * mp.mpf("1e-6"):
            break
    return c, worst


def remez_on(f, w, a, n):
    """remez on the symmetric interval [-a, a], returned as coefficients of
    the polynomial in the original variable (low to high)."""
    c, worst = remez(lambda y: f(y - a), lambda y: w(y - a), 2 * a, n)
    # p(t) = sum_k c_k (t + a)^k, expanded in powers of t
    out = [mp.mpf(0)] * (n + 1)
    for k, ck in enumerate(c):
        for j in range(k + 1):
            out[j] += ck * mp.binomial(k, j) * a ** (k - j)
    return out, worst


def G(t):
    # (e^t - e^0 - t) / t^2 from its series, accurate at and near t = 0
    return mp.fsum(t ** k / mp.factorial(k + 2) for k in range(60))


def L(x):
    return mp.fsum(x ** k / (2 * k + 3) for k in range(80))


def fit_all():
    out = {}
    for name, fn, w, b, n, lead in FITS:
        f = S if fn == "S" else C
        if lead is None:
            c, worst = remez(f, w, b, n)
        else:
            # f = lead + x g: fit g with degree n - 1 and weight x w(x)
            c, worst = remez(lambda x: (f(x) - lead) / x, lambda x: x * w(x), b, n - 1)
            c = [lead] + c
        out[name] = ([float(v) for v in c], float(worst))
    # exp: the weight t^2 / e^t vanishes at t = 0, inside the interval
    half_ln2 = mp.log(2) / 2
    c, worst = remez_on(G, lambda t: t * t / mp.exp(t) + mp.mpf("1e-40"), half_ln2, 9)
    out["exp_g"] = ([float(v) for v in c], float(worst))
    smax = (mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)
    c, worst = remez(L, lambda x: x, smax ** 2, 6)
    out["log_l"] = ([float(v) for v in c], float(worst))
    return out


if __name__ == "__main__":
    for name, (c, worst) in fit_all().items():
        print(f"{name}: max weighted error {worst:.3e}")
        for v in c:
            print(f"    {v!r}")
