"""Oracle for the one-dimensional scale-adaptive filter (Section 3).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP path and
never imports it.

What is computed (Section 3, the projections s[m] and Proposition 3.1).  A signal is given
by its samples f[k]; every sample m carries its own scale a[m] > 0; the continuous model is
    f(x) = sum_k c[k] beta^{n1}(x - k),
with the model degree n1 in {-1, 0, 1, 2, 3}: n1 = -1 is the impulse model f(x) = sum_k f[k]
delta(x - k) that the two-dimensional filter uses (Section 7, phi = delta); for n1 = 0 and
n1 = 1 the interpolation filter b^{n1}[k] = beta^{n1}(k) is the unit impulse, so c = f and no
prefilter is needed; for n1 = 2, 3 the coefficients are c = f_ext * (b^{n1})^{-1} (Section 3:
the model interpolates the samples), the bounded solution on all of Z of
    sum_j b^{n1}[j] c[k - j] = f_ext[k],   b^{n1}[0] = 3/4, 2/3 and b^{n1}[+-1] = 1/8, 1/6.
The oracle solves these equations directly (a tridiagonal system, exact rationals) on a block
reaching PREFILTER_MARGIN samples past every coefficient it needs, with the block's two end
coefficients set to the extended samples there.  The bounded solution's deviation from that
closure dies off like |z|^distance, z = 2 sqrt2 - 3 or sqrt3 - 2 (the roots of the symmetric
filter), so over 64 samples the truncation changes the result by less than 1e-34 of max|f|.
The output is the projection onto the B-spline of degree n - 1 and scale a = a[m] centred
at m:
    s[m] = <f, beta_a^{n-1}(. - m)> = sum_k c_ext[k] K_a(m - k),
    K_a = beta^{n1} * beta_a^{n-1}   (both kernels are even),
where n >= 1 is the number of running sums of the fast algorithm (n = n2 + 1 in
Proposition 3.1) and c_ext extends the samples past the ends by the nearest end value
(clamp) or by zeros (for n1 >= 2: the samples are extended first, and the prefilter runs on
the extended sequence).

beta_a^N is the symmetric B-spline of degree N and scale a (eq. definition): the (N+1)-fold
convolution of the box 1/a on (-a/2, a/2].  Written in truncated powers
(y)_+^N (with (y)_+^0 = 1 for y > 0 and 0 otherwise, which gives the half-open box),
    beta_a^N(x) = 1/(a^{N+1} N!) sum_j (-1)^j C(N+1, j) (x + a(N+1)/2 - a j)_+^N,
and the convolution of two truncated powers is a truncated power,
    (. - p)_+^A * (. - q)_+^B = A! B! / (A+B+1)! (. - p - q)_+^{A+B+1},
so that, with D = n1 + n,
    K_a(x) = 1/(a^n D!) sum_{i=0}^{n1+1} sum_{j=0}^{n} (-1)^{i+j} C(n1+1, i) C(n, j)
                                                       (x + (n1+1)/2 + a n/2 - i - a j)_+^D.
a is a float32 (the filter's scale format), so every term is a rational number; the oracle
sums each output exactly in integers and rounds once (Python's int/Fraction arithmetic),
so its float64 result is the correctly rounded exact projection (for n1 >= 2, of the
projection with the prefilter's block truncated as above).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

MODELS = (-1, 0, 1, 2, 3)
BORDERS = ("clamp", "zero")
PREFILTER_MARGIN = 64


def _scale_parts(a) -> tuple[int, int]:
    """a (rounded to float32) as A / 2^q with integers A > 0, q >= 0."""
    num, den = float(np.float32(a)).as_integer_ratio()
    if num <= 0:
        raise ValueError("scales must be positive")
    q = den.bit_length() - 1
    return num, q


def _tpow(X: int, D: int) -> int:
    """(X)_+^D for an integer X (the step function for D = 0)."""
    if X <= 0:
        return 0
    return X ** D if D > 0 else 1


def kernel_numerators(xs, a, n: int, n1: int):
    """Exact K_a(x) for integer offsets x: returns (numerators, denominator) as Python ints.

    With a = A / 2^q, every truncated-power argument times 2^(q+1) is the integer
        X_ij = 2^(q+1) x + 2^q (n1 + 1 - 2i) + A (n - 2j),
    and K_a(x) = [sum_ij (-1)^(i+j) C(n1+1,i) C(n,j) (X_ij)_+^D] 2^(q n) / (2^((q+1) D) A^n D!).
    """
    if n < 1 or n1 not in MODELS:
        raise ValueError("order n >= 1 and model degree in {-1, 0, 1, 2, 3}")
    A, q = _scale_parts(a)
    D = n1 + n
    terms = [((-1) ** (i + j) * math.comb(n1 + 1, i) * math.comb(n, j),
              (1 << q) * (n1 + 1 - 2 * i) + A * (n - 2 * j))
             for i in range(n1 + 2) for j in range(n + 1)]
    nums = []
    for x in xs:
        base = int(x) << (q + 1)
        nums.append(sum(w * _tpow(base + s, D) for w, s in terms))
    den = (1 << ((q + 1) * D)) * A ** n * math.factorial(D)
    # the factor 2^(q n) of the numerator is moved into the denominator's exponent
    return nums, Fraction(den, 1 << (q * n))


def kernel_value(x, a, n: int, n1: int = -1) -> Fraction:
    """K_a(x) = (beta^{n1} * beta_a^{n-1})(x) exactly, for an integer x."""
    nums, den = kernel_numerators([x], a, n, n1)
    return Fraction(nums[0]) / den


def support_radius(a, n: int, n1: int) -> float:
    """K_a vanishes for |x| >= (n1 + 1)/2 + a n / 2."""
    return (n1 + 1) / 2 + float(np.float32(a)) * n / 2


def bspline_at_integer(k: int, N: int) -> Fraction:
    """beta^N(k), the centred unit-scale B-spline of degree N at an integer k, exactly
    (1/N! sum_j (-1)^j C(N+1, j) (k + (N+1)/2 - j)_+^N)."""
    acc = Fraction(0)
    for j in range(N + 2):
        y = Fraction(k) + Fraction(N + 1, 2) - j
        if y > 0:
            acc += (-1) ** j * math.comb(N + 1, j) * (y ** N if N > 0 else 1)
    return acc / math.factorial(N)


def coefficients(f, n1: int, border: str, lo: int, hi: int) -> list[Fraction]:
    """c[k] for k = lo .. hi-1: the model coefficients c = f_ext * (b^{n1})^{-1} (Section 3).

    For n1 <= 1 they are the extended samples.  For n1 = 2, 3 the equations
    b1 c[k-1] + b0 c[k] + b1 c[k+1] = f_ext[k] are solved on the block [lo - M, hi + M),
    M = PREFILTER_MARGIN, with the block's end coefficients set to f_ext there (the
    tridiagonal elimination, in exact rationals)."""
    if n1 <= 1:
        return [Fraction(float(_ext(f, k, border))) for k in range(lo, hi)]
    M = PREFILTER_MARGIN
    rhs = [Fraction(float(_ext(f, k, border))) for k in range(lo - M, hi + M)]
    return solve_block(rhs, n1)[M:M + (hi - lo)]


def solve_block(rhs: list, n1: int) -> list[Fraction]:
    """The coefficients c of one block: b1 c[k-1] + b0 c[k] + b1 c[k+1] = rhs[k] for the inner
    k, with c at the block's two ends set to rhs there (tridiagonal elimination, exact)."""
    b0, b1 = bspline_at_integer(0, n1), bspline_at_integer(1, n1)
    rhs = [Fraction(v) for v in rhs]
    N = len(rhs)
    if N < 3:
        return rhs
    # unknowns c[1..N-2]; c[0], c[N-1] fixed to the block's end values
    first, last = rhs[0], rhs[-1]
    d = rhs[1:N - 1]
    d[0] -= b1 * first
    d[-1] -= b1 * last
    m = len(d)
    cp = [Fraction(0)] * m
    dp = [Fraction(0)] * m
    cp[0] = b1 / b0
    dp[0] = d[0] / b0
    for i in range(1, m):
        den = b0 - b1 * cp[i - 1]
        cp[i] = b1 / den
        dp[i] = (d[i] - b1 * dp[i - 1]) / den
    x = [Fraction(0)] * m
    x[-1] = dp[-1]
    for i in range(m - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return [first] + x + [last]


def _ext(f, k: int, border: str):
    L = len(f)
    if 0 <= k < L:
        return f[k]
    if border == "clamp":
        return f[min(max(k, 0), L - 1)]
    return 0.0


def filter1d_exact(f, scales, n: int, n1: int = -1, border: str = "clamp", samples=None) -> list[Fraction]:
    """The exact projections s[m] (Fractions) of one signal for the listed samples (default: all)."""
    if border not in BORDERS:
        raise ValueError("border must be 'clamp' or 'zero'")
    if n1 not in MODELS:
        raise ValueError("model degree must be one of -1, 0, 1, 2, 3")
    f = np.asarray(f)
    L = f.shape[0]
    ms = range(L) if samples is None else samples
    glob = None
    if samples is None and n1 >= 2:
        # one block for the whole signal: the coefficients every output reaches
        Rg = max(int(math.floor(support_radius(scales[m], n, n1))) for m in range(L))
        glob = (-Rg, coefficients(f, n1, border, -Rg, L + Rg))
    out = []
    for m in ms:
        a = scales[m]
        R = int(math.floor(support_radius(a, n, n1)))
        ks = list(range(m - R, m + R + 1))
        if glob is not None:
            cs = glob[1][m - R - glob[0]:m + R + 1 - glob[0]]
        else:
            cs = coefficients(f, n1, border, m - R, m + R + 1)
        nums, den = kernel_numerators([m - k for k in ks], a, n, n1)
        acc = Fraction(0)
        for cv, w in zip(cs, nums):
            if w:
                acc += cv * w
        out.append(acc / den)
    return out


def filter1d(f, scales, n: int, n1: int = -1, border: str = "clamp", samples=None) -> np.ndarray:
    """s[m] of one signal, float64 (each value the correctly rounded exact projection)."""
    return np.array([float(v) for v in filter1d_exact(f, scales, n, n1, border, samples)], dtype=np.float64)


def filter1d_batch(signals, scales, n: int, n1: int = -1, border: str = "clamp", samples=None) -> np.ndarray:
    """Row-wise filter1d of a [batch, length] array; ``samples`` lists (row, m) pairs or is None."""
    signals = np.asarray(signals)
    scales = np.asarray(scales)
    if samples is None:
        return np.stack([filter1d(signals[b], scales[b], n, n1, border) for b in range(signals.shape[0])])
    out = np.empty(len(samples))
    for i, (b, m) in enumerate(samples):
        out[i] = filter1d(signals[b], scales[b], n, n1, border, [m])[0]
    return out
