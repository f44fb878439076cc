#!/usr/bin/env python3
"""Generate the exact piecewise-polynomial tables of the lattice interpolant.

What is tabulated
-----------------
The adaptive step (Section 7, eq. ``final_eqn``) evaluates the pre-integrated
sequence g between lattice points with the interpolant built from the
four-direction box spline at the integration scale b = (1, sqrt2, 1, sqrt2)
(Section 7, the remark on the Zwart-Powell element, and Section 6, eq. ``NA``
with phi = delta).  At that scale the four generating segments are exactly the
lattice steps l1=(1,0), l2=(1,1), l3=(0,1), l4=(-1,1) (eq. ``RS_filter``).
For order n (the n-fold self-convolution of Section 4, last paragraph) every
direction appears n times, so the interpolant is the centred box spline

    beta_n(x) = M_Xi(x + c),   Xi = {l1^n, l2^n, l3^n, l4^n},   c = (n/2)(1, 3).

M_Xi is a piecewise polynomial of degree 4n-2 on the type-II triangulation of
Z^2 (unit squares cut by both diagonals).  Around the interpolation point the
kernel picks the cell whose centre is the nearest lattice point (odd n) or the
nearest half-integer point (even n), writes the point as  q + o + u  with
|u_i| <= 1/2, and uses the symmetry of beta_n under quarter turns to bring u
into the "right" triangle  u1 >= |u2|.  On that triangle

    sum_j g[q + j] beta_n(o + u - j) = sum_alpha G_alpha u^alpha,
    G_alpha = sum_j W[j, alpha] g[q + j],

and this script emits W (exact rationals with one common denominator per n).

How it is derived (independently of any numerical evaluator)
------------------------------------------------------------
1. The cone spline T_Xi (the kernel of n-fold running sums along Xi) is built
   by directional integration,  T_{Xi+xi}(x) = int_0^inf T_Xi(x - t xi) dt,
   starting from the two-direction cone indicator 1/|det(l1, l3)|.  On each of
   the three sectors between the rays l1, l2, l3, l4 it is a homogeneous
   polynomial; the integrals are done in exact rational arithmetic (sympy).
2. The box spline is its backward difference  M_Xi = prod_{xi in Xi} (1 - E^xi) T_Xi,
   the continuous counterpart of the finite-difference/running-sum factorisation
   of Section 5 (eq. ``factor``).
3. Restricting every translate to the reference triangle gives W.

Self-checks run before anything is written: partition of unity, the lattice
values 1/2 and 1/8 of the n=1 element, quarter-turn symmetry (all four triangles
computed independently), and continuity across the triangle edges.

Usage:  python gen_tables.py  [--out boxspline_tables.h] [--orders 1,2,3] [--models-out model_tables.h]
        [--models 0,1]  (--orders '' writes the model tables alone)
"""
import argparse
import itertools
import os
import sys
from fractions import Fraction
from math import comb, gcd

import sympy as sp

X1, X2, T = sp.symbols("x1 x2 t")
# lattice steps l1..l4; in angular order they are also the sector boundary rays
DIRS = [(1, 0), (1, 1), (0, 1), (-1, 1)]


def det(a, b):
    return a[0] * b[1] - a[1] * b[0]


def sector_of(p):
    """Index 0..2 of the open sector containing p, None if p is outside the
    cone spanned by l1 and l4.  Points on a boundary ray are rejected."""
    for s in range(3):
        d0 = det(DIRS[s], p)
        d1 = det(p, DIRS[s + 1])
        if d0 == 0 and (p[0] * DIRS[s][0] + p[1] * DIRS[s][1]) > 0:
            raise ValueError("point on a sector ray")
        if d0 > 0 and d1 > 0:
            return s
    if det(DIRS[3], p) == 0 and (p[0] * DIRS[3][0] + p[1] * DIRS[3][1]) > 0:
        raise ValueError("point on a sector ray")
    return None


# ----------------------------------------------------------------------------
# dictionary polynomials  {(a, b): Fraction}  in two variables
# ----------------------------------------------------------------------------
def sym_to_dict(expr):
    poly = sp.Poly(sp.expand(expr), X1, X2, domain="QQ")
    out = {}
    for (a, b), c in poly.terms():
        c = sp.Rational(c)
        out[(a, b)] = Fraction(int(c.p), int(c.q))
    return out


def shift(P, h1, h2):
    """P(y1 + h1, y2 + h2) as a polynomial in (y1, y2)."""
    out = {}
    for (a, b), c in P.items():
        for i in range(a + 1):
            ca = c * comb(a, i) * (Fraction(h1) ** (a - i))
            if ca == 0:
                continue
            for k in range(b + 1):
                cb = ca * comb(b, k) * (Fraction(h2) ** (b - k))
                if cb:
                    out[(i, k)] = out.get((i, k), 0) + cb
    return {m: c for m, c in out.items() if c != 0}


def padd(P, Q, s=1):
    out = dict(P)
    for m, c in Q.items():
        out[m] = out.get(m, 0) + s * c
    return {m: c for m, c in out.items() if c != 0}


def peval(P, u1, u2):
    return sum(c * Fraction(u1) ** a * Fraction(u2) ** b for (a, b), c in P.items())


def rotate_poly(P, quarter):
    """P(R^-quarter u): the polynomial in u obtained by rotating the argument."""
    out = dict(P)
    for _ in range(quarter % 4):
        # (R^-1 u) = (u2, -u1)  for R = rotation by +90 degrees
        nxt = {}
        for (a, b), c in out.items():
            # P(v1, v2) with v1 = u2, v2 = -u1  ->  c * u2^a * (-u1)^b
            nxt[(b, a)] = nxt.get((b, a), 0) + c * (-1) ** b
        out = nxt
    return out


# ----------------------------------------------------------------------------
# cone spline by directional integration
# ----------------------------------------------------------------------------
def add_direction(Tcone, xi):
    new = {}
    for s in range(3):
        xs = (DIRS[s][0] + DIRS[s + 1][0], DIRS[s][1] + DIRS[s + 1][1])  # inside sector s
        cross = []
        for r in DIRS:
            d = det(xi, r)
            if d == 0:
                continue
            tc = Fraction(det(xs, r), d)
            if tc <= 0:
                continue
            px = (xs[0] - tc * xi[0], xs[1] - tc * xi[1])
            if px[0] * r[0] + px[1] * r[1] <= 0:
                continue
            cross.append((tc, r))
        cross.sort(key=lambda e: e[0])
        bounds = [(Fraction(0), None)] + cross
        expr = sp.Integer(0)
        for i, (ta, ra) in enumerate(bounds):
            if i + 1 < len(bounds):
                tb, rb = bounds[i + 1]
                tmid = (ta + tb) / 2
            else:
                tb, rb = None, None
                tmid = ta + 1
            pm = (xs[0] - tmid * xi[0], xs[1] - tmid * xi[1])
            sm = sector_of(pm)
            if sm is None or sm not in Tcone:
                continue
            if tb is None:
                raise AssertionError("unbounded integration segment inside the support")
            lo = sp.Integer(0) if ra is None else sp.Rational(1, det(xi, ra)) * (X1 * ra[1] - X2 * ra[0])
            hi = sp.Rational(1, det(xi, rb)) * (X1 * rb[1] - X2 * rb[0])
            integrand = sp.expand(Tcone[sm].subs({X1: X1 - T * xi[0], X2: X2 - T * xi[1]}, simultaneous=True))
            F = sp.integrate(integrand, T)
            expr += F.subs(T, hi) - F.subs(T, lo)
        expr = sp.expand(expr)
        if expr != 0:
            new[s] = expr
    return new


def cone_spline(n, q=None):
    """T_Xi per sector as dict polynomials, Xi = {l1^n, l2^q, l3^n, l4^q} (q = n by default)."""
    q = n if q is None else q
    Tcone = {0: sp.Integer(1), 1: sp.Integer(1)}  # cone of l1, l3: 1/|det| = 1
    order = [DIRS[0]] * (n - 1) + [DIRS[2]] * (n - 1) + [DIRS[1]] * q + [DIRS[3]] * q
    for xi in order:
        Tcone = add_direction(Tcone, xi)
    return {s: sym_to_dict(e) for s, e in Tcone.items()}


# ----------------------------------------------------------------------------
# box spline pieces on cells
# ----------------------------------------------------------------------------
def box_piece(cone, n, base, centroid, q=None):
    """Polynomial in u of M_Xi(base + u) on the mesh triangle that contains
    base + centroid (base, centroid rational 2-vectors); Xi = {l1^n, l2^q, l3^n, l4^q}."""
    q = n if q is None else q
    P = {}
    for k in itertools.product(range(n + 1), range(q + 1), range(n + 1), range(q + 1)):
        coef = (-1) ** sum(k)
        for kd, md in zip(k, (n, q, n, q)):
            coef *= comb(md, kd)
        v = (k[0] * 1 + k[1] * 1 + k[3] * -1, k[1] + k[2] + k[3])
        z0 = (base[0] - v[0], base[1] - v[1])
        s = sector_of((z0[0] + centroid[0], z0[1] + centroid[1]))
        if s is None or s not in cone:
            continue
        P = padd(P, shift(cone[s], z0[0], z0[1]), coef)
    return P


# reference triangles of a cell in local coordinates u (|u_i| <= 1/2):
# 0 right (u1 >= |u2|), 1 top, 2 left, 3 bottom; a quarter turn maps i -> i+1
TRI_CENTROID = [(Fraction(1, 3), Fraction(0)), (Fraction(0), Fraction(1, 3)),
                (Fraction(-1, 3), Fraction(0)), (Fraction(0), Fraction(-1, 3))]
TRI_VERTS = [[(0, 0), (Fraction(1, 2), Fraction(-1, 2)), (Fraction(1, 2), Fraction(1, 2))]]
for _q in range(1, 4):
    TRI_VERTS.append([(-v[1], v[0]) for v in TRI_VERTS[-1]])


def cell_offset(n):
    """o: the cell centre relative to the anchor lattice point q."""
    return (Fraction(0), Fraction(0)) if n % 2 else (Fraction(1, 2), Fraction(1, 2))


def tables(n, check=True, q=None):
    """Pieces of the centred box spline of Xi = {l1^n, l2^q, l3^n, l4^q} (q = n: the order-n
    lattice box spline).  With q = order and n = order + model + 1 it is the interpolant of
    the continuous model of degree `model` (Section 6: phi * beta_b, phi = beta^model x
    beta^model adds model + 1 unit segments along l1 and l3)."""
    q = n if q is None else q
    cone = cone_spline(n, q)
    c = (Fraction(n, 2), Fraction(n, 2) + q)  # the centre: half of sum of the segments
    o = cell_offset(n)
    r = (n + 2 * q + 3) // 2 + 1
    pieces = {tri: {} for tri in range(4)}
    for tri in range(4):
        for j in itertools.product(range(-r, r + 1), repeat=2):
            base = (o[0] - j[0] + c[0], o[1] - j[1] + c[1])
            P = box_piece(cone, n, base, TRI_CENTROID[tri], q)
            if P:
                pieces[tri][j] = P
    if check:
        self_check(n, pieces, o, q)
    return pieces


def self_check(n, pieces, o, q=None):
    q = n if q is None else q
    deg = 2 * n + 2 * q - 2
    for tri in range(4):
        tot = {}
        for j, P in pieces[tri].items():
            assert max(a + b for (a, b) in P) <= deg
            tot = padd(tot, P)
        assert tot == {(0, 0): Fraction(1)}, f"partition of unity fails n={n} tri={tri}: {tot}"
    # quarter-turn symmetry: the piece on triangle tri+1 for stencil point R j equals
    # the piece on triangle tri for j with the argument rotated back
    for tri in range(3):
        for j, P in pieces[tri].items():
            # rotation about the cell centre o: j -> R(j - o) + o
            jr = (-(j[1] - o[1]) + o[0], (j[0] - o[0]) + o[1])
            jr = (int(jr[0]), int(jr[1]))
            Q = pieces[tri + 1].get(jr, {})
            assert rotate_poly(P, 1) == Q, f"quarter-turn symmetry fails n={n} tri={tri} j={j}"
    # continuity across the interior edges of the cell (u1 = u2 and u1 = -u2)
    for j in set(pieces[0]) | set(pieces[1]):
        A = pieces[0].get(j, {})
        B = pieces[1].get(j, {})
        for s in [Fraction(k, 7) for k in range(0, 4)]:
            assert peval(A, s, s) == peval(B, s, s)
    if n == 1 and q == 1:
        # lattice values of the unit-mass element: 1/2 at the centre, 1/8 at the axis neighbours
        P0 = pieces[0]
        assert peval(P0[(0, 0)], 0, 0) == Fraction(1, 2)
        for j in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
            assert peval(P0[j], 0, 0) == Fraction(1, 8), j
        # half-integer values (1/2,0) -> 3/8, (1/2,1/2) -> 1/4
        assert peval(P0[(0, 0)], Fraction(1, 2), 0) == Fraction(3, 8)
        assert peval(P0[(0, 0)], Fraction(1, 2), Fraction(1, 2)) == Fraction(1, 4)


def monomials(n, q=None):
    q = n if q is None else q
    deg = 2 * n + 2 * q - 2
    return [(a, b) for a in range(deg + 1) for b in range(deg + 1 - a)]


def lcm(a, b):
    return a * b // gcd(a, b)


def emit(all_tables, path, suffix=lambda key: str(key), title=None, label=lambda key: f"order n = {key}"):
    lines = []
    lines.append("// Generated by gen_tables.py -- do not edit.")
    for t in (title or ["Exact piecewise-polynomial pieces of the order-n four-direction lattice box spline",
                        "(the interpolant of the adaptive step, Section 7) on the reference triangle"]):
        lines.append("// " + t)
    lines.append("// u1 >= |u2| of an interpolation cell.  For anchor q and local offset u:")
    lines.append("//   sum_j g[q+j] beta_n(o + u - j) = (1/DEN) * sum_a u1^a1 u2^a2 * sum_j NUM[j][a] g[q+j]")
    lines.append("#pragma once")
    lines.append("namespace bsf_tables {")
    for key, (pieces, mono) in all_tables.items():
        n = suffix(key)
        deg = max(a + b for a, b in mono)
        stencil = sorted(pieces[0].keys(), key=lambda j: (j[1], j[0]))
        den = 1
        for j in stencil:
            for m, cf in pieces[0][j].items():
                den = lcm(den, cf.denominator)
        lines.append(f"// {label(key)}: {len(stencil)} stencil points, {len(mono)} monomials, degree {deg}")
        lines.append(f"constexpr int kStencil{n} = {len(stencil)};")
        lines.append(f"constexpr int kMono{n} = {len(mono)};")
        lines.append(f"constexpr double kDen{n} = {den}.0;")
        lines.append(f"#define BSF_J{n}_INIT {{" + ", ".join(f"{{{j[0]}, {j[1]}}}" for j in stencil) + "}")
        lines.append(f"constexpr int kJ{n}[{len(stencil)}][2] = BSF_J{n}_INIT;")
        lines.append(f"constexpr int kMonoExp{n}[{len(mono)}][2] = {{" +
                     ", ".join(f"{{{a}, {b}}}" for a, b in mono) + "};")
        lines.append(f"#define BSF_NUM{n}_INIT {{ \\")
        maxabs = 0
        for j in stencil:
            row = []
            for m in mono:
                v = pieces[0][j].get(m, Fraction(0)) * den
                assert v.denominator == 1
                maxabs = max(maxabs, abs(v.numerator))
                row.append(f"{v.numerator}.0")
            lines.append("  {" + ", ".join(row) + "}, \\")
        lines.append("}")
        lines.append(f"constexpr double kNum{n}[{len(stencil)}][{len(mono)}] = BSF_NUM{n}_INIT;")
        lines.append(f"// max |numerator| = {maxabs}")
    lines.append("}  // namespace bsf_tables")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(here, "boxspline_tables.h"))
    ap.add_argument("--orders", default="1,2,3")
    ap.add_argument("--models-out", default=os.path.join(here, "model_tables.h"),
                    help="tables of the continuous models (order 1, model degrees 0 and 1); '' to skip")
    ap.add_argument("--models", default="0,1")
    args = ap.parse_args()
    all_tables = {}
    if args.orders:
        for n in [int(s) for s in args.orders.split(",")]:
            pieces = tables(n)
            all_tables[n] = (pieces, monomials(n))
            print(f"n={n}: stencil {len(pieces[0])} points", file=sys.stderr)
        emit(all_tables, args.out, suffix=lambda n: str(n))
    if args.models_out:
        # order 1, model degree m: Xi = {l1^(m+2), l2, l3^(m+2), l4}, key 10 + m
        models = {}
        for m in [int(v) for v in args.models.split(",")]:
            pieces = tables(m + 2, q=1)
            models[10 + m] = (pieces, monomials(m + 2, 1))
            print(f"order 1, model {m}: stencil {len(pieces[0])} points", file=sys.stderr)
        emit(models, args.models_out, suffix=lambda k: f"M{k}", label=lambda k: f"order 1, model degree {k - 10}",
             title=["Exact piecewise-polynomial pieces of the interpolant phi * beta_b of the continuous model",
                    "of degree m (Section 6, phi = beta^m x beta^m) for the order-1 four-direction filter:",
                    "the box spline of {l1^(m+2), l2, l3^(m+2), l4}, table key 10 + m, on the reference triangle"])


if __name__ == "__main__":
    main()
