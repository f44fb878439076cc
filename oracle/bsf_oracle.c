/*
 * bsf_oracle.c -- plain CPU oracle for the space-variant four-direction box-spline filter.
 *
 * TEST INFRASTRUCTURE.  This is the reference that the HIP path is checked against.
 * Only the tests, the package smoke check and the benchmark's CPU-baseline leg may
 * load it; the product path never does.  It shares no code, header, table or
 * constant with the HIP library and it is built with plain gcc (-ffp-contract=off).
 *
 * What it computes
 * ----------------
 * The filter of Section 6 is the projection  s[m] = < f, B_{a(m)}(. - m) >  of the
 * image onto the box spline with the pixel's own scale vector a(m).  Section 7
 * chooses phi = delta, so the continuous image is the Dirac comb of the samples and
 *
 *     s[m] = sum_k f_ext[k] * B_{a(m)}(m - k)                                  (1)
 *
 * (B is even).  The paper's two-stage algorithm (pre-integration, eq. RS, then the
 * adaptive mesh, eq. final_eqn) reaches (1) exactly by the factorisation of
 * Section 5 (eq. factor); this file evaluates (1) directly, which involves only
 * non-negative terms.
 *
 *   * B_a is the four-direction box spline of Section 7 (eq. def with N = 4):
 *     the convolution of unit-mass segments of length a_d along
 *     r_d = (cos t_d, sin t_d), t_d = (d-1) pi/4  (Section 4, eq. generator).
 *   * Order n is the n-fold self-convolution of B_a (the closing remark of
 *     Section 4).  Each direction then carries the sum of n uniform variables,
 *     whose density is the scaled B-spline  beta^{n-1}_{a_d}  (Section 2,
 *     eq. definition; beta_a = rect(x/a)/a for degree 0).
 *   * f_ext is the image extended by the boundary rule.  The paper leaves 2-D
 *     boundaries open; clamp-to-edge (border 0) and zero (border 1) are offered.
 *
 * Evaluating B_a(x).  Write the two diagonal segment sums as coordinates
 * (s, t) along r2 = (1,1)/sqrt2 and r4 = (-1,1)/sqrt2; the axis sums then have
 * to make up the rest of x, so
 *
 *   B_a(x) = int int  b2(s) b4(t) b1(x1 - (s - t)/sqrt2) b3(x2 - (s + t)/sqrt2) ds dt,
 *
 * with b_d = beta^{n-1}_{a_d}.  The integrand is a polynomial on every cell cut
 * out of the (s, t) plane by the knots of the four factors (vertical, horizontal
 * and the two diagonal families), so the integral is computed exactly, up to
 * rounding: each cell is clipped as a convex polygon, fanned into triangles and
 * integrated with a collapsed Gauss-Legendre rule exact for the integrand's
 * degree 4(n-1).
 *
 * Stage 1 alone.  For the bit-exact check of the pre-integrator there is also
 * the running-sum recursion of Section 7 (eq. RS, steps (1)-(4)) applied n times
 * per direction on an integer window, in 128-bit integers with unit weights
 * (the two sqrt2 weights of the diagonal steps contribute a factor 2^n that the
 * caller applies).  The recursion of step (4) reads its predecessor down and to
 * the right, so it runs on the window extended to the right by a triangle of
 * zeros (row r from the bottom gets H-1-r extra columns); without it the
 * result is wrong wherever that ray leaves the window.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAX_GL 8

static double gl_x[MAX_GL + 1][MAX_GL];
static double gl_w[MAX_GL + 1][MAX_GL];
static int gl_ready = 0;

/* Gauss-Legendre nodes/weights on [0,1]: Newton iteration on the Legendre polynomial P_m. */
static double legendre(int m, double z, double* dp) {
    double p0 = 1.0, p1 = 0.0;
    for (int k = 1; k <= m; ++k) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
    }
    *dp = m * (z * p0 - p1) / (z * z - 1.0);
    return p0;
}

static void gl_init(void) {
    if (gl_ready) return;
    for (int m = 1; m <= MAX_GL; ++m) {
        for (int i = 0; i < m; ++i) {
            double z = cos(M_PI * (i + 0.75) / (m + 0.5)), dp;
            for (int it = 0; it < 100; ++it) {
                double dz = legendre(m, z, &dp) / dp;
                z -= dz;
                if (fabs(dz) < 1e-16) break;
            }
            legendre(m, z, &dp);
            gl_x[m][i] = 0.5 * (1.0 - z);
            gl_w[m][i] = 1.0 / ((1.0 - z * z) * dp * dp); /* half of 2/((1-z^2) P'(z)^2) */
        }
    }
    gl_ready = 1;
}

/* Centred cardinal B-spline of degree m (Section 2, eq. definition with a = 1):
 * the m+1 fold convolution of the unit box on (-1/2, 1/2]. */
static double cardinal_bspline(int m, double y) {
    if (m == 0) return (y > -0.5 && y <= 0.5) ? 1.0 : 0.0;
    double s = 0.0, binom = 1.0, fact = 1.0;
    for (int k = 1; k <= m; ++k) fact *= k;
    for (int k = 0; k <= m + 1; ++k) {
        double z = y + 0.5 * (m + 1) - k;
        if (z > 0.0) s += ((k & 1) ? -binom : binom) * pow(z, m);
        binom = binom * (m + 1 - k) / (k + 1);
    }
    return s / fact;
}

/* beta^m_a(y) = beta^m(y/a)/a */
static double scaled_bspline(int m, double a, double y) { return cardinal_bspline(m, y / a) / a; }

typedef struct { double s, t; } pt2;

/* keep the half plane  ca*s + cb*t <= cc  of a convex polygon */
static int clip_poly(const pt2* in, int nin, double ca, double cb, double cc, pt2* out) {
    int nout = 0;
    for (int i = 0; i < nin; ++i) {
        pt2 P = in[i], Q = in[(i + 1) % nin];
        double fp = ca * P.s + cb * P.t - cc;
        double fq = ca * Q.s + cb * Q.t - cc;
        if (fp <= 0.0) out[nout++] = P;
        if ((fp < 0.0 && fq > 0.0) || (fp > 0.0 && fq < 0.0)) {
            double r = fp / (fp - fq);
            pt2 X = {P.s + r * (Q.s - P.s), P.t + r * (Q.t - P.t)};
            out[nout++] = X;
        }
    }
    return nout;
}

double bsf_oracle_box_spline(double x1, double x2, const double* a, int n) {
    gl_init();
    const double a1 = a[0], a2 = a[1], a3 = a[2], a4 = a[3];
    const int m = n - 1;
    /* support: x = sum_d sigma_d r_d with |sigma_d| <= n a_d / 2 */
    const double h = 0.5 * n;
    const double R1 = h * (a1 + (a2 + a4) * M_SQRT1_2);
    const double R2 = h * (a3 + (a2 + a4) * M_SQRT1_2);
    if (fabs(x1) >= R1 || fabs(x2) >= R2) return 0.0;
    if (fabs(x1 + x2) >= h * (a1 + a3 + 2.0 * a2 * M_SQRT1_2)) return 0.0;
    if (fabs(x1 - x2) >= h * (a1 + a3 + 2.0 * a4 * M_SQRT1_2)) return 0.0;

    double ks[8], kt[8], c1[8], c3[8];
    for (int i = 0; i <= n; ++i) {
        ks[i] = a2 * (i - h);
        kt[i] = a4 * (i - h);
        c1[i] = M_SQRT2 * (x1 - a1 * (i - h)); /* line s - t = c1[i] */
        c3[i] = M_SQRT2 * (x2 - a3 * (i - h)); /* line s + t = c3[i] */
    }
    const int p = 4 * m;
    const int mu = (p + 3) / 2, mw = (p + 2) / 2;
    double total = 0.0;
    pt2 A[16], B[16];
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k)
            for (int ii = 0; ii < n; ++ii) {
                const double lo1 = c1[ii + 1], hi1 = c1[ii];
                for (int kk = 0; kk < n; ++kk) {
                    const double lo3 = c3[kk + 1], hi3 = c3[kk];
                    int np = 4;
                    A[0].s = ks[i];     A[0].t = kt[k];
                    A[1].s = ks[i + 1]; A[1].t = kt[k];
                    A[2].s = ks[i + 1]; A[2].t = kt[k + 1];
                    A[3].s = ks[i];     A[3].t = kt[k + 1];
                    np = clip_poly(A, np, 1.0, -1.0, hi1, B);
                    if (np < 3) continue;
                    np = clip_poly(B, np, -1.0, 1.0, -lo1, A);
                    if (np < 3) continue;
                    np = clip_poly(A, np, 1.0, 1.0, hi3, B);
                    if (np < 3) continue;
                    np = clip_poly(B, np, -1.0, -1.0, -lo3, A);
                    if (np < 3) continue;
                    for (int q = 1; q + 1 < np; ++q) {
                        const pt2 v0 = A[0], v1 = A[q], v2 = A[q + 1];
                        const double e1s = v1.s - v0.s, e1t = v1.t - v0.t;
                        const double e2s = v2.s - v0.s, e2t = v2.t - v0.t;
                        const double area2 = fabs(e1s * e2t - e1t * e2s);
                        if (area2 == 0.0) continue;
                        double acc = 0.0;
                        for (int iu = 0; iu < mu; ++iu) {
                            const double u = gl_x[mu][iu], wu = gl_w[mu][iu];
                            for (int iw = 0; iw < mw; ++iw) {
                                const double w = gl_x[mw][iw], ww = gl_w[mw][iw];
                                const double xi = u, eta = w * (1.0 - u);
                                const double s = v0.s + xi * e1s + eta * e2s;
                                const double t = v0.t + xi * e1t + eta * e2t;
                                const double val = scaled_bspline(m, a2, s) * scaled_bspline(m, a4, t) *
                                                   scaled_bspline(m, a1, x1 - (s - t) * M_SQRT1_2) *
                                                   scaled_bspline(m, a3, x2 - (s + t) * M_SQRT1_2);
                                acc += val * wu * ww * (1.0 - u);
                            }
                        }
                        total += acc * area2;
                    }
                }
            }
    return total;
}

/* s[m] of (1) for one pixel */
static double filter_pixel(const double* f, int H, int W, ptrdiff_t pitch, const float* sc, int n,
                           int border, int m1, int m2) {
    double a[4] = {sc[0], sc[1], sc[2], sc[3]};
    const double h = 0.5 * n;
    const double R1 = h * (a[0] + (a[1] + a[3]) * M_SQRT1_2);
    const double R2 = h * (a[2] + (a[1] + a[3]) * M_SQRT1_2);
    const int k1lo = (int)floor(m1 - R1), k1hi = (int)ceil(m1 + R1);
    const int k2lo = (int)floor(m2 - R2), k2hi = (int)ceil(m2 + R2);
    double acc = 0.0;
    for (int k2 = k2lo; k2 <= k2hi; ++k2) {
        int r = k2;
        if (r < 0 || r >= H) {
            if (border) continue;
            r = r < 0 ? 0 : H - 1;
        }
        for (int k1 = k1lo; k1 <= k1hi; ++k1) {
            int c = k1;
            if (c < 0 || c >= W) {
                if (border) continue;
                c = c < 0 ? 0 : W - 1;
            }
            const double v = f[(ptrdiff_t)r * pitch + c];
            if (v == 0.0) continue;
            acc += v * bsf_oracle_box_spline((double)(m1 - k1), (double)(m2 - k2), a, n);
        }
    }
    return acc;
}

/*
 * f: [H][pitch] doubles.  scales: [H][W][4] float32 (a1..a4 in paper units).
 * pix == NULL: every pixel in row-major order into out[H*W];
 * otherwise out[i] for the flat pixel index pix[i] = m2*W + m1.
 * Returns 0, or -1 on bad arguments.
 */
int bsf_oracle_filter(const double* f, int H, int W, ptrdiff_t pitch, const float* scales, int n,
                      int border, const int64_t* pix, int64_t npix, double* out) {
    if (!f || !scales || !out || H < 1 || W < 1 || pitch < W || n < 1 || n > 6) return -1;
    gl_init();
    const int64_t total = pix ? npix : (int64_t)H * W;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < total; ++i) {
        const int64_t id = pix ? pix[i] : i;
        const int m2 = (int)(id / W), m1 = (int)(id % W);
        out[i] = filter_pixel(f, H, W, pitch, scales + 4 * id, n, border, m1, m2);
    }
    return 0;
}

/*
 * Stage 1 on an integer window (eq. RS, steps (1)-(4), n times each, unit weights).
 * win: [Hq][Wq] int64 samples of the window (row 0 = bottom, i.e. smallest k2).
 * g:   [Hq][Wq] int64 output on the window.  Returns 0, -1 on bad arguments,
 * -2 if a result does not fit in int64.
 */
int bsf_oracle_preintegrate(const int64_t* win, int Hq, int Wq, int n, int64_t* g) {
    if (!win || !g || Hq < 1 || Wq < 1 || n < 1) return -1;
    const int Wt = Wq + Hq - 1;
    __int128* F = (__int128*)calloc((size_t)Hq * Wt, sizeof(__int128));
    if (!F) return -1;
#define AT(r, c) F[(size_t)(r) * Wt + (c)]
#define LEN(r) (Wq + (Hq - 1 - (r)))
    for (int r = 0; r < Hq; ++r)
        for (int c = 0; c < Wq; ++c) AT(r, c) = win[(size_t)r * Wq + c];
    for (int f = 0; f < n; ++f) /* (1) F0[k1,k2] = f[k1,k2] + F0[k1-1,k2] */
        for (int r = 0; r < Hq; ++r)
            for (int c = 1; c < LEN(r); ++c) AT(r, c) += AT(r, c - 1);
    for (int f = 0; f < n; ++f) /* (2) F45[k1,k2] = F0[k1,k2] + F45[k1-1,k2-1] */
        for (int r = 1; r < Hq; ++r)
            for (int c = LEN(r) - 1; c >= 1; --c) AT(r, c) += AT(r - 1, c - 1);
    for (int f = 0; f < n; ++f) /* (3) F90[k1,k2] = F45[k1,k2] + F90[k1,k2-1] */
        for (int r = 1; r < Hq; ++r)
            for (int c = 0; c < LEN(r); ++c) AT(r, c) += AT(r - 1, c);
    for (int f = 0; f < n; ++f) /* (4) g[k1,k2] = F90[k1,k2] + g[k1+1,k2-1] */
        for (int r = 1; r < Hq; ++r)
            for (int c = 0; c < LEN(r); ++c) AT(r, c) += AT(r - 1, c + 1);
    int rc = 0;
    const __int128 lim = ((__int128)1) << 63;
    for (int r = 0; r < Hq; ++r)
        for (int c = 0; c < Wq; ++c) {
            __int128 v = AT(r, c);
            if (v >= lim || v < -lim) rc = -2;
            g[(size_t)r * Wq + c] = (int64_t)(uint64_t)v; /* low 64 bits */
        }
#undef AT
#undef LEN
    free(F);
    return rc;
}

/*
 * Continuous models (Section 6): the image is f(x) = sum_k c[k] phi(x - k) with
 * phi = beta^{n1} (x) beta^{n1} (centred unit-scale B-splines of degree n1 along x and y;
 * n1 = -1 is phi = delta, Section 7's choice), and the projection onto the box spline is
 *
 *     s[m] = sum_k c[k] (phi * B_a)(m - k).                                       (2)
 *
 * phi is separable and B_a depends on x1 and x2 only through its two axis factors, so
 *
 *   (phi * B_a)(x) = int int b2(s) b4(t) K1(x1 - (s - t)/sqrt2) K3(x2 - (s + t)/sqrt2) ds dt,
 *
 * with K_d = beta^{n1} * b_d the one-dimensional model kernel of Section 3 at the scale
 * a_d.  K_d is evaluated as the integral of beta^{n1}(u) b_d(y - u) over u, piece by piece
 * between the knots of both factors (Gauss-Legendre exact for the product's degree; the
 * integrand is non-negative), and the outer integral as before, on the cells cut out by
 * the knots of b2, b4 and of K1, K3.
 */
#define MAX_KN 64

/* K(y) = (beta^{n1} * beta^{n-1}_a)(y); n1 = -1: beta^{n-1}_a(y) */
static double model_kernel(int n, int n1, double a, double y) {
    if (n1 < 0) return scaled_bspline(n - 1, a, y);
    double kn[MAX_KN];
    int nk = 0;
    for (int i = 0; i <= n1 + 1; ++i) kn[nk++] = -0.5 * (n1 + 1) + i;   /* beta^{n1}(u)   */
    for (int j = 0; j <= n; ++j) kn[nk++] = y - a * (j - 0.5 * n);        /* b(y - u)       */
    for (int i = 1; i < nk; ++i)                                           /* sort           */
        for (int k = i; k > 0 && kn[k - 1] > kn[k]; --k) {
            const double t = kn[k];
            kn[k] = kn[k - 1];
            kn[k - 1] = t;
        }
    const double lo = fmax(-0.5 * (n1 + 1), y - 0.5 * a * n), hi = fmin(0.5 * (n1 + 1), y + 0.5 * a * n);
    if (!(lo < hi)) return 0.0;
    const int deg = n1 + n - 1, mg = deg / 2 + 1;
    double total = 0.0;
    for (int i = 0; i + 1 < nk; ++i) {
        const double u0 = fmax(kn[i], lo), u1 = fmin(kn[i + 1], hi);
        if (!(u0 < u1)) continue;
        double acc = 0.0;
        for (int g = 0; g < mg; ++g) {
            const double u = u0 + (u1 - u0) * gl_x[mg][g];
            acc += gl_w[mg][g] * cardinal_bspline(n1, u) * scaled_bspline(n - 1, a, y - u);
        }
        total += acc * (u1 - u0);
    }
    return total;
}

/* knots of K (in y), sorted and de-duplicated */
static int model_knots(int n, int n1, double a, double* kn) {
    int nk = 0;
    const int ni = n1 < 0 ? 0 : n1 + 1;
    for (int i = 0; i <= ni; ++i)
        for (int j = 0; j <= n; ++j) kn[nk++] = (n1 < 0 ? 0.0 : -0.5 * (n1 + 1) + i) + a * (j - 0.5 * n);
    for (int i = 1; i < nk; ++i)
        for (int k = i; k > 0 && kn[k - 1] > kn[k]; --k) {
            const double t = kn[k];
            kn[k] = kn[k - 1];
            kn[k - 1] = t;
        }
    int m = 0;
    for (int i = 0; i < nk; ++i)
        if (m == 0 || kn[i] > kn[m - 1]) kn[m++] = kn[i];
    return m;
}

double bsf_oracle_box_spline_model(double x1, double x2, const double* a, int n, int n1) {
    gl_init();
    if (n < 1 || n1 < -1 || n1 > 3 || (n1 + 1) * (n + 1) + n + 1 > MAX_KN) return NAN;
    const double a1 = a[0], a2 = a[1], a3 = a[2], a4 = a[3];
    const int m = n - 1;
    const double h = 0.5 * n, e = n1 < 0 ? 0.0 : 0.5 * (n1 + 1);
    if (fabs(x1) >= h * (a1 + (a2 + a4) * M_SQRT1_2) + e || fabs(x2) >= h * (a3 + (a2 + a4) * M_SQRT1_2) + e)
        return 0.0;
    double ks[8], kt[8], k1[MAX_KN], k3[MAX_KN];
    for (int i = 0; i <= n; ++i) {
        ks[i] = a2 * (i - h);
        kt[i] = a4 * (i - h);
    }
    const int n1k = model_knots(n, n1, a1, k1), n3k = model_knots(n, n1, a3, k3);
    /* K1 knot kappa: the line s - t = sqrt2 (x1 - kappa); descending in kappa = ascending in s - t */
    const int dK = n1 < 0 ? m : n1 + n;
    const int p = 2 * m + 2 * dK;
    const int mu = (p + 3) / 2, mw = (p + 2) / 2;
    if (mu > MAX_GL || mw > MAX_GL) return NAN;
    double total = 0.0;
    pt2 A[24], B[24];
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k)
            for (int ii = 0; ii + 1 < n1k; ++ii) {
                /* x1 - (s-t)/sqrt2 in [k1[ii], k1[ii+1]]  <=>  s - t in [sqrt2 (x1 - k1[ii+1]), sqrt2 (x1 - k1[ii])] */
                const double lo1 = M_SQRT2 * (x1 - k1[ii + 1]), hi1 = M_SQRT2 * (x1 - k1[ii]);
                for (int kk = 0; kk + 1 < n3k; ++kk) {
                    const double lo3 = M_SQRT2 * (x2 - k3[kk + 1]), hi3 = M_SQRT2 * (x2 - k3[kk]);
                    int np = 4;
                    A[0].s = ks[i];     A[0].t = kt[k];
                    A[1].s = ks[i + 1]; A[1].t = kt[k];
                    A[2].s = ks[i + 1]; A[2].t = kt[k + 1];
                    A[3].s = ks[i];     A[3].t = kt[k + 1];
                    np = clip_poly(A, np, 1.0, -1.0, hi1, B);
                    if (np < 3) continue;
                    np = clip_poly(B, np, -1.0, 1.0, -lo1, A);
                    if (np < 3) continue;
                    np = clip_poly(A, np, 1.0, 1.0, hi3, B);
                    if (np < 3) continue;
                    np = clip_poly(B, np, -1.0, -1.0, -lo3, A);
                    if (np < 3) continue;
                    for (int q = 1; q + 1 < np; ++q) {
                        const pt2 v0 = A[0], v1 = A[q], v2 = A[q + 1];
                        const double e1s = v1.s - v0.s, e1t = v1.t - v0.t;
                        const double e2s = v2.s - v0.s, e2t = v2.t - v0.t;
                        const double area2 = fabs(e1s * e2t - e1t * e2s);
                        if (area2 == 0.0) continue;
                        double acc = 0.0;
                        for (int iu = 0; iu < mu; ++iu) {
                            const double u = gl_x[mu][iu], wu = gl_w[mu][iu];
                            for (int iw = 0; iw < mw; ++iw) {
                                const double w = gl_x[mw][iw], ww = gl_w[mw][iw];
                                const double xi = u, eta = w * (1.0 - u);
                                const double s = v0.s + xi * e1s + eta * e2s;
                                const double t = v0.t + xi * e1t + eta * e2t;
                                const double val = scaled_bspline(m, a2, s) * scaled_bspline(m, a4, t) *
                                                   model_kernel(n, n1, a1, x1 - (s - t) * M_SQRT1_2) *
                                                   model_kernel(n, n1, a3, x2 - (s + t) * M_SQRT1_2);
                                acc += val * wu * ww * (1.0 - u);
                            }
                        }
                        total += acc * area2;
                    }
                }
            }
    return total;
}

/*
 * (2) for a coefficient array that already holds c[k] for every k the sums reach:
 * c[(k2 + org) * pitch + (k1 + org)] for k in [-org, H + org) x [-org, W + org).
 * Output as bsf_oracle_filter.  Returns 0, or -1 on bad arguments (including an org too
 * small for a pixel's support).
 */
int bsf_oracle_filter_model(const double* c, int H, int W, ptrdiff_t pitch, int org, const float* scales, int n,
                            int n1, const int64_t* pix, int64_t npix, double* out) {
    if (!c || !scales || !out || H < 1 || W < 1 || n < 1 || n > 6 || n1 < -1 || n1 > 3 || org < 0 ||
        pitch < W + 2 * org)
        return -1;
    gl_init();
    const int64_t total = pix ? npix : (int64_t)H * W;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t i = 0; i < total; ++i) {
        const int64_t id = pix ? pix[i] : i;
        const int m2 = (int)(id / W), m1 = (int)(id % W);
        const float* sc = scales + 4 * id;
        double a[4] = {sc[0], sc[1], sc[2], sc[3]};
        const double h = 0.5 * n, e = n1 < 0 ? 0.0 : 0.5 * (n1 + 1);
        const double R1 = h * (a[0] + (a[1] + a[3]) * M_SQRT1_2) + e;
        const double R2 = h * (a[2] + (a[1] + a[3]) * M_SQRT1_2) + e;
        const int k1lo = (int)floor(m1 - R1), k1hi = (int)ceil(m1 + R1);
        const int k2lo = (int)floor(m2 - R2), k2hi = (int)ceil(m2 + R2);
        if (k1lo < -org || k2lo < -org || k1hi >= W + org || k2hi >= H + org) {
            bad = 1;
            out[i] = NAN;
            continue;
        }
        double acc = 0.0;
        for (int k2 = k2lo; k2 <= k2hi; ++k2)
            for (int k1 = k1lo; k1 <= k1hi; ++k1) {
                const double v = c[(ptrdiff_t)(k2 + org) * pitch + (k1 + org)];
                if (v == 0.0) continue;
                acc += v * bsf_oracle_box_spline_model((double)(m1 - k1), (double)(m2 - k2), a, n, n1);
            }
        out[i] = acc;
    }
    return bad ? -1 : 0;
}
