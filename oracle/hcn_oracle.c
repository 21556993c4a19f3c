/*
 * hcn_oracle.c -- plain, slow CPU oracle for the complex double-double (DD)
 * and quad-double (QD) Newton corrector of the path tracker in
 * "Accelerating Polynomial Homotopy Continuation on a Graphics Processing
 * Unit with Double Double and Quad Double Arithmetic" (Verschelde & Yu).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code with
 * the GPU path: it has its own arithmetic, written from the published
 * algorithm descriptions named below, and its own evaluation, QR and
 * control flow written from the plain definitions.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fused multiply-add is
 * formed except by the explicit fma() calls; glibc's fma is correctly
 * rounded).
 *
 * Number layout (also the library boundary's): a real is P doubles, most
 * significant limb first (P = 2: double-double, P = 4: quad-double); a
 * complex is [2][P] (real limbs, then imaginary limbs).
 *
 * Arithmetic (Section 1: DD/QD arithmetic as in the QD library):
 *   error-free transformations: TwoSum (Knuth), FastTwoSum (Dekker),
 *     TwoProd through a fused multiply-add;
 *   DD: the accurate double-word sum, the FMA double-word product, the
 *     double-word by double product and the double-word quotient of
 *     Joldes, Muller & Popescu (ACM TOMS 2017); square root by one Newton
 *     correction of the double square root (Karp & Markstein, TOMS 1997);
 *   QD: Hida, Li & Bailey (ARITH-15, 2001): renormalisation, the accurate
 *     sum (merge by magnitude, then accumulation in a two-word
 *     accumulator), products keeping all terms down to third order, long
 *     division, square root by Newton iteration on 1/sqrt.
 *   complex: 4-multiplication product (re*re - im*im, re*im + im*re).
 *
 * Method:
 *   eval      f_i = sum_m c_m prod_l x_l^a_ml and every partial derivative
 *             by its plain definition, each partial on its own with
 *             left-to-right products (Section 3.2 computes the same values
 *             by reverse-mode differentiation; exponents above one follow
 *             the generalisation stated in the design notes).
 *   homotopy  h = gamma (1-t)^k g + t^k f  (equation (1)).
 *   solve     modified Gram-Schmidt on [J | -h], then back substitution
 *             (Section 1 and Fig. 2, GPU_Modified_Gram_Schmidt).
 *   newton    the corrector of Fig. 2 with the tests of equation (3).
 *   track     the tracker of Fig. 3 with step bounds of equation (4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_OK 0
#define ORA_EINVAL (-1)
#define ORA_ENOMEM (-2)
#define ORA_ESINGULAR (-4)
#define ORA_NOT_CONVERGED 1
#define ORA_DIVERGED 2
#define ORA_MAX_STEPS 3
#define ORA_STEP_TOO_SMALL 4
#define ORA_NAN 5

/* ======================================================================
 * error-free transformations
 * ==================================================================== */

/* a + b = s + e exactly (Knuth), any magnitudes. */
static void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *e = (a - av) + (b - bv);
    *s = x;
}

/* a + b = s + e exactly when |a| >= |b| (Dekker). */
static void fast_two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double z = x - a;
    *e = b - z;
    *s = x;
}

/* a * b = p + e exactly (one rounded product, one fused multiply-add). */
static void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* ======================================================================
 * double-double (Joldes, Muller, Popescu 2017)
 * ==================================================================== */

/* accurate double-word + double-word */
static void dd_add(const double *x, const double *y, double *z)
{
    double sh, sl, th, tl, c, vh, vl, w, zh, zl;
    two_sum(x[0], y[0], &sh, &sl);
    two_sum(x[1], y[1], &th, &tl);
    c = sl + th;
    fast_two_sum(sh, c, &vh, &vl);
    w = tl + vl;
    fast_two_sum(vh, w, &zh, &zl);
    z[0] = zh;
    z[1] = zl;
}

/* double-word * double-word with fused multiply-adds */
static void dd_mul(const double *x, const double *y, double *z)
{
    double ch, cl1, tl0, tl1, cl2, cl3, zh, zl;
    two_prod(x[0], y[0], &ch, &cl1);
    tl0 = x[1] * y[1];
    tl1 = fma(x[0], y[1], tl0);
    cl2 = fma(x[1], y[0], tl1);
    cl3 = cl1 + cl2;
    fast_two_sum(ch, cl3, &zh, &zl);
    z[0] = zh;
    z[1] = zl;
}

/* double-word * double */
static void dd_mul_d(const double *x, double y, double *z)
{
    double ch, cl1, cl3, zh, zl;
    two_prod(x[0], y, &ch, &cl1);
    cl3 = fma(x[1], y, cl1);
    fast_two_sum(ch, cl3, &zh, &zl);
    z[0] = zh;
    z[1] = zl;
}

/* double-word / double-word */
static void dd_div(const double *x, const double *y, double *z)
{
    double th, r[2], pih, dl, d, tl, zh, zl;
    th = x[0] / y[0];
    dd_mul_d(y, th, r);
    pih = x[0] - r[0];
    dl = x[1] - r[1];
    d = pih + dl;
    tl = d / y[0];
    fast_two_sum(th, tl, &zh, &zl);
    z[0] = zh;
    z[1] = zl;
}

/* square root: double square root s, then s + (x - s^2) / (2 s) */
static void dd_sqrt(const double *x, double *z)
{
    double s, p, e, r, c, zh, zl;
    if (x[0] == 0.0) {
        z[0] = 0.0;
        z[1] = 0.0;
        return;
    }
    s = sqrt(x[0]);
    two_prod(s, s, &p, &e);
    r = ((x[0] - p) - e) + x[1];
    c = r / (2.0 * s);
    fast_two_sum(s, c, &zh, &zl);
    z[0] = zh;
    z[1] = zl;
}

/* ======================================================================
 * quad-double (Hida, Li, Bailey 2001)
 * ==================================================================== */

/* Five overlapping words (roughly decreasing) to four non-overlapping ones.
 * First fold the words bottom-up into a leading word with exact errors,
 * then walk top-down emitting a limb each time a sum leaves a non-zero
 * error; the fourth limb absorbs whatever remains. */
static void qd_renorm5(double c0, double c1, double c2, double c3, double c4,
                       double *out)
{
    double s, t0, t[4], o[4] = {0.0, 0.0, 0.0, 0.0}, e;
    int i, k = 0;
    two_sum(c3, c4, &s, &t[3]);
    two_sum(c2, s, &s, &t[2]);
    two_sum(c1, s, &s, &t[1]);
    two_sum(c0, s, &t0, &t[0]);
    s = t0;
    for (i = 0; i < 4; i++) {
        if (k == 3) {
            s = s + t[i];
            continue;
        }
        two_sum(s, t[i], &s, &e);
        if (e != 0.0) {
            o[k++] = s;
            s = e;
        }
    }
    o[k] = s;
    for (i = 0; i < 4; i++)
        out[i] = o[i];
}

/* a + b = (s, e1, e2) exactly */
static void three_sum(double a, double b, double c, double *s, double *e1,
                      double *e2)
{
    double t1, t2, t3;
    two_sum(a, b, &t1, &t2);
    two_sum(c, t1, s, &t3);
    two_sum(t2, t3, e1, e2);
}

/* Accurate sum: merge the eight limbs by decreasing magnitude (ties take a
 * first), then add them one by one into a two-word accumulator (u, v); when
 * an addition leaves three non-zero words the leading one is emitted as the
 * next limb.  At most four limbs are emitted; a final renormalisation. */
static void qd_add(const double *a, const double *b, double *out)
{
    double x[8], u = 0.0, v = 0.0, o[4] = {0.0, 0.0, 0.0, 0.0};
    int i = 0, j = 0, q, k = 0;
    for (q = 0; q < 8; q++) {
        if (j >= 4 || (i < 4 && fabs(a[i]) >= fabs(b[j])))
            x[q] = a[i++];
        else
            x[q] = b[j++];
    }
    for (q = 0; q < 8 && k < 4; q++) {
        double s1, e1, s2, e2;
        two_sum(v, x[q], &s1, &e1);
        two_sum(u, s1, &s2, &e2);
        if (e1 != 0.0 && e2 != 0.0) {
            o[k++] = s2;
            u = e2;
            v = e1;
        } else if (e1 == 0.0) {
            u = s2;
            v = e2;
        } else {
            u = s2;
            v = e1;
        }
    }
    if (k < 4)
        o[k++] = u;
    if (k < 4)
        o[k++] = v;
    qd_renorm5(o[0], o[1], o[2], o[3], 0.0, out);
}

/* product keeping every term down to third order */
static void qd_mul(const double *a, const double *b, double *out)
{
    double p0, e0, p1, e1, p2, e2, p3, e3, p4, e4, p5, e5;
    double s1, u1, u2, s2, w1, w2, w3, w4, w5, s3;
    two_prod(a[0], b[0], &p0, &e0);
    two_prod(a[0], b[1], &p1, &e1);
    two_prod(a[1], b[0], &p2, &e2);
    two_prod(a[0], b[2], &p3, &e3);
    two_prod(a[1], b[1], &p4, &e4);
    two_prod(a[2], b[0], &p5, &e5);
    /* first order: p1 + p2 + e0 */
    three_sum(p1, p2, e0, &s1, &u1, &u2);
    /* second order: p3 + p4 + p5 + e1 + e2 + u1 */
    two_sum(p3, p4, &s2, &w1);
    two_sum(s2, p5, &s2, &w2);
    two_sum(s2, e1, &s2, &w3);
    two_sum(s2, e2, &s2, &w4);
    two_sum(s2, u1, &s2, &w5);
    /* third order, rounded */
    s3 = a[0] * b[3];
    s3 = s3 + a[1] * b[2];
    s3 = s3 + a[2] * b[1];
    s3 = s3 + a[3] * b[0];
    s3 = s3 + e3;
    s3 = s3 + e4;
    s3 = s3 + e5;
    s3 = s3 + u2;
    s3 = s3 + w1;
    s3 = s3 + w2;
    s3 = s3 + w3;
    s3 = s3 + w4;
    s3 = s3 + w5;
    qd_renorm5(p0, s1, s2, s3, 0.0, out);
}

/* quad-double * double */
static void qd_mul_d(const double *a, double d, double *out)
{
    double p0, e0, p1, e1, p2, e2, p3, s1, u, s2, v1, v2, s3;
    two_prod(a[0], d, &p0, &e0);
    two_prod(a[1], d, &p1, &e1);
    two_prod(a[2], d, &p2, &e2);
    p3 = a[3] * d;
    two_sum(p1, e0, &s1, &u);
    three_sum(p2, e1, u, &s2, &v1, &v2);
    s3 = p3 + e2;
    s3 = s3 + v1;
    s3 = s3 + v2;
    qd_renorm5(p0, s1, s2, s3, 0.0, out);
}

static void qd_neg(const double *a, double *out)
{
    int i;
    for (i = 0; i < 4; i++)
        out[i] = -a[i];
}

/* long division: four quotient digits, each from the leading remainder */
static void qd_div(const double *a, const double *b, double *out)
{
    double q[4], r[4], t[4], nt[4];
    int i;
    for (i = 0; i < 4; i++)
        r[i] = a[i];
    for (i = 0; i < 4; i++) {
        q[i] = r[0] / b[0];
        if (i == 3)
            break;
        qd_mul_d(b, q[i], t);
        qd_neg(t, nt);
        qd_add(r, nt, r);
    }
    qd_renorm5(q[0], q[1], q[2], q[3], 0.0, out);
}

/* square root: three Newton steps y += y (1 - a y^2) / 2 on 1/sqrt(a) from
 * the double estimate, then sqrt(a) = a y */
static void qd_sqrt(const double *a, double *out)
{
    double y[4] = {0.0, 0.0, 0.0, 0.0}, h[4], e[4], one[4] = {1.0, 0.0, 0.0, 0.0};
    int it;
    if (a[0] == 0.0) {
        out[0] = out[1] = out[2] = out[3] = 0.0;
        return;
    }
    y[0] = 1.0 / sqrt(a[0]);
    for (it = 0; it < 3; it++) {
        qd_mul(y, y, h);
        qd_mul(a, h, h);
        qd_neg(h, h);
        qd_add(one, h, e);
        qd_mul(y, e, e);
        qd_mul_d(e, 0.5, e);
        qd_add(y, e, y);
    }
    qd_mul(a, y, out);
}

/* ======================================================================
 * precision-generic reals: P doubles (2 or 4)
 * ==================================================================== */

typedef struct {
    double v[4];
} rr;

typedef struct {
    rr re, im;
} cc;

static rr r_zero(void)
{
    rr z;
    memset(&z, 0, sizeof z);
    return z;
}

static rr r_from_d(double d)
{
    rr z = r_zero();
    z.v[0] = d;
    return z;
}

static rr r_add(int P, rr a, rr b)
{
    rr z = r_zero();
    if (P == 1)
        z.v[0] = a.v[0] + b.v[0];
    else if (P == 2)
        dd_add(a.v, b.v, z.v);
    else
        qd_add(a.v, b.v, z.v);
    return z;
}

static rr r_neg(int P, rr a)
{
    int i;
    for (i = 0; i < P; i++)
        a.v[i] = -a.v[i];
    return a;
}

static rr r_sub(int P, rr a, rr b)
{
    return r_add(P, a, r_neg(P, b));
}

static rr r_mul(int P, rr a, rr b)
{
    rr z = r_zero();
    if (P == 1)
        z.v[0] = a.v[0] * b.v[0];
    else if (P == 2)
        dd_mul(a.v, b.v, z.v);
    else
        qd_mul(a.v, b.v, z.v);
    return z;
}

static rr r_mul_d(int P, rr a, double d)
{
    rr z = r_zero();
    if (P == 1)
        z.v[0] = a.v[0] * d;
    else if (P == 2)
        dd_mul_d(a.v, d, z.v);
    else
        qd_mul_d(a.v, d, z.v);
    return z;
}

static rr r_div(int P, rr a, rr b)
{
    rr z = r_zero();
    if (P == 1)
        z.v[0] = a.v[0] / b.v[0];
    else if (P == 2)
        dd_div(a.v, b.v, z.v);
    else
        qd_div(a.v, b.v, z.v);
    return z;
}

static rr r_sqrt(int P, rr a)
{
    rr z = r_zero();
    if (P == 1)
        z.v[0] = sqrt(a.v[0]);
    else if (P == 2)
        dd_sqrt(a.v, z.v);
    else
        qd_sqrt(a.v, z.v);
    return z;
}

static rr r_load(int P, const double *p)
{
    rr z = r_zero();
    int i;
    for (i = 0; i < P; i++)
        z.v[i] = p[i];
    return z;
}

static void r_store(int P, rr a, double *p)
{
    int i;
    for (i = 0; i < P; i++)
        p[i] = a.v[i];
}

static cc c_zero(void)
{
    cc z;
    z.re = r_zero();
    z.im = r_zero();
    return z;
}

static cc c_one(void)
{
    cc z = c_zero();
    z.re.v[0] = 1.0;
    return z;
}

static cc c_load(int P, const double *p)
{
    cc z;
    z.re = r_load(P, p);
    z.im = r_load(P, p + P);
    return z;
}

static void c_store(int P, cc a, double *p)
{
    r_store(P, a.re, p);
    r_store(P, a.im, p + P);
}

static cc c_add(int P, cc a, cc b)
{
    cc z;
    z.re = r_add(P, a.re, b.re);
    z.im = r_add(P, a.im, b.im);
    return z;
}

static cc c_neg(int P, cc a)
{
    cc z;
    z.re = r_neg(P, a.re);
    z.im = r_neg(P, a.im);
    return z;
}

static cc c_sub(int P, cc a, cc b)
{
    return c_add(P, a, c_neg(P, b));
}

/* (ar br - ai bi) + i (ar bi + ai br) */
static cc c_mul(int P, cc a, cc b)
{
    rr rr_ = r_mul(P, a.re, b.re);
    rr ii = r_mul(P, a.im, b.im);
    rr ri = r_mul(P, a.re, b.im);
    rr ir = r_mul(P, a.im, b.re);
    cc z;
    z.re = r_sub(P, rr_, ii);
    z.im = r_add(P, ri, ir);
    return z;
}

/* conj(a) * b = (ar br + ai bi) + i (ar bi - ai br) */
static cc c_mul_conj(int P, cc a, cc b)
{
    rr rr_ = r_mul(P, a.re, b.re);
    rr ii = r_mul(P, a.im, b.im);
    rr ri = r_mul(P, a.re, b.im);
    rr ir = r_mul(P, a.im, b.re);
    cc z;
    z.re = r_add(P, rr_, ii);
    z.im = r_sub(P, ri, ir);
    return z;
}

/* |a|^2 = ar ar + ai ai */
static rr c_norm2(int P, cc a)
{
    return r_add(P, r_mul(P, a.re, a.re), r_mul(P, a.im, a.im));
}

/* real scaling: (s ar) + i (s ai) */
static cc c_scale(int P, rr s, cc a)
{
    cc z;
    z.re = r_mul(P, s, a.re);
    z.im = r_mul(P, s, a.im);
    return z;
}

static cc c_scale_d(int P, cc a, double d)
{
    cc z;
    z.re = r_mul_d(P, a.re, d);
    z.im = r_mul_d(P, a.im, d);
    return z;
}

/* infinity norm over the leading limbs of real and imaginary parts;
 * returns NaN when any leading limb is NaN */
static double lead_norm(int P, int len, const double *z)
{
    double m = 0.0;
    int i;
    for (i = 0; i < len; i++) {
        double a = fabs(z[(size_t)i * 2 * P]);
        double b = fabs(z[(size_t)i * 2 * P + P]);
        if (a != a || b != b)
            return NAN;
        if (a > m)
            m = a;
        if (b > m)
            m = b;
    }
    return m;
}

/* ======================================================================
 * elementwise entry points (for bitwise parity of the arithmetic layer)
 * ==================================================================== */

enum {
    OP_ADD = 0, OP_SUB = 1, OP_MUL = 2, OP_DIV = 3, OP_SQRT = 4, OP_MUL_D = 5,
    OP_CADD = 10, OP_CSUB = 11, OP_CMUL = 12, OP_CMUL_CONJ = 13,
    OP_CNORM2 = 14, OP_CSCALE = 15,
    OP_TWO_SUM = 20, OP_FAST_TWO_SUM = 21, OP_TWO_PROD = 22
};

int ora_elementwise(int op, int P, int count, const double *a, const double *b,
                    double *out)
{
    int q;
    if (P != 1 && P != 2 && P != 4 && op < 20)
        return ORA_EINVAL;
    for (q = 0; q < count; q++) {
        switch (op) {
        case OP_ADD: case OP_SUB: case OP_MUL: case OP_DIV: {
            rr x = r_load(P, a + (size_t)q * P), y = r_load(P, b + (size_t)q * P), z;
            z = op == OP_ADD ? r_add(P, x, y) : op == OP_SUB ? r_sub(P, x, y)
              : op == OP_MUL ? r_mul(P, x, y) : r_div(P, x, y);
            r_store(P, z, out + (size_t)q * P);
            break;
        }
        case OP_SQRT:
            r_store(P, r_sqrt(P, r_load(P, a + (size_t)q * P)), out + (size_t)q * P);
            break;
        case OP_MUL_D:
            r_store(P, r_mul_d(P, r_load(P, a + (size_t)q * P), b[q]),
                    out + (size_t)q * P);
            break;
        case OP_CADD: case OP_CSUB: case OP_CMUL: case OP_CMUL_CONJ: {
            cc x = c_load(P, a + (size_t)q * 2 * P), y = c_load(P, b + (size_t)q * 2 * P), z;
            z = op == OP_CADD ? c_add(P, x, y) : op == OP_CSUB ? c_sub(P, x, y)
              : op == OP_CMUL ? c_mul(P, x, y) : c_mul_conj(P, x, y);
            c_store(P, z, out + (size_t)q * 2 * P);
            break;
        }
        case OP_CNORM2:
            r_store(P, c_norm2(P, c_load(P, a + (size_t)q * 2 * P)), out + (size_t)q * P);
            break;
        case OP_CSCALE:
            c_store(P, c_scale(P, r_load(P, b + (size_t)q * P), c_load(P, a + (size_t)q * 2 * P)),
                    out + (size_t)q * 2 * P);
            break;
        case OP_TWO_SUM:
            two_sum(a[q], b[q], out + 2 * (size_t)q, out + 2 * (size_t)q + 1);
            break;
        case OP_FAST_TWO_SUM:
            fast_two_sum(a[q], b[q], out + 2 * (size_t)q, out + 2 * (size_t)q + 1);
            break;
        case OP_TWO_PROD:
            two_prod(a[q], b[q], out + 2 * (size_t)q, out + 2 * (size_t)q + 1);
            break;
        default:
            return ORA_EINVAL;
        }
    }
    return ORA_OK;
}

/* ======================================================================
 * polynomial systems
 * ==================================================================== */

typedef struct {
    int N, n, P;
    const int32_t *eq_ptr;   /* N+1 */
    const int32_t *mon_ptr;  /* nmon+1 */
    const int32_t *var;
    const int32_t *exp;
    const double *coef;      /* [nmon][2][P] */
} ora_sys;

/* f (N complex) and the column-major Jacobian J[k][i] = df_i/dx_k, each by
 * its definition: f_i = sum_m c_m prod_l x_l^a_l and
 * df_i/dx_k = sum_{m containing x_k} c_m a_k x_k^(a_k - 1) prod_{l != k} x_l^a_l.
 * Every partial is computed on its own with left-to-right products; the
 * sums run in ascending monomial order.  J may be NULL. */
int ora_eval(const ora_sys *S, const double *x, double *f, double *J)
{
    const int P = S->P, N = S->N, n = S->n;
    const size_t W = 2 * (size_t)P;
    int i, m, q, r, e;
    cc *xs;
    if (P != 1 && P != 2 && P != 4)
        return ORA_EINVAL;
    xs = (cc *)malloc(sizeof(cc) * (size_t)(n > 0 ? n : 1));
    if (!xs)
        return ORA_ENOMEM;
    for (i = 0; i < n; i++)
        xs[i] = c_load(P, x + i * W);
    if (J)
        memset(J, 0, sizeof(double) * (size_t)n * N * W);
    for (i = 0; i < N; i++) {
        cc fi = c_zero();
        for (m = S->eq_ptr[i]; m < S->eq_ptr[i + 1]; m++) {
            const int a0 = S->mon_ptr[m], a1 = S->mon_ptr[m + 1];
            cc c = c_load(P, S->coef + (size_t)m * W);
            cc val = c;
            for (q = a0; q < a1; q++)
                for (e = 0; e < S->exp[q]; e++)
                    val = c_mul(P, val, xs[S->var[q]]);
            fi = c_add(P, fi, val);
            if (!J)
                continue;
            for (q = a0; q < a1; q++) {
                const int k = S->var[q];
                cc d = c_scale_d(P, c, (double)S->exp[q]);
                for (r = a0; r < a1; r++) {
                    int pw = S->exp[r] - (r == q ? 1 : 0);
                    for (e = 0; e < pw; e++)
                        d = c_mul(P, d, xs[S->var[r]]);
                }
                {
                    double *dst = J + ((size_t)k * N + i) * W;
                    c_store(P, c_add(P, c_load(P, dst), d), dst);
                }
            }
        }
        c_store(P, fi, f + i * W);
    }
    free(xs);
    return ORA_OK;
}

/* homotopy h = gamma (1-t)^k g + t^k f and J_h = gamma (1-t)^k J_g + t^k J_f
 * (equation (1)).  G == NULL: h = f, J_h = J_f. */
int ora_eval_h(const ora_sys *F, const ora_sys *G, const double *gamma,
               int relax_k, double t, const double *x, double *h, double *Jh)
{
    const int P = F->P, N = F->N, n = F->n;
    const size_t W = 2 * (size_t)P;
    double *fg, *Jg;
    rr one_minus_t, sf, pw;
    cc sg;
    size_t q;
    int rc, j;
    rc = ora_eval(F, x, h, Jh);
    if (rc || !G)
        return rc;
    if (G->N != N || G->n != n || G->P != P || relax_k < 1)
        return ORA_EINVAL;
    fg = (double *)malloc(sizeof(double) * (size_t)N * W);
    Jg = (double *)malloc(sizeof(double) * (size_t)n * N * W);
    if (!fg || !Jg) {
        free(fg);
        free(Jg);
        return ORA_ENOMEM;
    }
    rc = ora_eval(G, x, fg, Jg);
    if (rc) {
        free(fg);
        free(Jg);
        return rc;
    }
    /* (1 - t) exactly as a two-word number, then the powers */
    {
        double s, e;
        two_sum(1.0, -t, &s, &e);
        one_minus_t = r_zero();
        one_minus_t.v[0] = s;
        one_minus_t.v[1] = e;
    }
    pw = one_minus_t;
    sf = r_from_d(t);
    for (j = 1; j < relax_k; j++) {
        pw = r_mul(P, pw, one_minus_t);
        sf = r_mul(P, sf, r_from_d(t));
    }
    sg = c_scale(P, pw, c_load(P, gamma));
    for (q = 0; q < (size_t)N; q++) {
        cc a = c_mul(P, sg, c_load(P, fg + q * W));
        cc b = c_scale(P, sf, c_load(P, h + q * W));
        c_store(P, c_add(P, a, b), h + q * W);
    }
    for (q = 0; q < (size_t)N * n; q++) {
        cc a = c_mul(P, sg, c_load(P, Jg + q * W));
        cc b = c_scale(P, sf, c_load(P, Jh + q * W));
        c_store(P, c_add(P, a, b), Jh + q * W);
    }
    free(fg);
    free(Jg);
    return ORA_OK;
}

/* ======================================================================
 * modified Gram-Schmidt on the augmented matrix [A | b], back substitution
 * ==================================================================== */

/* A: column-major N x n ([n][N][2][P]), overwritten by Q.  b: [N][2][P],
 * overwritten by its projections.  dx: [n][2][P].  R (may be NULL):
 * column-major [n+1][n][2][P], column j holds r_kj for k <= j (k < n);
 * column n holds y = Q^H b.  For k = 0..n-1: r_kk = ||a_k||_2,
 * q_k = a_k (1/r_kk), and for j > k (the column b last):
 * r_kj = q_k^H a_j, a_j -= r_kj q_k.  Then dx_k = (y_k - sum_{j>k} r_kj dx_j)
 * (1/r_kk) for k = n-1..0, the sum in ascending j. */
int ora_mgs_solve(int P, int N, int n, double *A, double *b, double *dx, double *R)
{
    const size_t W = 2 * (size_t)P;
    int i, j, k;
    rr *inv;
    cc *Rl;
    if ((P != 1 && P != 2 && P != 4) || n < 1 || N < n)
        return ORA_EINVAL;
    inv = (rr *)malloc(sizeof(rr) * (size_t)n);
    Rl = (cc *)malloc(sizeof(cc) * (size_t)(n + 1) * n);
    if (!inv || !Rl) {
        free(inv);
        free(Rl);
        return ORA_ENOMEM;
    }
#define ACOL(j) ((j) < n ? A + (size_t)(j) * N * W : b)
    for (j = 0; j < (n + 1) * n; j++)
        Rl[j] = c_zero();
    for (k = 0; k < n; k++) {
        double *ak = ACOL(k);
        rr s = r_zero(), rkk;
        for (i = 0; i < N; i++)
            s = r_add(P, s, c_norm2(P, c_load(P, ak + i * W)));
        rkk = r_sqrt(P, s);
        if (!(rkk.v[0] > 0.0) || !isfinite(rkk.v[0])) {
            free(inv);
            free(Rl);
            return ORA_ESINGULAR;
        }
        inv[k] = r_div(P, r_from_d(1.0), rkk);
        Rl[(size_t)k * n + k].re = rkk;
        for (i = 0; i < N; i++)
            c_store(P, c_scale(P, inv[k], c_load(P, ak + i * W)), ak + i * W);
        /* the columns j > k are independent of each other: large problems
         * spread them over threads (each column's operations, and so its
         * bits, are those of the serial loop) */
#pragma omp parallel for private(i) schedule(static) if ((size_t)N * (size_t)(n - k) >= 65536)
        for (j = k + 1; j <= n; j++) {
            double *aj = ACOL(j);
            cc r = c_zero();
            for (i = 0; i < N; i++)
                r = c_add(P, r, c_mul_conj(P, c_load(P, ak + i * W), c_load(P, aj + i * W)));
            Rl[(size_t)j * n + k] = r;
            for (i = 0; i < N; i++) {
                cc v = c_sub(P, c_load(P, aj + i * W), c_mul(P, r, c_load(P, ak + i * W)));
                c_store(P, v, aj + i * W);
            }
        }
    }
#undef ACOL
    for (k = n - 1; k >= 0; k--) {
        cc s = c_zero();
        for (j = k + 1; j < n; j++)
            s = c_add(P, s, c_mul(P, Rl[(size_t)j * n + k], c_load(P, dx + j * W)));
        c_store(P, c_scale(P, inv[k], c_sub(P, Rl[(size_t)n * n + k], s)), dx + k * W);
    }
    if (R)
        for (j = 0; j < (n + 1) * n; j++)
            c_store(P, Rl[j], R + (size_t)j * W);
    free(inv);
    free(Rl);
    return ORA_OK;
}

/* ======================================================================
 * the corrector (Section 2, equations (2) and (3); Fig. 2) and the
 * increment-and-fix tracker (equation (4); Fig. 3)
 * ==================================================================== */

typedef struct {
    int max_iter;
    double tol_res, tol_dx, max_eq_val;
} ora_newton_params;

typedef struct {
    int status;       /* ORA_OK = success, or a failure code */
    int iters;        /* evaluations performed */
    double res_norm;  /* last residual norm evaluated */
    double dx_norm;   /* last update norm, 0 if none */
} ora_newton_result;

/* What the corrector does next. */
typedef enum { CORR_EVALUATE, CORR_SOLVE, CORR_STOP } corr_phase;

/* Verdict on a residual norm r when the previous accepted residual (or
 * max_eq_val before the first) is `ceiling`: NaN stops, growth beyond the
 * ceiling is divergence, a residual under the tolerance is convergence;
 * -1 means keep going.  Norms are infinity norms of the leading limbs,
 * taken in double (the magnitude is all that matters). */
static int judge_residual(double r, double ceiling, double tol)
{
    if (r != r)
        return ORA_NAN;
    if (r > ceiling)
        return ORA_DIVERGED;
    if (r < tol)
        return ORA_OK;
    return -1;
}

/* Verdict on the size d of the update just applied. */
static int judge_update(double d, double tol)
{
    if (d != d)
        return ORA_NAN;
    if (d < tol)
        return ORA_OK;
    return -1;
}

/* Newton's method as a small machine with two phases.  EVALUATE forms the
 * residual h and the Jacobian at z and judges the residual (equation (3),
 * the backward error); SOLVE finds dz from J dz = -h, adds it to z and
 * judges the update (the forward error).  The residual of an iteration may
 * not exceed the one before it, which starts at max_eq_val.  Either test
 * ends the corrector with success; running out of evaluations ends it
 * unconverged. */
int ora_newton(const ora_sys *F, const ora_sys *G, const double *gamma,
               int relax_k, double t, double *z, const ora_newton_params *prm,
               ora_newton_result *res)
{
    const int P = F->P, N = F->N, n = F->n;
    const size_t W = 2 * (size_t)P;
    double *h, *J, *dz, ceiling = prm->max_eq_val, r_now = 0.0;
    int verdict = ORA_NOT_CONVERGED, q;
    corr_phase phase = CORR_EVALUATE;
    res->iters = 0;
    res->res_norm = 0.0;
    res->dx_norm = 0.0;
    h = (double *)malloc(sizeof(double) * (size_t)N * W);
    J = (double *)malloc(sizeof(double) * (size_t)N * n * W);
    dz = (double *)malloc(sizeof(double) * (size_t)n * W);
    if (!h || !J || !dz) {
        free(h); free(J); free(dz);
        return res->status = ORA_ENOMEM;
    }
    while (phase != CORR_STOP) {
        if (phase == CORR_EVALUATE) {
            int e, v;
            if (res->iters >= prm->max_iter) {
                verdict = ORA_NOT_CONVERGED;
                phase = CORR_STOP;
                continue;
            }
            e = ora_eval_h(F, G, gamma, relax_k, t, z, h, J);
            if (e) {
                verdict = e;
                phase = CORR_STOP;
                continue;
            }
            res->iters++;
            r_now = lead_norm(P, N, h);
            res->res_norm = r_now;
            v = judge_residual(r_now, ceiling, prm->tol_res);
            if (v >= 0) {
                verdict = v;
                phase = CORR_STOP;
            } else {
                phase = CORR_SOLVE;
            }
        } else {
            double d;
            int e, v;
            for (q = 0; q < N; q++)
                c_store(P, c_neg(P, c_load(P, h + q * W)), h + q * W);
            e = ora_mgs_solve(P, N, n, J, h, dz, NULL);
            if (e) {
                verdict = e;
                phase = CORR_STOP;
                continue;
            }
            d = lead_norm(P, n, dz);
            res->dx_norm = d;
            if (d != d) {
                verdict = ORA_NAN;  /* z is left as it was */
                phase = CORR_STOP;
                continue;
            }
            for (q = 0; q < n; q++)
                c_store(P, c_add(P, c_load(P, z + q * W), c_load(P, dz + q * W)), z + q * W);
            v = judge_update(d, prm->tol_dx);
            if (v >= 0) {
                verdict = v;
                phase = CORR_STOP;
            } else {
                ceiling = r_now;
                phase = CORR_EVALUATE;
            }
        }
    }
    free(h);
    free(J);
    free(dz);
    return res->status = verdict;
}

/* one Newton iteration without tests: evaluate, solve, update.  norms[0] =
 * residual norm before the update, norms[1] = update norm. */
int ora_newton_step(const ora_sys *F, const ora_sys *G, const double *gamma,
                    int relax_k, double t, double *x, double *norms)
{
    const int P = F->P, N = F->N, n = F->n;
    const size_t W = 2 * (size_t)P;
    double *h, *J, *dx;
    int e, q;
    h = (double *)malloc(sizeof(double) * (size_t)N * W);
    J = (double *)malloc(sizeof(double) * (size_t)N * n * W);
    dx = (double *)malloc(sizeof(double) * (size_t)n * W);
    if (!h || !J || !dx) {
        free(h); free(J); free(dx);
        return ORA_ENOMEM;
    }
    e = ora_eval_h(F, G, gamma, relax_k, t, x, h, J);
    if (!e) {
        norms[0] = lead_norm(P, N, h);
        for (q = 0; q < N; q++)
            c_store(P, c_neg(P, c_load(P, h + q * W)), h + q * W);
        e = ora_mgs_solve(P, N, n, J, h, dx, NULL);
    }
    if (!e) {
        norms[1] = lead_norm(P, n, dx);
        for (q = 0; q < n; q++)
            c_store(P, c_add(P, c_load(P, x + q * W), c_load(P, dx + q * W)), x + q * W);
    }
    free(h);
    free(J);
    free(dx);
    return e;
}

#define ORA_MAX_ORDER 4

/* The predictor of Section 3.1: the polynomial of degree d through the
 * points (ts[j], xs[j]), j = 0..d, evaluated at t, coordinate by
 * coordinate, in Lagrange form: x(t) = sum_j w_j xs[j] with
 * w_j = prod_{m != j} (t - ts[m]) / prod_{m != j} (ts[j] - ts[m]).
 * Each weight is its numerator product (m ascending) over its denominator
 * product, in the working precision from the double differences; the sum
 * runs over j ascending.  d = 0 copies xs[0].  xs: [d+1][n][2][P]. */
int ora_predict(int P, int n, int d, const double *ts, const double *xs, double t,
                double *out)
{
    const size_t W = 2 * (size_t)P;
    rr w[ORA_MAX_ORDER + 1];
    int i, j, m;
    if ((P != 1 && P != 2 && P != 4) || n < 0 || d < 0 || d > ORA_MAX_ORDER)
        return ORA_EINVAL;
    for (j = 0; j <= d; j++) {
        rr num = r_from_d(1.0), den = r_from_d(1.0);
        int first = 1;
        for (m = 0; m <= d; m++) {
            if (m == j)
                continue;
            if (first) {
                num = r_from_d(t - ts[m]);
                den = r_from_d(ts[j] - ts[m]);
                first = 0;
            } else {
                num = r_mul(P, num, r_from_d(t - ts[m]));
                den = r_mul(P, den, r_from_d(ts[j] - ts[m]));
            }
        }
        w[j] = d == 0 ? r_from_d(1.0) : r_div(P, num, den);
    }
    for (i = 0; i < n; i++) {
        cc acc;
        if (d == 0) {
            acc = c_load(P, xs + (size_t)i * W);
        } else {
            acc = c_scale(P, w[0], c_load(P, xs + (size_t)i * W));
            for (j = 1; j <= d; j++)
                acc = c_add(P, acc, c_scale(P, w[j], c_load(P, xs + ((size_t)j * n + i) * W)));
        }
        c_store(P, acc, out + (size_t)i * W);
    }
    return ORA_OK;
}

typedef struct {
    int max_iter;
    double tol_res, tol_dx, max_eq_val, max_dt, min_dt;
    int max_steps, end_iters;
    double end_tol;
    int predictor_order;
} ora_track_params;

typedef struct {
    int status, steps, newton_iters, end_iters, end_status, accepted;
    double t, res_norm, dx_norm;
} ora_path_result;

/* What the tracker does next. */
typedef enum { TRK_ADVANCE, TRK_PREDICT_CORRECT, TRK_REFINE, TRK_DONE } trk_phase;

/* Increment-and-fix continuation of the homotopy (equation (1)) along one
 * path, with the step bounds of equation (4), as a machine:
 *   ADVANCE: give up once more than max_steps steps were taken; otherwise
 *     the trial parameter is the last accepted t plus dt, clipped at 1;
 *   PREDICT_CORRECT: extrapolate the path to the trial t through the last
 *     accepted points (Section 3.1: degree up to predictor_order, one less
 *     than the points known) and correct with Newton's method.  Success
 *     accepts the point and counts a success; once the run of successes is
 *     longer than two, each further success doubles dt up to max_dt.
 *     Failure ends the run (count 0) and halves dt; below min_dt the path
 *     is given up.  Either way one step is counted.  Accepting t = 1 moves
 *     on to REFINE;
 *   REFINE: Newton's method at t = 1 with end_tol and end_iters.
 * Readings of the paper: a failed step leaves the accepted (t, x) in place
 * and the next trial starts from it; a NaN residual or update ends the
 * path.  trace (optional, trace_cap rows of 4 doubles): per step the trial
 * t, the dt that produced it, 1 for accepted / 0 for rejected, and the
 * corrector's evaluations. */
int ora_track_trace(const ora_sys *F, const ora_sys *G, const double *gamma,
                    int relax_k, const double *x0, const ora_track_params *prm,
                    double *x_out, ora_path_result *out, double *trace, int trace_cap)
{
    const int P = F->P, n = F->n;
    const size_t W = 2 * (size_t)P;
    const size_t xb = sizeof(double) * (size_t)n * W;
    const int order = prm->predictor_order < 0 ? 0
                    : prm->predictor_order > ORA_MAX_ORDER ? ORA_MAX_ORDER : prm->predictor_order;
    /* the accepted points, newest first: hist_t[j], hist_x + j n W */
    double hist_t[ORA_MAX_ORDER + 1], *hist_x, *z;
    double dt = prm->max_dt, t_try = 0.0;
    int known = 1, run = 0, status = ORA_OK, j;
    trk_phase phase = TRK_ADVANCE;
    ora_newton_params np;
    ora_newton_result nr;
    memset(out, 0, sizeof *out);
    if (order > ORA_MAX_ORDER)
        return out->status = ORA_EINVAL;
    hist_x = (double *)malloc(xb * (ORA_MAX_ORDER + 1));
    z = (double *)malloc(xb);
    if (!hist_x || !z) {
        free(hist_x); free(z);
        return out->status = ORA_ENOMEM;
    }
    hist_t[0] = 0.0;
    memcpy(hist_x, x0, xb);
    np.max_iter = prm->max_iter;
    np.tol_res = prm->tol_res;
    np.tol_dx = prm->tol_dx;
    np.max_eq_val = prm->max_eq_val;
    while (phase != TRK_DONE) {
        switch (phase) {
        case TRK_ADVANCE:
            if (hist_t[0] >= 1.0) {
                phase = TRK_REFINE;
            } else if (out->steps > prm->max_steps) {
                status = ORA_MAX_STEPS;
                phase = TRK_DONE;
            } else {
                t_try = hist_t[0] + dt;
                if (t_try > 1.0)
                    t_try = 1.0;
                phase = TRK_PREDICT_CORRECT;
            }
            break;
        case TRK_PREDICT_CORRECT: {
            const int deg = known - 1 < order ? known - 1 : order;
            int rc, accepted;
            ora_predict(P, n, deg, hist_t, hist_x, t_try, z);
            rc = ora_newton(F, G, gamma, relax_k, t_try, z, &np, &nr);
            out->newton_iters += nr.iters;
            out->res_norm = nr.res_norm;
            out->dx_norm = nr.dx_norm;
            accepted = rc == ORA_OK;
            if (trace && out->steps < trace_cap) {
                double *row = trace + 4 * (size_t)out->steps;
                row[0] = t_try;
                row[1] = dt;
                row[2] = accepted;
                row[3] = nr.iters;
            }
            out->steps++;
            if (rc == ORA_NAN || rc == ORA_EINVAL || rc == ORA_ENOMEM) {
                status = rc;
                phase = TRK_DONE;
                break;
            }
            if (accepted) {
                for (j = ORA_MAX_ORDER; j > 0; j--) {
                    hist_t[j] = hist_t[j - 1];
                    memcpy(hist_x + (size_t)j * n * W, hist_x + (size_t)(j - 1) * n * W, xb);
                }
                hist_t[0] = t_try;
                memcpy(hist_x, z, xb);
                if (known < ORA_MAX_ORDER + 1)
                    known++;
                out->accepted++;
                run++;
                if (run > 2)
                    dt = 2.0 * dt > prm->max_dt ? prm->max_dt : 2.0 * dt;
                phase = TRK_ADVANCE;
            } else {
                run = 0;
                dt = 0.5 * dt;
                phase = dt < prm->min_dt ? TRK_DONE : TRK_ADVANCE;
                if (phase == TRK_DONE)
                    status = ORA_STEP_TOO_SMALL;
            }
            break;
        }
        case TRK_REFINE:
            memcpy(z, hist_x, xb);
            if (prm->end_iters > 0) {
                ora_newton_params ep = np;
                ep.max_iter = prm->end_iters;
                ep.tol_res = prm->end_tol;
                ep.tol_dx = prm->end_tol;
                ora_newton(F, G, gamma, relax_k, 1.0, z, &ep, &nr);
                out->end_iters = nr.iters;
                out->end_status = nr.status;
                out->res_norm = nr.res_norm;
                out->dx_norm = nr.dx_norm;
            }
            phase = TRK_DONE;
            break;
        default:
            phase = TRK_DONE;
            break;
        }
    }
    out->t = hist_t[0];
    memcpy(x_out, status == ORA_OK ? z : hist_x, xb);
    free(hist_x);
    free(z);
    return out->status = status;
}

int ora_track(const ora_sys *F, const ora_sys *G, const double *gamma,
              int relax_k, const double *x0, const ora_track_params *prm,
              double *x_out, ora_path_result *out)
{
    return ora_track_trace(F, G, gamma, relax_k, x0, prm, x_out, out, NULL, 0);
}

/* accurate sum helper exposed for tests: sum of count reals in order */
int ora_sum(int P, int count, const double *a, double *out)
{
    rr s = r_zero();
    int q;
    for (q = 0; q < count; q++)
        s = r_add(P, s, r_load(P, a + (size_t)q * P));
    r_store(P, s, out);
    return ORA_OK;
}
