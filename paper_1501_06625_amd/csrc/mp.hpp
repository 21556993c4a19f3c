// mp.hpp -- device double-double / quad-double real and complex arithmetic
// for gfx950 (FP64 VALU; no matrix cores: every operation needs its own
// rounding).  Compiled with -ffp-contract=off: the only fused multiply-adds
// are the explicit __builtin_fma calls below, so the operation sequences are
// exactly the published ones:
//   TwoSum (Knuth), FastTwoSum (Dekker), TwoProd by fused multiply-add;
//   DD: Joldes, Muller & Popescu (ACM TOMS 2017) accurate double-word sum,
//       FMA double-word product, double-word times double and quotient;
//       square root by one Newton correction of the double square root
//       (Karp & Markstein 1997);
//   QD: Hida, Li & Bailey (ARITH-15, 2001): renormalisation, accurate sum
//       (merge by magnitude, accumulation in a two-word accumulator),
//       product down to third-order terms, long division, square root by
//       Newton iteration on the inverse square root.
// Complex products use the four-multiplication form.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define HCN_DEV __device__ __forceinline__

namespace hcn {

// ---------------------------------------------------------------------------
// error-free transformations
// ---------------------------------------------------------------------------

HCN_DEV void eft_sum(double a, double b, double &s, double &e) {
    const double x = a + b;
    const double bv = x - a;
    const double av = x - bv;
    e = (a - av) + (b - bv);
    s = x;
}

HCN_DEV void eft_fast_sum(double a, double b, double &s, double &e) {
    const double x = a + b;
    e = b - (x - a);
    s = x;
}

HCN_DEV void eft_prod(double a, double b, double &p, double &e) {
    const double x = a * b;
    e = __builtin_fma(a, b, -x);
    p = x;
}

// ---------------------------------------------------------------------------
// double-double
// ---------------------------------------------------------------------------

struct dd {
    double hi, lo;
};

HCN_DEV dd dd_make(double h) { return dd{h, 0.0}; }

HCN_DEV dd operator-(const dd &a) { return dd{-a.hi, -a.lo}; }

HCN_DEV dd add(const dd &x, const dd &y) {
    double sh, sl, th, tl, vh, vl, zh, zl;
    eft_sum(x.hi, y.hi, sh, sl);
    eft_sum(x.lo, y.lo, th, tl);
    const double c = sl + th;
    eft_fast_sum(sh, c, vh, vl);
    const double w = tl + vl;
    eft_fast_sum(vh, w, zh, zl);
    return dd{zh, zl};
}

HCN_DEV dd sub(const dd &x, const dd &y) { return add(x, -y); }

HCN_DEV dd mul(const dd &x, const dd &y) {
    double ch, cl1, zh, zl;
    eft_prod(x.hi, y.hi, ch, cl1);
    const double tl0 = x.lo * y.lo;
    const double tl1 = __builtin_fma(x.hi, y.lo, tl0);
    const double cl2 = __builtin_fma(x.lo, y.hi, tl1);
    const double cl3 = cl1 + cl2;
    eft_fast_sum(ch, cl3, zh, zl);
    return dd{zh, zl};
}

HCN_DEV dd mul_d(const dd &x, double y) {
    double ch, cl1, zh, zl;
    eft_prod(x.hi, y, ch, cl1);
    const double cl3 = __builtin_fma(x.lo, y, cl1);
    eft_fast_sum(ch, cl3, zh, zl);
    return dd{zh, zl};
}

HCN_DEV dd div(const dd &x, const dd &y) {
    const double th = x.hi / y.hi;
    const dd r = mul_d(y, th);
    const double pih = x.hi - r.hi;
    const double dl = x.lo - r.lo;
    const double d = pih + dl;
    const double tl = d / y.hi;
    double zh, zl;
    eft_fast_sum(th, tl, zh, zl);
    return dd{zh, zl};
}

HCN_DEV dd sqrt(const dd &x) {
    if (x.hi == 0.0) return dd{0.0, 0.0};
    const double s = ::sqrt(x.hi);
    double p, e, zh, zl;
    eft_prod(s, s, p, e);
    const double r = ((x.hi - p) - e) + x.lo;
    const double c = r / (2.0 * s);
    eft_fast_sum(s, c, zh, zl);
    return dd{zh, zl};
}

HCN_DEV double lead(const dd &a) { return a.hi; }

// ---------------------------------------------------------------------------
// quad-double
// ---------------------------------------------------------------------------

struct qd {
    double c0, c1, c2, c3;
};

HCN_DEV qd qd_make(double h) { return qd{h, 0.0, 0.0, 0.0}; }

HCN_DEV qd operator-(const qd &a) { return qd{-a.c0, -a.c1, -a.c2, -a.c3}; }

// three words to one rounded sum and two exact errors
HCN_DEV void eft_three(double a, double b, double c, double &s, double &e1, double &e2) {
    double t1, t2, t3;
    eft_sum(a, b, t1, t2);
    eft_sum(c, t1, s, t3);
    eft_sum(t2, t3, e1, e2);
}

// Renormalise five roughly decreasing words into four limbs: fold bottom-up
// into a leading word with exact errors, then emit top-down a limb whenever
// a sum leaves a non-zero error; the fourth limb absorbs the rest.
HCN_DEV qd renorm(double w0, double w1, double w2, double w3, double w4) {
    double s, t0, t1, t2, t3, t4;
    eft_sum(w3, w4, s, t4);
    eft_sum(w2, s, s, t3);
    eft_sum(w1, s, s, t2);
    eft_sum(w0, s, t0, t1);
    double o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0;
    int k = 0;
    s = t0;
    const double ts[4] = {t1, t2, t3, t4};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double ss, e;
        eft_sum(s, ts[i], ss, e);
        const bool emit = (k != 3) && (e != 0.0);
        o0 = (emit && k == 0) ? ss : o0;
        o1 = (emit && k == 1) ? ss : o1;
        o2 = (emit && k == 2) ? ss : o2;
        s = emit ? e : ss;
        k += emit ? 1 : 0;
    }
    o0 = (k == 0) ? s : o0;
    o1 = (k == 1) ? s : o1;
    o2 = (k == 2) ? s : o2;
    o3 = (k == 3) ? s : o3;
    return qd{o0, o1, o2, o3};
}

// Accurate sum: merge the eight limbs by decreasing magnitude (ties take x
// first), add them in that order into a two-word accumulator, emitting the
// leading word as a limb when three non-zero words remain; at most four
// limbs, then renormalise.
HCN_DEV qd add(const qd &x, const qd &y) {
    double a0 = x.c0, a1 = x.c1, a2 = x.c2, a3 = x.c3;
    double b0 = y.c0, b1 = y.c1, b2 = y.c2, b3 = y.c3;
    int na = 0, nb = 0;
    double u = 0.0, v = 0.0, o0 = 0.0, o1 = 0.0, o2 = 0.0, o3 = 0.0;
    int k = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const bool ta = (nb >= 4) || (na < 4 && fabs(a0) >= fabs(b0));
        const double w = ta ? a0 : b0;
        a0 = ta ? a1 : a0;
        a1 = ta ? a2 : a1;
        a2 = ta ? a3 : a2;
        b0 = ta ? b0 : b1;
        b1 = ta ? b1 : b2;
        b2 = ta ? b2 : b3;
        na += ta ? 1 : 0;
        nb += ta ? 0 : 1;
        double s1, e1, s2, e2;
        eft_sum(v, w, s1, e1);
        eft_sum(u, s1, s2, e2);
        const bool live = k < 4;
        const bool emit = live && (e1 != 0.0) && (e2 != 0.0);
        o0 = (emit && k == 0) ? s2 : o0;
        o1 = (emit && k == 1) ? s2 : o1;
        o2 = (emit && k == 2) ? s2 : o2;
        o3 = (emit && k == 3) ? s2 : o3;
        const double nu = emit ? e2 : s2;
        const double nv = emit ? e1 : ((e1 == 0.0) ? e2 : e1);
        u = live ? nu : u;
        v = live ? nv : v;
        k += emit ? 1 : 0;
    }
    // leftover accumulator words
    o0 = (k == 0) ? u : o0;
    o1 = (k == 1) ? u : o1;
    o2 = (k == 2) ? u : o2;
    o3 = (k == 3) ? u : o3;
    k += (k < 4) ? 1 : 0;
    o1 = (k == 1) ? v : o1;
    o2 = (k == 2) ? v : o2;
    o3 = (k == 3) ? v : o3;
    return renorm(o0, o1, o2, o3, 0.0);
}

HCN_DEV qd sub(const qd &x, const qd &y) { return add(x, -y); }

HCN_DEV qd mul(const qd &a, const qd &b) {
    double p0, e0, p1, e1, p2, e2, p3, e3, p4, e4, p5, e5;
    eft_prod(a.c0, b.c0, p0, e0);
    eft_prod(a.c0, b.c1, p1, e1);
    eft_prod(a.c1, b.c0, p2, e2);
    eft_prod(a.c0, b.c2, p3, e3);
    eft_prod(a.c1, b.c1, p4, e4);
    eft_prod(a.c2, b.c0, p5, e5);
    // first-order terms
    double s1, u1, u2;
    eft_three(p1, p2, e0, s1, u1, u2);
    // second-order terms
    double s2, w1, w2, w3, w4, w5;
    eft_sum(p3, p4, s2, w1);
    eft_sum(s2, p5, s2, w2);
    eft_sum(s2, e1, s2, w3);
    eft_sum(s2, e2, s2, w4);
    eft_sum(s2, u1, s2, w5);
    // third-order terms, rounded, in a fixed order
    double s3 = a.c0 * b.c3;
    s3 = s3 + a.c1 * b.c2;
    s3 = s3 + a.c2 * b.c1;
    s3 = s3 + a.c3 * b.c0;
    s3 = s3 + e3;
    s3 = s3 + e4;
    s3 = s3 + e5;
    s3 = s3 + u2;
    s3 = s3 + w1;
    s3 = s3 + w2;
    s3 = s3 + w3;
    s3 = s3 + w4;
    s3 = s3 + w5;
    return renorm(p0, s1, s2, s3, 0.0);
}

HCN_DEV qd mul_d(const qd &a, double d) {
    double p0, e0, p1, e1, p2, e2;
    eft_prod(a.c0, d, p0, e0);
    eft_prod(a.c1, d, p1, e1);
    eft_prod(a.c2, d, p2, e2);
    const double p3 = a.c3 * d;
    double s1, u, s2, v1, v2;
    eft_sum(p1, e0, s1, u);
    eft_three(p2, e1, u, s2, v1, v2);
    double s3 = p3 + e2;
    s3 = s3 + v1;
    s3 = s3 + v2;
    return renorm(p0, s1, s2, s3, 0.0);
}

// long division: four quotient digits taken from the leading remainder limb
HCN_DEV qd div(const qd &a, const qd &b) {
    qd r = a;
    const double q0 = r.c0 / b.c0;
    r = add(r, -mul_d(b, q0));
    const double q1 = r.c0 / b.c0;
    r = add(r, -mul_d(b, q1));
    const double q2 = r.c0 / b.c0;
    r = add(r, -mul_d(b, q2));
    const double q3 = r.c0 / b.c0;
    return renorm(q0, q1, q2, q3, 0.0);
}

// three Newton steps y += y (1 - a y^2) / 2 towards 1/sqrt(a), then a y
HCN_DEV qd sqrt(const qd &a) {
    if (a.c0 == 0.0) return qd{0.0, 0.0, 0.0, 0.0};
    qd y = qd{1.0 / ::sqrt(a.c0), 0.0, 0.0, 0.0};
    const qd one = qd{1.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int it = 0; it < 3; ++it) {
        qd h = mul(y, y);
        h = mul(a, h);
        const qd e = add(one, -h);
        qd c = mul(y, e);
        c = mul_d(c, 0.5);
        y = add(y, c);
    }
    return mul(a, y);
}

HCN_DEV double lead(const qd &a) { return a.c0; }

// ---------------------------------------------------------------------------
// plain double (the FP64 Jacobian and QR of the mixed-precision Newton step)
// ---------------------------------------------------------------------------

HCN_DEV double add(double a, double b) { return a + b; }
HCN_DEV double sub(double a, double b) { return a - b; }
HCN_DEV double mul(double a, double b) { return a * b; }
HCN_DEV double mul_d(double a, double b) { return a * b; }
HCN_DEV double div(double a, double b) { return a / b; }
HCN_DEV double sqrt(double a) { return ::sqrt(a); }
HCN_DEV double lead(double a) { return a; }

// ---------------------------------------------------------------------------
// precision traits: limbs and interleaved loads / stores
// ---------------------------------------------------------------------------

template <class R> struct limbs;
template <> struct limbs<double> { static constexpr int P = 1; };
template <> struct limbs<dd> { static constexpr int P = 2; };
template <> struct limbs<qd> { static constexpr int P = 4; };

template <class R> HCN_DEV R rmake(double h);
template <> HCN_DEV double rmake<double>(double h) { return h; }
template <> HCN_DEV dd rmake<dd>(double h) { return dd_make(h); }
template <> HCN_DEV qd rmake<qd>(double h) { return qd_make(h); }

HCN_DEV void rload(const double *p, double &r) { r = p[0]; }
HCN_DEV void rload(const double *p, dd &r) { r = dd{p[0], p[1]}; }
HCN_DEV void rload(const double *p, qd &r) { r = qd{p[0], p[1], p[2], p[3]}; }
HCN_DEV void rstore(double *p, double r) { p[0] = r; }
HCN_DEV void rstore(double *p, const dd &r) { p[0] = r.hi; p[1] = r.lo; }
HCN_DEV void rstore(double *p, const qd &r) { p[0] = r.c0; p[1] = r.c1; p[2] = r.c2; p[3] = r.c3; }

HCN_DEV bool rfinite(double a) { return __builtin_isfinite(a); }
HCN_DEV bool rfinite(const dd &a) { return __builtin_isfinite(a.hi); }
HCN_DEV bool rfinite(const qd &a) { return __builtin_isfinite(a.c0); }

// widen a double-precision value to R (exact)
HCN_DEV void rwiden(double a, double &r) { r = a; }
HCN_DEV void rwiden(double a, dd &r) { r = dd{a, 0.0}; }
HCN_DEV void rwiden(double a, qd &r) { r = qd{a, 0.0, 0.0, 0.0}; }

// ---------------------------------------------------------------------------
// complex numbers over R
// ---------------------------------------------------------------------------

template <class R> struct cx {
    R re, im;
};

template <class R> HCN_DEV cx<R> czero() { return cx<R>{rmake<R>(0.0), rmake<R>(0.0)}; }
template <class R> HCN_DEV cx<R> cone() { return cx<R>{rmake<R>(1.0), rmake<R>(0.0)}; }

template <class R> HCN_DEV cx<R> cload(const double *p) {
    constexpr int P = limbs<R>::P;
    cx<R> z;
    rload(p, z.re);
    rload(p + P, z.im);
    return z;
}

// a complex stored with Ps limbs per part, read in precision R (the leading
// limbs when R is narrower; Ps must be >= the limbs of R)
template <class R> HCN_DEV cx<R> cload_s(const double *p, int Ps) {
    cx<R> z;
    rload(p, z.re);
    rload(p + Ps, z.im);
    return z;
}

template <class R> HCN_DEV cx<R> cwiden(const cx<double> &a) {
    cx<R> z;
    rwiden(a.re, z.re);
    rwiden(a.im, z.im);
    return z;
}

template <class R> HCN_DEV void cstore(double *p, const cx<R> &z) {
    constexpr int P = limbs<R>::P;
    rstore(p, z.re);
    rstore(p + P, z.im);
}

template <class R> HCN_DEV cx<R> cadd(const cx<R> &a, const cx<R> &b) {
    return cx<R>{add(a.re, b.re), add(a.im, b.im)};
}

template <class R> HCN_DEV cx<R> cneg(const cx<R> &a) { return cx<R>{-a.re, -a.im}; }

template <class R> HCN_DEV cx<R> csub(const cx<R> &a, const cx<R> &b) { return cadd(a, cneg(b)); }

// (ar br - ai bi) + i (ar bi + ai br)
template <class R> HCN_DEV cx<R> cmul(const cx<R> &a, const cx<R> &b) {
    const R rr = mul(a.re, b.re);
    const R ii = mul(a.im, b.im);
    const R ri = mul(a.re, b.im);
    const R ir = mul(a.im, b.re);
    return cx<R>{sub(rr, ii), add(ri, ir)};
}

// conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
template <class R> HCN_DEV cx<R> cmul_conj(const cx<R> &a, const cx<R> &b) {
    const R rr = mul(a.re, b.re);
    const R ii = mul(a.im, b.im);
    const R ri = mul(a.re, b.im);
    const R ir = mul(a.im, b.re);
    return cx<R>{add(rr, ii), sub(ri, ir)};
}

template <class R> HCN_DEV R cnorm2(const cx<R> &a) { return add(mul(a.re, a.re), mul(a.im, a.im)); }

// s a for real s: (s ar) + i (s ai)
template <class R> HCN_DEV cx<R> cscale(const R &s, const cx<R> &a) {
    return cx<R>{mul(s, a.re), mul(s, a.im)};
}

// 2 a, exactly: every limb doubled
HCN_DEV double twice(double a) { return 2.0 * a; }
HCN_DEV dd twice(const dd &a) { return dd{2.0 * a.hi, 2.0 * a.lo}; }
HCN_DEV qd twice(const qd &a) { return qd{2.0 * a.c0, 2.0 * a.c1, 2.0 * a.c2, 2.0 * a.c3}; }
template <class R> HCN_DEV cx<R> cscale2(const cx<R> &a) { return cx<R>{twice(a.re), twice(a.im)}; }

template <class R> HCN_DEV cx<R> cscale_d(const cx<R> &a, double d) {
    return cx<R>{mul_d(a.re, d), mul_d(a.im, d)};
}

// infinity norm contribution of one complex number: max of the leading limbs
template <class R> HCN_DEV double clead_abs(const cx<R> &a) {
    const double x = fabs(lead(a.re));
    const double y = fabs(lead(a.im));
    // NaN propagates: (x != x) or (y != y) makes the result NaN
    if (x != x || y != y) return __builtin_nan("");
    return x > y ? x : y;
}

// max that propagates NaN
HCN_DEV double nanmax(double a, double b) {
    if (a != a || b != b) return __builtin_nan("");
    return a > b ? a : b;
}

}  // namespace hcn
