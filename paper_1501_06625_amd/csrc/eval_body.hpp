// eval_body.hpp -- per-lane bodies of the evaluation kernels, shared by the
// single-system kernels (eval.hip) and the slot-table kernels (batch.hip).
//
// mon_one: reverse mode on the product of the k distinct variables
// y_0..y_{k-1} of one monomial (Section 3.2, Table 1):
//   forward  F_0 = y_0, F_p = F_{p-1} y_p            (p = 1..k-2)
//   value    S = F_{k-2} y_{k-1}
//   backward dS/dy_{k-1} = F_{k-2}; B = y_{k-1};
//            for p = k-2..1: dS/dy_p = F_{p-1} B, B = B y_p;  dS/dy_0 = B
// i.e. 3k-5 complex products.  Exponents above one: m = c x^a is c' S with
// the common factor c' = c prod x_l^(a_l - 1), and dm/dx_l = a_l c' dS/dy_l.
// The factor c' is applied once, to the start of the backward product
// (B' = c' y_{k-1}), which carries it into every partial but the last:
// 3k-3 complex products for the value and all partials, coefficient
// included.
// The value and the k partials go to consecutive slots of the monomial's
// k-group (position-major, so a wavefront writes 64 consecutive slots).
//
// sum_one: one output, the sum of its slot list in input monomial order
// (Section 3.3), with the homotopy of equation (1) for the total-degree
// start system fused in.
#pragma once

#include "internal.hpp"
#include "mp.hpp"

namespace hcn {

enum { MON_FREG = 0, MON_FSLOT = 1, MON_VALUES = 2 };

// The dispatcher deals the workgroups of a launch to the 8 XCDs in turn
// (linear id w to XCD w mod 8), and each XCD has an L2 of its own.  The
// summation workgroups of one point share cache lines of its monomial
// slots, so they are given logical ids that keep them on one XCD: XCD x
// takes the contiguous range of logical ids starting at x (G / 8) +
// min(x, G mod 8), in dispatch order.  A bijection of 0..G-1.
HCN_DEV int xcd_logical(int w, int G) {
    constexpr int X = 8;
    const int x = w % X, q = G / X, r = G % X;
    return x * q + (x < r ? x : r) + w / X;
}

// The point a monomial kernel reads: variable v at x + v * stride, xP limbs
// (at least those of the compute precision).  pows (LDS, or NULL when the
// largest exponent is at most 2): pows + ((j - 2) n + v) W holds y_v^j for
// 2 <= j < maxe, so that the common factor can be formed with the same
// products in every lane (see mon_one).
struct PointView {
    const double *x;
    int stride, xP;
    const double *pows;
};

template <class R>
HCN_DEV cx<R> load_y(const SysView &s, const PointView &pv, int p, int m, int &v) {
    v = s.pos[(size_t)p * s.nmon + m];
    return cload_s<R>(pv.x + (size_t)v * pv.stride, pv.xP);
}

// the powers y^2 .. y^{maxe-1} of every variable of one point into LDS
// (pows: (maxe - 2) n complex numbers in the compute precision);
// y^j = y^{j-1} y, the products cpow_small forms
template <class R>
HCN_DEV void stage_pows(const SysView &s, const double *xb, int xP, double *pows) {
    constexpr int W = 2 * limbs<R>::P;
    for (int v = threadIdx.x; v < s.n; v += blockDim.x) {
        const cx<R> y = cload_s<R>(xb + (size_t)v * 2 * xP, xP);
        cx<R> r = y;
        for (int j = 2; j < s.max_e; ++j) {
            r = cmul(r, y);
            cstore(pows + ((size_t)(j - 2) * s.n + v) * W, r);
        }
    }
}

// LDS bytes of stage_pows for system s in compute precision RP; 0 when no
// power is needed (largest exponent at most 2) or the table would not fit
// the budget of one workgroup
HCN_DEV __host__ size_t mon_stage_bytes(const SysView &s, int RP) {
    if (s.max_e <= 2) return 0;
    const size_t b = (size_t)(s.max_e - 2) * s.n * 2 * RP * sizeof(double);
    return b <= 32 * 1024 ? b : 0;
}

// whether the monomial kernels use the uniform form of the common factor:
// some exponent above one, and the power table staged if needed (host side:
// also the process-wide switch mon_uniform_enabled)
HCN_DEV __host__ bool mon_uniform_fits(const SysView &s, int RP) {
    return s.max_e >= 2 && (s.max_e == 2 || mon_stage_bytes(s, RP) > 0);
}
bool mon_uniform_enabled();
inline bool mon_uniform(const SysView &s, int RP) { return mon_uniform_enabled() && mon_uniform_fits(s, RP); }

// a d for the exponent a of a variable: 1 leaves d, 2 doubles every limb
// (exact), larger exponents multiply by a double
template <class R>
HCN_DEV cx<R> exp_scale(const cx<R> &d, int a) {
    if (a == 1) return d;
    if (a == 2) return cscale2(d);
    return cscale_d(d, (double)a);
}

template <class R>
HCN_DEV cx<R> cpow_small(const cx<R> &y, int e) {
    // y^e for e >= 1 by repeated multiplication
    cx<R> r = y;
    for (int q = 1; q < e; ++q) r = cmul(r, y);
    return r;
}

// MODE: MON_FREG keeps the forward products in registers (KB-1 of them);
// MON_FSLOT parks them in the output slots of the partials they precede and
// reads them back in the backward sweep; MON_VALUES forms values only.
//
// Uniform form (mon_uniform: some exponent > 1):
// exponents differ from lane to lane, so a branch per variable would run
// both ways for the whole wavefront.  Instead every lane multiplies the
// common factor by y^{a-1} at every position, with y^0 = 1 (a product by 1
// returns a normalised FP64 / DD / QD number unchanged) and y^{a-1} from the staged
// table, and scales every partial by a with mul_d (exact for a = 1, 2):
// the same bits as the branching form, in the same operations for all lanes.
template <class R, int KB, int MODE, bool UNI = false>
HCN_DEV void mon_one(const SysView &s, int m, const PointView &pv, double *out) {
    constexpr int W = 2 * limbs<R>::P;
    constexpr bool uni = UNI;  // callers: mon_uniform
    const int k = s.mon_k[m];
    const int slot = s.mon_slot[m];
    const int stride = s.mon_stride[m];
    const cx<R> c = cload_s<R>(s.coef + (size_t)m * 2 * s.P, s.P);
    if (k == 0) {
        cstore(out + (size_t)slot * W, c);
        return;
    }
    auto escale = [&](const cx<R> &d, int a) -> cx<R> {
        if constexpr (uni) return cscale_d(d, (double)a);
        return exp_scale(d, a);
    };
    cx<R> F[MODE == MON_FREG ? (KB > 1 ? KB - 1 : 1) : 1];
    cx<R> Flast = czero<R>(), ylast = czero<R>(), pc = czero<R>();
    bool has_pc = false;
#pragma unroll
    for (int p = 0; p < KB; ++p) {
        if (p < k) {
            int v;
            const cx<R> y = load_y<R>(s, pv, p, m, v);
            const int e = s.ex[(size_t)p * s.nmon + m];
            if constexpr (uni) {
                cx<R> pw = y;
                if (e >= 3) pw = cload<R>(pv.pows + ((size_t)(e - 3) * s.n + v) * W);
                if (e == 1) pw = cone<R>();
                pc = (p == 0) ? pw : cmul(pc, pw);
            } else if (e >= 2) {
                const cx<R> pw = cpow_small(y, e - 1);
                pc = has_pc ? cmul(pc, pw) : pw;
                has_pc = true;
            }
            if (p <= k - 2) {
                const cx<R> Fp = (p == 0) ? y : cmul(Flast, y);
                if (MODE == MON_FREG) {
                    F[MODE == MON_FREG ? p : 0] = Fp;
                } else if (MODE == MON_FSLOT) {
                    cstore(out + (size_t)(slot + (p + 2) * stride) * W, Fp);
                }
                Flast = Fp;
            } else {
                ylast = y;
            }
        }
    }
    const cx<R> cp = uni ? cmul(c, pc) : (has_pc ? cmul(c, pc) : c);
    if (k == 1) {
        cstore(out + (size_t)slot * W, cmul(cp, ylast));
        if (MODE != MON_VALUES) cstore(out + (size_t)(slot + stride) * W, escale(cp, s.ex[m]));
        return;
    }
    // the coefficient rides on the backward product: B' = c' y_{k-1}
    cx<R> Bk = cmul(cp, ylast);
    cstore(out + (size_t)slot * W, cmul(Flast, Bk));
    if (MODE == MON_VALUES) return;
    cstore(out + (size_t)(slot + k * stride) * W,
           escale(cmul(cp, Flast), s.ex[(size_t)(k - 1) * s.nmon + m]));
#pragma unroll
    for (int p = KB - 2; p >= 1; --p) {
        if (p <= k - 2) {
            cx<R> Fpm1;
            if (MODE == MON_FREG) {
                Fpm1 = F[MODE == MON_FREG ? p - 1 : 0];
            } else {
                Fpm1 = cload<R>(out + (size_t)(slot + (p + 1) * stride) * W);
            }
            cstore(out + (size_t)(slot + (p + 1) * stride) * W,
                   escale(cmul(Fpm1, Bk), s.ex[(size_t)p * s.nmon + m]));
            int v;
            Bk = cmul(Bk, load_y<R>(s, pv, p, m, v));
        }
    }
    cstore(out + (size_t)(slot + stride) * W, escale(Bk, s.ex[m]));
}

// mon_one for monomials of any size (more variables than the unrolled forms
// cover): the same operations in the same order as mon_one with MON_FSLOT
// (or MON_VALUES), with loops over the monomial's own k, so the bits are
// those of mon_one; forward products parked in the output slots.  The loops
// take LONG_AHEAD positions at a time and issue their loads (positions,
// exponents, variables, parked products) before the products that use
// them, so that a lane waits for memory once per group, not once per
// position.
constexpr int LONG_AHEAD = 4;

template <class R, int MODE, bool UNI = false>
HCN_DEV void mon_one_long(const SysView &s, int m, const PointView &pv, double *out) {
    static_assert(MODE != MON_FREG, "the long form parks its forward products in the slots");
    constexpr int W = 2 * limbs<R>::P;
    constexpr int U = LONG_AHEAD;
    const int k = s.mon_k[m];
    const int slot = s.mon_slot[m];
    const int stride = s.mon_stride[m];
    const cx<R> c = cload_s<R>(s.coef + (size_t)m * 2 * s.P, s.P);
    if (k == 0) {
        cstore(out + (size_t)slot * W, c);
        return;
    }
    auto escale = [&](const cx<R> &d, int a) -> cx<R> {
        if constexpr (UNI) return cscale_d(d, (double)a);
        return exp_scale(d, a);
    };
    cx<R> Flast = czero<R>(), ylast = czero<R>(), pc = czero<R>();
    bool has_pc = false;
    for (int p0 = 0; p0 < k; p0 += U) {
        cx<R> yb[U];
        int vb[U], eb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 + u;
            vb[u] = 0;
            eb[u] = 1;
            yb[u] = czero<R>();
            if (p < k) {
                yb[u] = load_y<R>(s, pv, p, m, vb[u]);
                eb[u] = s.ex[(size_t)p * s.nmon + m];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 + u;
            if (p >= k) break;
            const cx<R> y = yb[u];
            const int v = vb[u], e = eb[u];
            if constexpr (UNI) {
                cx<R> pw = y;
                if (e >= 3) pw = cload<R>(pv.pows + ((size_t)(e - 3) * s.n + v) * W);
                if (e == 1) pw = cone<R>();
                pc = (p == 0) ? pw : cmul(pc, pw);
            } else if (e >= 2) {
                const cx<R> pw = cpow_small(y, e - 1);
                pc = has_pc ? cmul(pc, pw) : pw;
                has_pc = true;
            }
            if (p <= k - 2) {
                const cx<R> Fp = (p == 0) ? y : cmul(Flast, y);
                if (MODE == MON_FSLOT) cstore(out + (size_t)(slot + (p + 2) * stride) * W, Fp);
                Flast = Fp;
            } else {
                ylast = y;
            }
        }
    }
    const cx<R> cp = UNI ? cmul(c, pc) : (has_pc ? cmul(c, pc) : c);
    if (k == 1) {
        cstore(out + (size_t)slot * W, cmul(cp, ylast));
        if (MODE != MON_VALUES) cstore(out + (size_t)(slot + stride) * W, escale(cp, s.ex[m]));
        return;
    }
    cx<R> Bk = cmul(cp, ylast);
    cstore(out + (size_t)slot * W, cmul(Flast, Bk));
    if (MODE == MON_VALUES) return;
    cstore(out + (size_t)(slot + k * stride) * W,
           escale(cmul(cp, Flast), s.ex[(size_t)(k - 1) * s.nmon + m]));
    // positions k-2 down to 1; position p reads F_{p-1} from slot p+1 and
    // writes its partial there (each slot read, then written, by the same
    // position)
    for (int p0 = k - 2; p0 >= 1; p0 -= U) {
        cx<R> Fb[U], yb[U];
        int eb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 - u;
            eb[u] = 1;
            Fb[u] = yb[u] = czero<R>();
            if (p >= 1) {
                Fb[u] = cload<R>(out + (size_t)(slot + (p + 1) * stride) * W);
                eb[u] = s.ex[(size_t)p * s.nmon + m];
                int v;
                yb[u] = load_y<R>(s, pv, p, m, v);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int p = p0 - u;
            if (p < 1) break;
            cstore(out + (size_t)(slot + (p + 1) * stride) * W, escale(cmul(Fb[u], Bk), eb[u]));
            Bk = cmul(Bk, yb[u]);
        }
    }
    cstore(out + (size_t)(slot + stride) * W, escale(Bk, s.ex[m]));
}

// Tree mode (Section 3.2: the product of a monomial and all its products
// with one factor left out as a circuit of G cooperating lanes, log G
// levels, instead of one lane's reverse sweep).  Lane j of a group of G
// (a power of two >= k) holds y_j (one past k), forms y_j^(a_j - 1), and
// the group forms by shuffles, log2 G levels each:
//   the product of those powers (a butterfly whose products take the lower
//     lane's value first, so every lane holds the same bits), times c: c';
//   the exclusive prefix products L_j = y_0 ... y_{j-1} and suffix products
//     R_j = y_{j+1} ... y_{k-1} (Hillis-Steele scans);
// then dm/dx_j = a_j (c' (L_j R_j)) and the value c' (L_{G-1} y_{G-1}) (the
// total product, formed by the last lane's inclusive scan and broadcast).
// Outputs go to the same slots as mon_one's.  The products are the same
// mathematically as the reverse mode's, rounded in another order.
template <class R>
HCN_DEV cx<R> shfl_cx(const cx<R> &v, int src, int width);
template <>
HCN_DEV cx<double> shfl_cx(const cx<double> &v, int src, int width) {
    return cx<double>{__shfl(v.re, src, width), __shfl(v.im, src, width)};
}
template <>
HCN_DEV cx<dd> shfl_cx(const cx<dd> &v, int src, int width) {
    return cx<dd>{dd{__shfl(v.re.hi, src, width), __shfl(v.re.lo, src, width)},
                  dd{__shfl(v.im.hi, src, width), __shfl(v.im.lo, src, width)}};
}
template <>
HCN_DEV cx<qd> shfl_cx(const cx<qd> &v, int src, int width) {
    return cx<qd>{qd{__shfl(v.re.c0, src, width), __shfl(v.re.c1, src, width),
                     __shfl(v.re.c2, src, width), __shfl(v.re.c3, src, width)},
                  qd{__shfl(v.im.c0, src, width), __shfl(v.im.c1, src, width),
                     __shfl(v.im.c2, src, width), __shfl(v.im.c3, src, width)}};
}

// every lane of the group calls this (lanes beyond the last monomial with
// m = -1, which only take part in the shuffles)
template <class R, int G, bool UNI>
HCN_DEV void mon_tree(const SysView &s, int m, int j, const PointView &pv, double *out) {
    constexpr int W = 2 * limbs<R>::P;
    const bool live = m >= 0;
    const int k = live ? s.mon_k[m] : 0;
    const bool mine = j < k;
    int v = 0, e = 1;
    cx<R> y = cone<R>();
    if (mine) {
        y = load_y<R>(s, pv, j, m, v);
        e = s.ex[(size_t)j * s.nmon + m];
    }
    // y^(a - 1): 1, y, or powers (from the staged table in the uniform form)
    cx<R> pw = cone<R>();
    if (e == 2) {
        pw = y;
    } else if (e >= 3) {
        if constexpr (UNI)
            pw = cload<R>(pv.pows + ((size_t)(e - 3) * s.n + v) * W);
        else
            pw = cpow_small(y, e - 1);
    }
    // c' = c * prod of the powers (butterfly, lower lane's value first)
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const cx<R> o = shfl_cx(pw, (int)(threadIdx.x & 63) ^ d, 64);
        pw = (j & d) ? cmul(o, pw) : cmul(pw, o);
    }
    // inclusive prefix products (Hillis-Steele), then exclusive by one lane
    cx<R> pre = y;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const int src = (int)(threadIdx.x & 63) - d;
        const cx<R> o = shfl_cx(pre, src < 0 ? 0 : src, 64);
        if (j >= d) pre = cmul(o, pre);
    }
    const int lane = (int)(threadIdx.x & 63);
    const cx<R> total = shfl_cx(pre, lane - j + G - 1, 64);
    cx<R> L = shfl_cx(pre, lane > 0 ? lane - 1 : 0, 64);
    if (j == 0) L = cone<R>();
    // exclusive suffix products
    cx<R> suf = y;
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
        const int src = lane + d;
        const cx<R> o = shfl_cx(suf, src > 63 ? 63 : src, 64);
        if (j + d < G) suf = cmul(suf, o);
    }
    cx<R> Rr = shfl_cx(suf, lane < 63 ? lane + 1 : 63, 64);
    if (j == G - 1) Rr = cone<R>();
    if (!live) return;
    const int slot = s.mon_slot[m];
    const int stride = s.mon_stride[m];
    const cx<R> c = cload_s<R>(s.coef + (size_t)m * 2 * s.P, s.P);
    if (k == 0) {
        if (j == 0) cstore(out + (size_t)slot * W, c);
        return;
    }
    const cx<R> cp = cmul(c, pw);
    if (j == 0) cstore(out + (size_t)slot * W, cmul(cp, total));
    if (mine) cstore(out + (size_t)(slot + (j + 1) * stride) * W, cscale_d(cmul(cp, cmul(L, Rr)), (double)e));
}

// The sum of the slots list[0], list[step], ..., list[(len-1) step], added
// in list order.  The slot loads of SUM_BATCH entries (8; 4 in QD, whose
// slots take twice the registers) are issued before their additions, so
// that each lane keeps that many gathers in flight instead of one; the
// order of the additions, and so every bit, is that of the plain loop.
template <class R>
HCN_DEV cx<R> sum_strided(const double *sc, const int32_t *list, int step, int len) {
    constexpr int W = 2 * limbs<R>::P;
    constexpr int SUM_BATCH = limbs<R>::P == 4 ? 4 : 8;
    cx<R> acc = czero<R>();
    int c = 0;
    for (; c + SUM_BATCH <= len; c += SUM_BATCH) {
        cx<R> v[SUM_BATCH];
#pragma unroll
        for (int u = 0; u < SUM_BATCH; ++u) v[u] = cload<R>(sc + (size_t)list[(c + u) * step] * W);
#pragma unroll
        for (int u = 0; u < SUM_BATCH; ++u) acc = c + u == 0 ? v[u] : cadd(acc, v[u]);
    }
    if (c < len) {
        const int rem = len - c;
        cx<R> v[SUM_BATCH];
#pragma unroll
        for (int u = 0; u < SUM_BATCH; ++u)
            if (u < rem) v[u] = cload<R>(sc + (size_t)list[(c + u) * step] * W);
#pragma unroll
        for (int u = 0; u < SUM_BATCH; ++u)
            if (u < rem) acc = c + u == 0 ? v[u] : cadd(acc, v[u]);
    }
    return acc;
}

template <class R>
HCN_DEV cx<R> sum_list(const double *sc, const int32_t *list, int a, int b) {
    return a >= b ? czero<R>() : sum_strided<R>(sc, list + a, 1, b - a);
}

template <class R>
HCN_DEV R r_from_two(double s, double e);
template <>
HCN_DEV double r_from_two<double>(double s, double e) { return s + e; }
template <>
HCN_DEV dd r_from_two<dd>(double s, double e) { return dd{s, e}; }
template <>
HCN_DEV qd r_from_two<qd>(double s, double e) { return qd{s, e, 0.0, 0.0}; }

// where one path's sums go
struct SumOut {
    int jac;            // 0: values only (entries 0..N-1 are f)
    double *J;          // column k at J + k*J_cstride, or NULL
    long J_cstride;
    double *f;          // or NULL
    int f_neg, f_lead_only;
};

// output e of one path (e < n N: Jacobian entry (e / N, e % N); else f_{e - nN});
// returns the leading-limb magnitude of an f entry (0 for Jacobian entries)
template <class R>
HCN_DEV double sum_one(const SysView &s, long e, const double *sc, const double *xb, int xP,
                       int hom_on, int relax_k, double t, const double *gamma, int gP,
                       const SumOut &o) {
    constexpr int W = 2 * limbs<R>::P;
    const long nJ = o.jac ? (long)s.n * s.N : 0;
    if (e >= nJ + s.N) return 0.0;
    const bool isJ = e < nJ;
    // Jacobian lanes equation-major: lane e forms entry (k, i) = (e mod n,
    // e / n), whose list is that of the column-major index ej = k N + i
    const int k = isJ ? (int)(e % s.n) : -1;
    const int i = isJ ? (int)(e / s.n) : (int)(e - nJ);
    const long ej = (long)k * s.N + i;
    cx<R> acc;
    if (isJ && s.J_ilv) {
        // the interleaved copy of the list: lanes of a wavefront read their
        // c-th indices from consecutive words
        const int32_t *li = s.J_ilv + s.J_wbase[e >> 6] + (e & 63);
        acc = sum_strided<R>(sc, li, 64, s.J_ptr[ej + 1] - s.J_ptr[ej]);
    } else {
        acc = isJ ? sum_list<R>(sc, s.J_list, s.J_ptr[ej], s.J_ptr[ej + 1])
                  : sum_list<R>(sc, s.f_list, s.f_ptr[i], s.f_ptr[i + 1]);
    }
    if (hom_on) {
        // s_f = t^k, s_g = gamma (1-t)^k (1-t formed exactly)
        const R tt = rmake<R>(t);
        R sf = tt;
        for (int q = 1; q < relax_k; ++q) sf = mul(sf, tt);
        if (!isJ || k == i) {
            double os, oe;
            eft_sum(1.0, -t, os, oe);
            const R omt = r_from_two<R>(os, oe);
            R pw = omt;
            for (int q = 1; q < relax_k; ++q) pw = mul(pw, omt);
            const cx<R> gam = cload_s<R>(gamma, gP);
            const cx<R> sg = cscale(pw, gam);
            const cx<R> xi = cload_s<R>(xb + (size_t)i * 2 * xP, xP);
            const int d = s.deg[i];
            cx<R> xpm1 = cone<R>();
            if (d >= 2) xpm1 = cpow_small(xi, d - 1);
            if (isJ) {
                const cx<R> dg = cscale_d(xpm1, (double)d);
                acc = cadd(cmul(sg, dg), cscale(sf, acc));
            } else {
                const cx<R> xd = (d >= 2) ? cmul(xpm1, xi) : xi;
                const cx<R> g = csub(xd, cone<R>());
                acc = cadd(cmul(sg, g), cscale(sf, acc));
            }
        } else {
            acc = cscale(sf, acc);
        }
    }
    if (isJ) {
        if (o.J) cstore(o.J + (size_t)k * o.J_cstride + (size_t)i * W, acc);
        return 0.0;
    }
    const double mx = clead_abs(acc);
    if (o.f_neg) acc = cneg(acc);
    if (o.f) {
        if (o.f_lead_only) {
            double *p = o.f + (size_t)i * 2;
            p[0] = lead(acc.re);
            p[1] = lead(acc.im);
        } else {
            cstore(o.f + (size_t)i * W, acc);
        }
    }
    return mx;
}

// maximum over a 256-lane workgroup (NaN propagates); every lane returns it
HCN_DEV double block_max(double mx, double *red) {
    for (int off = 32; off >= 1; off >>= 1) mx = nanmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = nanmax(r, red[w]);
    __syncthreads();
    return r;
}

}  // namespace hcn
