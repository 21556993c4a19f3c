// eval.hip -- evaluation and differentiation of a polynomial system
// (Sections 3.2 and 3.3).
//
// k_mon: one lane per monomial, a wavefront per 64 monomials of (after the
// sort by number of variables) equal size k.  Reverse mode on the product of
// the k distinct variables y_0..y_{k-1} (Table 1):
//   forward  F_0 = y_0, F_p = F_{p-1} y_p            (p = 1..k-2)
//   value    S = F_{k-2} y_{k-1}
//   backward dS/dy_{k-1} = F_{k-2}; B = y_{k-1};
//            for p = k-2..1: dS/dy_p = F_{p-1} B, B = B y_p;  dS/dy_0 = B
// i.e. 3k-5 complex products.  Exponents above one: m = c x^a is
// c' S with the common factor c' = c prod x_l^(a_l - 1), and
// dm/dx_l = a_l c' dS/dy_l.  Each lane writes its value and k partials to
// consecutive slots of its k-group (position-major, coalesced).
//
// k_sum: one lane per output; the value of f_i and every dense Jacobian
// entry J[k][i] is the sum of its slot list in input monomial order.  The
// homotopy with the total-degree start system and the residual max norm are
// fused into the same pass.
#include "internal.hpp"
#include "mp.hpp"
#include "prof.hpp"

namespace hcn {

template <class R>
HCN_DEV cx<R> load_y(const SysView &s, const double *xb, int p, int m) {
    constexpr int W = 2 * limbs<R>::P;
    const int v = s.pos[(size_t)p * s.nmon + m];
    return cload<R>(xb + (size_t)v * W);
}

template <class R>
HCN_DEV cx<R> cpow_small(const cx<R> &y, int e) {
    // y^e for e >= 1 by repeated multiplication
    cx<R> r = y;
    for (int q = 1; q < e; ++q) r = cmul(r, y);
    return r;
}

// FREG: forward products held in registers (KB-1 of them); otherwise they
// are parked in the output slots of the partials they precede and read back
// in the backward sweep.
template <class R, int KB, bool FREG>
__global__ __launch_bounds__(256) void k_mon(SysView s, int B, const double *__restrict__ x,
                                             long x_pstride, double *__restrict__ scratch,
                                             long sc_pstride, const PathState *st) {
    constexpr int W = 2 * limbs<R>::P;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= s.nmon) return;
    for (int b = blockIdx.y; b < B; b += gridDim.y) {
        if (st && !st[b].c_active) continue;
        const double *xb = x + (size_t)b * x_pstride;
        double *out = scratch + (size_t)b * sc_pstride;
        const int k = s.mon_k[m];
        const int slot = s.mon_slot[m];
        const int stride = s.mon_stride[m];
        const cx<R> c = cload<R>(s.coef + (size_t)m * W);
        if (k == 0) {
            cstore(out + (size_t)slot * W, c);
            continue;
        }
        cx<R> F[FREG ? (KB > 1 ? KB - 1 : 1) : 1];
        cx<R> Flast = czero<R>(), ylast = czero<R>(), pc = czero<R>();
        bool has_pc = false;
#pragma unroll
        for (int p = 0; p < KB; ++p) {
            if (p < k) {
                const cx<R> y = load_y<R>(s, xb, p, m);
                const int e = s.ex[(size_t)p * s.nmon + m];
                if (e >= 2) {
                    const cx<R> pw = cpow_small(y, e - 1);
                    pc = has_pc ? cmul(pc, pw) : pw;
                    has_pc = true;
                }
                if (p <= k - 2) {
                    const cx<R> Fp = (p == 0) ? y : cmul(Flast, y);
                    if (FREG) {
                        F[FREG ? p : 0] = Fp;
                    } else {
                        cstore(out + (size_t)(slot + (p + 2) * stride) * W, Fp);
                    }
                    Flast = Fp;
                } else {
                    ylast = y;
                }
            }
        }
        const cx<R> cp = has_pc ? cmul(c, pc) : c;
        if (k == 1) {
            cstore(out + (size_t)slot * W, cmul(cp, ylast));
            const int a0 = s.ex[m];
            const cx<R> d = (a0 == 1) ? cp : cscale_d(cp, (double)a0);
            cstore(out + (size_t)(slot + stride) * W, d);
            continue;
        }
        const cx<R> S = cmul(Flast, ylast);
        cstore(out + (size_t)slot * W, cmul(cp, S));
        {
            const int a = s.ex[(size_t)(k - 1) * s.nmon + m];
            cx<R> d = cmul(cp, Flast);
            if (a != 1) d = cscale_d(d, (double)a);
            cstore(out + (size_t)(slot + k * stride) * W, d);
        }
        cx<R> Bk = ylast;
#pragma unroll
        for (int p = KB - 2; p >= 1; --p) {
            if (p <= k - 2) {
                cx<R> Fpm1;
                if (FREG) {
                    Fpm1 = F[FREG ? p - 1 : 0];
                } else {
                    Fpm1 = cload<R>(out + (size_t)(slot + (p + 1) * stride) * W);
                }
                const int a = s.ex[(size_t)p * s.nmon + m];
                cx<R> d = cmul(cp, cmul(Fpm1, Bk));
                if (a != 1) d = cscale_d(d, (double)a);
                cstore(out + (size_t)(slot + (p + 1) * stride) * W, d);
                Bk = cmul(Bk, load_y<R>(s, xb, p, m));
            }
        }
        {
            const int a = s.ex[m];
            cx<R> d = cmul(cp, Bk);
            if (a != 1) d = cscale_d(d, (double)a);
            cstore(out + (size_t)(slot + stride) * W, d);
        }
    }
}

template <class R>
HCN_DEV cx<R> sum_list(const double *sc, const int32_t *list, int a, int b) {
    constexpr int W = 2 * limbs<R>::P;
    if (a >= b) return czero<R>();
    cx<R> acc = cload<R>(sc + (size_t)list[a] * W);
    for (int q = a + 1; q < b; ++q) acc = cadd(acc, cload<R>(sc + (size_t)list[q] * W));
    return acc;
}

template <class R>
HCN_DEV R r_from_two(double s, double e);
template <>
HCN_DEV dd r_from_two<dd>(double s, double e) { return dd{s, e}; }
template <>
HCN_DEV qd r_from_two<qd>(double s, double e) { return qd{s, e, 0.0, 0.0}; }

template <class R>
__global__ __launch_bounds__(256) void k_sum(SysView s, int B, const double *__restrict__ scratch,
                                             long sc_pstride, const double *__restrict__ x,
                                             long x_pstride, Homotopy hom, double *__restrict__ J,
                                             long J_cstride, long J_pstride, double *__restrict__ f,
                                             long f_pstride, int f_neg, double *norm_part,
                                             const PathState *st) {
    constexpr int W = 2 * limbs<R>::P;
    __shared__ double red[256 / 64];
    const long nJ = (long)s.n * s.N;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    for (int b = blockIdx.y; b < B; b += gridDim.y) {
        if (st && !st[b].c_active) continue;
        const double *sc = scratch + (size_t)b * sc_pstride;
        double mx = 0.0;
        if (e < nJ + s.N) {
            const bool isJ = e < nJ;
            const int k = isJ ? (int)(e / s.N) : -1;
            const int i = isJ ? (int)(e % s.N) : (int)(e - nJ);
            cx<R> acc = isJ ? sum_list<R>(sc, s.J_list, s.J_ptr[e], s.J_ptr[e + 1])
                            : sum_list<R>(sc, s.f_list, s.f_ptr[i], s.f_ptr[i + 1]);
            if (hom.on && (!isJ || k == i)) {
                // s_f = t^k, s_g = gamma (1-t)^k (1-t formed exactly)
                const double t = hom.t[b];
                double os, oe;
                eft_sum(1.0, -t, os, oe);
                const R omt = r_from_two<R>(os, oe);
                const R tt = rmake<R>(t);
                R pw = omt, sf = tt;
                for (int q = 1; q < hom.relax_k; ++q) {
                    pw = mul(pw, omt);
                    sf = mul(sf, tt);
                }
                const cx<R> gam = cload<R>(hom.gamma);
                const cx<R> sg = cscale(pw, gam);
                const double *xb = x + (size_t)b * x_pstride;
                const cx<R> xi = cload<R>(xb + (size_t)i * W);
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
            } else if (hom.on) {
                const double t = hom.t[b];
                const R tt = rmake<R>(t);
                R sf = tt;
                for (int q = 1; q < hom.relax_k; ++q) sf = mul(sf, tt);
                acc = cscale(sf, acc);
            }
            if (isJ) {
                if (J) cstore(J + (size_t)b * J_pstride + (size_t)k * J_cstride + (size_t)i * W, acc);
            } else {
                mx = clead_abs(acc);
                if (f_neg) acc = cneg(acc);
                if (f) cstore(f + (size_t)b * f_pstride + (size_t)i * W, acc);
            }
        }
        if (norm_part) {
            // block max of the residual leading limbs (order-independent, exact)
            for (int off = 32; off >= 1; off >>= 1) mx = nanmax(mx, __shfl_xor(mx, off));
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
            __syncthreads();
            if (threadIdx.x == 0) {
                double r = red[0];
                for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = nanmax(r, red[w]);
                norm_part[(size_t)b * gridDim.x + blockIdx.x] = r;
            }
            __syncthreads();
        }
    }
}

static int kbucket(int max_k) {
    if (max_k <= 4) return 4;
    if (max_k <= 8) return 8;
    if (max_k <= 16) return 16;
    if (max_k <= 32) return 32;
    return 64;
}

template <class R>
static int launch_mon_t(const SysView &s, int B, const double *x, long x_pstride, double *scratch,
                        long sc_pstride, const PathState *st, hipStream_t stream) {
    if (s.nmon == 0 || B == 0) return 0;
    dim3 grid((s.nmon + 255) / 256, B < 65535 ? B : 65535);
    ProfScope prof("eval_monomials", stream);
    const int kb = kbucket(s.max_k);
    constexpr bool isdd = limbs<R>::P == 2;
    switch (kb) {
        case 4: hipLaunchKernelGGL((k_mon<R, 4, isdd>), grid, dim3(256), 0, stream, s, B, x, x_pstride, scratch, sc_pstride, st); break;
        case 8: hipLaunchKernelGGL((k_mon<R, 8, isdd>), grid, dim3(256), 0, stream, s, B, x, x_pstride, scratch, sc_pstride, st); break;
        case 16: hipLaunchKernelGGL((k_mon<R, 16, isdd>), grid, dim3(256), 0, stream, s, B, x, x_pstride, scratch, sc_pstride, st); break;
        case 32: hipLaunchKernelGGL((k_mon<R, 32, false>), grid, dim3(256), 0, stream, s, B, x, x_pstride, scratch, sc_pstride, st); break;
        default: hipLaunchKernelGGL((k_mon<R, 64, false>), grid, dim3(256), 0, stream, s, B, x, x_pstride, scratch, sc_pstride, st); break;
    }
    return (int)hipGetLastError();
}

int launch_mon(int P, const SysView &s, int B, const double *x, long x_pstride, double *scratch,
               long sc_pstride, const PathState *st, hipStream_t stream) {
    return P == 2 ? launch_mon_t<dd>(s, B, x, x_pstride, scratch, sc_pstride, st, stream)
                  : launch_mon_t<qd>(s, B, x, x_pstride, scratch, sc_pstride, st, stream);
}

int sum_nparts(const SysView &s) {
    const long E = (long)s.n * s.N + s.N;
    return (int)((E + 255) / 256);
}

int launch_sum(int P, const SysView &s, int B, const double *scratch, long sc_pstride,
               const double *x, long x_pstride, const Homotopy &hom, double *J, long J_cstride,
               long J_pstride, double *f, long f_pstride, int f_neg, double *norm_part,
               const PathState *st, hipStream_t stream) {
    if (B == 0) return 0;
    dim3 grid(sum_nparts(s), B < 65535 ? B : 65535);
    ProfScope prof("eval_sums", stream);
    if (P == 2)
        hipLaunchKernelGGL(k_sum<dd>, grid, dim3(256), 0, stream, s, B, scratch, sc_pstride, x,
                           x_pstride, hom, J, J_cstride, J_pstride, f, f_pstride, f_neg, norm_part,
                           st);
    else
        hipLaunchKernelGGL(k_sum<qd>, grid, dim3(256), 0, stream, s, B, scratch, sc_pstride, x,
                           x_pstride, hom, J, J_cstride, J_pstride, f, f_pstride, f_neg, norm_part,
                           st);
    return (int)hipGetLastError();
}

}  // namespace hcn
