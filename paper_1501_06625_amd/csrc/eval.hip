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
// consecutive slots of its k-group (position-major, coalesced).  A
// values-only mode (for residuals) forms just c' S.
//
// k_sum: one lane per output; the value of f_i and every dense Jacobian
// entry J[k][i] is the sum of its slot list in input monomial order.  The
// homotopy with the total-degree start system and the residual max norm are
// fused into the same pass.
//
// The compute precision R (double, DD or QD) may be narrower than the
// storage of the coefficients (the system's limbs) and of x: loads take the
// leading limbs.
#include "internal.hpp"
#include "mp.hpp"
#include "prof.hpp"

namespace hcn {

enum { MON_FREG = 0, MON_FSLOT = 1, MON_VALUES = 2 };

template <class R>
HCN_DEV cx<R> load_y(const SysView &s, const double *xb, int xP, int p, int m) {
    const int v = s.pos[(size_t)p * s.nmon + m];
    return cload_s<R>(xb + (size_t)v * 2 * xP, xP);
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
template <class R, int KB, int MODE>
__global__ __launch_bounds__(256) void k_mon(MonArgs a) {
    constexpr int W = 2 * limbs<R>::P;
    const SysView &s = a.s;
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= s.nmon) return;
    for (int b = blockIdx.y; b < a.B; b += gridDim.y) {
        if (a.st && !a.st[b].c_active) continue;
        const double *xb = a.x + (size_t)b * a.x_pstride;
        double *out = a.scratch + (size_t)b * a.sc_pstride;
        const int k = s.mon_k[m];
        const int slot = s.mon_slot[m];
        const int stride = s.mon_stride[m];
        const cx<R> c = cload_s<R>(s.coef + (size_t)m * 2 * s.P, s.P);
        if (k == 0) {
            cstore(out + (size_t)slot * W, c);
            continue;
        }
        cx<R> F[MODE == MON_FREG ? (KB > 1 ? KB - 1 : 1) : 1];
        cx<R> Flast = czero<R>(), ylast = czero<R>(), pc = czero<R>();
        bool has_pc = false;
#pragma unroll
        for (int p = 0; p < KB; ++p) {
            if (p < k) {
                const cx<R> y = load_y<R>(s, xb, a.xP, p, m);
                const int e = s.ex[(size_t)p * s.nmon + m];
                if (e >= 2) {
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
        const cx<R> cp = has_pc ? cmul(c, pc) : c;
        if (k == 1) {
            cstore(out + (size_t)slot * W, cmul(cp, ylast));
            if (MODE != MON_VALUES) {
                const int a0 = s.ex[m];
                const cx<R> d = (a0 == 1) ? cp : cscale_d(cp, (double)a0);
                cstore(out + (size_t)(slot + stride) * W, d);
            }
            continue;
        }
        const cx<R> S = cmul(Flast, ylast);
        cstore(out + (size_t)slot * W, cmul(cp, S));
        if (MODE == MON_VALUES) continue;
        {
            const int e = s.ex[(size_t)(k - 1) * s.nmon + m];
            cx<R> d = cmul(cp, Flast);
            if (e != 1) d = cscale_d(d, (double)e);
            cstore(out + (size_t)(slot + k * stride) * W, d);
        }
        cx<R> Bk = ylast;
#pragma unroll
        for (int p = KB - 2; p >= 1; --p) {
            if (p <= k - 2) {
                cx<R> Fpm1;
                if (MODE == MON_FREG) {
                    Fpm1 = F[MODE == MON_FREG ? p - 1 : 0];
                } else {
                    Fpm1 = cload<R>(out + (size_t)(slot + (p + 1) * stride) * W);
                }
                const int e = s.ex[(size_t)p * s.nmon + m];
                cx<R> d = cmul(cp, cmul(Fpm1, Bk));
                if (e != 1) d = cscale_d(d, (double)e);
                cstore(out + (size_t)(slot + (p + 1) * stride) * W, d);
                Bk = cmul(Bk, load_y<R>(s, xb, a.xP, p, m));
            }
        }
        {
            const int e = s.ex[m];
            cx<R> d = cmul(cp, Bk);
            if (e != 1) d = cscale_d(d, (double)e);
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
HCN_DEV double r_from_two<double>(double s, double e) { return s + e; }
template <>
HCN_DEV dd r_from_two<dd>(double s, double e) { return dd{s, e}; }
template <>
HCN_DEV qd r_from_two<qd>(double s, double e) { return qd{s, e, 0.0, 0.0}; }

template <class R>
__global__ __launch_bounds__(256) void k_sum(SumArgs a) {
    constexpr int W = 2 * limbs<R>::P;
    const SysView &s = a.s;
    __shared__ double red[256 / 64];
    const long nJ = a.jac ? (long)s.n * s.N : 0;
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const Homotopy &hom = a.hom;
    for (int b = blockIdx.y; b < a.B; b += gridDim.y) {
        if (a.st && !a.st[b].c_active) continue;
        const double *sc = a.scratch + (size_t)b * a.sc_pstride;
        double mx = 0.0;
        if (e < nJ + s.N) {
            const bool isJ = e < nJ;
            const int k = isJ ? (int)(e / s.N) : -1;
            const int i = isJ ? (int)(e % s.N) : (int)(e - nJ);
            cx<R> acc = isJ ? sum_list<R>(sc, s.J_list, s.J_ptr[e], s.J_ptr[e + 1])
                            : sum_list<R>(sc, s.f_list, s.f_ptr[i], s.f_ptr[i + 1]);
            if (hom.on) {
                // s_f = t^k, s_g = gamma (1-t)^k (1-t formed exactly)
                const double t = hom.t[b];
                const R tt = rmake<R>(t);
                R sf = tt;
                for (int q = 1; q < hom.relax_k; ++q) sf = mul(sf, tt);
                if (!isJ || k == i) {
                    double os, oe;
                    eft_sum(1.0, -t, os, oe);
                    const R omt = r_from_two<R>(os, oe);
                    R pw = omt;
                    for (int q = 1; q < hom.relax_k; ++q) pw = mul(pw, omt);
                    const cx<R> gam = cload_s<R>(hom.gamma, hom.gP);
                    const cx<R> sg = cscale(pw, gam);
                    const double *xb = a.x + (size_t)b * a.x_pstride;
                    const cx<R> xi = cload_s<R>(xb + (size_t)i * 2 * a.xP, a.xP);
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
                if (a.J) cstore(a.J + (size_t)b * a.J_pstride + (size_t)k * a.J_cstride + (size_t)i * W, acc);
            } else {
                mx = clead_abs(acc);
                if (a.f_neg) acc = cneg(acc);
                if (a.f) {
                    if (a.f_lead_only) {
                        double *p = a.f + (size_t)b * a.f_pstride + (size_t)i * 2;
                        p[0] = lead(acc.re);
                        p[1] = lead(acc.im);
                    } else {
                        cstore(a.f + (size_t)b * a.f_pstride + (size_t)i * W, acc);
                    }
                }
            }
        }
        if (a.norm_part) {
            // block max of the residual leading limbs (order-independent, exact)
            for (int off = 32; off >= 1; off >>= 1) mx = nanmax(mx, __shfl_xor(mx, off));
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
            __syncthreads();
            if (threadIdx.x == 0) {
                double r = red[0];
                for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = nanmax(r, red[w]);
                a.norm_part[(size_t)b * gridDim.x + blockIdx.x] = r;
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

template <class R, int KB>
static void mon_kb(const MonArgs &a, dim3 grid, hipStream_t stream) {
    // forward products in registers where they fit (DD up to 16, FP64 up to
    // 32 variables); QD and longer products park them in their output slots
    constexpr bool freg = (limbs<R>::P == 2 && KB <= 16) || (limbs<R>::P == 1 && KB <= 32);
    if (a.values_only)
        hipLaunchKernelGGL((k_mon<R, KB, MON_VALUES>), grid, dim3(256), 0, stream, a);
    else if (freg)
        hipLaunchKernelGGL((k_mon<R, KB, MON_FREG>), grid, dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((k_mon<R, KB, MON_FSLOT>), grid, dim3(256), 0, stream, a);
}

template <class R>
static int launch_mon_t(const MonArgs &a, hipStream_t stream) {
    if (a.s.nmon == 0 || a.B == 0) return 0;
    dim3 grid((a.s.nmon + 255) / 256, a.B < 65535 ? a.B : 65535);
    ProfScope prof("eval_monomials", stream);
    switch (kbucket(a.s.max_k)) {
        case 4: mon_kb<R, 4>(a, grid, stream); break;
        case 8: mon_kb<R, 8>(a, grid, stream); break;
        case 16: mon_kb<R, 16>(a, grid, stream); break;
        case 32: mon_kb<R, 32>(a, grid, stream); break;
        default: mon_kb<R, 64>(a, grid, stream); break;
    }
    return (int)hipGetLastError();
}

int launch_mon(int RP, const MonArgs &a, hipStream_t stream) {
    switch (RP) {
        case 1: return launch_mon_t<double>(a, stream);
        case 2: return launch_mon_t<dd>(a, stream);
        default: return launch_mon_t<qd>(a, stream);
    }
}

int sum_nparts(const SysView &s, int jac) {
    const long E = (jac ? (long)s.n * s.N : 0) + s.N;
    return (int)((E + 255) / 256);
}

int launch_sum(int RP, const SumArgs &a, hipStream_t stream) {
    if (a.B == 0) return 0;
    dim3 grid(sum_nparts(a.s, a.jac), a.B < 65535 ? a.B : 65535);
    ProfScope prof("eval_sums", stream);
    switch (RP) {
        case 1: hipLaunchKernelGGL(k_sum<double>, grid, dim3(256), 0, stream, a); break;
        case 2: hipLaunchKernelGGL(k_sum<dd>, grid, dim3(256), 0, stream, a); break;
        default: hipLaunchKernelGGL(k_sum<qd>, grid, dim3(256), 0, stream, a); break;
    }
    return (int)hipGetLastError();
}

}  // namespace hcn
