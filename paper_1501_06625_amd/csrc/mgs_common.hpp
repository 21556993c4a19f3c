// mgs_common.hpp -- the parts of the solve shared by every MGS variant: the
// Fig. 2 tests taken before a solve, and the epilogue after the
// factorisation (column-oriented back substitution dx_k = y_k / r_kk,
// y_i -= r_ik dx_k for i < k; the Newton update x += dx with its norm and the
// Fig. 2 tests that follow it).  The epilogue runs in one workgroup of
// MGS_THREADS lanes per problem.
#pragma once

#include "internal.hpp"
#include "mp.hpp"

namespace hcn {

constexpr int MGS_THREADS = 256;

// Fig. 2 before the solve: fail if the residual grew beyond the previous one
// (initially max_eq_val), succeed if it is below the tolerance, stop on NaN.
// Called by one lane; returns 1 when this problem needs no solve.
HCN_DEV int fig2_decide(const MgsArgs &a, int b) {
    PathState &st = a.st[b];
    if (!st.c_active) return 1;
    double res = 0.0;
    for (int q = 0; q < a.nparts; ++q) res = nanmax(res, a.norm_part[(size_t)b * a.nparts + q]);
    st.res = res;
    st.c_iter += 1;
    int decided = 0;
    if (res != res) {
        st.c_status = HCN_NAN;
        decided = 1;
    } else if (res > st.last) {
        st.c_status = HCN_DIVERGED;
        decided = 1;
    } else if (res < st.tol_res) {
        st.c_status = HCN_OK;
        decided = 1;
    }
    if (decided) st.c_active = 0;
    return decided;
}

template <class R>
HCN_DEV void mgs_epilogue(const MgsArgs &a, int b, bool singular) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    const int tid = threadIdx.x;
    const int n = a.n;
    double *Rb = a.R + (size_t)b * a.R_pstride;
    double *invb = a.inv + (size_t)b * a.inv_pstride;
    double *dxb = a.dx + (size_t)b * a.dx_pstride;
    if (singular) {
        if (tid == 0) {
            if (a.status) a.status[b] = HCN_ESINGULAR;
            if (a.mode == MGS_NEWTON_FIG2 || a.mode == MGS_MIXED_SOLVE) {
                a.st[b].c_status = HCN_ESINGULAR;
                a.st[b].c_active = 0;
            }
            if (a.mode == MGS_NEWTON_STEP && a.norms) {
                double res = 0.0;
                for (int q = 0; q < a.nparts; ++q) res = nanmax(res, a.norm_part[(size_t)b * a.nparts + q]);
                a.norms[2 * b] = res;
                a.norms[2 * b + 1] = __builtin_nan("");
            }
        }
        return;
    }

    // ---- back substitution, in place in dx (starts as y = column n of R)
    for (int i = tid; i < n; i += MGS_THREADS)
        cstore(dxb + (size_t)i * W, cload<R>(Rb + ((size_t)n * n + i) * W));
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
        if (tid == 0) {
            R iv;
            rload(invb + (size_t)k * P, iv);
            cstore(dxb + (size_t)k * W, cscale(iv, cload<R>(dxb + (size_t)k * W)));
        }
        __syncthreads();
        const cx<R> xk = cload<R>(dxb + (size_t)k * W);
        for (int i = tid; i < k; i += MGS_THREADS) {
            double *p = dxb + (size_t)i * W;
            cstore(p, csub(cload<R>(p), cmul(cload<R>(Rb + ((size_t)k * n + i) * W), xk)));
        }
        __syncthreads();
    }

    if (a.mode == MGS_SOLVE || a.mode == MGS_MIXED_SOLVE) {
        if (tid == 0 && a.status) a.status[b] = HCN_OK;
        return;
    }

    // ---- Newton: update norm, NaN check, x += dx
    __shared__ double s_red[MGS_THREADS / 64];
    double m = 0.0;
    for (int i = tid; i < n; i += MGS_THREADS) m = nanmax(m, clead_abs(cload<R>(dxb + (size_t)i * W)));
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
    if ((tid & 63) == 0) s_red[tid >> 6] = m;
    __syncthreads();
    double dxn = s_red[0];
    for (int w = 1; w < MGS_THREADS / 64; ++w) dxn = nanmax(dxn, s_red[w]);
    const bool isnan_dx = dxn != dxn;
    if (!isnan_dx) {
        double *xb = a.x + (size_t)b * a.x_pstride;
        for (int i = tid; i < n; i += MGS_THREADS) {
            double *p = xb + (size_t)i * W;
            cstore(p, cadd(cload<R>(p), cload<R>(dxb + (size_t)i * W)));
        }
    }
    if (tid == 0) {
        if (a.mode == MGS_NEWTON_STEP) {
            double res = 0.0;
            for (int q = 0; q < a.nparts; ++q) res = nanmax(res, a.norm_part[(size_t)b * a.nparts + q]);
            if (a.norms) {
                a.norms[2 * b] = res;
                a.norms[2 * b + 1] = dxn;
            }
            if (a.status) a.status[b] = isnan_dx ? HCN_NAN : HCN_OK;
        } else {
            PathState &st = a.st[b];
            st.dxn = dxn;
            if (isnan_dx) {
                st.c_status = HCN_NAN;
                st.c_active = 0;
            } else if (dxn < st.tol_dx) {
                st.c_status = HCN_OK;
                st.c_active = 0;
            } else {
                st.last = st.res;
                if (st.c_iter >= st.c_maxit) {
                    st.c_status = HCN_NOT_CONVERGED;
                    st.c_active = 0;
                }
            }
        }
    }
}

}  // namespace hcn
