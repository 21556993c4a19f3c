// mgs.hip -- modified Gram-Schmidt on the augmented matrix [A | b] and back
// substitution (Section 1; Fig. 2, GPU_Modified_Gram_Schmidt), fused with
// the Newton update and the device-side tests of Fig. 2.
//
// One workgroup of 256 lanes per problem, right-looking: for column k the
// first lane group forms ||a_k||^2, one lane takes r_kk = sqrt, 1/r_kk,
// every lane scales its rows of a_k, then each of the 16 lane groups owns
// trailing columns j > k (the right-hand side last), forms r_kj = q_k^H a_j
// from its rows and a butterfly across its 16 lanes, and updates
// a_j -= r_kj q_k on its rows.  Butterflies always add the lower lane's
// value first, so all lanes of a group hold bitwise the same sum.  Back
// substitution is column-oriented: dx_k = y_k / r_kk, then
// y_i -= r_ik dx_k for i < k.
#include "internal.hpp"
#include "mp.hpp"
#include "prof.hpp"
#include "mgs_common.hpp"

namespace hcn {

constexpr int GROUP = 16;  // lanes per column group
constexpr int NGROUPS = MGS_THREADS / GROUP;

HCN_DEV double shfl_x(double v, int m) { return __shfl_xor(v, m); }

HCN_DEV dd shfl_x(const dd &v, int m) { return dd{shfl_x(v.hi, m), shfl_x(v.lo, m)}; }
HCN_DEV qd shfl_x(const qd &v, int m) {
    return qd{shfl_x(v.c0, m), shfl_x(v.c1, m), shfl_x(v.c2, m), shfl_x(v.c3, m)};
}

// sum over the GROUP lanes of a group (lanes of a group are consecutive)
template <class R>
HCN_DEV R group_sum(R v, int lane) {
#pragma unroll
    for (int m = 1; m < GROUP; m <<= 1) {
        const R o = shfl_x(v, m);
        v = (lane & m) ? add(o, v) : add(v, o);
    }
    return v;
}

template <class R>
HCN_DEV cx<R> group_csum(cx<R> v, int lane) {
#pragma unroll
    for (int m = 1; m < GROUP; m <<= 1) {
        const cx<R> o{shfl_x(v.re, m), shfl_x(v.im, m)};
        v = (lane & m) ? cadd(o, v) : cadd(v, o);
    }
    return v;
}

template <class R>
__global__ __launch_bounds__(MGS_THREADS) void k_mgs(MgsArgs a) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    const int b = blockIdx.x;
    const int tid = threadIdx.x;
    const int g = tid / GROUP;
    const int lane = tid % GROUP;
    const int N = a.N, n = a.n;
    __shared__ int s_flag;
    __shared__ double s_inv[4];

    // ---- Fig. 2 tests before the solve (residual norm vs previous, tolerance)
    if (a.mode == MGS_NEWTON_FIG2 || a.mode == MGS_MIXED_SOLVE) {
        // one lane reads and decides; the others learn it through LDS
        if (tid == 0) s_flag = a.mode == MGS_NEWTON_FIG2 ? fig2_decide(a, b) : !a.st[b].c_active;
        __syncthreads();
        if (s_flag) return;
    }

    double *Ab = a.A + (size_t)b * a.A_pstride;
    double *bb = a.bcol ? a.bcol + (size_t)b * a.b_pstride : Ab + (size_t)n * a.A_cstride;
    double *Rb = a.R + (size_t)b * a.R_pstride;
    double *invb = a.inv + (size_t)b * a.inv_pstride;
    double *dxb = a.dx + (size_t)b * a.dx_pstride;
    auto col = [&](int j) -> double * { return j < n ? Ab + (size_t)j * a.A_cstride : bb; };

    if (tid == 0) s_flag = 0;
    __syncthreads();

    for (int k = 0; k < n; ++k) {
        double *ak = col(k);
        if (g == 0) {
            R s = rmake<R>(0.0);
            bool first = true;
            for (int i = lane; i < N; i += GROUP) {
                const R v = cnorm2(cload<R>(ak + (size_t)i * W));
                s = first ? v : add(s, v);
                first = false;
            }
            s = group_sum(s, lane);
            if (lane == 0) {
                const R rkk = sqrt(s);
                const bool bad = !(lead(rkk) > 0.0) || !rfinite(rkk);
                if (bad) {
                    s_flag = 1;
                } else {
                    const R iv = div(rmake<R>(1.0), rkk);
                    rstore(invb + (size_t)k * P, iv);
                    rstore(s_inv, iv);
                    const cx<R> rc{rkk, rmake<R>(0.0)};
                    cstore(Rb + ((size_t)k * n + k) * W, rc);
                }
            }
        }
        __syncthreads();
        if (s_flag) break;
        R iv;
        rload(s_inv, iv);
        for (int i = tid; i < N; i += MGS_THREADS) {
            double *p = ak + (size_t)i * W;
            cstore(p, cscale(iv, cload<R>(p)));
        }
        __syncthreads();
        for (int j = k + 1 + g; j <= n; j += NGROUPS) {
            double *aj = col(j);
            cx<R> r = czero<R>();
            bool first = true;
            for (int i = lane; i < N; i += GROUP) {
                const cx<R> v = cmul_conj(cload<R>(ak + (size_t)i * W), cload<R>(aj + (size_t)i * W));
                r = first ? v : cadd(r, v);
                first = false;
            }
            r = group_csum(r, lane);
            if (lane == 0) cstore(Rb + ((size_t)j * n + k) * W, r);
            for (int i = lane; i < N; i += GROUP) {
                double *p = aj + (size_t)i * W;
                cstore(p, csub(cload<R>(p), cmul(r, cload<R>(ak + (size_t)i * W))));
            }
        }
        __syncthreads();
    }

    mgs_epilogue<R>(a, b, s_flag != 0);
}

int launch_mgs(int P, const MgsArgs &a, hipStream_t stream) {
    if (a.B == 0) return 0;
    ProfScope prof("mgs", stream);
    if (P == 1)
        hipLaunchKernelGGL(k_mgs<double>, dim3(a.B), dim3(MGS_THREADS), 0, stream, a);
    else if (P == 2)
        hipLaunchKernelGGL(k_mgs<dd>, dim3(a.B), dim3(MGS_THREADS), 0, stream, a);
    else
        hipLaunchKernelGGL(k_mgs<qd>, dim3(a.B), dim3(MGS_THREADS), 0, stream, a);
    return (int)hipGetLastError();
}

}  // namespace hcn
