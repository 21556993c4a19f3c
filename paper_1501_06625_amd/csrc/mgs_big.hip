// mgs_big.hip -- modified Gram-Schmidt for large systems (hundreds of
// columns), where the linear algebra dominates the cost of a Newton step
// (Section 1: sparse systems of low degree need dimensions of several
// hundreds; the right-looking algorithm gives the most thread parallelism,
// and combining it with left-looking tiles cuts memory traffic).
//
// Every variant applies, to every column j, the projections k = 0, 1, ...,
// j-1 in that order.
//
// Right-looking: one launch per column step k; the workgroup of trailing
// column j > k forms r_kj = q_k^H a_j and a_j -= r_kj q_k on global memory
// (lane t sums rows t, t+256, ... in order; a 64-lane butterfly adding the
// lower lane first; the four wavefront sums added in order); the workgroup
// of column k+1 then also normalises it (r_{k+1,k+1}, q_{k+1}).  The
// trailing matrix is read and written once per step.
//
// Tiled (panel width T; mgs_tiled.hpp): the columns are taken T at a time.
// A panel launch factors columns k0..k0+T-1 in one workgroup of T
// wavefronts, each holding one column in registers; a trailing launch gives
// every later column (the right-hand side included) a wavefront that applies
// the panel's T projections in order, so a trailing column is read and
// written once per panel rather than once per column.  Reductions are per
// wavefront, so this variant agrees with the other two to rounding, not
// bitwise.
#include <algorithm>

#include "internal.hpp"
#include "mgs_common.hpp"
#include "mgs_tiled.hpp"
#include "mp.hpp"
#include "prof.hpp"

namespace hcn {

constexpr int BT = MGS_THREADS;

HCN_DEV double bshfl(double v, int m) { return __shfl_xor(v, m); }
HCN_DEV dd bshfl(const dd &v, int m) { return dd{bshfl(v.hi, m), bshfl(v.lo, m)}; }
HCN_DEV qd bshfl(const qd &v, int m) {
    return qd{bshfl(v.c0, m), bshfl(v.c1, m), bshfl(v.c2, m), bshfl(v.c3, m)};
}

// full workgroup sums; every lane returns the same bits
template <class R>
HCN_DEV cx<R> wg_csum(cx<R> v, cx<R> *s_part) {
    const int tid = threadIdx.x, lane = tid & 63;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const cx<R> o{bshfl(v.re, m), bshfl(v.im, m)};
        v = (lane & m) ? cadd(o, v) : cadd(v, o);
    }
    if (lane == 0) s_part[tid >> 6] = v;
    __syncthreads();
    cx<R> s = s_part[0];
#pragma unroll
    for (int w = 1; w < BT / 64; ++w) s = cadd(s, s_part[w]);
    __syncthreads();
    return s;
}

template <class R>
HCN_DEV R wg_rsum(R v, R *s_part) {
    const int tid = threadIdx.x, lane = tid & 63;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const R o = bshfl(v, m);
        v = (lane & m) ? add(o, v) : add(v, o);
    }
    if (lane == 0) s_part[tid >> 6] = v;
    __syncthreads();
    R s = s_part[0];
#pragma unroll
    for (int w = 1; w < BT / 64; ++w) s = add(s, s_part[w]);
    __syncthreads();
    return s;
}

template <class R>
HCN_DEV cx<R> col_dot(const double *q, const double *a, int N, cx<R> *s_part) {
    constexpr int W = 2 * limbs<R>::P;
    cx<R> acc = czero<R>();
    bool first = true;
    for (int i = threadIdx.x; i < N; i += BT) {
        const cx<R> v = cmul_conj(cload<R>(q + (size_t)i * W), cload<R>(a + (size_t)i * W));
        acc = first ? v : cadd(acc, v);
        first = false;
    }
    return wg_csum(acc, s_part);
}

template <class R>
HCN_DEV void col_axpy(const double *q, double *a, const cx<R> &r, int N) {
    constexpr int W = 2 * limbs<R>::P;
    for (int i = threadIdx.x; i < N; i += BT) {
        double *p = a + (size_t)i * W;
        cstore(p, csub(cload<R>(p), cmul(r, cload<R>(q + (size_t)i * W))));
    }
}

template <class R>
HCN_DEV R col_norm2(const double *a, int N, R *s_part) {
    constexpr int W = 2 * limbs<R>::P;
    R acc = rmake<R>(0.0);
    bool first = true;
    for (int i = threadIdx.x; i < N; i += BT) {
        const R v = cnorm2(cload<R>(a + (size_t)i * W));
        acc = first ? v : add(acc, v);
        first = false;
    }
    return wg_rsum(acc, s_part);
}

template <class R>
HCN_DEV void col_scale(double *a, const R &iv, int N) {
    constexpr int W = 2 * limbs<R>::P;
    for (int i = threadIdx.x; i < N; i += BT) {
        double *p = a + (size_t)i * W;
        cstore(p, cscale(iv, cload<R>(p)));
    }
}

// r_jj = ||a_j||, 1/r_jj and q_j = a_j / r_jj on the column at `aj`; writes
// R[j][j] and inv[j].  Returns false (on every lane) for a singular column.
template <class R>
HCN_DEV bool col_normalise(const MgsArgs &a, int b, int j, double *aj, R *s_part, R *s_inv,
                           int *s_bad) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    const R s = col_norm2<R>(aj, a.N, s_part);
    if (threadIdx.x == 0) {
        const R rkk = sqrt(s);
        const bool bad = !(lead(rkk) > 0.0) || !rfinite(rkk);
        *s_bad = bad ? 1 : 0;
        if (!bad) {
            const R iv = div(rmake<R>(1.0), rkk);
            *s_inv = iv;
            rstore(a.inv + (size_t)b * a.inv_pstride + (size_t)j * P, iv);
            const cx<R> rc{rkk, rmake<R>(0.0)};
            cstore(a.R + (size_t)b * a.R_pstride + ((size_t)j * a.n + j) * W, rc);
        }
    }
    __syncthreads();
    if (*s_bad) return false;
    col_scale<R>(aj, *s_inv, a.N);
    return true;
}

HCN_DEV double *col_ptr(const MgsArgs &a, int b, int j) {
    double *Ab = a.A + (size_t)b * a.A_pstride;
    if (j < a.n) return Ab + (size_t)j * a.A_cstride;
    return a.bcol ? a.bcol + (size_t)b * a.b_pstride : Ab + (size_t)a.n * a.A_cstride;
}

HCN_DEV bool problem_live(const MgsArgs &a, int b) {
    return (a.mode != MGS_NEWTON_FIG2 && a.mode != MGS_MIXED_SOLVE) || a.st[b].c_active;
}

// ---------------------------------------------------------------------------
// right-looking: one launch per column step (k = -1 normalises column 0)
// ---------------------------------------------------------------------------
template <class R>
__global__ __launch_bounds__(BT) void k_mgs_rl(MgsArgs a, int k, int *sing) {
    constexpr int W = 2 * limbs<R>::P;
    __shared__ cx<R> s_part[BT / 64];
    __shared__ R s_rpart[BT / 64];
    __shared__ R s_inv;
    __shared__ int s_bad;
    const int b = blockIdx.y;
    if (!problem_live(a, b) || sing[b]) return;
    const int j = (k < 0) ? 0 : k + 1 + (int)blockIdx.x;
    if (j > a.n) return;
    double *aj = col_ptr(a, b, j);
    if (k >= 0) {
        const double *qk = col_ptr(a, b, k);
        const cx<R> r = col_dot<R>(qk, aj, a.N, s_part);
        if (threadIdx.x == 0)
            cstore(a.R + (size_t)b * a.R_pstride + ((size_t)j * a.n + k) * W, r);
        col_axpy<R>(qk, aj, r, a.N);
    }
    if (j == k + 1 && j < a.n) {
        if (!col_normalise<R>(a, b, j, aj, s_rpart, &s_inv, &s_bad) && threadIdx.x == 0) sing[b] = 1;
    }
}

// ---------------------------------------------------------------------------
// tiled: panel and trailing launches over the bodies in mgs_tiled.hpp
// ---------------------------------------------------------------------------
// Panel k0..k1-1 of problem blockIdx.x; blockDim.x = 64 (k1 - k0).  The
// columns before k0 have been projected out of every panel column already.
template <class R, int RPL>
__global__ __launch_bounds__((64 * tiled_max_waves<R, RPL>())) void k_mgs_tpanel(MgsArgs a, int k0,
                                                                                   int k1, int *sing) {
    extern __shared__ double qbuf[];  // [N][W]: the newest q_k
    const int b = blockIdx.x;
    if (!problem_live(a, b) || sing[b]) return;
    tiled_panel<R, RPL>(problem_of(a, b), k0, k1, sing + b, qbuf);
}

// Columns j >= k1 (the right-hand side j = n included), four per workgroup.
template <class R, int RPL>
__global__ __launch_bounds__(BT) void k_mgs_ttrail(MgsArgs a, int k0, int k1, int *sing) {
    const int b = blockIdx.y;
    if (!problem_live(a, b) || sing[b]) return;
    const int j = k1 + 4 * (int)blockIdx.x + (int)(threadIdx.x >> 6);
    if (j > a.n) return;
    tiled_trail<R, RPL>(problem_of(a, b), k0, k1, j);
}

int mgs_tiled_rpl(int N, int P) { return tiled_rpl(N, P); }

static int g_panel = 16;

int mgs_panel_width() { return g_panel; }
void set_mgs_panel_width(int T) { g_panel = T; }

template <class R, int RPL>
static void launch_tiled_rpl(const MgsArgs &a, int *sing, hipStream_t s) {
    const int T = std::min(g_panel, tiled_max_waves<R, RPL>());
    const size_t lds = (size_t)a.N * 2 * limbs<R>::P * sizeof(double);
    (void)hipFuncSetAttribute((const void *)k_mgs_tpanel<R, RPL>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    for (int k0 = 0; k0 < a.n; k0 += T) {
        const int k1 = std::min(k0 + T, a.n);
        hipLaunchKernelGGL((k_mgs_tpanel<R, RPL>), dim3(a.B), dim3(64 * (k1 - k0)), lds, s, a, k0, k1,
                           sing);
        const int cols = a.n + 1 - k1;
        hipLaunchKernelGGL((k_mgs_ttrail<R, RPL>), dim3((cols + 3) / 4, a.B), dim3(BT), 0, s, a, k0, k1,
                           sing);
    }
}

template <class R>
static void launch_tiled(const MgsArgs &a, int *sing, hipStream_t s) {
    switch (mgs_tiled_rpl(a.N, limbs<R>::P)) {
        case 1: launch_tiled_rpl<R, 1>(a, sing, s); break;
        case 2: launch_tiled_rpl<R, 2>(a, sing, s); break;
        case 4: launch_tiled_rpl<R, 4>(a, sing, s); break;
        default:
            if constexpr (limbs<R>::P != 4) launch_tiled_rpl<R, 8>(a, sing, s);
            break;
    }
}

// ---------------------------------------------------------------------------
// pre-solve Fig. 2 tests and the epilogue for the multi-workgroup variants
// ---------------------------------------------------------------------------
__global__ void k_fig2_pre(MgsArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < a.B) (void)fig2_decide(problem_of(a, b));
}

template <class R>
__global__ __launch_bounds__(BT) void k_mgs_finish(MgsArgs a, const int *sing) {
    const int b = blockIdx.x;
    if (!problem_live(a, b)) return;
    mgs_epilogue<R>(problem_of(a, b), sing[b] != 0);
}

__global__ void k_zero_int(int *p, int count) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) p[q] = 0;
}

template <class R>
static int launch_big_t(const MgsArgs &a, int variant, int *ints, hipStream_t s) {
    // ints: sing[B]
    int *sing = ints;
    hipLaunchKernelGGL(k_zero_int, dim3((a.B + 255) / 256), dim3(256), 0, s, ints, a.B);
    if (a.mode == MGS_NEWTON_FIG2)
        hipLaunchKernelGGL(k_fig2_pre, dim3((a.B + 255) / 256), dim3(256), 0, s, a);
    {
        ProfScope prof("mgs", s);
        if (variant == 4) {
            launch_tiled<R>(a, sing, s);
        } else {
            hipLaunchKernelGGL(k_mgs_rl<R>, dim3(1, a.B), dim3(BT), 0, s, a, -1, sing);
            for (int k = 0; k < a.n; ++k)
                hipLaunchKernelGGL(k_mgs_rl<R>, dim3(a.n - k, a.B), dim3(BT), 0, s, a, k, sing);
        }
        hipLaunchKernelGGL(k_mgs_finish<R>, dim3(a.B), dim3(BT), 0, s, a, sing);
    }
    return (int)hipGetLastError();
}

int launch_mgs_big(int P, const MgsArgs &a, int variant, int *ints, hipStream_t s) {
    if (a.B == 0) return 0;
    if (variant == 4 && mgs_tiled_rpl(a.N, P) == 0) variant = 2;
    if (P == 1) return launch_big_t<double>(a, variant, ints, s);
    return P == 2 ? launch_big_t<dd>(a, variant, ints, s) : launch_big_t<qd>(a, variant, ints, s);
}

int launch_fig2_pre(const MgsArgs &a, hipStream_t s) {
    if (a.B == 0) return 0;
    hipLaunchKernelGGL(k_fig2_pre, dim3((a.B + 255) / 256), dim3(256), 0, s, a);
    return (int)hipGetLastError();
}

}  // namespace hcn
