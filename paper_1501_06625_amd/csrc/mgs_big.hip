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
// Pipelined (one cooperative launch): a persistent workgroup per slice of
// columns (column j belongs to workgroup j mod G and stays in its LDS for
// the whole factorisation).  The owner of column k normalises it and
// publishes q_k in place in A (the column's final value) with a flag;
// every workgroup waits for the flags in order, reads q_k from A and
// projects it out of its own later columns, the next column first, so that
// the owner of column k+1 can publish q_{k+1} while the others still work
// on q_k (look-ahead).  The column operations are the right-looking
// variant's (same lanes, rows, butterflies and order), so the results are
// bitwise the same; the trailing matrix never leaves LDS and the step
// boundaries cost a flag instead of a launch.  Waits are bounded: a wait
// that times out (a workgroup not resident, which the cooperative launch
// rules out) or a singular column stops every workgroup of the problem, and
// the epilogue reports the problem as failed (HCN_EDEVICE or ESINGULAR).
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

// full workgroup sums: a 64-lane butterfly adding the lower lane first
// (group_csum / group_sum: DPP moves within rows of 16 lanes, permutes
// beyond), then the four wavefront sums in order; every lane returns the
// same bits
template <class R>
HCN_DEV cx<R> wg_csum(cx<R> v, cx<R> *s_part) {
    const int tid = threadIdx.x, lane = tid & 63;
    v = group_csum<R, 64>(v, lane);
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
    v = group_sum<R, 64>(v, lane);
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
// R[j][j] and inv[j].  Every lane holds the same squared norm, so every lane
// forms r_jj and 1/r_jj itself (the same bits; no broadcast).  Returns false
// (on every lane) for a singular column.
template <class R>
HCN_DEV bool col_normalise(const MgsArgs &a, int b, int j, double *aj, R *s_part) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    const R s = col_norm2<R>(aj, a.N, s_part);
    const R rkk = sqrt(s);
    if (!(lead(rkk) > 0.0) || !rfinite(rkk)) return false;
    const R iv = div(rmake<R>(1.0), rkk);
    if (threadIdx.x == 0) {
        rstore(a.inv + (size_t)b * a.inv_pstride + (size_t)j * P, iv);
        const cx<R> rc{rkk, rmake<R>(0.0)};
        cstore(a.R + (size_t)b * a.R_pstride + ((size_t)j * a.n + j) * W, rc);
    }
    col_scale<R>(aj, iv, a.N);
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
        if (!col_normalise<R>(a, b, j, aj, s_rpart) && threadIdx.x == 0) sing[b] = 1;
    }
}

// ---------------------------------------------------------------------------
// pipelined: one cooperative launch, columns resident in LDS
// ---------------------------------------------------------------------------
// sing[b]: 0 running, 1 singular column, 2 a wait timed out
constexpr int PIPE_SINGULAR = 1, PIPE_TIMEOUT = 2;

// Thread 0 waits (bounded) until flags[k] is set or the problem stopped;
// the acquire fence then makes the published column visible to the
// workgroup.  Returns false (on every thread) when the problem stopped.
HCN_DEV bool pipe_wait(const int *flag, int *stop_word, long spin_limit, int *s_go) {
    if (threadIdx.x == 0) {
        int go = 1;
        long spins = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            if (__hip_atomic_load(stop_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                go = 0;
                break;
            }
            if (++spins > spin_limit) {
                __hip_atomic_store(stop_word, PIPE_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                go = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *s_go = go;
    }
    __syncthreads();
    return *s_go != 0;
}

template <class R>
__global__ __launch_bounds__(BT) void k_mgs_pipe(MgsArgs a, int *sing, int *flags, long spin_limit) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    extern __shared__ double lds[];  // own columns [c][N][W]
    __shared__ cx<R> s_part[BT / 64];
    __shared__ R s_rpart[BT / 64];
    __shared__ int s_go;
    const int b = blockIdx.y;
    if (!problem_live(a, b)) return;
    const int G = gridDim.x, w = blockIdx.x, n = a.n, N = a.N;
    const size_t cst = (size_t)N * W;
    if (w > n) return;
    const int mine = (n - w) / G + 1;  // columns w, w + G, ...
    int *flg = flags + (size_t)b * (n + 1);
    int *stop = sing + b;
    for (int c = 0; c < mine; ++c) {
        const double *src = col_ptr(a, b, w + c * G);
        for (size_t t = threadIdx.x; t < cst; t += BT) lds[(size_t)c * cst + t] = src[t];
    }
    __syncthreads();
    // column j (owned, in LDS slot c), fully projected: r_jj, 1/r_jj, q_j;
    // q_j goes to its place in A and its flag is raised.  False: singular.
    auto publish = [&](int c) -> bool {
        const int j = w + c * G;
        double *aj = lds + (size_t)c * cst;
        if (!col_normalise<R>(a, b, j, aj, s_rpart)) {
            if (threadIdx.x == 0)
                __hip_atomic_store(stop, PIPE_SINGULAR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __syncthreads();  // the scaled rows, written row-wise, are copied element-wise
        double *dst = col_ptr(a, b, j);
        for (size_t t = threadIdx.x; t < cst; t += BT) dst[t] = aj[t];
        // the workgroup's stores complete before the barrier; the release
        // store writes them back beyond this XCD's L2 before the flag
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(flg + j, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    };
    bool live = true;
    if (w == 0 && n > 0) live = publish(0);
    for (int k = 0; k < n && live; ++k) {
        const double *qk;
        if (k % G == w) {
            qk = lds + (size_t)(k / G) * cst;
        } else {
            // q_k is needed only while this workgroup has a column beyond k
            if (k >= w && w + ((k - w) / G + 1) * G > n) break;
            if (!pipe_wait(flg + k, stop, spin_limit, &s_go)) {
                live = false;
                break;
            }
            // each lane reads its own rows of the published q_k (the first
            // column's dot product fetches them, later ones hit the caches)
            qk = col_ptr(a, b, k);
        }
        // own columns j > k in increasing order (column k+1 first)
        const int c0 = k < w ? 0 : (k - w) / G + 1;
        for (int c = c0; c < mine && live; ++c) {
            const int j = w + c * G;
            double *aj = lds + (size_t)c * cst;
            const cx<R> r = col_dot<R>(qk, aj, N, s_part);
            if (threadIdx.x == 0)
                cstore(a.R + (size_t)b * a.R_pstride + ((size_t)j * n + k) * W, r);
            col_axpy<R>(qk, aj, r, N);
            if (j == k + 1 && j < n) live = publish(c);
        }
    }
    // the projected right-hand side (column n) goes back to its place
    if (live && n % G == w) {
        __syncthreads();
        const double *src = lds + (size_t)(n / G) * cst;
        double *dst = col_ptr(a, b, n);
        for (size_t t = threadIdx.x; t < cst; t += BT) dst[t] = src[t];
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
    const MgsProblem p = problem_of(a, b);
    if (sing[b] == PIPE_TIMEOUT) {
        // a wait of the pipelined variant timed out: the factorisation is
        // incomplete, reported as a device error of this problem
        if (threadIdx.x == 0) {
            if (p.status) *p.status = HCN_EDEVICE;
            if (p.mode == MGS_NEWTON_FIG2 || p.mode == MGS_MIXED_SOLVE) {
                p.st->c_status = HCN_EDEVICE;
                p.st->c_active = 0;
            }
            if (p.mode == MGS_NEWTON_STEP && p.norms) {
                p.norms[0] = residual_norm(p);
                p.norms[1] = __builtin_nan("");
            }
        }
        return;
    }
    mgs_epilogue<R>(p, sing[b] != 0);
}

__global__ void k_zero_int(int *p, int count) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) p[q] = 0;
}

// workgroups of the pipelined variant for one problem (0: it does not fit):
// at most one per CU-slot the occupancy calculator allows with the LDS of
// its columns, and B of them must be resident together
template <class R>
static int pipe_groups(const MgsArgs &a, size_t *lds_out) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
    }
    const size_t cst = (size_t)a.N * 2 * limbs<R>::P * sizeof(double);
    int G = std::min(cus / std::max(a.B, 1), a.n + 1);
    if (G < 1) return 0;
    const int mine = a.n / G + 1;
    const size_t lds = (size_t)mine * cst;
    if (lds > 160 * 1024) return 0;
    (void)hipFuncSetAttribute((const void *)k_mgs_pipe<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mgs_pipe<R>, BT, lds) != hipSuccess ||
        per_cu < 1)
        return 0;
    *lds_out = lds;
    return G;
}

// bounded waits: about a second of polling before a wait gives up
constexpr long PIPE_SPIN_LIMIT = 1L << 22;

template <class R>
static int launch_big_t(const MgsArgs &a, int variant, int *ints, hipStream_t s) {
    // ints: sing[B], then (after 2B + 1) the column flags [B][n + 1]
    int *sing = ints;
    int *flags = ints + 2 * a.B + 1;
    size_t pipe_lds = 0;
    const int G = variant == 5 ? pipe_groups<R>(a, &pipe_lds) : 0;
    if (variant == 5 && G == 0) variant = 2;
    const long nz = variant == 5 ? 2L * a.B + 1 + (long)a.B * (a.n + 1) : a.B;
    hipLaunchKernelGGL(k_zero_int, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, ints, (int)nz);
    if (a.mode == MGS_NEWTON_FIG2)
        hipLaunchKernelGGL(k_fig2_pre, dim3((a.B + 255) / 256), dim3(256), 0, s, a);
    {
        ProfScope prof("mgs", s);
        if (variant == 5) {
            MgsArgs av = a;
            long spin = PIPE_SPIN_LIMIT;
            void *args[] = {&av, &sing, &flags, &spin};
            const hipError_t e = hipLaunchCooperativeKernel((const void *)k_mgs_pipe<R>, dim3(G, a.B),
                                                            dim3(BT), args, (unsigned)pipe_lds, s);
            if (e != hipSuccess) return (int)e;
        } else if (variant == 4) {
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
