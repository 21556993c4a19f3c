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
// (lane t sums rows t, t+256, ... in order; a 64-lane butterfly; the four
// wavefront sums added pairwise); the workgroup
// of column k+1 then also normalises it (r_{k+1,k+1}, q_{k+1}).  The
// trailing matrix is read and written once per step.
//
// Pipelined (one cooperative launch): a persistent workgroup per slice of
// columns (column j belongs to workgroup j mod G and stays in its LDS for
// the whole factorisation; one workgroup per CU, so the chain of column
// steps always has a CU of its own).  At the start every workgroup marks
// the places of its columns in A empty (a signalling-NaN pattern) and the
// workgroups of a problem meet once.  The owner of column k normalises it
// and publishes q_k in place in A (the column's final value) with
// device-coherent stores: for the workgroups next on the chain (whose next
// column is k+1 or k+2) the data are their own flag, each lane polling its
// own rows until none is empty, with no fence or flag word on the chain;
// the others wait for a flag the owner raises once its stores are complete.
// Every workgroup takes the q_k in order and projects each out of its own
// later columns, its next column first (while that column is k+2 the
// others wait), so that the owner of column k+1 can publish q_{k+1} while
// the others still work on q_k (look-ahead).  The column operations are
// the right-looking variant's (same lanes, rows, butterflies and order), so
// the results are bitwise the same; the trailing matrix never leaves LDS
// and the step boundaries cost no launch.  Waits
// are bounded: a wait that times out (a workgroup not resident, which the
// cooperative launch rules out) or a singular column stops every workgroup
// of the problem, and the epilogue reports the problem as failed
// (HCN_EDEVICE or ESINGULAR).
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

// Team operations on one column.  A team is 256 lanes (four wavefronts);
// lane t of the team holds rows t, t + 256, ... .  A sum over the column is
// lane t's rows in order, a 64-lane butterfly (group_csum / group_sum: DPP
// moves within rows of 16 lanes, permutes beyond), then the four wavefront
// sums added pairwise, so every lane of the team returns the same bits.  The right-looking workgroup is one team; the
// pipelined workgroup is one team too.  `act` false: the lane adds no rows
// (its part of the sum is zero) but keeps the barriers.
constexpr int TEAM = MGS_THREADS;

template <class T>
HCN_DEV T sum2(const T &a, const T &b) { return add(a, b); }
template <class R>
HCN_DEV cx<R> sum2(const cx<R> &a, const cx<R> &b) { return cadd(a, b); }

// The TEAM / 64 wavefront sums added pairwise, (w0 + w1) + (w2 + w3): two
// dependent additions instead of three, the same order on every lane
template <class T>
HCN_DEV T wave_tree(const T *part) {
    T v[TEAM / 64];
#pragma unroll
    for (int w = 0; w < TEAM / 64; ++w) v[w] = part[w];
#pragma unroll
    for (int h = 1; h < TEAM / 64; h <<= 1)
#pragma unroll
        for (int w = 0; w + h < TEAM / 64; w += 2 * h) v[w] = sum2(v[w], v[w + h]);
    return v[0];
}

// The partial sums go through a ring of two slots, taken in turn (`ph`
// flips at every call; every lane of the team makes the same calls): a slot
// is written again only two sums later, after the barrier of the sum in
// between, which every lane passes only once it has read the slot.  One
// barrier per sum.  A complex slot holds two sums' partials (team_csum2).
constexpr int CSLOT = 2 * (TEAM / 64);

template <class R>
HCN_DEV cx<R> team_csum(cx<R> v, int t, cx<R> *ring, int &ph) {
    cx<R> *s_part = ring + ph * CSLOT;
    ph ^= 1;
    const int lane = t & 63;
    v = group_csum<R, 64>(v, lane);
    if (lane == 0) s_part[t >> 6] = v;
    lds_barrier();
    return wave_tree(s_part);
}

// two independent sums side by side, each in team_csum's order
template <class R>
HCN_DEV void team_csum2(cx<R> &v0, cx<R> &v1, int t, cx<R> *ring, int &ph) {
    cx<R> *s_part = ring + ph * CSLOT;
    ph ^= 1;
    const int lane = t & 63;
    v0 = group_csum<R, 64>(v0, lane);
    v1 = group_csum<R, 64>(v1, lane);
    if (lane == 0) {
        s_part[t >> 6] = v0;
        s_part[TEAM / 64 + (t >> 6)] = v1;
    }
    lds_barrier();
    v0 = wave_tree(s_part);
    v1 = wave_tree(s_part + TEAM / 64);
}

template <class R>
HCN_DEV R team_rsum(R v, int t, R *ring, int &ph) {
    R *s_part = ring + ph * (TEAM / 64);
    ph ^= 1;
    const int lane = t & 63;
    v = group_sum<R, 64>(v, lane);
    if (lane == 0) s_part[t >> 6] = v;
    lds_barrier();
    return wave_tree(s_part);
}

// the two rings of a team's sums (complex dot products, real squared norms)
template <class R>
struct TeamSums {
    cx<R> *c;
    R *r;
    int pc, pr;
    HCN_DEV TeamSums(cx<R> *c_ring, R *r_ring) : c(c_ring), r(r_ring), pc(0), pr(0) {}
};

// A column as rows of complex numbers: limb l of row i at p[i * step + l * ld].
// In global memory a column is interleaved (step = 2P, ld = 1, the
// boundary's layout); the pipelined variant keeps its columns planar in
// LDS (step = 1, ld = N: limb planes of N doubles), so that the 64 lanes of
// a wavefront reading one limb of consecutive rows touch consecutive
// doubles instead of doubles 2P apart (bank conflicts).
struct Col {
    double *p;
    int ld, step;
};
template <class R>
HCN_DEV Col interleaved(double *p) {
    return Col{p, 1, 2 * limbs<R>::P};
}
HCN_DEV Col planar(double *p, int N) { return Col{p, N, 1}; }

template <class R>
HCN_DEV cx<R> col_ld(const Col &c, int i) {
    constexpr int W = 2 * limbs<R>::P;
    double v[W];
#pragma unroll
    for (int l = 0; l < W; ++l) v[l] = c.p[(size_t)i * c.step + (size_t)l * c.ld];
    return cload<R>(v);
}
template <class R>
HCN_DEV void col_st(const Col &c, int i, const cx<R> &x) {
    constexpr int W = 2 * limbs<R>::P;
    double v[W];
    cstore(v, x);
#pragma unroll
    for (int l = 0; l < W; ++l) c.p[(size_t)i * c.step + (size_t)l * c.ld] = v[l];
}

// q^H a over the column
template <class R>
HCN_DEV cx<R> col_dot(const Col &q, const Col &a, int N, int t, TeamSums<R> &ts, bool act = true) {
    cx<R> acc = czero<R>();
    bool first = true;
    if (act) {
        for (int i = t; i < N; i += TEAM) {
            const cx<R> v = cmul_conj(col_ld<R>(q, i), col_ld<R>(a, i));
            acc = first ? v : cadd(acc, v);
            first = false;
        }
    }
    return team_csum(acc, t, ts.c, ts.pc);
}

template <class R>
HCN_DEV void col_axpy(const Col &q, const Col &a, const cx<R> &r, int N, int t) {
    for (int i = t; i < N; i += TEAM) col_st<R>(a, i, csub(col_ld<R>(a, i), cmul(r, col_ld<R>(q, i))));
}

// r0 = q^H a0, r1 = q^H a1 and a0 -= r0 q, a1 -= r1 q side by side: two
// independent chains for the scheduler, each in the order of col_dot and
// col_axpy (the same bits)
template <class R>
HCN_DEV void col_update2(const Col &q, const Col &a0, const Col &a1, int N, int t, TeamSums<R> &ts,
                         cx<R> &r0, cx<R> &r1) {
    cx<R> acc0 = czero<R>(), acc1 = czero<R>();
    bool first = true;
    for (int i = t; i < N; i += TEAM) {
        const cx<R> qi = col_ld<R>(q, i);
        const cx<R> v0 = cmul_conj(qi, col_ld<R>(a0, i));
        const cx<R> v1 = cmul_conj(qi, col_ld<R>(a1, i));
        acc0 = first ? v0 : cadd(acc0, v0);
        acc1 = first ? v1 : cadd(acc1, v1);
        first = false;
    }
    team_csum2(acc0, acc1, t, ts.c, ts.pc);
    r0 = acc0;
    r1 = acc1;
    for (int i = t; i < N; i += TEAM) {
        const cx<R> qi = col_ld<R>(q, i);
        col_st<R>(a0, i, csub(col_ld<R>(a0, i), cmul(r0, qi)));
        col_st<R>(a1, i, csub(col_ld<R>(a1, i), cmul(r1, qi)));
    }
}

template <class R>
HCN_DEV R col_norm2(const Col &a, int N, int t, TeamSums<R> &ts, bool act = true) {
    R acc = rmake<R>(0.0);
    bool first = true;
    if (act) {
        for (int i = t; i < N; i += TEAM) {
            const R v = cnorm2(col_ld<R>(a, i));
            acc = first ? v : add(acc, v);
            first = false;
        }
    }
    return team_rsum(acc, t, ts.r, ts.pr);
}

// a -= r q, returning the lane's part of ||a||^2 over the updated rows, in
// col_norm2's order (team_rsum of it gives col_norm2's bits)
template <class R>
HCN_DEV R col_axpy_norm2(const Col &q, const Col &a, const cx<R> &r, int N, int t) {
    R acc = rmake<R>(0.0);
    bool first = true;
    for (int i = t; i < N; i += TEAM) {
        const cx<R> u = csub(col_ld<R>(a, i), cmul(r, col_ld<R>(q, i)));
        col_st<R>(a, i, u);
        const R v = cnorm2(u);
        acc = first ? v : add(acc, v);
        first = false;
    }
    return acc;
}

// Loads and stores coherent across the device (agent-scope atomics: they
// reach the memory side, past the per-XCD L2), for columns handed from one
// workgroup to another inside a launch
HCN_DEV double ld_device(const double *p) {
    return __longlong_as_double(
        __hip_atomic_load((long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
HCN_DEV void st_device(double *p, double v) {
    __hip_atomic_store((long long *)p, __double_as_longlong(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// a *= iv in place; with `copy` (interleaved, global), the scaled rows also
// go there with device-coherent stores
template <class R>
HCN_DEV void col_scale(const Col &a, const R &iv, int N, int t, double *copy = nullptr) {
    constexpr int W = 2 * limbs<R>::P;
    for (int i = t; i < N; i += TEAM) {
        const cx<R> v = cscale(iv, col_ld<R>(a, i));
        col_st<R>(a, i, v);
        if (copy) {
            double tmp[W];
            cstore(tmp, v);
#pragma unroll
            for (int l = 0; l < W; ++l) st_device(copy + (size_t)i * W + l, tmp[l]);
        }
    }
}

// r_jj = ||a_j|| and 1/r_jj from the squared norm s (the same bits on every
// lane of the team); stores R[j][j] and inv[j] (lane t == 0).  False for a
// singular column.
template <class R>
HCN_DEV bool col_pivot(const MgsArgs &a, int b, int j, const R &s, int t, R *iv_out) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    const R rkk = sqrt(s);
    if (!(lead(rkk) > 0.0) || !rfinite(rkk)) return false;
    const R iv = div(rmake<R>(1.0), rkk);
    if (t == 0) {
        rstore(a.inv + (size_t)b * a.inv_pstride + (size_t)j * P, iv);
        const cx<R> rc{rkk, rmake<R>(0.0)};
        cstore(a.R + (size_t)b * a.R_pstride + ((size_t)j * a.n + j) * W, rc);
    }
    *iv_out = iv;
    return true;
}

// r_jj, 1/r_jj and q_j = a_j / r_jj on the column at `aj` by the one-team
// workgroup; false (on every lane) for a singular column
template <class R>
HCN_DEV bool col_normalise(const MgsArgs &a, int b, int j, double *aj, const R &s2) {
    const int t = threadIdx.x;
    const Col c = interleaved<R>(aj);
    R iv;
    if (!col_pivot<R>(a, b, j, s2, t, &iv)) return false;
    col_scale<R>(c, iv, a.N, t);
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
    __shared__ cx<R> s_part[2 * CSLOT];
    __shared__ R s_rpart[2 * (BT / 64)];
    TeamSums<R> ts(s_part, s_rpart);
    const int b = blockIdx.y;
    if (!problem_live(a, b) || sing[b]) return;
    const int j = (k < 0) ? 0 : k + 1 + (int)blockIdx.x;
    if (j > a.n) return;
    double *aj = col_ptr(a, b, j);
    const Col c = interleaved<R>(aj);
    const bool next = j == k + 1 && j < a.n;
    R part = rmake<R>(0.0);  // the lane's part of the squared norm of column k+1
    if (k >= 0) {
        const double *qk = col_ptr(a, b, k);
        const Col q = interleaved<R>((double *)qk);
        const cx<R> r = col_dot<R>(q, c, a.N, threadIdx.x, ts);
        if (threadIdx.x == 0)
            cstore(a.R + (size_t)b * a.R_pstride + ((size_t)j * a.n + k) * W, r);
        if (next)
            part = col_axpy_norm2<R>(q, c, r, a.N, threadIdx.x);
        else
            col_axpy<R>(q, c, r, a.N, threadIdx.x);
    }
    if (next) {
        const R s2 = k >= 0 ? team_rsum(part, (int)threadIdx.x, ts.r, ts.pr) : col_norm2<R>(c, a.N, threadIdx.x, ts);
        if (!col_normalise<R>(a, b, j, aj, s2) && threadIdx.x == 0) sing[b] = 1;
    }
}

// ---------------------------------------------------------------------------
// pipelined: one cooperative launch, columns resident in LDS
// ---------------------------------------------------------------------------
// sing[b]: 0 running, 1 singular column, 2 a wait timed out
constexpr int PIPE_SINGULAR = 1, PIPE_TIMEOUT = 2;

// Bit pattern of a not-yet-published word of a column: a signalling NaN.
// Published words are results of floating-point arithmetic (q_k = a_k / r_kk
// limb by limb), which never yields a signalling NaN, so a word differing
// from this pattern holds its final value.
constexpr long long PIPE_EMPTY = 0x7FF0DEAD5EA1BEEFLL;

HCN_DEV long long ld_device_bits(const double *p) {
    return __hip_atomic_load((long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One lane's wait for its rows of a published column: the data are their
// own flag.  The lane loads its words of the column at src (interleaved)
// with device-coherent loads into its rows of the staging column qs
// (planar), every word at every poll, until no word is empty.  Bounded:
// false once the problem stopped (stop word set by another workgroup) or
// the spin limit passed (the lane then sets the stop word to PIPE_TIMEOUT).
// Two polls in flight, half a round trip apart, for up to FETCH_ROWS rows
// per lane: the words are seen sooner after they land.
constexpr int FETCH_ROWS = 2;

template <class R>
HCN_DEV bool pipe_fetch2(const double *src, double *qs, int N, int t, int *stop_word, long spin_limit) {
    constexpr int W = 2 * limbs<R>::P;
    // a poll: the lane's words and the stop word, loaded together
    struct Poll {
        long long w[FETCH_ROWS][W];
        int stop;
    };
    Poll a, b;
    // rows past N read row t again (their words are not used)
    auto issue = [&](Poll &x) {
#pragma unroll
        for (int r = 0; r < FETCH_ROWS; ++r) {
            const int i = t + r * TEAM < N ? t + r * TEAM : t;
#pragma unroll
            for (int l = 0; l < W; ++l) x.w[r][l] = ld_device_bits(src + (size_t)i * W + l);
        }
        x.stop = __hip_atomic_load(stop_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };
    // 1: complete (staged), 0: not yet, -1: give up
    long spins = 0;
    auto take = [&](const Poll &x) -> int {
        bool all = true;
#pragma unroll
        for (int r = 0; r < FETCH_ROWS; ++r)
#pragma unroll
            for (int l = 0; l < W; ++l) all = all && x.w[r][l] != PIPE_EMPTY;
        if (all) {
#pragma unroll
            for (int r = 0; r < FETCH_ROWS; ++r) {
                const int i = t + r * TEAM;
                if (i < N)
#pragma unroll
                    for (int l = 0; l < W; ++l) qs[(size_t)l * N + i] = __longlong_as_double(x.w[r][l]);
            }
            return 1;
        }
        if (x.stop != 0) return -1;
        if (++spins > spin_limit) {
            __hip_atomic_store(stop_word, PIPE_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
        return 0;
    };
    issue(a);
    for (;;) {
        __builtin_amdgcn_s_sleep(8);
        issue(b);
        int r = take(a);
        if (r != 0) return r > 0;
        __builtin_amdgcn_s_sleep(8);
        issue(a);
        r = take(b);
        if (r != 0) return r > 0;
    }
}

template <class R>
HCN_DEV bool pipe_fetch(const double *src, double *qs, int N, int t, int *stop_word, long spin_limit) {
    constexpr int W = 2 * limbs<R>::P;
    if (t >= N) return true;
    if (N <= FETCH_ROWS * TEAM) return pipe_fetch2<R>(src, qs, N, t, stop_word, spin_limit);
    long spins = 0;
    for (;;) {
        bool all = true;
        for (int i = t; i < N; i += TEAM)
#pragma unroll
            for (int l = 0; l < W; ++l) {
                const long long v = ld_device_bits(src + (size_t)i * W + l);
                all = all && v != PIPE_EMPTY;
                qs[(size_t)l * N + i] = __longlong_as_double(v);
            }
        if (all) return true;
        if (__hip_atomic_load(stop_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (++spins > spin_limit) {
            __hip_atomic_store(stop_word, PIPE_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Thread 0's bounded wait until flags[k] is set or the problem stopped
// (false on every thread then); the column's stores completed before its
// flag was raised.
HCN_DEV bool pipe_wait(int *flag, int *stop_word, long spin_limit, int *s_go) {
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
        *s_go = go;
    }
    __syncthreads();
    return *s_go != 0;
}

// Workgroups whose next columns are this close to column k poll q_k's data
// themselves; the others wait for its flag (fewer loads on the lines being
// written)
constexpr int PIPE_EAGER = 2;

template <class R>
__global__ __launch_bounds__(TEAM) void k_mgs_pipe(MgsArgs a, int *sing, int *arrived, int *flags, long spin_limit, int qslots) {
    constexpr int W = 2 * limbs<R>::P;
    extern __shared__ double lds[];  // own columns [c][W][N] (planar), then qslots staging columns
    __shared__ cx<R> s_part[2 * CSLOT];
    __shared__ R s_rpart[2 * (TEAM / 64)];
    __shared__ int s_go;
    TeamSums<R> ts(s_part, s_rpart);
    const int b = blockIdx.y;
    if (!problem_live(a, b)) return;
    const int G = gridDim.x, w = blockIdx.x, n = a.n, N = a.N, t = threadIdx.x;
    if (w > n) return;
    const int mine = (n - w) / G + 1;  // columns w, w + G, ...
    const size_t cst = (size_t)N * W;
    double *qs0 = lds + (size_t)mine * cst;  // q_k received, in slot k mod qslots
    int *stop = sing + b;
    int *flg = flags + (size_t)b * (n + 1);
    // own columns into LDS; their places in A (columns j < n, where q_j
    // will be published) marked empty
    for (int c = 0; c < mine; ++c) {
        double *src = col_ptr(a, b, w + c * G);
        for (size_t e = t; e < cst; e += TEAM) lds[(size_t)c * cst + (e % W) * N + e / W] = src[e];
        if (w + c * G < n) {
            __syncthreads();  // the column is read whole before it is marked
            for (size_t e = t; e < cst; e += TEAM) st_device(src + e, __longlong_as_double(PIPE_EMPTY));
        }
    }
    // every workgroup of the problem has marked its columns before any
    // reads one: each wave's stores complete (an agent-scope release), then
    // the workgroup's arrival is counted and all G awaited (bounded)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (t == 0) {
        int *cnt = arrived + b;
        __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int go = 1;
        long spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < G) {
            if (++spins > spin_limit) {
                __hip_atomic_store(stop, PIPE_TIMEOUT, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                go = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        s_go = go;
    }
    __syncthreads();
    if (!s_go) return;
    auto own = [&](int c) { return planar(lds + (size_t)c * cst, N); };
    // own column j (slot c), fully projected: r_jj, 1/r_jj and q_j, written
    // to LDS and to its place in A (which publishes it to the polling
    // workgroups), then, once every wave's stores have completed (an
    // agent-scope release; a workgroup barrier alone does not wait for
    // global stores), its flag.  False: singular.
    auto publish = [&](int c, const R *part) -> bool {
        const int j = w + c * G;
        const Col aj = own(c);
        R iv;
        const R s2 = part ? team_rsum(*part, t, ts.r, ts.pr) : col_norm2<R>(aj, N, t, ts);
        if (!col_pivot<R>(a, b, j, s2, t, &iv)) {
            if (t == 0) __hip_atomic_store(stop, PIPE_SINGULAR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        col_scale<R>(aj, iv, N, t, col_ptr(a, b, j));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (t == 0) __hip_atomic_store(flg + j, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return true;
    };
    bool live = true;
    if (w == 0 && n > 0) live = publish(0, nullptr);
    // q_m for m <= k: in its owner's LDS slot, or received into staging slot
    // m mod qslots
    auto qcol = [&](int m) {
        return m % G == w ? own(m / G) : planar(qs0 + (size_t)(m % qslots) * cst, N);
    };
    auto rstore = [&](int j, int k, const cx<R> &r) {
        if (t == 0) cstore(a.R + (size_t)b * a.R_pstride + ((size_t)j * n + k) * W, r);
    };
    // q_k applied to own column slot c
    auto apply1 = [&](const Col &qk, int k, int c) {
        const Col aj = own(c);
        const cx<R> r = col_dot<R>(qk, aj, N, t, ts);
        rstore(w + c * G, k, r);
        col_axpy<R>(qk, aj, r, N, t);
    };
    // q_k applied to own columns from slot c on, two at a time
    auto apply_from = [&](const Col &qk, int k, int c) {
        for (; c + 1 < mine; c += 2) {
            cx<R> r0, r1;
            col_update2<R>(qk, own(c), own(c + 1), N, t, ts, r0, r1);
            rstore(w + c * G, k, r0);
            rstore(w + (c + 1) * G, k, r1);
        }
        if (c < mine) apply1(qk, k, c);
    };
    // The lead is this workgroup's first column beyond k that is not the
    // right-hand side.  While it is k+2 (with two staging slots), q_k goes
    // to the lead alone and the other columns wait; once the lead is k+1 it
    // takes q_k and is published first, then the other columns take every q
    // they still lack, in order.  So the lead is ready for q_{k+1} as soon
    // as it comes; every column still takes q_0, q_1, ... in order.
    int tp = 0;  // columns other than the lead have q_0 .. q_{tp-1}
    for (int k = 0; k < n && live; ++k) {
        const int next = k < w ? w : w + ((k - w) / G + 1) * G;  // first own column > k
        if (k % G != w) {
            // q_k is needed only while this workgroup has a column beyond k
            if (next > n) break;
            // q_k into its staging slot, each lane its own rows (read back
            // only by the same lane); the workgroup goes on only if every
            // lane got its rows
            bool ok = true;
            if (next - k > PIPE_EAGER) ok = pipe_wait(flg + k, stop, spin_limit, &s_go);
            if (ok) ok = pipe_fetch<R>(col_ptr(a, b, k), qs0 + (size_t)(k % qslots) * cst, N, t, stop, spin_limit);
            if (__syncthreads_or(!ok)) {
                live = false;
                break;
            }
        }
        const Col qk = qcol(k);
        const int c = k < w ? 0 : (k - w) / G + 1;  // slot of column next
        if (c >= mine) continue;
        if (next == k + 1 && next < n) {
            // the lead: its update forms its squared norm on the way
            const Col aj = own(c);
            const cx<R> r = col_dot<R>(qk, aj, N, t, ts);
            rstore(next, k, r);
            const R part = col_axpy_norm2<R>(qk, aj, r, N, t);
            live = publish(c, &part);
            for (int m = tp; m <= k && live; ++m) apply_from(qcol(m), m, c + 1);
            tp = k + 1;
        } else if (qslots > 1 && next == k + 2 && next < n) {
            apply1(qk, k, c);
        } else {
            apply_from(qk, k, c);
            tp = k + 1;
        }
    }
    // the projected right-hand side (column n) goes back to its place
    if (live && n % G == w) {
        const Col src = own(n / G);
        double *dst = col_ptr(a, b, n);
        for (int i = t; i < N; i += TEAM) cstore(dst + (size_t)i * W, col_ld<R>(src, i));
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

// Back substitution of mgs_backsub with y in LDS (ys: [ROWS BT][2P]
// doubles) and the rows of R fetched BS_AHEAD steps ahead into registers,
// for n <= ROWS * BT: lane t holds rows t, t + BT, ... of y and forms dx_k
// when it holds row k, which it hands to the others through one of two LDS
// slots (one barrier per step, ordering LDS only: a slot is written again
// two steps later, after the barrier of the step in between).  A step has
// no branch around its loads and updates (rows at or beyond k keep their
// value by a select, loads of rows not needed read r_k0), so that the
// fetches of the steps ahead stay in flight.  The same operations in the
// same order as mgs_backsub, so the same bits; dx written to global memory
// at the end.
constexpr int BS_AHEAD = 4;

template <class R, int ROWS>
HCN_DEV void mgs_backsub_lds(const MgsProblem &p, double *ys) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    __shared__ cx<R> s_x[2];
    const int t = threadIdx.x;
    const int n = p.n;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int i = t + r * BT;
        const cx<R> y = i < n ? cload<R>(p.R + ((size_t)n * n + i) * W) : czero<R>();
        cstore(ys + (size_t)i * W, y);
    }
    // what step k reads from global memory, fetched ahead: r_ki for the
    // lane's rows i < k (other rows read r_k0, unused) and 1/r_kk
    struct Ahead {
        cx<R> rk[ROWS];
        R iv;
    };
    auto fetch = [&](int k, Ahead &f) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int i = t + r * BT;
            f.rk[r] = cload<R>(p.R + ((size_t)k * n + (i < k ? i : 0)) * W);
        }
        rload(p.inv + (size_t)k * P, f.iv);
    };
    // one step: dx_k by its owner, then y_i -= r_ki dx_k for i < k
    auto step = [&](int k, const Ahead &f) {
        if (k % BT == t) {
            const cx<R> x = cscale(f.iv, cload<R>(ys + (size_t)k * W));
            cstore(ys + (size_t)k * W, x);
            s_x[k & 1] = x;
        }
        lds_barrier();  // the fetches of the steps ahead stay in flight
        const cx<R> xk = s_x[k & 1];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const int i = t + r * BT;
            double *q = ys + (size_t)i * W;
            const cx<R> y = cload<R>(q);
            const cx<R> u = csub(y, cmul(f.rk[r], xk));
            cstore(q, i < k ? u : y);
        }
    };
    // buffer u serves the steps k with (n - 1 - k) % BS_AHEAD == u
    Ahead fb[BS_AHEAD];
#pragma unroll
    for (int u = 0; u < BS_AHEAD; ++u) fetch(n - 1 - u >= 0 ? n - 1 - u : 0, fb[u]);
    int k0 = n - 1;
    for (; k0 >= BS_AHEAD - 1; k0 -= BS_AHEAD) {
#pragma unroll
        for (int u = 0; u < BS_AHEAD; ++u) {
            const int k = k0 - u;
            step(k, fb[u]);
            fetch(k - BS_AHEAD >= 0 ? k - BS_AHEAD : 0, fb[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < BS_AHEAD - 1; ++u)
        if (k0 - u >= 0) step(k0 - u, fb[u]);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int i = t + r * BT;
        if (i < n) cstore(p.dx + (size_t)i * W, cload<R>(ys + (size_t)i * W));
    }
    __syncthreads();
}

// rows per lane of the LDS back substitution for n unknowns (0: the plain
// one), and its dynamic LDS: y padded to ROWS * BT rows, within the 64 KB a
// launch gets without an attribute (with the kernel's own slots)
template <class R>
HCN_DEV __host__ inline int backsub_rows(int n) {
    const int rows = (n + BT - 1) / BT;
    const size_t b = (size_t)rows * BT * 2 * limbs<R>::P * sizeof(double);
    return rows >= 1 && rows <= 4 && b <= 60 * 1024 ? rows : 0;
}
template <class R>
HCN_DEV __host__ inline size_t backsub_lds_bytes(int n) {
    return (size_t)backsub_rows<R>(n) * BT * 2 * limbs<R>::P * sizeof(double);
}

template <class R>
__global__ __launch_bounds__(BT) void k_mgs_finish(MgsArgs a, const int *sing) {
    extern __shared__ double ys[];  // y of the back substitution, when it fits
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
    if (sing[b] != 0) {
        mgs_singular<R>(p);
        return;
    }
    switch (backsub_rows<R>(p.n)) {
        case 1: mgs_backsub_lds<R, 1>(p, ys); break;
        case 2: mgs_backsub_lds<R, 2>(p, ys); break;
        case 3: mgs_backsub_lds<R, 3>(p, ys); break;
        case 4: mgs_backsub_lds<R, 4>(p, ys); break;
        default: mgs_backsub<R>(p); break;
    }
    mgs_after_backsub<R>(p);
}

__global__ void k_zero_int(int *p, int count) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < count) p[q] = 0;
}

// workgroups of the pipelined variant for one problem (0: it does not fit):
// the columns dealt round G workgroups, each holding its columns in LDS,
// all B x G of them resident at once.  G starts at one workgroup per CU per
// problem (several problems then share CUs, their chains interleaving) and
// halves until the B x G workgroups fit the device's residency.
constexpr size_t PIPE_MAX_DYN_LDS = 159 * 1024;

template <class R>
static int pipe_groups(const MgsArgs &a, size_t *lds_out, int *qslots_out) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
    }
    const size_t cst = (size_t)a.N * 2 * limbs<R>::P * sizeof(double);
    for (int G = std::min(cus, a.n + 1); G >= 1; G /= 2) {
        const int mine = a.n / G + 1;
        // two staging columns where they fit (the lead column goes first),
        // else one
        for (int qslots = 2; qslots >= 1; --qslots) {
            const size_t lds = (size_t)(mine + qslots) * cst;
            // the LDS of a CU (160 KB) holds the dynamic part and the
            // kernel's own few hundred bytes of reduction slots
            if (lds > PIPE_MAX_DYN_LDS) continue;
            if (hipFuncSetAttribute((const void *)k_mgs_pipe<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds) != hipSuccess) {
                (void)hipGetLastError();
                return 0;
            }
            int per_cu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mgs_pipe<R>, TEAM, lds) !=
                hipSuccess)
                return 0;
            if ((long)per_cu * cus >= (long)G * a.B) {
                *lds_out = lds;
                *qslots_out = qslots;
                return G;
            }
        }
    }
    return 0;
}

// bounded waits: seconds of polling before a wait gives up
static long g_wait_limit = 1L << 22;

void set_mgs_wait_limit(long long polls) { g_wait_limit = (long)polls; }

template <class R>
static int launch_big_t(const MgsArgs &a, int variant, int *ints, hipStream_t s) {
    // ints: sing[B], then (after 2B + 1) the pipelined variant's column
    // flags [B][n + 1], then its arrival counters [B] in the words B + 1 ..
    // 2B (free in that variant)
    int *sing = ints;
    int *arrived = ints + a.B + 1;
    int *flags = ints + 2 * a.B + 1;
    size_t pipe_lds = 0;
    int qslots = 1;
    const int G = variant == 5 ? pipe_groups<R>(a, &pipe_lds, &qslots) : 0;
    if (variant == 5 && G == 0) variant = 2;
    const long nz = variant == 5 ? 2L * a.B + 1 + (long)a.B * (a.n + 1) : a.B;
    hipLaunchKernelGGL(k_zero_int, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, s, ints, (int)nz);
    if (a.mode == MGS_NEWTON_FIG2)
        hipLaunchKernelGGL(k_fig2_pre, dim3((a.B + 255) / 256), dim3(256), 0, s, a);
    {
        ProfScope prof("mgs", s);
        if (variant == 5) {
            MgsArgs av = a;
            long spin = g_wait_limit;
            void *args[] = {&av, &sing, &arrived, &flags, &spin, &qslots};
            const hipError_t e = hipLaunchCooperativeKernel((const void *)k_mgs_pipe<R>, dim3(G, a.B),
                                                            dim3(TEAM), args, (unsigned)pipe_lds, s);
            // a launch the device cannot take whole goes right-looking
            if (e != hipSuccess) {
                (void)hipGetLastError();
                variant = 2;
            }
        }
        if (variant == 4) {
            launch_tiled<R>(a, sing, s);
        } else if (variant == 2) {
            hipLaunchKernelGGL(k_mgs_rl<R>, dim3(1, a.B), dim3(BT), 0, s, a, -1, sing);
            for (int k = 0; k < a.n; ++k)
                hipLaunchKernelGGL(k_mgs_rl<R>, dim3(a.n - k, a.B), dim3(BT), 0, s, a, k, sing);
        }
        hipLaunchKernelGGL(k_mgs_finish<R>, dim3(a.B), dim3(BT), backsub_lds_bytes<R>(a.n), s, a, sing);
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
