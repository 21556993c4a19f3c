// mgs_common.hpp -- modified Gram-Schmidt on the augmented matrix [A | b] in
// one workgroup per problem (Section 1; Fig. 2, GPU_Modified_Gram_Schmidt),
// the Fig. 2 tests around a solve, and the epilogue every MGS variant shares
// (column-oriented back substitution dx_k = y_k / r_kk, y_i -= r_ik dx_k for
// i < k; the Newton update x += dx with its norm and the Fig. 2 tests that
// follow it).
//
// mgs_wg: right-looking.  At step k each lane group owns trailing columns
// j > k (the right-hand side last), forms r_kj = q_k^H a_j over its rows and
// a butterfly across its GROUP lanes, and updates a_j -= r_kj q_k on its
// rows; the group that updates column k+1 then forms its norm, r_{k+1,k+1},
// 1/r_{k+1,k+1} and q_{k+1} on its rows right away (look-ahead), so one
// barrier per column separates the steps.  Butterflies add the lower lane's
// value first, so every lane of a group holds bitwise the same sum.  When
// [A | b] fits in LDS the workgroup copies it there first; the arithmetic is
// the same either way.
#pragma once

#include "internal.hpp"
#include "mp.hpp"

namespace hcn {

constexpr int MGS_THREADS = 256;

// A workgroup barrier that orders LDS accesses only: global loads and
// stores still in flight stay in flight (a plain __syncthreads waits for
// every one of them first)
HCN_DEV void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// one problem with every pointer resolved
struct MgsProblem {
    int N, n, mode, lds;
    double *A;          // column j at A + j*A_cstride (j < n)
    long A_cstride;
    double *bcol;       // column n
    double *R;          // [n+1][n][2P]
    double *inv;        // [n][P]
    double *dx;         // [n][2P]
    int32_t *status;    // or NULL
    double *x;          // Newton modes: [n][2P]
    const double *norm_part;
    int nparts;
    double *norms;      // [2] or NULL
    PathState *st;      // Fig. 2 modes
};

HCN_DEV MgsProblem problem_of(const MgsArgs &a, int b) {
    MgsProblem p;
    p.N = a.N;
    p.n = a.n;
    p.mode = a.mode;
    p.lds = 0;
    p.A = a.A + (size_t)b * a.A_pstride;
    p.A_cstride = a.A_cstride;
    p.bcol = a.bcol ? a.bcol + (size_t)b * a.b_pstride : p.A + (size_t)a.n * a.A_cstride;
    p.R = a.R + (size_t)b * a.R_pstride;
    p.inv = a.inv + (size_t)b * a.inv_pstride;
    p.dx = a.dx + (size_t)b * a.dx_pstride;
    p.status = a.status ? a.status + b : nullptr;
    p.x = a.x ? a.x + (size_t)b * a.x_pstride : nullptr;
    p.norm_part = a.norm_part ? a.norm_part + (size_t)b * a.nparts : nullptr;
    p.nparts = a.nparts;
    p.norms = a.norms ? a.norms + 2 * (size_t)b : nullptr;
    p.st = a.st ? a.st + b : nullptr;
    return p;
}

HCN_DEV double residual_norm(const MgsProblem &p) {
    double res = 0.0;
    for (int q = 0; q < p.nparts; ++q) res = nanmax(res, p.norm_part[q]);
    return res;
}

// residual_norm by every lane of the workgroup (MGS_THREADS lanes, all of
// which call it), the same value on each: the maximum is exact and a NaN
// anywhere gives NaN, so the grouping does not matter
HCN_DEV double residual_norm_wg(const MgsProblem &p) {
    __shared__ double s_rn[MGS_THREADS / 64];
    double m = 0.0;
    for (int q = threadIdx.x; q < p.nparts; q += MGS_THREADS) m = nanmax(m, p.norm_part[q]);
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) s_rn[threadIdx.x >> 6] = m;
    __syncthreads();
    double r = s_rn[0];
    for (int w = 1; w < MGS_THREADS / 64; ++w) r = nanmax(r, s_rn[w]);
    return r;
}

// Fig. 2 before the solve: fail if the residual grew beyond the previous one
// (initially max_eq_val), succeed if it is below the tolerance, stop on NaN.
// Called by one lane; returns 1 when this problem needs no solve.
HCN_DEV int fig2_decide(const MgsProblem &p) {
    PathState &st = *p.st;
    if (!st.c_active) return 1;
    const double res = residual_norm(p);
    st.res = res;
    st.c_iter += 1;
    st.evals += 1;
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

// Fig. 2 after the update
HCN_DEV void fig2_after_update(PathState &st, double dxn) {
    st.dxn = dxn;
    st.solves += 1;
    if (dxn != dxn) {
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

// The epilogue's two parts, after a solve that found no singular column.
// Back substitution R dx = y in place in dx (it starts as y = column n of
// R): for k = n-1 down to 0, dx_k = y_k / r_kk (times the stored 1/r_kk),
// then y_i -= r_ik dx_k for every i < k.
template <class R>
HCN_DEV void mgs_backsub(const MgsProblem &p) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    const int tid = threadIdx.x;
    const int n = p.n;
    for (int i = tid; i < n; i += MGS_THREADS)
        cstore(p.dx + (size_t)i * W, cload<R>(p.R + ((size_t)n * n + i) * W));
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
        if (tid == 0) {
            R iv;
            rload(p.inv + (size_t)k * P, iv);
            cstore(p.dx + (size_t)k * W, cscale(iv, cload<R>(p.dx + (size_t)k * W)));
        }
        __syncthreads();
        const cx<R> xk = cload<R>(p.dx + (size_t)k * W);
        for (int i = tid; i < k; i += MGS_THREADS) {
            double *q = p.dx + (size_t)i * W;
            cstore(q, csub(cload<R>(q), cmul(cload<R>(p.R + ((size_t)k * n + i) * W), xk)));
        }
        __syncthreads();
    }
}

// Then the status of a plain solve, or for Newton the update norm, the NaN
// check, x += dx and the Fig. 2 bookkeeping (dx complete in global memory,
// the workgroup synchronised).
template <class R>
HCN_DEV void mgs_after_backsub(const MgsProblem &p) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    const int tid = threadIdx.x;
    const int n = p.n;
    if (p.mode == MGS_SOLVE || p.mode == MGS_MIXED_SOLVE) {
        if (tid == 0 && p.status) *p.status = HCN_OK;
        return;
    }
    __shared__ double s_red[MGS_THREADS / 64];
    double m = 0.0;
    for (int i = tid; i < n; i += MGS_THREADS) m = nanmax(m, clead_abs(cload<R>(p.dx + (size_t)i * W)));
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
    if ((tid & 63) == 0) s_red[tid >> 6] = m;
    __syncthreads();
    double dxn = s_red[0];
    for (int w = 1; w < MGS_THREADS / 64; ++w) dxn = nanmax(dxn, s_red[w]);
    const bool isnan_dx = dxn != dxn;
    if (!isnan_dx) {
        for (int i = tid; i < n; i += MGS_THREADS) {
            double *q = p.x + (size_t)i * W;
            cstore(q, cadd(cload<R>(q), cload<R>(p.dx + (size_t)i * W)));
        }
    }
    const double res = p.mode == MGS_NEWTON_STEP && p.norms ? residual_norm_wg(p) : 0.0;
    if (tid == 0) {
        if (p.mode == MGS_NEWTON_STEP) {
            if (p.norms) {
                p.norms[0] = res;
                p.norms[1] = dxn;
            }
            if (p.status) *p.status = isnan_dx ? HCN_NAN : HCN_OK;
        } else {
            fig2_after_update(*p.st, dxn);
        }
    }
}

// a singular column: the problem's status, and for Newton its norms
template <class R>
HCN_DEV void mgs_singular(const MgsProblem &p) {
    if (threadIdx.x == 0) {
        if (p.status) *p.status = HCN_ESINGULAR;
        if (p.mode == MGS_NEWTON_FIG2 || p.mode == MGS_MIXED_SOLVE) {
            p.st->c_status = HCN_ESINGULAR;
            p.st->c_active = 0;
        }
        if (p.mode == MGS_NEWTON_STEP && p.norms) {
            p.norms[0] = residual_norm(p);
            p.norms[1] = __builtin_nan("");
        }
    }
}

template <class R>
HCN_DEV void mgs_epilogue(const MgsProblem &p, bool singular) {
    if (singular) {
        mgs_singular<R>(p);
        return;
    }
    mgs_backsub<R>(p);
    mgs_after_backsub<R>(p);
}

// The partner's value at butterfly level M (lanes l and l ^ M).  Inside a
// row of 16 lanes by DPP: quad_perm for M = 1, 2; for M = 4 and 8 the
// half-row and row mirrors (l <-> 7 - l, l <-> 15 - l), which reach a lane
// of the same quad / half-row as l ^ M and so the same value once the
// earlier levels have made every quad / half-row uniform.  Beyond a row by
// ds_bpermute.
template <int M>
HCN_DEV double xshfl(double v) {
    if constexpr (M <= 8) {
        constexpr int ctrl = M == 1 ? 0xB1 : M == 2 ? 0x4E : M == 4 ? 0x141 : 0x140;
        const unsigned long long u = (unsigned long long)__double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, ctrl, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), ctrl, 0xF, 0xF, false);
        return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    } else {
        return __shfl_xor(v, M);
    }
}
template <int M>
HCN_DEV dd xshfl(const dd &v) {
    return dd{xshfl<M>(v.hi), xshfl<M>(v.lo)};
}
template <int M>
HCN_DEV qd xshfl(const qd &v) {
    return qd{xshfl<M>(v.c0), xshfl<M>(v.c1), xshfl<M>(v.c2), xshfl<M>(v.c3)};
}

// sum over the GRP consecutive lanes of a group (levels M, 2M, ... < GRP),
// lower lane first in QD, so every lane of the group holds the same bits
// (in FP64 and DD the order does not matter: the error-free sums of an
// addition give the same pair whichever operand comes first)
template <class R, int GRP, int M = 1>
HCN_DEV R group_sum(R v, int lane) {
    if constexpr (M >= GRP) {
        return v;
    } else {
        const R o = xshfl<M>(v);
        if constexpr (limbs<R>::P == 4)
            v = (lane & M) ? add(o, v) : add(v, o);
        else
            v = add(v, o);  // add(v, o) and add(o, v) have the same bits in FP64 and DD
        return group_sum<R, GRP, 2 * M>(v, lane);
    }
}

template <class R, int GRP, int M = 1>
HCN_DEV cx<R> group_csum(cx<R> v, int lane) {
    if constexpr (M >= GRP) {
        return v;
    } else {
        const cx<R> o{xshfl<M>(v.re), xshfl<M>(v.im)};
        if constexpr (limbs<R>::P == 4)
            v = (lane & M) ? cadd(o, v) : cadd(v, o);
        else
            v = cadd(v, o);
        return group_csum<R, GRP, 2 * M>(v, lane);
    }
}

// bytes of LDS that hold [A | b] of one problem
HCN_DEV __host__ inline size_t mgs_lds_bytes(int N, int n, int P) {
    return (size_t)(n + 1) * N * 2 * P * sizeof(double);
}

// STORE: where [A | b] lives, fixed at compile time (0 global memory, 1 LDS:
// the loads and stores are then LDS or global instructions) or -1, p.lds at
// run time (generic addressing)
template <class R, int GRP, int STORE = -1>
HCN_DEV void mgs_wg(const MgsProblem &p) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    constexpr int NGRP = MGS_THREADS / GRP;
    extern __shared__ double lds_cols[];
    const bool in_lds = STORE < 0 ? p.lds != 0 : STORE == 1;
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    const int g = tid / GRP;
    const int lane = tid % GRP;
    const int N = p.N, n = p.n;

    // Fig. 2 tests before the solve (residual norm against the previous one)
    if (p.mode == MGS_NEWTON_FIG2 || p.mode == MGS_MIXED_SOLVE) {
        if (tid == 0) s_flag = p.mode == MGS_NEWTON_FIG2 ? fig2_decide(p) : !p.st->c_active;
        __syncthreads();
        if (s_flag) return;
    }
    const size_t cst = (size_t)N * W;
    if (in_lds) {
        for (size_t q = tid; q < (size_t)(n + 1) * cst; q += MGS_THREADS) {
            const int j = (int)(q / cst);
            const size_t off = q - (size_t)j * cst;
            const double *src = j < n ? p.A + (size_t)j * p.A_cstride : p.bcol;
            lds_cols[q] = src[off];
        }
    }
    auto col = [&](int j) -> double * {
        if constexpr (STORE == 1) return lds_cols + (size_t)j * cst;
        if constexpr (STORE == 0) return j < n ? p.A + (size_t)j * p.A_cstride : p.bcol;
        if (in_lds) return lds_cols + (size_t)j * cst;
        return j < n ? p.A + (size_t)j * p.A_cstride : p.bcol;
    };
    // ||a_k||^2 over the rows of group 0, lower lane first
    auto group0_norm2 = [&](const double *ak) -> R {
        R s = rmake<R>(0.0);
        bool first = true;
        for (int i = lane; i < N; i += GRP) {
            const R v = cnorm2(cload<R>(ak + (size_t)i * W));
            s = first ? v : add(s, v);
            first = false;
        }
        return group_sum<R, GRP>(s, lane);
    };
    // column j, just updated by the calling group, with n2 = ||a_j||^2:
    // r_jj = sqrt(n2), 1/r_jj and q_j = a_j / r_jj on the group's rows;
    // false when singular
    auto normalise = [&](int j, double *aj, const R &n2) -> bool {
        const R rkk = sqrt(n2);
        if (!(lead(rkk) > 0.0) || !rfinite(rkk)) return false;
        const R iv = div(rmake<R>(1.0), rkk);
        if (lane == 0) {
            rstore(p.inv + (size_t)j * P, iv);
            const cx<R> rc{rkk, rmake<R>(0.0)};
            cstore(p.R + ((size_t)j * n + j) * W, rc);
        }
        for (int i = lane; i < N; i += GRP) {
            double *q = aj + (size_t)i * W;
            cstore(q, cscale(iv, cload<R>(q)));
        }
        return true;
    };
    // singular column seen, by the parity of the column (written while the
    // previous step runs, read after its barrier: every thread decides alike)
    __shared__ int s_bad[2];
    if (tid < 2) s_bad[tid] = 0;
    __syncthreads();
    if (g == 0 && !normalise(0, col(0), group0_norm2(col(0))) && lane == 0) s_bad[0] = 1;
    __syncthreads();

    bool singular = false;
    for (int k = 0; k < n; ++k) {
        if (s_bad[k & 1]) {
            singular = true;
            break;
        }
        double *ak = col(k);
        for (int j = k + 1 + g; j <= n; j += NGRP) {
            double *aj = col(j);
            cx<R> r = czero<R>();
            bool first = true;
            for (int i = lane; i < N; i += GRP) {
                const cx<R> v = cmul_conj(cload<R>(ak + (size_t)i * W), cload<R>(aj + (size_t)i * W));
                r = first ? v : cadd(r, v);
                first = false;
            }
            r = group_csum<R, GRP>(r, lane);
            if (lane == 0) cstore(p.R + ((size_t)j * n + k) * W, r);
            // look ahead: the group of column k+1 normalises it right away,
            // in DD and FP64 with its squared norm formed from the updated
            // values as they are stored (the rows and order of group0_norm2,
            // so the same bits); QD reads the column again, as the extra
            // accumulator would cost it registers
            constexpr bool fused = P != 4;
            const bool next = j == k + 1 && j < n;
            R n2 = rmake<R>(0.0);
            bool first_n2 = true;
            for (int i = lane; i < N; i += GRP) {
                double *q = aj + (size_t)i * W;
                const cx<R> u = csub(cload<R>(q), cmul(r, cload<R>(ak + (size_t)i * W)));
                cstore(q, u);
                if (fused && next) {
                    const R v = cnorm2(u);
                    n2 = first_n2 ? v : add(n2, v);
                    first_n2 = false;
                }
            }
            if (next && !normalise(j, aj, fused ? group_sum<R, GRP>(n2, lane) : group0_norm2(aj)) &&
                lane == 0)
                s_bad[(k + 1) & 1] = 1;
        }
        __syncthreads();
    }
    // a plain solve returns Q and the projected right-hand side in place
    if (in_lds && p.mode == MGS_SOLVE && !singular) {
        for (size_t q = tid; q < (size_t)(n + 1) * cst; q += MGS_THREADS) {
            const int j = (int)(q / cst);
            const size_t off = q - (size_t)j * cst;
            double *dst = j < n ? p.A + (size_t)j * p.A_cstride : p.bcol;
            dst[off] = lds_cols[q];
        }
    }
    mgs_epilogue<R>(p, singular);
}

// Register-resident form of mgs_wg, for problems with N <= GRP * RPL rows and
// n + 1 <= NGRP * CPG columns.  Column j belongs to lane group j % NGRP (its
// slot j / NGRP); lane l of the group holds rows l, l + GRP, ... of each of
// its columns in registers for the whole factorisation.  At step k every
// group projects q_k (read from LDS) out of its columns j > k; the owner of
// column k + 1 then forms its norm, r, 1/r and q_{k+1}, which it writes to the
// other of two LDS buffers; one barrier per column.  Each element sees the
// same operations as in mgs_wg and every reduction runs over the same rows in
// the same order with the same butterfly, so the results are bitwise those of
// mgs_wg; [A | b] is read once and only R (and Q for a plain solve) written.
template <class R, int GRP, int RPL, int CPG>
HCN_DEV void mgs_reg(const MgsProblem &p) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    constexpr int NGRP = MGS_THREADS / GRP;
    __shared__ double s_q[2][GRP * RPL * W];
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    const int g = tid / GRP;
    const int lane = tid % GRP;
    const int N = p.N, n = p.n;

    if (p.mode == MGS_NEWTON_FIG2 || p.mode == MGS_MIXED_SOLVE) {
        if (tid == 0) s_flag = p.mode == MGS_NEWTON_FIG2 ? fig2_decide(p) : !p.st->c_active;
        __syncthreads();
        if (s_flag) return;
    }
    auto col = [&](int j) -> double * { return j < n ? p.A + (size_t)j * p.A_cstride : p.bcol; };
    cx<R> v[CPG][RPL];
#pragma unroll
    for (int c = 0; c < CPG; ++c) {
        const int j = g + c * NGRP;
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + r * GRP;
            v[c][r] = (j <= n && i < N) ? cload<R>(col(j) + (size_t)i * W) : czero<R>();
        }
    }
    // ||column||^2 over this lane's rows, then the group butterfly
    auto norm2 = [&](const cx<R>(&u)[RPL]) -> R {
        R t = rmake<R>(0.0);
#pragma unroll
        for (int r = 0; r < RPL; ++r)
            if (lane + r * GRP < N) t = r == 0 ? cnorm2(u[r]) : add(t, cnorm2(u[r]));
        return group_sum<R, GRP>(t, lane);
    };
    // column j in slot c of the calling group, just updated: r_jj, 1/r_jj
    // and q_j into the registers and into the LDS buffer q; false when singular
    auto normalise = [&](int j, cx<R>(&u)[RPL], double *q) -> bool {
        const R rkk = sqrt(norm2(u));
        if (!(lead(rkk) > 0.0) || !rfinite(rkk)) return false;
        const R iv = div(rmake<R>(1.0), rkk);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            u[r] = cscale(iv, u[r]);
            cstore(q + (size_t)(lane + r * GRP) * W, u[r]);
        }
        if (lane == 0) {
            rstore(p.inv + (size_t)j * P, iv);
            const cx<R> rc{rkk, rmake<R>(0.0)};
            cstore(p.R + ((size_t)j * n + j) * W, rc);
        }
        return true;
    };
    // singular column seen, by the parity of the column (written while the
    // previous step runs, read after its barrier: every thread decides alike)
    __shared__ int s_bad[2];
    if (tid < 2) s_bad[tid] = 0;
    __syncthreads();
    if (g == 0 && !normalise(0, v[0], s_q[0]) && lane == 0) s_bad[0] = 1;
    __syncthreads();

    bool singular = false;
    for (int k = 0; k < n; ++k) {
        if (s_bad[k & 1]) {
            singular = true;
            break;
        }
        const double *q = s_q[k & 1];
#pragma unroll
        for (int c = 0; c < CPG; ++c) {
            const int j = g + c * NGRP;
            if (j <= k || j > n) continue;
            cx<R> acc = czero<R>();
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                if (lane + r * GRP < N) {
                    const cx<R> t = cmul_conj(cload<R>(q + (size_t)(lane + r * GRP) * W), v[c][r]);
                    acc = r == 0 ? t : cadd(acc, t);
                }
            }
            acc = group_csum<R, GRP>(acc, lane);
            if (lane == 0) cstore(p.R + ((size_t)j * n + k) * W, acc);
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                if (lane + r * GRP < N)
                    v[c][r] = csub(v[c][r], cmul(acc, cload<R>(q + (size_t)(lane + r * GRP) * W)));
            // look ahead: the owner of column k+1 normalises it into the
            // other LDS buffer right away
            if (j == k + 1 && j < n && !normalise(j, v[c], s_q[(k + 1) & 1]) && lane == 0)
                s_bad[(k + 1) & 1] = 1;
        }
        __syncthreads();
    }
    // a plain solve returns Q and the projected right-hand side in place
    if (p.mode == MGS_SOLVE && !singular) {
#pragma unroll
        for (int c = 0; c < CPG; ++c) {
            const int j = g + c * NGRP;
            if (j > n) continue;
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + r * GRP;
                if (i < N) cstore(col(j) + (size_t)i * W, v[c][r]);
            }
        }
    }
    __syncthreads();
    mgs_epilogue<R>(p, singular);
}

// Left-looking by panels, one workgroup per problem (Section 1: left-looking
// tiles cut the memory traffic of the right-looking form): the workgroup
// takes the columns NGRP at a time, lane group g holding column j0 + g of the
// panel in registers (lane l: rows l, l + GRP, ...).  The panel first
// receives the projections of every earlier column k < j0, in order, with
// q_k read from memory (final since its own panel); then the panel is
// factored as in mgs_reg (the owner of column k normalises it into LDS and
// memory, one barrier per column).  Every column sees the projections
// k = 0, 1, ... in the same order, over the same rows with the same
// butterflies, as in mgs_wg, so the results are bitwise those of mgs_wg;
// [A | b] is read once and each q column once per later panel, instead of
// the whole trailing matrix at every column step.
template <class R, int GRP, int RPL>
HCN_DEV void mgs_panel(const MgsProblem &p) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    constexpr int NGRP = MGS_THREADS / GRP;
    __shared__ double s_q[2][GRP * RPL * W];
    __shared__ int s_flag;
    __shared__ int s_bad[2];
    const int tid = threadIdx.x;
    const int g = tid / GRP;
    const int lane = tid % GRP;
    const int N = p.N, n = p.n;

    if (p.mode == MGS_NEWTON_FIG2 || p.mode == MGS_MIXED_SOLVE) {
        if (tid == 0) s_flag = p.mode == MGS_NEWTON_FIG2 ? fig2_decide(p) : !p.st->c_active;
        __syncthreads();
        if (s_flag) return;
    }
    auto col = [&](int j) -> double * { return j < n ? p.A + (size_t)j * p.A_cstride : p.bcol; };
    auto norm2 = [&](const cx<R>(&u)[RPL]) -> R {
        R t = rmake<R>(0.0);
#pragma unroll
        for (int r = 0; r < RPL; ++r)
            if (lane + r * GRP < N) t = r == 0 ? cnorm2(u[r]) : add(t, cnorm2(u[r]));
        return group_sum<R, GRP>(t, lane);
    };
    // q_k^H u over the lane's rows and the group butterfly, then u -= r q_k
    auto project = [&](const double *q, cx<R>(&u)[RPL], int j, int k) {
        cx<R> acc = czero<R>();
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            if (lane + r * GRP < N) {
                const cx<R> t = cmul_conj(cload<R>(q + (size_t)(lane + r * GRP) * W), u[r]);
                acc = r == 0 ? t : cadd(acc, t);
            }
        }
        acc = group_csum<R, GRP>(acc, lane);
        if (lane == 0) cstore(p.R + ((size_t)j * n + k) * W, acc);
#pragma unroll
        for (int r = 0; r < RPL; ++r)
            if (lane + r * GRP < N) u[r] = csub(u[r], cmul(acc, cload<R>(q + (size_t)(lane + r * GRP) * W)));
    };
    // column j of the calling group, fully projected: r_jj, 1/r_jj and q_j
    // into the registers, the LDS buffer q and memory; false when singular
    auto normalise = [&](int j, cx<R>(&u)[RPL], double *q) -> bool {
        const R rkk = sqrt(norm2(u));
        if (!(lead(rkk) > 0.0) || !rfinite(rkk)) return false;
        const R iv = div(rmake<R>(1.0), rkk);
        double *aj = col(j);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            u[r] = cscale(iv, u[r]);
            cstore(q + (size_t)(lane + r * GRP) * W, u[r]);
            if (lane + r * GRP < N) cstore(aj + (size_t)(lane + r * GRP) * W, u[r]);
        }
        if (lane == 0) {
            rstore(p.inv + (size_t)j * P, iv);
            const cx<R> rc{rkk, rmake<R>(0.0)};
            cstore(p.R + ((size_t)j * n + j) * W, rc);
        }
        return true;
    };
    if (tid < 2) s_bad[tid] = 0;
    __syncthreads();
    bool singular = false;
    for (int j0 = 0; j0 <= n && !singular; j0 += NGRP) {
        const int j = j0 + g;
        const bool own = j <= n;
        cx<R> v[RPL];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = lane + r * GRP;
            v[r] = (own && i < N) ? cload<R>(col(j) + (size_t)i * W) : czero<R>();
        }
        // the projections of the earlier panels' columns, in order
        if (own)
            for (int k = 0; k < j0; ++k) project(col(k), v, j, k);
        // the panel itself
        const int k1 = j0 + NGRP < n ? j0 + NGRP : n;
        if (own && j == j0 && j0 < n && !normalise(j, v, s_q[j0 & 1]) && lane == 0) s_bad[j0 & 1] = 1;
        __syncthreads();
        for (int k = j0; k < k1; ++k) {
            if (s_bad[k & 1]) {
                singular = true;
                break;
            }
            if (own && j > k) {
                project(s_q[k & 1], v, j, k);
                if (j == k + 1 && j < n && !normalise(j, v, s_q[(k + 1) & 1]) && lane == 0)
                    s_bad[(k + 1) & 1] = 1;
            }
            __syncthreads();
        }
        // a plain solve returns the projected right-hand side in place
        if (!singular && own && j == n && p.mode == MGS_SOLVE) {
#pragma unroll
            for (int r = 0; r < RPL; ++r)
                if (lane + r * GRP < N) cstore(col(n) + (size_t)(lane + r * GRP) * W, v[r]);
        }
    }
    __syncthreads();
    mgs_epilogue<R>(p, singular);
}

// rows per lane of mgs_panel (0 when a column does not fit the register
// budget of 16 rows per lane, and for QD, whose columns spill to the stack)
HCN_DEV __host__ inline int mgs_panel_rpl(int N, int P, int grp) {
    if (P == 4) return 0;
    const int need = (N + grp - 1) / grp;
    int r = 1;
    while (r < need) r <<= 1;
    return r <= 16 ? r : 0;
}

// rows per lane and columns per group of mgs_reg for a problem (0 when it
// does not fit the register budget: at most 8 complex numbers per lane in
// DD and FP64; in QD at most 4 and one column per group)
HCN_DEV __host__ inline void mgs_reg_shape(int N, int n, int P, int grp, int *rpl, int *cpg) {
    const int ngrp = MGS_THREADS / grp;
    auto up = [](int x) { return x <= 1 ? 1 : x <= 2 ? 2 : x <= 4 ? 4 : 8; };
    const int r = up((N + grp - 1) / grp), c = up((n + 1 + ngrp - 1) / ngrp);
    const int cap = P == 4 ? 4 : 8;
    if (r * c > cap || r > 4 || c > 4 || (P == 4 && c > 1)) {
        *rpl = *cpg = 0;
    } else {
        *rpl = r;
        *cpg = c;
    }
}

}  // namespace hcn
