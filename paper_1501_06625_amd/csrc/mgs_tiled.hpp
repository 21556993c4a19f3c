// mgs_tiled.hpp -- tiled modified Gram-Schmidt on one problem [A | b]
// (Section 1: right-looking, taken a panel of T columns at a time), shared by
// the single-system solver (mgs_big.hip) and the slot-table batch
// (batch.hip), where every launch covers many problems of different sizes.
//
// One wavefront per column: lane l holds rows l, l+64, ... of its column in
// registers (RPL rows per lane, zero past N), and every reduction is the
// lane's rows in ascending order followed by a 64-lane butterfly that adds
// the lower lane first, so all lanes of the wavefront hold the same bits.
//
// tiled_panel: the workgroup's wavefront w owns column k0 + w of the panel
// k0..k1-1 (wavefronts past k1 - k0 only keep the barriers).  For each k the
// owner of column k forms r_kk, 1/r_kk and q_k (every lane the same bits),
// writes q_k to LDS and to A; the owners of later panel columns form
// r_kj = q_k^H a_j from the LDS copy and update a_j -= r_kj q_k.
//
// tiled_trail: one wavefront applies the panel's projections k0..k1-1, in
// order, to one later column j (the right-hand side is column n), held in
// registers from load to store.
#pragma once

#include "internal.hpp"
#include "mgs_common.hpp"
#include "mp.hpp"

namespace hcn {

// wavefronts (columns) per panel workgroup: 16, or 8 where a column and the
// temporaries of its arithmetic would not fit the register budget of 1024
// lanes (DD and FP64 beyond four rows per lane, QD beyond one)
template <class R, int RPL>
constexpr int tiled_max_waves() {
    return (limbs<R>::P == 4 ? RPL == 1 : limbs<R>::P * RPL <= 8) ? 16 : 8;
}

// rows per lane for N rows in precision P, 0 when a column does not fit in
// registers (N > 512 for DD and FP64, N > 256 for QD)
HCN_DEV __host__ inline int tiled_rpl(int N, int P) {
    const int need = (N + 63) / 64;
    const int cap = P == 4 ? 4 : 8;
    int rpl = 1;
    while (rpl < need) rpl <<= 1;
    return rpl <= cap ? rpl : 0;
}

template <class R>
HCN_DEV cx<R> wave_csum(cx<R> v) {
    return group_csum<R, 64>(v, threadIdx.x & 63);
}

template <class R>
HCN_DEV R wave_rsum(R v) {
    return group_sum<R, 64>(v, threadIdx.x & 63);
}

template <class R, int RPL>
HCN_DEV void wcol_load(cx<R> (&v)[RPL], const double *col, int N, int lane) {
    constexpr int W = 2 * limbs<R>::P;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        v[r] = i < N ? cload<R>(col + (size_t)i * W) : czero<R>();
    }
}

template <class R, int RPL>
HCN_DEV void wcol_store(const cx<R> (&v)[RPL], double *col, int N, int lane) {
    constexpr int W = 2 * limbs<R>::P;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < N) cstore(col + (size_t)i * W, v[r]);
    }
}

// q^H v over the wavefront's column
template <class R, int RPL>
HCN_DEV cx<R> wcol_dot(const double *q, const cx<R> (&v)[RPL], int N, int lane) {
    constexpr int W = 2 * limbs<R>::P;
    cx<R> acc = czero<R>();
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < N) {
            const cx<R> t = cmul_conj(cload<R>(q + (size_t)i * W), v[r]);
            acc = r == 0 ? t : cadd(acc, t);
        }
    }
    return wave_csum(acc);
}

template <class R, int RPL>
HCN_DEV void wcol_axpy(const double *q, cx<R> (&v)[RPL], const cx<R> &rv, int N, int lane) {
    constexpr int W = 2 * limbs<R>::P;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i < N) v[r] = csub(v[r], cmul(rv, cload<R>(q + (size_t)i * W)));
    }
}

HCN_DEV double *tiled_col(const MgsProblem &p, int j) {
    return j < p.n ? p.A + (size_t)j * p.A_cstride : p.bcol;
}

// Panel k0..k1-1 (k1 <= n) of problem p by the calling workgroup; qbuf holds
// N complex numbers in LDS.  Raises *sing (and returns) on a singular column.
template <class R, int RPL>
HCN_DEV void tiled_panel(const MgsProblem &p, int k0, int k1, int *sing, double *qbuf) {
    constexpr int P = limbs<R>::P;
    constexpr int W = 2 * P;
    __shared__ int s_bad;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, N = p.N;
    const int j = k0 + w;
    const bool own = j < k1;
    double *aj = own ? tiled_col(p, j) : nullptr;
    cx<R> v[RPL];
    if (own) wcol_load<R, RPL>(v, aj, N, lane);
    for (int k = k0; k < k1; ++k) {
        if (own && j == k) {
            R s = rmake<R>(0.0);
#pragma unroll
            for (int r = 0; r < RPL; ++r) {
                const int i = lane + 64 * r;
                if (i < N) s = r == 0 ? cnorm2(v[r]) : add(s, cnorm2(v[r]));
            }
            s = wave_rsum(s);
            const R rkk = sqrt(s);
            const bool bad = !(lead(rkk) > 0.0) || !rfinite(rkk);
            if (!bad) {
                const R iv = div(rmake<R>(1.0), rkk);
#pragma unroll
                for (int r = 0; r < RPL; ++r) v[r] = cscale(iv, v[r]);
                wcol_store<R, RPL>(v, qbuf, N, lane);
                wcol_store<R, RPL>(v, aj, N, lane);
                if (lane == 0) {
                    rstore(p.inv + (size_t)k * P, iv);
                    const cx<R> rc{rkk, rmake<R>(0.0)};
                    cstore(p.R + ((size_t)k * p.n + k) * W, rc);
                }
            }
            if (lane == 0) s_bad = bad ? 1 : 0;
        }
        __syncthreads();
        if (s_bad) {
            if (threadIdx.x == 0) *sing = 1;
            return;
        }
        if (own && j > k) {
            const cx<R> rv = wcol_dot<R, RPL>(qbuf, v, N, lane);
            if (lane == 0) cstore(p.R + ((size_t)j * p.n + k) * W, rv);
            wcol_axpy<R, RPL>(qbuf, v, rv, N, lane);
        }
        __syncthreads();
    }
}

// Projections k0..k1-1 applied to column j (k1 <= j <= n) by the calling
// wavefront.
template <class R, int RPL>
HCN_DEV void tiled_trail(const MgsProblem &p, int k0, int k1, int j) {
    constexpr int W = 2 * limbs<R>::P;
    const int lane = threadIdx.x & 63, N = p.N;
    double *aj = tiled_col(p, j);
    cx<R> v[RPL];
    wcol_load<R, RPL>(v, aj, N, lane);
    for (int k = k0; k < k1; ++k) {
        const double *qk = tiled_col(p, k);
        const cx<R> rv = wcol_dot<R, RPL>(qk, v, N, lane);
        if (lane == 0) cstore(p.R + ((size_t)j * p.n + k) * W, rv);
        wcol_axpy<R, RPL>(qk, v, rv, N, lane);
    }
    wcol_store<R, RPL>(v, aj, N, lane);
}

}  // namespace hcn
