// batch.hip -- a slot table of paths of many systems (one precision), all
// advanced together: every kernel launch covers every occupied slot, each
// workgroup finding its path's system and workspace from the slot index.
//
// Per step: begin (one workgroup per slot: trial t, predictor), then
// max_iter times { monomials (one workgroup per (slot, block of 256
// monomials)), sums (one per (slot, block of 256 outputs)), MGS (one per
// slot, one launch per lane-group width; or, for slots whose system has at
// least split_n unknowns, the tiled MGS of mgs_tiled.hpp: a panel launch and
// a trailing launch per panel of columns, each covering all such slots) },
// then end (controller).  The
// work lists are rebuilt on the host when slots are added or released; the
// step is captured once into a HIP graph and replayed.  Each slot's
// arithmetic depends only on its own system, point and tuning entry, so a
// path gives the same bits alone and in any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

#include "eval_body.hpp"
#include "internal.hpp"
#include "mgs_common.hpp"
#include "mgs_tiled.hpp"
#include "mp.hpp"
#include "prof.hpp"
#include "registry.hpp"
#include "track_body.hpp"

namespace hcn {

struct BatchDev {
    int P, max_n, max_nparts, relax_k;
    int mixed;            // FP64 Jacobian and solve, DD/QD residual and update
    const SysView *sys;   // registry
    const int *slot_sys;  // [cap] registry index, -1 empty
    const int *slot_lds;  // [cap] stage [A | b] in LDS
    double *x, *x_acc, *x_prev, *x_out, *sc, *J, *R, *inv, *dx, *np, *t, *gamma;
    double *x_old;        // [cap][3][xs] older accepted points (NULL: predictor order <= 1)
    PathState *st;
    hcn_path_result *res;
    int *sing;            // [cap] singular column seen by the tiled MGS
    long xs, scs, Js, Rs, invs, nps;
    TrackArgs prm;
};

HCN_DEV TrackPath slot_path(const BatchDev &d, int slot) {
    TrackPath p;
    p.n = d.sys[d.slot_sys[slot]].n;
    p.st = d.st + slot;
    p.x = d.x + (size_t)slot * d.xs;
    p.x_acc = d.x_acc + (size_t)slot * d.xs;
    p.x_prev = d.x_prev + (size_t)slot * d.xs;
    p.x_out = d.x_out + (size_t)slot * d.xs;
    p.old_stride = d.xs;
    p.x_old = d.x_old ? d.x_old + (size_t)slot * (MAX_PREDICTOR_ORDER - 1) * d.xs : nullptr;
    p.t = d.t + slot;
    p.res = d.res + slot;
    return p;
}

template <class R>
__global__ void k_b_init(BatchDev d, int slot, const double *x0) {
    track_init_one<R>(d.prm, slot_path(d, slot), x0);
}

template <class R>
__global__ void k_b_begin(BatchDev d, const int *slots) {
    track_begin_one<R>(d.prm, slot_path(d, slots[blockIdx.x]));
}

template <class R>
__global__ void k_b_end(BatchDev d, const int *slots) {
    track_end_one<R>(d.prm, slot_path(d, slots[blockIdx.x]));
}

// UNI (every registered system mon_uniform): the workgroup first tabulates
// the slot point's powers in LDS when its system has exponents above two
template <class R, int KB, int MODE, bool UNI>
__global__ __launch_bounds__(256) void k_b_mon(BatchDev d, const int2 *work) {
    extern __shared__ double pows[];
    const int2 w = work[blockIdx.x];
    const int slot = w.x;
    if (!d.st[slot].c_active) return;
    const SysView &s = d.sys[d.slot_sys[slot]];
    const double *xb = d.x + (size_t)slot * d.xs;
    const bool table = UNI && s.max_e > 2;
    if (table) {
        stage_pows<R>(s, xb, d.P, pows);
        __syncthreads();
    }
    const PointView pv{xb, 2 * d.P, d.P, table ? pows : nullptr};
    const int m = w.y * 256 + threadIdx.x;
    if (m >= s.nmon) return;
    if constexpr (KB == 0)
        mon_one_long<R, MODE, UNI>(s, m, pv, d.sc + (size_t)slot * d.scs);
    else
        mon_one<R, KB, MODE, UNI>(s, m, pv, d.sc + (size_t)slot * d.scs);
}

// what a sum launch forms: the full [J | -h] with its norm parts, the
// residual only (rounded -h into the FP64 matrix, with norm parts), or the
// FP64 Jacobian only
enum { BSUM_FULL = 0, BSUM_RESIDUAL = 1, BSUM_JACOBIAN = 2 };

template <class R, int VARIANT>
__global__ __launch_bounds__(256) void k_b_sum(BatchDev d, const int2 *work) {
    constexpr int W = 2 * limbs<R>::P;
    constexpr int WJ = VARIANT == BSUM_RESIDUAL ? 2 : W;  // element width of the matrix
    __shared__ double red[256 / 64];
    const int2 w = work[xcd_logical(blockIdx.x, gridDim.x)];
    const int slot = w.x;
    if (!d.st[slot].c_active) return;
    const SysView &s = d.sys[d.slot_sys[slot]];
    double *J = d.J + (size_t)slot * d.Js;
    SumOut o;
    o.jac = VARIANT == BSUM_RESIDUAL ? 0 : 1;
    o.J = VARIANT == BSUM_RESIDUAL ? nullptr : J;
    o.J_cstride = (long)s.N * WJ;
    o.f = VARIANT == BSUM_JACOBIAN ? nullptr : J + (size_t)s.n * s.N * WJ;
    o.f_neg = 1;
    o.f_lead_only = VARIANT == BSUM_RESIDUAL ? 1 : 0;
    const long e = (long)w.y * 256 + threadIdx.x;
    const double mx = sum_one<R>(s, e, d.sc + (size_t)slot * d.scs, d.x + (size_t)slot * d.xs, d.P,
                                 1, d.relax_k, d.t[slot], d.gamma + (size_t)slot * 2 * d.P, d.P, o);
    if (VARIANT == BSUM_JACOBIAN) return;
    const double r = block_max(mx, red);
    if (threadIdx.x == 0) d.np[(size_t)slot * d.nps + w.y] = r;
}

__global__ void k_b_fig2_pre(BatchDev d, const int *slots, int count) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const int slot = slots[q];
    const SysView &s = d.sys[d.slot_sys[slot]];
    MgsProblem p = {};
    p.norm_part = d.np + (size_t)slot * d.nps;
    p.nparts = (s.N + 255) / 256;
    p.st = d.st + slot;
    (void)fig2_decide(p);
}

template <class Rx>
__global__ __launch_bounds__(MGS_THREADS) void k_b_mixed_update(BatchDev d, const int *slots) {
    constexpr int Wx = 2 * limbs<Rx>::P;
    __shared__ double s_red[MGS_THREADS / 64];
    const int slot = slots[blockIdx.x];
    PathState &st = d.st[slot];
    if (!st.c_active) return;
    const int n = d.sys[d.slot_sys[slot]].n;
    const double *dx = d.sc + (size_t)slot * d.scs;
    double *x = d.x + (size_t)slot * d.xs;
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += MGS_THREADS)
        m = nanmax(m, nanmax(fabs(dx[2 * i]), fabs(dx[2 * i + 1])));
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = m;
    __syncthreads();
    double dxn = s_red[0];
    for (int w = 1; w < MGS_THREADS / 64; ++w) dxn = nanmax(dxn, s_red[w]);
    if (dxn == dxn) {
        for (int i = threadIdx.x; i < n; i += MGS_THREADS) {
            double *q = x + (size_t)i * Wx;
            const cx<double> dd{dx[2 * i], dx[2 * i + 1]};
            cstore(q, cadd(cload<Rx>(q), cwiden<Rx>(dd)));
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) fig2_after_update(st, dxn);
}

// the solve of one slot with every pointer resolved (R: solve precision)
template <class R>
HCN_DEV MgsProblem slot_problem(const BatchDev &d, int slot) {
    constexpr int W = 2 * limbs<R>::P;
    const SysView &s = d.sys[d.slot_sys[slot]];
    MgsProblem p;
    p.N = s.N;
    p.n = s.n;
    p.mode = d.mixed ? MGS_MIXED_SOLVE : MGS_NEWTON_FIG2;
    p.lds = d.slot_lds[slot];
    p.A = d.J + (size_t)slot * d.Js;
    p.A_cstride = (long)s.N * W;
    p.bcol = p.A + (size_t)s.n * s.N * W;
    p.R = d.R + (size_t)slot * d.Rs;
    p.inv = d.inv + (size_t)slot * d.invs;
    p.dx = d.sc + (size_t)slot * d.scs;  // the scratch is free once the sums are formed
    p.status = nullptr;
    p.x = d.x + (size_t)slot * d.xs;
    p.norm_part = d.np + (size_t)slot * d.nps;
    p.nparts = (int)(((long)s.n * s.N + s.N + 255) / 256);
    p.norms = nullptr;
    p.st = d.st + slot;
    return p;
}

template <class R, int GRP>
__global__ __launch_bounds__(MGS_THREADS) void k_b_mgs(BatchDev d, const int *slots) {
    mgs_wg<R, GRP>(slot_problem<R>(d, slots[blockIdx.x]));
}

// left-looking panel MGS (bitwise that of k_b_mgs) for slots whose table
// entry asks for it; RPL covers the largest row count of the launch
template <class R, int GRP, int RPL>
__global__ __launch_bounds__(MGS_THREADS) void k_b_mgs_panel(BatchDev d, const int *slots) {
    mgs_panel<R, GRP, RPL>(slot_problem<R>(d, slots[blockIdx.x]));
}

// Persistent form of a plain step for one slot per workgroup: begin, then
// max_iter times {monomials, sums, one-workgroup MGS with the Fig. 2 tests},
// then end; the same device functions on the same data in the same order as
// the launches of a captured step, so a path gets bitwise the same results.
// The workgroup runs up to `steps` steps of its path without returning to
// the host, and stops once the path is done (every later step would leave a
// finished path unchanged).  The monomials take the general form (forward
// products parked in their output slots, any size up to 64 variables,
// exponents by branching), which gives the same bits as the register and
// uniform forms of the captured step and keeps this kernel to one instance
// per precision and lane-group width.  The dynamic LDS holds [A | b] during
// a solve staged in LDS.
template <class R>
HCN_DEV void b_sum_full(const BatchDev &d, int slot, const SysView &s, int nparts, double *red) {
    constexpr int W = 2 * limbs<R>::P;
    double *J = d.J + (size_t)slot * d.Js;
    SumOut o;
    o.jac = 1;
    o.J = J;
    o.J_cstride = (long)s.N * W;
    o.f = J + (size_t)s.n * s.N * W;
    o.f_neg = 1;
    o.f_lead_only = 0;
    for (int part = 0; part < nparts; ++part) {
        const long e = (long)part * 256 + threadIdx.x;
        const double mx = sum_one<R>(s, e, d.sc + (size_t)slot * d.scs, d.x + (size_t)slot * d.xs, d.P,
                                     1, d.relax_k, d.t[slot], d.gamma + (size_t)slot * 2 * d.P, d.P, o);
        const double r = block_max(mx, red);
        if (threadIdx.x == 0) d.np[(size_t)slot * d.nps + part] = r;
    }
}

template <class R, int GRP>
__global__ __launch_bounds__(MGS_THREADS) void k_b_persist(BatchDev d, const int *slots, int steps) {
    __shared__ double red[256 / 64];
    const int slot = slots[blockIdx.x];
    const TrackPath path = slot_path(d, slot);
    const SysView &s = d.sys[d.slot_sys[slot]];
    const double *xb = d.x + (size_t)slot * d.xs;
    double *sc = d.sc + (size_t)slot * d.scs;
    const int nparts = (int)(((long)s.n * s.N + s.N + 255) / 256);
    for (int q = 0; q < steps; ++q) {
        __syncthreads();
        if (d.st[slot].phase == PHASE_DONE) return;
        track_begin_one<R>(d.prm, path);
        for (int it = 0; it < d.prm.max_iter; ++it) {
            // the state written by one lane is read by all after a barrier
            __syncthreads();
            if (d.st[slot].c_active) {
                const PointView pv{xb, 2 * d.P, d.P, nullptr};
                for (int m = threadIdx.x; m < s.nmon; m += MGS_THREADS) {
                    if (s.mon_k[m] > 64)
                        mon_one_long<R, MON_FSLOT, false>(s, m, pv, sc);
                    else
                        mon_one<R, 64, MON_FSLOT, false>(s, m, pv, sc);
                }
                __syncthreads();
                b_sum_full<R>(d, slot, s, nparts, red);
                __syncthreads();
            }
            mgs_wg<R, GRP>(slot_problem<R>(d, slot));
        }
        __syncthreads();
        track_end_one<R>(d.prm, path);
    }
}

// tiled MGS of the large slots: the Fig. 2 tests before the solve (already
// taken by the residual pass in mixed mode) and a cleared singular flag
__global__ void k_bt_pre(BatchDev d, const int *slots, int count) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    const int slot = slots[q];
    d.sing[slot] = 0;
    if (!d.mixed) (void)fig2_decide(slot_problem<double>(d, slot));
}

template <class R, int RPL>
__global__ __launch_bounds__((64 * tiled_max_waves<R, RPL>())) void k_bt_panel(BatchDev d, const int *slots,
                                                                                 int k0, int T) {
    extern __shared__ double qbuf[];
    const int slot = slots[blockIdx.x];
    if (!d.st[slot].c_active || d.sing[slot]) return;
    const MgsProblem p = slot_problem<R>(d, slot);
    if (k0 >= p.n) return;
    tiled_panel<R, RPL>(p, k0, min(k0 + T, p.n), d.sing + slot, qbuf);
}

template <class R, int RPL>
__global__ __launch_bounds__(MGS_THREADS) void k_bt_trail(BatchDev d, const int *slots, int k0, int T) {
    const int slot = slots[blockIdx.y];
    if (!d.st[slot].c_active || d.sing[slot]) return;
    const MgsProblem p = slot_problem<R>(d, slot);
    if (k0 >= p.n) return;
    const int k1 = min(k0 + T, p.n);
    const int j = k1 + 4 * (int)blockIdx.x + (int)(threadIdx.x >> 6);
    if (j > p.n) return;
    tiled_trail<R, RPL>(p, k0, k1, j);
}

template <class R>
__global__ __launch_bounds__(MGS_THREADS) void k_bt_finish(BatchDev d, const int *slots) {
    const int slot = slots[blockIdx.x];
    if (!d.st[slot].c_active) return;
    mgs_epilogue<R>(slot_problem<R>(d, slot), d.sing[slot] != 0);
}

__global__ void k_b_counts(BatchDev d, int cap, int32_t *out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= cap) return;
    const bool occ = d.slot_sys[s] >= 0;
    out[2 * s] = occ ? d.st[s].evals : 0;
    out[2 * s + 1] = occ ? d.st[s].solves : 0;
}

__global__ void k_b_flags(BatchDev d, int cap, int32_t *done, int32_t *running) {
    __shared__ int red[256 / 64];
    int c = 0;
    for (int s = threadIdx.x; s < cap; s += blockDim.x) {
        const bool occ = d.slot_sys[s] >= 0;
        const bool fin = occ && d.st[s].phase == PHASE_DONE;
        done[s] = fin ? 1 : 0;
        c += (occ && !fin) ? 1 : 0;
    }
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        *running = t;
    }
}

}  // namespace hcn

using namespace hcn;

namespace {

thread_local std::string g_berr;

int bfail(int code, const char *msg) {
    g_berr = msg;
    return code;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

// one-workgroup MGS forms per lane-group width: k_b_mgs, and k_b_mgs_panel
// with 1, 2, 4, 8 or 16 rows per lane
constexpr int NFORM = 6;
constexpr int NMGS_GROUPS = 3 * NFORM;

int kbucket_b(int k) {
    if (k <= 4) return 4;
    if (k <= 8) return 8;
    if (k <= 16) return 16;
    if (k <= 32) return 32;
    if (k <= 64) return 64;
    return 1 << 30;  // the loop form
}

}  // namespace

struct hcn_batch_s {
    int P = 2, cap = 0, max_n = 0, max_nslots = 0, max_sys = 0;
    BatchDev d = {};
    void *dmem = nullptr;
    size_t bytes = 0;
    // registry: the systems the slots refer to (holding a reference on
    // each) and their device views, by registry index
    SysRegistry<hcn_sys> reg{0};
    std::vector<SysView> views;
    SysView *d_sys = nullptr;
    int kb = 4;
    // slots
    std::vector<int> slot_sys, slot_lds;
    int *d_slot_sys = nullptr, *d_slot_lds = nullptr;
    // work lists
    int2 *d_mon = nullptr, *d_sum = nullptr, *d_sumf = nullptr;
    int *d_slots = nullptr;
    int n_mon = 0, n_sum = 0, n_sumf = 0, n_slots = 0;
    // large slots (n >= split_n; 0: none) solve with the tiled MGS
    int split_n = 0;
    // plain steps as one persistent workgroup per slot (no tiled slots)
    bool persistent = false;
    int *d_big = nullptr;
    int n_big = 0, big_maxn = 0, big_maxN = 0;
    // one-workgroup MGS launches: lane-group width index g (8, 16, 32) times
    // form f (0: k_b_mgs, 1 + log2 RPL: k_b_mgs_panel), group g * NFORM + f
    int grp_off[NMGS_GROUPS] = {}, grp_cnt[NMGS_GROUPS] = {};
    size_t grp_lds[NMGS_GROUPS] = {};
    long mon_cap = 0, sum_cap = 0;
    int32_t *d_done = nullptr, *d_running = nullptr;
    int32_t *h_running = nullptr, *h_done = nullptr;
    bool dirty = true;
    hipGraphExec_t exec = nullptr;
    // for callers on the legacy null stream (which cannot be captured) the
    // graph runs on a stream of the batch's own, created at first use
    hipStream_t own = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

extern "C" const char *hcn_batch_last_error(void) { return g_berr.c_str(); }

namespace {

template <class R, int MODE, bool UNI>
void launch_b_mon_u(hcn_batch_s *b, size_t lds, hipStream_t s) {
    const BatchDev &d = b->d;
    constexpr int ML = MODE == MON_VALUES ? MON_VALUES : MON_FSLOT;
    const dim3 g(b->n_mon), t(256);
    switch (b->kb) {
        case 4: hipLaunchKernelGGL((k_b_mon<R, 4, MODE, UNI>), g, t, lds, s, d, b->d_mon); break;
        case 8: hipLaunchKernelGGL((k_b_mon<R, 8, MODE, UNI>), g, t, lds, s, d, b->d_mon); break;
        case 16: hipLaunchKernelGGL((k_b_mon<R, 16, MODE, UNI>), g, t, lds, s, d, b->d_mon); break;
        case 32: hipLaunchKernelGGL((k_b_mon<R, 32, ML, UNI>), g, t, lds, s, d, b->d_mon); break;
        case 64: hipLaunchKernelGGL((k_b_mon<R, 64, ML, UNI>), g, t, lds, s, d, b->d_mon); break;
        default: hipLaunchKernelGGL((k_b_mon<R, 0, ML, UNI>), g, t, lds, s, d, b->d_mon); break;
    }
}

template <class R, int MODE>
void launch_b_mon(hcn_batch_s *b, hipStream_t s) {
    // the power table of the largest registered system (each workgroup uses
    // its own); the uniform form of the common factor when every system
    // allows it (both forms give the same bits)
    size_t lds = 0;
    bool uni = false;  // every registered system allows the uniform form
    for (int q = 0; q < b->reg.size(); ++q) {
        if (!b->reg.live(q)) continue;
        const SysView &v = b->views[q];
        if (lds == 0 && !uni) uni = true;
        lds = std::max(lds, mon_stage_bytes(v, limbs<R>::P));
        if (!mon_uniform(v, limbs<R>::P)) uni = false;
    }
    if (uni)
        launch_b_mon_u<R, MODE, true>(b, lds, s);
    else
        launch_b_mon_u<R, MODE, false>(b, lds, s);
}

template <class R, int RPL>
void launch_b_tiled_rpl(hcn_batch_s *b, hipStream_t s) {
    const BatchDev &d = b->d;
    constexpr int T = tiled_max_waves<R, RPL>();
    const size_t lds = (size_t)b->big_maxN * 2 * limbs<R>::P * sizeof(double);
    for (int k0 = 0; k0 < b->big_maxn; k0 += T) {
        hipLaunchKernelGGL((k_bt_panel<R, RPL>), dim3(b->n_big), dim3(64 * T), lds, s, d, b->d_big, k0, T);
        const int cols = b->big_maxn + 1 - std::min(k0 + T, b->big_maxn);
        hipLaunchKernelGGL((k_bt_trail<R, RPL>), dim3((cols + 3) / 4, b->n_big), dim3(MGS_THREADS), 0, s, d,
                           b->d_big, k0, T);
    }
}

template <class R>
void launch_b_tiled(hcn_batch_s *b, hipStream_t s) {
    if (b->n_big == 0) return;
    hipLaunchKernelGGL(k_bt_pre, dim3((b->n_big + 255) / 256), dim3(256), 0, s, b->d, b->d_big, b->n_big);
    switch (tiled_rpl(b->big_maxN, limbs<R>::P)) {
        case 1: launch_b_tiled_rpl<R, 1>(b, s); break;
        case 2: launch_b_tiled_rpl<R, 2>(b, s); break;
        case 4: launch_b_tiled_rpl<R, 4>(b, s); break;
        default:
            if constexpr (limbs<R>::P != 4) launch_b_tiled_rpl<R, 8>(b, s);
            break;
    }
    hipLaunchKernelGGL(k_bt_finish<R>, dim3(b->n_big), dim3(MGS_THREADS), 0, s, b->d, b->d_big);
}

template <class R, int GRP>
void launch_b_mgs_grp(hcn_batch_s *b, int g, hipStream_t s) {
    const BatchDev &d = b->d;
    for (int f = 0; f < NFORM; ++f) {
        const int q = g * NFORM + f;
        const int cnt = b->grp_cnt[q];
        if (cnt == 0) continue;
        const int *list = b->d_slots + b->grp_off[q];
        const dim3 grid(cnt), block(MGS_THREADS);
        if (f == 0) {
            hipLaunchKernelGGL((k_b_mgs<R, GRP>), grid, block, b->grp_lds[q], s, d, list);
            continue;
        }
        if constexpr (limbs<R>::P != 4) {
            switch (f) {
                case 1: hipLaunchKernelGGL((k_b_mgs_panel<R, GRP, 1>), grid, block, 0, s, d, list); break;
                case 2: hipLaunchKernelGGL((k_b_mgs_panel<R, GRP, 2>), grid, block, 0, s, d, list); break;
                case 3: hipLaunchKernelGGL((k_b_mgs_panel<R, GRP, 4>), grid, block, 0, s, d, list); break;
                case 4: hipLaunchKernelGGL((k_b_mgs_panel<R, GRP, 8>), grid, block, 0, s, d, list); break;
                default: hipLaunchKernelGGL((k_b_mgs_panel<R, GRP, 16>), grid, block, 0, s, d, list); break;
            }
        }
    }
}

template <class R>
void launch_b_mgs(hcn_batch_s *b, hipStream_t s) {
    launch_b_tiled<R>(b, s);
    launch_b_mgs_grp<R, 8>(b, 0, s);
    launch_b_mgs_grp<R, 16>(b, 1, s);
    launch_b_mgs_grp<R, 32>(b, 2, s);
}

// `steps` plain steps of every slot by the persistent kernels, one launch
// per lane-group width (the slots of one width are contiguous in the list)
template <class R>
int enqueue_persist(hcn_batch_s *b, int steps, hipStream_t s) {
    const int lim = (int)mgs_lds_limit();
    for (int g = 0; g < 3; ++g) {
        int cnt = 0;
        for (int f = 0; f < NFORM; ++f) cnt += b->grp_cnt[g * NFORM + f];
        if (cnt == 0) continue;
        const int *list = b->d_slots + b->grp_off[g * NFORM];
        const size_t lds = b->grp_lds[g * NFORM];
        const dim3 grid(cnt), block(MGS_THREADS);
        const void *fn = g == 0 ? (const void *)k_b_persist<R, 8>
                       : g == 1 ? (const void *)k_b_persist<R, 16> : (const void *)k_b_persist<R, 32>;
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (g == 0)
            hipLaunchKernelGGL((k_b_persist<R, 8>), grid, block, lds, s, b->d, list, steps);
        else if (g == 1)
            hipLaunchKernelGGL((k_b_persist<R, 16>), grid, block, lds, s, b->d, list, steps);
        else
            hipLaunchKernelGGL((k_b_persist<R, 32>), grid, block, lds, s, b->d, list, steps);
    }
    return (int)hipGetLastError();
}

template <class R>
int enqueue_step(hcn_batch_s *b, hipStream_t s) {
    const BatchDev &d = b->d;
    if (b->n_slots == 0) return 0;
    hipLaunchKernelGGL(k_b_begin<R>, dim3(b->n_slots), dim3(64), 0, s, d, b->d_slots);
    constexpr bool isdd = limbs<R>::P == 2;
    for (int it = 0; it < d.prm.max_iter; ++it) {
        if (!d.mixed) {
            launch_b_mon<R, isdd ? MON_FREG : MON_FSLOT>(b, s);
            hipLaunchKernelGGL((k_b_sum<R, BSUM_FULL>), dim3(b->n_sum), dim3(256), 0, s, d, b->d_sum);
            launch_b_mgs<R>(b, s);
        } else {
            // residual in DD/QD, its rounding the right-hand side; Fig. 2 tests
            launch_b_mon<R, MON_VALUES>(b, s);
            hipLaunchKernelGGL((k_b_sum<R, BSUM_RESIDUAL>), dim3(b->n_sumf), dim3(256), 0, s, d, b->d_sumf);
            hipLaunchKernelGGL(k_b_fig2_pre, dim3((b->n_slots + 255) / 256), dim3(256), 0, s, d,
                               b->d_slots, b->n_slots);
            // Jacobian and solve in FP64, update in DD/QD
            launch_b_mon<double, MON_FREG>(b, s);
            hipLaunchKernelGGL((k_b_sum<double, BSUM_JACOBIAN>), dim3(b->n_sum), dim3(256), 0, s, d, b->d_sum);
            launch_b_mgs<double>(b, s);
            hipLaunchKernelGGL(k_b_mixed_update<R>, dim3(b->n_slots), dim3(MGS_THREADS), 0, s, d, b->d_slots);
        }
    }
    hipLaunchKernelGGL(k_b_end<R>, dim3(b->n_slots), dim3(64), 0, s, d, b->d_slots);
    return (int)hipGetLastError();
}

template <class R>
void set_lds_attributes() {
    const int lim = (int)mgs_lds_limit();
    (void)hipFuncSetAttribute((const void *)k_b_mgs<R, 8>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void *)k_b_mgs<R, 16>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void *)k_b_mgs<R, 32>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

// a slot solves with the tiled MGS when its system has at least split_n
// unknowns and its columns fit the tiled kernels' registers; this depends
// on the slot's own system only, so a path's bits do not depend on the mix
bool big_slot(const hcn_batch_s *b, const SysView &v) {
    const int Ps = b->d.mixed ? 1 : b->P;
    return b->split_n > 0 && v.n >= b->split_n && tiled_rpl(v.N, Ps) > 0;
}

// work lists from the occupied slots; slots grouped by MGS lane-group width
int rebuild(hcn_batch_s *b) {
    std::vector<int2> mon, sum, sumf;
    std::vector<int> lists[NMGS_GROUPS], big;
    const int Ps = b->d.mixed ? 1 : b->P;  // precision of the solve
    b->big_maxn = b->big_maxN = 0;
    size_t lds_need[NMGS_GROUPS] = {};
    for (int s = 0; s < b->cap; ++s) {
        if (b->slot_sys[s] < 0) continue;
        const SysView &v = b->views[b->slot_sys[s]];
        const int mb = (v.nmon + 255) / 256;
        for (int q = 0; q < mb; ++q) mon.push_back(make_int2(s, q));
        const int sb = sum_nparts(v, 1);
        for (int q = 0; q < sb; ++q) sum.push_back(make_int2(s, q));
        const int sf = sum_nparts(v, 0);
        for (int q = 0; q < sf; ++q) sumf.push_back(make_int2(s, q));
        b->slot_lds[s] = 0;
        if (big_slot(b, v)) {
            big.push_back(s);
            b->big_maxn = std::max(b->big_maxn, v.n);
            b->big_maxN = std::max(b->big_maxN, v.N);
            continue;
        }
        const int grp = tune_mgs_group(Ps, v.N), choice = tune_mgs_lds(Ps, v.N);
        const int g = grp == 8 ? 0 : grp == 32 ? 2 : 1;
        const int prpl = choice == 3 ? mgs_panel_rpl(v.N, Ps, grp) : 0;
        if (prpl > 0) {
            int f = 1;
            while ((1 << (f - 1)) < prpl) ++f;
            lists[g * NFORM + f].push_back(s);
            continue;
        }
        lists[g * NFORM].push_back(s);
        const size_t bytes = mgs_lds_bytes(v.N, v.n, Ps);
        const int lds = (bytes <= mgs_lds_limit() && choice == 1) ? 1 : 0;
        b->slot_lds[s] = lds;
        if (lds) lds_need[g * NFORM] = std::max(lds_need[g * NFORM], bytes);
    }
    std::vector<int> slots;
    for (int g = 0; g < NMGS_GROUPS; ++g) {
        b->grp_off[g] = (int)slots.size();
        b->grp_cnt[g] = (int)lists[g].size();
        b->grp_lds[g] = lds_need[g];
        slots.insert(slots.end(), lists[g].begin(), lists[g].end());
    }
    b->n_mon = (int)mon.size();
    b->n_sum = (int)sum.size();
    b->n_sumf = (int)sumf.size();
    // the large slots follow the others in the slot list: begin, end and the
    // mixed-precision kernels cover all, the one-workgroup MGS its groups only
    b->n_big = (int)big.size();
    slots.insert(slots.end(), big.begin(), big.end());
    b->d_big = b->d_slots + (slots.size() - big.size());
    b->n_slots = (int)slots.size();
    if ((long)mon.size() > b->mon_cap || (long)sum.size() > b->sum_cap)
        return bfail(HCN_EINVAL, "hcn_batch: work list exceeds its capacity");
    hipError_t e = hipSuccess;
    if (!mon.empty()) e = hipMemcpy(b->d_mon, mon.data(), mon.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (!e && !sum.empty()) e = hipMemcpy(b->d_sum, sum.data(), sum.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (!e && !sumf.empty()) e = hipMemcpy(b->d_sumf, sumf.data(), sumf.size() * sizeof(int2), hipMemcpyHostToDevice);
    if (!e && !slots.empty()) e = hipMemcpy(b->d_slots, slots.data(), slots.size() * sizeof(int), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(b->d_slot_sys, b->slot_sys.data(), b->cap * sizeof(int), hipMemcpyHostToDevice);
    if (!e) e = hipMemcpy(b->d_slot_lds, b->slot_lds.data(), b->cap * sizeof(int), hipMemcpyHostToDevice);
    if (e) return bfail(HCN_EDEVICE, hipGetErrorString(e));
    b->dirty = false;
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    return HCN_OK;
}

}  // namespace

extern "C" {

int hcn_batch_create(hcn_batch *out, int P, int capacity, int max_n, int max_nslots,
                     int max_systems, const hcn_track_params *prm, int relax_k, int flags) {
    if (!out || !prm) return bfail(HCN_EINVAL, "hcn_batch_create: NULL argument");
    *out = nullptr;
    if ((P != 2 && P != 4) || capacity < 1 || max_n < 1 || max_n > 1024 || max_nslots < 1 ||
        max_systems < 1 || relax_k < 1)
        return bfail(HCN_EINVAL, "hcn_batch_create: bad sizes (P 2/4, capacity >= 1, 1 <= max_n <= 1024)");
    if (prm->max_iter < 1 || prm->max_iter > 100 || prm->max_steps < 0 || prm->end_iters < 0 ||
        !(prm->max_dt > 0.0) || prm->max_dt > 1.0 || !(prm->min_dt > 0.0) ||
        prm->predictor_order < 0 || prm->predictor_order > MAX_PREDICTOR_ORDER)
        return bfail(HCN_EINVAL, "hcn_batch_create: bad tracking parameters");
    auto *b = new hcn_batch_s;
    b->P = P;
    b->cap = capacity;
    b->max_n = max_n;
    b->max_nslots = max_nslots;
    b->max_sys = max_systems;
    b->reg = SysRegistry<hcn_sys>(max_systems);
    const long W = 2 * P;
    const long cap = capacity;
    const long xs = max_n * W;
    const long scs = std::max<long>((long)max_nslots * W, xs);  // scratch also holds dx
    const long Js = (long)(max_n + 1) * max_n * W;
    const long Rs = Js;
    const long invs = (long)max_n * P;
    const long nps = ((long)max_n * max_n + max_n + 255) / 256;
    b->mon_cap = cap * ((max_nslots + 255) / 256 + 1);
    b->sum_cap = cap * nps;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += al(bytes);
        return o;
    };
    const size_t o_x = take(cap * xs * 8), o_xa = take(cap * xs * 8), o_xp = take(cap * xs * 8),
                 o_xo = take(cap * xs * 8), o_sc = take(cap * scs * 8), o_J = take(cap * Js * 8),
                 o_R = take(cap * Rs * 8), o_inv = take(cap * invs * 8), o_np = take(cap * nps * 8),
                 o_t = take(cap * 8), o_g = take(cap * W * 8), o_st = take(cap * sizeof(PathState)),
                 o_res = take(cap * sizeof(hcn_path_result)), o_sys = take(max_systems * sizeof(SysView)),
                 o_ss = take(cap * 4), o_sl = take(cap * 4), o_mon = take(b->mon_cap * sizeof(int2)),
                 o_sum = take(b->sum_cap * sizeof(int2)), o_sumf = take(cap * ((max_n + 255) / 256) * sizeof(int2)),
                 o_slots = take(cap * 4), o_done = take(cap * 4),
                 o_run = take(4), o_sing = take(cap * 4),
                 o_old = prm->predictor_order >= 2 ? take(cap * (MAX_PREDICTOR_ORDER - 1) * xs * 8) : 0;
    b->bytes = off;
    if (hipMalloc(&b->dmem, off) != hipSuccess) {
        delete b;
        return bfail(HCN_ENOMEM, "hcn_batch_create: device allocation failed");
    }
    char *base = (char *)b->dmem;
    BatchDev &d = b->d;
    d.P = P;
    d.max_n = max_n;
    d.relax_k = relax_k;
    d.mixed = (flags & HCN_BATCH_MIXED) ? 1 : 0;
    d.x = (double *)(base + o_x);
    d.x_acc = (double *)(base + o_xa);
    d.x_prev = (double *)(base + o_xp);
    d.x_out = (double *)(base + o_xo);
    d.x_old = prm->predictor_order >= 2 ? (double *)(base + o_old) : nullptr;
    d.sc = (double *)(base + o_sc);
    d.J = (double *)(base + o_J);
    d.R = (double *)(base + o_R);
    d.inv = (double *)(base + o_inv);
    d.np = (double *)(base + o_np);
    d.t = (double *)(base + o_t);
    d.gamma = (double *)(base + o_g);
    d.st = (PathState *)(base + o_st);
    d.res = (hcn_path_result *)(base + o_res);
    d.sing = (int *)(base + o_sing);
    d.xs = xs;
    d.scs = scs;
    d.Js = Js;
    d.Rs = Rs;
    d.invs = invs;
    d.nps = nps;
    d.max_nparts = (int)nps;
    b->d_sys = (SysView *)(base + o_sys);
    b->d_slot_sys = (int *)(base + o_ss);
    b->d_slot_lds = (int *)(base + o_sl);
    b->d_mon = (int2 *)(base + o_mon);
    b->d_sum = (int2 *)(base + o_sum);
    b->d_sumf = (int2 *)(base + o_sumf);
    b->d_slots = (int *)(base + o_slots);
    b->d_done = (int32_t *)(base + o_done);
    b->d_running = (int32_t *)(base + o_run);
    d.sys = b->d_sys;
    d.slot_sys = b->d_slot_sys;
    d.slot_lds = b->d_slot_lds;
    TrackArgs &ta = d.prm;
    ta.P = P;
    ta.max_iter = prm->max_iter;
    ta.max_steps = prm->max_steps;
    ta.end_iters = prm->end_iters;
    ta.predictor_order = prm->predictor_order;
    ta.tol_res = prm->tol_res;
    ta.tol_dx = prm->tol_dx;
    ta.max_eq_val = prm->max_eq_val;
    ta.max_dt = prm->max_dt;
    ta.min_dt = prm->min_dt;
    ta.end_tol = prm->end_tol;
    b->slot_sys.assign(capacity, -1);
    b->slot_lds.assign(capacity, 0);
    if (hipHostMalloc((void **)&b->h_running, sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc((void **)&b->h_done, sizeof(int32_t) * capacity) != hipSuccess) {
        (void)hipFree(b->dmem);
        delete b;
        return bfail(HCN_ENOMEM, "hcn_batch_create: pinned allocation failed");
    }
    if (P == 2)
        set_lds_attributes<dd>();
    else
        set_lds_attributes<qd>();
    set_lds_attributes<double>();
    *out = b;
    return HCN_OK;
}

int hcn_batch_destroy(hcn_batch b) {
    if (!b) return HCN_OK;
    if (b->own) (void)hipStreamSynchronize(b->own);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->own) (void)hipStreamDestroy(b->own);
    (void)hipHostFree(b->h_running);
    (void)hipHostFree(b->h_done);
    (void)hipFree(b->dmem);
    for (hcn_sys h : b->reg.all()) sys_release(h);
    delete b;
    return HCN_OK;
}

size_t hcn_batch_device_bytes(hcn_batch b) { return b ? b->bytes : 0; }

int hcn_batch_add(hcn_batch b, int slot, hcn_sys sys, const double *gamma, const double *x0,
                  void *stream) {
    if (!b || !sys || !gamma || !x0) return bfail(HCN_EINVAL, "hcn_batch_add: NULL argument");
    if (slot < 0 || slot >= b->cap) return bfail(HCN_EINVAL, "hcn_batch_add: slot out of range");
    if (b->slot_sys[slot] >= 0) return bfail(HCN_EINVAL, "hcn_batch_add: slot is occupied");
    hcn_sys_info_t info;
    if (hcn_sys_info(sys, &info) != HCN_OK) return bfail(HCN_EINVAL, "hcn_batch_add: bad system");
    if (info.P != b->P) return bfail(HCN_EINVAL, "hcn_batch_add: precision differs from the batch");
    if (info.N != info.n) return bfail(HCN_EINVAL, "hcn_batch_add: tracking needs N == n");
    if (info.n > b->max_n || info.nslots > b->max_nslots)
        return bfail(HCN_EINVAL, "hcn_batch_add: system larger than the batch was sized for");
    bool fresh = false;
    int idx = b->reg.acquire(sys, &fresh);
    if (idx < 0) {
        // every entry is listed: once the queued work has finished, entries
        // that no slot uses any more can go
        if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
            return bfail(HCN_EDEVICE, "hcn_batch_add: sync");
        for (hcn_sys h : b->reg.collect()) sys_release(h);
        idx = b->reg.acquire(sys, &fresh);
        if (idx < 0) return bfail(HCN_EINVAL, "hcn_batch_add: too many distinct systems in the slots");
    }
    if (fresh) {
        sys_retain(sys);
        const SysView v = sys_view(sys);
        if ((int)b->views.size() < b->reg.size()) b->views.resize(b->reg.size());
        b->views[idx] = v;
        if (hipMemcpy(b->d_sys + idx, &v, sizeof(SysView), hipMemcpyHostToDevice) != hipSuccess) {
            b->reg.drop(idx);
            return bfail(HCN_EDEVICE, "hcn_batch_add: registry upload failed");
        }
        b->kb = std::max(b->kb, kbucket_b(v.max_k));
    }
    hipStream_t s = (hipStream_t)stream;
    const long W = 2 * b->P;
    if (hipMemcpyAsync(b->d.gamma + (size_t)slot * W, gamma, sizeof(double) * W,
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return bfail(HCN_EDEVICE, "hcn_batch_add: gamma upload failed");
    b->slot_sys[slot] = idx;
    // the slot table on the device must know the slot before its init runs
    if (hipMemcpyAsync(b->d_slot_sys + slot, &b->slot_sys[slot], sizeof(int), hipMemcpyHostToDevice,
                       s) != hipSuccess)
        return bfail(HCN_EDEVICE, "hcn_batch_add: slot upload failed");
    if (b->P == 2)
        hipLaunchKernelGGL(k_b_init<dd>, dim3(1), dim3(64), 0, s, b->d, slot, x0);
    else
        hipLaunchKernelGGL(k_b_init<qd>, dim3(1), dim3(64), 0, s, b->d, slot, x0);
    b->dirty = true;
    return hipGetLastError() == hipSuccess ? HCN_OK : bfail(HCN_EDEVICE, "hcn_batch_add: launch failed");
}

int hcn_batch_set_split(hcn_batch b, int min_n) {
    if (!b || min_n < 0) return bfail(HCN_EINVAL, "hcn_batch_set_split: bad argument");
    b->split_n = min_n;
    b->dirty = true;
    return HCN_OK;
}

int hcn_batch_set_persistent(hcn_batch b, int on) {
    if (!b) return bfail(HCN_EINVAL, "hcn_batch_set_persistent: NULL batch");
    b->persistent = on != 0;
    return HCN_OK;
}

int hcn_batch_release(hcn_batch b, int slot) {
    if (!b || slot < 0 || slot >= b->cap) return bfail(HCN_EINVAL, "hcn_batch_release: bad slot");
    if (b->slot_sys[slot] < 0) return HCN_OK;
    b->reg.drop(b->slot_sys[slot]);
    b->slot_sys[slot] = -1;
    b->dirty = true;
    return HCN_OK;
}

int hcn_batch_step(hcn_batch b, int steps, void *stream) {
    if (!b || steps < 0) return bfail(HCN_EINVAL, "hcn_batch_step: bad argument");
    hipStream_t s = (hipStream_t)stream;
    if (b->dirty) {
        // the slot table may only change between steps: wait for pending work
        if (hipStreamSynchronize(s) != hipSuccess) return bfail(HCN_EDEVICE, "hcn_batch_step: sync");
        const int rc = rebuild(b);
        if (rc) return rc;
    }
    if (b->n_slots == 0 || steps == 0) return HCN_OK;
    if (b->persistent && !b->d.mixed && b->n_big == 0) {
        ProfScope prof("batch_step", s);
        const int e = b->P == 2 ? enqueue_persist<dd>(b, steps, s) : enqueue_persist<qd>(b, steps, s);
        return e ? bfail(HCN_EDEVICE, "hcn_batch_step: persistent launch failed") : HCN_OK;
    }
    // the graph is captured and replayed on the caller's stream; the legacy
    // null stream cannot be captured, so its callers go through the batch's
    // own stream, joined with events on both sides
    if (!s && !b->own) {
        if (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)
            return bfail(HCN_EDEVICE, "hcn_batch_step: stream or event creation failed");
    }
    hipStream_t run = s ? s : b->own;
    if (!b->exec) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(run, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return bfail(HCN_EDEVICE, "hcn_batch_step: capture begin failed");
        const int e = b->P == 2 ? enqueue_step<dd>(b, run) : enqueue_step<qd>(b, run);
        const hipError_t ec = hipStreamEndCapture(run, &g);
        if (e || ec != hipSuccess) return bfail(HCN_EDEVICE, "hcn_batch_step: capture failed");
        const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) return bfail(HCN_EDEVICE, "hcn_batch_step: instantiate failed");
    }
    if (!s && (hipEventRecord(b->ev_in, s) != hipSuccess || hipStreamWaitEvent(run, b->ev_in, 0) != hipSuccess))
        return bfail(HCN_EDEVICE, "hcn_batch_step: stream join failed");
    {
        ProfScope prof("batch_step", run);
        for (int q = 0; q < steps; ++q)
            if (hipGraphLaunch(b->exec, run) != hipSuccess)
                return bfail(HCN_EDEVICE, "hcn_batch_step: graph launch failed");
    }
    if (!s && (hipEventRecord(b->ev_out, run) != hipSuccess || hipStreamWaitEvent(s, b->ev_out, 0) != hipSuccess))
        return bfail(HCN_EDEVICE, "hcn_batch_step: stream join failed");
    return HCN_OK;
}

int hcn_batch_poll(hcn_batch b, int32_t *done, void *stream) {
    if (!b) return bfail(HCN_EINVAL, "hcn_batch_poll: NULL batch");
    hipStream_t s = (hipStream_t)stream;
    if (b->dirty) {
        if (hipStreamSynchronize(s) != hipSuccess) return bfail(HCN_EDEVICE, "hcn_batch_poll: sync");
        const int rc = rebuild(b);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_b_flags, dim3(1), dim3(256), 0, s, b->d, b->cap, b->d_done, b->d_running);
    hipError_t e = hipMemcpyAsync(b->h_running, b->d_running, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (!e && done) e = hipMemcpyAsync(b->h_done, b->d_done, sizeof(int32_t) * b->cap, hipMemcpyDeviceToHost, s);
    if (!e) e = hipStreamSynchronize(s);
    if (e) return bfail(HCN_EDEVICE, "hcn_batch_poll: copy failed");
    if (done) std::memcpy(done, b->h_done, sizeof(int32_t) * b->cap);
    return *b->h_running;
}

int hcn_batch_counts(hcn_batch b, int32_t *counts, void *stream) {
    if (!b || !counts) return bfail(HCN_EINVAL, "hcn_batch_counts: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    int32_t *dbuf = nullptr;
    if (hipMallocAsync((void **)&dbuf, sizeof(int32_t) * 2 * b->cap, s) != hipSuccess)
        return bfail(HCN_ENOMEM, "hcn_batch_counts: allocation failed");
    if (b->dirty) {
        if (hipStreamSynchronize(s) != hipSuccess) return bfail(HCN_EDEVICE, "hcn_batch_counts: sync");
        const int rc = rebuild(b);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_b_counts, dim3((b->cap + 255) / 256), dim3(256), 0, s, b->d, b->cap, dbuf);
    hipError_t e = hipMemcpyAsync(counts, dbuf, sizeof(int32_t) * 2 * b->cap, hipMemcpyDeviceToHost, s);
    (void)hipFreeAsync(dbuf, s);
    if (!e) e = hipStreamSynchronize(s);
    return e ? bfail(HCN_EDEVICE, "hcn_batch_counts: copy failed") : HCN_OK;
}

int hcn_batch_result(hcn_batch b, int slot, double *x_out, hcn_path_result *res, void *stream) {
    if (!b || slot < 0 || slot >= b->cap || b->slot_sys[slot] < 0)
        return bfail(HCN_EINVAL, "hcn_batch_result: bad slot");
    hipStream_t s = (hipStream_t)stream;
    const SysView &v = b->views[b->slot_sys[slot]];
    hipError_t e = hipSuccess;
    if (x_out)
        e = hipMemcpyAsync(x_out, b->d.x_out + (size_t)slot * b->d.xs, sizeof(double) * v.n * 2 * b->P,
                           hipMemcpyDeviceToDevice, s);
    if (!e && res) {
        e = hipMemcpyAsync(res, b->d.res + slot, sizeof(hcn_path_result), hipMemcpyDeviceToHost, s);
        if (!e) e = hipStreamSynchronize(s);
    }
    return e ? bfail(HCN_EDEVICE, "hcn_batch_result: copy failed") : HCN_OK;
}

int hcn_batch_run(hcn_batch b, int chunk, void *stream) {
    if (!b || chunk < 1) return bfail(HCN_EINVAL, "hcn_batch_run: bad argument");
    const long bound = (long)b->d.prm.max_steps + 3 +
                       (b->d.prm.end_iters + b->d.prm.max_iter - 1) / b->d.prm.max_iter + 2;
    long done_steps = 0;
    int running = hcn_batch_poll(b, nullptr, stream);
    while (running > 0 && done_steps < bound + chunk) {
        const int rc = hcn_batch_step(b, chunk, stream);
        if (rc) return rc;
        done_steps += chunk;
        running = hcn_batch_poll(b, nullptr, stream);
        if (running < 0) return running;
    }
    return running == 0 ? HCN_OK : bfail(HCN_EDEVICE, "hcn_batch_run: paths unfinished after the step bound");
}

}  // extern "C"
