// internal.hpp -- structures shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/hcn.h"

namespace hcn {

// Device view of a loaded system.  Monomials are stored sorted by their
// number of variables k (Section 3.2: threads of one block get products of
// similar size); `perm` maps a sorted monomial back to its input index.
// Per monomial m (sorted order):
//   mon_k[m]      number of variables,
//   mon_slot[m]   slot of its value; partial p is at mon_slot + (p+1)*mon_stride,
//   mon_stride[m] size of its group of equal k (slots of a group are laid out
//                 position-major so that lanes of a wavefront write
//                 consecutive slots at the same step, Section 3.2),
//   pos[p*nmon+m] variable of position p, ex[p*nmon+m] its exponent,
//   coef[m]       [2][P] coefficient.
// Sums (Section 3.3): the value slots of equation i are
// f_list[f_ptr[i] .. f_ptr[i+1]); the partial slots of the dense Jacobian
// entry e = k*N + i (column-major) are J_list[J_ptr[e] .. J_ptr[e+1]), in
// input monomial order.
struct SysView {
    int N, n, P, nmon, max_k, nslots;
    int max_e;  // largest exponent
    const int32_t *mon_k;
    const int32_t *mon_slot;
    const int32_t *mon_stride;
    const uint16_t *pos;
    const uint8_t *ex;
    const double *coef;
    const int32_t *f_ptr;
    const int32_t *f_list;
    const int32_t *J_ptr;
    const int32_t *J_list;
    // J_list in the summation's lane order (lane q = i n + k takes entry
    // e = k N + i) interleaved per wavefront of 64 lanes (or NULL): entry c
    // of the list of lane q at J_ilv[J_wbase[q / 64] + 64 c + q % 64]
    const int32_t *J_wbase;
    const int32_t *J_ilv;
    const int32_t *deg;
};

// Homotopy h = gamma (1-t)^k g + t^k f with g_i = x_i^{d_i} - 1.
struct Homotopy {
    int on;            // 0: plain f
    int relax_k;
    int gP;            // limbs of gamma
    double gamma[8];   // [2][gP]
    const double *t;   // device [B]
};

// Per-path corrector (Fig. 2) and tracker (Fig. 3) state, in device memory.
struct PathState {
    // corrector
    double last, res, dxn, tol_res, tol_dx;
    int32_t c_status, c_iter, c_active, c_maxit;
    // tracker: accepted t values newest first (t_acc, t_prev, t_old[0..2])
    double t_acc, t_prev, dt, t;
    double t_old[3];
    int32_t phase, nsucc, steps, accepted, newton_iters, end_iters, end_status,
        known, status, refine_started, finalized;
    // work counters: residual evaluations and solves since the path started
    int32_t evals, solves;
};

enum { PHASE_TRACK = 0, PHASE_REFINE = 1, PHASE_DONE = 2 };
// highest degree of the predictor's extrapolation (Section 3.1)
constexpr int MAX_PREDICTOR_ORDER = 4;
enum { C_RUNNING = 100 };

// MGS_MIXED_SOLVE: solve only (no update), for problems whose corrector is
// still active; a singular matrix ends the corrector
enum MgsMode { MGS_SOLVE = 0, MGS_NEWTON_STEP = 1, MGS_NEWTON_FIG2 = 2, MGS_MIXED_SOLVE = 3 };

struct MgsArgs {
    int B, N, n, mode;
    double *A;          // column j of path b: A + b*A_pstride + j*A_cstride
    long A_cstride, A_pstride;
    double *bcol;       // column n when separate (else column n of A)
    long b_pstride;
    double *R;          // [B][n+1][n][2P]
    long R_pstride;
    double *inv;        // [B][n][P] 1/r_kk
    long inv_pstride;
    double *dx;         // [B][n][2P]
    long dx_pstride;
    int32_t *status;    // [B] or NULL
    double *x;          // Newton: [B][n][2P] updated in place
    long x_pstride;
    const double *norm_part;  // Newton: [B][nparts] partial residual maxima
    int nparts;
    double *norms;      // Newton step: [B][2]
    PathState *st;      // Fig. 2 mode
};

// monomial values and partials of B points (compute precision: 1, 2 or 4
// limbs, at most the storage limbs of x and of the coefficients)
struct MonArgs {
    SysView s;
    int B;
    const double *x;     // [B] points, x_pstride doubles apart, xP limbs
    long x_pstride;
    int xP;
    double *scratch;     // [B] nslots complex numbers in compute precision
    long sc_pstride;
    const PathState *st; // skip paths whose corrector is idle (or NULL)
    int values_only;
};

// sums of the slots into f (or -h) and the column-major Jacobian
struct SumArgs {
    SysView s;
    int B;
    const double *scratch;
    long sc_pstride;
    const double *x;     // for the start-system terms of the homotopy
    long x_pstride;
    int xP;
    Homotopy hom;
    int jac;             // 0: values only
    double *J;           // entry (k, i) of path b at J + b*J_pstride + k*J_cstride + i*2P
    long J_cstride, J_pstride;
    double *f;
    long f_pstride;
    int f_neg;           // store -f
    int f_lead_only;     // store the leading limbs only ([2] doubles per entry)
    double *norm_part;   // [B][nparts] block maxima of the leading limbs, or NULL
    const PathState *st;
};

// launchers (return hipError_t as int); RP = limbs of the compute precision
int launch_mon(int RP, const MonArgs &a, hipStream_t stream);
int launch_sum(int RP, const SumArgs &a, hipStream_t stream);
int sum_nparts(const SysView &s, int jac);
void set_mon_uniform(bool on);
void set_mon_tree(bool on);
int launch_mgs(int RP, const MgsArgs &a, hipStream_t stream);
// multi-workgroup MGS for large single problems: variant 2 right-looking
// (one launch per column step), 4 tiled; ints_dev holds B ints of workspace
int launch_mgs_big(int P, const MgsArgs &a, int variant, int *ints_dev, hipStream_t stream);
int mgs_tiled_rpl(int N, int P);
int mgs_panel_width();
void set_mgs_panel_width(int T);
void set_mgs_wait_limit(long long polls);
// the device tables of a loaded system (capi.hip); references held by
// batches and queued requests, the tables freed with the last
SysView sys_view(hcn_sys s);
void sys_retain(hcn_sys s);
void sys_release(hcn_sys s);

// kernel-variant table (tune.hip)
int tune_mgs_group(int P, int N);
int tune_mgs_lds(int P, int N);
size_t mgs_lds_limit();
void tune_set(int P, int N, int group, int lds);

// Fig. 2 tests before a solve, one lane per problem (norm parts of a.norm_part)
int launch_fig2_pre(const MgsArgs &a, hipStream_t stream);
// mixed precision: x (xP limbs) += dx (double), the update norm and the Fig. 2
// tests after a solve
int launch_mixed_update(int xP, const MgsArgs &a, hipStream_t stream);
int launch_elementwise(int op, int P, int count, const double *a, const double *b,
                       double *out, hipStream_t stream);

// tracker kernels
struct TrackArgs {
    int B, n, P, max_iter, max_steps, end_iters, predictor_order;
    double tol_res, tol_dx, max_eq_val, max_dt, min_dt, end_tol;
    PathState *st;
    double *x;       // working point [B][n][2P]
    double *x_acc;   // last accepted
    double *x_prev;  // the one before
    double *x_old;   // the three before that, [B][3][n][2P] (NULL for order <= 1)
    double *x_out;
    double *t;       // trial t per path [B]
    hcn_path_result *res;
    int32_t *active_count;
};
int launch_newton_init(int B, PathState *st, const hcn_newton_params &p, hipStream_t s);
int launch_newton_finish(int B, const PathState *st, double *norms, int32_t *status,
                         int32_t *iters, hipStream_t s);
int launch_track_init(const TrackArgs &a, const double *x0, hipStream_t s);
int launch_track_begin(const TrackArgs &a, hipStream_t s);
int launch_track_end(const TrackArgs &a, hipStream_t s);
int launch_track_count(const TrackArgs &a, hipStream_t s);

}  // namespace hcn
