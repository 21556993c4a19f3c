// track_body.hpp -- one path's step-size controller (Fig. 3, equation (4)),
// run by one workgroup per path; shared by the single-system tracker
// (track.hip) and the slot-table batch (batch.hip).
//
// begin: trial t = min(1, t_acc + dt) and the predicted point (Section 3.1:
// the polynomial through the last accepted points, of degree
// predictor_order or one less than the points known, evaluated in Lagrange
// form); arms the corrector.  end: on success accept, count
// it and once more than two successes are counted double dt up to max_dt;
// on failure reset the count and halve dt, failing below min_dt; more than
// max_steps steps fail the path.  After t = 1 the corrector refines with
// end_tol for up to end_iters evaluations, across as many steps as needed.
#pragma once

#include "internal.hpp"
#include "mp.hpp"

namespace hcn {

struct TrackPath {
    int n;
    PathState *st;
    double *x, *x_acc, *x_prev, *x_out;
    double *x_old;      // the 3rd..5th newest accepted points (NULL: order <= 1)
    long old_stride;    // doubles between two of them
    double *t;
    hcn_path_result *res;
};

// accepted point j (0 the newest) of a path
HCN_DEV const double *hist_point(const TrackPath &p, int j) {
    return j == 0 ? p.x_acc : j == 1 ? p.x_prev : p.x_old + (size_t)(j - 2) * p.old_stride;
}

template <class R>
HCN_DEV void track_init_one(const TrackArgs &a, const TrackPath &p, const double *x0) {
    constexpr int W = 2 * limbs<R>::P;
    for (int q = threadIdx.x; q < p.n * W; q += blockDim.x) {
        p.x_acc[q] = x0[q];
        p.x[q] = x0[q];
    }
    if (threadIdx.x == 0) {
        PathState s = {};
        s.t_acc = 0.0;
        s.known = 1;
        s.dt = a.max_dt;
        s.phase = PHASE_TRACK;
        s.status = HCN_OK;
        s.c_status = C_RUNNING;
        *p.st = s;
    }
}

template <class R>
HCN_DEV void track_begin_one(const TrackArgs &a, const TrackPath &p) {
    constexpr int W = 2 * limbs<R>::P;
    __shared__ int s_mode;  // 0 idle, 1 predict, 2 copy x_acc (refine start)
    __shared__ int s_deg;
    __shared__ double s_t, s_ts[MAX_PREDICTOR_ORDER + 1];
    PathState &st = *p.st;
    if (threadIdx.x == 0) {
        int mode = 0;
        if (st.phase == PHASE_TRACK) {
            if (st.steps > a.max_steps) {
                st.status = HCN_MAX_STEPS;
                st.phase = PHASE_DONE;
                st.c_active = 0;
            } else {
                double t = st.t_acc + st.dt;
                if (t > 1.0) t = 1.0;
                st.t = t;
                *p.t = t;
                st.last = a.max_eq_val;
                st.tol_res = a.tol_res;
                st.tol_dx = a.tol_dx;
                st.c_maxit = a.max_iter;
                st.c_iter = 0;
                st.res = 0.0;
                st.dxn = 0.0;
                st.c_active = a.max_iter > 0 ? 1 : 0;
                st.c_status = a.max_iter > 0 ? C_RUNNING : HCN_NOT_CONVERGED;
                s_t = t;
                int deg = st.known - 1;
                if (deg > a.predictor_order) deg = a.predictor_order;
                if (deg < 0) deg = 0;
                s_deg = deg;
                s_ts[0] = st.t_acc;
                s_ts[1] = st.t_prev;
                for (int j = 2; j <= MAX_PREDICTOR_ORDER; ++j) s_ts[j] = st.t_old[j - 2];
                mode = 1;
            }
        } else if (st.phase == PHASE_REFINE && !st.refine_started) {
            st.refine_started = 1;
            st.t = 1.0;
            *p.t = 1.0;
            st.last = a.max_eq_val;
            st.tol_res = a.end_tol;
            st.tol_dx = a.end_tol;
            st.c_maxit = a.end_iters;
            st.c_iter = 0;
            st.res = 0.0;
            st.dxn = 0.0;
            st.c_active = 1;
            st.c_status = C_RUNNING;
            mode = 2;
        }
        s_mode = mode;
    }
    __syncthreads();
    const int mode = s_mode;
    if (mode == 0) return;
    const int deg = mode == 2 ? 0 : s_deg;
    if (deg == 0) {
        for (int q = threadIdx.x; q < p.n * W; q += blockDim.x) p.x[q] = p.x_acc[q];
        return;
    }
    // Lagrange weights w_j = prod_{m != j} (t - t_m) / prod_{m != j} (t_j - t_m),
    // products in m order from the double differences, formed alike in every
    // lane; then x = sum_j w_j x_j over j ascending
    const double t = s_t;
    R w[MAX_PREDICTOR_ORDER + 1];
    for (int j = 0; j <= deg; ++j) {
        R num = rmake<R>(1.0), den = rmake<R>(1.0);
        bool first = true;
        for (int m = 0; m <= deg; ++m) {
            if (m == j) continue;
            const R a_m = rmake<R>(t - s_ts[m]);
            const R b_m = rmake<R>(s_ts[j] - s_ts[m]);
            num = first ? a_m : mul(num, a_m);
            den = first ? b_m : mul(den, b_m);
            first = false;
        }
        w[j] = div(num, den);
    }
    for (int i = threadIdx.x; i < p.n; i += blockDim.x) {
        cx<R> acc = cscale(w[0], cload<R>(p.x_acc + (size_t)i * W));
        for (int j = 1; j <= deg; ++j) acc = cadd(acc, cscale(w[j], cload<R>(hist_point(p, j) + (size_t)i * W)));
        cstore(p.x + (size_t)i * W, acc);
    }
}

HCN_DEV void track_write_result(const TrackPath &p, const PathState &st) {
    hcn_path_result r;
    r.status = st.status;
    r.steps = st.steps;
    r.newton_iters = st.newton_iters;
    r.end_iters = st.end_iters;
    r.end_status = st.end_status;
    r.accepted = st.accepted;
    r.t = st.t_acc;
    r.res_norm = st.res;
    r.dx_norm = st.dxn;
    *p.res = r;
}

template <class R>
HCN_DEV void track_end_one(const TrackArgs &a, const TrackPath &p) {
    constexpr int W = 2 * limbs<R>::P;
    __shared__ int s_copy;  // 0 none, 1 accept (the accepted points move one
                            // back, x_acc <- x),
                            // 2 out <- x, 3 out <- x_acc, 4 accept and out <- x
    PathState &st = *p.st;
    if (threadIdx.x == 0) {
        int copy = 0;
        if (st.phase == PHASE_TRACK) {
            const int cs = st.c_status;
            st.newton_iters += st.c_iter;
            if (cs == HCN_OK) {
                st.t_old[2] = st.t_old[1];
                st.t_old[1] = st.t_old[0];
                st.t_old[0] = st.t_prev;
                st.t_prev = st.t_acc;
                st.t_acc = st.t;
                if (st.known <= MAX_PREDICTOR_ORDER) st.known += 1;
                st.accepted += 1;
                st.nsucc += 1;
                if (st.nsucc > 2) {
                    const double dt = 2.0 * st.dt;
                    st.dt = dt > a.max_dt ? a.max_dt : dt;
                }
                st.steps += 1;
                copy = 1;
                if (st.t_acc >= 1.0) {
                    if (a.end_iters > 0) {
                        st.phase = PHASE_REFINE;
                    } else {
                        st.phase = PHASE_DONE;
                        copy = 4;
                    }
                }
            } else if (cs == HCN_NAN) {
                st.status = HCN_NAN;
                st.phase = PHASE_DONE;
                st.steps += 1;
                copy = 3;
            } else {
                st.nsucc = 0;
                st.dt = 0.5 * st.dt;
                st.steps += 1;
                if (st.dt < a.min_dt) {
                    st.status = HCN_STEP_TOO_SMALL;
                    st.phase = PHASE_DONE;
                    copy = 3;
                }
            }
            if (st.phase == PHASE_DONE) st.c_active = 0;
        } else if (st.phase == PHASE_REFINE && st.refine_started && !st.c_active) {
            st.end_iters = st.c_iter;
            st.end_status = st.c_status == C_RUNNING ? HCN_NOT_CONVERGED : st.c_status;
            st.phase = PHASE_DONE;
            st.status = HCN_OK;
            copy = 2;
        }
        if (st.phase == PHASE_DONE && !st.finalized) {
            // paths stopped by the step limit in begin end here
            if (copy == 0) copy = 3;
            track_write_result(p, st);
            st.finalized = 1;
        }
        s_copy = copy;
    }
    __syncthreads();
    const int copy = s_copy;
    if (copy == 0) return;
    for (int q = threadIdx.x; q < p.n * W; q += blockDim.x) {
        if (copy == 1 || copy == 4) {
            if (p.x_old) {
                double *o = p.x_old + q;
                o[2 * p.old_stride] = o[p.old_stride];
                o[p.old_stride] = o[0];
                o[0] = p.x_prev[q];
            }
            const double xa = p.x_acc[q];
            p.x_prev[q] = xa;
            p.x_acc[q] = p.x[q];
            if (copy == 4) p.x_out[q] = p.x[q];
        } else if (copy == 2) {
            p.x_out[q] = p.x[q];
        } else {
            p.x_out[q] = p.x_acc[q];
        }
    }
}

}  // namespace hcn
