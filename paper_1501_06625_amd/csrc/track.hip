// track.hip -- per-path corrector state (Fig. 2) and the step-size
// controller of the path tracker (Fig. 3, equation (4)), on the device.
//
// One workgroup per path.  k_track_begin forms the trial t = min(1, t_acc +
// dt) and the predicted point (linear extrapolation through the two last
// accepted points, constant before the second; Section 3.1), and arms the
// corrector.  The corrector's iterations are the evaluation and solve
// kernels.  k_track_end accepts or rejects: on success the point is
// accepted, the success count grows and once it exceeds two dt doubles up
// to max_dt; on failure the count resets and dt halves, failing below
// min_dt; paths taking more than max_steps steps fail.  After t = 1 the
// corrector refines with end_tol for up to end_iters evaluations, across as
// many steps as needed.
#include "internal.hpp"
#include "mp.hpp"

namespace hcn {

constexpr int TRK_THREADS = 64;

__global__ void k_newton_init(int B, PathState *st, hcn_newton_params p) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    PathState s = {};
    s.last = p.max_eq_val;
    s.tol_res = p.tol_res;
    s.tol_dx = p.tol_dx;
    s.c_maxit = p.max_iter;
    s.c_active = p.max_iter > 0 ? 1 : 0;
    s.c_status = p.max_iter > 0 ? C_RUNNING : HCN_NOT_CONVERGED;
    st[b] = s;
}

__global__ void k_newton_finish(int B, const PathState *st, double *norms, int32_t *status,
                                int32_t *iters) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const PathState s = st[b];
    if (norms) {
        norms[2 * b] = s.res;
        norms[2 * b + 1] = s.dxn;
    }
    if (status) status[b] = s.c_status == C_RUNNING ? HCN_NOT_CONVERGED : s.c_status;
    if (iters) iters[b] = s.c_iter;
}

int launch_newton_init(int B, PathState *st, const hcn_newton_params &p, hipStream_t s) {
    if (B == 0) return 0;
    hipLaunchKernelGGL(k_newton_init, dim3((B + 255) / 256), dim3(256), 0, s, B, st, p);
    return (int)hipGetLastError();
}

int launch_newton_finish(int B, const PathState *st, double *norms, int32_t *status,
                         int32_t *iters, hipStream_t s) {
    if (B == 0) return 0;
    hipLaunchKernelGGL(k_newton_finish, dim3((B + 255) / 256), dim3(256), 0, s, B, st, norms,
                       status, iters);
    return (int)hipGetLastError();
}

template <class R>
__global__ void k_track_init(TrackArgs a, const double *x0) {
    constexpr int W = 2 * limbs<R>::P;
    const int b = blockIdx.x;
    const size_t off = (size_t)b * a.n * W;
    for (int q = threadIdx.x; q < a.n * W; q += blockDim.x) {
        a.x_acc[off + q] = x0[off + q];
        a.x[off + q] = x0[off + q];
    }
    if (threadIdx.x == 0) {
        PathState s = {};
        s.t_acc = 0.0;
        s.dt = a.max_dt;
        s.phase = PHASE_TRACK;
        s.status = HCN_OK;
        s.c_status = C_RUNNING;
        a.st[b] = s;
    }
}

template <class R>
__global__ void k_track_begin(TrackArgs a) {
    constexpr int W = 2 * limbs<R>::P;
    const int b = blockIdx.x;
    __shared__ int s_mode;  // 0 idle, 1 predict, 2 copy x_acc (refine start)
    __shared__ double s_t;
    PathState &st = a.st[b];
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
                a.t[b] = t;
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
                mode = 1;
            }
        } else if (st.phase == PHASE_REFINE && !st.refine_started) {
            st.refine_started = 1;
            st.t = 1.0;
            a.t[b] = 1.0;
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
    const size_t off = (size_t)b * a.n * W;
    if (mode == 2 || !st.have_prev || a.predictor_order < 1) {
        for (int q = threadIdx.x; q < a.n * W; q += blockDim.x) a.x[off + q] = a.x_acc[off + q];
        return;
    }
    // secant: x = x1 + r (x1 - x0), r = (t - t1) / (t1 - t0)
    const double t = s_t;
    const R num = rmake<R>(t - st.t_acc);
    const R den = rmake<R>(st.t_acc - st.t_prev);
    const R ratio = div(num, den);
    for (int i = threadIdx.x; i < a.n; i += blockDim.x) {
        const cx<R> x1 = cload<R>(a.x_acc + off + (size_t)i * W);
        const cx<R> xp = cload<R>(a.x_prev + off + (size_t)i * W);
        const cx<R> d = csub(x1, xp);
        cstore(a.x + off + (size_t)i * W, cadd(x1, cscale(ratio, d)));
    }
}

__device__ void write_result(const TrackArgs &a, int b, const PathState &st) {
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
    a.res[b] = r;
}

template <class R>
__global__ void k_track_end(TrackArgs a) {
    constexpr int W = 2 * limbs<R>::P;
    const int b = blockIdx.x;
    __shared__ int s_copy;  // 0 none, 1 accept (x_prev <- x_acc, x_acc <- x),
                            // 2 out <- x, 3 out <- x_acc
    PathState &st = a.st[b];
    if (threadIdx.x == 0) {
        int copy = 0;
        if (st.phase == PHASE_TRACK) {
            const int cs = st.c_status;
            st.newton_iters += st.c_iter;
            if (cs == HCN_OK) {
                st.t_prev = st.t_acc;
                st.have_prev = 1;
                st.t_acc = st.t;
                st.accepted += 1;
                st.nsucc += 1;
                if (st.nsucc > 2) {
                    double dt = 2.0 * st.dt;
                    st.dt = dt > a.max_dt ? a.max_dt : dt;
                }
                st.steps += 1;
                copy = 1;
                if (st.t_acc >= 1.0) {
                    if (a.end_iters > 0) {
                        st.phase = PHASE_REFINE;
                    } else {
                        st.phase = PHASE_DONE;
                        copy = 4;  // accept, then out <- x_acc
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
            // paths stopped by the step limit in k_track_begin end here
            if (copy == 0) copy = 3;
            write_result(a, b, st);
            st.finalized = 1;
        }
        s_copy = copy;
    }
    __syncthreads();
    const int copy = s_copy;
    if (copy == 0) return;
    const size_t off = (size_t)b * a.n * W;
    for (int q = threadIdx.x; q < a.n * W; q += blockDim.x) {
        if (copy == 1 || copy == 4) {
            const double xa = a.x_acc[off + q];
            a.x_prev[off + q] = xa;
            a.x_acc[off + q] = a.x[off + q];
            if (copy == 4) a.x_out[off + q] = a.x[off + q];
        } else if (copy == 2) {
            a.x_out[off + q] = a.x[off + q];
        } else {
            a.x_out[off + q] = a.x_acc[off + q];
        }
    }
}

__global__ void k_track_count(TrackArgs a) {
    __shared__ int red[256 / 64];
    int c = 0;
    for (int b = threadIdx.x; b < a.B; b += blockDim.x) c += a.st[b].phase != PHASE_DONE ? 1 : 0;
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        *a.active_count = s;
    }
}

int launch_track_init(const TrackArgs &a, const double *x0, hipStream_t s) {
    if (a.B == 0) return 0;
    if (a.P == 2)
        hipLaunchKernelGGL(k_track_init<dd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a, x0);
    else
        hipLaunchKernelGGL(k_track_init<qd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a, x0);
    return (int)hipGetLastError();
}

int launch_track_begin(const TrackArgs &a, hipStream_t s) {
    if (a.B == 0) return 0;
    if (a.P == 2)
        hipLaunchKernelGGL(k_track_begin<dd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL(k_track_begin<qd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a);
    return (int)hipGetLastError();
}

int launch_track_end(const TrackArgs &a, hipStream_t s) {
    if (a.B == 0) return 0;
    if (a.P == 2)
        hipLaunchKernelGGL(k_track_end<dd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL(k_track_end<qd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a);
    return (int)hipGetLastError();
}

int launch_track_count(const TrackArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_track_count, dim3(1), dim3(256), 0, s, a);
    return (int)hipGetLastError();
}

}  // namespace hcn
