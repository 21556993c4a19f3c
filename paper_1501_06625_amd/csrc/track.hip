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
#include "track_body.hpp"

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

HCN_DEV TrackPath path_of(const TrackArgs &a, int b) {
    const size_t off = (size_t)b * a.n * 2 * a.P;
    TrackPath p;
    p.n = a.n;
    p.st = a.st + b;
    p.x = a.x + off;
    p.x_acc = a.x_acc + off;
    p.x_prev = a.x_prev + off;
    p.old_stride = (long)a.n * 2 * a.P;
    p.x_old = a.x_old ? a.x_old + (size_t)(MAX_PREDICTOR_ORDER - 1) * off : nullptr;
    p.x_out = a.x_out + off;
    p.t = a.t + b;
    p.res = a.res + b;
    return p;
}

template <class R>
__global__ void k_track_init(TrackArgs a, const double *x0) {
    track_init_one<R>(a, path_of(a, blockIdx.x), x0 + (size_t)blockIdx.x * a.n * 2 * a.P);
}

template <class R>
__global__ void k_track_begin(TrackArgs a) {
    track_begin_one<R>(a, path_of(a, blockIdx.x));
}

template <class R>
__global__ void k_track_end(TrackArgs a) {
    track_end_one<R>(a, path_of(a, blockIdx.x));
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
    if (a.P == 1)
        hipLaunchKernelGGL(k_track_init<double>, dim3(a.B), dim3(TRK_THREADS), 0, s, a, x0);
    else if (a.P == 2)
        hipLaunchKernelGGL(k_track_init<dd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a, x0);
    else
        hipLaunchKernelGGL(k_track_init<qd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a, x0);
    return (int)hipGetLastError();
}

int launch_track_begin(const TrackArgs &a, hipStream_t s) {
    if (a.B == 0) return 0;
    if (a.P == 1)
        hipLaunchKernelGGL(k_track_begin<double>, dim3(a.B), dim3(TRK_THREADS), 0, s, a);
    else if (a.P == 2)
        hipLaunchKernelGGL(k_track_begin<dd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL(k_track_begin<qd>, dim3(a.B), dim3(TRK_THREADS), 0, s, a);
    return (int)hipGetLastError();
}

int launch_track_end(const TrackArgs &a, hipStream_t s) {
    if (a.B == 0) return 0;
    if (a.P == 1)
        hipLaunchKernelGGL(k_track_end<double>, dim3(a.B), dim3(TRK_THREADS), 0, s, a);
    else if (a.P == 2)
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
