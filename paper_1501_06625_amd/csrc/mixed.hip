// mixed.hip -- the update of the mixed-precision Newton step: the Jacobian
// and its QR are formed in FP64, the residual and x stay in DD or QD, so the
// FP64 correction dx is added to x in extended precision and the iteration
// recovers full extended accuracy (the refinement converges while
// kappa(J) 2^-53 < 1).  One workgroup per problem: the update norm, the
// NaN check, x += dx, and the Fig. 2 tests that follow a solve.
#include "internal.hpp"
#include "mgs_common.hpp"
#include "mp.hpp"

namespace hcn {

template <class Rx>
__global__ __launch_bounds__(MGS_THREADS) void k_mixed_update(MgsArgs a) {
    constexpr int Wx = 2 * limbs<Rx>::P;
    __shared__ double s_red[MGS_THREADS / 64];
    const int b = blockIdx.x, tid = threadIdx.x, n = a.n;
    PathState &st = a.st[b];
    if (!st.c_active) return;
    const double *dxb = a.dx + (size_t)b * a.dx_pstride;  // [n][2] doubles
    double m = 0.0;
    for (int i = tid; i < n; i += MGS_THREADS) {
        const double re = dxb[2 * i], im = dxb[2 * i + 1];
        m = nanmax(m, nanmax(fabs(re), fabs(im)));
    }
    for (int off = 32; off >= 1; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
    if ((tid & 63) == 0) s_red[tid >> 6] = m;
    __syncthreads();
    double dxn = s_red[0];
    for (int w = 1; w < MGS_THREADS / 64; ++w) dxn = nanmax(dxn, s_red[w]);
    const bool isnan_dx = dxn != dxn;
    if (!isnan_dx) {
        double *xb = a.x + (size_t)b * a.x_pstride;
        for (int i = tid; i < n; i += MGS_THREADS) {
            double *p = xb + (size_t)i * Wx;
            const cx<double> d{dxb[2 * i], dxb[2 * i + 1]};
            cstore(p, cadd(cload<Rx>(p), cwiden<Rx>(d)));
        }
    }
    __syncthreads();
    if (tid == 0) fig2_after_update(st, dxn);
}

int launch_mixed_update(int xP, const MgsArgs &a, hipStream_t s) {
    if (a.B == 0) return 0;
    if (xP == 2)
        hipLaunchKernelGGL(k_mixed_update<dd>, dim3(a.B), dim3(MGS_THREADS), 0, s, a);
    else
        hipLaunchKernelGGL(k_mixed_update<qd>, dim3(a.B), dim3(MGS_THREADS), 0, s, a);
    return (int)hipGetLastError();
}

}  // namespace hcn
