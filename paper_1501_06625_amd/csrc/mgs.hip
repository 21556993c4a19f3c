// mgs.hip -- modified Gram-Schmidt solve, one workgroup of 256 lanes per
// problem (mgs_wg / mgs_reg in mgs_common.hpp), with the lane-group width
// and the storage of [A | b] (global memory, LDS, registers) chosen by the
// tuner (hcn_tune).
#include "internal.hpp"
#include "mgs_common.hpp"
#include "mp.hpp"
#include "prof.hpp"

namespace hcn {

// LDS: [A | b] staged in LDS (1) or left in global memory (0)
template <class R, int GRP, int LDS>
__global__ __launch_bounds__(MGS_THREADS) void k_mgs(MgsArgs a) {
    MgsProblem p = problem_of(a, blockIdx.x);
    p.lds = LDS;
    mgs_wg<R, GRP, LDS>(p);
}

template <class R, int GRP, int RPL, int CPG>
__global__ __launch_bounds__(MGS_THREADS) void k_mgs_reg(MgsArgs a) {
    mgs_reg<R, GRP, RPL, CPG>(problem_of(a, blockIdx.x));
}

template <class R, int GRP>
static bool launch_reg(const MgsArgs &a, hipStream_t stream) {
    int rpl = 0, cpg = 0;
    mgs_reg_shape(a.N, a.n, limbs<R>::P, GRP, &rpl, &cpg);
    const dim3 grid(a.B), block(MGS_THREADS);
    switch (rpl * 8 + cpg) {
        case 9: hipLaunchKernelGGL((k_mgs_reg<R, GRP, 1, 1>), grid, block, 0, stream, a); return true;
        case 17: hipLaunchKernelGGL((k_mgs_reg<R, GRP, 2, 1>), grid, block, 0, stream, a); return true;
        case 33: hipLaunchKernelGGL((k_mgs_reg<R, GRP, 4, 1>), grid, block, 0, stream, a); return true;
        default: break;
    }
    // QD columns beyond one per group spill to the stack
    if constexpr (limbs<R>::P != 4) {
        switch (rpl * 8 + cpg) {
            case 10: hipLaunchKernelGGL((k_mgs_reg<R, GRP, 1, 2>), grid, block, 0, stream, a); return true;
            case 12: hipLaunchKernelGGL((k_mgs_reg<R, GRP, 1, 4>), grid, block, 0, stream, a); return true;
            case 18: hipLaunchKernelGGL((k_mgs_reg<R, GRP, 2, 2>), grid, block, 0, stream, a); return true;
            case 20: hipLaunchKernelGGL((k_mgs_reg<R, GRP, 2, 4>), grid, block, 0, stream, a); return true;
            case 34: hipLaunchKernelGGL((k_mgs_reg<R, GRP, 4, 2>), grid, block, 0, stream, a); return true;
            default: break;
        }
    }
    return false;
}

template <class R, int GRP, int RPL>
__global__ __launch_bounds__(MGS_THREADS) void k_mgs_panel(MgsArgs a) {
    mgs_panel<R, GRP, RPL>(problem_of(a, blockIdx.x));
}

template <class R, int GRP>
static bool launch_panel(const MgsArgs &a, hipStream_t stream) {
    if constexpr (limbs<R>::P != 4) {
        const dim3 grid(a.B), block(MGS_THREADS);
        switch (mgs_panel_rpl(a.N, limbs<R>::P, GRP)) {
            case 1: hipLaunchKernelGGL((k_mgs_panel<R, GRP, 1>), grid, block, 0, stream, a); return true;
            case 2: hipLaunchKernelGGL((k_mgs_panel<R, GRP, 2>), grid, block, 0, stream, a); return true;
            case 4: hipLaunchKernelGGL((k_mgs_panel<R, GRP, 4>), grid, block, 0, stream, a); return true;
            case 8: hipLaunchKernelGGL((k_mgs_panel<R, GRP, 8>), grid, block, 0, stream, a); return true;
            case 16: hipLaunchKernelGGL((k_mgs_panel<R, GRP, 16>), grid, block, 0, stream, a); return true;
            default: break;
        }
    }
    return false;
}

template <class R, int GRP>
static void launch_grp(const MgsArgs &a, hipStream_t stream) {
    // storage of [A | b]: 0 global memory, 1 LDS (when it fits), 2 registers
    // (when they fit), 3 registers a panel of columns at a time (left-looking,
    // when a column fits); all give the same bits.  A few problems (latency
    // rather than throughput) always go to registers when they fit.
    const int mode = tune_mgs_lds(limbs<R>::P, a.N);
    if ((mode == 2 || a.B <= 64) && launch_reg<R, GRP>(a, stream)) return;
    if (mode == 3 && launch_panel<R, GRP>(a, stream)) return;
    const size_t bytes = mgs_lds_bytes(a.N, a.n, limbs<R>::P);
    const int lds = (bytes <= mgs_lds_limit() && mode == 1) ? 1 : 0;
    if (lds) {
        (void)hipFuncSetAttribute((const void *)k_mgs<R, GRP, 1>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        hipLaunchKernelGGL((k_mgs<R, GRP, 1>), dim3(a.B), dim3(MGS_THREADS), bytes, stream, a);
    } else {
        hipLaunchKernelGGL((k_mgs<R, GRP, 0>), dim3(a.B), dim3(MGS_THREADS), 0, stream, a);
    }
}

template <class R>
static void launch_t(const MgsArgs &a, int grp, hipStream_t stream) {
    switch (grp) {
        case 8: launch_grp<R, 8>(a, stream); break;
        case 32: launch_grp<R, 32>(a, stream); break;
        default: launch_grp<R, 16>(a, stream); break;
    }
}

int launch_mgs(int P, const MgsArgs &a, hipStream_t stream) {
    if (a.B == 0) return 0;
    ProfScope prof("mgs", stream);
    const int grp = tune_mgs_group(P, a.N);
    if (P == 1)
        launch_t<double>(a, grp, stream);
    else if (P == 2)
        launch_t<dd>(a, grp, stream);
    else
        launch_t<qd>(a, grp, stream);
    return (int)hipGetLastError();
}

}  // namespace hcn
