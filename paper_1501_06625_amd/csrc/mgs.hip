// mgs.hip -- modified Gram-Schmidt solve, one workgroup of 256 lanes per
// problem (mgs_wg in mgs_common.hpp), with the lane-group width chosen by
// the tuner (hcn_tune) and [A | b] staged in LDS when it fits.
#include "internal.hpp"
#include "mgs_common.hpp"
#include "mp.hpp"
#include "prof.hpp"

namespace hcn {

template <class R, int GRP>
__global__ __launch_bounds__(MGS_THREADS) void k_mgs(MgsArgs a, int lds) {
    MgsProblem p = problem_of(a, blockIdx.x);
    p.lds = lds;
    mgs_wg<R, GRP>(p);
}

template <class R, int GRP>
static void launch_grp(const MgsArgs &a, hipStream_t stream) {
    const size_t bytes = mgs_lds_bytes(a.N, a.n, limbs<R>::P);
    const int lds = (bytes <= mgs_lds_limit() && tune_mgs_lds(limbs<R>::P, a.N)) ? 1 : 0;
    if (lds)
        (void)hipFuncSetAttribute((const void *)k_mgs<R, GRP>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    hipLaunchKernelGGL((k_mgs<R, GRP>), dim3(a.B), dim3(MGS_THREADS), lds ? bytes : 0, stream, a,
                       lds);
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
