// eval.hip -- evaluation and differentiation of one polynomial system at a
// batch of points (Sections 3.2 and 3.3).
//
// k_mon: one lane per monomial, a wavefront per 64 monomials of (after the
// sort by number of variables) equal size k; reverse mode per lane
// (mon_one).  k_sum: one lane per output (sum_one), the residual max norm as
// per-block maxima.  The compute precision R (double, DD or QD) may be
// narrower than the storage of the coefficients and of x: loads take the
// leading limbs.
#include "eval_body.hpp"
#include "internal.hpp"
#include "mp.hpp"
#include "prof.hpp"

namespace hcn {

// UNI (mon_uniform): the workgroup first tabulates its point's powers in
// LDS when some exponent exceeds two (dynamic LDS, mon_stage_bytes).
template <class R, int KB, int MODE, bool UNI>
__global__ __launch_bounds__(256) void k_mon(MonArgs a) {
    extern __shared__ double pows[];
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const bool table = UNI && a.s.max_e > 2;
    for (int b = blockIdx.y; b < a.B; b += gridDim.y) {
        if (a.st && !a.st[b].c_active) continue;
        const double *xb = a.x + (size_t)b * a.x_pstride;
        if (table) {
            stage_pows<R>(a.s, xb, a.xP, pows);
            __syncthreads();
        }
        const PointView pv{xb, 2 * a.xP, a.xP, table ? pows : nullptr};
        if (m < a.s.nmon) {
            double *out = a.scratch + (size_t)b * a.sc_pstride;
            if constexpr (KB == 0)
                mon_one_long<R, MODE, UNI>(a.s, m, pv, out);
            else
                mon_one<R, KB, MODE, UNI>(a.s, m, pv, out);
        }
        if (table) __syncthreads();
    }
}

// tree mode: G lanes per monomial (mon_tree), 256 / G monomials per workgroup
template <class R, int G, bool UNI>
__global__ __launch_bounds__(256) void k_mon_tree(MonArgs a) {
    extern __shared__ double pows[];
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int m = gid / G < a.s.nmon ? (int)(gid / G) : -1;
    const int j = (int)(threadIdx.x % G);
    const bool table = UNI && a.s.max_e > 2;
    for (int b = blockIdx.y; b < a.B; b += gridDim.y) {
        if (a.st && !a.st[b].c_active) continue;
        const double *xb = a.x + (size_t)b * a.x_pstride;
        if (table) {
            stage_pows<R>(a.s, xb, a.xP, pows);
            __syncthreads();
        }
        const PointView pv{xb, 2 * a.xP, a.xP, table ? pows : nullptr};
        mon_tree<R, G, UNI>(a.s, m, j, pv, a.scratch + (size_t)b * a.sc_pstride);
        if (table) __syncthreads();
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_sum(SumArgs a) {
    __shared__ double red[256 / 64];
    // (part, point) from the XCD-aware logical id of the workgroup
    const int L = xcd_logical(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
    const int part = L % gridDim.x;
    const long e = (long)part * blockDim.x + threadIdx.x;
    for (int b = L / gridDim.x; b < a.B; b += gridDim.y) {
        if (a.st && !a.st[b].c_active) continue;
        SumOut o;
        o.jac = a.jac;
        o.J = a.J ? a.J + (size_t)b * a.J_pstride : nullptr;
        o.J_cstride = a.J_cstride;
        o.f = a.f ? a.f + (size_t)b * a.f_pstride : nullptr;
        o.f_neg = a.f_neg;
        o.f_lead_only = a.f_lead_only;
        const double t = a.hom.on ? a.hom.t[b] : 0.0;
        const double mx = sum_one<R>(a.s, e, a.scratch + (size_t)b * a.sc_pstride,
                                     a.x + (size_t)b * a.x_pstride, a.xP, a.hom.on, a.hom.relax_k,
                                     t, a.hom.gamma, a.hom.gP, o);
        if (a.norm_part) {
            const double r = block_max(mx, red);
            if (threadIdx.x == 0) a.norm_part[(size_t)b * gridDim.x + part] = r;
        }
    }
}

// the unrolled monomial forms cover up to 64 variables; 0: the loop form
static int kbucket(int max_k) {
    if (max_k <= 4) return 4;
    if (max_k <= 8) return 8;
    if (max_k <= 16) return 16;
    if (max_k <= 32) return 32;
    if (max_k <= 64) return 64;
    return 0;
}

static bool g_mon_uniform = true;
static bool g_mon_tree = false;

bool mon_uniform_enabled() { return g_mon_uniform; }
void set_mon_uniform(bool on) { g_mon_uniform = on; }
void set_mon_tree(bool on) { g_mon_tree = on; }

template <class R, int G>
static void mon_tree_g(const MonArgs &a, hipStream_t stream) {
    const long lanes = (long)a.s.nmon * G;
    const dim3 grid((unsigned)((lanes + 255) / 256), a.B < 65535 ? a.B : 65535);
    if (mon_uniform(a.s, limbs<R>::P))
        hipLaunchKernelGGL((k_mon_tree<R, G, true>), grid, dim3(256), mon_stage_bytes(a.s, limbs<R>::P),
                           stream, a);
    else
        hipLaunchKernelGGL((k_mon_tree<R, G, false>), grid, dim3(256), 0, stream, a);
}

// the tree form for the values and gradients of monomials of at most 64
// variables, when enabled; false when the reverse form should run
template <class R>
static bool launch_mon_tree(const MonArgs &a, hipStream_t stream) {
    if (!g_mon_tree || a.values_only || a.s.max_k > 64) return false;
    const int k = a.s.max_k;
    if (k <= 4) mon_tree_g<R, 4>(a, stream);
    else if (k <= 8) mon_tree_g<R, 8>(a, stream);
    else if (k <= 16) mon_tree_g<R, 16>(a, stream);
    else if (k <= 32) mon_tree_g<R, 32>(a, stream);
    else mon_tree_g<R, 64>(a, stream);
    return true;
}

template <class R, int KB, bool UNI>
static void mon_kb_u(const MonArgs &a, dim3 grid, size_t lds, hipStream_t stream) {
    // forward products in registers where they fit (DD up to 16, FP64 up to
    // 32 variables); QD and longer products park them in their output slots
    constexpr bool freg = KB > 0 && ((limbs<R>::P == 2 && KB <= 16) || (limbs<R>::P == 1 && KB <= 32));
    if (a.values_only) {
        hipLaunchKernelGGL((k_mon<R, KB, MON_VALUES, UNI>), grid, dim3(256), lds, stream, a);
    } else if constexpr (freg) {
        hipLaunchKernelGGL((k_mon<R, KB, MON_FREG, UNI>), grid, dim3(256), lds, stream, a);
    } else {
        hipLaunchKernelGGL((k_mon<R, KB, MON_FSLOT, UNI>), grid, dim3(256), lds, stream, a);
    }
}

template <class R, int KB>
static void mon_kb(const MonArgs &a, dim3 grid, hipStream_t stream) {
    if (mon_uniform(a.s, limbs<R>::P))
        mon_kb_u<R, KB, true>(a, grid, mon_stage_bytes(a.s, limbs<R>::P), stream);
    else
        mon_kb_u<R, KB, false>(a, grid, 0, stream);
}

template <class R>
static int launch_mon_t(const MonArgs &a, hipStream_t stream) {
    if (a.s.nmon == 0 || a.B == 0) return 0;
    dim3 grid((a.s.nmon + 255) / 256, a.B < 65535 ? a.B : 65535);
    ProfScope prof("eval_monomials", stream);
    if (launch_mon_tree<R>(a, stream)) return (int)hipGetLastError();
    switch (kbucket(a.s.max_k)) {
        case 4: mon_kb<R, 4>(a, grid, stream); break;
        case 8: mon_kb<R, 8>(a, grid, stream); break;
        case 16: mon_kb<R, 16>(a, grid, stream); break;
        case 32: mon_kb<R, 32>(a, grid, stream); break;
        case 64: mon_kb<R, 64>(a, grid, stream); break;
        default: mon_kb<R, 0>(a, grid, stream); break;
    }
    return (int)hipGetLastError();
}

int launch_mon(int RP, const MonArgs &a, hipStream_t stream) {
    switch (RP) {
        case 1: return launch_mon_t<double>(a, stream);
        case 2: return launch_mon_t<dd>(a, stream);
        default: return launch_mon_t<qd>(a, stream);
    }
}

int sum_nparts(const SysView &s, int jac) {
    const long E = (jac ? (long)s.n * s.N : 0) + s.N;
    return (int)((E + 255) / 256);
}

int launch_sum(int RP, const SumArgs &a, hipStream_t stream) {
    if (a.B == 0) return 0;
    dim3 grid(sum_nparts(a.s, a.jac), a.B < 65535 ? a.B : 65535);
    ProfScope prof("eval_sums", stream);
    switch (RP) {
        case 1: hipLaunchKernelGGL(k_sum<double>, grid, dim3(256), 0, stream, a); break;
        case 2: hipLaunchKernelGGL(k_sum<dd>, grid, dim3(256), 0, stream, a); break;
        default: hipLaunchKernelGGL(k_sum<qd>, grid, dim3(256), 0, stream, a); break;
    }
    return (int)hipGetLastError();
}

}  // namespace hcn
