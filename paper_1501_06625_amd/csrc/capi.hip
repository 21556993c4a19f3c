// capi.hip -- host side of the C ABI declared in include/hcn.h: argument
// checks, system tables, workspace layout and the launch sequences of the
// evaluation, solve, Newton and tracking entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "prof.hpp"

using namespace hcn;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int dev_fail(int err, const char *where) {
    if (err == 0) return HCN_OK;
    return fail(HCN_EDEVICE, "%s: %s", where, hipGetErrorString((hipError_t)err));
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// carves consecutive 256-byte-aligned pieces out of one buffer
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <class T>
    T *take(size_t count) {
        T *p = base ? (T *)(base + off) : nullptr;
        off += align_up(count * sizeof(T));
        return p;
    }
};

// workspace given by the caller, or allocated on the stream for this call
struct Workspace {
    void *ptr = nullptr;
    bool owned = false;
    hipStream_t stream = nullptr;
    int acquire(void *user, size_t user_bytes, size_t need, hipStream_t s) {
        stream = s;
        if (user) {
            if (user_bytes < need)
                return fail(HCN_EINVAL, "workspace too small: %zu bytes given, %zu needed",
                            user_bytes, need);
            ptr = user;
            return HCN_OK;
        }
        if (need == 0) return HCN_OK;
        hipError_t e = hipMallocAsync(&ptr, need, s);
        if (e != hipSuccess) return fail(HCN_ENOMEM, "workspace allocation of %zu bytes failed", need);
        owned = true;
        return HCN_OK;
    }
    ~Workspace() {
        if (owned && ptr) (void)hipFreeAsync(ptr, stream);
    }
};

int g_mgs_variant = 0;  // 0 auto, 1 workgroup per problem, 2 right-looking, 4 tiled, 5 pipelined

// integers of an MGS workspace: per problem a status word, counters, and
// the column flags of the pipelined variant
size_t mgs_ints(int B, int n) { return (size_t)2 * B + 1 + (size_t)B * (n + 1); }
size_t g_chunk_bytes = 0;  // 0: every launch covers the whole batch

// the MGS variant for B problems with n unknowns
int mgs_variant_for(int n, int B) {
    if (g_mgs_variant != 0) return g_mgs_variant;
    return (n >= 160 && B <= 4) ? 5 : 1;
}

int enqueue_mgs_variant(int P, const MgsArgs &a, int variant, int *ints, hipStream_t s) {
    if (variant == 1) return launch_mgs(P, a, s);
    return launch_mgs_big(P, a, variant, ints, s);
}

// choose and launch the MGS variant for B problems of size N x n
int enqueue_mgs(int P, const MgsArgs &a, int *ints, hipStream_t s) {
    return enqueue_mgs_variant(P, a, mgs_variant_for(a.n, a.B), ints, s);
}

// Points per chunk of the evaluation: the monomial scratch of one chunk
// takes about g_chunk_bytes, so that what the monomial launch writes is
// still in the last-level cache when the summation reads it (the solve runs
// over the whole batch, which it needs to fill the GPU).  A multiple of 64,
// at least 64, at most B.
int chunk_points(const SysView &v, int B, int RP) {
    if (g_chunk_bytes == 0) return B;
    const size_t per = (size_t)v.nslots * 2 * (size_t)RP * sizeof(double);
    long c = (long)(g_chunk_bytes / std::max<size_t>(per, 1));
    c = std::max<long>(64, c / 64 * 64);
    return (int)std::min<long>(c, B);
}

// the same launch arguments restricted to points b0 .. b0 + Bc - 1
MonArgs chunk_of(MonArgs m, int b0, int Bc) {
    m.B = Bc;
    m.x += (size_t)b0 * m.x_pstride;
    m.scratch += (size_t)b0 * m.sc_pstride;
    if (m.st) m.st += b0;
    return m;
}

SumArgs chunk_of(SumArgs a, int b0, int Bc) {
    a.B = Bc;
    a.scratch += (size_t)b0 * a.sc_pstride;
    a.x += (size_t)b0 * a.x_pstride;
    if (a.hom.on) a.hom.t += b0;
    if (a.J) a.J += (size_t)b0 * a.J_pstride;
    if (a.f) a.f += (size_t)b0 * a.f_pstride;
    if (a.norm_part) a.norm_part += (size_t)b0 * sum_nparts(a.s, a.jac);
    if (a.st) a.st += b0;
    return a;
}

MgsArgs chunk_of(MgsArgs a, int b0, int Bc) {
    a.B = Bc;
    a.A += (size_t)b0 * a.A_pstride;
    if (a.bcol) a.bcol += (size_t)b0 * a.b_pstride;
    a.R += (size_t)b0 * a.R_pstride;
    a.inv += (size_t)b0 * a.inv_pstride;
    a.dx += (size_t)b0 * a.dx_pstride;
    if (a.status) a.status += b0;
    if (a.x) a.x += (size_t)b0 * a.x_pstride;
    if (a.norm_part) a.norm_part += (size_t)b0 * a.nparts;
    if (a.norms) a.norms += 2 * (size_t)b0;
    if (a.st) a.st += b0;
    return a;
}

}  // namespace

// A loaded system.  References: the caller's (from hcn_sys_load, given up
// by hcn_sys_free) and one per batch registry entry or queued serving
// request that names it; the device tables are freed with the last one.
struct hcn_sys_s {
    SysView v;
    void *dmem = nullptr;
    size_t bytes = 0;
    int nnz = 0;
    std::vector<int32_t> deg;
    std::atomic<int> refs{1};
};

SysView hcn::sys_view(hcn_sys s) { return s->v; }

void hcn::sys_retain(hcn_sys s) {
    if (s) s->refs.fetch_add(1);
}

void hcn::sys_release(hcn_sys s) {
    if (s && s->refs.fetch_sub(1) == 1) {
        (void)hipFree(s->dmem);
        delete s;
    }
}

extern "C" {

const char *hcn_last_error(void) { return g_err.c_str(); }

int hcn_version(void) { return 100; }

int hcn_sys_load(hcn_sys *out, int N, int n, int P, const int32_t *eq_ptr, const int32_t *mon_ptr,
                 const int32_t *var, const int32_t *exp, const double *coef) {
    if (!out) return fail(HCN_EINVAL, "hcn_sys_load: out is NULL");
    *out = nullptr;
    if (P != 1 && P != 2 && P != 4) return fail(HCN_EINVAL, "hcn_sys_load: P must be 1, 2 or 4, got %d", P);
    if (n < 1 || N < n || N > 4096)
        return fail(HCN_EINVAL, "hcn_sys_load: need 1 <= n <= N <= 4096 (N=%d n=%d)", N, n);
    if (!eq_ptr || !mon_ptr || !coef) return fail(HCN_EINVAL, "hcn_sys_load: NULL table");
    if (eq_ptr[0] != 0) return fail(HCN_EINVAL, "hcn_sys_load: eq_ptr[0] must be 0");
    for (int i = 0; i < N; ++i)
        if (eq_ptr[i + 1] < eq_ptr[i]) return fail(HCN_EINVAL, "hcn_sys_load: eq_ptr not monotone");
    const int nmon = eq_ptr[N];
    if (nmon < 1) return fail(HCN_EINVAL, "hcn_sys_load: no monomials");
    if (mon_ptr[0] != 0) return fail(HCN_EINVAL, "hcn_sys_load: mon_ptr[0] must be 0");
    int max_k = 0;
    for (int m = 0; m < nmon; ++m) {
        const int k = mon_ptr[m + 1] - mon_ptr[m];
        if (k < 0 || k > n)
            return fail(HCN_EINVAL, "hcn_sys_load: monomial %d has %d pairs (0..n allowed)", m, k);
        max_k = std::max(max_k, k);
    }
    const int npairs = mon_ptr[nmon];
    if (npairs > 0 && (!var || !exp)) return fail(HCN_EINVAL, "hcn_sys_load: NULL var/exp");
    {
        std::vector<int> seen(n, -1);
        for (int m = 0; m < nmon; ++m)
            for (int q = mon_ptr[m]; q < mon_ptr[m + 1]; ++q) {
                if (var[q] < 0 || var[q] >= n)
                    return fail(HCN_EINVAL, "hcn_sys_load: variable %d out of range", var[q]);
                if (exp[q] < 1 || exp[q] > 255)
                    return fail(HCN_EINVAL, "hcn_sys_load: exponent %d out of 1..255", exp[q]);
                if (seen[var[q]] == m)
                    return fail(HCN_EINVAL, "hcn_sys_load: variable %d repeated in monomial %d",
                                var[q], m);
                seen[var[q]] = m;
            }
    }
    const int W = 2 * P;

    // sort monomials by number of variables (stable)
    std::vector<int> perm(nmon), inv(nmon), eq_of(nmon);
    for (int i = 0; i < N; ++i)
        for (int m = eq_ptr[i]; m < eq_ptr[i + 1]; ++m) eq_of[m] = i;
    std::iota(perm.begin(), perm.end(), 0);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
        return (mon_ptr[a + 1] - mon_ptr[a]) < (mon_ptr[b + 1] - mon_ptr[b]);
    });
    for (int s = 0; s < nmon; ++s) inv[perm[s]] = s;

    std::vector<int32_t> h_k(nmon), h_slot(nmon), h_stride(nmon);
    long nslots = 0;
    for (int s = 0; s < nmon;) {
        const int k = mon_ptr[perm[s] + 1] - mon_ptr[perm[s]];
        int e = s;
        while (e < nmon && mon_ptr[perm[e] + 1] - mon_ptr[perm[e]] == k) ++e;
        const int Mg = e - s;
        for (int q = s; q < e; ++q) {
            h_k[q] = k;
            h_slot[q] = (int32_t)(nslots + (q - s));
            h_stride[q] = Mg;
        }
        nslots += (long)(k + 1) * Mg;
        s = e;
    }
    if (nslots > (1L << 30)) return fail(HCN_EINVAL, "hcn_sys_load: system too large");
    const int kk = std::max(max_k, 1);
    std::vector<uint16_t> h_pos((size_t)kk * nmon, 0);
    std::vector<uint8_t> h_ex((size_t)kk * nmon, 0);
    std::vector<double> h_coef((size_t)nmon * W);
    for (int s = 0; s < nmon; ++s) {
        const int m = perm[s];
        for (int p = 0; p < h_k[s]; ++p) {
            h_pos[(size_t)p * nmon + s] = (uint16_t)var[mon_ptr[m] + p];
            h_ex[(size_t)p * nmon + s] = (uint8_t)exp[mon_ptr[m] + p];
        }
        std::memcpy(&h_coef[(size_t)s * W], coef + (size_t)m * W, sizeof(double) * W);
    }
    // sums: value slots per equation, partial slots per dense Jacobian entry
    std::vector<int32_t> f_ptr(N + 1, 0), f_list(nmon);
    for (int i = 0; i < N; ++i) {
        f_ptr[i + 1] = eq_ptr[i + 1];
        for (int m = eq_ptr[i]; m < eq_ptr[i + 1]; ++m) f_list[m] = h_slot[inv[m]];
    }
    const long nJ = (long)n * N;
    std::vector<int32_t> J_ptr(nJ + 1, 0), J_list(std::max(npairs, 1));
    for (int m = 0; m < nmon; ++m)
        for (int q = mon_ptr[m]; q < mon_ptr[m + 1]; ++q) J_ptr[(long)var[q] * N + eq_of[m] + 1] += 1;
    for (long e = 0; e < nJ; ++e) J_ptr[e + 1] += J_ptr[e];
    int nnz = 0;
    for (long e = 0; e < nJ; ++e) nnz += J_ptr[e + 1] > J_ptr[e] ? 1 : 0;
    {
        std::vector<int32_t> fill(J_ptr.begin(), J_ptr.end() - 1);
        for (int i = 0; i < N; ++i)
            for (int m = eq_ptr[i]; m < eq_ptr[i + 1]; ++m) {
                const int s = inv[m];
                for (int p = 0; p < h_k[s]; ++p) {
                    const long e = (long)var[mon_ptr[m] + p] * N + i;
                    J_list[fill[e]++] = h_slot[s] + (p + 1) * h_stride[s];
                }
            }
    }
    // The summation takes the Jacobian entries equation-major: lane index
    // q = i n + k forms entry (k, i), whose list is that of e = k N + i.  The
    // partials of neighbouring monomials share cache lines (slots are
    // position-major within a size group) and belong, mostly, to one
    // equation, so their lines are read by lanes of one wavefront at nearly
    // the same list position.  The lists are interleaved per wavefront of 64
    // consecutive lanes (entry c of lane q at J_wbase[q / 64] + 64 c +
    // q % 64), so that the lanes read their c-th slot indices from one cache
    // line; the copy is dropped when the padding to each wavefront's longest
    // list would cost more than four times the lists.
    auto lane_entry = [&](long q) -> long { return (q % n) * N + q / n; };
    const long nwv = (nJ + 63) / 64;
    std::vector<int32_t> J_wbase(nwv + 1, 0), J_ilv;
    {
        long total = 0;
        for (long w = 0; w < nwv; ++w) {
            int mx = 0;
            for (long q = w * 64; q < std::min(nJ, (w + 1) * 64); ++q) {
                const long e = lane_entry(q);
                mx = std::max(mx, J_ptr[e + 1] - J_ptr[e]);
            }
            total += 64L * mx;
            if (total > (1L << 30)) break;
            J_wbase[w + 1] = (int32_t)total;
        }
        if (total <= 4L * std::max(npairs, 1) + 4096) {
            J_ilv.assign(std::max<long>(total, 1), 0);
            for (long q = 0; q < nJ; ++q) {
                const long e = lane_entry(q);
                for (int c = 0; c < J_ptr[e + 1] - J_ptr[e]; ++c)
                    J_ilv[J_wbase[q / 64] + 64L * c + q % 64] = J_list[J_ptr[e] + c];
            }
        }
    }
    std::vector<int32_t> deg(N, 0);
    for (int i = 0; i < N; ++i)
        for (int m = eq_ptr[i]; m < eq_ptr[i + 1]; ++m) {
            int d = 0;
            for (int q = mon_ptr[m]; q < mon_ptr[m + 1]; ++q) d += exp[q];
            deg[i] = std::max(deg[i], d);
        }

    // one device allocation for every table
    Carver c(nullptr);
    c.take<int32_t>(nmon);
    c.take<int32_t>(nmon);
    c.take<int32_t>(nmon);
    c.take<uint16_t>(h_pos.size());
    c.take<uint8_t>(h_ex.size());
    c.take<double>(h_coef.size());
    c.take<int32_t>(f_ptr.size());
    c.take<int32_t>(f_list.size());
    c.take<int32_t>(J_ptr.size());
    c.take<int32_t>(J_list.size());
    c.take<int32_t>(J_wbase.size());
    c.take<int32_t>(std::max<size_t>(J_ilv.size(), 1));
    c.take<int32_t>(deg.size());
    const size_t bytes = c.off;
    void *dmem = nullptr;
    if (hipMalloc(&dmem, bytes) != hipSuccess)
        return fail(HCN_ENOMEM, "hcn_sys_load: device allocation of %zu bytes failed", bytes);
    Carver d(dmem);
    auto up = [&](auto *dst, const auto &vec) {
        return hipMemcpy(dst, vec.data(), vec.size() * sizeof(vec[0]), hipMemcpyHostToDevice);
    };
    auto *d_k = d.take<int32_t>(nmon);
    auto *d_slot = d.take<int32_t>(nmon);
    auto *d_stride = d.take<int32_t>(nmon);
    auto *d_pos = d.take<uint16_t>(h_pos.size());
    auto *d_ex = d.take<uint8_t>(h_ex.size());
    auto *d_coef = d.take<double>(h_coef.size());
    auto *d_fptr = d.take<int32_t>(f_ptr.size());
    auto *d_flist = d.take<int32_t>(f_list.size());
    auto *d_Jptr = d.take<int32_t>(J_ptr.size());
    auto *d_Jlist = d.take<int32_t>(J_list.size());
    auto *d_Jwbase = d.take<int32_t>(J_wbase.size());
    auto *d_Jilv = d.take<int32_t>(std::max<size_t>(J_ilv.size(), 1));
    auto *d_deg = d.take<int32_t>(deg.size());
    hipError_t e = hipSuccess;
    e = e ? e : up(d_k, h_k);
    e = e ? e : up(d_slot, h_slot);
    e = e ? e : up(d_stride, h_stride);
    e = e ? e : up(d_pos, h_pos);
    e = e ? e : up(d_ex, h_ex);
    e = e ? e : up(d_coef, h_coef);
    e = e ? e : up(d_fptr, f_ptr);
    e = e ? e : up(d_flist, f_list);
    e = e ? e : up(d_Jptr, J_ptr);
    e = e ? e : up(d_Jlist, J_list);
    e = e ? e : up(d_Jwbase, J_wbase);
    if (!J_ilv.empty()) e = e ? e : up(d_Jilv, J_ilv);
    e = e ? e : up(d_deg, deg);
    if (e != hipSuccess) {
        (void)hipFree(dmem);
        return dev_fail(e, "hcn_sys_load: upload");
    }
    auto *sys = new hcn_sys_s;
    sys->dmem = dmem;
    sys->bytes = bytes;
    sys->nnz = nnz;
    sys->deg = deg;
    SysView &v = sys->v;
    v.N = N;
    v.n = n;
    v.P = P;
    v.nmon = nmon;
    v.max_k = max_k;
    v.max_e = 1;
    for (int q = 0; q < npairs; ++q) v.max_e = std::max(v.max_e, (int)exp[q]);
    v.nslots = (int)nslots;
    v.mon_k = d_k;
    v.mon_slot = d_slot;
    v.mon_stride = d_stride;
    v.pos = d_pos;
    v.ex = d_ex;
    v.coef = d_coef;
    v.f_ptr = d_fptr;
    v.f_list = d_flist;
    v.J_ptr = d_Jptr;
    v.J_list = d_Jlist;
    v.J_wbase = d_Jwbase;
    v.J_ilv = J_ilv.empty() ? nullptr : d_Jilv;
    v.deg = d_deg;
    *out = sys;
    return HCN_OK;
}

int hcn_sys_free(hcn_sys sys) {
    sys_release(sys);
    return HCN_OK;
}

int hcn_sys_info(hcn_sys sys, hcn_sys_info_t *info) {
    if (!sys || !info) return fail(HCN_EINVAL, "hcn_sys_info: NULL argument");
    info->N = sys->v.N;
    info->n = sys->v.n;
    info->P = sys->v.P;
    info->nmon = sys->v.nmon;
    info->max_k = sys->v.max_k;
    info->nslots = sys->v.nslots;
    info->nnz_jac = sys->nnz;
    info->device_bytes = sys->bytes;
    return HCN_OK;
}

int hcn_sys_degrees(hcn_sys sys, int32_t *degrees) {
    if (!sys || !degrees) return fail(HCN_EINVAL, "hcn_sys_degrees: NULL argument");
    std::memcpy(degrees, sys->deg.data(), sizeof(int32_t) * sys->deg.size());
    return HCN_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// workspace layouts
// ---------------------------------------------------------------------------

namespace {

struct EvalWs {
    double *scratch;
    double *norm_part;
};

template <class C>
EvalWs carve_eval(C &c, const SysView &v, int B) {
    EvalWs w;
    w.scratch = c.template take<double>((size_t)B * v.nslots * 2 * v.P);
    w.norm_part = c.template take<double>((size_t)B * sum_nparts(v, 1));
    return w;
}

struct NewtonWs {
    EvalWs ev;
    double *Jaug, *R, *inv, *dx;
    PathState *st;
    int *ints;
};

template <class C>
NewtonWs carve_newton(C &c, const SysView &v, int B) {
    NewtonWs w;
    const size_t W = 2 * v.P;
    w.ev = carve_eval(c, v, B);
    w.Jaug = c.template take<double>((size_t)B * (v.n + 1) * v.N * W);
    w.R = c.template take<double>((size_t)B * (v.n + 1) * v.n * W);
    w.inv = c.template take<double>((size_t)B * v.n * v.P);
    w.dx = c.template take<double>((size_t)B * v.n * W);
    w.st = c.template take<PathState>((size_t)B);
    w.ints = c.template take<int>(mgs_ints(B, v.n));
    return w;
}

struct TrackWs {
    NewtonWs nw;
    double *x, *x_acc, *x_prev, *x_old, *t;
    int32_t *count;
};

template <class C>
TrackWs carve_track(C &c, const SysView &v, int B) {
    TrackWs w;
    const size_t W = 2 * v.P;
    w.nw = carve_newton(c, v, B);
    w.x = c.template take<double>((size_t)B * v.n * W);
    w.x_acc = c.template take<double>((size_t)B * v.n * W);
    w.x_prev = c.template take<double>((size_t)B * v.n * W);
    w.x_old = c.template take<double>((size_t)B * (MAX_PREDICTOR_ORDER - 1) * v.n * W);
    w.t = c.template take<double>((size_t)B);
    w.count = c.template take<int32_t>(1);
    return w;
}

MonArgs mon_args(const SysView &v, int B, const double *x, double *scratch, int RP,
                 const PathState *st, int values_only) {
    MonArgs m = {};
    m.s = v;
    m.B = B;
    m.x = x;
    m.x_pstride = (long)v.n * 2 * v.P;
    m.xP = v.P;
    m.scratch = scratch;
    m.sc_pstride = (long)v.nslots * 2 * RP;
    m.st = st;
    m.values_only = values_only;
    return m;
}

SumArgs sum_args(const SysView &v, int B, const double *scratch, int RP, const double *x,
                 const Homotopy &hom, const PathState *st) {
    SumArgs a = {};
    a.s = v;
    a.B = B;
    a.scratch = scratch;
    a.sc_pstride = (long)v.nslots * 2 * RP;
    a.x = x;
    a.x_pstride = (long)v.n * 2 * v.P;
    a.xP = v.P;
    a.hom = hom;
    a.jac = 1;
    a.st = st;
    return a;
}

// evaluation of f (or h) and J into the augmented [J | -h] of the Newton
// workspace, with the residual norm parts
int enqueue_eval_aug(const SysView &v, int B, const double *x, const Homotopy &hom,
                     const NewtonWs &w, const PathState *st, hipStream_t s, int b0 = 0, int Bc = -1) {
    const long W = 2 * v.P;
    if (Bc < 0) Bc = B - b0;
    int e = launch_mon(v.P, chunk_of(mon_args(v, B, x, w.ev.scratch, v.P, st, 0), b0, Bc), s);
    if (e) return dev_fail(e, "evaluation launch");
    SumArgs a = sum_args(v, B, w.ev.scratch, v.P, x, hom, st);
    a.J = w.Jaug;
    a.J_cstride = v.N * W;
    a.J_pstride = (long)(v.n + 1) * v.N * W;
    a.f = w.Jaug + (size_t)v.n * v.N * W;
    a.f_pstride = (long)(v.n + 1) * v.N * W;
    a.f_neg = 1;
    a.norm_part = w.ev.norm_part;
    e = launch_sum(v.P, chunk_of(a, b0, Bc), s);
    if (e) return dev_fail(e, "summation launch");
    return HCN_OK;
}

// One Newton iteration over the batch (evaluation into [J | -h], then the
// solve), a chunk of points at a time; every point's arithmetic is the same
// whatever the chunk.
int enqueue_newton_iter(const SysView &v, int B, const double *x, const Homotopy &hom,
                        const NewtonWs &w, const PathState *st, const MgsArgs &a, hipStream_t s) {
    const int C = chunk_points(v, B, v.P);
    for (int b0 = 0; b0 < B; b0 += C) {
        const int rc = enqueue_eval_aug(v, B, x, hom, w, st, s, b0, std::min(C, B - b0));
        if (rc) return rc;
    }
    const int e = enqueue_mgs(v.P, a, w.ints, s);
    return e ? dev_fail(e, "solve launch") : HCN_OK;
}

MgsArgs newton_mgs_args(const SysView &v, int B, const NewtonWs &w, double *x, int mode) {
    const long W = 2 * v.P;
    MgsArgs a = {};
    a.B = B;
    a.N = v.N;
    a.n = v.n;
    a.mode = mode;
    a.A = w.Jaug;
    a.A_cstride = v.N * W;
    a.A_pstride = (long)(v.n + 1) * v.N * W;
    a.bcol = nullptr;
    a.R = w.R;
    a.R_pstride = (long)(v.n + 1) * v.n * W;
    a.inv = w.inv;
    a.inv_pstride = (long)v.n * v.P;
    a.dx = w.dx;
    a.dx_pstride = v.n * W;
    a.x = x;
    a.x_pstride = v.n * W;
    a.norm_part = w.ev.norm_part;
    a.nparts = sum_nparts(v, 1);
    a.st = w.st;
    return a;
}

int make_homotopy(const SysView &v, const double *gamma, int relax_k, const double *t,
                  Homotopy &hom) {
    std::memset(&hom, 0, sizeof hom);
    if (!gamma) return HCN_OK;
    if (v.N != v.n) return fail(HCN_EINVAL, "homotopy with the total-degree start system needs N == n");
    if (relax_k < 1) return fail(HCN_EINVAL, "relaxation exponent k must be >= 1");
    if (!t) return fail(HCN_EINVAL, "homotopy needs a device array of t values");
    hom.on = 1;
    hom.relax_k = relax_k;
    hom.gP = v.P;
    std::memcpy(hom.gamma, gamma, sizeof(double) * 2 * v.P);
    hom.t = t;
    return HCN_OK;
}

}  // namespace

extern "C" {

size_t hcn_eval_ws_bytes(hcn_sys sys, int B) {
    if (!sys || B < 0) return 0;
    Carver c(nullptr);
    carve_eval(c, sys->v, B);
    return c.off;
}

int hcn_eval_jac(hcn_sys sys, int B, const double *x, double *f, double *J, void *ws,
                 size_t ws_bytes, void *stream) {
    if (!sys) return fail(HCN_EINVAL, "hcn_eval_jac: NULL system");
    if (B < 0) return fail(HCN_EINVAL, "hcn_eval_jac: negative batch");
    if (B == 0) return HCN_OK;
    if (!x || !f) return fail(HCN_EINVAL, "hcn_eval_jac: NULL x or f");
    const SysView &v = sys->v;
    hipStream_t s = (hipStream_t)stream;
    Workspace wsp;
    int rc = wsp.acquire(ws, ws_bytes, hcn_eval_ws_bytes(sys, B), s);
    if (rc) return rc;
    Carver c(wsp.ptr);
    EvalWs w = carve_eval(c, v, B);
    const long W = 2 * v.P;
    int e = launch_mon(v.P, mon_args(v, B, x, w.scratch, v.P, nullptr, J ? 0 : 1), s);
    if (e) return dev_fail(e, "hcn_eval_jac: evaluation launch");
    Homotopy hom;
    std::memset(&hom, 0, sizeof hom);
    SumArgs a = sum_args(v, B, w.scratch, v.P, x, hom, nullptr);
    a.jac = J ? 1 : 0;
    a.J = J;
    a.J_cstride = v.N * W;
    a.J_pstride = (long)v.n * v.N * W;
    a.f = f;
    a.f_pstride = v.N * W;
    e = launch_sum(v.P, a, s);
    if (e) return dev_fail(e, "hcn_eval_jac: summation launch");
    return HCN_OK;
}

size_t hcn_mgs_ws_bytes(int B, int N, int n, int P) {
    if (B < 0 || n < 1 || (P != 1 && P != 2 && P != 4)) return 0;
    Carver c(nullptr);
    c.take<double>((size_t)B * (n + 1) * n * 2 * P);
    c.take<double>((size_t)B * n * P);
    c.take<int>(mgs_ints(B, n));
    return c.off;
}

int hcn_mgs_solve(int B, int N, int n, int P, double *A, double *b, double *dx, double *R,
                  int32_t *status, void *ws, size_t ws_bytes, void *stream) {
    if (P != 1 && P != 2 && P != 4) return fail(HCN_EINVAL, "hcn_mgs_solve: P must be 1, 2 or 4");
    if (n < 1 || N < n || N > 4096)
        return fail(HCN_EINVAL, "hcn_mgs_solve: need 1 <= n <= N <= 4096 (N=%d n=%d)", N, n);
    if (B < 0) return fail(HCN_EINVAL, "hcn_mgs_solve: negative batch");
    if (B == 0) return HCN_OK;
    if (!A || !b || !dx) return fail(HCN_EINVAL, "hcn_mgs_solve: NULL A, b or dx");
    hipStream_t s = (hipStream_t)stream;
    Workspace wsp;
    int rc = wsp.acquire(ws, ws_bytes, hcn_mgs_ws_bytes(B, N, n, P), s);
    if (rc) return rc;
    Carver c(wsp.ptr);
    double *Rw = c.take<double>((size_t)B * (n + 1) * n * 2 * P);
    double *inv = c.take<double>((size_t)B * n * P);
    int *ints = c.take<int>(mgs_ints(B, n));
    const long W = 2 * P;
    MgsArgs a = {};
    a.B = B;
    a.N = N;
    a.n = n;
    a.mode = MGS_SOLVE;
    a.A = A;
    a.A_cstride = N * W;
    a.A_pstride = (long)n * N * W;
    a.bcol = b;
    a.b_pstride = N * W;
    a.R = R ? R : Rw;
    a.R_pstride = (long)(n + 1) * n * W;
    a.inv = inv;
    a.inv_pstride = (long)n * P;
    a.dx = dx;
    a.dx_pstride = n * W;
    a.status = status;
    return dev_fail(enqueue_mgs(P, a, ints, s), "hcn_mgs_solve: launch");
}

size_t hcn_newton_ws_bytes(hcn_sys sys, int B) {
    if (!sys || B < 0) return 0;
    Carver c(nullptr);
    carve_newton(c, sys->v, B);
    return c.off;
}

int hcn_newton_step(hcn_sys sys, const double *gamma, int relax_k, int B, const double *t,
                    double *x, double *norms, int32_t *status, void *ws, size_t ws_bytes,
                    void *stream) {
    if (!sys) return fail(HCN_EINVAL, "hcn_newton_step: NULL system");
    if (B < 0) return fail(HCN_EINVAL, "hcn_newton_step: negative batch");
    if (B == 0) return HCN_OK;
    if (!x) return fail(HCN_EINVAL, "hcn_newton_step: NULL x");
    const SysView &v = sys->v;
    Homotopy hom;
    int rc = make_homotopy(v, gamma, relax_k, t, hom);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Workspace wsp;
    rc = wsp.acquire(ws, ws_bytes, hcn_newton_ws_bytes(sys, B), s);
    if (rc) return rc;
    Carver c(wsp.ptr);
    NewtonWs w = carve_newton(c, v, B);
    MgsArgs a = newton_mgs_args(v, B, w, x, MGS_NEWTON_STEP);
    a.norms = norms;
    a.status = status;
    return enqueue_newton_iter(v, B, x, hom, w, nullptr, a, s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// hcn_newton_step_static: hcn_newton_step on a fixed device workspace
// ---------------------------------------------------------------------------

// The workspace of hcn_newton_step_static, a device array of the library's
// code object: every GPU the library runs on holds its own copy, at its own
// address, until the process ends.  In host code its name is a host-side
// stand-in, never a device address; kernels receive the address that
// hipGetSymbolAddress returns for the device (static_ws below).
static __device__ __align__(256) char scratch[HCN_STATIC_WS_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ws[MAX_DEVICES];  // per device, set once

// the device the stream's work runs on (the current one for the null stream)
int stream_device(hipStream_t s, int *dev) {
    if (s) {
        if (hipStreamGetDevice(s, dev) != hipSuccess)
            return fail(HCN_EDEVICE, "hcn_newton_step_static: stream without a device");
    } else if (hipGetDevice(dev) != hipSuccess) {
        return fail(HCN_EDEVICE, "hcn_newton_step_static: no current device");
    }
    if (*dev < 0 || *dev >= MAX_DEVICES)
        return fail(HCN_EDEVICE, "hcn_newton_step_static: device %d beyond the table", *dev);
    return HCN_OK;
}

// address of the device's copy of `scratch`: looked up on the first call on
// that device, with that device current, and kept
int static_ws(hipStream_t s, void **out) {
    int dev = -1;
    int rc = stream_device(s, &dev);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ws[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess)
            return fail(HCN_EDEVICE, "hcn_newton_step_static: no current device");
        if (cur != dev && hipSetDevice(dev) != hipSuccess)
            return fail(HCN_EDEVICE, "hcn_newton_step_static: cannot select device %d", dev);
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !p)
            return fail(HCN_EDEVICE, "hcn_newton_step_static: workspace address on device %d: %s",
                        dev, hipGetErrorString(e));
        g_static_ws[dev] = p;
    }
    *out = g_static_ws[dev];
    return HCN_OK;
}

}  // namespace

extern "C" {

int hcn_newton_step_static(hcn_sys sys, const double *gamma, int relax_k, int B,
                           const double *t, double *x, double *norms, int32_t *status,
                           void *stream) {
    if (!sys) return fail(HCN_EINVAL, "hcn_newton_step_static: NULL system");
    if (B < 0) return fail(HCN_EINVAL, "hcn_newton_step_static: negative batch");
    const size_t need = hcn_newton_ws_bytes(sys, B);
    if (need > (size_t)HCN_STATIC_WS_BYTES)
        return fail(HCN_EINVAL,
                    "hcn_newton_step_static: %d points need %zu bytes of workspace, more than "
                    "the fixed %zu (use hcn_newton_step with a workspace of its own)",
                    B, need, (size_t)HCN_STATIC_WS_BYTES);
    if (B == 0) return HCN_OK;
    hipStream_t s = (hipStream_t)stream;
    void *ws = nullptr;
    const int rc = static_ws(s, &ws);
    if (rc) return rc;
    // the launches create no profiling events either
    ProfPause no_events;
    return hcn_newton_step(sys, gamma, relax_k, B, t, x, norms, status, ws,
                           (size_t)HCN_STATIC_WS_BYTES, stream);
}

int hcn_newton(hcn_sys sys, const double *gamma, int relax_k, int B, const double *t, double *x,
               const hcn_newton_params *prm, double *norms, int32_t *status, int32_t *iters,
               void *ws, size_t ws_bytes, void *stream) {
    if (!sys || !prm) return fail(HCN_EINVAL, "hcn_newton: NULL system or parameters");
    if (B < 0) return fail(HCN_EINVAL, "hcn_newton: negative batch");
    if (prm->max_iter < 0 || prm->max_iter > 1000)
        return fail(HCN_EINVAL, "hcn_newton: max_iter out of 0..1000");
    if (B == 0) return HCN_OK;
    if (!x) return fail(HCN_EINVAL, "hcn_newton: NULL x");
    const SysView &v = sys->v;
    Homotopy hom;
    int rc = make_homotopy(v, gamma, relax_k, t, hom);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Workspace wsp;
    rc = wsp.acquire(ws, ws_bytes, hcn_newton_ws_bytes(sys, B), s);
    if (rc) return rc;
    Carver c(wsp.ptr);
    NewtonWs w = carve_newton(c, v, B);
    int e = launch_newton_init(B, w.st, *prm, s);
    if (e) return dev_fail(e, "hcn_newton: init launch");
    const MgsArgs a = newton_mgs_args(v, B, w, x, MGS_NEWTON_FIG2);
    for (int it = 0; it < prm->max_iter; ++it) {
        rc = enqueue_newton_iter(v, B, x, hom, w, w.st, a, s);
        if (rc) return rc;
    }
    e = launch_newton_finish(B, w.st, norms, status, iters, s);
    return dev_fail(e, "hcn_newton: finish launch");
}

size_t hcn_track_ws_bytes(hcn_sys sys, int B) {
    if (!sys || B < 0) return 0;
    Carver c(nullptr);
    carve_track(c, sys->v, B);
    return c.off;
}

int hcn_track_paths(hcn_sys sys, const double *gamma, int relax_k, int B, const double *x0,
                    const hcn_track_params *prm, double *x_out, hcn_path_result *results,
                    void *ws, size_t ws_bytes, void *stream) {
    if (!sys || !prm || !gamma) return fail(HCN_EINVAL, "hcn_track_paths: NULL system, gamma or parameters");
    if (B < 0) return fail(HCN_EINVAL, "hcn_track_paths: negative batch");
    if (prm->max_iter < 1 || prm->max_iter > 100)
        return fail(HCN_EINVAL, "hcn_track_paths: max_iter out of 1..100");
    if (prm->max_steps < 0 || prm->end_iters < 0 || prm->end_iters > 1000)
        return fail(HCN_EINVAL, "hcn_track_paths: bad max_steps or end_iters");
    if (!(prm->max_dt > 0.0) || !(prm->min_dt > 0.0) || prm->max_dt > 1.0)
        return fail(HCN_EINVAL, "hcn_track_paths: need 0 < min_dt and 0 < max_dt <= 1");
    if (prm->predictor_order < 0 || prm->predictor_order > MAX_PREDICTOR_ORDER)
        return fail(HCN_EINVAL, "hcn_track_paths: predictor_order out of 0..%d", MAX_PREDICTOR_ORDER);
    if (B == 0) return HCN_OK;
    if (!x0 || !x_out || !results) return fail(HCN_EINVAL, "hcn_track_paths: NULL x0, x_out or results");
    const SysView &v = sys->v;
    hipStream_t s = (hipStream_t)stream;
    Workspace wsp;
    int rc = wsp.acquire(ws, ws_bytes, hcn_track_ws_bytes(sys, B), s);
    if (rc) return rc;
    Carver c(wsp.ptr);
    TrackWs w = carve_track(c, v, B);
    Homotopy hom;
    rc = make_homotopy(v, gamma, relax_k, w.t, hom);
    if (rc) return rc;
    TrackArgs ta = {};
    ta.B = B;
    ta.n = v.n;
    ta.P = v.P;
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
    ta.st = w.nw.st;
    ta.x = w.x;
    ta.x_acc = w.x_acc;
    ta.x_prev = w.x_prev;
    ta.x_old = w.x_old;
    ta.x_out = x_out;
    ta.t = w.t;
    ta.res = results;
    ta.active_count = w.count;
    int e = launch_track_init(ta, x0, s);
    if (e) return dev_fail(e, "hcn_track_paths: init launch");
    const MgsArgs a = newton_mgs_args(v, B, w.nw, w.x, MGS_NEWTON_FIG2);
    int32_t *host_count = nullptr;
    if (hipHostMalloc((void **)&host_count, sizeof(int32_t)) != hipSuccess)
        return fail(HCN_ENOMEM, "hcn_track_paths: pinned allocation failed");
    // every path ends within max_steps + 1 tracking steps plus the steps of
    // its refinement; the bound only guards against a logic error
    const long max_total = (long)prm->max_steps + 3 + (prm->end_iters + prm->max_iter - 1) / prm->max_iter + 2;
    const int chunk = 8;
    long done_steps = 0;
    rc = HCN_OK;
    while (done_steps < max_total) {
        for (int q = 0; q < chunk && rc == HCN_OK; ++q) {
            e = launch_track_begin(ta, s);
            if (e) { rc = dev_fail(e, "hcn_track_paths: begin launch"); break; }
            for (int it = 0; it < prm->max_iter && rc == HCN_OK; ++it)
                rc = enqueue_newton_iter(v, B, w.x, hom, w.nw, w.nw.st, a, s);
            if (rc) break;
            e = launch_track_end(ta, s);
            if (e) rc = dev_fail(e, "hcn_track_paths: end launch");
        }
        if (rc) break;
        done_steps += chunk;
        e = launch_track_count(ta, s);
        if (e) { rc = dev_fail(e, "hcn_track_paths: count launch"); break; }
        e = hipMemcpyAsync(host_count, w.count, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (!e) e = hipStreamSynchronize(s);
        if (e) { rc = dev_fail(e, "hcn_track_paths: poll"); break; }
        if (*host_count == 0) break;
    }
    if (rc == HCN_OK && *host_count != 0)
        rc = fail(HCN_EDEVICE, "hcn_track_paths: %d paths unfinished after %ld steps", *host_count,
                  done_steps);
    (void)hipHostFree(host_count);
    return rc;
}

}  // extern "C"

namespace {

struct MixedWs {
    double *sc_ext;    // values of the monomials in DD/QD
    double *np;        // residual norm parts
    double *sc64;      // values and partials in FP64
    double *J64;       // [B][n+1][N][2]: FP64 Jacobian and rounded -h
    double *R64, *inv64, *dx64;
    PathState *st;
    int *ints;
};

template <class C>
MixedWs carve_mixed(C &c, const SysView &v, int B) {
    MixedWs w;
    w.sc_ext = c.template take<double>((size_t)B * v.nslots * 2 * v.P);
    w.np = c.template take<double>((size_t)B * sum_nparts(v, 0));
    w.sc64 = c.template take<double>((size_t)B * v.nslots * 2);
    w.J64 = c.template take<double>((size_t)B * (v.n + 1) * v.N * 2);
    w.R64 = c.template take<double>((size_t)B * (v.n + 1) * v.n * 2);
    w.inv64 = c.template take<double>((size_t)B * v.n);
    w.dx64 = c.template take<double>((size_t)B * v.n * 2);
    w.st = c.template take<PathState>((size_t)B);
    w.ints = c.template take<int>(mgs_ints(B, v.n));
    return w;
}

}  // namespace

extern "C" {

size_t hcn_newton_mixed_ws_bytes(hcn_sys sys, int B) {
    if (!sys || B < 0) return 0;
    Carver c(nullptr);
    carve_mixed(c, sys->v, B);
    return c.off;
}

int hcn_newton_mixed(hcn_sys sys, const double *gamma, int relax_k, int B, const double *t,
                     double *x, const hcn_newton_params *prm, double *norms, int32_t *status,
                     int32_t *iters, void *ws, size_t ws_bytes, void *stream) {
    if (!sys || !prm) return fail(HCN_EINVAL, "hcn_newton_mixed: NULL system or parameters");
    if (B < 0) return fail(HCN_EINVAL, "hcn_newton_mixed: negative batch");
    if (prm->max_iter < 0 || prm->max_iter > 1000)
        return fail(HCN_EINVAL, "hcn_newton_mixed: max_iter out of 0..1000");
    if (sys->v.P == 1)
        return fail(HCN_EINVAL, "hcn_newton_mixed: the system is in double precision already");
    if (B == 0) return HCN_OK;
    if (!x) return fail(HCN_EINVAL, "hcn_newton_mixed: NULL x");
    const SysView &v = sys->v;
    Homotopy hom;
    int rc = make_homotopy(v, gamma, relax_k, t, hom);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Workspace wsp;
    rc = wsp.acquire(ws, ws_bytes, hcn_newton_mixed_ws_bytes(sys, B), s);
    if (rc) return rc;
    Carver c(wsp.ptr);
    MixedWs w = carve_mixed(c, v, B);
    int e = launch_newton_init(B, w.st, *prm, s);
    if (e) return dev_fail(e, "hcn_newton_mixed: init launch");
    const long colN = (long)v.N * 2;
    MgsArgs a = {};
    a.B = B;
    a.N = v.N;
    a.n = v.n;
    a.mode = MGS_MIXED_SOLVE;
    a.A = w.J64;
    a.A_cstride = colN;
    a.A_pstride = (long)(v.n + 1) * colN;
    a.R = w.R64;
    a.R_pstride = (long)(v.n + 1) * v.n * 2;
    a.inv = w.inv64;
    a.inv_pstride = v.n;
    a.dx = w.dx64;
    a.dx_pstride = (long)v.n * 2;
    a.x = x;
    a.x_pstride = (long)v.n * 2 * v.P;
    a.norm_part = w.np;
    a.nparts = sum_nparts(v, 0);
    a.st = w.st;
    SumArgs sr = sum_args(v, B, w.sc_ext, v.P, x, hom, w.st);
    sr.jac = 0;
    sr.f = w.J64 + (size_t)v.n * colN;
    sr.f_pstride = (long)(v.n + 1) * colN;
    sr.f_neg = 1;
    sr.f_lead_only = 1;
    sr.norm_part = w.np;
    SumArgs sj = sum_args(v, B, w.sc64, 1, x, hom, w.st);
    sj.J = w.J64;
    sj.J_cstride = colN;
    sj.J_pstride = (long)(v.n + 1) * colN;
    const MonArgs mr = mon_args(v, B, x, w.sc_ext, v.P, w.st, 1);
    const MonArgs mj = mon_args(v, B, x, w.sc64, 1, w.st, 0);
    const int Cr = chunk_points(v, B, v.P), Cj = chunk_points(v, B, 1);
    for (int it = 0; it < prm->max_iter; ++it) {
        // residual in extended precision; its rounding is the right-hand side
        for (int b0 = 0; b0 < B; b0 += Cr) {
            const int Bc = std::min(Cr, B - b0);
            e = launch_mon(v.P, chunk_of(mr, b0, Bc), s);
            if (e) return dev_fail(e, "hcn_newton_mixed: residual launch");
            e = launch_sum(v.P, chunk_of(sr, b0, Bc), s);
            if (e) return dev_fail(e, "hcn_newton_mixed: residual sum launch");
        }
        e = launch_fig2_pre(a, s);
        if (e) return dev_fail(e, "hcn_newton_mixed: test launch");
        // the Jacobian in FP64 at the leading limbs of x
        for (int b0 = 0; b0 < B; b0 += Cj) {
            const int Bc = std::min(Cj, B - b0);
            e = launch_mon(1, chunk_of(mj, b0, Bc), s);
            if (e) return dev_fail(e, "hcn_newton_mixed: Jacobian launch");
            e = launch_sum(1, chunk_of(sj, b0, Bc), s);
            if (e) return dev_fail(e, "hcn_newton_mixed: Jacobian sum launch");
        }
        e = enqueue_mgs(1, a, w.ints, s);
        if (e) return dev_fail(e, "hcn_newton_mixed: solve launch");
        e = launch_mixed_update(v.P, a, s);
        if (e) return dev_fail(e, "hcn_newton_mixed: update launch");
    }
    e = launch_newton_finish(B, w.st, norms, status, iters, s);
    return dev_fail(e, "hcn_newton_mixed: finish launch");
}

int hcn_set_mgs_variant(int variant) {
    if (variant < 0 || variant > 5 || variant == 3)
        return fail(HCN_EINVAL, "hcn_set_mgs_variant: 0, 1, 2, 4 or 5 (3 is not available)");
    g_mgs_variant = variant;
    return HCN_OK;
}

int hcn_set_mon_uniform(int on) {
    set_mon_uniform(on != 0);
    return HCN_OK;
}

int hcn_set_mon_tree(int on) {
    set_mon_tree(on != 0);
    return HCN_OK;
}

int hcn_set_chunk_bytes(size_t bytes) {
    g_chunk_bytes = bytes;
    return HCN_OK;
}

int hcn_set_mgs_panel(int T) {
    if (T < 1 || T > 16) return fail(HCN_EINVAL, "hcn_set_mgs_panel: 1..16");
    set_mgs_panel_width(T);
    return HCN_OK;
}

int hcn_set_mgs_wait_limit(long long polls) {
    if (polls < 0) return fail(HCN_EINVAL, "hcn_set_mgs_wait_limit: polls must be >= 0");
    set_mgs_wait_limit(polls);
    return HCN_OK;
}

int hcn_elementwise(int op, int P, int count, const double *a, const double *b, double *out,
                    void *stream) {
    if (P != 1 && P != 2 && P != 4) return fail(HCN_EINVAL, "hcn_elementwise: P must be 1, 2 or 4");
    static const int ops[] = {0, 1, 2, 3, 4, 5, 10, 11, 12, 13, 14, 15, 20, 21, 22};
    if (std::find(std::begin(ops), std::end(ops), op) == std::end(ops))
        return fail(HCN_EINVAL, "hcn_elementwise: unknown op %d", op);
    if (count < 0) return fail(HCN_EINVAL, "hcn_elementwise: negative count");
    if (count == 0) return HCN_OK;
    const bool needs_b = !(op == 4 || op == 14);
    if (!a || !out || (needs_b && !b)) return fail(HCN_EINVAL, "hcn_elementwise: NULL array");
    return dev_fail(launch_elementwise(op, P, count, a, b, out, (hipStream_t)stream),
                    "hcn_elementwise: launch");
}

}  // extern "C"
