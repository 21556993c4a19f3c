// tune.hip -- kernel-variant table and the autotuner.
//
// Choices: the lane-group width of the one-workgroup MGS (8, 16 or 32 lanes
// per column) and where [A | b] lives during the factorisation (0 global
// memory, 1 staged in LDS, 2 held in registers by the owning lane groups,
// 3 in registers a panel of columns at a time, left-looking), per precision
// and row count bucket.  hcn_autotune times a Newton step of a given system for every
// choice (HIP events on the caller's stream) and keeps the fastest, or [A | b]
// staged in LDS when that is within 5 % of it and fits the whole bucket; the
// table can be saved to and loaded from a text file (one line per entry:
// "P Nbucket group lds").  A choice depends only on (P, N), never on what
// else is in a batch, so a path gives the same bits alone and in a mix.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "mgs_common.hpp"

namespace hcn {
namespace {
struct Choice {
    int group = 16;
    int lds = 0;
};
std::mutex g_mu;
std::map<std::pair<int, int>, Choice> g_table;

int nbucket(int N) {
    int b = 8;
    while (b < N && b < 4096) b <<= 1;
    return b;
}

// untuned: 16 lanes per column; from 33 to 256 rows in DD and FP64 the
// left-looking panel form, which reads [A | b] once instead of the trailing
// matrix at every column step, with 32 lanes per column beyond 128 rows in
// DD (at most 8 rows per lane: 16 take every register of a lane) and beyond
// 64 rows in FP64 (the solve of the mixed-precision corrector)
Choice default_choice(int P, int N) {
    Choice c;
    if (P != 4 && N > 32 && N <= 256) {
        c.group = N > (P == 1 ? 64 : 128) ? 32 : 16;
        c.lds = 3;
    }
    return c;
}

Choice lookup(int P, int N) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find({P, nbucket(N)});
    return it == g_table.end() ? default_choice(P, N) : it->second;
}
}  // namespace

int tune_mgs_group(int P, int N) { return lookup(P, N).group; }

int tune_mgs_lds(int P, int N) { return lookup(P, N).lds; }

size_t mgs_lds_limit() { return 80 * 1024; }

void tune_set(int P, int N, int group, int lds) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[{P, nbucket(N)}] = Choice{group, lds};
}

}  // namespace hcn

using namespace hcn;

extern "C" {

int hcn_tune_set(int P, int N, int mgs_group, int mgs_lds) {
    if ((P != 1 && P != 2 && P != 4) || N < 1 ||
        (mgs_group != 8 && mgs_group != 16 && mgs_group != 32) || mgs_lds < 0 || mgs_lds > 3)
        return HCN_EINVAL;
    tune_set(P, N, mgs_group, mgs_lds);
    return HCN_OK;
}

int hcn_tune_get(int P, int N, int *mgs_group, int *mgs_lds) {
    if (!mgs_group || !mgs_lds) return HCN_EINVAL;
    *mgs_group = tune_mgs_group(P, N);
    *mgs_lds = tune_mgs_lds(P, N);
    return HCN_OK;
}

int hcn_tune_save(const char *path) {
    if (!path) return HCN_EINVAL;
    FILE *f = std::fopen(path, "w");
    if (!f) return HCN_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &kv : g_table)
        std::fprintf(f, "%d %d %d %d\n", kv.first.first, kv.first.second, kv.second.group,
                     kv.second.lds);
    std::fclose(f);
    return HCN_OK;
}

int hcn_tune_load(const char *path) {
    if (!path) return HCN_EINVAL;
    FILE *f = std::fopen(path, "r");
    if (!f) return HCN_EINVAL;
    int P, Nb, grp, lds, rc = HCN_OK;
    while (std::fscanf(f, "%d %d %d %d", &P, &Nb, &grp, &lds) == 4)
        if (hcn_tune_set(P, Nb, grp, lds) != HCN_OK) rc = HCN_EINVAL;
    std::fclose(f);
    return rc;
}

}  // extern "C"

extern "C" {

// Time hcn_newton_step of `sys` at the B points x_dev ([B][n][2][P], not
// modified) for every lane-group width and storage choice, and keep in the
// table for (P, N) the fastest, or LDS staging when it is within 5 % of the
// fastest and fits every row count of the bucket.  Outputs the choice and
// its time.
int hcn_autotune(hcn_sys sys, int B, const double *x_dev, int reps, int *best_group,
                 int *best_lds, double *best_ms, void *stream) {
    if (!sys || !x_dev || B < 1 || reps < 1) return HCN_EINVAL;
    hcn_sys_info_t info;
    if (hcn_sys_info(sys, &info) != HCN_OK) return HCN_EINVAL;
    const int P = info.P, N = info.N, n = info.n;
    hipStream_t s = (hipStream_t)stream;
    const size_t xbytes = (size_t)B * n * 2 * P * sizeof(double);
    const size_t wsb = hcn_newton_ws_bytes(sys, B);
    double *x = nullptr, *norms = nullptr;
    int32_t *status = nullptr;
    void *ws = nullptr;
    hipEvent_t e0, e1;
    if (hipMalloc((void **)&x, xbytes) != hipSuccess) return HCN_ENOMEM;
    if (hipMalloc((void **)&norms, 2 * B * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&status, B * sizeof(int32_t)) != hipSuccess ||
        hipMalloc(&ws, wsb) != hipSuccess) {
        (void)hipFree(x);
        (void)hipFree(norms);
        (void)hipFree(status);
        return HCN_ENOMEM;
    }
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    const int prev_group = tune_mgs_group(P, N), prev_lds = tune_mgs_lds(P, N);
    int bg = prev_group, bl = prev_lds, rc = HCN_OK;
    double bms = 1e300;
    struct Timed {
        int grp, lds;
        double ms;
    };
    std::vector<Timed> timed;
    const bool lds_fits = mgs_lds_bytes(N, n, P) <= mgs_lds_limit();
    for (int grp : {8, 16, 32}) {
        int rpl = 0, cpg = 0;
        mgs_reg_shape(N, n, P, grp, &rpl, &cpg);
        for (int lds = 0; lds <= 3; ++lds) {
            if ((lds == 1 && !lds_fits) || (lds == 2 && rpl == 0) ||
                (lds == 3 && mgs_panel_rpl(N, P, grp) == 0))
                continue;
            tune_set(P, N, grp, lds);
            float ms = 0.0f;
            for (int pass = 0; pass < 2 && rc == HCN_OK; ++pass) {  // warm-up, then timed
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < reps && rc == HCN_OK; ++r) {
                    (void)hipMemcpyAsync(x, x_dev, xbytes, hipMemcpyDeviceToDevice, s);
                    rc = hcn_newton_step(sys, nullptr, 1, B, nullptr, x, norms, status, ws, wsb, s);
                }
                (void)hipEventRecord(e1, s);
                if (hipEventSynchronize(e1) != hipSuccess) rc = HCN_EDEVICE;
                (void)hipEventElapsedTime(&ms, e0, e1);
            }
            if (rc) break;
            timed.push_back({grp, lds, ms / reps});
            bms = std::min(bms, (double)ms / reps);
        }
    }
    // among the choices within 5 % of the fastest (run-to-run noise of the
    // timings, and under 2 % of a Newton step for the solve), keep [A | b]
    // staged in LDS when that fits every row count of the bucket: the
    // global-memory form's in-place column updates reach HBM.  Otherwise
    // the fastest.
    {
        const int Nb = nbucket(N);
        const bool bucket_fits = mgs_lds_bytes(Nb, Nb, P) <= mgs_lds_limit();
        const Timed *fastest = nullptr, *staged = nullptr;
        for (const Timed &t : timed) {
            if (!fastest || t.ms < fastest->ms) fastest = &t;
            if (bucket_fits && t.lds == 1 && (!staged || t.ms < staged->ms)) staged = &t;
        }
        const Timed *pick = (staged && staged->ms <= 1.05 * bms) ? staged : fastest;
        if (pick) {
            bg = pick->grp;
            bl = pick->lds;
            bms = pick->ms;
        }
    }
    tune_set(P, N, rc ? prev_group : bg, rc ? prev_lds : bl);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(norms);
    (void)hipFree(status);
    (void)hipFree(ws);
    if (rc) return rc;
    if (best_group) *best_group = bg;
    if (best_lds) *best_lds = bl;
    if (best_ms) *best_ms = bms;
    return HCN_OK;
}

}  // extern "C"
