// server.hip -- continuous batching of path-tracking requests.
//
// One slot-table batch per precision (DD, QD).  The number of slots of each
// batch is its share of a device-memory budget divided by the footprint of
// one slot (sized for the largest system the server accepts), so admission
// is by device-memory footprint: a request waits in its precision's FIFO
// queue until a slot is free.  Each scheduling round (hcn_server_pump)
//   1. harvests finished paths (result copied out, slot released),
//   2. admits queued requests into free slots (start point staged on the
//      device, path state initialised on the device),
//   3. advances every unfinished path by a fixed number of steps.
// Paths admitted while others are running join the same launches; each
// path's arithmetic is independent of the others, so its result is the
// same alone and in the mix.  Timestamps use a monotonic clock in seconds
// since the server was created (hcn_server_now).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

#include "internal.hpp"

namespace {

thread_local std::string g_serr;

int sfail(int code, const char *msg) {
    g_serr = msg;
    return code;
}

struct Request {
    int64_t id = 0;
    hcn_sys sys = nullptr;
    int P = 2, n = 0;
    double gamma[8] = {};
    std::vector<double> x0;
    double t_arrival = 0, t_admit = 0, t_done = 0;
    hcn_path_result res = {};
    std::vector<double> x_out;
};

struct Lane {
    int P = 2, cap = 0;
    hcn_batch batch = nullptr;
    double *stage = nullptr;  // [cap][max_n][2][P] start points on the device
    std::deque<Request *> queue;
    std::vector<Request *> slots;
    int running = 0;
};

}  // namespace

struct hcn_server_s {
    Lane lane[2];  // 0: DD, 1: QD
    int max_n = 0, steps_per_round = 4, serial = 0;
    hipStream_t stream = nullptr;
    std::chrono::steady_clock::time_point t0;
    std::deque<Request *> done;
    int64_t admitted = 0, completed = 0, rejected = 0;
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

extern "C" {

const char *hcn_server_last_error(void) { return g_serr.c_str(); }

int hcn_server_create(hcn_server *out, size_t budget_bytes, double qd_share, int max_n,
                      int max_nslots, const hcn_track_params *dd_prm, const hcn_track_params *qd_prm,
                      int steps_per_round, int serial) {
    if (!out || !dd_prm || !qd_prm) return sfail(HCN_EINVAL, "hcn_server_create: NULL argument");
    *out = nullptr;
    if (!(qd_share >= 0.0 && qd_share <= 1.0) || max_n < 1 || max_nslots < 1 || steps_per_round < 1)
        return sfail(HCN_EINVAL, "hcn_server_create: bad arguments");
    auto *s = new hcn_server_s;
    s->max_n = max_n;
    s->steps_per_round = steps_per_round;
    s->serial = serial ? 1 : 0;
    s->t0 = std::chrono::steady_clock::now();
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
        delete s;
        return sfail(HCN_EDEVICE, "hcn_server_create: stream");
    }
    const double share[2] = {1.0 - qd_share, qd_share};
    for (int l = 0; l < 2; ++l) {
        Lane &ln = s->lane[l];
        ln.P = l == 0 ? 2 : 4;
        // footprint of one slot: measured on a one-slot batch
        hcn_batch probe = nullptr;
        int rc = hcn_batch_create(&probe, ln.P, 1, max_n, max_nslots, 64, l == 0 ? dd_prm : qd_prm, 1, 0);
        if (rc) {
            hcn_server_destroy(s);
            return sfail(rc, hcn_batch_last_error());
        }
        const size_t per = hcn_batch_device_bytes(probe) + (size_t)max_n * 2 * ln.P * sizeof(double);
        hcn_batch_destroy(probe);
        long cap = s->serial ? 1 : (long)(share[l] * (double)budget_bytes / (double)per);
        if (share[l] > 0.0 && cap < 1) cap = 1;
        if (cap > 65536) cap = 65536;
        ln.cap = (int)cap;
        if (cap == 0) continue;
        rc = hcn_batch_create(&ln.batch, ln.P, ln.cap, max_n, max_nslots, 4096,
                              l == 0 ? dd_prm : qd_prm, 1, 0);
        if (rc) {
            hcn_server_destroy(s);
            return sfail(rc, hcn_batch_last_error());
        }
        if (hipMalloc((void **)&ln.stage, (size_t)ln.cap * max_n * 2 * ln.P * sizeof(double)) != hipSuccess) {
            hcn_server_destroy(s);
            return sfail(HCN_ENOMEM, "hcn_server_create: staging allocation");
        }
        ln.slots.assign(ln.cap, nullptr);
    }
    *out = s;
    return HCN_OK;
}

int hcn_server_destroy(hcn_server s) {
    if (!s) return HCN_OK;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto &ln : s->lane) {
        if (ln.batch) hcn_batch_destroy(ln.batch);
        if (ln.stage) (void)hipFree(ln.stage);
        for (auto *r : ln.queue) delete r;
        for (auto *r : ln.slots) delete r;
    }
    for (auto *r : s->done) delete r;
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return HCN_OK;
}

double hcn_server_now(hcn_server s) { return s ? s->now() : 0.0; }

int hcn_server_capacity(hcn_server s, int *dd_slots, int *qd_slots) {
    if (!s) return sfail(HCN_EINVAL, "hcn_server_capacity: NULL server");
    if (dd_slots) *dd_slots = s->lane[0].cap;
    if (qd_slots) *qd_slots = s->lane[1].cap;
    return HCN_OK;
}

// Queue a request: system (DD or QD, N == n <= max_n), gamma (host [2][P]),
// start solution x0 (host [n][2][P]), arrival time on the server clock.
int hcn_server_submit(hcn_server s, int64_t id, hcn_sys sys, const double *gamma,
                      const double *x0, double t_arrival) {
    if (!s || !sys || !gamma || !x0) return sfail(HCN_EINVAL, "hcn_server_submit: NULL argument");
    hcn_sys_info_t info;
    hcn_sys_info(sys, &info);
    const int l = info.P == 2 ? 0 : 1;
    if (info.N != info.n || info.n > s->max_n || s->lane[l].cap == 0) {
        ++s->rejected;
        return sfail(HCN_EINVAL, "hcn_server_submit: system does not fit the server");
    }
    auto *r = new Request;
    r->id = id;
    r->sys = sys;
    r->P = info.P;
    r->n = info.n;
    std::memcpy(r->gamma, gamma, sizeof(double) * 2 * info.P);
    r->x0.assign(x0, x0 + (size_t)info.n * 2 * info.P);
    r->t_arrival = t_arrival;
    s->lane[l].queue.push_back(r);
    return HCN_OK;
}

// One scheduling round; returns the number of paths in flight (>= 0).
int hcn_server_pump(hcn_server s) {
    if (!s) return sfail(HCN_EINVAL, "hcn_server_pump: NULL server");
    hipStream_t st = s->stream;
    int in_flight = 0;
    // 1. harvest finished paths
    for (auto &ln : s->lane) {
        if (!ln.batch || ln.running == 0) continue;
        std::vector<int32_t> done(ln.cap);
        const int run = hcn_batch_poll(ln.batch, done.data(), st);
        if (run < 0) return sfail(run, hcn_batch_last_error());
        const double t = s->now();
        for (int q = 0; q < ln.cap; ++q) {
            Request *r = ln.slots[q];
            if (!r || !done[q]) continue;
            r->x_out.resize((size_t)r->n * 2 * r->P);
            double *dx = ln.stage + (size_t)q * s->max_n * 2 * ln.P;
            int rc = hcn_batch_result(ln.batch, q, dx, &r->res, st);
            if (!rc && hipMemcpyAsync(r->x_out.data(), dx, sizeof(double) * r->x_out.size(),
                                      hipMemcpyDeviceToHost, st) != hipSuccess)
                rc = HCN_EDEVICE;
            if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = HCN_EDEVICE;
            if (rc) return sfail(HCN_EDEVICE, "hcn_server_pump: result copy failed");
            r->t_done = t;
            hcn_batch_release(ln.batch, q);
            ln.slots[q] = nullptr;
            --ln.running;
            ++s->completed;
            s->done.push_back(r);
        }
    }
    // 2. admit queued requests into free slots
    const bool busy = s->lane[0].running + s->lane[1].running > 0;
    for (auto &ln : s->lane) {
        if (!ln.batch) continue;
        for (int q = 0; q < ln.cap && !ln.queue.empty(); ++q) {
            if (ln.slots[q]) continue;
            if (s->serial && (busy || s->lane[0].running + s->lane[1].running > 0)) break;
            Request *r = ln.queue.front();
            ln.queue.pop_front();
            double *x0d = ln.stage + (size_t)q * s->max_n * 2 * ln.P;
            if (hipMemcpyAsync(x0d, r->x0.data(), sizeof(double) * r->x0.size(), hipMemcpyHostToDevice,
                               st) != hipSuccess)
                return sfail(HCN_EDEVICE, "hcn_server_pump: start point upload failed");
            const int rc = hcn_batch_add(ln.batch, q, r->sys, r->gamma, x0d, st);
            if (rc) return sfail(rc, hcn_batch_last_error());
            r->t_admit = s->now();
            ln.slots[q] = r;
            ++ln.running;
            ++s->admitted;
        }
    }
    // 3. advance every unfinished path
    for (auto &ln : s->lane) {
        if (!ln.batch || ln.running == 0) continue;
        const int rc = hcn_batch_step(ln.batch, s->steps_per_round, st);
        if (rc) return sfail(rc, hcn_batch_last_error());
        in_flight += ln.running;
    }
    return in_flight;
}

// Pop one completed request; returns 1 when one was available, 0 if none.
// x_out (host, [n][2][P] of the request's system) may be NULL; times on the
// server clock.
int hcn_server_fetch(hcn_server s, int64_t *id, double *x_out, hcn_path_result *res,
                     double *t_arrival, double *t_admit, double *t_done) {
    if (!s) return sfail(HCN_EINVAL, "hcn_server_fetch: NULL server");
    if (s->done.empty()) return 0;
    Request *r = s->done.front();
    s->done.pop_front();
    if (id) *id = r->id;
    if (x_out) std::memcpy(x_out, r->x_out.data(), sizeof(double) * r->x_out.size());
    if (res) *res = r->res;
    if (t_arrival) *t_arrival = r->t_arrival;
    if (t_admit) *t_admit = r->t_admit;
    if (t_done) *t_done = r->t_done;
    delete r;
    return 1;
}

// queued (not yet admitted) requests per precision
int hcn_server_queued(hcn_server s, int *dd, int *qd) {
    if (!s) return sfail(HCN_EINVAL, "hcn_server_queued: NULL server");
    if (dd) *dd = (int)s->lane[0].queue.size();
    if (qd) *qd = (int)s->lane[1].queue.size();
    return HCN_OK;
}

}  // extern "C"
