// server.hip -- continuous batching of path-tracking requests.
//
// Lanes: one slot-table batch per precision (DD, QD) and size class of the
// system (n <= 24, 25..63, >= 64 unknowns), each on a stream of its own.
// The slot count of a lane is its share of a device-memory budget divided
// by the footprint of one slot sized for the largest system of its class,
// so admission is by device-memory footprint: a request waits in its lane's
// FIFO queue until a slot is free.  Lanes advance independently: a pump
// looks at every lane whose last round has finished on the device (an
// event query, no wait) and
//   1. harvests its finished paths (result copied out, slot released),
//   2. admits queued requests into its free slots (start point staged on
//      the device, path state initialised on the device),
//   3. launches its next round: a fixed number of steps of every unfinished
//      path in the lane,
// so small systems are not held back by the step time of large ones.
// Slots of systems with at least SPLIT_N unknowns solve with the tiled MGS
// across workgroups (lower latency per step).  Paths admitted while others
// are running join the same launches; each path's arithmetic depends only on
// its own system, point and lane settings, so its result is the same alone
// and in the mix.  Timestamps use a monotonic clock in seconds since the
// server was created (hcn_server_now).
#include <hip/hip_runtime.h>

#include <algorithm>
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

constexpr int NCLASS = 3;
constexpr int CLASS_HI[NCLASS] = {24, 63, 1 << 30};  // largest n of each size class
constexpr int SPLIT_N = 48;

int size_class(int n) {
    int c = 0;
    while (c < NCLASS - 1 && n > CLASS_HI[c]) ++c;
    return c;
}

// A request holds a reference on its system from submission until it is
// fetched or the server is destroyed.
struct Request {
    int64_t id = 0, seq = 0;
    hcn_sys sys = nullptr;
    int P = 2, n = 0;
    double gamma[8] = {};
    std::vector<double> x0;
    double t_arrival = 0, t_admit = 0, t_done = 0;
    hcn_path_result res = {};
    std::vector<double> x_out;
    ~Request() { hcn::sys_release(sys); }
};

struct Lane {
    int P = 2, max_n = 0, cap = 0;
    hcn_batch batch = nullptr;
    double *stage = nullptr;  // [cap][max_n][2][P] start points and results on the device
    std::deque<Request *> queue;
    std::vector<Request *> slots;
    std::vector<int32_t> done;
    int running = 0;
    bool inflight = false;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
};

}  // namespace

struct hcn_server_s {
    Lane lane[2][NCLASS];  // [DD, QD][size class]
    int max_n = 0, steps_per_round = 4, serial = 0;
    std::chrono::steady_clock::time_point t0;
    std::deque<Request *> done;
    int64_t seq = 0, admitted = 0, completed = 0, rejected = 0;
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// finished paths of an idle lane: results to the host, slots released
int harvest(hcn_server_s *s, Lane &ln) {
    if (ln.running == 0) return HCN_OK;
    const int run = hcn_batch_poll(ln.batch, ln.done.data(), ln.stream);
    if (run < 0) return sfail(run, hcn_batch_last_error());
    const double t = s->now();
    for (int q = 0; q < ln.cap; ++q) {
        Request *r = ln.slots[q];
        if (!r || !ln.done[q]) continue;
        r->x_out.resize((size_t)r->n * 2 * r->P);
        double *dx = ln.stage + (size_t)q * ln.max_n * 2 * ln.P;
        int rc = hcn_batch_result(ln.batch, q, dx, &r->res, ln.stream);
        if (!rc && hipMemcpyAsync(r->x_out.data(), dx, sizeof(double) * r->x_out.size(),
                                  hipMemcpyDeviceToHost, ln.stream) != hipSuccess)
            rc = HCN_EDEVICE;
        if (!rc && hipStreamSynchronize(ln.stream) != hipSuccess) rc = HCN_EDEVICE;
        if (rc) return sfail(HCN_EDEVICE, "hcn_server_pump: result copy failed");
        r->t_done = t;
        hcn_batch_release(ln.batch, q);
        ln.slots[q] = nullptr;
        --ln.running;
        ++s->completed;
        s->done.push_back(r);
    }
    return HCN_OK;
}

// the head of the lane's queue into a free slot; false when none is free
int admit_one(hcn_server_s *s, Lane &ln, bool *admitted) {
    *admitted = false;
    if (ln.queue.empty()) return HCN_OK;
    int q = 0;
    while (q < ln.cap && ln.slots[q]) ++q;
    if (q == ln.cap) return HCN_OK;
    // the request leaves the queue only once its slot is set up
    Request *r = ln.queue.front();
    double *x0d = ln.stage + (size_t)q * ln.max_n * 2 * ln.P;
    if (hipMemcpyAsync(x0d, r->x0.data(), sizeof(double) * r->x0.size(), hipMemcpyHostToDevice,
                       ln.stream) != hipSuccess)
        return sfail(HCN_EDEVICE, "hcn_server_pump: start point upload failed");
    const int rc = hcn_batch_add(ln.batch, q, r->sys, r->gamma, x0d, ln.stream);
    if (rc) return sfail(rc, hcn_batch_last_error());
    ln.queue.pop_front();
    r->t_admit = s->now();
    ln.slots[q] = r;
    ++ln.running;
    ++s->admitted;
    *admitted = true;
    return HCN_OK;
}

}  // namespace

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
    const int nclass = size_class(max_n) + 1;
    const double share[2] = {1.0 - qd_share, qd_share};
    for (int l = 0; l < 2; ++l) {
        for (int c = 0; c < nclass; ++c) {
            Lane &ln = s->lane[l][c];
            ln.P = l == 0 ? 2 : 4;
            ln.max_n = std::min(max_n, CLASS_HI[c]);
            // footprint of one slot: measured on a one-slot batch
            hcn_batch probe = nullptr;
            int rc = hcn_batch_create(&probe, ln.P, 1, ln.max_n, max_nslots, 64, l == 0 ? dd_prm : qd_prm,
                                      1, 0);
            if (rc) {
                hcn_server_destroy(s);
                return sfail(rc, hcn_batch_last_error());
            }
            const size_t per = hcn_batch_device_bytes(probe) + (size_t)ln.max_n * 2 * ln.P * sizeof(double);
            hcn_batch_destroy(probe);
            long cap = s->serial ? 1 : (long)(share[l] * (double)budget_bytes / nclass / (double)per);
            if (share[l] > 0.0 && cap < 1) cap = 1;
            if (cap > 65536) cap = 65536;
            ln.cap = (int)cap;
            if (cap == 0) continue;
            rc = hcn_batch_create(&ln.batch, ln.P, ln.cap, ln.max_n, max_nslots, 4096,
                                  l == 0 ? dd_prm : qd_prm, 1, 0);
            if (!rc) rc = hcn_batch_set_split(ln.batch, SPLIT_N);
            if (rc) {
                hcn_server_destroy(s);
                return sfail(rc, hcn_batch_last_error());
            }
            if (hipMalloc((void **)&ln.stage, (size_t)ln.cap * ln.max_n * 2 * ln.P * sizeof(double)) !=
                    hipSuccess ||
                hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming) != hipSuccess) {
                hcn_server_destroy(s);
                return sfail(HCN_ENOMEM, "hcn_server_create: lane allocation");
            }
            ln.slots.assign(ln.cap, nullptr);
            ln.done.assign(ln.cap, 0);
        }
    }
    *out = s;
    return HCN_OK;
}

int hcn_server_destroy(hcn_server s) {
    if (!s) return HCN_OK;
    for (auto &row : s->lane) {
        for (auto &ln : row) {
            if (ln.stream) (void)hipStreamSynchronize(ln.stream);
            if (ln.batch) hcn_batch_destroy(ln.batch);
            if (ln.stage) (void)hipFree(ln.stage);
            if (ln.ev) (void)hipEventDestroy(ln.ev);
            if (ln.stream) (void)hipStreamDestroy(ln.stream);
            for (auto *r : ln.queue) delete r;
            for (auto *r : ln.slots) delete r;
        }
    }
    for (auto *r : s->done) delete r;
    delete s;
    return HCN_OK;
}

double hcn_server_now(hcn_server s) { return s ? s->now() : 0.0; }

int hcn_server_capacity(hcn_server s, int *dd_slots, int *qd_slots) {
    if (!s) return sfail(HCN_EINVAL, "hcn_server_capacity: NULL server");
    int cap[2] = {0, 0};
    for (int l = 0; l < 2; ++l)
        for (auto &ln : s->lane[l]) cap[l] += ln.cap;
    if (dd_slots) *dd_slots = cap[0];
    if (qd_slots) *qd_slots = cap[1];
    return HCN_OK;
}

// Queue a request: system (DD or QD, N == n <= max_n), gamma (host [2][P]),
// start solution x0 (host [n][2][P]), arrival time on the server clock.
int hcn_server_submit(hcn_server s, int64_t id, hcn_sys sys, const double *gamma,
                      const double *x0, double t_arrival) {
    if (!s || !sys || !gamma || !x0) return sfail(HCN_EINVAL, "hcn_server_submit: NULL argument");
    hcn_sys_info_t info;
    if (hcn_sys_info(sys, &info) != HCN_OK) return sfail(HCN_EINVAL, "hcn_server_submit: bad system");
    if (info.P != 2 && info.P != 4) return sfail(HCN_EINVAL, "hcn_server_submit: DD or QD systems only");
    const int l = info.P == 2 ? 0 : 1;
    if (info.N != info.n || info.n > s->max_n) {
        ++s->rejected;
        return sfail(HCN_EINVAL, "hcn_server_submit: system does not fit the server");
    }
    Lane &ln = s->lane[l][size_class(info.n)];
    if (ln.cap == 0) {
        ++s->rejected;
        return sfail(HCN_EINVAL, "hcn_server_submit: no slots for this precision");
    }
    auto *r = new Request;
    r->id = id;
    r->seq = s->seq++;
    hcn::sys_retain(sys);
    r->sys = sys;
    r->P = info.P;
    r->n = info.n;
    std::memcpy(r->gamma, gamma, sizeof(double) * 2 * info.P);
    r->x0.assign(x0, x0 + (size_t)info.n * 2 * info.P);
    r->t_arrival = t_arrival;
    ln.queue.push_back(r);
    return HCN_OK;
}

// One scheduling pass over the lanes (never waits for a lane that is still
// busy); returns the number of paths in flight (>= 0).
int hcn_server_pump(hcn_server s) {
    if (!s) return sfail(HCN_EINVAL, "hcn_server_pump: NULL server");
    // 1. lanes whose last round has finished: harvest
    int running = 0;
    bool all_idle = true;
    for (auto &row : s->lane) {
        for (auto &ln : row) {
            if (!ln.batch) continue;
            if (ln.inflight) {
                const hipError_t e = hipEventQuery(ln.ev);
                if (e == hipErrorNotReady) {
                    running += ln.running;
                    all_idle = false;
                    continue;
                }
                if (e != hipSuccess) return sfail(HCN_EDEVICE, "hcn_server_pump: lane failed");
                ln.inflight = false;
            }
            const int rc = harvest(s, ln);
            if (rc) return rc;
            running += ln.running;
        }
    }
    // 2. admission: every idle lane from its own queue, or (one at a time)
    //    the oldest request of all once nothing runs
    if (s->serial) {
        if (all_idle && running == 0) {
            Lane *best = nullptr;
            for (auto &row : s->lane)
                for (auto &ln : row)
                    if (ln.batch && !ln.queue.empty() && (!best || ln.queue.front()->seq < best->queue.front()->seq))
                        best = &ln;
            if (best) {
                bool ok = false;
                const int rc = admit_one(s, *best, &ok);
                if (rc) return rc;
            }
        }
    } else {
        for (auto &row : s->lane) {
            for (auto &ln : row) {
                if (!ln.batch || ln.inflight) continue;
                bool ok = true;
                while (ok) {
                    const int rc = admit_one(s, ln, &ok);
                    if (rc) return rc;
                }
            }
        }
    }
    // 3. the next round of every idle lane with paths
    int in_flight = 0;
    for (auto &row : s->lane) {
        for (auto &ln : row) {
            if (!ln.batch) continue;
            in_flight += ln.running;
            if (ln.inflight || ln.running == 0) continue;
            const int rc = hcn_batch_step(ln.batch, s->steps_per_round, ln.stream);
            if (rc) return sfail(rc, hcn_batch_last_error());
            if (hipEventRecord(ln.ev, ln.stream) != hipSuccess)
                return sfail(HCN_EDEVICE, "hcn_server_pump: event record failed");
            ln.inflight = true;
        }
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
    size_t q[2] = {0, 0};
    for (int l = 0; l < 2; ++l)
        for (auto &ln : s->lane[l]) q[l] += ln.queue.size();
    if (dd) *dd = (int)q[0];
    if (qd) *qd = (int)q[1];
    return HCN_OK;
}

}  // extern "C"
