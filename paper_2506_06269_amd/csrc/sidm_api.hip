// sidm_api.hip -- host side of the libsidm C ABI: argument validation,
// context and scratch memory, per-configuration launch plans, and the
// sequencing of the kernels of each entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sidm_internal.hpp"

namespace sidm {
hipError_t launch_kick_drift(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                             double* x, double* y, double* z, double* vx, double* vy, double* vz,
                             const double* ax, const double* ay, const double* az, hipStream_t st);
hipError_t launch_open_kick(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                            double* vx, double* vy, double* vz, const double* ax, const double* ay,
                            const double* az, int8_t* bin, hipStream_t st);
hipError_t launch_tick_drift(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                             double* x, double* y, double* z, double* vx, double* vy, double* vz,
                             int tick, int bmax, hipStream_t st);
hipError_t launch_diag(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                       int n_halos, const double* x, const double* y, const double* z,
                       const double* vx, const double* vy, const double* vz, const double* m,
                       const double* pot, double* bsum, const long long* ev_counts,
                       const unsigned long long* tree_terms, const int* status, sidm_diag* diag,
                       hipStream_t st);

hipError_t launch_center(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                         int n_halos, const double* radius, const double* x, const double* y,
                         const double* z, const double* m, const double* pot, double* bsum,
                         sidm_center* out, hipStream_t st);
hipError_t launch_tidal(const StreamBlock* d_blocks, int64_t n_blocks, const HaloDev* d_halos,
                        int n_halos, const double* x, const double* y, const double* z,
                        const double* m, const double* pot, double* bsum, sidm_center* cen,
                        double* tid, sidm_tidal* out, hipStream_t st);
}  // namespace sidm

#include "sidm_plan.hpp"

namespace sidm {
hipError_t launch_gravity(bool mixed, const Plan& P, Scratch& w, const sidm_state* s, int kick,
                          hipStream_t st, hipEvent_t tile_begin, hipEvent_t tile_end, int tick = 0,
                          int bmax = 0);
int64_t gravity_slots(int device);
int64_t gravity_slots(int device, const GravShape& shape, bool mixed);
int64_t gravity_sym_slots(int device, const GravShape& shape);
hipError_t launch_cell_list(const Plan& plan, const sidm_state* s, Scratch& w, hipStream_t st,
                            int tick = 0, int bmax = 0);
hipError_t launch_knn(const Plan& plan, const sidm_state* s, Scratch& w, uint32_t* nbr, int k_max,
                      hipStream_t st);
hipError_t launch_tree_hmax(const Plan& plan, Scratch& w, hipStream_t st);
hipError_t launch_reset(const Plan& plan, Scratch& w, hipStream_t st);
hipError_t launch_tree_terms_reset(Scratch& w, int n_halos, hipStream_t st);
hipError_t launch_scatter(const Plan& plan, const sidm_state* s, Scratch& w, uint32_t step,
                          sidm_event* out_events, int64_t out_cap, hipStream_t st,
                          hipEvent_t after_pairs);
hipError_t launch_publish_status(const Plan& P, Scratch& w, hipStream_t st);
hipError_t launch_fingerprint(const Plan& P, Scratch& w, unsigned long long fp, bool captured,
                              hipStream_t st);
hipError_t launch_copy_events(Scratch& w, sidm_event* out, int64_t cap, hipStream_t st);
hipError_t launch_clear_sticky(Scratch& w, hipStream_t st);
}  // namespace sidm

using namespace sidm;

const char* sidm_static_error_text();

struct sidm_ctx {
    int device = 0;
    int64_t max_particles = 0;
    int32_t max_halos = 0;
    std::string err;
    Scratch w;
    Plan plan;
    std::vector<sidm_halo> plan_key;
    std::vector<double> radius;       // host copy of the last central-density radii
    bool plan_valid = false;
    bool timing = false;
    bool timed = false;               // the last step recorded its events
    hipEvent_t ev[SIDM_N_PASSES + 2] = {};
    // device status not yet reported: the sticky word is copied to pinned host
    // memory at the end of each call outside capture and read by a later call
    int* sticky_host = nullptr;
    hipEvent_t sticky_ev = nullptr;
    bool sticky_pending = false;
    // fingerprint of the halos, the state pointers and the scratch memory of
    // the last call outside capture; scratch_gen changes when scratch moves
    uint64_t scratch_gen = 1;
    uint64_t fp_eager = 0;
    bool fp_valid = false;
    GravShape shape;                  // launch shape of the direct-sum tiles
    int64_t sym_min_n = kSymMinN;     // smallest halo of the symmetric tiles (0: none)
};

namespace {

void set_err(sidm_ctx* c, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
}

sidm_status hip_fail(sidm_ctx* c, hipError_t e, const char* where)
{
    set_err(c, "%s: %s", where, hipGetErrorString(e));
    return SIDM_ERR_HIP;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

sidm_status validate(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos, const sidm_state* s,
                     int need)
{
    if (!c) return SIDM_ERR_INVALID;
    if (!halos || n_halos <= 0) {
        set_err(c, "need at least one halo (halos=%p, n_halos=%d)", (const void*)halos, n_halos);
        return SIDM_ERR_INVALID;
    }
    if (n_halos > c->max_halos) {
        set_err(c, "n_halos=%d exceeds the context's max_halos=%d", n_halos, c->max_halos);
        return SIDM_ERR_INVALID;
    }
    if (!s) {
        set_err(c, "state is NULL");
        return SIDM_ERR_INVALID;
    }
    const bool need_pos = true;
    if (need_pos && (!s->x || !s->y || !s->z || !s->m)) {
        set_err(c, "state x, y, z and m must be device pointers");
        return SIDM_ERR_INVALID;
    }
    if ((need & (NEED_GRAV | NEED_STEP)) && (!s->ax || !s->ay || !s->az || !s->pot)) {
        set_err(c, "state ax, ay, az and pot are required");
        return SIDM_ERR_INVALID;
    }
    if ((need & (NEED_KNN | NEED_SCATTER | NEED_STEP)) && (!s->id || !s->h)) {
        set_err(c, "state id and h are required");
        return SIDM_ERR_INVALID;
    }
    if ((need & (NEED_SCATTER | NEED_STEP)) && (!s->vx || !s->vy || !s->vz)) {
        set_err(c, "state vx, vy and vz are required");
        return SIDM_ERR_INVALID;
    }
    std::vector<std::pair<int64_t, int64_t>> ranges;
    int64_t total = 0;
    for (int32_t h = 0; h < n_halos; ++h) {
        const sidm_halo& H = halos[h];
        char msg[256];
        const sidm_status r = check_halo(H, need, msg, sizeof msg);
        if (r != SIDM_OK) {
            set_err(c, "halo %d: %s", h, msg);
            return r;
        }
        ranges.push_back({H.offset, H.offset + H.n});
        total = std::max(total, H.offset + H.n);
    }
    if (total > c->max_particles) {
        set_err(c, "particles up to index %lld exceed the context's max_particles=%lld",
                (long long)total, (long long)c->max_particles);
        return SIDM_ERR_INVALID;
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t r = 1; r < ranges.size(); ++r)
        if (ranges[r].first < ranges[r - 1].second) {
            set_err(c, "halo particle ranges overlap");
            return SIDM_ERR_INVALID;
        }
    return SIDM_OK;
}

sidm_status ensure_plan(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos, hipStream_t st)
{
    if (c->plan_valid && (int32_t)c->plan_key.size() == n_halos &&
        std::memcmp(c->plan_key.data(), halos, sizeof(sidm_halo) * (size_t)n_halos) == 0)
        return SIDM_OK;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
        set_err(c, "the halo configuration changed during stream capture; call once before "
                   "capturing so the launch plan is built");
        return SIDM_ERR_INVALID;
    }
    std::string why;
    const GravItem* items_tick = c->w.items_tick;
    const double4* partial_tick = c->w.partial_tick;
    const SymItem* sym_items = c->w.sym_items;
    const unsigned long long* symacc = c->w.symacc;
    c->w.slots_mixed = gravity_slots(c->device, c->shape, true);
    c->w.slots_fp64 = gravity_slots(c->device, c->shape, false);
    c->w.slots_sym = c->sym_min_n > 0 ? gravity_sym_slots(c->device, c->shape) : 0;
    if (!build_plan(c->plan, c->w, halos, n_halos, c->shape, c->w.slots_mixed, why, c->sym_min_n,
                    c->w.slots_sym) ||
        !ensure_tick_tables(c->w, c->plan, why) || !ensure_sym_tables(c->w, c->plan, why)) {
        c->plan_valid = false;
        set_err(c, "%s", why.c_str());
        return SIDM_ERR_CAPACITY;
    }
    if (items_tick != c->w.items_tick || partial_tick != c->w.partial_tick ||
        sym_items != c->w.sym_items || symacc != c->w.symacc)
        ++c->scratch_gen;
    hipError_t e = upload_plan(c->plan, c->w);
    if (e != hipSuccess) return hip_fail(c, e, "uploading the launch plan");
    c->plan_key.assign(halos, halos + n_halos);
    c->plan_valid = true;
    return SIDM_OK;
}

bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Status code and text for device status bits.
sidm_status report_bits(sidm_ctx* c, int bits, const char* when)
{
    std::string what;
    if (bits & SIDM_DEV_EVENT_OVERFLOW) what += " event buffer overflow (no kicks applied);";
    if (bits & SIDM_DEV_KNN_OVERFLOW) what += " kNN refinement overflow (h is NaN there);";
    if (bits & SIDM_DEV_UNEQUAL_MASS) what += " sigma_m > 0 with unequal masses (not scattered);";
    if (bits & SIDM_DEV_DUPLICATE_ID) what += " repeated ids within a halo (not scattered);";
    if (bits & SIDM_DEV_STALE_GRAPH)
        what += " a captured call was replayed after the halos, state or scratch changed;";
    set_err(c, "%s:%s", when, what.c_str());
    if (bits & (SIDM_DEV_EVENT_OVERFLOW | SIDM_DEV_KNN_OVERFLOW)) return SIDM_ERR_CAPACITY;
    if (bits & (SIDM_DEV_DUPLICATE_ID | SIDM_DEV_STALE_GRAPH)) return SIDM_ERR_INVALID;
    if (bits & SIDM_DEV_UNEQUAL_MASS) return SIDM_ERR_UNSUPPORTED;
    return SIDM_OK;
}

// Conditions a previous call's kernels found, once its copy of the sticky
// word has arrived (no waiting); they are reported once, and clear.
sidm_status take_sticky(sidm_ctx* c, hipStream_t st)
{
    if (!c->sticky_pending || hipEventQuery(c->sticky_ev) != hipSuccess) return SIDM_OK;
    c->sticky_pending = false;
    const int bits = *(volatile int*)c->sticky_host;
    if (!bits) return SIDM_OK;
    *(volatile int*)c->sticky_host = 0;
    (void)launch_clear_sticky(c->w, st);
    const sidm_status r =
        report_bits(c, bits, "an earlier call on this context found (this call was not run)");
    return r == SIDM_OK ? SIDM_ERR_INVALID : r;
}

// After a call's kernels: the status words (when the call reset and set them)
// into the sticky word and, outside capture, its copy to the host.
void publish(sidm_ctx* c, hipStream_t st, bool captured, bool with_status = true)
{
    if (with_status) (void)launch_publish_status(c->plan, c->w, st);
    if (captured) return;
    if (hipMemcpyAsync(c->sticky_host, c->w.sticky, sizeof(int), hipMemcpyDeviceToHost, st) ==
            hipSuccess &&
        hipEventRecord(c->sticky_ev, st) == hipSuccess)
        c->sticky_pending = true;
}

uint64_t fingerprint(const sidm_ctx* c, const sidm_halo* halos, int32_t n_halos,
                     const sidm_state* s)
{
    uint64_t h = 1469598103934665603ull;   // FNV-1a, 64 bit
    auto mix = [&](const void* p, size_t n) {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    mix(halos, sizeof(sidm_halo) * (size_t)n_halos);
    mix(s, sizeof(sidm_state));
    mix(&c->scratch_gen, sizeof c->scratch_gen);
    return h;
}

// Common start of the calls that enqueue kernels (after validation): reports
// conditions found by earlier calls, builds the launch plan, and records the
// fingerprint (outside capture) or enqueues its check (inside capture: the
// last call outside capture must have used the same halos and state).
sidm_status enter(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos, const sidm_state* s,
                  hipStream_t st, bool& captured)
{
    captured = capturing(st);
    sidm_status r;
    if (!captured && (r = take_sticky(c, st)) != SIDM_OK) return r;
    if ((r = ensure_plan(c, halos, n_halos, st)) != SIDM_OK) return r;
    const uint64_t fp = fingerprint(c, halos, n_halos, s);
    if (captured) {
        if (!c->fp_valid || fp != c->fp_eager) {
            set_err(c, "the halos or the state pointers differ from the last call outside "
                       "capture; call once outside capture with them before capturing");
            return SIDM_ERR_INVALID;
        }
        return SIDM_OK;   // the check is enqueued by guard(), after the status reset
    }
    if (c->fp_valid && fp == c->fp_eager) return SIDM_OK;
    const hipError_t e = launch_fingerprint(c->plan, c->w, fp, false, st);
    if (e != hipSuccess) return hip_fail(c, e, "fingerprint launch");
    c->fp_eager = fp;
    c->fp_valid = true;
    return SIDM_OK;
}

// Inside capture: the kernel that flags a replay whose fingerprint is no
// longer the device's (placed after the call's reset of the status words).
sidm_status guard(sidm_ctx* c, hipStream_t st, bool captured)
{
    if (!captured) return SIDM_OK;
    const hipError_t e = launch_fingerprint(c->plan, c->w, c->fp_eager, true, st);
    return e == hipSuccess ? SIDM_OK : hip_fail(c, e, "guard launch");
}

int max_k(const sidm_halo* halos, int32_t n)
{
    int k = 0;
    for (int32_t h = 0; h < n; ++h) k = std::max(k, (int)halos[h].k);
    return k;
}

}  // namespace

extern "C" {

const char* sidm_status_string(sidm_status s)
{
    switch (s) {
    case SIDM_OK: return "ok";
    case SIDM_ERR_INVALID: return "invalid argument";
    case SIDM_ERR_NOMEM: return "out of device memory";
    case SIDM_ERR_HIP: return "HIP runtime error";
    case SIDM_ERR_CAPACITY: return "device capacity exceeded";
    case SIDM_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* sidm_last_error(const sidm_ctx* c) { return c ? c->err.c_str() : sidm_static_error_text(); }

sidm_status sidm_create(sidm_ctx** out, int device, int64_t max_particles, int32_t max_halos)
{
    if (!out) return SIDM_ERR_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return SIDM_ERR_INVALID;
    if (max_particles < 2 || max_halos < 1 || max_particles > (int64_t(1) << 31))
        return SIDM_ERR_INVALID;
    sidm_ctx* c = new sidm_ctx();
    c->device = device;
    c->max_particles = max_particles;
    c->max_halos = max_halos;
    DeviceGuard g(device);
    std::string why;
    const int64_t max_events = std::max<int64_t>(4096, max_particles / 8);
    if (!alloc_scratch(c->w, max_particles, max_halos, max_events, why)) {
        free_scratch(c->w);
        delete c;
        return SIDM_ERR_NOMEM;
    }
    c->w.grav_slots = gravity_slots(device);
    if (hipHostMalloc((void**)&c->sticky_host, sizeof(int), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&c->sticky_ev, hipEventDisableTiming) != hipSuccess) {
        if (c->sticky_host) (void)hipHostFree(c->sticky_host);
        free_scratch(c->w);
        delete c;
        return SIDM_ERR_NOMEM;
    }
    *c->sticky_host = 0;
    *out = c;
    return SIDM_OK;
}

sidm_status sidm_set_event_capacity(sidm_ctx* c, int64_t max_events)
{
    if (!c || max_events < 1) return SIDM_ERR_INVALID;
    DeviceGuard g(c->device);
    std::string why;
    (void)hipDeviceSynchronize();   // the old buffer may still be in use
    ++c->scratch_gen;                // graphs captured before hold the old buffer
    if (!realloc_events(c->w, max_events, why)) {
        set_err(c, "%s", why.c_str());
        return SIDM_ERR_NOMEM;
    }
    return SIDM_OK;
}

void sidm_destroy(sidm_ctx* c)
{
    if (!c) return;
    {
        DeviceGuard g(c->device);
        (void)hipDeviceSynchronize();
        free_scratch(c->w);
        for (auto& ev : c->ev)
            if (ev) (void)hipEventDestroy(ev);
        if (c->sticky_ev) (void)hipEventDestroy(c->sticky_ev);
        if (c->sticky_host) (void)hipHostFree(c->sticky_host);
    }
    delete c;
}

sidm_status sidm_gravity(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos,
                         const sidm_state* s, sidm_precision prec, void* stream)
{
    sidm_status r = validate(c, halos, n_halos, s, NEED_GRAV);
    if (r != SIDM_OK) return r;
    if (prec != SIDM_PREC_FP64 && prec != SIDM_PREC_MIXED) {
        set_err(c, "unknown precision %d", (int)prec);
        return SIDM_ERR_INVALID;
    }
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    if ((r = enter(c, halos, n_halos, s, st, cap)) != SIDM_OK) return r;
    if ((r = guard(c, st, cap)) != SIDM_OK) return r;
    hipError_t e = launch_tree_terms_reset(c->w, n_halos, st);
    if (e == hipSuccess) e = launch_cell_list(c->plan, s, c->w, st);
    if (e == hipSuccess)
        e = launch_gravity(prec == SIDM_PREC_MIXED, c->plan, c->w, s, 0, st, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "gravity launch");
    publish(c, st, cap, false);
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_knn_h(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos, const sidm_state* s,
                       uint32_t* nbr, void* stream)
{
    sidm_status r = validate(c, halos, n_halos, s, NEED_KNN);
    if (r != SIDM_OK) return r;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    if ((r = enter(c, halos, n_halos, s, st, cap)) != SIDM_OK) return r;
    hipError_t e = launch_reset(c->plan, c->w, st);
    if (e == hipSuccess && (r = guard(c, st, cap)) != SIDM_OK) return r;
    if (e == hipSuccess) e = launch_cell_list(c->plan, s, c->w, st);
    if (e == hipSuccess) e = launch_knn(c->plan, s, c->w, nbr, max_k(halos, n_halos), st);
    if (e != hipSuccess) return hip_fail(c, e, "kNN launch");
    publish(c, st, cap);
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_scatter(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos,
                         const sidm_state* s, uint32_t step, sidm_event* events, int64_t cap,
                         int64_t* n_events_host, void* stream)
{
    sidm_status r = validate(c, halos, n_halos, s, NEED_SCATTER);
    if (r != SIDM_OK) return r;
    if (events && cap < 0) {
        set_err(c, "negative event capacity");
        return SIDM_ERR_INVALID;
    }
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    bool captured = false;
    if ((r = enter(c, halos, n_halos, s, st, captured)) != SIDM_OK) return r;
    if (n_events_host && captured) {
        set_err(c, "n_events_host waits for the device: not possible during stream capture");
        return SIDM_ERR_INVALID;
    }
    hipError_t e = launch_reset(c->plan, c->w, st);
    if (e == hipSuccess && (r = guard(c, st, captured)) != SIDM_OK) return r;
    if (e == hipSuccess) e = launch_cell_list(c->plan, s, c->w, st);
    if (e == hipSuccess) e = launch_tree_hmax(c->plan, c->w, st);
    if (e == hipSuccess)
        e = launch_scatter(c->plan, s, c->w, step, events, events ? cap : 0, st, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "scatter launch");
    if (!n_events_host) {
        publish(c, st, captured);
        c->err.clear();
        return SIDM_OK;
    }
    // synchronous: the count and the conditions of this pass are reported here
    unsigned long long cnt = 0;
    std::vector<int> status((size_t)n_halos, 0);
    e = hipMemcpyAsync(&cnt, &c->w.counters->n_events_total, sizeof cnt, hipMemcpyDeviceToHost,
                       st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(status.data(), c->w.status, sizeof(int) * (size_t)n_halos,
                           hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(c, e, "reading the event count");
    *n_events_host = (int64_t)cnt;
    int bits = 0;
    for (int v : status) bits |= v;
    if ((int64_t)cnt > c->w.max_events || (events && (int64_t)cnt > cap)) {
        set_err(c, "%llu events exceed the capacity (context %lld, caller %lld)", cnt,
                (long long)c->w.max_events, (long long)(events ? cap : -1));
        return SIDM_ERR_CAPACITY;
    }
    if (bits) return report_bits(c, bits, "the scattering pass found");
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_last_events(sidm_ctx* c, sidm_event* out, int64_t cap, int64_t* n_events_host,
                             void* stream)
{
    if (!c) return SIDM_ERR_INVALID;
    if ((cap > 0 && !out) || cap < 0) {
        set_err(c, "need a device buffer for cap >= 0 events");
        return SIDM_ERR_INVALID;
    }
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    if (n_events_host && capturing(st)) {
        set_err(c, "n_events_host waits for the device: not possible during stream capture");
        return SIDM_ERR_INVALID;
    }
    hipError_t e = hipSuccess;
    if (cap > 0) e = launch_copy_events(c->w, out, cap, st);
    if (e != hipSuccess) return hip_fail(c, e, "event copy launch");
    if (n_events_host) {
        unsigned long long cnt = 0;
        e = hipMemcpyAsync(&cnt, &c->w.counters->n_events_total, sizeof cnt,
                           hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "reading the event count");
        *n_events_host = (int64_t)cnt;
        if ((int64_t)cnt > c->w.max_events || (int64_t)cnt > cap) {
            set_err(c, "%llu events exceed the capacity (context %lld, caller %lld)", cnt,
                    (long long)c->w.max_events, (long long)cap);
            return SIDM_ERR_CAPACITY;
        }
    }
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_kdk_step(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos,
                          const sidm_state* s, uint32_t step, sidm_precision prec,
                          sidm_diag* diag, void* stream)
{
    sidm_status r = validate(c, halos, n_halos, s, NEED_STEP);
    if (r != SIDM_OK) return r;
    if (prec != SIDM_PREC_FP64 && prec != SIDM_PREC_MIXED) {
        set_err(c, "unknown precision %d", (int)prec);
        return SIDM_ERR_INVALID;
    }
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    bool captured = false;
    if ((r = enter(c, halos, n_halos, s, st, captured)) != SIDM_OK) return r;
    const Plan& P = c->plan;
    // events: 0 start, 1 after kick+drift, 5 after the cell list, 2/3 around
    // the gravity tiles, 4 after gravity, 6 after kNN, 7 after the pair search,
    // 8 after the kicks, 9 after the diagnostics
    hipEvent_t* E = c->ev;
    const bool tm = c->timing && !captured;
    auto mark = [&](int i) {
        if (tm) (void)hipEventRecord(E[i], st);
    };
    // block time steps: the deepest bin of the halos that use them
    int bmax = -1;
    for (int32_t h = 0; h < n_halos; ++h)
        if (halos[h].eta > 0.0) bmax = std::max(bmax, (int)halos[h].max_bin);
    mark(0);
    hipError_t e = launch_reset(P, c->w, st);
    if (e == hipSuccess && (r = guard(c, st, captured)) != SIDM_OK) return r;
    if (e == hipSuccess) e = launch_tree_terms_reset(c->w, n_halos, st);
    if (bmax < 0) {
        if (e == hipSuccess)
            e = launch_kick_drift(c->w.blocks, P.n_blocks, c->w.halos, s->x, s->y, s->z, s->vx,
                                  s->vy, s->vz, s->ax, s->ay, s->az, st);
        mark(1);
        if (e == hipSuccess) e = launch_cell_list(P, s, c->w, st);
        mark(5);
        if (e == hipSuccess)
            e = launch_gravity(prec == SIDM_PREC_MIXED, P, c->w, s, 1, st, tm ? E[2] : nullptr,
                               tm ? E[3] : nullptr);
    } else {
        if (e == hipSuccess)
            e = launch_open_kick(c->w.blocks, P.n_blocks, c->w.halos, s->vx, s->vy, s->vz, s->ax,
                                 s->ay, s->az, c->w.bin, st);
        mark(1);
        mark(5);
        mark(2);
        for (int tick = 1; tick <= (1 << bmax) && e == hipSuccess; ++tick) {
            e = launch_tick_drift(c->w.blocks, P.n_blocks, c->w.halos, s->x, s->y, s->z, s->vx,
                                  s->vy, s->vz, tick, bmax, st);
            if (e == hipSuccess) e = launch_cell_list(P, s, c->w, st, tick, bmax);
            if (e == hipSuccess)
                e = launch_gravity(prec == SIDM_PREC_MIXED, P, c->w, s, 1, st, nullptr, nullptr,
                                   tick, bmax);
        }
        mark(3);
    }
    mark(4);
    if (e == hipSuccess) e = launch_knn(P, s, c->w, nullptr, max_k(halos, n_halos), st);
    if (e == hipSuccess) e = launch_tree_hmax(P, c->w, st);
    mark(6);
    if (e == hipSuccess) e = launch_scatter(P, s, c->w, step, nullptr, 0, st, tm ? E[7] : nullptr);
    mark(8);
    if (e == hipSuccess && diag)
        e = launch_diag(c->w.blocks, P.n_blocks, c->w.halos, n_halos, s->x, s->y, s->z, s->vx,
                        s->vy, s->vz, s->m, s->pot, c->w.bsum, c->w.ev_counts, c->w.tree_terms,
                        c->w.status, diag, st);
    mark(9);
    c->timed = tm;
    if (e != hipSuccess) return hip_fail(c, e, "step launch");
    publish(c, st, captured);
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_diagnostics(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos,
                             const sidm_state* s, sidm_diag* diag, void* stream)
{
    sidm_status r = validate(c, halos, n_halos, s, 0);
    if (r != SIDM_OK) return r;
    if (!diag || !s->vx || !s->vy || !s->vz || !s->pot) {
        set_err(c, "diag, vx, vy, vz and pot are required");
        return SIDM_ERR_INVALID;
    }
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    if ((r = enter(c, halos, n_halos, s, st, cap)) != SIDM_OK) return r;
    if ((r = guard(c, st, cap)) != SIDM_OK) return r;
    const Plan& P = c->plan;
    hipError_t e = launch_diag(c->w.blocks, P.n_blocks, c->w.halos, n_halos, s->x, s->y, s->z,
                               s->vx, s->vy, s->vz, s->m, s->pot, c->w.bsum, c->w.ev_counts,
                               c->w.tree_terms,
                               c->w.status, diag, st);
    if (e != hipSuccess) return hip_fail(c, e, "diagnostics launch");
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_central_density(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos,
                                 const sidm_state* s, const double* radius, sidm_center* out,
                                 void* stream)
{
    sidm_status r = validate(c, halos, n_halos, s, 0);
    if (r != SIDM_OK) return r;
    if (!out || !radius || !s->pot) {
        set_err(c, "radius, out and pot are required");
        return SIDM_ERR_INVALID;
    }
    for (int h = 0; h < n_halos; ++h)
        if (!(radius[h] > 0.0) || !std::isfinite(radius[h])) {
            set_err(c, "halo %d: radius must be positive and finite", h);
            return SIDM_ERR_INVALID;
        }
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    if ((r = enter(c, halos, n_halos, s, st, cap)) != SIDM_OK) return r;
    if ((r = guard(c, st, cap)) != SIDM_OK) return r;
    const Plan& P = c->plan;
    c->radius.assign(radius, radius + n_halos);
    hipError_t e = hipMemcpyAsync(c->w.radius, c->radius.data(), sizeof(double) * (size_t)n_halos,
                                  hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(c, e, "radius upload");
    e = launch_center(c->w.blocks, P.n_blocks, c->w.halos, n_halos, c->w.radius, s->x, s->y,
                      s->z, s->m, s->pot, c->w.bsum, out, st);
    if (e != hipSuccess) return hip_fail(c, e, "central density launch");
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_tidal_radius(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos,
                              const sidm_state* s, sidm_tidal* out, void* stream)
{
    sidm_status r = validate(c, halos, n_halos, s, 0);
    if (r != SIDM_OK) return r;
    if (!out || !s->pot) {
        set_err(c, "out and pot are required");
        return SIDM_ERR_INVALID;
    }
    for (int h = 0; h < n_halos; ++h)
        if (halos[h].host_kind == 0) {
            set_err(c, "halo %d: the tidal radius needs a host (host_kind != 0)", h);
            return SIDM_ERR_INVALID;
        }
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    bool cap = false;
    if ((r = enter(c, halos, n_halos, s, st, cap)) != SIDM_OK) return r;
    if ((r = guard(c, st, cap)) != SIDM_OK) return r;
    const Plan& P = c->plan;
    hipError_t e = launch_tidal(c->w.blocks, P.n_blocks, c->w.halos, n_halos, s->x, s->y, s->z,
                                s->m, s->pot, c->w.bsum, c->w.center, c->w.tidal, out, st);
    if (e != hipSuccess) return hip_fail(c, e, "tidal radius launch");
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_take_status(sidm_ctx* c, int32_t* bits)
{
    if (!c || !bits) return SIDM_ERR_INVALID;
    DeviceGuard g(c->device);
    int v = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&v, c->w.sticky, sizeof v, hipMemcpyDeviceToHost);
    if (e == hipSuccess && v) e = hipMemset(c->w.sticky, 0, sizeof v);
    if (e != hipSuccess) return hip_fail(c, e, "reading the status");
    c->sticky_pending = false;
    *(volatile int*)c->sticky_host = 0;
    *bits = v;
    return SIDM_OK;
}

sidm_status sidm_enable_timing(sidm_ctx* c, int on)
{
    if (!c) return SIDM_ERR_INVALID;
    DeviceGuard g(c->device);
    if (on && !c->ev[0])
        for (auto& ev : c->ev)
            if (hipEventCreate(&ev) != hipSuccess) return hip_fail(c, hipGetLastError(), "events");
    c->timing = on != 0;
    return SIDM_OK;
}

sidm_status sidm_pass_times(sidm_ctx* c, double ms[SIDM_N_PASSES])
{
    if (!c || !ms) return SIDM_ERR_INVALID;
    if (!c->timed) {
        set_err(c, "no timed step recorded (enable timing, then run sidm_kdk_step)");
        return SIDM_ERR_INVALID;
    }
    DeviceGuard g(c->device);
    hipError_t e = hipEventSynchronize(c->ev[9]);
    if (e != hipSuccess) return hip_fail(c, e, "waiting for the timed step");
    const int from[SIDM_N_PASSES] = {0, 5, 2, 1, 4, 6, 7, 8};
    const int to[SIDM_N_PASSES] = {1, 4, 3, 5, 6, 7, 8, 9};
    for (int p = 0; p < SIDM_N_PASSES; ++p) {
        float t = 0.f;
        e = hipEventElapsedTime(&t, c->ev[from[p]], c->ev[to[p]]);
        if (e != hipSuccess) return hip_fail(c, e, "reading pass times");
        ms[p] = t;
    }
    return SIDM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- launch shapes
namespace {

bool shape_supported(int ireg, int nt)
{
    for (int k = 0; k < kNumShapes; ++k)
        if (kShapeIreg[k] == ireg && kShapeNt[k] == nt) return true;
    return false;
}

// Key of a tuning-cache entry: device architecture and compute units,
// precision, and the call's direct-sum size class (log2 of the particles in
// direct-sum halos, and of the number of halos, both rounded to nearest).
// sym_min_n: the context's threshold of the symmetric tiles; a mixed call
// with a halo that takes them is keyed apart (":sym"), as it times them.
std::string tune_key(int device, const sidm_halo* halos, int32_t n_halos, sidm_precision prec,
                     int64_t sym_min_n)
{
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch.resize(colon);
        cus = prop.multiProcessorCount;
    }
    double ndir = 0.0;
    int nh = 0;
    bool sym = false;
    for (int32_t h = 0; h < n_halos; ++h)
        if (!(halos[h].tree_alpha > 0.0)) {
            ndir += (double)halos[h].n;
            ++nh;
            if (sym_min_n > 0 && halos[h].n >= std::max<int64_t>(sym_min_n, 2) &&
                halos[h].eps > 0.0)
                sym = true;
        }
    const int ln = ndir > 0.0 ? (int)std::lround(std::log2(ndir)) : 0;
    const int lh = nh > 0 ? (int)std::lround(std::log2((double)nh)) : 0;
    char buf[160];
    snprintf(buf, sizeof buf, "%s:%dcu:%s:n2^%d:h2^%d%s", arch.c_str(), cus,
             prec == SIDM_PREC_MIXED ? "mixed" : "fp64", ln, lh,
             prec == SIDM_PREC_MIXED && sym ? ":sym" : "");
    return buf;
}

// The cache file: one JSON object, one entry per line,
//   "key": {"ireg": I, "threads": T, "persistent": P, "ms": X, "ms_default": Y},
// read back line by line (the file is only ever written by tune_write).
bool tune_read(const char* path, const std::string& key, GravShape& shape)
{
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char line[512];
    const std::string want = "\"" + key + "\":";
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        const char* p = strstr(line, want.c_str());
        if (!p) continue;
        int ireg = 0, nt = 0, persist = 0;
        if (sscanf(p + want.size(), " {\"ireg\": %d, \"threads\": %d, \"persistent\": %d", &ireg,
                   &nt, &persist) == 3 && shape_supported(ireg, nt)) {
            shape.ireg = ireg;
            shape.nt = nt;
            shape.persist = persist ? 1 : 0;
            found = true;
        }
        break;
    }
    fclose(f);
    return found;
}

bool tune_write(const char* path, const std::string& key, const GravShape& s, double ms,
                double ms_default)
{
    std::vector<std::string> lines;
    if (FILE* f = fopen(path, "r")) {
        char line[512];
        const std::string want = "\"" + key + "\":";
        while (fgets(line, sizeof line, f)) {
            std::string l(line);
            while (!l.empty() && (l.back() == '\n' || l.back() == ',' || l.back() == ' '))
                l.pop_back();
            if (l.find("\": {\"ireg\"") == std::string::npos) continue;   // braces, junk
            if (l.find(want) != std::string::npos) continue;              // replaced below
            size_t a = l.find('"');
            lines.push_back(a == std::string::npos ? l : l.substr(a));
        }
        fclose(f);
    }
    char buf[320];
    snprintf(buf, sizeof buf,
             "\"%s\": {\"ireg\": %d, \"threads\": %d, \"persistent\": %d, \"ms\": %.4f, "
             "\"ms_default\": %.4f}",
             key.c_str(), s.ireg, s.nt, s.persist, ms, ms_default);
    lines.push_back(buf);
    std::sort(lines.begin(), lines.end());
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fputs("{\n", f);
    for (size_t i = 0; i < lines.size(); ++i)
        fprintf(f, "  %s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
    fputs("}\n", f);
    const bool ok = fclose(f) == 0;
    return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

sidm_status sidm_set_launch_shape(sidm_ctx* c, int32_t ireg, int32_t threads, int32_t persistent)
{
    if (!c) return SIDM_ERR_INVALID;
    if (!shape_supported(ireg, threads)) {
        set_err(c, "no gravity tiles of shape ireg=%d threads=%d", ireg, threads);
        return SIDM_ERR_UNSUPPORTED;
    }
    DeviceGuard g(c->device);
    GravShape s;
    s.ireg = ireg;
    s.nt = threads;
    s.persist = persistent ? 1 : 0;
    if (s.persist && gravity_slots(c->device, s, true) <= 0) {
        set_err(c, "no resident blocks known for the persistent launch of this shape");
        return SIDM_ERR_UNSUPPORTED;
    }
    if (s.ireg != c->shape.ireg || s.nt != c->shape.nt || s.persist != c->shape.persist) {
        c->shape = s;
        c->plan_valid = false;   // the work items follow the shape
        ++c->scratch_gen;        // graphs captured before launch the old shape
    }
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_set_symmetric(sidm_ctx* c, int64_t min_n)
{
    if (!c) return SIDM_ERR_INVALID;
    if (min_n < 0) {
        set_err(c, "min_n must be >= 0");
        return SIDM_ERR_INVALID;
    }
    if (min_n != c->sym_min_n) {
        c->sym_min_n = min_n;
        c->plan_valid = false;
        ++c->scratch_gen;
    }
    c->err.clear();
    return SIDM_OK;
}

sidm_status sidm_autotune(sidm_ctx* c, const sidm_halo* halos, int32_t n_halos,
                          const sidm_state* s, sidm_precision prec, const char* cache_path,
                          int32_t flags, sidm_tune_result* out, void* stream)
{
    sidm_status r = validate(c, halos, n_halos, s, NEED_GRAV);
    if (r != SIDM_OK) return r;
    if (prec != SIDM_PREC_FP64 && prec != SIDM_PREC_MIXED) {
        set_err(c, "unknown precision %d", (int)prec);
        return SIDM_ERR_INVALID;
    }
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    if (capturing(st)) {
        set_err(c, "the tuner times launches: not possible during stream capture");
        return SIDM_ERR_INVALID;
    }
    const std::string key = tune_key(c->device, halos, n_halos, prec, c->sym_min_n);
    sidm_tune_result res;
    std::memset(&res, 0, sizeof res);
    snprintf(res.key, sizeof res.key, "%s", key.c_str());
    GravShape best;
    bool have = false;
    if (cache_path && !(flags & SIDM_TUNE_FORCE)) have = tune_read(cache_path, key, best);
    if (!have && (flags & SIDM_TUNE_CACHE_ONLY)) {
        best = c->shape;   // no entry: the current shape stays, nothing is timed
        res.ireg = best.ireg;
        res.threads = best.nt;
        res.persistent = best.persist;
        if (out) *out = res;
        c->err.clear();
        return sidm_gravity(c, halos, n_halos, s, prec, stream);
    }
    const GravShape saved = c->shape;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipSuccess;
    if (!have) {
        // time every shape on the caller's halos: the cell list once, then the
        // gravity pass (all its kernels) per shape, the best of a few runs
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
            return hip_fail(c, e, "tuner events");
        bool cap = false;
        double best_ms = 1e300, default_ms = 0.0;
        for (int k = 0; k < 2 * kNumShapes && e == hipSuccess; ++k) {
            GravShape cand;
            cand.ireg = kShapeIreg[k % kNumShapes];
            cand.nt = kShapeNt[k % kNumShapes];
            cand.persist = k >= kNumShapes ? 1 : 0;
            if (gravity_slots(c->device, cand, prec == SIDM_PREC_MIXED) <= 0) continue;
            c->shape = cand;
            c->plan_valid = false;
            if ((r = enter(c, halos, n_halos, s, st, cap)) != SIDM_OK) break;
            e = launch_cell_list(c->plan, s, c->w, st);
            double ms = 1e300;
            const int runs = (flags & SIDM_TUNE_QUICK) ? 2 : 4;
            for (int rep = 0; rep < runs && e == hipSuccess; ++rep) {
                (void)hipEventRecord(e0, st);
                e = launch_gravity(prec == SIDM_PREC_MIXED, c->plan, c->w, s, 0, st, nullptr,
                                   nullptr);
                (void)hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float t = 0.f;
                if (e == hipSuccess && rep > 0 && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
                    ms = std::min(ms, (double)t);
            }
            if (cand.ireg == 4 && cand.nt == 256 && !cand.persist) default_ms = ms;
            if (ms < best_ms) {
                best_ms = ms;
                best = cand;
            }
            ++res.n_tried;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (r != SIDM_OK || e != hipSuccess) {
            c->shape = saved;
            c->plan_valid = false;
            return r != SIDM_OK ? r : hip_fail(c, e, "tuner launch");
        }
        res.ms = best_ms;
        res.ms_default = default_ms;
        if (cache_path && !tune_write(cache_path, key, best, best_ms, default_ms)) {
            set_err(c, "cannot write the tuning cache %s", cache_path);
            c->shape = best;
            c->plan_valid = false;
            return SIDM_ERR_INVALID;
        }
    } else {
        res.from_cache = 1;
    }
    // the chosen shape, and a and pot as sidm_gravity computes them with it
    c->shape = best;
    c->plan_valid = false;
    res.ireg = best.ireg;
    res.threads = best.nt;
    res.persistent = best.persist;
    if (out) *out = res;
    c->err.clear();
    return sidm_gravity(c, halos, n_halos, s, prec, stream);
}

}  // extern "C"
