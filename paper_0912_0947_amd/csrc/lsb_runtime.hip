// lsb_runtime.hip -- error reporting, device properties and the launch
// configuration table of liblsb.so.
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>

#include "lsb_host.hpp"

namespace lsb {

static thread_local std::string g_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

void clear_error() { g_error.clear(); }

static thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

void take_launch_events(hipEvent_t *start, hipEvent_t *stop) {
    *start = g_ev_start;
    *stop = g_ev_stop;
    g_ev_start = g_ev_stop = nullptr;
}

int set_launch_events(void *start, void *stop) {
    g_ev_start = (hipEvent_t)start;
    g_ev_stop = (hipEvent_t)stop;
    return 0;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(LSB_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

int device_cus() {
    static std::mutex mu;
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> g(mu);
    if (!cus[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            v = 256;
        cus[dev] = v;
    }
    return cus[dev];
}

// ---------------------------------------------------------------------------
// Launch configuration table.
static std::mutex g_tune_mu;
static lsb_launch_cfg g_tune[2][9][kBuckets];
static bool g_tune_init = false;

static void tune_defaults() {
    // 256 threads, two 16-byte vectors per lane per step, one wave group per
    // wave (no grid cap), cached loads/stores.  Replaced by tuned entries.
    for (int op = 0; op < 2; ++op)
        for (int k = 0; k <= 8; ++k)
            for (int b = 0; b < kBuckets; ++b) g_tune[op][k][b] = lsb_launch_cfg{256, 2, 0, 0, 0, 0};
    g_tune_init = true;
}

bool cfg_valid(const lsb_launch_cfg &c) {
    return c.block >= 64 && c.block <= 1024 && c.block % 64 == 0 &&
           (c.unroll == 1 || c.unroll == 2 || c.unroll == 4) && c.blocks_per_cu >= 0 &&
           c.blocks_per_cu <= 64 && (c.nontemporal == 0 || c.nontemporal == 1) && (c.pack == 0 || c.pack == 1) &&
           (c.order == 0 || c.order == 1);
}

static int bucket_of(uint64_t n) {
    int b = 0;
    while (b + 1 < kBuckets && (n >> (b + 1))) ++b;
    return b;
}

lsb_launch_cfg tune_lookup(int op, int k, uint64_t n) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (!g_tune_init) tune_defaults();
    return g_tune[op][k][bucket_of(n)];
}

}  // namespace lsb

using namespace lsb;

extern "C" {

const char *lsb_last_error(void) { return g_error.c_str(); }

const char *lsb_version(void) { return "liblsb 0.1 gfx950"; }

int lsb_time_next_launch(void *start_event, void *stop_event) { return set_launch_events(start_event, stop_event); }

int lsb_tune_get(int op, int k, uint64_t n, lsb_launch_cfg *cfg) {
    if ((op != LSB_OP_EMBED && op != LSB_OP_EXTRACT) || k < 1 || k > 8 || !cfg)
        return fail(LSB_E_ARG, "lsb_tune_get: bad op/k/cfg");
    *cfg = tune_lookup(op, k, n);
    return LSB_OK;
}

int lsb_tune_set(int op, int k, int bucket, const lsb_launch_cfg *cfg) {
    if ((op != LSB_OP_EMBED && op != LSB_OP_EXTRACT) || k < 1 || k > 8 || !cfg || bucket < -1 ||
        bucket >= kBuckets)
        return fail(LSB_E_ARG, "lsb_tune_set: bad op/k/bucket/cfg");
    if (!cfg_valid(*cfg)) return fail(LSB_E_ARG, "lsb_tune_set: invalid configuration");
    std::lock_guard<std::mutex> g(g_tune_mu);
    if (!g_tune_init) tune_defaults();
    if (bucket < 0) {  // -1: every bucket
        for (int b = 0; b < kBuckets; ++b) g_tune[op][k][b] = *cfg;
    } else {
        g_tune[op][k][bucket] = *cfg;
    }
    return LSB_OK;
}

}  // extern "C"
