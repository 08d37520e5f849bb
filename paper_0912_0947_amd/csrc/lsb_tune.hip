// lsb_tune.hip -- autotuner for the plain embed / extract launch
// configuration: times every candidate (block size, vectors per lane,
// grid cap, streaming cache policy) on caller-provided device buffers and
// installs the fastest for the size bucket of n.
//
// The paper fixes the launch at 4 blocks of min(32, data length) threads per
// image row (Section VI step 6, Section VII step 5); here the launch shape is
// a measured choice per (op, k, size bucket).
#include <vector>

#include "lsb_host.hpp"

using namespace lsb;

namespace {

// Write a scratch buffer larger than the 256 MB Infinity Cache before each
// timed launch so that reads come from HBM.
struct Flush {
    void *buf = nullptr;
    size_t bytes = 0;
    int init(size_t b) {
        bytes = b;
        hipError_t e = hipMalloc(&buf, bytes);
        return e == hipSuccess ? LSB_OK : hip_fail(e, "hipMalloc(flush buffer)");
    }
    int run(hipStream_t s) {
        hipError_t e = hipMemsetAsync(buf, 0x5A, bytes, s);
        return e == hipSuccess ? LSB_OK : hip_fail(e, "hipMemsetAsync(flush)");
    }
    ~Flush() {
        if (buf) (void)hipFree(buf);
    }
};

}  // namespace

extern "C" int lsb_autotune(int op, int k, uint64_t n, uint8_t *cover, uint8_t *stego, uint8_t *msg, int reps,
                            lsb_launch_cfg *best, double *best_us, void *stream_v) {
    const TimedCall timed_call;
    if ((op != LSB_OP_EMBED && op != LSB_OP_EXTRACT) || k < 1 || k > 8 || !cover || !stego || !msg || reps < 1 ||
        reps > 1000)
        return fail(LSB_E_ARG, "lsb_autotune: bad arguments");
    hipStream_t stream = (hipStream_t)stream_v;
    const int64_t cap = lsb_capacity(n, k);
    if (cap < 0) return (int)cap;
    if (overlaps(cover, n, stego, n) || overlaps(msg, (uint64_t)cap, stego, n) || overlaps(msg, (uint64_t)cap, cover, n))
        return fail(LSB_E_ARG, "lsb_autotune: buffers overlap");

    Flush flush;
    int rc = flush.init((size_t)512 << 20);
    if (rc) return rc;
    uint32_t *status = nullptr;
    hipError_t e = hipMalloc((void **)&status, 16);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(status)");
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    // both events exist in a recorded state before the first timing
    if (e == hipSuccess) e = hipEventRecord(ev0, stream);
    if (e == hipSuccess) e = hipEventRecord(ev1, stream);
    if (e != hipSuccess) {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        (void)hipFree(status);
        return hip_fail(e, "hipEventCreate/Record(autotune)");
    }

    // For extract, the stego buffer must carry a full-capacity stream.
    Span base{};
    base.n = n;
    base.k = k;
    base.hdr_len = 4;
    base.t0 = 0;
    if (op == LSB_OP_EXTRACT) {
        Span s = base;
        s.src = cover;
        s.dst = stego;
        s.body = msg;
        s.bits = 8 * (4 + (uint64_t)cap);
        s.hdr = (uint32_t)cap;
        rc = launch_embed(s, tune_lookup(LSB_OP_EMBED, k, n), stream);
    }
    const int blocks[] = {256, 512, 1024};
    const int unrolls[] = {1, 2, 4};
    const int caps[] = {0, 1, 2, 4, 8, 16};
    double best_t = 1e30;
    lsb_launch_cfg best_c = tune_lookup(op, k, n);
    const int packs = (op == LSB_OP_EXTRACT && k == 1) ? 2 : 1;  // ballot packing exists for k = 1
    for (int ord = 0; ord < 2 && rc == LSB_OK; ++ord)
    for (int pk = 0; pk < packs && rc == LSB_OK; ++pk)
    for (int nt = 0; nt < 2 && rc == LSB_OK; ++nt)
        for (int b : blocks)
            for (int u : unrolls)
                for (int c : caps) {
                    if (rc != LSB_OK) break;
                    const lsb_launch_cfg cfg{b, u, c, nt, pk, ord};
                    double total = 0;
                    for (int r = 0; r < reps && rc == LSB_OK; ++r) {
                        rc = flush.run(stream);
                        if (rc) break;
                        set_launch_events(ev0, ev1);  // bound to the kernel's own begin and end
                        if (op == LSB_OP_EMBED) {
                            Span s = base;
                            s.src = cover;
                            s.dst = stego;
                            s.body = msg;
                            s.bits = 8 * (4 + (uint64_t)cap);
                            s.hdr = (uint32_t)cap;
                            rc = launch_embed(s, cfg, stream);
                        } else {
                            Span s = base;
                            s.src = stego;
                            s.out = msg;
                            const uint64_t v_stream = ceil_div(4 + (uint64_t)cap, 2 * (uint64_t)k);
                            const uint64_t v_buf = ceil_div(n, 16);
                            rc = launch_extract(s, 1, (uint64_t)cap, status, (int32_t *)(status + 1),
                                                v_stream < v_buf ? v_stream : v_buf, cfg, stream);
                        }
                        e = hipEventSynchronize(ev1);
                        if (e != hipSuccess) {
                            rc = hip_fail(e, "hipEventSynchronize(autotune)");
                            break;
                        }
                        float ms = 0;
                        e = hipEventElapsedTime(&ms, ev0, ev1);
                        if (e != hipSuccess) {
                            rc = hip_fail(e, "hipEventElapsedTime(autotune)");
                            break;
                        }
                        total += ms;
                    }
                    const double t = total / reps;
                    if (rc == LSB_OK && t < best_t) {
                        best_t = t;
                        best_c = cfg;
                    }
                }
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    (void)hipFree(status);
    if (rc != LSB_OK) return rc;
    int bucket = 0;
    while (bucket + 1 < kBuckets && (n >> (bucket + 1))) ++bucket;
    rc = lsb_tune_set(op, k, bucket, &best_c);
    if (rc != LSB_OK) return rc;
    if (best) *best = best_c;
    if (best_us) *best_us = best_t * 1e3;
    return LSB_OK;
}
