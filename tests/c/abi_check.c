/* abi_check.c -- the C ABI of liblsb.so used from plain C (and C++): every
 * entry point of lsb.h is referenced with its declared type, the record
 * layouts that bindings rely on are fixed, and the host-only calls run
 * without a GPU (capacity, tuning tables, the serving scheduler on its
 * modelled clock).  Prints "ok" on success. */
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include "lsb.h"

#ifdef __cplusplus
#define STATIC_ASSERT static_assert
#else
#define STATIC_ASSERT _Static_assert
#endif

STATIC_ASSERT(sizeof(lsb_job) == 64, "lsb_job is 64 bytes");
STATIC_ASSERT(offsetof(lsb_job, msg_cap) == 32 && offsetof(lsb_job, t0) == 40 &&
                  offsetof(lsb_job, stream_bits) == 48 && offsetof(lsb_job, len) == 56 &&
                  offsetof(lsb_job, flags) == 62,
              "lsb_job field offsets");
STATIC_ASSERT(sizeof(lsb_launch_cfg) == 24, "lsb_launch_cfg is six int32");
STATIC_ASSERT(sizeof(lsb_server_cfg) == 48, "lsb_server_cfg is 48 bytes");
STATIC_ASSERT(sizeof(lsb_request) == 48, "lsb_request is 48 bytes");
STATIC_ASSERT(sizeof(lsb_result) == 56, "lsb_result is 56 bytes");
STATIC_ASSERT(sizeof(lsb_serve_stats) == 104, "lsb_serve_stats is 104 bytes");

typedef void (*any_fn)(void);

/* Every entry point, through its declared type (a mismatch fails to compile). */
static const any_fn entry_points[] = {
    (any_fn)lsb_capacity,       (any_fn)lsb_embed,           (any_fn)lsb_extract,
    (any_fn)lsb_extract_sync,   (any_fn)lsb_embed_raw,       (any_fn)lsb_extract_raw,
    (any_fn)lsb_paper_capacity, (any_fn)lsb_paper_embed,     (any_fn)lsb_paper_extract,
    (any_fn)lsb_embed_plane,    (any_fn)lsb_extract_plane,   (any_fn)lsb_sse,
    (any_fn)lsb_video_embed_host, (any_fn)lsb_verify,        (any_fn)lsb_plan_create,
    (any_fn)lsb_plan_update,    (any_fn)lsb_plan_run,        (any_fn)lsb_embed_batch,
    (any_fn)lsb_extract_batch,  (any_fn)lsb_plan_tiles,      (any_fn)lsb_plan_destroy,
    (any_fn)lsb_tune_get,       (any_fn)lsb_tune_set,        (any_fn)lsb_autotune,
    (any_fn)lsb_batch_tune_get, (any_fn)lsb_batch_tune_set,  (any_fn)lsb_serve,
    (any_fn)lsb_time_next_launch, (any_fn)lsb_stream_reference, (any_fn)lsb_serve_simulate,
    (any_fn)lsb_last_error,     (any_fn)lsb_version,         (any_fn)lsb_job_extents,
    (any_fn)lsb_slice_stream_bytes, (any_fn)lsb_embed_verify,  (any_fn)lsb_batch_run_static,
    (any_fn)lsb_batch_tune_get_op, (any_fn)lsb_batch_tune_set_op, (any_fn)lsb_roundtrip_latency,
};

static int check(int cond, const char *what) {
    if (!cond) fprintf(stderr, "FAILED: %s (%s)\n", what, lsb_last_error());
    return cond ? 0 : 1;
}

int main(void) {
    int bad = 0;
    size_t i;
    for (i = 0; i < sizeof entry_points / sizeof entry_points[0]; ++i) bad += check(entry_points[i] != NULL, "symbol");

    /* capacity: floor(n*k/8) - 4, capped by the 32-bit header */
    bad += check(lsb_capacity(786432, 1) == 98300, "capacity 512x512x3 at k = 1");
    bad += check(lsb_capacity(201326592, 4) == 100663292, "capacity 8192x8192x3 at k = 4");
    bad += check(lsb_capacity(1ull << 40, 8) == 0xFFFFFFFFll, "capacity capped at 2^32 - 1");
    bad += check(lsb_capacity(31, 1) == LSB_E_CAPACITY, "no room for the header");
    bad += check(lsb_capacity(100, 9) == LSB_E_ARG && lsb_last_error()[0] != '\0', "k outside 1..8");
    bad += check(lsb_paper_capacity(7, 1024) == 7 * 256, "paper-layout capacity");
    bad += check(lsb_version() != NULL && strlen(lsb_version()) > 0, "version string");

    /* stream bytes a raw slice touches: ceil(min(k*(t0+n), bits) / 8) */
    bad += check(lsb_slice_stream_bytes(1, 0, 100, 4000) == 13, "slice stream bytes, k = 1");
    bad += check(lsb_slice_stream_bytes(2, 4, 10, 1000) == 4, "slice stream bytes, k = 2, t0 = 4");
    bad += check(lsb_slice_stream_bytes(3, 10, 50, 30) == 0, "slice past the stream touches nothing");
    bad += check(lsb_slice_stream_bytes(9, 0, 1, 8) == LSB_E_ARG, "slice stream bytes, bad k");

    /* the allocation-free batched call refuses more jobs than its table
     * before touching a device */
    bad += check(lsb_batch_run_static(NULL, LSB_STATIC_MAX_JOBS + 1, LSB_OP_EMBED, NULL, NULL, NULL, NULL, NULL,
                                      NULL) == LSB_E_ARG, "static batch refuses n_jobs > LSB_STATIC_MAX_JOBS");

    /* arena extents of a job list */
    {
        lsb_job jobs[2];
        uint64_t ext[3] = {0, 0, 0};
        memset(jobs, 0, sizeof jobs);
        jobs[0].cover_off = 0;      jobs[0].stego_off = 512;  jobs[0].msg_off = 0;
        jobs[0].n = 1000;           jobs[0].len = 100;        jobs[0].k = 1; /* capacity 121 */
        jobs[1].cover_off = 4096;   jobs[1].stego_off = 0;    jobs[1].msg_off = 256;
        jobs[1].n = 100;            jobs[1].len = 30;         jobs[1].k = 1; /* capacity 8: no work */
        bad += check(lsb_job_extents(jobs, 2, LSB_OP_EMBED, ext) == LSB_OK, "job extents");
        bad += check(ext[0] == 4196 && ext[1] == 1512 && ext[2] == 100, "embed extents");
        jobs[0].msg_cap = 500;      jobs[1].msg_cap = 3;
        bad += check(lsb_job_extents(jobs, 2, LSB_OP_EXTRACT, ext) == LSB_OK, "extract extents");
        bad += check(ext[0] == 0 && ext[1] == 1512 && ext[2] == 259, "extract extents: min(msg_cap, capacity)");
        jobs[1].k = 0;
        bad += check(lsb_job_extents(jobs, 2, LSB_OP_EMBED, ext) == LSB_E_ARG, "extents refuse k = 0");
    }

    /* the serving loop refuses a null cover pool before touching a device */
    {
        lsb_server_cfg cfg;
        lsb_request req;
        lsb_result res;
        memset(&cfg, 0, sizeof cfg);
        memset(&req, 0, sizeof req);
        cfg.arena = (uint8_t *)(uintptr_t)4096; /* never dereferenced: the call fails first */
        cfg.arena_bytes = 1u << 20;
        cfg.msg_pool = (const uint8_t *)(uintptr_t)8192;
        cfg.max_batch = 1;
        cfg.n_slots = 1;
        req.n = 4096;
        req.k = 1;
        bad += check(lsb_serve(&cfg, &req, 1, &res, NULL) == LSB_E_ARG, "serve refuses a null cover pool");
        cfg.cover_pool = (const uint8_t *)(uintptr_t)8192;
        cfg.msg_pool = NULL;
        bad += check(lsb_serve(&cfg, &req, 1, &res, NULL) == LSB_E_ARG, "serve refuses a null message pool");
    }

    /* tuning tables round trip */
    {
        lsb_launch_cfg c, back;
        int64_t tv = 0;
        bad += check(lsb_tune_get(LSB_OP_EMBED, 3, 1u << 20, &c) == LSB_OK, "tune_get");
        bad += check(lsb_tune_set(LSB_OP_EMBED, 3, 20, &c) == LSB_OK, "tune_set");
        bad += check(lsb_tune_get(LSB_OP_EMBED, 3, 1u << 20, &back) == LSB_OK && memcmp(&c, &back, sizeof c) == 0,
                     "tune round trip");
        bad += check(lsb_batch_tune_get(&c, &tv) == LSB_OK && tv >= 64, "batch tune_get");
        c.block = 100;
        bad += check(lsb_tune_set(LSB_OP_EMBED, 3, 20, &c) == LSB_E_ARG, "invalid block refused");
        c.block = 256;
        c.order = 2;
        bad += check(lsb_tune_set(LSB_OP_EMBED, 3, 20, &c) == LSB_E_ARG, "invalid block order refused");
    }

    /* the serving scheduler on its modelled clock: four embeds, then two
     * extracts of the first two stegos */
    {
        lsb_server_cfg cfg;
        lsb_request req[6];
        lsb_result res[6];
        lsb_serve_stats st;
        memset(&cfg, 0, sizeof cfg);
        memset(req, 0, sizeof req);
        cfg.arena_bytes = 1u << 24;
        cfg.max_batch = 4;
        cfg.n_slots = 2;
        for (i = 0; i < 6; ++i) {
            req[i].arrival_s = 1e-4 * (double)i;
            req[i].n = 65536;
            req[i].cover_off = 65536 * (i % 4);
            req[i].msg_off = 4096 * (i % 4);
            req[i].len = 1000;
            req[i].k = 1;
            req[i].op = i < 4 ? LSB_OP_EMBED : LSB_OP_EXTRACT;
            req[i].target = i < 4 ? -1 : (int64_t)(i - 4);
        }
        bad += check(lsb_serve_simulate(&cfg, req, 6, res, &st, 5.0, 1000.0) == LSB_OK, "serve_simulate");
        for (i = 0; i < 6; ++i) bad += check(res[i].status == LSB_OK, "request served");
        bad += check(res[4].op_run == LSB_OP_EXTRACT && res[4].target == 0 && res[4].len == 1000, "extract of request 0");
        bad += check(res[5].op_run == LSB_OP_EXTRACT && res[5].target == 1, "extract of request 1");
        bad += check(st.launches >= 1 && st.p50_ms > 0 && st.p99_ms >= st.p50_ms, "latency figures");
    }
    if (bad) {
        fprintf(stderr, "%d checks failed\n", bad);
        return 1;
    }
    printf("ok\n");
    return 0;
}
