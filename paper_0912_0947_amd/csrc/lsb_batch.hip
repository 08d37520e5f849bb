// lsb_batch.hip -- batched embed/extract over thousands of covers of uneven
// size and k in one persistent launch.
//
// The paper loops on the host over the rows of an image (Section VI steps
// 4-5 split the data across rows; Section VII steps 3-4 likewise), paying a
// copy and a launch per row.  Here every cover of a batch is a job, each job
// is cut into tiles of T 16-byte vectors (2T for extract jobs), and one
// persistent grid walks the global tile list, each block taking the next
// tile from a counter.  Tile t of a job starts 16*T*t fields after the job's
// first field, a whole number of stream bytes, so no two tiles of a job share
// an output byte.  A job is a whole cover with its length header or a raw
// slice [t0, t0 + n) of a longer logical cover; slices of one stream may be
// spread over many jobs (the frames of a clip).
//
// One run: an asynchronous copy of the job table from the plan's pinned
// host mirror, only when the table changed since the last upload, then the
// persistent kernel.  The kernel also reports each job's status (and, for
// extract jobs, the decoded length), and its last block resets the tile
// counter, so a run whose table is already on the device is one kernel
// launch.  (While a prologue kernel ran before the persistent one, the run
// was a HIP graph of three nodes; with one kernel left, launching the graph
// cost about 25 us more host time per run than launching the kernel.)
#include <stddef.h>
#include <string.h>

#include <mutex>
#include <new>

#include "lsb_batch_device.hpp"

namespace lsb {

// Kernel for a launch shape, plan class and raw-slice support.
static BatchFn batch_fn(int unroll, int nt, int cls, bool raw) {
    return raw ? batch_fn_raw(unroll, nt, cls) : batch_fn_for<false>(unroll, nt, cls);
}

// Batched-kernel configuration (global, read at each run): the launch shape
// of plans with embed jobs (entry 0) and of extract-only plans (entry 1),
// and the tile size of both.
static std::mutex g_batch_mu;
static lsb_launch_cfg g_batch_cfg[2] = {{1024, 2, 2, 1, 0}, {1024, 4, 2, 1, 0}};
static int64_t g_tile_vectors = 4096;

// Launch shape of a plan: extract-only plans have their own entry.
static lsb_launch_cfg batch_cfg_for(bool has_embed, bool has_extract, int64_t *tv) {
    std::lock_guard<std::mutex> g(g_batch_mu);
    *tv = g_tile_vectors;
    return g_batch_cfg[has_extract && !has_embed ? 1 : 0];
}

}  // namespace lsb

using namespace lsb;

struct lsb_plan {
    int device = -1;
    int max_jobs = 0;
    int n_jobs = 0;
    int op_mode = LSB_OP_MIXED;  // LSB_OP_EMBED / LSB_OP_EXTRACT: every job of that kind
    bool has_extract = false;
    bool has_embed = false;
    bool has_raw = false;  // some job is a raw slice: the raw-capable kernels run
    int cls = 0;  // 1 + 8*op + (k-1) when every job shares (op, k); kClsExtractAnyK; else 0
    uint64_t total_tiles = 0;
    size_t table_bytes = 0;  // bytes of header + (max_jobs + 1) records
    size_t used_bytes = 0;   // bytes the next upload copies
    uint8_t *host = nullptr;  // pinned mirror of the device table
    uint8_t *dev = nullptr;
    hipEvent_t done = nullptr;  // recorded after each run
    hipStream_t last_stream = nullptr;  // stream of the last run
    bool ran = false;
    bool table_dirty = true;  // the host table changed since the last upload
    int64_t tile_vectors = 0;  // tile size the table was filled with
};

// ---------------------------------------------------------------------------
// Table of lsb_batch_run_static: the job table and tile counter live in this
// file-scope device array (one copy per device, held until the process
// ends) instead of plan memory.  Host code never uses the array's name as an
// address: static_table() looks up each device's copy once, with that
// device current, and the launches take that pointer.
constexpr size_t kStaticTableBytes = sizeof(PlanHeader) + sizeof(DevJob) * ((size_t)LSB_STATIC_MAX_JOBS + 1);
static __device__ __align__(256) uint8_t scratch[kStaticTableBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;                    // guards the two below and the launches' upload order
static uint8_t *g_static_dev[kMaxDevices] = {};  // device address of `scratch`, per device
alignas(256) static uint8_t g_static_host[kStaticTableBytes];  // host staging of the table

// Device address of the current device's copy of `scratch` (caller holds
// g_static_mu).
static int static_table(uint8_t **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(LSB_E_ARG, "lsb_batch_run_static: device %d not supported", dev);
    if (!g_static_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
        g_static_dev[dev] = (uint8_t *)ptr;
    }
    *out = g_static_dev[dev];
    return LSB_OK;
}

// Host-side checks of a job list (nothing is touched on failure).
static int validate_jobs(const lsb_job *jobs, int n_jobs, int op_mode) {
    for (int i = 0; i < n_jobs; ++i) {
        const lsb_job &J = jobs[i];
        if (J.k < 1 || J.k > 8) return fail(LSB_E_ARG, "job %d: k=%d outside 1..8", i, (int)J.k);
        if (op_mode == LSB_OP_MIXED && J.op != LSB_OP_EMBED && J.op != LSB_OP_EXTRACT)
            return fail(LSB_E_ARG, "job %d: bad op %d", i, (int)J.op);
        if ((J.cover_off | J.stego_off | J.msg_off) & 255)
            return fail(LSB_E_ARG, "job %d: arena offsets must be multiples of 256", i);
        if (J.n > (1ull << 48)) return fail(LSB_E_ARG, "job %d: n out of range", i);
        if (J.reserved) return fail(LSB_E_ARG, "job %d: reserved field must be 0", i);
        if (J.flags & ~LSB_JOB_RAW) return fail(LSB_E_ARG, "job %d: unknown flags 0x%x", i, (unsigned)J.flags);
        if (!(J.flags & LSB_JOB_RAW)) {
            if (J.t0 || J.stream_bits) return fail(LSB_E_ARG, "job %d: t0/stream_bits set on a header job", i);
            continue;
        }
        if (J.t0 > (1ull << 56) || J.stream_bits > (1ull << 60))
            return fail(LSB_E_ARG, "job %d: t0/stream_bits out of range", i);
        const uint8_t op = op_mode == LSB_OP_MIXED ? J.op : (uint8_t)op_mode;
        if (op == LSB_OP_EXTRACT) {
            // slices of one stream may not share an output byte
            const uint64_t begin = (uint64_t)J.k * J.t0;
            uint64_t end = (uint64_t)J.k * (J.t0 + J.n);
            if (end > J.stream_bits) end = J.stream_bits;
            if (begin % 8) return fail(LSB_E_ARG, "job %d: raw extract with k*t0 not byte aligned", i);
            if (begin < end && end % 8 && end != J.stream_bits)
                return fail(LSB_E_ARG, "job %d: raw extract ends inside a stream byte", i);
        }
    }
    return LSB_OK;
}

// What a filled job table holds, for the launch.
struct TableInfo {
    uint64_t tiles = 0;
    bool has_extract = false, has_embed = false, has_raw = false;
    int cls = 0;            // kernel class (see lsb_batch_device.hpp)
    size_t used_bytes = 0;  // header + (n_jobs + 1) records
};

// Fill a job table (header, records, sentinel) at `host` for validated
// jobs: per-job status for work the host can already refuse, tile counts
// and their exclusive prefix, the kernel class.  The header's tile counter
// is zero, so uploading the table resets it.
static TableInfo fill_table(const lsb_job *jobs, int n_jobs, int op_mode, int64_t tv, uint8_t *host) {
    PlanHeader *h = (PlanHeader *)host;
    DevJob *d = (DevJob *)(host + sizeof(PlanHeader));
    TableInfo t;
    uint64_t tiles = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const lsb_job &J = jobs[i];
        const uint8_t op = op_mode == LSB_OP_MIXED ? J.op : (uint8_t)op_mode;
        DevJob &D = d[i];
        memset(&D, 0, sizeof D);
        D.cover_off = J.cover_off;
        D.stego_off = J.stego_off;
        D.msg_off = J.msg_off;
        D.n = J.n;
        D.raw = (J.flags & LSB_JOB_RAW) ? 1 : 0;
        t.has_raw |= D.raw != 0;
        D.len = D.raw ? 0 : J.len;  // what the kernel reports in len_dev
        D.k = J.k;
        D.op = op;
        D.tile_begin = tiles;
        D.status = LSB_OK;
        uint64_t vectors = ceil_div(J.n, 16);
        if (D.raw) {
            D.t0 = J.t0;
            if (op == LSB_OP_EMBED) {
                t.has_embed = true;
                D.cap_bits = J.stream_bits;  // stream bits past the slice fall back to copies
            } else {
                t.has_extract = true;
                const uint64_t begin = (uint64_t)J.k * J.t0;
                uint64_t end = (uint64_t)J.k * (J.t0 + J.n);
                if (end > J.stream_bits) end = J.stream_bits;
                D.cap_bits = end;
                // only the fields that carry stream bits [begin, end) are read
                const uint64_t fields = end > begin ? ceil_div(end - begin, (uint64_t)J.k) : 0;
                const uint64_t v_stream = ceil_div(fields, 16);
                if (v_stream < vectors) vectors = v_stream;
            }
        } else if (op == LSB_OP_EMBED) {
            D.cap_bits = 0;
            t.has_embed = true;
            const uint64_t room = room_bytes(J.n, J.k);
            if (room < 4 || (uint64_t)J.len > room - 4) {
                D.status = LSB_E_CAPACITY;
                vectors = 0;
            }
        } else {
            t.has_extract = true;
            D.cap_bits = J.msg_cap;
            // worst case: the stream may fill the cover or the output buffer
            const uint64_t room = room_bytes(J.n, J.k);
            const uint64_t cap = room >= 4 ? room - 4 : 0;
            const uint64_t max_len = J.msg_cap < cap ? J.msg_cap : cap;
            const uint64_t v_stream = ceil_div(4 + max_len, 2 * (uint64_t)J.k);
            if (v_stream < vectors) vectors = v_stream;
            if ((uint64_t)J.k * J.n < 32) vectors = 0;
        }
        // an extract tile moves about half the bytes of an embed tile (no
        // stego write), so it covers twice the vectors to carry the same
        // traffic per job lookup
        const uint64_t jtv = op == LSB_OP_EMBED ? (uint64_t)tv : 2 * (uint64_t)tv;
        tiles += ceil_div(vectors, jtv);
    }
    DevJob &S = d[n_jobs];  // sentinel
    memset(&S, 0, sizeof S);
    S.tile_begin = tiles;
    memset(h, 0, sizeof *h);
    h->n_jobs = (uint64_t)n_jobs;
    h->total_tiles = tiles;
    h->tile_vectors = (uint64_t)tv;
    t.tiles = tiles;
    if (n_jobs > 0) {
        bool same = true;
        bool same_op = true;
        for (int i = 1; i < n_jobs && same; ++i) same = d[i].op == d[0].op && d[i].k == d[0].k;
        for (int i = 1; i < n_jobs && same_op; ++i) same_op = d[i].op == d[0].op;
        if (same) t.cls = 1 + 8 * d[0].op + (d[0].k - 1);
        else if (same_op && d[0].op == LSB_OP_EXTRACT) t.cls = kClsExtractAnyK;
    }
    t.used_bytes = sizeof(PlanHeader) + sizeof(DevJob) * ((size_t)n_jobs + 1);
    return t;
}

// Grid of the persistent kernel: capped at blocks_per_cu blocks per CU,
// never more blocks than tiles.
static unsigned main_grid_for(const lsb_launch_cfg &cfg, uint64_t total_tiles) {
    const uint64_t cap_blocks = (uint64_t)(cfg.blocks_per_cu > 0 ? cfg.blocks_per_cu : 8) * (uint64_t)device_cus();
    return (unsigned)(total_tiles < cap_blocks ? (total_tiles ? total_tiles : 1) : cap_blocks);
}

static int64_t batch_tile_vectors() {
    std::lock_guard<std::mutex> g(g_batch_mu);
    return g_tile_vectors;
}

extern "C" {

int lsb_plan_create(lsb_plan **out, const lsb_job *jobs, int n_jobs, int op) {
    clear_error();
    if (!out) return fail(LSB_E_ARG, "lsb_plan_create: null plan pointer");
    *out = nullptr;
    if (n_jobs < 1 || n_jobs > (1 << 24)) return fail(LSB_E_ARG, "lsb_plan_create: n_jobs=%d", n_jobs);
    if (op != LSB_OP_EMBED && op != LSB_OP_EXTRACT && op != LSB_OP_MIXED)
        return fail(LSB_E_ARG, "lsb_plan_create: op=%d", op);
    lsb_plan *p = new (std::nothrow) lsb_plan();
    if (!p) return fail(LSB_E_NOMEM, "lsb_plan_create: out of host memory");
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) return delete p, hip_fail(e, "hipGetDevice");
    p->max_jobs = n_jobs;
    p->op_mode = op;
    p->table_bytes = sizeof(PlanHeader) + sizeof(DevJob) * ((size_t)n_jobs + 1);
    e = hipHostMalloc((void **)&p->host, p->table_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return delete p, fail(LSB_E_NOMEM, "lsb_plan_create: hipHostMalloc failed");
    e = hipMalloc((void **)&p->dev, p->table_bytes);
    if (e != hipSuccess)
        return (void)hipHostFree(p->host), delete p, fail(LSB_E_NOMEM, "lsb_plan_create: hipMalloc failed");
    e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) return (void)hipFree(p->dev), (void)hipHostFree(p->host), delete p, hip_fail(e, "hipEventCreate");
    memset(p->host, 0, p->table_bytes);
    p->used_bytes = sizeof(PlanHeader) + sizeof(DevJob);
    if (jobs) {
        const int rc = lsb_plan_update(p, jobs, n_jobs);
        if (rc != LSB_OK) {
            lsb_plan_destroy(p);
            return rc;
        }
    }
    *out = p;
    return LSB_OK;
}

int lsb_plan_update(lsb_plan *p, const lsb_job *jobs, int n_jobs) {
    clear_error();
    if (!p) return fail(LSB_E_ARG, "lsb_plan_update: null plan");
    if (n_jobs < 0 || n_jobs > p->max_jobs)
        return fail(LSB_E_ARG, "lsb_plan_update: n_jobs=%d outside 0..%d", n_jobs, p->max_jobs);
    if (n_jobs && !jobs) return fail(LSB_E_ARG, "lsb_plan_update: null job list");
    const int64_t tv = batch_tile_vectors();
    // validate everything before touching the mirror
    const int rc = validate_jobs(jobs, n_jobs, p->op_mode);
    if (rc != LSB_OK) return rc;
    // the previous run's upload must have read the mirror before it changes
    if (p->ran) {
        hipError_t e = hipEventSynchronize(p->done);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(plan)");
    }
    const TableInfo t = fill_table(jobs, n_jobs, p->op_mode, tv, p->host);
    p->n_jobs = n_jobs;
    p->total_tiles = t.tiles;
    p->has_extract = t.has_extract;
    p->has_embed = t.has_embed;
    p->has_raw = t.has_raw;
    p->cls = t.cls;
    p->tile_vectors = tv;
    p->used_bytes = t.used_bytes;
    p->table_dirty = true;
    return LSB_OK;
}

int64_t lsb_plan_tiles(const lsb_plan *p) { return p ? (int64_t)p->total_tiles : fail(LSB_E_ARG, "null plan"); }

int lsb_job_extents(const lsb_job *jobs, int n_jobs, int op, uint64_t *extents) {
    clear_error();
    if (!extents || (n_jobs && !jobs) || n_jobs < 0) return fail(LSB_E_ARG, "lsb_job_extents: null argument");
    if (op != LSB_OP_EMBED && op != LSB_OP_EXTRACT && op != LSB_OP_MIXED)
        return fail(LSB_E_ARG, "lsb_job_extents: op=%d", op);
    uint64_t cover = 0, stego = 0, msg = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const lsb_job &J = jobs[i];
        if (J.k < 1 || J.k > 8) return fail(LSB_E_ARG, "job %d: k=%d outside 1..8", i, (int)J.k);
        const uint8_t jop = op == LSB_OP_MIXED ? J.op : (uint8_t)op;
        if (jop != LSB_OP_EMBED && jop != LSB_OP_EXTRACT) return fail(LSB_E_ARG, "job %d: bad op %d", i, (int)J.op);
        if (J.n > (1ull << 48) || J.cover_off >= (1ull << 62) || J.stego_off >= (1ull << 62) ||
            J.msg_off >= (1ull << 62) || J.t0 > (1ull << 56) || J.stream_bits > (1ull << 60))
            return fail(LSB_E_ARG, "job %d: offset or size out of range", i);
        if (!J.n) continue;
        const uint64_t k = J.k;
        uint64_t mbytes;  // message-arena bytes from msg_off that the job reads or writes
        if (J.flags & LSB_JOB_RAW) {
            // stream bytes k*t0/8 .. ceil(min(k*(t0+n), stream_bits)/8) - 1
            const uint64_t begin = k * J.t0;
            uint64_t end = k * (J.t0 + J.n);
            if (end > J.stream_bits) end = J.stream_bits;
            mbytes = end > begin ? ceil_div(end, 8) : 0;
        } else {
            const uint64_t room = room_bytes(J.n, J.k);
            uint64_t cap = room >= 4 ? room - 4 : 0;
            if (cap > 0xFFFFFFFFull) cap = 0xFFFFFFFFull;
            if (jop == LSB_OP_EMBED) mbytes = (uint64_t)J.len <= cap ? J.len : 0;  // over capacity: no work
            else mbytes = J.msg_cap < cap ? J.msg_cap : cap;
        }
        if (jop == LSB_OP_EMBED && J.cover_off + J.n > cover) cover = J.cover_off + J.n;
        if (J.stego_off + J.n > stego) stego = J.stego_off + J.n;
        if (mbytes && J.msg_off + mbytes > msg) msg = J.msg_off + mbytes;
    }
    extents[0] = cover;
    extents[1] = stego;
    extents[2] = msg;
    return LSB_OK;
}

int lsb_plan_run(lsb_plan *p, const uint8_t *cover_arena, uint8_t *stego_arena, uint8_t *msg_arena, uint32_t *len_dev,
                 int32_t *status_dev, void *stream) {
    clear_error();
    if (!p) return fail(LSB_E_ARG, "lsb_plan_run: null plan");
    if (p->n_jobs == 0) return LSB_OK;
    if (!status_dev) return fail(LSB_E_ARG, "lsb_plan_run: null status_dev");
    if (p->has_extract && !len_dev) return fail(LSB_E_ARG, "lsb_plan_run: extract jobs need len_dev");
    if (!stego_arena || !msg_arena) return fail(LSB_E_ARG, "lsb_plan_run: null arena");
    if (p->has_embed && !cover_arena) return fail(LSB_E_ARG, "lsb_plan_run: embed jobs need a cover arena");
    if (((uintptr_t)cover_arena | (uintptr_t)stego_arena | (uintptr_t)msg_arena) & 255)
        return fail(LSB_E_ARG, "lsb_plan_run: arena base pointers must be 256-byte aligned");
    int dev = -1;
    const hipError_t de = hipGetDevice(&dev);
    if (de != hipSuccess) return hip_fail(de, "hipGetDevice");
    if (dev != p->device) return fail(LSB_E_ARG, "lsb_plan_run: plan belongs to device %d, current is %d", p->device, dev);
    int64_t tv;
    const lsb_launch_cfg cfg = batch_cfg_for(p->has_embed, p->has_extract, &tv);
    if (tv != p->tile_vectors) return fail(LSB_E_ARG, "lsb_plan_run: tile size changed since lsb_plan_update");
    hipStream_t st = (hipStream_t)stream;
    // A captured run would replay its upload and kernel outside the plan's
    // tracking (the upload state, the completion event that updates wait
    // for, the kernel chosen for the table's class): refused before
    // anything is enqueued.
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    const hipError_t ce = hipStreamIsCapturing(st, &capture);
    if (ce != hipSuccess) return hip_fail(ce, "hipStreamIsCapturing");
    if (capture != hipStreamCaptureStatusNone)
        return fail(LSB_E_ARG, "lsb_plan_run: the stream is capturing a graph (a captured run would replay outside "
                               "the plan's tracking of its table and runs)");
    const BatchFn fn = batch_fn(cfg.unroll, cfg.nontemporal, p->cls, p->has_raw);
    const PlanHeader *hdr = (const PlanHeader *)p->dev;
    const DevJob *jobs = (const DevJob *)(p->dev + sizeof(PlanHeader));
    hipError_t e;
    if (p->ran && st != p->last_stream) {
        // every run shares the device job table and its tile counters: a run
        // on another stream starts only after the previous run has finished
        e = hipStreamWaitEvent(st, p->done, 0);
        if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(plan)");
    }
    // upload the job table only when it changed since the last upload (the
    // kernel's last block resets the tile counters either way)
    const bool upload = p->table_dirty;
    if (upload) {
        e = hipMemcpyAsync(p->dev, p->host, p->used_bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(job table)");
    }
    void *argv[] = {&hdr, &jobs, &cover_arena, &stego_arena, &msg_arena, &len_dev, &status_dev};
    e = hipLaunchKernel((const void *)fn, dim3(main_grid_for(cfg, p->total_tiles)), dim3(cfg.block), argv, 0, st);
    if (e != hipSuccess) {
        // an enqueued upload still reads the pinned mirror: let it finish
        // before a later update may refill the mirror
        if (upload) (void)hipStreamSynchronize(st);
        return hip_fail(e, "persistent kernel launch");
    }
    e = hipEventRecord(p->done, st);
    if (e != hipSuccess) {
        // without the event nothing tracks the launch: wait for it here so
        // that a later update or destroy cannot overtake it
        (void)hipStreamSynchronize(st);
        return hip_fail(e, "hipEventRecord(plan)");
    }
    p->ran = true;
    p->table_dirty = false;
    p->last_stream = st;
    return LSB_OK;
}

int lsb_embed_batch(lsb_plan *p, const uint8_t *cover_arena, uint8_t *stego_arena, const uint8_t *msg_arena,
                    int32_t *status_dev, void *stream) {
    clear_error();
    if (!p) return fail(LSB_E_ARG, "lsb_embed_batch: null plan");
    if (p->has_extract) return fail(LSB_E_ARG, "lsb_embed_batch: the plan holds extract jobs");
    if (p->n_jobs && !cover_arena) return fail(LSB_E_ARG, "lsb_embed_batch: null cover arena");
    // embed jobs only read the message arena
    return lsb_plan_run(p, cover_arena, stego_arena, const_cast<uint8_t *>(msg_arena), nullptr, status_dev, stream);
}

int lsb_extract_batch(lsb_plan *p, const uint8_t *stego_arena, uint8_t *msg_arena, uint32_t *len_dev,
                      int32_t *status_dev, void *stream) {
    clear_error();
    if (!p) return fail(LSB_E_ARG, "lsb_extract_batch: null plan");
    if (p->has_embed) return fail(LSB_E_ARG, "lsb_extract_batch: the plan holds embed jobs");
    if (p->n_jobs && !len_dev) return fail(LSB_E_ARG, "lsb_extract_batch: null len_dev");
    // extract jobs only read the stego arena
    return lsb_plan_run(p, nullptr, const_cast<uint8_t *>(stego_arena), msg_arena, len_dev, status_dev, stream);
}

void lsb_plan_destroy(lsb_plan *p) {
    if (!p) return;
    // teardown: nothing useful can be done with a failure here
    if (p->ran) (void)hipEventSynchronize(p->done);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->dev) (void)hipFree(p->dev);
    if (p->host) (void)hipHostFree(p->host);
    delete p;
}

int lsb_batch_run_static(const lsb_job *jobs, int n_jobs, int op, const uint8_t *cover_arena,
                         uint8_t *stego_arena, uint8_t *msg_arena, uint32_t *len_dev, int32_t *status_dev,
                         void *stream) {
    clear_error();
    if (op != LSB_OP_EMBED && op != LSB_OP_EXTRACT && op != LSB_OP_MIXED)
        return fail(LSB_E_ARG, "lsb_batch_run_static: op=%d", op);
    if (n_jobs < 0 || n_jobs > LSB_STATIC_MAX_JOBS)
        return fail(LSB_E_ARG, "lsb_batch_run_static: n_jobs=%d outside 0..%d (larger batches need a plan)", n_jobs,
                    LSB_STATIC_MAX_JOBS);
    if (n_jobs == 0) return LSB_OK;
    if (!jobs) return fail(LSB_E_ARG, "lsb_batch_run_static: null job list");
    if (!status_dev) return fail(LSB_E_ARG, "lsb_batch_run_static: null status_dev");
    if (!stego_arena || !msg_arena) return fail(LSB_E_ARG, "lsb_batch_run_static: null arena");
    if (((uintptr_t)cover_arena | (uintptr_t)stego_arena | (uintptr_t)msg_arena) & 255)
        return fail(LSB_E_ARG, "lsb_batch_run_static: arena base pointers must be 256-byte aligned");
    int rc = validate_jobs(jobs, n_jobs, op);
    if (rc != LSB_OK) return rc;
    const int64_t tv = batch_tile_vectors();
    hipStream_t st = (hipStream_t)stream;
    // Under stream capture the table upload would become a graph node that
    // reads the staging buffer below at every replay, after later calls may
    // have refilled it: such a call is refused before anything is enqueued.
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(st, &capture);
    if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
    if (capture != hipStreamCaptureStatusNone)
        return fail(LSB_E_ARG, "lsb_batch_run_static: the stream is capturing a graph (the job table's upload "
                               "would read a shared staging buffer at each replay)");
    // One host staging table for all devices: filled and uploaded under the
    // lock.  An upload from pageable memory has read the source when
    // hipMemcpyAsync returns, so the next call may refill it.
    std::lock_guard<std::mutex> g(g_static_mu);
    uint8_t *table = nullptr;
    rc = static_table(&table);
    if (rc != LSB_OK) return rc;
    const TableInfo t = fill_table(jobs, n_jobs, op, tv, g_static_host);
    int64_t tv_now;
    const lsb_launch_cfg cfg = batch_cfg_for(t.has_embed, t.has_extract, &tv_now);
    if (tv_now != tv) return fail(LSB_E_ARG, "lsb_batch_run_static: tile size changed during the call");
    if (t.has_extract && !len_dev) return fail(LSB_E_ARG, "lsb_batch_run_static: extract jobs need len_dev");
    if (t.has_embed && !cover_arena) return fail(LSB_E_ARG, "lsb_batch_run_static: embed jobs need a cover arena");
    e = hipMemcpyAsync(table, g_static_host, t.used_bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(static job table)");
    const PlanHeader *hdr = (const PlanHeader *)table;
    const DevJob *dj = (const DevJob *)(table + sizeof(PlanHeader));
    const BatchFn fn = batch_fn(cfg.unroll, cfg.nontemporal, t.cls, t.has_raw);
    void *main_args[] = {&hdr, &dj, &cover_arena, &stego_arena, &msg_arena, &len_dev, &status_dev};
    e = hipLaunchKernel((const void *)fn, dim3(main_grid_for(cfg, t.tiles)), dim3(cfg.block), main_args, 0, st);
    if (e != hipSuccess) return hip_fail(e, "persistent kernel launch");
    return LSB_OK;
}

int lsb_batch_tune_get(lsb_launch_cfg *cfg, int64_t *tile_vectors) {
    std::lock_guard<std::mutex> g(g_batch_mu);
    if (cfg) *cfg = g_batch_cfg[0];
    if (tile_vectors) *tile_vectors = g_tile_vectors;
    return LSB_OK;
}

static bool batch_cfg_valid(const lsb_launch_cfg *cfg) {
    // one wave of every block hands out tiles, the others stream them
    return cfg && cfg_valid(*cfg) && cfg->block >= 128;
}

int lsb_batch_tune_set(const lsb_launch_cfg *cfg, int64_t tile_vectors) {
    if (!batch_cfg_valid(cfg))
        return fail(LSB_E_ARG, "lsb_batch_tune_set: invalid configuration (blocks need at least 128 threads)");
    if (tile_vectors < 64 || tile_vectors > (1ll << 30) || tile_vectors % 64)
        return fail(LSB_E_ARG, "lsb_batch_tune_set: tile_vectors must be a multiple of 64 in [64, 2^30]");
    std::lock_guard<std::mutex> g(g_batch_mu);
    g_batch_cfg[0] = g_batch_cfg[1] = *cfg;
    g_tile_vectors = tile_vectors;
    return LSB_OK;
}

int lsb_batch_tune_get_op(int op, lsb_launch_cfg *cfg) {
    if ((op != LSB_OP_EMBED && op != LSB_OP_EXTRACT) || !cfg) return fail(LSB_E_ARG, "lsb_batch_tune_get_op: bad op or null");
    std::lock_guard<std::mutex> g(g_batch_mu);
    *cfg = g_batch_cfg[op == LSB_OP_EXTRACT ? 1 : 0];
    return LSB_OK;
}

int lsb_batch_tune_set_op(int op, const lsb_launch_cfg *cfg) {
    if (op != LSB_OP_EMBED && op != LSB_OP_EXTRACT) return fail(LSB_E_ARG, "lsb_batch_tune_set_op: op=%d", op);
    if (!batch_cfg_valid(cfg))
        return fail(LSB_E_ARG, "lsb_batch_tune_set_op: invalid configuration (blocks need at least 128 threads)");
    std::lock_guard<std::mutex> g(g_batch_mu);
    g_batch_cfg[op == LSB_OP_EXTRACT ? 1 : 0] = *cfg;
    return LSB_OK;
}

}  // extern "C"
