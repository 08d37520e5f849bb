/*
 * lsb.h -- C ABI of liblsb.so: k-bit least-significant-bit embedding and
 * extraction on AMD Instinct MI355X (gfx950).
 *
 * The operation is the one of Patel, Pradhan and Ambegaokar, "A Novel
 * Approach for Implementing Steganography with Computing Power Obtained by
 * Combining CUDA and MATLAB" (arXiv:0912.0947):
 *   - embedding (Section VI, step 7): each cover byte keeps its high bits and
 *     takes a piece of the data in its low bits (the paper: 2 bits, masks
 *     1111 1100 / 0000 0011); here the field width k is a parameter, 1..8;
 *   - extraction (Section VII, step 6): the low bits of each stego byte are
 *     masked, shifted into place and ORed into zero-initialised data bytes;
 *   - capacity (Section VI step 5, Section VII step 4): at 2 bits per byte a
 *     data byte needs 4 cover bytes; in general n cover bytes hold n*k bits.
 *
 * Readings fixed by this library where the paper is silent:
 *   - stream S = BE32(len) || msg: a 32-bit big-endian byte count, then the
 *     message; bits are read most-significant first;
 *   - cover layout: flat bytes (an HWC image or video frame in raster order,
 *     every channel byte carries data); cover byte t carries stream bits
 *     k*t .. k*t+k-1, the first of them in the highest bit of the k-bit field;
 *   - F = ceil(8*|S| / k) cover bytes carry the stream; if k does not divide
 *     8*|S|, the last field carries nb < k bits in its top nb bits and keeps
 *     the cover's other low bits; bytes t >= F are copied unchanged.
 *
 * Conventions for every call below:
 *   - Buffer pointers are DEVICE pointers owned by the caller (for example
 *     torch uint8 tensors on the GPU); the library never frees them.  Plain
 *     embed/extract calls never allocate.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls enqueue work and return after host-side validation; results are
 *     ready once the stream reaches that point.
 *   - Return value: LSB_OK (0) once enqueued, or a negative LSB_E_* code, in
 *     which case nothing was enqueued and outputs are untouched.  No C++
 *     exception crosses the ABI.  lsb_last_error() gives a message for the
 *     last failed call on the calling thread.
 *   - Any alignment is accepted.  The fast kernels need the cover and stego
 *     (or stego) pointers 16-byte aligned; otherwise a per-byte kernel runs
 *     (same results, lower bandwidth).
 *   - Threads: every call may be made from several host threads at once,
 *     except that one lsb_plan is used by one thread at a time (distinct
 *     plans are independent).  The shared state is the launch-configuration
 *     tables (guarded; a launch uses the entry current at its call) and
 *     per-thread state (error message, lsb_time_next_launch events,
 *     lsb_extract_sync buffer).
 *   - Devices: calls launch on the current HIP device; a plan belongs to the
 *     device current when it was created.
 */
#ifndef LSB_H
#define LSB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LSB_OK = 0,
    LSB_E_ARG = -1,      /* bad argument: k outside 1..8, null or overlapping buffers */
    LSB_E_CAPACITY = -2, /* message longer than the cover can hold */
    LSB_E_HEADER = -3,   /* decoded length does not fit the stego cover */
    LSB_E_BUFFER = -4,   /* decoded length exceeds the output buffer */
    LSB_E_HIP = -5,      /* a HIP runtime call failed */
    LSB_E_NOMEM = -6     /* a plan could not be allocated */
};

enum { LSB_OP_EMBED = 0, LSB_OP_EXTRACT = 1, LSB_OP_MIXED = 2 };

/* Message capacity in bytes of an n-byte cover at k bits per byte:
 * floor(n*k/8) - 4, capped at 2^32 - 1 by the header width (Section VI step 5
 * generalised).  LSB_E_ARG if k is outside 1..8; LSB_E_CAPACITY if
 * floor(n*k/8) < 4.  Host-only; touches no GPU. */
int64_t lsb_capacity(uint64_t n, int k);

/* Embed msg[0..len) into cover[0..n) at k bits per byte, writing
 * stego[0..n) (Section VI step 7).  stego == cover is the in-place form: only
 * bytes t < F are rewritten.  Any other overlap between cover, stego and msg
 * is LSB_E_ARG.  len > lsb_capacity(n, k) is LSB_E_CAPACITY. */
int lsb_embed(const uint8_t *cover, uint8_t *stego, uint64_t n,
              const uint8_t *msg, uint32_t len, int k, void *stream);

/* Extract the message from stego[0..n) (Section VII step 6).  The 32-bit
 * header is decoded on the device; nothing returns to the host.  When the
 * stream is done: *len_out_dev = decoded length (0 if n*k < 32) and
 * *status_out_dev = LSB_OK, LSB_E_HEADER (length does not fit the cover;
 * msg_out untouched) or LSB_E_BUFFER (length > out_cap; msg_out untouched).
 * msg_out may be NULL when out_cap == 0. */
int lsb_extract(const uint8_t *stego, uint64_t n, int k, uint8_t *msg_out,
                uint64_t out_cap, uint32_t *len_out_dev,
                int32_t *status_out_dev, void *stream);

/* As lsb_extract, then waits for the stream and returns the device status
 * as the return value (LSB_OK, LSB_E_HEADER, LSB_E_BUFFER) with the decoded
 * length in *len_out_host.  Uses a small per-thread device buffer that is
 * allocated on the first call. */
int lsb_extract_sync(const uint8_t *stego, uint64_t n, int k,
                     uint8_t *msg_out, uint64_t out_cap,
                     uint32_t *len_out_host, void *stream);

/* Raw slices: no header.  The buffer holds cover bytes [t0, t0+n) of a
 * longer logical cover (one video frame of a clip, one shard of a cover);
 * `stream_bytes` points at byte 0 of a logical stream of `stream_bits` bits.
 * Buffer byte t carries stream bits k*(t0+t) .. k*(t0+t)+k-1.
 *
 * lsb_embed_raw: stego[t] as in lsb_embed for stream bits < stream_bits,
 * cover[t] past them; any t0.  Reads stream bytes k*t0/8 onwards only.
 *
 * lsb_extract_raw: writes stream bits [k*t0, e), e = min(k*(t0+n),
 * stream_bits), into stream_out (byte 0 = logical byte 0), i.e. bytes
 * k*t0/8 .. ceil(e/8)-1, pad bits past stream_bits as zero.  Requires
 * k*t0 % 8 == 0 and (e % 8 == 0 or e == stream_bits), so that slices never
 * share an output byte; LSB_E_ARG otherwise. */
int lsb_embed_raw(const uint8_t *cover, uint8_t *stego, uint64_t n,
                  uint64_t t0, const uint8_t *stream_bytes,
                  uint64_t stream_bits, int k, void *stream);
int lsb_extract_raw(const uint8_t *stego, uint64_t n, uint64_t t0,
                    uint8_t *stream_out, uint64_t stream_bits, int k,
                    void *stream);

/* Bytes of a logical stream that a raw slice touches, counted from stream
 * byte 0: ceil(min(k*(t0+n), stream_bits) / 8), or 0 when the slice carries
 * no stream bit (k*(t0+n) <= k*t0 or stream_bits <= k*t0).  The stream
 * buffer passed to lsb_embed_raw / lsb_extract_raw must hold at least this
 * many bytes.  LSB_E_ARG for k outside 1..8 or t0, n, stream_bits beyond
 * the raw calls' ranges (2^56, 2^56, 2^60).  Host-only. */
int64_t lsb_slice_stream_bytes(int k, uint64_t t0, uint64_t n,
                               uint64_t stream_bits);

/* ------------------------------------------------------------------------
 * The paper's own layout (Section VI steps 2-7, Section VII steps 2-6), kept
 * for fidelity: 2 bits per byte in ONE colour plane `plane` of an h x w x c
 * HWC image; the data is split greedily over the rows in order, row y taking
 * L = min(remaining, floor(w/4)) bytes (Section VI step 5: size(B)*4 <=
 * size(A)); bit pair i (bits 2i+1..2i) of the row's data byte j goes to the
 * low two bits of plane pixel L*i + j of that row.  No length header: the
 * caller passes `len`, as the paper's extract call passes N.
 *
 * lsb_paper_capacity: h * floor(w/4) bytes.  Host-only.
 * lsb_paper_embed: stego = cover with the data placed as above; every other
 *   byte copied (stego == cover: in place).  LSB_E_CAPACITY if len exceeds
 *   the capacity, LSB_E_ARG if plane >= c, h*w*c > 2^48 or buffers overlap
 *   otherwise.
 * lsb_paper_extract: data_out[0..len) from the stego image (data_out's
 *   bytes are all written).
 */
int64_t lsb_paper_capacity(uint32_t h, uint32_t w);
int lsb_paper_embed(const uint8_t *cover, uint8_t *stego, uint32_t h,
                    uint32_t w, uint32_t c, uint32_t plane,
                    const uint8_t *data, uint64_t len, void *stream);
int lsb_paper_extract(const uint8_t *stego, uint32_t h, uint32_t w,
                      uint32_t c, uint32_t plane, uint8_t *data_out,
                      uint64_t len, void *stream);

/* ------------------------------------------------------------------------
 * One colour plane with the general method (the paper separates one plane
 * before embedding, Section VI step 2 / Section VII step 2): the fields are
 * the bytes p*c + plane of an HWC image of `pixels` pixels, in raster order;
 * stream, header, bit order and errors as lsb_embed / lsb_extract, with the
 * capacity lsb_capacity(pixels, k).  lsb_embed_plane copies the other bytes
 * (stego == cover: in place, only plane bytes are rewritten).  LSB_E_ARG
 * also for plane >= c, pixels > 2^48 or c > 65536.
 */
int lsb_embed_plane(const uint8_t *cover, uint8_t *stego, uint64_t pixels,
                    uint32_t c, uint32_t plane, const uint8_t *msg,
                    uint32_t len, int k, void *stream);
int lsb_extract_plane(const uint8_t *stego, uint64_t pixels, uint32_t c,
                      uint32_t plane, int k, uint8_t *msg_out,
                      uint64_t out_cap, uint32_t *len_out_dev,
                      int32_t *status_out_dev, void *stream);

/* Sum over i < n of (a[i] - b[i])^2 into the device word *sse_dev (which
 * the call overwrites).  The paper's quality figure (Section VIII) is
 * PSNR = 10*log10(255^2 * count / sse), with count the bytes the mean is
 * taken over (all bytes of the cover). */
int lsb_sse(const uint8_t *a, const uint8_t *b, uint64_t n, uint64_t *sse_dev,
            void *stream);

/* ------------------------------------------------------------------------
 * Host-streamed video (the paper's copy-in / launch / copy-out flow of
 * Sections III and V, pipelined): `frames` frames of `frame_bytes` bytes in
 * pinned host memory are embedded in place as raw slices t0 = f *
 * frame_bytes of one logical stream (stream_dev, a device buffer of
 * stream_bits bits) and copied back to host_stego.  Frame f goes to stream
 * streams[f % n_streams] (1 <= n_streams <= 16, distinct streams), which
 * copies it into ring slot f % ring_slots (dev_ring holds ring_slots *
 * frame_bytes bytes), embeds it and copies it back, in stream order.
 * ring_slots must be a positive multiple of n_streams, so that a slot is
 * only reused by a later frame of the same stream: no events or cross-stream
 * waits are needed, and the copies of different streams run in both PCIe
 * directions at once.  Returns after enqueueing; host_stego is complete once
 * every stream has drained.  Errors: LSB_E_ARG. */
int lsb_video_embed_host(const uint8_t *host_frames, uint8_t *host_stego,
                         uint64_t frame_bytes, uint64_t frames,
                         const uint8_t *stream_dev, uint64_t stream_bits, int k,
                         uint8_t *dev_ring, uint32_t ring_slots,
                         void *const *streams, int n_streams);

/* ------------------------------------------------------------------------
 * Round-trip checks in one launch (extraction, Section VII step 6, is the
 * reverse of embedding, Section VI step 7).  A stego byte is counted as
 * wrong unless (a) the bits of its field that carry stream bits, read back
 * as extraction reads them, equal those bits of S = BE32(len) || msg, and
 * (b) every other bit equals the cover byte's (bytes past the stream: the
 * whole byte).  Both checks run on the extraction side of the method, so a
 * wrong embedding is caught, not reproduced.  *mismatches_dev (a device
 * word, overwritten) receives the count; 0 means that extraction returns msg
 * and that the stego differs from the cover only where the stream is.
 * Errors as lsb_embed (k, capacity, null or overlapping buffers, also the
 * counter overlapping any buffer).
 *
 * lsb_verify: checks an existing stego buffer (read only).  Reads cover,
 * stego and the stream once (2n + |S| bytes).
 *
 * lsb_embed_verify: lsb_embed(cover, stego, n, msg, len, k) and, in the same
 * launch, the check of every byte it writes (each vector is extracted again
 * in registers right after it is embedded).  stego == cover is the in-place
 * form.  Same memory traffic as lsb_embed (2n + |S|; in place 2F + |S|). */
int lsb_verify(const uint8_t *cover, const uint8_t *stego, uint64_t n,
               const uint8_t *msg, uint32_t len, int k,
               uint64_t *mismatches_dev, void *stream);
int lsb_embed_verify(const uint8_t *cover, uint8_t *stego, uint64_t n,
                     const uint8_t *msg, uint32_t len, int k,
                     uint64_t *mismatches_dev, void *stream);

/* ------------------------------------------------------------------------
 * Batched form: thousands of covers of uneven size and k in one persistent
 * launch (the paper's per-row loop over an image, Section VI steps 4-5, and
 * its frame loop over a video, generalised to independent covers).
 *
 * A job names byte offsets into three caller-owned device arenas.  Every
 * offset must be a multiple of 256 (LSB_E_ARG otherwise).  The caller
 * guarantees that each job's buffers lie inside the arenas and that no job
 * writes bytes another job reads or writes.
 *
 * A job is either a whole cover with its 32-bit length header (flags = 0, as
 * lsb_embed / lsb_extract) or a raw slice (flags = LSB_JOB_RAW, as
 * lsb_embed_raw / lsb_extract_raw): the cover buffer holds bytes [t0, t0+n)
 * of a longer logical cover and msg_off names byte 0 of a logical stream of
 * stream_bits bits, which several slice jobs of one plan may share (the
 * frames of a clip, the shards of a cover).  A raw extract job obeys the
 * alignment rules of lsb_extract_raw; breaking them is LSB_E_ARG for the
 * whole call.  Header jobs leave t0 and stream_bits at 0.
 */
enum { LSB_JOB_RAW = 1 };

typedef struct lsb_job {
    uint64_t cover_off;   /* embed: cover input (cover arena)                  */
    uint64_t stego_off;   /* embed: stego output; extract: stego input         */
    uint64_t msg_off;     /* embed: message / stream input; extract: output    */
    uint64_t n;           /* cover bytes of this job's buffer                  */
    uint64_t msg_cap;     /* header extract: output capacity in bytes          */
    uint64_t t0;          /* raw: logical field index of buffer byte 0         */
    uint64_t stream_bits; /* raw: bits of the logical stream                   */
    uint32_t len;         /* header embed: message length                      */
    uint8_t k;            /* bits per cover byte, 1..8                         */
    uint8_t op;           /* LSB_OP_EMBED or LSB_OP_EXTRACT (LSB_OP_MIXED plans) */
    uint8_t flags;        /* 0 or LSB_JOB_RAW                                  */
    uint8_t reserved;     /* must be 0                                         */
} lsb_job;                /* 64 bytes */

typedef struct lsb_plan lsb_plan;

/* Create a plan for n_jobs jobs (1 <= n_jobs <= 2^24).  Allocates device and
 * pinned host memory (this is the only allocating call of the batched form).
 * A run is an asynchronous upload of the job table from the plan's pinned
 * mirror (only when the table changed since the last upload), then one
 * persistent kernel launch.
 *   jobs_host  host array of n_jobs jobs, or NULL to reserve room for n_jobs
 *              jobs and set them later with lsb_plan_update.
 *   op         LSB_OP_EMBED or LSB_OP_EXTRACT: every job of the plan is of
 *              that kind (the jobs' own op fields are ignored);
 *              LSB_OP_MIXED: each job's op field says which it is.
 * On error *plan is NULL and nothing is left allocated. */
int lsb_plan_create(lsb_plan **plan, const lsb_job *jobs_host, int n_jobs, int op);

/* Replace the plan's job list (n_jobs <= the n_jobs given at creation),
 * keeping its memory.  Validates every job on the host: a job with bad k,
 * offsets, flags or raw-slice alignment is LSB_E_ARG for the whole call; a
 * header embed job whose len exceeds its
 * capacity is not an error of the call: it gets status LSB_E_CAPACITY and no
 * work.  Waits for the plan's previous run to have read the job table. */
int lsb_plan_update(lsb_plan *plan, const lsb_job *jobs_host, int n_jobs);

/* Run every job of the plan on `stream`.  Every run of a plan uses the
 * plan's device job table and tile counter: a run on another stream than
 * the plan's previous run first makes `stream` wait for that run.  The job
 * table is uploaded again only after lsb_plan_update.
 * For job j: status_dev[j] <- LSB_OK
 * or its error; for extract jobs len_dev[j] <- decoded length, 0 for raw
 * slices (len_dev may be NULL if the plan has no extract job).  Results are
 * identical to one lsb_embed / lsb_extract call per job (raw slices:
 * lsb_embed_raw / lsb_extract_raw).  The arena base pointers must be
 * 256-byte aligned.  LSB_E_ARG if the current device is not the plan's, if
 * the batch tile size (lsb_batch_tune_set) changed since the plan's last
 * lsb_plan_update (update the plan again first), or if `stream` is capturing
 * a graph (a captured run would replay outside the plan's tracking of its
 * table and runs); nothing is enqueued then. */
int lsb_plan_run(lsb_plan *plan, const uint8_t *cover_arena,
                 uint8_t *stego_arena, uint8_t *msg_arena, uint32_t *len_dev,
                 int32_t *status_dev, void *stream);

/* lsb_plan_run for a plan whose jobs are all embeds (LSB_E_ARG otherwise):
 * job j reads cover_arena + cover_off and msg_arena + msg_off, writes
 * stego_arena + stego_off and status_dev[j]. */
int lsb_embed_batch(lsb_plan *plan, const uint8_t *cover_arena,
                    uint8_t *stego_arena, const uint8_t *msg_arena,
                    int32_t *status_dev, void *stream);

/* lsb_plan_run for a plan whose jobs are all extracts (LSB_E_ARG otherwise):
 * job j reads stego_arena + stego_off, writes msg_arena + msg_off (at most
 * msg_cap bytes), len_dev[j] and status_dev[j]. */
int lsb_extract_batch(lsb_plan *plan, const uint8_t *stego_arena,
                      uint8_t *msg_arena, uint32_t *len_dev,
                      int32_t *status_dev, void *stream);

/* Arena extents of a job list: extents[0], [1], [2] receive one past the
 * furthest byte that any job reads or writes in the cover, stego and message
 * arenas (0 when none).  A job of n = 0 touches nothing; a header embed job
 * over its capacity reads no message byte (it gets LSB_E_CAPACITY and no
 * work) but still counts in the cover and stego extents; a header extract
 * job writes at most
 * min(msg_cap, capacity) bytes; a raw job reads or writes stream bytes up to
 * lsb_slice_stream_bytes.  `op` as for lsb_plan_create.  LSB_E_ARG for a
 * bad k or op, or offsets of 2^62 and beyond.  Host-only: callers check arena sizes
 * with it before lsb_plan_run, which trusts them. */
int lsb_job_extents(const lsb_job *jobs, int n_jobs, int op,
                    uint64_t *extents);

/* For callers that cannot allocate (serving loops and harnesses that may not
 * call hipMalloc): lsb_plan_create + lsb_plan_run in one call that allocates
 * nothing.  The job table and its tile counter go into a
 * fixed device array of the library (one per device, about 256 KiB, held
 * until the process ends) instead of plan memory; the table is staged in a
 * library host buffer and uploaded with an asynchronous copy on `stream`,
 * then the persistent kernel is launched on `stream` (no graph).  Jobs, arenas, len_dev and status_dev mean what they mean for
 * lsb_plan_create(op) + lsb_plan_run, and the results are identical.
 * At most LSB_STATIC_MAX_JOBS jobs: more is LSB_E_ARG (use a plan).  Every
 * call on one device shares that device's table: calls on one stream run in
 * order, but calls on different streams of one device whose work overlaps
 * race and must not be made.  Host threads are serialised while the table is
 * filled and uploaded.  A stream that is capturing a graph is refused
 * (LSB_E_ARG, nothing enqueued): the captured upload would read the shared
 * staging buffer at each replay, after later calls may have refilled it. */
enum { LSB_STATIC_MAX_JOBS = 4096 };
int lsb_batch_run_static(const lsb_job *jobs, int n_jobs, int op,
                         const uint8_t *cover_arena, uint8_t *stego_arena,
                         uint8_t *msg_arena, uint32_t *len_dev,
                         int32_t *status_dev, void *stream);

/* Total tiles (work units) of the current job list, for reporting. */
int64_t lsb_plan_tiles(const lsb_plan *plan);

void lsb_plan_destroy(lsb_plan *plan);

/* ------------------------------------------------------------------------
 * Launch configuration (autotuning).  A configuration is chosen per
 * (op, k, size bucket); size bucket b covers n in [2^b, 2^(b+1)).  The
 * library starts with built-in defaults; lsb_tune_set overrides an entry
 * (the Python package loads its tuned table through it), lsb_autotune times
 * every candidate on caller-provided device buffers and installs the best.
 */
typedef struct lsb_launch_cfg {
    int32_t block;          /* threads per block: 64..1024, multiple of 64 */
    int32_t unroll;         /* 16-byte vectors per lane per step: 1, 2, 4  */
    int32_t blocks_per_cu;  /* grid cap = blocks_per_cu * CUs; 0 = no cap  */
    int32_t nontemporal;    /* 1 = streaming (non-temporal) loads/stores   */
    int32_t pack;           /* extract, k = 1: 0 = per-lane multiply pack,
                               1 = wavefront ballots staged through LDS    */
    int32_t order;          /* block order on the 8 XCDs, which take blocks
                               in turn: 0 = launch order, 1 = runs of 16
                               consecutive blocks per XCD (neighbouring
                               blocks then share an L2); embed and extract */
} lsb_launch_cfg;

int lsb_tune_get(int op, int k, uint64_t n, lsb_launch_cfg *cfg);
int lsb_tune_set(int op, int k, int bucket, const lsb_launch_cfg *cfg);

/* Time every candidate configuration for (op, k, n) on the given buffers
 * (cover/stego of n bytes, msg of lsb_capacity(n,k) bytes; contents are
 * overwritten), `reps` launches each, install the fastest for n's bucket and
 * return it in *best (and its mean kernel time in *best_us). */
int lsb_autotune(int op, int k, uint64_t n, uint8_t *cover, uint8_t *stego,
                 uint8_t *msg, int reps, lsb_launch_cfg *best,
                 double *best_us, void *stream);

/* Batched-kernel configuration: tile size in 16-byte vectors per embed tile
 * (extract tiles span twice as many; a multiple of 64 in [64, 2^30]), the
 * kernel's block/unroll/nontemporal choice and its grid cap.  Blocks need at
 * least 128 threads: one wave of each block hands out the tiles that the
 * others stream.  Plans read the tile size at lsb_plan_update and the rest
 * at each run. */
int lsb_batch_tune_get(lsb_launch_cfg *cfg, int64_t *tile_vectors);
int lsb_batch_tune_set(const lsb_launch_cfg *cfg, int64_t tile_vectors);

/* The batched kernel keeps two launch shapes: one for plans with embed jobs
 * (op = LSB_OP_EMBED, also used by mixed plans) and one for extract-only
 * plans (op = LSB_OP_EXTRACT), which move about half the bytes per vector
 * and do best with more vectors in flight per lane.  lsb_batch_tune_get
 * returns the embed shape and lsb_batch_tune_set sets both (and the tile
 * size); these read or set one. */
int lsb_batch_tune_get_op(int op, lsb_launch_cfg *cfg);
int lsb_batch_tune_set_op(int op, const lsb_launch_cfg *cfg);

/* ------------------------------------------------------------------------
 * Serving loop: an open-loop stream of embed and extract requests served
 * with continuous batching.  Requests are admitted in arrival order when the
 * HBM budget (the caller's arena) has room for their outputs; admitted
 * requests are packed into the next launch on any free slot (one stream
 * each), so launches overlap on the device and requests that arrive while
 * others run join the next launch.  A launch of up to four jobs of one
 * operation runs them through lsb_embed / lsb_extract (one kernel each);
 * more go through the slot's batched plan for that operation.  Either way
 * each job's result and status are the same.  Stego buffers stay device
 * resident until an extract consumes them (then they are freed) or the budget
 * needs their space (oldest first, counted as evictions).
 */
typedef struct lsb_server_cfg {
    uint8_t *arena;             /* device memory for stego and message outputs */
    uint64_t arena_bytes;       /* its size: the HBM admission budget          */
    const uint8_t *cover_pool;  /* device-resident covers (requests index it)  */
    const uint8_t *msg_pool;    /* device-resident messages                    */
    int32_t max_batch;          /* jobs per launch, 1..65536                   */
    int32_t n_slots;            /* launches in flight, 1..16                   */
    int32_t keep_outputs;       /* 1: never free or evict outputs (checking)   */
    int32_t reserved;           /* must be 0                                   */
} lsb_server_cfg;

typedef struct lsb_request {
    double arrival_s;   /* scheduled arrival, seconds after the run starts     */
    uint64_t cover_off; /* embed: cover bytes [cover_off, +n) of cover_pool    */
    uint64_t n;
    uint64_t msg_off;   /* embed: message bytes [msg_off, +len) of msg_pool    */
    uint32_t len;
    uint8_t k;          /* embed: bits per byte                                */
    uint8_t op;         /* LSB_OP_EMBED, or LSB_OP_EXTRACT of a live stego     */
    uint16_t reserved;  /* must be 0                                           */
    int64_t target;     /* extract: index of the embed request whose stego to
                           read, or -1 for the oldest live one; an extract with
                           no live stego to read is served as an embed         */
} lsb_request;

typedef struct lsb_result {
    double admit_s, launch_s, done_s; /* seconds after the run starts          */
    uint64_t out_off;  /* arena offset of the output (stego for embed, message
                          for extract); UINT64_MAX once freed or evicted       */
    int32_t status;    /* device status of the job, or LSB_E_NOMEM if the
                          request can never fit the budget                     */
    uint32_t len;      /* message length (decoded, for extract)                */
    int64_t target;    /* extract: the embed request it read; else -1         */
    uint8_t op_run;    /* the operation actually served                        */
    uint8_t k;
    uint8_t reserved[6];
} lsb_result;

typedef struct lsb_serve_stats {
    double makespan_s;        /* first arrival to last completion             */
    double bytes;             /* algorithmic bytes of all served requests     */
    double gbps;              /* bytes / makespan                             */
    double p50_ms, p99_ms, max_ms, mean_ms; /* latency = done - arrival       */
    int64_t launches, evictions, admission_stalls, rejected;
    double mean_batch;
    uint64_t peak_arena_bytes; /* high-water mark of the budget in use        */
} lsb_serve_stats;

/* Serve `n_requests` requests (sorted by arrival) in real time on the
 * current device; returns when every request has completed.  results[i]
 * describes request i.  A request that cannot be served fails alone, its
 * status in results[i] and counted in stats->rejected: LSB_E_CAPACITY when
 * the request is served as an embed and its message does not fit its cover
 * (decided at admission, nothing launched), LSB_E_NOMEM when its output can
 * never fit the budget.  Bad fields (op, k, alignment, order) are LSB_E_ARG
 * for the whole call.  Allocates its plans, streams and events on entry and
 * frees them on exit; never allocates device memory outside cfg->arena. */
int lsb_serve(const lsb_server_cfg *cfg, const lsb_request *requests, int n_requests, lsb_result *results,
              lsb_serve_stats *stats);

/* Measurement support: the next kernel launched by an embed, extract,
 * paper-layout, plane, squared-error, verify, reference-stream or
 * host-streamed video call (there: the first frame's) of the calling thread
 * records `start_event` and `stop_event` (hipEvent_t
 * handles passed as void*, created with timing enabled) at the kernel's own
 * begin and end, so that per-launch durations exclude queueing and marker
 * packets.  Applies to the next such call only: the request clears when
 * that call returns, also if it failed or had nothing to launch (then the
 * events are not recorded).  lsb_autotune replaces a pending request with
 * its own events and clears it.  Both may be NULL to clear. */
int lsb_time_next_launch(void *start_event, void *stop_event);

/* Measurement support: reference streams with the traffic mixes of the
 * method's kernels, so that a kernel's duration can be set against a plain
 * stream of the same bytes on the same device.  Computes nothing of the
 * method.  At k bits per cover byte (k in {1, 2, 4}) a 16-byte cover vector
 * goes with 2k stream bytes.  Over the nv = n / 16 vectors of `src`:
 *   LSB_REF_COPY         dst vector i = src vector i (read n, write n; k
 *                        only checked)
 *   LSB_REF_EMBED_MIX    as COPY with the 2k bytes side[i] XORed into the
 *                        first dword (k = 4: first two dwords) of the vector
 *                        (read n + nk/8, write n: the embed mix)
 *   LSB_REF_EXTRACT_MIX  the 2k bytes dst[i] = for k = 1 the low half, for
 *                        k = 2 all of the XOR of src vector i's four dwords;
 *                        for k = 4 {v0 ^ v1, v2 ^ v3} (read n, write nk/8:
 *                        the extract mix); side unused
 * n must be a multiple of 16; src (and dst for the first two kinds) 16-byte
 * aligned, side and the EXTRACT_MIX dst 2k-byte aligned; dst holds n bytes
 * (nk/8 for EXTRACT_MIX), side nk/8, and dst overlaps no input.  Launch
 * shape: block in {256, 512, 1024}, unroll in {1, 2, 4} vectors in flight
 * per lane (one grid stride apart), grid 0 = enough blocks for one pass,
 * else capped at that.  Device pointers, asynchronous on `stream`; timed
 * like the embed kernel through lsb_time_next_launch.  Errors: LSB_E_ARG. */
enum { LSB_REF_COPY = 0, LSB_REF_EMBED_MIX = 1, LSB_REF_EXTRACT_MIX = 2 };
int lsb_stream_reference(int kind, int k, const uint8_t *src, uint8_t *dst, const uint8_t *side, uint64_t n,
                         int block, int unroll, uint32_t grid, void *stream);

/* The same scheduler without a GPU: launches are modelled (a launch of
 * jobs moving B algorithmic bytes finishes launch_us + B / device_gbps after
 * it starts, every job succeeds, nothing is computed) on a virtual clock
 * that jumps to the next arrival or completion when idle.  cfg's buffers are
 * not touched (they may be NULL); arena_bytes is the budget.  For testing
 * admission, batching and eviction on the host. */
int lsb_serve_simulate(const lsb_server_cfg *cfg, const lsb_request *requests, int n_requests,
                       lsb_result *results, lsb_serve_stats *stats, double launch_us,
                       double device_gbps);

/* Measurement support: the host-observed latency of `reps` round trips
 * lsb_embed(cover -> stego) + lsb_extract_sync(stego -> msg_out), issued
 * from C++ on `stream` (each round trip ends with the synchronisation of
 * lsb_extract_sync), so that the launch and synchronisation cost of the
 * library can be told apart from the cost of a binding above it.  Median and
 * minimum microseconds per round trip.  Arguments as for the two calls
 * (msg_out holds len bytes); LSB_E_HEADER if a round trip decodes another
 * length; LSB_E_ARG for reps outside 1..100000. */
int lsb_roundtrip_latency(const uint8_t *cover, uint8_t *stego, uint64_t n,
                          const uint8_t *msg, uint32_t len, int k,
                          uint8_t *msg_out, int reps, double *us_median,
                          double *us_min, void *stream);

/* Message for the last failed call on this thread ("" if none). */
const char *lsb_last_error(void);

/* Library version string. */
const char *lsb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LSB_H */
