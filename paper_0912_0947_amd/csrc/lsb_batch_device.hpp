// lsb_batch_device.hpp -- device side of the batched embed/extract: the job
// table records and the persistent kernel, shared by the translation unit of
// header-only plans and the one of plans with raw-slice jobs.
#pragma once

#include <stddef.h>

#include <utility>

#include "lsb_host.hpp"

namespace lsb {

// The tile counter has a 128-byte cache line of its own: sharing a line with
// the job records that every block reads made each atomic contend with those
// reads (a one-job batch ran at 40 % of a many-job batch).  Both counters
// are zero in an uploaded table, and the last block of each run sets them
// back to zero, so a run whose table is already on the device starts from
// zero without an upload.
struct PlanHeader {
    uint64_t n_jobs;
    uint64_t total_tiles;
    uint64_t tile_vectors;
    uint64_t pad0[13];
    uint64_t next_tile;    // tile counter of the persistent kernel
    uint64_t blocks_done;  // blocks whose producer has taken its last tile id this run
    uint64_t pad1[14];
};
static_assert(sizeof(PlanHeader) == 256 && offsetof(PlanHeader, next_tile) == 128 &&
                  offsetof(PlanHeader, blocks_done) == 136,
              "counters on their own line, job records 256-byte aligned");

struct DevJob {
    uint64_t cover_off, stego_off, msg_off, n;
    uint64_t cap_bits;    // header extract: msg_cap; raw: end bit (embed: stream_bits, extract: e)
    uint64_t tile_begin;  // tiles of jobs before this one; entry n_jobs = total
    uint64_t t0;          // raw: logical field index of buffer byte 0; header jobs: 0
    uint32_t len;
    uint8_t k, op;
    int8_t status;  // host-validated status; header extract: decoded on device
    uint8_t raw;    // 1: raw slice, no header
};
static_assert(sizeof(DevJob) == 64, "DevJob is one 64-byte record");
static_assert(sizeof(lsb_job) == 64 && offsetof(lsb_job, len) == 56, "lsb_job layout of the C ABI");

// One tile of a job: ranges with k known at compile time, then the walk
// over the tile's vectors.
template <int K, int UNR, bool NT>
__device__ __forceinline__ void embed_tile(const Span &s, uint64_t v_begin, uint64_t tile_vectors, uint32_t wave,
                                           uint32_t n_waves, uint32_t lane) {
    const Ranges r = embed_ranges<K>(s);
    uint64_t v_end = v_begin + tile_vectors;
    if (v_end > r.count) v_end = r.count;
    if (v_begin < v_end) embed_walk<K, UNR, NT>(s, r, v_begin, v_end, wave, n_waves, lane);
}

template <int K, int UNR, bool NT>
__device__ __forceinline__ void extract_tile(const Span &s, uint64_t v_begin, uint64_t tile_vectors, uint32_t wave,
                                             uint32_t n_waves, uint32_t lane) {
    const Ranges r = extract_ranges<K>(s);
    uint64_t v_end = v_begin + tile_vectors;
    if (v_end > r.count) v_end = r.count;
    if (v_begin < v_end) extract_walk<K, UNR, NT>(s, r, v_begin, v_end, wave, n_waves, lane);
}

// Job classes of a plan.  CLS = 1 + 8*op + (k - 1): every job has that
// (op, k), and only its walker is compiled in.  CLS = 17: every job is an
// extract, k dispatched by a switch over the eight extract walkers (61 VGPRs
// at two vectors per lane, so two 1024-thread blocks fit a CU; the same for
// the embed walkers needs more than the sixteen-way switch and spills).
// CLS = 0: (op, k) read from each job, a switch over all sixteen.
// Header and raw-slice jobs share the walkers: only the span's stream fields
// differ.  RAW = false compiles the raw-slice case out (the plan has none):
// the header span's constant t0, header length and dword stream side then
// fold into the walk.
constexpr int kClsExtractAnyK = 17, kClasses = 18;

template <int UNR, bool NT, int CLS, bool RAW>
__device__ __forceinline__ void run_tile(const DevJob &J, uint64_t v_begin, uint64_t tile_vectors,
                                         const uint8_t *cover_arena, uint8_t *stego_arena, uint8_t *msg_arena,
                                         uint32_t len, uint32_t wave, uint32_t n_waves, uint32_t lane) {
    constexpr bool EMB = CLS == 0 || (CLS >= 1 && CLS <= 8);
    constexpr bool EXT = CLS == 0 || CLS == kClsExtractAnyK || (CLS >= 9 && CLS <= 16);
    constexpr int KC = CLS >= 1 && CLS <= 16 ? (CLS - 1) % 8 + 1 : 0;  // fixed k, 0: any
    Span s{};
    s.n = J.n;
    s.t0 = 0;
    s.k = J.k;
    s.hdr_len = 4;
    s.words = 1;  // offsets are multiples of 256: stream side is dword aligned
    const bool raw = RAW && J.raw;
    if (raw) {
        // stream byte 0 sits at a 256-byte aligned offset, so the stream side
        // is dword aligned exactly when field t0 starts on a 32-bit boundary
        s.t0 = J.t0;
        s.hdr_len = 0;
        s.words = (((uint64_t)J.k * J.t0) & 31u) == 0;
    }
    if constexpr (EMB) {
        if (!EXT || J.op == LSB_OP_EMBED) {
            s.src = cover_arena + J.cover_off;
            s.dst = stego_arena + J.stego_off;
            s.body = msg_arena + J.msg_off;
            s.bits = raw ? J.cap_bits : 8 * (4 + (uint64_t)J.len);
            s.hdr = J.len;
            if constexpr (KC > 0) {
                embed_tile<KC, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane);
            } else {
                switch (J.k) {
                    case 1: embed_tile<1, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                    case 2: embed_tile<2, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                    case 3: embed_tile<3, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                    case 4: embed_tile<4, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                    case 5: embed_tile<5, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                    case 6: embed_tile<6, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                    case 7: embed_tile<7, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                    default: embed_tile<8, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                }
            }
            return;
        }
    }
    if constexpr (EXT) {
        s.src = stego_arena + J.stego_off;
        s.out = msg_arena + J.msg_off;
        s.bits = raw ? J.cap_bits : 8 * (4 + (uint64_t)len);
        if constexpr (KC > 0) {
            extract_tile<KC, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane);
        } else {
            switch (J.k) {
                case 1: extract_tile<1, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                case 2: extract_tile<2, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                case 3: extract_tile<3, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                case 4: extract_tile<4, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                case 5: extract_tile<5, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                case 6: extract_tile<6, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                case 7: extract_tile<7, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
                default: extract_tile<8, UNR, NT>(s, v_begin, tile_vectors, wave, n_waves, lane); break;
            }
        }
    }
}

// Waves per SIMD the launch bound asks for.  A 1024-thread block puts 4
// waves on each SIMD (so at most 128 VGPRs), and anything from 4 to 7 keeps
// one block per CU; only 8 (64 VGPRs) fits two.  8 at one vector per lane
// (about 30-40 VGPRs) and for the extract-any-k class at two (47 VGPRs; with
// raw slices it would spill under 64 and takes 6); 6 for the others at two,
// 5 for the raw-capable kernels with the widest walkers (all sixteen behind
// the switch: 85 VGPRs; k = 1 embed), where 6 would spill; 4 at four (the
// extract-any-k class then uses 88 VGPRs, 97 with raw slices: one block per
// CU).
template <int UNR, int CLS, bool RAW>
constexpr int batch_min_waves() {
    if constexpr (UNR == 1) return 8;
    else if constexpr (UNR == 2) return CLS == kClsExtractAnyK && !RAW ? 8 : (RAW && CLS <= 1 ? 5 : 6);
    else return 4;
}

// Tile hand-off inside a block.  Wave 0 is the block's producer and does no
// streaming itself: it takes the next tile id from the plan's counter,
// resolves the tile's job (forward search over the tile prefix, 64 jobs per
// ballot; jobs only move forward as the tile id grows), reads the job record
// (and, for a header extract job, decodes the job's length header), and
// publishes all of it in a slot of a two-slot LDS ring.  The producer that
// takes a job's first tile also reports the job's length and status; jobs
// without tiles are reported by a sweep over the job table that every
// producer runs once.  The other waves (the workers) read their next tile
// from the ring when they finish the current one, so they never wait for
// each other at a tile boundary, and the latency of the counter, the search
// and the record reads is spent by the producer while the workers stream.
// The producer publishes tile m + 1 once every worker has taken tile m (the
// slot it overwrites was read before that), so a block holds at most one
// tile beyond the one its slowest worker is on.  Every wait is
// bounded (kSpinLimit polls): a wave whose partner never answers gives up
// instead of hanging the device (its tiles are then left undone).
constexpr int kRing = 2;
constexpr uint32_t kSpinLimit = 1u << 26;

struct TileSlot {
    DevJob job;       // the tile's job record
    uint64_t tile;    // global tile id; >= total ends the block
    uint32_t len;     // header extract: decoded message length
    uint32_t run;     // 1: the job has work (status OK)
};

// Ordering of the hand-off.  The LDS instructions of one wave execute in
// the order they are issued, and a wave observes another wave's LDS write
// once it has executed.  So the ring needs only relaxed LDS accesses kept in
// program order by compiler barriers: the producer writes a slot, then its
// sequence number; a worker reads the sequence number, then the slot, then
// counts itself as a reader.  (Release/acquire atomics would also order the
// waves' global memory traffic: a worker would wait for its previous tile's
// stores to complete at every tile boundary.)
__device__ __forceinline__ void lds_order() { asm volatile("" ::: "memory"); }

__device__ __forceinline__ uint32_t lds_read(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void lds_write(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait (wave-uniform) until *p == want; false if the limit ran out.
__device__ __forceinline__ bool lds_wait_eq(const uint32_t *p, uint32_t want) {
    for (uint32_t i = 0; i < kSpinLimit; ++i) {
        const uint32_t v = lds_read(p);
        lds_order();
        if (v == want) return true;
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

__device__ __forceinline__ uint32_t uniform32(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    return ((uint64_t)uniform32((uint32_t)(v >> 32)) << 32) | uniform32((uint32_t)v);
}

// What a job reports in len_dev / status_dev.  The host-validated status
// and length, except for a header extract job that the host let through:
// its length is the stego's 32-bit header (Section VII, the stream's first
// 32 bits), which must fit the cover's room and the job's output buffer.
// J is wave-uniform: the decode spreads the header's bits over the lanes.
struct JobReport {
    uint32_t len;
    int32_t status;
};

__device__ __forceinline__ JobReport job_report(const DevJob &J, const uint8_t *stego_arena, uint32_t lane) {
    JobReport r{J.len, J.status};
    if (J.op == LSB_OP_EXTRACT && !J.raw && J.status == LSB_OK) {
        r.len = 0;
        r.status = LSB_E_HEADER;
        if ((uint64_t)J.k * J.n >= 32) {
            r.len = decode_header(stego_arena + J.stego_off, J.k, lane);
            if (4 + (uint64_t)r.len > room_bytes(J.n, J.k)) r.status = LSB_E_HEADER;
            else if ((uint64_t)r.len > J.cap_bits) r.status = LSB_E_BUFFER;
            else r.status = LSB_OK;
        }
    }
    return r;
}

// Reports of the jobs without tiles (refused on the host, empty slices, and
// header extract jobs whose cover holds fewer than 32 bits), lane-parallel
// over the table: block b's producer takes jobs 64b + lane, then every
// 64 G-th.  No tile is ever handed out for these jobs, so nothing else
// writes their entries.  A header extract job the host let through has a
// tile whenever k n >= 32, so one without tiles is refused here.
__device__ __forceinline__ void report_empty_jobs(const DevJob *jobs, uint64_t n_jobs, uint32_t *len_dev,
                                                  int32_t *status_dev, uint32_t lane) {
    for (uint64_t j = (uint64_t)blockIdx.x * 64 + lane; j < n_jobs; j += (uint64_t)gridDim.x * 64) {
        const DevJob &J = jobs[j];
        if (J.tile_begin != jobs[j + 1].tile_begin) continue;  // the producer of its first tile reports it
        uint32_t len = J.len;
        int32_t status = J.status;
        if (J.op == LSB_OP_EXTRACT && !J.raw && status == LSB_OK) {
            len = 0;
            status = LSB_E_HEADER;
        }
        if (len_dev) len_dev[j] = len;
        status_dev[j] = status;
    }
}

// A producer is done with the counter (lane 0): the last one of the grid
// sets both counters back to zero for the plan's next run.  Every producer
// has taken its last tile id before it counts itself (its atomics return
// values that it has used), so after the last count nothing else touches
// the counters in this run.
__device__ __forceinline__ void producer_done(const PlanHeader *hdr) {
    PlanHeader *h = const_cast<PlanHeader *>(hdr);
    const unsigned long long before = atomicAdd((unsigned long long *)&h->blocks_done, 1ull);
    if (before == (unsigned long long)gridDim.x - 1) {
        __hip_atomic_store(&h->next_tile, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&h->blocks_done, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Persistent kernel: tiles come from one counter in arrival order, so the
// tiles in flight at any moment are neighbours in the arenas (a static b,
// b + G, ... order lets blocks drift apart over the run).  Blocks have at
// least two waves (one producer, at least one worker).
template <int UNR, bool NT, int CLS, bool RAW>
__global__ void __launch_bounds__(1024, (batch_min_waves<UNR, CLS, RAW>()))
    lsb_batch_kernel(const PlanHeader *hdr, const DevJob *jobs, const uint8_t *cover_arena, uint8_t *stego_arena,
                     uint8_t *msg_arena, uint32_t *len_dev, int32_t *status_dev) {
    __shared__ TileSlot ring[kRing];
    __shared__ uint32_t seq[kRing];      // iteration whose tile the slot holds
    __shared__ uint32_t readers[kRing];  // workers that have read the slot's current content
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t workers = (blockDim.x >> 6) - 1;
    const uint64_t total = hdr->total_tiles;
    if (threadIdx.x < kRing) {
        seq[threadIdx.x] = ~0u;
        readers[threadIdx.x] = workers;  // free
    }
    __syncthreads();

    if (wave == 0) {
        // ---- producer
        unsigned long long *counter = (unsigned long long *)&const_cast<PlanHeader *>(hdr)->next_tile;
        const uint64_t n_jobs = hdr->n_jobs;
        uint64_t j = 0;  // job search cursor
        uint64_t t = 0;
        if (lane == 0) t = atomicAdd(counter, 1ull);
        for (uint32_t m = 0;; ++m) {
            t = uniform64(t);
            const uint32_t sl = m % kRing;
            uint32_t run = 0, len = 0;
            DevJob J{};
            if (t < total) {
                // largest j with jobs[j].tile_begin <= t (entry n_jobs holds total > t)
                for (;;) {
                    const uint64_t idx = j + 1 + lane;
                    const uint64_t tb = idx <= n_jobs ? jobs[idx].tile_begin : ~0ull;
                    const uint64_t below = __ballot(tb <= t);
                    const uint32_t cnt = (uint32_t)__popcll(below);
                    j += cnt;
                    if (cnt < 64) break;
                }
                j = uniform64(j);
                J = jobs[j];
                const JobReport r = job_report(J, stego_arena, lane);
                run = r.status == LSB_OK;
                len = r.len;
                if (t == J.tile_begin && lane == 0) {  // the job's first tile: report the job
                    if (len_dev) len_dev[j] = r.len;
                    status_dev[j] = r.status;
                }
            }
            // every worker must have taken tile m - 1 (and so every earlier one)
            if (m && !lds_wait_eq(&readers[(m - 1) % kRing], workers)) {
                if (lane == 0) producer_done(hdr);
                return;
            }
            if (lane == 0) {
                if (t < total) ring[sl].job = J;
                ring[sl].tile = t;
                ring[sl].len = len;
                ring[sl].run = run;
                lds_write(&readers[sl], 0);
                lds_order();
                lds_write(&seq[sl], m);
            }
            // after the first hand-off, so that the workers start at once
            if (m == 0) report_empty_jobs(jobs, n_jobs, len_dev, status_dev, lane);
            if (t >= total) {  // the end mark is out
                if (lane == 0) producer_done(hdr);
                return;
            }
            if (lane == 0) t = atomicAdd(counter, 1ull);
        }
    }

    // ---- workers
    const uint64_t tv_embed = hdr->tile_vectors;
    for (uint32_t m = 0;; ++m) {
        const uint32_t sl = m % kRing;
        if (!lds_wait_eq(&seq[sl], m)) return;
        // the slot, read into wave-uniform registers
        const uint64_t tile = uniform64(ring[sl].tile);
        DevJob J;
        {
            const uint32_t *src = reinterpret_cast<const uint32_t *>(&ring[sl].job);
            uint32_t *dst = reinterpret_cast<uint32_t *>(&J);
#pragma unroll
            for (int i = 0; i < (int)(sizeof(DevJob) / 4); ++i) dst[i] = uniform32(src[i]);
        }
        const uint32_t len = uniform32(ring[sl].len);
        const uint32_t run = uniform32(ring[sl].run);
        lds_order();
        if (lane == 0) __hip_atomic_fetch_add(&readers[sl], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (tile >= total) return;
        if (run) {
            // an extract tile covers twice the vectors of an embed tile; the
            // workers' shares of a tile rotate from tile to tile
            const uint64_t tv = J.op == LSB_OP_EXTRACT ? 2 * tv_embed : tv_embed;
            const uint32_t w = (wave - 1 + m) % workers;
            run_tile<UNR, NT, CLS, RAW>(J, (tile - J.tile_begin) * tv, tv, cover_arena, stego_arena, msg_arena, len,
                                        w, workers, lane);
        }
    }
}

typedef void (*BatchFn)(const PlanHeader *, const DevJob *, const uint8_t *, uint8_t *, uint8_t *, uint32_t *,
                        int32_t *);

// Kernel table of one launch shape: entry CLS of the class sequence.
template <int UNR, bool NT, bool RAW, int... C>
BatchFn batch_fn_of(int cls, std::integer_sequence<int, C...>) {
    static const BatchFn table[] = {lsb_batch_kernel<UNR, NT, C, RAW>...};
    return table[cls];
}

// Kernel for a launch shape and plan class (0 = mixed jobs).
template <bool RAW>
BatchFn batch_fn_for(int unroll, int nt, int cls) {
    using Classes = std::make_integer_sequence<int, kClasses>;
    if (unroll == 1)
        return nt ? batch_fn_of<1, true, RAW>(cls, Classes{}) : batch_fn_of<1, false, RAW>(cls, Classes{});
    if (unroll == 2)
        return nt ? batch_fn_of<2, true, RAW>(cls, Classes{}) : batch_fn_of<2, false, RAW>(cls, Classes{});
    return nt ? batch_fn_of<4, true, RAW>(cls, Classes{}) : batch_fn_of<4, false, RAW>(cls, Classes{});
}

// Kernels of plans holding raw-slice jobs (instantiated in their own
// translation unit, which builds in parallel with the header-only one).
BatchFn batch_fn_raw(int unroll, int nt, int cls);

}  // namespace lsb
