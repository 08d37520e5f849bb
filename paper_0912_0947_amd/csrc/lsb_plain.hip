// lsb_plain.hip -- single-buffer embed / extract kernels for gfx950 and the
// C-ABI entry points lsb_capacity, lsb_embed, lsb_extract(_sync),
// lsb_embed_raw, lsb_extract_raw.
//
// Embedding follows Section VI step 7 of arXiv:0912.0947 (keep the cover
// byte's bits above the field, OR in the data bits), extraction Section VII
// step 6 (mask the field, shift it into place, OR into zeroed data), both
// generalised to k bits per byte with an MSB-first stream; capacity follows
// Section VI step 5 (n*k/8 stream bytes fit n cover bytes).
//
// The paper's kernel uses 4 blocks of at most 32 threads per image row, one
// byte per thread, with every data byte spread over 4 strided positions and
// four blocks ORing into the same output byte during extraction.  Here a
// lane moves 16 contiguous cover bytes per access, a wave 1 KiB, the grid
// covers the whole image in one launch, and every output byte has exactly
// one writer.
#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <vector>

#include "lsb_host.hpp"

namespace lsb {

// ---------------------------------------------------------------------------
// Kernels.

// Block order of the embed and extract kernels (launch configuration field
// `order`; Span.block_order).  Workgroups go to the eight XCDs in turn, so
// neighbouring blocks sit on different XCDs (each with its own L2), and a
// line that two neighbours share is moved by both: the embed's
// stream bytes straddle a line at each end of a block (the 4-byte header sits
// in front of the message), and an extract block's 2k-byte outputs end
// inside a line.  Logical blocks are therefore handed out in runs of 16 per
// XCD (physical block b on XCD b % 8 takes logical block
// 128 (s / 16) + 16 x + s % 16, s = b / 8): the neighbours inside a run share
// an L2, and the XCDs still interleave at 16-block granularity (handing each
// XCD one contiguous eighth removed the shared lines too, but made every
// XCD stream its own distant region and slowed the grid-stride launches).
// Blocks past the last whole round of 128 keep their index.
__device__ __forceinline__ uint32_t xcd_run_block(uint32_t b, uint32_t grid) {
    constexpr uint32_t kXcds = 8, kRun = 16, kRound = kXcds * kRun;
    if (b >= grid / kRound * kRound) return b;
    const uint32_t x = b % kXcds, slot = b / kXcds;
    return (slot / kRun) * kRound + x * kRun + slot % kRun;
}

// Vector embed over the whole span; grid-stride over wave groups.
template <int K, int UNR, bool NT>
__global__ void __launch_bounds__(1024) lsb_embed_kernel(Span s) {
    const Ranges r = embed_ranges<K>(s);
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t block = s.block_order ? xcd_run_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint64_t wave = (block * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    embed_walk<K, UNR, NT>(s, r, 0, r.count, wave, n_waves, lane);
}

__device__ uint8_t header_dummy = 0;  // global (not constant) address space: the loads stay global_load
constexpr int kMaxUnroll = 4;
__device__ __attribute__((aligned(16))) uint8_t group_dummy[16 * 64 * kMaxUnroll] = {};

// Vector extract.  header != 0: decode the length on the device, report it
// and the status through block 0, and extract the message; header == 0: raw
// slice, s.bits already holds the end bit.
template <int K, int UNR, bool NT, bool BALLOT>
__global__ void __launch_bounds__(1024)
    lsb_extract_kernel(Span s, int header, uint64_t out_cap, uint32_t *len_out, int32_t *status_out) {
    constexpr uint64_t G = 64 * UNR;
    static_assert(UNR <= kMaxUnroll, "the dummy group holds kMaxUnroll*64 vectors");
    // ballot packing stages 1 KiB per wave (16 waves per block at most)
    __shared__ __attribute__((aligned(16))) uint8_t stage_all[BALLOT ? 16 * 1024 : 16];
    uint8_t *stage = BALLOT ? stage_all + 1024 * (threadIdx.x >> 6) : nullptr;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t block = s.block_order ? xcd_run_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const uint64_t wave = (block * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    if (!header) {
        const Ranges r = extract_ranges<K>(s);
        extract_walk<K, UNR, NT, BALLOT>(s, r, 0, r.count, wave, n_waves, lane, stage);
        return;
    }
    // Header mode.  Lane j reads the stego byte holding stream bit j % 32
    // (a wave-uniform branch, so the load is issued first), then the wave
    // loads its first group of stego vectors, which do not depend on the
    // decoded length: the header's memory latency overlaps the group's.  A
    // wave whose first group lies past the buffer loads group 0 instead and
    // drops it.
    const bool fits = (uint64_t)K * s.n >= 32;
    const uint64_t u_first = wave * G;
    const bool pre = (u_first + G) * 16 <= s.n;
    // Branch-free: a buffer too short for a header reads a dummy byte.
    const uint8_t *hp = fits ? s.src + (lane & 31u) / K : &header_dummy;
    const uint32_t hbyte = *hp;
    asm volatile("" ::: "memory");
    // The loads are unconditional (no merge of register values after them):
    // a buffer smaller than one group reads the dummy group instead.  The
    // compiler barriers keep the header load first and stop the group loads
    // from being sunk below the decode into the block that consumes them.
    const uint8_t *gp = s.n >= 16 * G ? s.src + 16 * (pre ? u_first : 0) : group_dummy;
    u32x4 c[UNR];
#pragma unroll
    for (int j = 0; j < UNR; ++j) c[j] = load16<NT>(gp + 16 * ((uint64_t)j * 64 + lane));
    asm volatile("" ::: "memory");
    uint32_t len = 0;
    int status = LSB_E_HEADER;
    if (fits) {
        const uint32_t bit = lane < 32 ? (hbyte >> (K - 1 - lane % K)) & 1u : 0u;
        len = __builtin_bitreverse32((uint32_t)__ballot(bit));
        if (4 + (uint64_t)len > room_bytes(s.n, K)) status = LSB_E_HEADER;
        else if ((uint64_t)len > out_cap) status = LSB_E_BUFFER;
        else status = LSB_OK;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *len_out = len;
        *status_out = status;
    }
    if (status != LSB_OK) return;
    s.bits = 8 * (4 + (uint64_t)len);
    const Ranges r = extract_ranges<K>(s);
    uint64_t v_begin = 0;
    if (pre && u_first >= r.fast_begin && u_first + G <= r.fast_end && u_first + G <= r.count) {
        if constexpr (BALLOT && K == 1)
            extract_store_group_ballot<UNR>(s, extract_out_base(s), u_first, c, lane, stage);
        else
            extract_store_group<K, UNR>(s, extract_out_base(s), u_first, c, lane);
        v_begin = n_waves * G;  // the walk resumes at this wave's second group
    }
    extract_walk<K, UNR, NT, BALLOT>(s, r, v_begin, r.count, wave, n_waves, lane, stage);
}

// Per-byte embed for buffers whose cover or stego pointer is not 16-byte
// aligned: one buffer byte per thread step.
__global__ void __launch_bounds__(256) lsb_embed_bytes_kernel(Span s, uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += stride)
        embed_byte(s, t);
}

// Per-byte extract for a misaligned stego pointer: one output stream byte
// per thread step.
__global__ void __launch_bounds__(256)
    lsb_extract_bytes_kernel(Span s, int header, uint64_t out_cap, uint32_t *len_out, int32_t *status_out) {
    const uint32_t lane = threadIdx.x & 63u;
    if (header) {
        uint32_t len = 0;
        int status = LSB_E_HEADER;
        if ((uint64_t)s.k * s.n >= 32) {
            len = decode_header(s.src, s.k, lane);
            if (4 + (uint64_t)len > room_bytes(s.n, s.k)) status = LSB_E_HEADER;
            else if ((uint64_t)len > out_cap) status = LSB_E_BUFFER;
            else status = LSB_OK;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *len_out = len;
            *status_out = status;
        }
        if (status != LSB_OK) return;
        s.bits = 8 * (4 + (uint64_t)len);
    }
    const uint64_t first = stream_byte0(s) > s.hdr_len ? stream_byte0(s) : s.hdr_len;
    const uint64_t end = ceil_div(s.bits, 8);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = first + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < end; i += stride)
        s.out[i - s.hdr_len] = (uint8_t)extract_stream_byte(s, i);
}

// ---------------------------------------------------------------------------
// Dispatch tables: [k-1][unroll index][nontemporal].
typedef void (*EmbedFn)(Span);
typedef void (*ExtractFn)(Span, int, uint64_t, uint32_t *, int32_t *);

static int unroll_index(int u) { return u == 1 ? 0 : (u == 2 ? 1 : 2); }

template <int K>
struct Table {
    static constexpr EmbedFn embed[3][2] = {
        {lsb_embed_kernel<K, 1, false>, lsb_embed_kernel<K, 1, true>},
        {lsb_embed_kernel<K, 2, false>, lsb_embed_kernel<K, 2, true>},
        {lsb_embed_kernel<K, 4, false>, lsb_embed_kernel<K, 4, true>}};
    static constexpr ExtractFn extract[3][2] = {
        {lsb_extract_kernel<K, 1, false, false>, lsb_extract_kernel<K, 1, true, false>},
        {lsb_extract_kernel<K, 2, false, false>, lsb_extract_kernel<K, 2, true, false>},
        {lsb_extract_kernel<K, 4, false, false>, lsb_extract_kernel<K, 4, true, false>}};
};

// k = 1 extract with wavefront-ballot packing.
static constexpr ExtractFn extract_ballot_k1[3][2] = {
    {lsb_extract_kernel<1, 1, false, true>, lsb_extract_kernel<1, 1, true, true>},
    {lsb_extract_kernel<1, 2, false, true>, lsb_extract_kernel<1, 2, true, true>},
    {lsb_extract_kernel<1, 4, false, true>, lsb_extract_kernel<1, 4, true, true>}};

static EmbedFn embed_fn(int k, int u, int nt) {
    const int ui = unroll_index(u);
    switch (k) {
        case 1: return Table<1>::embed[ui][nt];
        case 2: return Table<2>::embed[ui][nt];
        case 3: return Table<3>::embed[ui][nt];
        case 4: return Table<4>::embed[ui][nt];
        case 5: return Table<5>::embed[ui][nt];
        case 6: return Table<6>::embed[ui][nt];
        case 7: return Table<7>::embed[ui][nt];
        default: return Table<8>::embed[ui][nt];
    }
}

static ExtractFn extract_fn(int k, int u, int nt, int pack) {
    const int ui = unroll_index(u);
    if (k == 1 && pack == 1) return extract_ballot_k1[ui][nt];
    switch (k) {
        case 1: return Table<1>::extract[ui][nt];
        case 2: return Table<2>::extract[ui][nt];
        case 3: return Table<3>::extract[ui][nt];
        case 4: return Table<4>::extract[ui][nt];
        case 5: return Table<5>::extract[ui][nt];
        case 6: return Table<6>::extract[ui][nt];
        case 7: return Table<7>::extract[ui][nt];
        default: return Table<8>::extract[ui][nt];
    }
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Stream-side accesses may use dword (even k) / short (odd k) width when the
// address of the first stream byte of vector 0 is 4-byte aligned and k*t0 is
// byte aligned.
static int stream_words(const void *base, uint32_t hdr_len, const Span &s) {
    if (((uint64_t)s.k * s.t0) & 7) return 0;
    const uintptr_t a = (uintptr_t)base - hdr_len + stream_byte0(s);
    return (a & 3u) == 0;
}

int launch_embed(const Span &s0, const lsb_launch_cfg &c, hipStream_t stream) {
    Span s = s0;
    s.words = stream_words(s.body, s.hdr_len, s);
    s.block_order = c.order;
    if (!aligned16(s.src) || !aligned16(s.dst)) {
        // per-byte kernel over the bytes that must be written
        uint64_t count = s.n;
        if (s.inplace) {
            const uint64_t any = ceil_div(s.bits, (uint64_t)s.k);
            count = any > s.t0 ? any - s.t0 : 0;
            if (count > s.n) count = s.n;
        }
        if (!count) return LSB_OK;
        uint64_t blocks = ceil_div(count, 256);
        if (blocks > 65536) blocks = 65536;
        hipEvent_t e0, e1;
        take_launch_events(&e0, &e1);
        hipExtLaunchKernelGGL(lsb_embed_bytes_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, e0, e1, 0, s, count);
    } else {
        const Ranges r = embed_ranges(s);
        if (!r.count) return LSB_OK;
        EmbedFn fn = embed_fn(s.k, c.unroll, c.nontemporal);
        hipEvent_t e0, e1;
        take_launch_events(&e0, &e1);
        hipExtLaunchKernelGGL(fn, dim3(grid_for(c, r.count)), dim3(c.block), 0, stream, e0, e1, 0, s);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "embed kernel launch");
}

int launch_extract(const Span &s0, int header, uint64_t out_cap, uint32_t *len_out, int32_t *status_out,
                   uint64_t max_vectors, const lsb_launch_cfg &c, hipStream_t stream) {
    Span s = s0;
    s.words = stream_words(s.out, s.hdr_len, s);
    s.block_order = c.order;
    if (!aligned16(s.src)) {
        uint64_t bytes = max_vectors * 2 * (uint64_t)s.k;  // output stream bytes bound
        uint64_t blocks = ceil_div(bytes ? bytes : 1, 256);
        if (blocks > 65536) blocks = 65536;
        hipEvent_t e0, e1;
        take_launch_events(&e0, &e1);
        hipExtLaunchKernelGGL(lsb_extract_bytes_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, e0, e1, 0, s,
                              header, out_cap, len_out, status_out);
    } else {
        ExtractFn fn = extract_fn(s.k, c.unroll, c.nontemporal, c.pack);
        hipEvent_t e0, e1;
        take_launch_events(&e0, &e1);
        hipExtLaunchKernelGGL(fn, dim3(grid_for(c, max_vectors)), dim3(c.block), 0, stream, e0, e1, 0, s, header,
                              out_cap, len_out, status_out);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "extract kernel launch");
}

}  // namespace lsb

using namespace lsb;

// ---------------------------------------------------------------------------
// C ABI.
extern "C" {

int64_t lsb_capacity(uint64_t n, int k) {
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_capacity: k=%d outside 1..8", k);
    const uint64_t room = room_bytes(n, k);
    if (room < 4) return fail(LSB_E_CAPACITY, "lsb_capacity: %llu bytes at k=%d cannot hold the 4-byte header",
                              (unsigned long long)n, k);
    uint64_t cap = room - 4;
    if (cap > 0xFFFFFFFFull) cap = 0xFFFFFFFFull;
    return (int64_t)cap;
}

int64_t lsb_slice_stream_bytes(int k, uint64_t t0, uint64_t n, uint64_t stream_bits) {
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_slice_stream_bytes: k=%d outside 1..8", k);
    if (t0 > (1ull << 56) || n > (1ull << 56) || stream_bits > (1ull << 60))
        return fail(LSB_E_ARG, "lsb_slice_stream_bytes: t0/n/stream_bits out of range");
    const uint64_t begin = (uint64_t)k * t0;
    uint64_t end = (uint64_t)k * (t0 + n);
    if (end > stream_bits) end = stream_bits;
    return end > begin ? (int64_t)ceil_div(end, 8) : 0;
}

int lsb_embed(const uint8_t *cover, uint8_t *stego, uint64_t n, const uint8_t *msg, uint32_t len, int k,
              void *stream) {
    const TimedCall timed_call;
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_embed: k=%d outside 1..8", k);
    const int64_t cap = lsb_capacity(n, k);
    if (cap < 0) return (int)cap;
    if ((uint64_t)len > (uint64_t)cap)
        return fail(LSB_E_CAPACITY, "lsb_embed: message of %u bytes exceeds capacity %lld", len, (long long)cap);
    if (!cover || !stego) return fail(LSB_E_ARG, "lsb_embed: null cover/stego");
    if (len && !msg) return fail(LSB_E_ARG, "lsb_embed: null msg");
    if (cover != stego && overlaps(cover, n, stego, n))
        return fail(LSB_E_ARG, "lsb_embed: cover and stego overlap (only stego == cover is allowed)");
    if (overlaps(msg, len, stego, n)) return fail(LSB_E_ARG, "lsb_embed: msg overlaps stego");

    Span s{};
    s.src = cover;
    s.dst = stego;
    s.body = msg;
    s.n = n;
    s.t0 = 0;
    s.bits = 8 * (4 + (uint64_t)len);
    s.hdr = len;
    s.hdr_len = 4;
    s.k = k;
    s.inplace = cover == stego;
    return launch_embed(s, tune_lookup(LSB_OP_EMBED, k, n), (hipStream_t)stream);
}

int lsb_embed_raw(const uint8_t *cover, uint8_t *stego, uint64_t n, uint64_t t0, const uint8_t *stream_bytes,
                  uint64_t stream_bits, int k, void *stream) {
    const TimedCall timed_call;
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_embed_raw: k=%d outside 1..8", k);
    if (n == 0) return LSB_OK;
    if (!cover || !stego) return fail(LSB_E_ARG, "lsb_embed_raw: null cover/stego");
    if (t0 > (1ull << 56) || n > (1ull << 56) || stream_bits > (1ull << 60))
        return fail(LSB_E_ARG, "lsb_embed_raw: t0/n/stream_bits out of range");
    const uint64_t sb = ((uint64_t)k * t0) / 8;
    const uint64_t s_end = ceil_div(stream_bits, 8);
    const uint64_t read_end = ceil_div((uint64_t)k * (t0 + n) < stream_bits ? (uint64_t)k * (t0 + n) : stream_bits, 8);
    if (sb < s_end && !stream_bytes) return fail(LSB_E_ARG, "lsb_embed_raw: null stream");
    if (cover != stego && overlaps(cover, n, stego, n))
        return fail(LSB_E_ARG, "lsb_embed_raw: cover and stego overlap (only stego == cover is allowed)");
    if (sb < read_end && overlaps(stream_bytes + sb, read_end - sb, stego, n))
        return fail(LSB_E_ARG, "lsb_embed_raw: stream overlaps stego");

    Span s{};
    s.src = cover;
    s.dst = stego;
    s.body = stream_bytes;
    s.n = n;
    s.t0 = t0;
    s.bits = stream_bits;
    s.hdr_len = 0;
    s.k = k;
    s.inplace = cover == stego;
    return launch_embed(s, tune_lookup(LSB_OP_EMBED, k, n), (hipStream_t)stream);
}

int lsb_extract(const uint8_t *stego, uint64_t n, int k, uint8_t *msg_out, uint64_t out_cap, uint32_t *len_out_dev,
                int32_t *status_out_dev, void *stream) {
    const TimedCall timed_call;
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_extract: k=%d outside 1..8", k);
    if (!len_out_dev || !status_out_dev) return fail(LSB_E_ARG, "lsb_extract: null len/status pointer");
    if (n && !stego) return fail(LSB_E_ARG, "lsb_extract: null stego");
    if (out_cap && !msg_out) return fail(LSB_E_ARG, "lsb_extract: null msg_out with out_cap > 0");
    if (n > (1ull << 56)) return fail(LSB_E_ARG, "lsb_extract: n out of range");
    const uint64_t room = room_bytes(n, k);
    const uint64_t cap = room >= 4 ? room - 4 : 0;
    const uint64_t max_len = out_cap < cap ? out_cap : cap;
    if (overlaps(msg_out, max_len, stego, n)) return fail(LSB_E_ARG, "lsb_extract: msg_out overlaps stego");
    if (overlaps(len_out_dev, 4, stego, n) || overlaps(status_out_dev, 4, stego, n) ||
        overlaps(len_out_dev, 4, msg_out, max_len) || overlaps(status_out_dev, 4, msg_out, max_len))
        return fail(LSB_E_ARG, "lsb_extract: len/status overlap a data buffer");

    // Upper bound on vectors: the longest stream that can pass both checks.
    uint64_t max_vectors = 0;
    if ((uint64_t)k * n >= 32) {
        const uint64_t v_stream = ceil_div(4 + max_len, 2 * (uint64_t)k);
        const uint64_t v_buf = ceil_div(n, 16);
        max_vectors = v_stream < v_buf ? v_stream : v_buf;
    }
    Span s{};
    s.src = stego;
    s.out = msg_out;
    s.n = n;
    s.t0 = 0;
    s.hdr_len = 4;
    s.k = k;
    return launch_extract(s, 1, out_cap, len_out_dev, status_out_dev, max_vectors,
                          tune_lookup(LSB_OP_EXTRACT, k, n), (hipStream_t)stream);
}

int lsb_extract_raw(const uint8_t *stego, uint64_t n, uint64_t t0, uint8_t *stream_out, uint64_t stream_bits, int k,
                    void *stream) {
    const TimedCall timed_call;
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_extract_raw: k=%d outside 1..8", k);
    if (t0 > (1ull << 56) || n > (1ull << 56) || stream_bits > (1ull << 60))
        return fail(LSB_E_ARG, "lsb_extract_raw: t0/n/stream_bits out of range");
    const uint64_t begin = (uint64_t)k * t0;
    uint64_t end = (uint64_t)k * (t0 + n);
    if (end > stream_bits) end = stream_bits;
    if (begin % 8) return fail(LSB_E_ARG, "lsb_extract_raw: k*t0 = %llu is not byte aligned", (unsigned long long)begin);
    if (begin >= end) return LSB_OK;
    if (end % 8 && end != stream_bits)
        return fail(LSB_E_ARG, "lsb_extract_raw: slice ends inside a stream byte that the next slice also needs");
    if (!stego || !stream_out) return fail(LSB_E_ARG, "lsb_extract_raw: null stego/stream_out");
    const uint64_t first = begin / 8, last = ceil_div(end, 8);
    if (overlaps(stream_out + first, last - first, stego, n))
        return fail(LSB_E_ARG, "lsb_extract_raw: stream_out overlaps stego");

    Span s{};
    s.src = stego;
    s.out = stream_out;
    s.n = n;
    s.t0 = t0;
    s.bits = end;
    s.hdr_len = 0;
    s.k = k;
    const Ranges r = extract_ranges(s);
    if (!r.count) return LSB_OK;
    return launch_extract(s, 0, 0, nullptr, nullptr, r.count, tune_lookup(LSB_OP_EXTRACT, k, n),
                          (hipStream_t)stream);
}

int lsb_extract_sync(const uint8_t *stego, uint64_t n, int k, uint8_t *msg_out, uint64_t out_cap,
                     uint32_t *len_out_host, void *stream) {
    struct Scratch {
        int dev = -1;
        void *buf = nullptr;
    };
    static thread_local Scratch scratch[16];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 16) return fail(LSB_E_ARG, "lsb_extract_sync: device %d not supported", dev);
    Scratch &sc = scratch[dev];
    if (!sc.buf) {
        e = hipMalloc(&sc.buf, 256);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc(extract_sync scratch)");
        sc.dev = dev;
    }
    uint32_t *len_dev = (uint32_t *)sc.buf;
    int32_t *status_dev = (int32_t *)((char *)sc.buf + 4);
    int rc = lsb_extract(stego, n, k, msg_out, out_cap, len_dev, status_dev, stream);
    if (rc != LSB_OK) return rc;
    uint32_t host[2] = {0, 0};
    e = hipMemcpyAsync(host, sc.buf, 8, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(extract_sync status)");
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (len_out_host) *len_out_host = host[0];
    const int status = (int)(int32_t)host[1];
    if (status != LSB_OK)
        fail(status, "lsb_extract_sync: %s (decoded length %u)",
             status == LSB_E_HEADER ? "header does not fit the cover" : "output buffer too small", host[0]);
    return status;
}

int lsb_roundtrip_latency(const uint8_t *cover, uint8_t *stego, uint64_t n, const uint8_t *msg, uint32_t len, int k,
                          uint8_t *msg_out, int reps, double *us_median, double *us_min, void *stream) {
    if (reps < 1 || reps > 100000 || !us_median || !us_min) return fail(LSB_E_ARG, "lsb_roundtrip_latency: bad reps");
    std::vector<double> us;
    us.reserve((size_t)reps);
    for (int r = 0; r < reps; ++r) {
        const auto t0 = std::chrono::steady_clock::now();
        int rc = lsb_embed(cover, stego, n, msg, len, k, stream);
        if (rc != LSB_OK) return rc;
        uint32_t got = 0;
        rc = lsb_extract_sync(stego, n, k, msg_out, len, &got, stream);
        if (rc != LSB_OK) return rc;
        if (got != len) return fail(LSB_E_HEADER, "lsb_roundtrip_latency: decoded %u of %u bytes", got, len);
        us.push_back(std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count());
    }
    std::sort(us.begin(), us.end());
    *us_median = us[us.size() / 2];
    *us_min = us.front();
    return LSB_OK;
}

}  // extern "C"
