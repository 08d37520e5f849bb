// lsb_device.hpp -- device-side building blocks of k-bit LSB embed/extract
// for gfx950 (CDNA4, wave64).
//
// Operation (arXiv:0912.0947): embedding, Section VI step 7 -- a cover byte
// keeps its bits above the field and takes k stream bits in the field;
// extraction, Section VII step 6 -- the field is masked out of the stego byte
// and its bits are placed back into the zero-initialised data byte.
//
// Stream: S = BE32(len) || msg in header mode, or a caller stream in raw
// mode, read most-significant bit first.  Buffer byte t is logical field
// g = t0 + t and carries stream bits k*g .. k*g+k-1, first bit highest.
//
// Work unit: one "vector" = 16 consecutive buffer bytes = 16 fields = 16k
// stream bits = 2k whole stream bytes (16k is a multiple of 8, so when k*t0
// is byte aligned every vector starts on a stream byte).  A lane moves one
// 16-byte vector of cover/stego per step with a single dwordx4 access and the
// matching 2k stream bytes with dword (k even) or short (k odd) accesses.
// Vectors are grouped 64 per wave access so that every load and store
// instruction of a wave touches one contiguous 1 KiB span.
//
// Each span of vectors splits into (computed once per wave, in scalars):
//   fast  -- all 16 fields full and every stream byte past the header,
//   copy  -- no stream bits at all (embed copies the cover),
//   edge  -- the rest (header bytes, the partial last field, the buffer tail),
//            handled byte by byte; only a few vectors per buffer are edges.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsb {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// -------------------------------------------------------------------------
// Description of one embed or extract over one buffer.
struct Span {
    const uint8_t *src;   // embed: cover; extract: stego
    uint8_t *dst;         // embed: stego; extract: unused
    const uint8_t *body;  // embed: stream source (msg in header mode)
    uint8_t *out;         // extract: destination of stream bytes >= hdr_len
    uint64_t n;           // buffer bytes
    uint64_t t0;          // logical field index of buffer byte 0
    uint64_t bits;        // embed: stream bits; extract: end bit e (exclusive)
    uint32_t hdr;         // header value (header mode)
    uint32_t hdr_len;     // 4 in header mode, 0 in raw mode
    int k;
    int inplace;          // embed: dst == src, skip copy-only bytes
    int words;            // stream side may use dword/short accesses
    int block_order;      // plain kernels: 1 = blocks in runs of 16 per XCD
};

// Vector classes of a span (all in the span's own vector index space).
struct Ranges {
    uint64_t fast_begin, fast_end;  // fast vectors: [fast_begin, fast_end)
    uint64_t copy_begin, copy_end;  // copy vectors: [copy_begin, copy_end)
    uint64_t count;                 // vectors to visit: [0, count)
};

__host__ __device__ inline uint64_t stream_byte0(const Span &s) {
    return ((uint64_t)s.k * s.t0) >> 3;  // stream byte holding field t0's first bit
}

// The range functions take k as a compile-time constant on the device
// (KC > 0), so that their divisions by k and 2k become shifts or constant
// multiplies instead of 64-bit division sequences; KC = 0 reads s.k (host).
template <int KC = 0>
__host__ __device__ inline Ranges embed_ranges(const Span &s) {
    Ranges r;
    const uint64_t k = KC > 0 ? (uint64_t)KC : (uint64_t)s.k;
    const uint64_t full = s.bits / k;            // fields fully inside the stream
    const uint64_t any = ceil_div(s.bits, k);    // fields carrying any stream bit
    const uint64_t whole = s.n / 16;             // vectors fully inside the buffer
    const uint64_t sb = stream_byte0(s);
    r.fast_begin = sb >= s.hdr_len ? 0 : ceil_div(s.hdr_len - sb, 2 * k);
    const uint64_t f_end = full > s.t0 ? (full - s.t0) / 16 : 0;
    r.fast_end = f_end < whole ? f_end : whole;
    r.copy_begin = any > s.t0 ? ceil_div(any - s.t0, 16) : 0;
    r.copy_end = whole;
    const uint64_t all = ceil_div(s.n, 16);
    r.count = s.inplace ? (r.copy_begin < all ? r.copy_begin : all) : all;
    return r;
}

// For extract, s.bits is the end bit e <= k*(t0+n), and k*t0 % 8 == 0.
template <int KC = 0>
__host__ __device__ inline Ranges extract_ranges(const Span &s) {
    Ranges r;
    const uint64_t k = KC > 0 ? (uint64_t)KC : (uint64_t)s.k;
    const uint64_t full = s.bits / k;
    const uint64_t whole = s.n / 16;
    const uint64_t sb = stream_byte0(s);
    r.fast_begin = sb >= s.hdr_len ? 0 : ceil_div(s.hdr_len - sb, 2 * k);
    const uint64_t f_end = full > s.t0 ? (full - s.t0) / 16 : 0;
    r.fast_end = f_end < whole ? f_end : whole;
    r.copy_begin = r.copy_end = 0;
    const uint64_t end_byte = ceil_div(s.bits, 8);  // exclusive
    const uint64_t by_stream = end_byte > sb ? ceil_div(end_byte - sb, 2 * k) : 0;
    const uint64_t all = ceil_div(s.n, 16);
    r.count = by_stream < all ? by_stream : all;
    return r;
}

// -------------------------------------------------------------------------
// Memory access helpers.
template <bool NT>
__device__ __forceinline__ u32x4 load16(const uint8_t *p) {
    const u32x4 *q = reinterpret_cast<const u32x4 *>(p);
    if constexpr (NT) return __builtin_nontemporal_load(q);
    else return *q;
}

template <bool NT>
__device__ __forceinline__ void store16(uint8_t *p, u32x4 v) {
    u32x4 *q = reinterpret_cast<u32x4 *>(p);
    if constexpr (NT) __builtin_nontemporal_store(v, q);
    else *q = v;
}

__device__ __forceinline__ uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

// Logical stream byte s (header bytes come from the header value).
__device__ __forceinline__ uint32_t stream_byte(const Span &s, uint64_t i) {
    if (i < s.hdr_len) return (s.hdr >> (8 * (3 - (uint32_t)i))) & 0xFFu;
    return s.body[i - s.hdr_len];
}

// Number of 32-bit words holding one vector's 16k stream bits.
template <int K> struct Chunk { static constexpr int NW = (K + 1) / 2; };

// Load one vector's 2K stream bytes that start at `p` as big-endian words
// (bit 31 of w[0] is the vector's first stream bit).  `p` is 4-byte aligned
// for even K, 2-byte aligned for odd K.
template <int K>
__device__ __forceinline__ void load_chunk_words(const uint8_t *p, uint32_t *w) {
    if constexpr (K % 2 == 0) {
#pragma unroll
        for (int i = 0; i < K / 2; ++i)
            w[i] = bswap32(reinterpret_cast<const uint32_t *>(p)[i]);
    } else {
        const uint16_t *h = reinterpret_cast<const uint16_t *>(p);
#pragma unroll
        for (int i = 0; i < K / 2; ++i)
            w[i] = bswap32((uint32_t)h[2 * i] | ((uint32_t)h[2 * i + 1] << 16));
        w[K / 2] = bswap32((uint32_t)h[K - 1]);
    }
}

// Same with byte accesses and a bit offset r in 0..7 (misaligned stream
// pointer or k*t0 not byte aligned).  Reads 2K bytes, plus one if r > 0.
template <int K>
__device__ __forceinline__ void load_chunk_bytes(const uint8_t *p, uint32_t r, uint32_t *w) {
    constexpr int NB = 2 * K;
    uint32_t b[NB + 1];
#pragma unroll
    for (int i = 0; i < NB; ++i) b[i] = p[i];
    b[NB] = r ? p[NB] : 0u;
    uint32_t W[Chunk<K>::NW + 1];
#pragma unroll
    for (int i = 0; i <= Chunk<K>::NW; ++i) {
        uint32_t v = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int idx = 4 * i + j;
            v = (v << 8) | (idx <= NB ? b[idx] : 0u);
        }
        W[i] = v;
    }
#pragma unroll
    for (int i = 0; i < Chunk<K>::NW; ++i)
        w[i] = r ? ((W[i] << r) | (W[i + 1] >> (32 - r))) : W[i];
}

// Field f (0..15) of a vector: K bits at chunk bit offset K*f.
template <int K>
__device__ __forceinline__ uint32_t get_field(const uint32_t *w, int f) {
    constexpr uint32_t low = (1u << K) - 1u;
    const int off = K * f;
    const int i = off >> 5, sh = off & 31;
    if (sh + K <= 32) return (w[i] >> (32 - sh - K)) & low;
    return ((w[i] << (sh + K - 32)) | (w[i + 1] >> (64 - sh - K))) & low;
}

template <int K>
__device__ __forceinline__ void put_field(uint32_t *w, int f, uint32_t v) {
    const int off = K * f;
    const int i = off >> 5, sh = off & 31;
    if (sh + K <= 32) {
        w[i] |= v << (32 - sh - K);
    } else {
        w[i] |= v >> (sh + K - 32);
        w[i + 1] |= v << (64 - sh - K);
    }
}

// Embed 16 fields: byte f of the vector keeps its bits above the field and
// takes field f of the chunk (Section VI step 7f, k-bit masks).
template <int K>
__device__ __forceinline__ u32x4 embed_vec(u32x4 c, const uint32_t *w) {
    u32x4 o;
    if constexpr (K == 1) {
        // The 16 stream bits sit in w[0] bits 31..16.  Reverse them so stream
        // bit f is bit f, then spread each nibble to the LSBs of 4 bytes with
        // one 24-bit multiply (shifts 0, 7, 14, 21 never overlap).
        const uint32_t r = __builtin_bitreverse32(w[0]);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t nib = (r >> (4 * d)) & 0xFu;
            const uint32_t spread = (nib * 0x204081u) & 0x01010101u;
            o[d] = (c[d] & 0xFEFEFEFEu) | spread;
        }
    } else if constexpr (K == 8) {
#pragma unroll
        for (int d = 0; d < 4; ++d) o[d] = bswap32(w[d]);
    } else {
        constexpr uint32_t low = (1u << K) - 1u;
        constexpr uint32_t keep = ~(low * 0x01010101u);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t f = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) f |= get_field<K>(w, 4 * d + j) << (8 * j);
            o[d] = (c[d] & keep) | f;
        }
    }
    return o;
}

// Extract 16 fields into the chunk's big-endian words (Section VII step 6:
// mask the field, shift it to its place, OR into zeroed data).
template <int K>
__device__ __forceinline__ void extract_vec(u32x4 c, uint32_t *w) {
#pragma unroll
    for (int i = 0; i < Chunk<K>::NW; ++i) w[i] = 0;
    if constexpr (K == 1) {
        // Gather the 4 LSBs of a dword into a nibble, first byte highest:
        // one multiply moves byte j's LSB (bit 8j) to bit 31-j.
        uint32_t v = 0;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t nib = ((c[d] & 0x01010101u) * 0x80402010u) >> 28;
            v |= nib << (28 - 4 * d);
        }
        w[0] = v;
    } else if constexpr (K == 8) {
#pragma unroll
        for (int d = 0; d < 4; ++d) w[d] = bswap32(c[d]);
    } else {
        constexpr uint32_t low = (1u << K) - 1u;
#pragma unroll
        for (int f = 0; f < 16; ++f) put_field<K>(w, f, (c[f >> 2] >> (8 * (f & 3))) & low);
    }
}

// Store one vector's 2K stream bytes from big-endian words at `p` (4-byte
// aligned for even K, 2-byte aligned for odd K).
template <int K>
__device__ __forceinline__ void store_chunk_words(uint8_t *p, const uint32_t *w) {
    if constexpr (K % 2 == 0) {
#pragma unroll
        for (int i = 0; i < K / 2; ++i) reinterpret_cast<uint32_t *>(p)[i] = bswap32(w[i]);
    } else {
        uint16_t *h = reinterpret_cast<uint16_t *>(p);
#pragma unroll
        for (int i = 0; i < K / 2; ++i) {
            const uint32_t le = bswap32(w[i]);
            h[2 * i] = (uint16_t)le;
            h[2 * i + 1] = (uint16_t)(le >> 16);
        }
        h[K - 1] = (uint16_t)bswap32(w[K / 2]);
    }
}

// -------------------------------------------------------------------------
// Per-byte forms used for edge vectors and for misaligned buffers.

// Embed buffer byte t.  Writes nothing for a copy-only byte of an in-place span.
// KC > 0 fixes k at compile time (as in the range functions); 0 reads s.k.
template <int KC = 0>
__device__ __forceinline__ void embed_byte(const Span &s, uint64_t t) {
    const uint32_t k = KC > 0 ? (uint32_t)KC : (uint32_t)s.k;
    const uint64_t first = (uint64_t)k * (s.t0 + t);
    const uint32_t c = s.src[t];
    if (first >= s.bits) {
        if (!s.inplace) s.dst[t] = (uint8_t)c;
        return;
    }
    const uint64_t left = s.bits - first;
    const uint32_t nb = left < k ? (uint32_t)left : k;
    // the nb bits start at bit (first % 8) of stream byte first/8 and span at
    // most two bytes
    const uint64_t byte = first >> 3;
    const uint32_t bit = (uint32_t)(first & 7);
    uint32_t pair = stream_byte(s, byte) << 8;
    if (bit + nb > 8) pair |= stream_byte(s, byte + 1);
    const uint32_t v = (pair >> (16 - bit - nb)) & ((1u << nb) - 1u);
    const uint32_t shift = k - nb;
    const uint32_t mask = ((1u << nb) - 1u) << shift;
    s.dst[t] = (uint8_t)((c & ~mask) | (v << shift));
}

// Compute logical stream byte i (which must start at or after field t0 and
// before the span's end bit s.bits) from the stego bytes; bits at or past
// s.bits read as zero.
template <int KC = 0>
__device__ __forceinline__ uint32_t extract_stream_byte(const Span &s, uint64_t i) {
    const uint32_t k = KC > 0 ? (uint32_t)KC : (uint32_t)s.k;
    const uint32_t low = (1u << k) - 1u;
    const uint64_t b0 = 8 * i;
    const uint64_t b1 = (b0 + 8 < s.bits) ? b0 + 8 : s.bits;  // exclusive, > b0
    const uint64_t g_first = b0 / k, g_last = (b1 - 1) / k;
    uint32_t acc = 0, nbits = 0;  // fields g_first..g_last, first bit highest
    for (uint64_t g = g_first; g <= g_last; ++g) {
        acc = (acc << k) | (s.src[g - s.t0] & low);
        nbits += k;
    }
    const uint32_t skip = (uint32_t)(b0 - (uint64_t)k * g_first);
    uint32_t v = ((acc << (32 - nbits)) << skip) >> 24;
    const uint32_t valid = (uint32_t)(b1 - b0);
    return v & ((0xFF00u >> valid) & 0xFFu);
}

// -------------------------------------------------------------------------
// Span walkers.  A team of `n_waves` waves (a whole grid, or one block) walks
// vectors [v_begin, v_end) of a span in groups of 64*UNR vectors; wave
// `wave` takes groups wave, wave + n_waves, ...

template <int K, int UNR, bool NT>
__device__ __forceinline__ void embed_walk(const Span &s, const Ranges &r, uint64_t v_begin,
                                           uint64_t v_end, uint64_t wave, uint64_t n_waves,
                                           uint32_t lane) {
    constexpr uint64_t G = 64 * UNR;
    const uint64_t sb = stream_byte0(s);
    const uint32_t rbit = (uint32_t)(((uint64_t)K * s.t0) & 7);
    // address of stream byte sb + 2K*u is body_base + 2K*u, valid for fast u
    const uintptr_t body_base = (uintptr_t)s.body + sb - s.hdr_len;
    for (uint64_t u0 = v_begin + wave * G; u0 < v_end; u0 += n_waves * G) {
        const uint64_t u_hi = u0 + G;
        if (u0 >= r.fast_begin && u_hi <= r.fast_end && u_hi <= v_end) {
            u32x4 c[UNR];
            uint32_t w[UNR][Chunk<K>::NW];
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const uint64_t u = u0 + (uint64_t)j * 64 + lane;
                c[j] = load16<NT>(s.src + 16 * u);
                const uint8_t *p = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u);
                if (s.words) load_chunk_words<K>(p, w[j]);
                else load_chunk_bytes<K>(p, rbit, w[j]);
            }
#pragma unroll
            for (int j = 0; j < UNR; ++j) {
                const uint64_t u = u0 + (uint64_t)j * 64 + lane;
                store16<NT>(s.dst + 16 * u, embed_vec<K>(c[j], w[j]));
            }
        } else if (u0 >= r.copy_begin && u_hi <= r.copy_end && u_hi <= v_end) {
            if (!s.inplace) {
                u32x4 c[UNR];
#pragma unroll
                for (int j = 0; j < UNR; ++j)
                    c[j] = load16<NT>(s.src + 16 * (u0 + (uint64_t)j * 64 + lane));
#pragma unroll
                for (int j = 0; j < UNR; ++j)
                    store16<NT>(s.dst + 16 * (u0 + (uint64_t)j * 64 + lane), c[j]);
            }
        } else {
            for (int j = 0; j < UNR; ++j) {
                const uint64_t u = u0 + (uint64_t)j * 64 + lane;
                if (u >= v_end) continue;
                if (u >= r.fast_begin && u < r.fast_end) {
                    uint32_t w[Chunk<K>::NW];
                    const uint8_t *p = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u);
                    if (s.words) load_chunk_words<K>(p, w);
                    else load_chunk_bytes<K>(p, rbit, w);
                    store16<NT>(s.dst + 16 * u, embed_vec<K>(load16<NT>(s.src + 16 * u), w));
                } else if (u >= r.copy_begin && u < r.copy_end) {
                    if (!s.inplace) store16<NT>(s.dst + 16 * u, load16<NT>(s.src + 16 * u));
                } else {
                    const uint64_t t_end = 16 * u + 16 < s.n ? 16 * u + 16 : s.n;
                    for (uint64_t t = 16 * u; t < t_end; ++t) embed_byte<K>(s, t);
                }
            }
        }
    }
}

// Store the stream bytes of one fast wave group whose stego vectors are in c.
// Every vector of the group is extracted before the first store, and the
// stores sit in one branch on the stream side's width: with a branch per
// vector, the wait inserted where the two store paths join made the wave
// wait for each vector's store to complete before extracting the next.
template <int K, int UNR>
__device__ __forceinline__ void extract_store_group(const Span &s, uintptr_t out_base, uint64_t u0,
                                                    const u32x4 *c, uint32_t lane) {
    uint32_t w[UNR][Chunk<K>::NW];
#pragma unroll
    for (int j = 0; j < UNR; ++j) extract_vec<K>(c[j], w[j]);
    uint8_t *p0 = reinterpret_cast<uint8_t *>(out_base + 2 * K * (u0 + lane));
    if (s.words) {
#pragma unroll
        for (int j = 0; j < UNR; ++j) store_chunk_words<K>(p0 + 2 * K * 64 * j, w[j]);
    } else {
#pragma unroll
        for (int j = 0; j < UNR; ++j)
#pragma unroll
            for (int i = 0; i < 2 * K; ++i)
                p0[2 * K * 64 * j + i] = (uint8_t)(w[j][i >> 2] >> (24 - 8 * (i & 3)));
    }
}

// Same for k = 1 with wavefront ballots.  The wave's 1 KiB of stego bytes
// per vector set is staged in LDS so that lane L can read bytes L, L+64, ...,
// L+960; ballot m over their LSBs then holds 64 consecutive stream bits
// (bit L = stream bit 64m + L), i.e. 8 output bytes, which a per-byte bit
// reversal puts in MSB-first order.  Lanes 0..15 store the 16 ballots.
// `stage` is this wave's 1 KiB of LDS.  Must be called by all 64 lanes.
template <int UNR>
__device__ __forceinline__ void extract_store_group_ballot(const Span &s, uintptr_t out_base, uint64_t u0,
                                                           const u32x4 *c, uint32_t lane, uint8_t *stage) {
#pragma unroll
    for (int j = 0; j < UNR; ++j) {
        *reinterpret_cast<u32x4 *>(stage + 16 * lane) = c[j];
        uint32_t bits = 0;
#pragma unroll
        for (int m = 0; m < 16; ++m) bits |= ((uint32_t)stage[lane + 64 * m] & 1u) << m;
        uint64_t mine = 0;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const uint64_t mask = __ballot((bits >> m) & 1u);
            mine = lane == (uint32_t)m ? mask : mine;
        }
        if (lane < 16) {
            const uint64_t v = __builtin_bswap64(__builtin_bitreverse64(mine));
            uint8_t *p = reinterpret_cast<uint8_t *>(out_base + 2 * (u0 + (uint64_t)j * 64) + 8 * lane);
            if (s.words) {
                reinterpret_cast<uint32_t *>(p)[0] = (uint32_t)v;
                reinterpret_cast<uint32_t *>(p)[1] = (uint32_t)(v >> 32);
            } else {
#pragma unroll
                for (int b = 0; b < 8; ++b) p[b] = (uint8_t)(v >> (8 * b));
            }
        }
    }
}

__host__ __device__ inline uintptr_t extract_out_base(const Span &s) {
    return (uintptr_t)s.out + stream_byte0(s) - s.hdr_len;
}

// BALLOT (k = 1 only): pack fast groups with wavefront ballots through the
// wave's 1 KiB LDS `stage` instead of per-lane multiplies.
template <int K, int UNR, bool NT, bool BALLOT = false>
__device__ __forceinline__ void extract_walk(const Span &s, const Ranges &r, uint64_t v_begin,
                                             uint64_t v_end, uint64_t wave, uint64_t n_waves,
                                             uint32_t lane, uint8_t *stage = nullptr) {
    constexpr uint64_t G = 64 * UNR;
    const uint64_t sb = stream_byte0(s);
    const uintptr_t out_base = extract_out_base(s);
    for (uint64_t u0 = v_begin + wave * G; u0 < v_end; u0 += n_waves * G) {
        const uint64_t u_hi = u0 + G;
        if (u0 >= r.fast_begin && u_hi <= r.fast_end && u_hi <= v_end) {
            u32x4 c[UNR];
#pragma unroll
            for (int j = 0; j < UNR; ++j)
                c[j] = load16<NT>(s.src + 16 * (u0 + (uint64_t)j * 64 + lane));
            if constexpr (BALLOT && K == 1)
                extract_store_group_ballot<UNR>(s, out_base, u0, c, lane, stage);
            else
                extract_store_group<K, UNR>(s, out_base, u0, c, lane);
        } else {
            for (int j = 0; j < UNR; ++j) {
                const uint64_t u = u0 + (uint64_t)j * 64 + lane;
                if (u >= v_end) continue;
                uint8_t *p = reinterpret_cast<uint8_t *>(out_base + 2 * K * u);
                if (u >= r.fast_begin && u < r.fast_end) {
                    uint32_t w[Chunk<K>::NW];
                    extract_vec<K>(load16<NT>(s.src + 16 * u), w);
                    if (s.words) {
                        store_chunk_words<K>(p, w);
                    } else {
                        for (int i = 0; i < 2 * K; ++i) p[i] = (uint8_t)(w[i >> 2] >> (24 - 8 * (i & 3)));
                    }
                } else {
                    const uint64_t i0 = sb + 2 * K * u;
                    const uint64_t end_byte = ceil_div(s.bits, 8);
                    for (uint64_t i = i0; i < i0 + 2 * K && i < end_byte; ++i) {
                        if (i < s.hdr_len) continue;
                        s.out[i - s.hdr_len] = (uint8_t)extract_stream_byte<K>(s, i);
                    }
                }
            }
        }
    }
}

// Decode the 32-bit length header from the first ceil(32/k) stego bytes with
// one ballot: lane j (< 32) reads stream bit j, the ballot's low 32 bits are
// the header bits in reverse order.  Caller guarantees n*k >= 32.
__device__ __forceinline__ uint32_t decode_header(const uint8_t *stego, int k, uint32_t lane) {
    uint32_t bit = 0;
    if (lane < 32) {
        const uint32_t t = lane / (uint32_t)k, q = lane % (uint32_t)k;
        bit = (stego[t] >> ((uint32_t)k - 1 - q)) & 1u;
    }
    const uint64_t m = __ballot(bit);
    return __builtin_bitreverse32((uint32_t)m);
}

// floor(n*k/8) without overflow.
__host__ __device__ inline uint64_t room_bytes(uint64_t n, int k) {
    return (n / 8) * (uint64_t)k + ((n % 8) * (uint64_t)k) / 8;
}

}  // namespace lsb
