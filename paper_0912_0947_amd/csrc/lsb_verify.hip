// lsb_verify.hip -- round-trip checks of a stego buffer in one launch
// (arXiv:0912.0947: embedding is Section VI step 7, extraction Section VII
// step 6; extraction reverses embedding).
//
// A stego byte t is right when
//   - the bits of its field that carry stream bits, read back as extraction
//     reads them (mask the field, shift it down), equal those stream bits, and
//   - every other bit (above the field; the low bits of a partial last field;
//     all bits of a byte past the stream) equals the cover's.
// Both checks go through the extraction side of the method (extract_vec on a
// whole vector, or the per-byte field read), never through the embedding
// arithmetic, so an embedding mistake shows up as a mismatch.
//
// lsb_verify reads cover, stego and stream once (2n + |S| bytes) and counts
// wrong stego bytes.  lsb_embed_verify embeds (as lsb_embed) and, in the same
// launch, checks every byte it writes in this way: the round trip of each
// vector happens in registers, so the check costs no memory traffic beyond
// the embed's own 2n + |S| bytes.
#include <hip/hip_ext.h>

#include "lsb_host.hpp"

namespace lsb {

// Stream bits carried by field t: their count nb (0 past the stream) and
// value v, first bit highest.
__device__ __forceinline__ uint32_t stream_field(const Span &s, uint64_t t, uint32_t *nb_out) {
    const uint32_t k = (uint32_t)s.k;
    const uint64_t first = (uint64_t)k * (s.t0 + t);
    if (first >= s.bits) {
        *nb_out = 0;
        return 0;
    }
    const uint64_t left = s.bits - first;
    const uint32_t nb = left < k ? (uint32_t)left : k;
    const uint64_t byte = first >> 3;
    const uint32_t bit = (uint32_t)(first & 7);
    uint32_t pair = stream_byte(s, byte) << 8;
    if (bit + nb > 8) pair |= stream_byte(s, byte + 1);
    *nb_out = nb;
    return (pair >> (16 - bit - nb)) & ((1u << nb) - 1u);
}

// 1 if stego byte g at buffer position t is wrong for cover byte c.
__device__ __forceinline__ uint32_t byte_wrong(const Span &s, uint64_t t, uint32_t c, uint32_t g) {
    uint32_t nb;
    const uint32_t v = stream_field(s, t, &nb);
    if (!nb) return g != c;
    const uint32_t shift = (uint32_t)s.k - nb;
    const uint32_t mask = ((1u << nb) - 1u) << shift;
    const uint32_t read_back = (g & mask) >> shift;  // Section VII step 6 on this byte
    return (read_back != v) | (((g ^ c) & ~mask & 0xFFu) != 0);
}

// Wrong bytes of a fast vector (all 16 fields carry K stream bits): extract
// the stego vector's fields into stream words, compare them with the stream
// chunk w, and compare the bits above the fields with the cover's.  Whole
// words first: when every word reads back and no kept bit changed (a
// correct embedding) the vector costs a few compares; only a vector with a
// difference is counted field by field and byte by byte.
template <int K>
__device__ __forceinline__ uint32_t vec_wrong(u32x4 c, u32x4 g, const uint32_t *w) {
    uint32_t got[Chunk<K>::NW];
    extract_vec<K>(g, got);
    uint32_t diff[Chunk<K>::NW];
    uint32_t any = 0;
#pragma unroll
    for (int i = 0; i < Chunk<K>::NW; ++i) {
        diff[i] = got[i] ^ w[i];
        any |= diff[i];
    }
    if constexpr (K < 8) {
        constexpr uint32_t keep_bits = ~(((1u << K) - 1u) * 0x01010101u);
#pragma unroll
        for (int d = 0; d < 4; ++d) any |= (c[d] ^ g[d]) & keep_bits;
    }
    if (!any) return 0;
    uint32_t bad = 0;  // bit f: byte f of the vector is wrong
#pragma unroll
    for (int f = 0; f < 16; ++f) bad |= (get_field<K>(diff, f) != 0 ? 1u : 0u) << f;
    if constexpr (K < 8) {
        constexpr uint32_t keep = ~(((1u << K) - 1u) * 0x01010101u);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t x = (c[d] ^ g[d]) & keep;
#pragma unroll
            for (int j = 0; j < 4; ++j) bad |= (((x >> (8 * j)) & 0xFFu) != 0 ? 1u : 0u) << (4 * d + j);
        }
    }
    return (uint32_t)__builtin_popcount(bad);
}

__device__ __forceinline__ uint32_t bytes_differ(u32x4 a, u32x4 b) {
    uint32_t n = 0;
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        const uint32_t x = a[d] ^ b[d];
#pragma unroll
        for (int j = 0; j < 4; ++j) n += ((x >> (8 * j)) & 0xFFu) != 0;
    }
    return n;
}

// Sum `bad` over the block (256 threads) and add it to the counter.
__device__ __forceinline__ void add_block_count(uint32_t bad, unsigned long long *mismatches) {
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
    __shared__ uint32_t part[4];
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t sum = part[0] + part[1] + part[2] + part[3];
        if (sum) atomicAdd(mismatches, (unsigned long long)sum);
    }
}

// Check only: s.src = cover, s.dst = stego (read only here).  One vector u
// of the span (any class).
template <int K>
__device__ __forceinline__ uint32_t verify_one(const Span &s, const Ranges &r, uintptr_t body_base, uint64_t u) {
    if (u >= r.fast_begin && u < r.fast_end) {
        uint32_t w[Chunk<K>::NW];
        const uint8_t *p = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u);
        if (s.words) load_chunk_words<K>(p, w);
        else load_chunk_bytes<K>(p, 0, w);
        return vec_wrong<K>(load16<true>(s.src + 16 * u), load16<true>(s.dst + 16 * u), w);
    }
    if (u >= r.copy_begin && u < r.copy_end)
        return bytes_differ(load16<true>(s.src + 16 * u), load16<true>(s.dst + 16 * u));
    uint32_t bad = 0;
    const uint64_t t_end = 16 * u + 16 < s.n ? 16 * u + 16 : s.n;
    for (uint64_t t = 16 * u; t < t_end; ++t) bad += byte_wrong(s, t, s.src[t], s.dst[t]);
    return bad;
}

// A block covers 512 vectors per pass, two per thread (vectors v and v + 256
// of the pass), as in the embedding form below.
template <int K>
__global__ void __launch_bounds__(256) lsb_verify_kernel(Span s, unsigned long long *mismatches) {
    const Ranges r = embed_ranges<K>(s);  // inplace = 0: every vector is visited
    const uint64_t stride = (uint64_t)gridDim.x * 512;
    const uintptr_t body_base = (uintptr_t)s.body - s.hdr_len;
    uint32_t bad = 0;
    for (uint64_t u0 = (uint64_t)blockIdx.x * 512 + threadIdx.x; u0 < r.count; u0 += stride) {
        const uint64_t u1 = u0 + 256;
        if (u0 >= r.fast_begin && u1 < r.fast_end) {
            uint32_t w0[Chunk<K>::NW], w1[Chunk<K>::NW];
            const uint8_t *p0 = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u0);
            const uint8_t *p1 = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u1);
            if (s.words) {
                load_chunk_words<K>(p0, w0);
                load_chunk_words<K>(p1, w1);
            } else {
                load_chunk_bytes<K>(p0, 0, w0);
                load_chunk_bytes<K>(p1, 0, w1);
            }
            const u32x4 c0 = load16<true>(s.src + 16 * u0), g0 = load16<true>(s.dst + 16 * u0);
            const u32x4 c1 = load16<true>(s.src + 16 * u1), g1 = load16<true>(s.dst + 16 * u1);
            bad += vec_wrong<K>(c0, g0, w0) + vec_wrong<K>(c1, g1, w1);
        } else {
            bad += verify_one<K>(s, r, body_base, u0);
            if (u1 < r.count) bad += verify_one<K>(s, r, body_base, u1);
        }
    }
    add_block_count(bad, mismatches);
}

// Embed and check one vector u of the span (any class).  A fast vector is
// embedded in registers, stored, and its stored value is checked against
// the stream through extraction; an edge vector is embedded byte by byte
// and each byte this thread wrote is read back.
template <int K>
__device__ __forceinline__ uint32_t embed_verify_one(const Span &s, const Ranges &r, uintptr_t body_base,
                                                     uint64_t u) {
    if (u >= r.fast_begin && u < r.fast_end) {
        uint32_t w[Chunk<K>::NW];
        const uint8_t *p = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u);
        if (s.words) load_chunk_words<K>(p, w);
        else load_chunk_bytes<K>(p, 0, w);
        const u32x4 c = load16<true>(s.src + 16 * u);
        const u32x4 g = embed_vec<K>(c, w);
        store16<true>(s.dst + 16 * u, g);
        return vec_wrong<K>(c, g, w);
    }
    if (u >= r.copy_begin && u < r.copy_end) {
        if (!s.inplace) store16<true>(s.dst + 16 * u, load16<true>(s.src + 16 * u));
        return 0;
    }
    uint32_t bad = 0;
    const uint64_t t_end = 16 * u + 16 < s.n ? 16 * u + 16 : s.n;
    for (uint64_t t = 16 * u; t < t_end; ++t) {
        const uint32_t c = s.src[t];
        embed_byte<K>(s, t);
        bad += byte_wrong(s, t, c, s.dst[t]);
    }
    return bad;
}

// Embed and check in one launch: s.src = cover, s.dst = stego (may equal
// cover).  A block covers 512 vectors per pass, two per thread (vectors v
// and v + 256 of the pass, so each load instruction of a wave stays
// contiguous); when both are fast their loads are issued before either is
// embedded.
template <int K>
__global__ void __launch_bounds__(256) lsb_embed_verify_kernel(Span s, unsigned long long *mismatches) {
    const Ranges r = embed_ranges<K>(s);
    const uint64_t stride = (uint64_t)gridDim.x * 512;
    const uintptr_t body_base = (uintptr_t)s.body - s.hdr_len;
    uint32_t bad = 0;
    for (uint64_t u0 = (uint64_t)blockIdx.x * 512 + threadIdx.x; u0 < r.count; u0 += stride) {
        const uint64_t u1 = u0 + 256;
        if (u0 >= r.fast_begin && u1 < r.fast_end) {
            uint32_t w0[Chunk<K>::NW], w1[Chunk<K>::NW];
            const uint8_t *p0 = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u0);
            const uint8_t *p1 = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u1);
            if (s.words) {
                load_chunk_words<K>(p0, w0);
                load_chunk_words<K>(p1, w1);
            } else {
                load_chunk_bytes<K>(p0, 0, w0);
                load_chunk_bytes<K>(p1, 0, w1);
            }
            const u32x4 c0 = load16<true>(s.src + 16 * u0);
            const u32x4 c1 = load16<true>(s.src + 16 * u1);
            const u32x4 g0 = embed_vec<K>(c0, w0);
            const u32x4 g1 = embed_vec<K>(c1, w1);
            store16<true>(s.dst + 16 * u0, g0);
            store16<true>(s.dst + 16 * u1, g1);
            bad += vec_wrong<K>(c0, g0, w0) + vec_wrong<K>(c1, g1, w1);
        } else {
            bad += embed_verify_one<K>(s, r, body_base, u0);
            if (u1 < r.count) bad += embed_verify_one<K>(s, r, body_base, u1);
        }
    }
    add_block_count(bad, mismatches);
}

// Per-byte forms for buffers whose cover or stego pointer is not 16-byte
// aligned.
__global__ void __launch_bounds__(256) lsb_verify_bytes_kernel(Span s, unsigned long long *mismatches) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < s.n; t += stride)
        bad += byte_wrong(s, t, s.src[t], s.dst[t]);
    add_block_count(bad, mismatches);
}

__global__ void __launch_bounds__(256) lsb_embed_verify_bytes_kernel(Span s, unsigned long long *mismatches) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < s.n; t += stride) {
        const uint32_t c = s.src[t];
        embed_byte(s, t);
        bad += byte_wrong(s, t, c, s.dst[t]);
    }
    add_block_count(bad, mismatches);
}

// The counter is cleared by a kernel (not a memset node), so that the call
// can sit in a captured graph.
__global__ void lsb_verify_zero_kernel(unsigned long long *p) { *p = 0; }

typedef void (*VerifyFn)(Span, unsigned long long *);

template <int K>
struct VerifyK {
    static constexpr VerifyFn fn = lsb_verify_kernel<K>;
};
template <int K>
struct EmbedVerifyK {
    static constexpr VerifyFn fn = lsb_embed_verify_kernel<K>;
};

template <template <int> class F>
static VerifyFn fn_for_k(int k) {
    switch (k) {
        case 1: return F<1>::fn;
        case 2: return F<2>::fn;
        case 3: return F<3>::fn;
        case 4: return F<4>::fn;
        case 5: return F<5>::fn;
        case 6: return F<6>::fn;
        case 7: return F<7>::fn;
        default: return F<8>::fn;
    }
}

// Shared argument checks and launch of both entry points.
static int verify_call(const char *name, bool embed, const uint8_t *cover, uint8_t *stego, uint64_t n,
                       const uint8_t *msg, uint32_t len, int k, uint64_t *mismatches_dev, void *stream) {
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "%s: k=%d outside 1..8", name, k);
    const int64_t cap = lsb_capacity(n, k);
    if (cap < 0) return (int)cap;
    if ((uint64_t)len > (uint64_t)cap)
        return fail(LSB_E_CAPACITY, "%s: message of %u bytes exceeds capacity %lld", name, len, (long long)cap);
    if (!cover || !stego || !mismatches_dev) return fail(LSB_E_ARG, "%s: null pointer", name);
    if (len && !msg) return fail(LSB_E_ARG, "%s: null msg", name);
    if (overlaps(mismatches_dev, 8, cover, n) || overlaps(mismatches_dev, 8, stego, n) ||
        overlaps(mismatches_dev, 8, msg, len))
        return fail(LSB_E_ARG, "%s: counter overlaps a buffer", name);
    if (embed) {
        if (cover != stego && overlaps(cover, n, stego, n))
            return fail(LSB_E_ARG, "%s: cover and stego overlap (only stego == cover is allowed)", name);
        if (overlaps(msg, len, stego, n)) return fail(LSB_E_ARG, "%s: msg overlaps stego", name);
    }
    Span s{};
    s.src = cover;
    s.dst = stego;
    s.body = msg;
    s.n = n;
    s.bits = 8 * (4 + (uint64_t)len);
    s.hdr = len;
    s.hdr_len = 4;
    s.k = k;
    s.inplace = embed && cover == stego;
    s.words = (((uintptr_t)msg - 4) & 3u) == 0;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *cnt = (unsigned long long *)mismatches_dev;
    hipLaunchKernelGGL(lsb_verify_zero_kernel, dim3(1), dim3(1), 0, st, cnt);
    const bool vec = (((uintptr_t)cover | (uintptr_t)stego) & 15u) == 0;
    uint64_t items = vec ? ceil_div(n, 16) : n;
    if (vec && s.inplace) items = embed_ranges(s).count;  // in place: bytes past the stream stay untouched
    // The vector kernels' blocks cover 512 vectors per pass, and the grid
    // gives every pair of vectors a thread: on a grid capped at 8 blocks
    // per CU the waves loop, and a looping wave's wait for its next loads
    // also waits for its previous stores (one counter covers both).  The
    // capped grid measured slower for the check alone too.  A correct
    // embedding adds nothing to the counter, so the larger grid costs no
    // atomics.
    uint64_t blocks = ceil_div(items ? items : 1, vec ? 512 : 256);
    if (blocks > (uint64_t)INT32_MAX) blocks = (uint64_t)INT32_MAX;
    VerifyFn fn = vec ? (embed ? fn_for_k<EmbedVerifyK>(k) : fn_for_k<VerifyK>(k))
                      : (embed ? lsb_embed_verify_bytes_kernel : lsb_verify_bytes_kernel);
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    hipExtLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(256), 0, st, e0, e1, 0, s, cnt);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "verify kernel launch");
}

}  // namespace lsb

using namespace lsb;

extern "C" int lsb_verify(const uint8_t *cover, const uint8_t *stego, uint64_t n, const uint8_t *msg, uint32_t len,
                          int k, uint64_t *mismatches_dev, void *stream) {
    const TimedCall timed_call;
    return verify_call("lsb_verify", false, cover, const_cast<uint8_t *>(stego), n, msg, len, k, mismatches_dev,
                       stream);
}

extern "C" int lsb_embed_verify(const uint8_t *cover, uint8_t *stego, uint64_t n, const uint8_t *msg, uint32_t len,
                                int k, uint64_t *mismatches_dev, void *stream) {
    const TimedCall timed_call;
    return verify_call("lsb_embed_verify", true, cover, stego, n, msg, len, k, mismatches_dev, stream);
}
