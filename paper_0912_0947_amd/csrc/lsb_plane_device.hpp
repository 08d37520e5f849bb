// lsb_plane_device.hpp -- device code for one colour plane with the general
// method (arXiv:0912.0947, Section VI step 2 / Section VII step 2 select the
// plane; steps VI.7 / VII.6 place and gather the bits).  Included by
// lsb_plane.hip.
#pragma once

#include "../../include/lsb.h"
#include "lsb_device.hpp"

namespace lsb {

// Buffer byte of field t in a plane view.
__device__ __forceinline__ uint64_t plane_byte(uint64_t t, uint32_t c, uint32_t plane) {
    return t * c + plane;
}

// Embed field t of the plane view (Section VI step 7, k-bit fields).
__device__ __forceinline__ void plane_embed_field(const Span &s, uint64_t t, uint32_t c, uint32_t plane) {
    const uint32_t k = (uint32_t)s.k;
    const uint64_t first = (uint64_t)k * t;
    if (first >= s.bits) return;
    const uint64_t left = s.bits - first;
    const uint32_t nb = left < k ? (uint32_t)left : k;
    const uint64_t byte = first >> 3;
    const uint32_t bit = (uint32_t)(first & 7);
    uint32_t pair = stream_byte(s, byte) << 8;
    if (bit + nb > 8) pair |= stream_byte(s, byte + 1);
    const uint32_t v = (pair >> (16 - bit - nb)) & ((1u << nb) - 1u);
    const uint32_t shift = k - nb;
    const uint32_t mask = ((1u << nb) - 1u) << shift;
    const uint64_t at = plane_byte(t, c, plane);
    s.dst[at] = (uint8_t)((s.src[at] & ~mask) | (v << shift));
}

// Stream byte i (>= 4) of a plane view from its fields (Section VII step 6).
__device__ __forceinline__ uint32_t plane_stream_byte(const Span &s, uint64_t i, uint32_t c, uint32_t plane) {
    const uint32_t k = (uint32_t)s.k;
    const uint32_t low = (1u << k) - 1u;
    const uint64_t b0 = 8 * i;
    const uint64_t b1 = (b0 + 8 < s.bits) ? b0 + 8 : s.bits;
    const uint64_t g_first = b0 / k, g_last = (b1 - 1) / k;
    uint32_t acc = 0, nbits = 0;
    for (uint64_t g = g_first; g <= g_last; ++g) {
        acc = (acc << k) | (s.src[plane_byte(g, c, plane)] & low);
        nbits += k;
    }
    const uint32_t skip = (uint32_t)(b0 - (uint64_t)k * g_first);
    const uint32_t v = ((acc << (32 - nbits)) << skip) >> 24;
    const uint32_t valid = (uint32_t)(b1 - b0);
    return v & ((0xFF00u >> valid) & 0xFFu);
}

__global__ void __launch_bounds__(256) lsb_copy_kernel(const uint8_t *src, uint8_t *dst, uint64_t n, int vec) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (vec) {
        const uint64_t nv = n / 16;
        for (uint64_t u = gid; u < nv; u += stride) store16<true>(dst + 16 * u, load16<true>(src + 16 * u));
        for (uint64_t t = 16 * nv + gid; t < n; t += stride) dst[t] = src[t];
    } else {
        for (uint64_t t = gid; t < n; t += stride) dst[t] = src[t];
    }
}

__global__ void __launch_bounds__(256) lsb_plane_embed_kernel(Span s, uint64_t fields, uint32_t c, uint32_t plane) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < fields; t += stride)
        plane_embed_field(s, t, c, plane);
}

// Header decode on the plane view (lane j < 32 reads stream bit j), status
// through block 0, then one lane per message byte.
__global__ void __launch_bounds__(256) lsb_plane_extract_kernel(Span s, uint32_t c, uint32_t plane, uint64_t out_cap,
                                                                uint32_t *len_out, int32_t *status_out) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t k = (uint32_t)s.k;
    uint32_t len = 0;
    int status = LSB_E_HEADER;
    if ((uint64_t)k * s.n >= 32) {
        uint32_t bit = 0;
        if (lane < 32) bit = (s.src[plane_byte(lane / k, c, plane)] >> (k - 1 - lane % k)) & 1u;
        len = __builtin_bitreverse32((uint32_t)__ballot(bit));
        if (4 + (uint64_t)len > room_bytes(s.n, (int)k)) status = LSB_E_HEADER;
        else if ((uint64_t)len > out_cap) status = LSB_E_BUFFER;
        else status = LSB_OK;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *len_out = len;
        *status_out = status;
    }
    if (status != LSB_OK) return;
    s.bits = 8 * (4 + (uint64_t)len);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; m < len; m += stride)
        s.out[m] = (uint8_t)plane_stream_byte(s, m + 4, c, plane);
}

// ---------------------------------------------------------------------------
// Vector form for C in {2, 3, 4} channels: a lane moves 16 pixels = C
// 16-byte vectors, gathers their plane bytes into one 16-field vector, runs
// the plain vector embed / extract on it and scatters the result back.  All
// byte positions are compile-time constants (C and PLANE are template
// parameters), so the gather and scatter are register bit-field moves.
template <int C, int PLANE>
__device__ __forceinline__ u32x4 plane_gather(const u32x4 *v) {
    u32x4 p = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int f = 0; f < 16; ++f) {
        const int b = f * C + PLANE;
        const uint32_t byte = (v[b >> 4][(b & 15) >> 2] >> (8 * (b & 3))) & 0xFFu;
        p[f >> 2] |= byte << (8 * (f & 3));
    }
    return p;
}

template <int C, int PLANE>
__device__ __forceinline__ void plane_scatter(u32x4 *v, u32x4 p) {
#pragma unroll
    for (int f = 0; f < 16; ++f) {
        const int b = f * C + PLANE;
        const uint32_t byte = (p[f >> 2] >> (8 * (f & 3))) & 0xFFu;
        const int sh = 8 * (b & 3);
        v[b >> 4][(b & 15) >> 2] = (v[b >> 4][(b & 15) >> 2] & ~(0xFFu << sh)) | (byte << sh);
    }
}

template <int K, int C, int PLANE>
__device__ __forceinline__ void plane_embed_vec(u32x4 *v, const uint32_t *w) {
    plane_scatter<C, PLANE>(v, embed_vec<K>(plane_gather<C, PLANE>(v), w));
}

template <int K, int C>
__device__ __forceinline__ void plane_embed_vec_any(u32x4 *v, const uint32_t *w, uint32_t plane) {
    switch (plane) {  // uniform across the grid
        case 0: plane_embed_vec<K, C, 0>(v, w); break;
        case 1: plane_embed_vec<K, C, 1>(v, w); break;
        case 2: if constexpr (C > 2) plane_embed_vec<K, C, 2>(v, w); break;
        default: if constexpr (C > 3) plane_embed_vec<K, C, 3>(v, w); break;
    }
}

template <int K, int C>
__device__ __forceinline__ u32x4 plane_gather_any(const u32x4 *v, uint32_t plane) {
    switch (plane) {
        case 0: return plane_gather<C, 0>(v);
        case 1: return plane_gather<C, 1>(v);
        case 2: if constexpr (C > 2) return plane_gather<C, 2>(v); break;
        default: if constexpr (C > 3) return plane_gather<C, 3>(v); break;
    }
    return u32x4{0u, 0u, 0u, 0u};
}

// Wave groups: a wave takes 64 consecutive 16-pixel units (64*C vectors,
// C KiB of the interleaved buffer).  When the whole group is fast, the wave
// loads it with C contiguous 1 KiB accesses into LDS, each lane reads back
// its own C vectors (16 pixels), and, for embed, the results go back through
// LDS to C contiguous stores: every global access of the wave covers one
// contiguous span, instead of 64 lanes touching C-vector runs at a stride of
// 16*C bytes.  Other groups (header, stream end, buffer tail) go lane by lane.

// stage[64*i + lane] = vector 64*i + lane of the group.
template <int C>
__device__ __forceinline__ void plane_group_load(const uint8_t *src, u32x4 *stage, uint32_t lane) {
#pragma unroll
    for (int i = 0; i < C; ++i) stage[64 * i + lane] = load16<true>(src + 16 * (64 * i + lane));
}

template <int C>
__device__ __forceinline__ void plane_group_store(uint8_t *dst, const u32x4 *stage, uint32_t lane) {
#pragma unroll
    for (int i = 0; i < C; ++i) store16<true>(dst + 16 * (64 * i + lane), stage[64 * i + lane]);
}

// Embed unit u (16 pixels) whose C vectors are in stage[C*lane .. C*lane + C).
template <int K, int C>
__device__ __forceinline__ void plane_group_embed(const Span &s, u32x4 *stage, uint64_t u, uint32_t lane,
                                                  uint32_t plane) {
    const uintptr_t body_base = (uintptr_t)s.body - s.hdr_len;  // stream byte i at body_base + i
    u32x4 v[C];
#pragma unroll
    for (int i = 0; i < C; ++i) v[i] = stage[C * lane + i];
    uint32_t w[Chunk<K>::NW];
    const uint8_t *p = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u);
    if (s.words) load_chunk_words<K>(p, w);
    else load_chunk_bytes<K>(p, 0, w);
    plane_embed_vec_any<K, C>(v, w, plane);
#pragma unroll
    for (int i = 0; i < C; ++i) stage[C * lane + i] = v[i];
}

// One unit lane by lane (groups that are not wholly fast).
template <int K, int C>
__device__ __forceinline__ void plane_embed_unit(const Span &s, const Ranges &r, uint64_t u, uint32_t plane) {
    uint8_t *dst = s.dst + 16 * C * u;
    const uint8_t *src = s.src + 16 * C * u;
    if (u >= r.fast_begin && u < r.fast_end) {
        const uintptr_t body_base = (uintptr_t)s.body - s.hdr_len;
        u32x4 v[C];
#pragma unroll
        for (int i = 0; i < C; ++i) v[i] = load16<true>(src + 16 * i);
        uint32_t w[Chunk<K>::NW];
        const uint8_t *p = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u);
        if (s.words) load_chunk_words<K>(p, w);
        else load_chunk_bytes<K>(p, 0, w);
        plane_embed_vec_any<K, C>(v, w, plane);
#pragma unroll
        for (int i = 0; i < C; ++i) store16<true>(dst + 16 * i, v[i]);
    } else if (u >= r.copy_begin && u < r.copy_end) {
        if (!s.inplace) {
#pragma unroll
            for (int i = 0; i < C; ++i) store16<true>(dst + 16 * i, load16<true>(src + 16 * i));
        }
    } else {
        const uint64_t px_end = 16 * u + 16 < s.n ? 16 * u + 16 : s.n;
        for (uint64_t px = 16 * u; px < px_end; ++px) {
            if (!s.inplace)
                for (uint32_t ch = 0; ch < (uint32_t)C; ++ch)
                    if (ch != plane) s.dst[px * C + ch] = s.src[px * C + ch];
            const uint64_t at = plane_byte(px, C, plane);
            if ((uint64_t)s.k * px >= s.bits) {
                if (!s.inplace) s.dst[at] = s.src[at];
            } else {
                plane_embed_field(s, px, C, plane);
            }
        }
    }
}

// Group classes (wave-uniform).
enum PlaneGroup { PLANE_FAST = 0, PLANE_COPY = 1, PLANE_EDGE = 2 };

__device__ __forceinline__ int plane_group_class(const Ranges &r, uint64_t u0) {
    if (u0 >= r.fast_begin && u0 + 64 <= r.fast_end) return PLANE_FAST;
    if (u0 >= r.copy_begin && u0 + 64 <= r.copy_end) return PLANE_COPY;
    return PLANE_EDGE;
}

// Embed over the plane view; s.n = pixels, s.src/s.dst the interleaved
// cover/stego (16-byte aligned), header mode (t0 = 0).
template <int K, int C>
__global__ void __launch_bounds__(256) lsb_plane_embed_vec_kernel(Span s, uint32_t plane) {
    __shared__ u32x4 stage_all[4][64 * C];  // one stage per wave of the 256-thread block
    const Ranges r = embed_ranges<K>(s);
    const uint32_t lane = threadIdx.x & 63u;
    u32x4 *stage = stage_all[threadIdx.x >> 6];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t groups = ceil_div(r.count, 64);
    for (uint64_t g = wave; g < groups; g += n_waves) {
        const uint64_t u0 = 64 * g;
        const int cls = plane_group_class(r, u0);
        if (cls == PLANE_FAST) {
            plane_group_load<C>(s.src + 16 * C * u0, stage, lane);
            __builtin_amdgcn_wave_barrier();
            plane_group_embed<K, C>(s, stage, u0 + lane, lane, plane);
            __builtin_amdgcn_wave_barrier();
            plane_group_store<C>(s.dst + 16 * C * u0, stage, lane);
            __builtin_amdgcn_wave_barrier();
        } else if (cls == PLANE_COPY) {
            if (!s.inplace) {
#pragma unroll
                for (int i = 0; i < C; ++i)
                    store16<true>(s.dst + 16 * (C * u0 + 64 * i + lane), load16<true>(s.src + 16 * (C * u0 + 64 * i + lane)));
            }
        } else if (u0 + lane < r.count) {
            plane_embed_unit<K, C>(s, r, u0 + lane, plane);
        }
    }
}

// Extract unit u from its C vectors v (fast units).
template <int K, int C>
__device__ __forceinline__ void plane_extract_vec_out(const Span &s, const u32x4 *v, uint64_t u, uint32_t plane) {
    const uintptr_t out_base = (uintptr_t)s.out - s.hdr_len;
    uint32_t w[Chunk<K>::NW];
    extract_vec<K>(plane_gather_any<K, C>(v, plane), w);
    uint8_t *p = reinterpret_cast<uint8_t *>(out_base + 2 * K * u);
    if (s.words) {
        store_chunk_words<K>(p, w);
    } else {
#pragma unroll
        for (int i = 0; i < 2 * K; ++i) p[i] = (uint8_t)(w[i >> 2] >> (24 - 8 * (i & 3)));
    }
}

template <int K, int C>
__device__ __forceinline__ void plane_group_extract(const Span &s, const u32x4 *stage, uint64_t u, uint32_t lane,
                                                    uint32_t plane) {
    u32x4 v[C];
#pragma unroll
    for (int i = 0; i < C; ++i) v[i] = stage[C * lane + i];
    plane_extract_vec_out<K, C>(s, v, u, plane);
}

template <int K, int C>
__device__ __forceinline__ void plane_extract_unit(const Span &s, const Ranges &r, uint64_t u, uint32_t plane) {
    if (u >= r.fast_begin && u < r.fast_end) {
        u32x4 v[C];
#pragma unroll
        for (int i = 0; i < C; ++i) v[i] = load16<true>(s.src + 16 * (C * u + i));
        plane_extract_vec_out<K, C>(s, v, u, plane);
    } else {
        const uint64_t end_byte = ceil_div(s.bits, 8);
        const uint64_t i0 = 2 * K * u;
        for (uint64_t i = i0; i < i0 + 2 * K && i < end_byte; ++i)
            if (i >= s.hdr_len) s.out[i - s.hdr_len] = (uint8_t)plane_stream_byte(s, i, C, plane);
    }
}

// Extract over the plane view: header decode per wave (lane j < 32 reads
// stream bit j), status through block 0, then 2K message bytes per lane.
template <int K, int C>
__global__ void __launch_bounds__(256)
    lsb_plane_extract_vec_kernel(Span s, uint32_t plane, uint64_t out_cap, uint32_t *len_out, int32_t *status_out) {
    __shared__ u32x4 stage_all[4][64 * C];
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t len = 0;
    int status = LSB_E_HEADER;
    if ((uint64_t)K * s.n >= 32) {
        uint32_t bit = 0;
        if (lane < 32) bit = (s.src[plane_byte(lane / K, C, plane)] >> (K - 1 - lane % K)) & 1u;
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
    u32x4 *stage = stage_all[threadIdx.x >> 6];
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t groups = ceil_div(r.count, 64);
    for (uint64_t g = wave; g < groups; g += n_waves) {
        const uint64_t u0 = 64 * g;
        if (plane_group_class(r, u0) == PLANE_FAST) {
            plane_group_load<C>(s.src + 16 * C * u0, stage, lane);
            __builtin_amdgcn_wave_barrier();
            plane_group_extract<K, C>(s, stage, u0 + lane, lane, plane);
            __builtin_amdgcn_wave_barrier();
        } else if (u0 + lane < r.count) {
            plane_extract_unit<K, C>(s, r, u0 + lane, plane);
        }
    }
}

}  // namespace lsb
