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

}  // namespace lsb
