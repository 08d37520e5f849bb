// lsb_paper_device.hpp -- device code of the paper's own layout
// (arXiv:0912.0947, Section VI steps 2-7, Section VII steps 2-6): 2 bits per
// byte in one colour plane, greedy per-row data chunks, bit pair i of data
// byte j in plane pixel L*i + j.  Included by lsb_paper.hip.
#pragma once

#include "lsb_device.hpp"

namespace lsb {

struct PaperSpan {
    const uint8_t *src;
    uint8_t *dst;
    const uint8_t *data;
    uint8_t *out;
    uint64_t n;         // h * w * c
    uint64_t len;       // data bytes
    uint64_t rowbytes;  // w * c
    uint32_t w, c, plane, q;  // q = w / 4 data bytes per full row
    int inplace;
};

// New value of the plane byte at row y, pixel x (Section VI step 7: clear
// the low two bits, OR in bits 2i+1..2i of data byte j, with x = L*i + j).
__device__ __forceinline__ uint32_t paper_pixel(const PaperSpan &p, uint64_t y, uint32_t x, uint32_t byte) {
    const uint64_t first = y * p.q;  // first data byte of row y
    if (first >= p.len) return byte;
    const uint64_t left = p.len - first;
    const uint32_t L = left < p.q ? (uint32_t)left : p.q;
    if (x >= 4 * L) return byte;
    const uint32_t i = (x >= L) + (x >= 2 * L) + (x >= 3 * L);
    const uint32_t j = x - i * L;
    const uint32_t d = p.data[first + j];
    return (byte & 0xFCu) | ((d >> (2 * i)) & 3u);
}

// Bytes [t, t_end) of one row-ordered run, with (y, x, ch) the position of t.
// Walks positions by increments; applies paper_pixel to plane bytes.
__device__ __forceinline__ void paper_walk_bytes(const PaperSpan &p, uint64_t t, uint64_t t_end, uint8_t *bytes) {
    uint64_t y = t / p.rowbytes;
    const uint64_t rem = t - y * p.rowbytes;
    uint32_t x = (uint32_t)(rem / p.c);
    uint32_t ch = (uint32_t)(rem - (uint64_t)x * p.c);
    for (uint64_t k = 0; t + k < t_end; ++k) {
        if (ch == p.plane) bytes[k] = (uint8_t)paper_pixel(p, y, x, bytes[k]);
        if (++ch == p.c) {
            ch = 0;
            if (++x == p.w) {
                x = 0;
                ++y;
            }
        }
    }
}

// One 16-byte vector starting at cover byte t, for rows of at least 16
// bytes (so the vector touches at most two rows).  Positions advance by
// selects, all data-byte gathers of the vector are issued together, then the
// plane bytes of carrying rows are updated (Section VI step 7).
__device__ __forceinline__ u32x4 paper_vec16(const PaperSpan &p, uint64_t t, u32x4 v) {
    const uint64_t y = t / p.rowbytes;
    const uint32_t rem = (uint32_t)(t - y * p.rowbytes);
    uint32_t x = rem / p.c;
    uint32_t ch = rem - x * p.c;
    // data chunk of row y and of row y + 1
    uint64_t first[2];
    uint32_t L[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        first[r] = (y + r) * p.q;
        const uint64_t left = first[r] < p.len ? p.len - first[r] : 0;
        L[r] = left < p.q ? (uint32_t)left : p.q;
    }
    uint32_t row = 0;
    bool need[16];
    uint32_t pair[16];
    uint64_t at[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const uint32_t Lr = row ? L[1] : L[0];
        need[k] = ch == p.plane && x < 4 * Lr;
        const uint32_t i = (x >= Lr) + (x >= 2 * Lr) + (x >= 3 * Lr);
        pair[k] = 2 * i;
        at[k] = (row ? first[1] : first[0]) + (x - i * Lr);
        // advance to the next byte: channel, then pixel, then row
        const bool ch_wrap = ch + 1 == p.c;
        const bool x_wrap = ch_wrap && x + 1 == p.w;
        ch = ch_wrap ? 0 : ch + 1;
        x = x_wrap ? 0 : (ch_wrap ? x + 1 : x);
        row = x_wrap ? 1 : row;
    }
    uint32_t d[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) d[k] = need[k] ? p.data[at[k]] : 0u;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (need[k]) {
            const int sh = 8 * (k & 3);
            const uint32_t val = (d[k] >> pair[k]) & 3u;
            v[k >> 2] = (v[k >> 2] & ~(3u << sh)) | (val << sh);
        }
    }
    return v;
}

// Embed: every cover byte is read once and written once (16 bytes per lane
// when both pointers are 16-byte aligned and rows hold at least 16 bytes,
// else one byte per lane).
template <bool VEC>
__global__ void __launch_bounds__(256) lsb_paper_embed_kernel(PaperSpan p) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t rows_with_data = p.q ? ceil_div(p.len, p.q) : 0;
    const uint64_t data_end = rows_with_data * p.rowbytes;  // bytes past it never change
    if constexpr (VEC) {
        const uint64_t vecs = ceil_div(p.n, 16);
        for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < vecs; u += stride) {
            const uint64_t t = 16 * u;
            if (t + 16 <= p.n) {
                u32x4 v = load16<true>(p.src + t);
                if (t >= data_end) {  // no data in this vector's rows
                    if (!p.inplace) store16<true>(p.dst + t, v);
                    continue;
                }
                store16<true>(p.dst + t, paper_vec16(p, t, v));
            } else {
                uint8_t b[16];
                const uint64_t m = p.n - t;
                for (uint64_t k = 0; k < m; ++k) b[k] = p.src[t + k];
                paper_walk_bytes(p, t, p.n, b);
                for (uint64_t k = 0; k < m; ++k) p.dst[t + k] = b[k];
            }
        }
    } else {
        for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < p.n; t += stride) {
            uint8_t b = p.src[t];
            if (t < data_end) paper_walk_bytes(p, t, t + 1, &b);
            if (!p.inplace || t < data_end) p.dst[t] = b;
        }
    }
}

// -------------------------------------------------------------------------
// Row-per-block embed.  Block y handles image row y: it stages the row's data
// chunk (data bytes [y*q, y*q + L)) in LDS with dword loads, then each lane
// streams 16-byte vectors of the row and rewrites their plane bytes from LDS
// (Section VI steps 5-7).  No 64-bit division and no scattered global gathers.
// Used when the row length is a multiple of 16, both image pointers are
// 16-byte aligned and the chunk fits the block's LDS.

struct PaperRow {
    const uint8_t *src;
    uint8_t *dst;
    uint64_t first;  // first data byte of the row
    uint32_t L;      // data bytes of the row (0: the row carries none)
    uint32_t h0;     // (data + first) % 4: LDS offset of data byte `first`
};

__device__ __forceinline__ PaperRow paper_row(const PaperSpan &p, uint64_t y) {
    PaperRow r;
    r.src = p.src + y * p.rowbytes;
    r.dst = p.dst + y * p.rowbytes;
    r.first = y * p.q;
    const uint64_t left = r.first < p.len ? p.len - r.first : 0;
    r.L = left < p.q ? (uint32_t)left : p.q;
    r.h0 = (uint32_t)((uintptr_t)(p.data + r.first) & 3u);
    return r;
}

// Copy a row that carries no data (out-of-place only).
__device__ __forceinline__ void paper_row_copy(const PaperSpan &p, const PaperRow &r, uint32_t tid, uint32_t nthreads) {
    const uint32_t rowvecs = (uint32_t)(p.rowbytes / 16);
    for (uint32_t u = tid; u < rowvecs; u += nthreads) store16<true>(r.dst + 16 * (uint64_t)u, load16<true>(r.src + 16 * (uint64_t)u));
}

// Stage data bytes [first, first + L) at chunk[h0 .. h0 + L): whole dwords
// of the data buffer land on aligned LDS dwords; the partial dwords at the
// two ends are copied byte by byte, so no byte outside the chunk is read.
__device__ __forceinline__ void paper_row_stage(const PaperSpan &p, const PaperRow &r, uint8_t *chunk, uint32_t tid,
                                                uint32_t nthreads) {
    const uint8_t *a = p.data + r.first;
    const uint32_t *aw = reinterpret_cast<const uint32_t *>(a - r.h0);
    const uint32_t end = r.h0 + r.L;
    const uint32_t nw = (end + 3) / 4;
    for (uint32_t w = tid; w < nw; w += nthreads) {
        const uint32_t lo = 4 * w;
        if (lo >= r.h0 && lo + 4 <= end) {
            reinterpret_cast<uint32_t *>(chunk)[w] = aw[w];
        } else {
            for (uint32_t b = lo; b < lo + 4; ++b)
                if (b >= r.h0 && b < end) chunk[b] = a[b - r.h0];
        }
    }
}

// New value of the 16 row bytes at row offset o (Section VI step 7): for a
// plane byte of pixel x < 4L, i = x / L (by three compares) and j = x - i*L;
// its low two bits become bits 2i+1..2i of data byte j (data = the staged
// chunk, data[j] = data byte first + j).  All 16 LDS reads are issued before
// any is used; bytes that take no data read data[0] and keep their value.
template <int C>
__device__ __forceinline__ u32x4 paper_row_vec(const PaperSpan &p, const uint8_t *data, uint32_t L, uint32_t o,
                                               u32x4 v) {
    const uint32_t c = C > 0 ? (uint32_t)C : p.c;
    uint32_t x = o / c;
    uint32_t ch = o - x * c;
    const uint32_t four_l = 4 * L;
    bool need[16];
    uint32_t shift[16], d[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        need[k] = ch == p.plane && x < four_l;
        const uint32_t i = (x >= L) + (x >= 2 * L) + (x >= 3 * L);
        shift[k] = 2 * i;
        d[k] = data[need[k] ? x - i * L : 0];
        const bool wrap = ch + 1 == c;
        ch = wrap ? 0 : ch + 1;
        x = wrap ? x + 1 : x;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int sh = 8 * (k & 3);
        const uint32_t nv = (v[k >> 2] & ~(3u << sh)) | (((d[k] >> shift[k]) & 3u) << sh);
        v[k >> 2] = need[k] ? nv : v[k >> 2];
    }
    return v;
}

// Window form for c = 1, 3, 4.  The plane bytes of a 16-byte vector are
// the pixels xf, xf + 1, ... (16, 5 or 6, 4 of them), so their data bytes
// are a contiguous run of the chunk, read with a few LDS dwords and a funnel
// shift.  With L >= the window length a window meets at most one quarter
// boundary: pixels before it take bit pair i of data[j0 + m], pixels after
// it bit pair i + 1 of data[m - ms] (ms = L - j0 pixels remain in quarter
// i), read as a second window starting L bytes earlier.  Pixels at or past
// 4L take no data.  LDS holds kPaperGuard readable bytes before the chunk
// and 32 after it, so both windows stay inside the allocation.
constexpr uint32_t kPaperGuard = 16;

template <int C>
struct PaperWindow {
    static constexpr uint32_t len = C == 1 ? 16 : (C == 3 ? 6 : 4);  // plane pixels read per vector
};

__device__ __forceinline__ uint32_t funnel8(uint32_t hi, uint32_t lo, uint32_t s) {
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> (8 * s));
}

// Bytes chunk[a .. a + 4*NW) as NW dwords (little-endian), a >= 0 relative
// to the 4-byte aligned chunk base.
template <int NW>
__device__ __forceinline__ void lds_window(const uint8_t *chunk, uint32_t a, uint32_t *out) {
    const uint32_t *w = reinterpret_cast<const uint32_t *>(chunk) + (a >> 2);
    const uint32_t s = a & 3u;
    uint32_t d[NW + 1];
#pragma unroll
    for (int t = 0; t <= NW; ++t) d[t] = w[t];
#pragma unroll
    for (int t = 0; t < NW; ++t) out[t] = funnel8(d[t + 1], d[t], s);
}

// Data-bit pairs and keep masks (0x03 per byte that takes data) of the
// window's pixels, packed one per byte in NW dwords.
template <int NW>
__device__ __forceinline__ void paper_pairs(const uint8_t *chunk, uint32_t h0, uint32_t L, uint32_t xf,
                                            uint32_t *pairs, uint32_t *keep) {
    const bool any = xf < 4 * L;
    const uint32_t i = (xf >= L) + (xf >= 2 * L) + (xf >= 3 * L);
    const uint32_t j0 = any ? xf - i * L : 0;
    const uint32_t ms = L - j0;  // >= 1: window pixels still in quarter i
    const bool cross = ms < 4 * NW;
    const bool next = cross && i < 3;  // pixels after the boundary take quarter i + 1
    uint32_t a[NW], b[NW];
    lds_window<NW>(chunk, kPaperGuard + h0 + j0, a);
    lds_window<NW>(chunk, kPaperGuard + h0 + j0 - (cross ? L : 0), b);
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        // bytes of dword t below ms come from window a
        const uint32_t lo = ms >= 4u * t + 4 ? 0xFFFFFFFFu : (ms <= 4u * t ? 0u : (1u << (8 * (ms - 4 * t))) - 1u);
        const uint32_t pa = (a[t] >> (2 * i)) & 0x03030303u;
        const uint32_t pb = (b[t] >> (2 * (i + 1) & 7)) & 0x03030303u;
        const uint32_t hi_ok = next ? ~lo : 0u;
        pairs[t] = any ? (pa & lo) | (pb & hi_ok) : 0u;
        keep[t] = any ? 0x03030303u & (lo | hi_ok) : 0u;
    }
}

// 128-bit value t shifted left by r bytes (r < 4), dword 0 lowest.
__device__ __forceinline__ void shl_bytes(uint32_t *t, uint32_t r) {
    const uint32_t sh = 32 - 8 * r;
#pragma unroll
    for (int d = 3; d >= 0; --d) t[d] = (uint32_t)((((uint64_t)t[d] << 32) | (d ? t[d - 1] : 0u)) >> sh);
}

// Six packed bytes (bytes 0..3 of p0, 0..1 of p1) to bytes 0, 3, 6, 9, 12,
// 15 of a 128-bit value, then shifted left by r bytes.
__device__ __forceinline__ void spread3(uint32_t p0, uint32_t p1, uint32_t r, uint32_t *t) {
    t[0] = (p0 & 0xFFu) | ((p0 & 0xFF00u) << 16);
    t[1] = p0 & 0xFF0000u;
    t[2] = (p0 >> 16) & 0xFF00u;
    t[3] = (p1 & 0xFFu) | ((p1 & 0xFF00u) << 16);
    shl_bytes(t, r);
}

template <int C>
__device__ __forceinline__ u32x4 paper_row_vec_window(const PaperSpan &p, const uint8_t *chunk, uint32_t h0,
                                                      uint32_t L, uint32_t o, u32x4 v) {
    if constexpr (C == 1) {
        uint32_t pr[4], kp[4];
        paper_pairs<4>(chunk, h0, L, o, pr, kp);
#pragma unroll
        for (int d = 0; d < 4; ++d) v[d] = (v[d] & ~kp[d]) | pr[d];
    } else if constexpr (C == 3) {
        const uint32_t ch0 = o % 3u;
        const uint32_t r = (p.plane + 3u - ch0) % 3u;  // first plane byte of the vector
        const uint32_t xf = (o + r) / 3u;
        uint32_t pr[2], kp[2], tp[4], tk[4];
        paper_pairs<2>(chunk, h0, L, xf, pr, kp);
        spread3(pr[0], pr[1], r, tp);
        spread3(kp[0], kp[1], r, tk);
#pragma unroll
        for (int d = 0; d < 4; ++d) v[d] = (v[d] & ~tk[d]) | tp[d];
    } else {
        static_assert(C == 4, "window form for c = 1, 3, 4");
        const uint32_t sh = 8 * p.plane;  // o % 4 == 0: byte `plane` of each dword
        uint32_t pr[1], kp[1];
        paper_pairs<1>(chunk, h0, L, o / 4u, pr, kp);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t pd = ((pr[0] >> (8 * d)) & 3u) << sh, kd = ((kp[0] >> (8 * d)) & 3u) << sh;
            v[d] = (v[d] & ~kd) | pd;
        }
    }
    return v;
}

// This lane's vectors of a data-carrying row: UNR loads in flight, then the
// updates and stores.  `lds` is the block's LDS area: kPaperGuard bytes,
// then the staged chunk.  WIN selects the window form (c = 1, 3, 4 and
// L >= its window length, a block-uniform choice).
template <int C, bool WIN>
__device__ __forceinline__ void paper_row_update(const PaperSpan &p, const PaperRow &r, const uint8_t *lds,
                                                 uint32_t tid, uint32_t nthreads) {
    constexpr int UNR = 4;
    const uint32_t rowvecs = (uint32_t)(p.rowbytes / 16);
    const uint8_t *data = lds + kPaperGuard + r.h0;
    for (uint32_t base = tid; base < rowvecs; base += UNR * nthreads) {
        u32x4 v[UNR];
#pragma unroll
        for (int m = 0; m < UNR; ++m) {
            const uint32_t u = base + m * nthreads;
            if (u < rowvecs) v[m] = load16<true>(r.src + 16 * (uint64_t)u);
        }
#pragma unroll
        for (int m = 0; m < UNR; ++m) {
            const uint32_t u = base + m * nthreads;
            if (u >= rowvecs) continue;
            u32x4 w;
            if constexpr (WIN) w = paper_row_vec_window<C>(p, lds, r.h0, r.L, 16 * u, v[m]);
            else w = paper_row_vec<C>(p, data, r.L, 16 * u, v[m]);
            store16<true>(r.dst + 16 * (uint64_t)u, w);
        }
    }
}

// LDS bytes of the row kernel for rows of q data bytes: guard, chunk (with
// the data pointer's offset mod 4), and the window reads' overrun.
__host__ __device__ constexpr uint64_t paper_row_lds_bytes(uint64_t q) { return kPaperGuard + (q + 3 + 32 + 15) / 16 * 16; }

// Extract: one lane per data byte d; row y = d / q holds bytes
// [y*q, y*q + L); byte j of the row is ORed together from the low two bits
// of pixels L*i + j, shifted left by 2i (Section VII step 6).
__global__ void __launch_bounds__(256) lsb_paper_extract_kernel(PaperSpan p) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t d = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; d < p.len; d += stride) {
        const uint64_t y = d / p.q;
        const uint64_t first = y * p.q;
        const uint32_t j = (uint32_t)(d - first);
        const uint64_t left = p.len - first;
        const uint32_t L = left < p.q ? (uint32_t)left : p.q;
        const uint8_t *row = p.src + y * p.rowbytes + p.plane;
        uint32_t v = 0;
#pragma unroll
        for (uint32_t i = 0; i < 4; ++i) v |= ((uint32_t)row[(uint64_t)(L * i + j) * p.c] & 3u) << (2 * i);
        p.out[d] = (uint8_t)v;
    }
}

}  // namespace lsb
