// lsb_plane.hip -- one colour plane with the general method, and the squared
// error behind the paper's PSNR figures (arXiv:0912.0947).
//
// Section VI step 2 / Section VII step 2 separate one plane of the image
// before embedding.  Here the fields are the bytes of plane `plane` of an
// HWC image (byte p*c + plane for pixel p), in raster order; the stream, bit
// order, header and partial last field are those of lsb_embed.  Out of
// place, a vector copy kernel first copies the cover, then a strided kernel
// rewrites the plane bytes that carry stream bits.
//
// Section VIII reports PSNR = 10*log10(255^2 / MSE).  lsb_sse sums the
// squared byte differences of two buffers on the device (16 bytes per lane,
// wave reduction, one 64-bit atomic per wave).
#include <hip/hip_ext.h>

#include "lsb_host.hpp"

#include "lsb_plane_device.hpp"

namespace lsb {

__global__ void lsb_zero_u64_kernel(uint64_t *p) { *p = 0; }

__device__ __forceinline__ uint32_t sq_diff4(uint32_t a, uint32_t b) {
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int d = (int)((a >> (8 * j)) & 0xFFu) - (int)((b >> (8 * j)) & 0xFFu);
        sum += (uint32_t)(d * d);
    }
    return sum;
}

// Sum of squared byte differences; one 64-bit atomic per wave.
__global__ void __launch_bounds__(256) lsb_sse_kernel(const uint8_t *a, const uint8_t *b, uint64_t n, int vec,
                                                     unsigned long long *out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc = 0;
    uint64_t tail = 0;
    if (vec) {
        const uint64_t nv = n / 16;
        for (uint64_t u = gid; u < nv; u += stride) {
            const u32x4 x = load16<true>(a + 16 * u), y = load16<true>(b + 16 * u);
            acc += sq_diff4(x[0], y[0]) + sq_diff4(x[1], y[1]) + sq_diff4(x[2], y[2]) + sq_diff4(x[3], y[3]);
        }
        tail = 16 * nv;
    }
    for (uint64_t t = tail + gid; t < n; t += stride) {
        const int d = (int)a[t] - (int)b[t];
        acc += (uint64_t)(d * d);
    }
    // wave reduction of the 64-bit partial sums, then across the block's
    // waves in LDS, then one atomic per block
    uint32_t lo = (uint32_t)acc, hi = (uint32_t)(acc >> 32);
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t olo = __shfl_xor(lo, off), ohi = __shfl_xor(hi, off);
        const uint64_t sum = ((uint64_t)hi << 32 | lo) + ((uint64_t)ohi << 32 | olo);
        lo = (uint32_t)sum;
        hi = (uint32_t)(sum >> 32);
    }
    __shared__ unsigned long long part[4];  // 256 threads = 4 waves
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = (unsigned long long)hi << 32 | lo;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

typedef void (*PlaneEmbedFn)(Span, uint32_t);
typedef void (*PlaneExtractFn)(Span, uint32_t, uint64_t, uint32_t *, int32_t *);

template <int K>
struct PlaneTable {
    static constexpr PlaneEmbedFn embed[3] = {lsb_plane_embed_vec_kernel<K, 2>, lsb_plane_embed_vec_kernel<K, 3>,
                                              lsb_plane_embed_vec_kernel<K, 4>};
    static constexpr PlaneExtractFn extract[3] = {lsb_plane_extract_vec_kernel<K, 2>,
                                                  lsb_plane_extract_vec_kernel<K, 3>,
                                                  lsb_plane_extract_vec_kernel<K, 4>};
};

static PlaneEmbedFn plane_embed_fn(int k, uint32_t c) {
    const int ci = (int)c - 2;
    switch (k) {
        case 1: return PlaneTable<1>::embed[ci];
        case 2: return PlaneTable<2>::embed[ci];
        case 3: return PlaneTable<3>::embed[ci];
        case 4: return PlaneTable<4>::embed[ci];
        case 5: return PlaneTable<5>::embed[ci];
        case 6: return PlaneTable<6>::embed[ci];
        case 7: return PlaneTable<7>::embed[ci];
        default: return PlaneTable<8>::embed[ci];
    }
}

static PlaneExtractFn plane_extract_fn(int k, uint32_t c) {
    const int ci = (int)c - 2;
    switch (k) {
        case 1: return PlaneTable<1>::extract[ci];
        case 2: return PlaneTable<2>::extract[ci];
        case 3: return PlaneTable<3>::extract[ci];
        case 4: return PlaneTable<4>::extract[ci];
        case 5: return PlaneTable<5>::extract[ci];
        case 6: return PlaneTable<6>::extract[ci];
        case 7: return PlaneTable<7>::extract[ci];
        default: return PlaneTable<8>::extract[ci];
    }
}

// Grid of the plane kernels: a thread per item.  They are grid-stride
// loops, and a looping wave's wait for its next loads also waits for its
// previous stores; capped at 16 blocks per CU, the plane embed of an
// 8192x8192x3 image took 70-72 us against 66-67 us uncapped (extract
// 37.8-38.2 against 37.3-37.6 us).
static unsigned grid_cap(uint64_t items) {
    const uint64_t blocks = ceil_div(items ? items : 1, 256);
    return (unsigned)(blocks < (uint64_t)INT32_MAX ? blocks : (uint64_t)INT32_MAX);
}

}  // namespace lsb

using namespace lsb;

extern "C" {

int lsb_embed_plane(const uint8_t *cover, uint8_t *stego, uint64_t pixels, uint32_t c, uint32_t plane,
                    const uint8_t *msg, uint32_t len, int k, void *stream) {
    const TimedCall timed_call;
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_embed_plane: k=%d outside 1..8", k);
    if (c == 0 || plane >= c) return fail(LSB_E_ARG, "lsb_embed_plane: plane %u outside 0..%u", plane, c ? c - 1 : 0);
    if (pixels > (1ull << 48) || c > 65536) return fail(LSB_E_ARG, "lsb_embed_plane: pixels or channels out of range");
    const int64_t cap = lsb_capacity(pixels, k);
    if (cap < 0) return (int)cap;
    if ((uint64_t)len > (uint64_t)cap)
        return fail(LSB_E_CAPACITY, "lsb_embed_plane: message of %u bytes exceeds capacity %lld", len, (long long)cap);
    const uint64_t n = pixels * c;
    if (!cover || !stego) return fail(LSB_E_ARG, "lsb_embed_plane: null cover/stego");
    if (len && !msg) return fail(LSB_E_ARG, "lsb_embed_plane: null msg");
    if (cover != stego && overlaps(cover, n, stego, n))
        return fail(LSB_E_ARG, "lsb_embed_plane: cover and stego overlap (only stego == cover is allowed)");
    if (overlaps(msg, len, stego, n)) return fail(LSB_E_ARG, "lsb_embed_plane: msg overlaps stego");
    hipStream_t st = (hipStream_t)stream;
    const bool aligned = (((uintptr_t)cover | (uintptr_t)stego) & 15u) == 0;
    if (c == 1) return lsb_embed(cover, stego, pixels, msg, len, k, stream);  // the plane is the image
    if (aligned && c <= 4) {
        // one pass: each lane moves 16 pixels (c vectors) and rewrites their plane bytes
        Span s{};
        s.src = cover;
        s.dst = stego;
        s.body = msg;
        s.n = pixels;
        s.bits = 8 * (4 + (uint64_t)len);
        s.hdr = len;
        s.hdr_len = 4;
        s.k = k;
        s.inplace = cover == stego;
        s.words = (((uintptr_t)msg - 4) & 3u) == 0;
        const Ranges r = embed_ranges(s);
        if (!r.count) return LSB_OK;
        hipEvent_t e0, e1;
        take_launch_events(&e0, &e1);
        hipExtLaunchKernelGGL(plane_embed_fn(k, c), dim3(grid_cap(r.count)), dim3(256), 0, st, e0, e1, 0, s, plane);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? LSB_OK : hip_fail(e, "plane embed kernel launch");
    }
    // other channel counts or misaligned buffers: copy, then rewrite the plane bytes
    if (cover != stego) {
        const int vec = aligned;
        hipLaunchKernelGGL(lsb_copy_kernel, dim3(grid_cap(vec ? n / 16 : n)), dim3(256), 0, st, cover, stego, n, vec);
    }
    Span s{};
    s.src = stego;  // after the copy the plane bytes are read back from stego
    s.dst = stego;
    s.body = msg;
    s.n = pixels;
    s.bits = 8 * (4 + (uint64_t)len);
    s.hdr = len;
    s.hdr_len = 4;
    s.k = k;
    const uint64_t fields = ceil_div(s.bits, (uint64_t)k);
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    hipExtLaunchKernelGGL(lsb_plane_embed_kernel, dim3(grid_cap(fields)), dim3(256), 0, st, e0, e1, 0, s, fields, c,
                          plane);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "plane embed kernel launch");
}

int lsb_extract_plane(const uint8_t *stego, uint64_t pixels, uint32_t c, uint32_t plane, int k, uint8_t *msg_out,
                      uint64_t out_cap, uint32_t *len_out_dev, int32_t *status_out_dev, void *stream) {
    const TimedCall timed_call;
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_extract_plane: k=%d outside 1..8", k);
    if (c == 0 || plane >= c) return fail(LSB_E_ARG, "lsb_extract_plane: plane %u outside 0..%u", plane, c ? c - 1 : 0);
    if (!len_out_dev || !status_out_dev) return fail(LSB_E_ARG, "lsb_extract_plane: null len/status pointer");
    if (pixels && !stego) return fail(LSB_E_ARG, "lsb_extract_plane: null stego");
    if (out_cap && !msg_out) return fail(LSB_E_ARG, "lsb_extract_plane: null msg_out with out_cap > 0");
    if (pixels > (1ull << 48) || c > 65536)
        return fail(LSB_E_ARG, "lsb_extract_plane: pixels or channels out of range");
    const uint64_t n = pixels * c;
    const uint64_t room = room_bytes(pixels, k);
    const uint64_t cap = room >= 4 ? room - 4 : 0;
    const uint64_t max_len = out_cap < cap ? out_cap : cap;
    if (overlaps(msg_out, max_len, stego, n)) return fail(LSB_E_ARG, "lsb_extract_plane: msg_out overlaps stego");
    if (overlaps(len_out_dev, 4, stego, n) || overlaps(status_out_dev, 4, stego, n) ||
        overlaps(len_out_dev, 4, msg_out, max_len) || overlaps(status_out_dev, 4, msg_out, max_len))
        return fail(LSB_E_ARG, "lsb_extract_plane: len/status overlap a data buffer");
    if (c == 1) return lsb_extract(stego, pixels, k, msg_out, out_cap, len_out_dev, status_out_dev, stream);
    Span s{};
    s.src = stego;
    s.out = msg_out;
    s.n = pixels;
    s.hdr_len = 4;
    s.k = k;
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    if (c <= 4 && ((uintptr_t)stego & 15u) == 0) {
        s.words = (((uintptr_t)msg_out - 4) & 3u) == 0;
        uint64_t vectors = 0;  // bound on the vectors a decodable stream can need
        if ((uint64_t)k * pixels >= 32) {
            const uint64_t v_stream = ceil_div(4 + max_len, 2 * (uint64_t)k);
            const uint64_t v_buf = ceil_div(pixels, 16);
            vectors = v_stream < v_buf ? v_stream : v_buf;
        }
        hipExtLaunchKernelGGL(plane_extract_fn(k, c), dim3(grid_cap(vectors)), dim3(256), 0, (hipStream_t)stream, e0,
                              e1, 0, s, plane, out_cap, len_out_dev, status_out_dev);
    } else {
        hipExtLaunchKernelGGL(lsb_plane_extract_kernel, dim3(grid_cap(max_len)), dim3(256), 0, (hipStream_t)stream,
                              e0, e1, 0, s, c, plane, out_cap, len_out_dev, status_out_dev);
    }
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "plane extract kernel launch");
}

int lsb_sse(const uint8_t *a, const uint8_t *b, uint64_t n, uint64_t *sse_dev, void *stream) {
    const TimedCall timed_call;
    if (!sse_dev) return fail(LSB_E_ARG, "lsb_sse: null result pointer");
    if (n && (!a || !b)) return fail(LSB_E_ARG, "lsb_sse: null buffer");
    if (overlaps(sse_dev, 8, a, n) || overlaps(sse_dev, 8, b, n))
        return fail(LSB_E_ARG, "lsb_sse: result overlaps an input");
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(lsb_zero_u64_kernel, dim3(1), dim3(1), 0, st, sse_dev);
    const int vec = (((uintptr_t)a | (uintptr_t)b) & 15u) == 0;
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    uint64_t blocks = ceil_div((vec ? n / 16 : n) + 1, 256);
    const uint64_t cap = (uint64_t)device_cus() * 4;  // few atomics on the one result word
    if (blocks > cap) blocks = cap;
    hipExtLaunchKernelGGL(lsb_sse_kernel, dim3((unsigned)blocks), dim3(256), 0, st, e0, e1, 0, a, b, n, vec,
                          (unsigned long long *)sse_dev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "sse kernel launch");
}

}  // extern "C"
