// lsb_paper.hip -- the paper's own layout on gfx950 (arXiv:0912.0947,
// Section VI steps 2-7 and Section VII steps 2-6): 2 bits per byte in one
// colour plane of an h x w x c image, the data split greedily over the rows
// (each row takes L = min(remaining, w/4) bytes, Section VI step 5), and bit
// pair i of data byte j in plane pixel L*i + j of its row.
//
// The paper runs this as 4 blocks of at most 32 threads per row, one MEX call
// per row.  Here one launch covers the whole image: the embed kernel streams
// every cover byte once (16 bytes per lane, copy plus in-plane update) and
// the extract kernel gives each data byte one lane that gathers its four
// pixels, so each output byte has a single writer (the paper's four blocks
// OR into the same byte).
#include <hip/hip_ext.h>

#include "lsb_host.hpp"
#include "lsb_paper_device.hpp"

namespace lsb {

// One block per row; dynamic LDS holds the row's data chunk.  C > 0 fixes
// the channel count at compile time (1, 3, 4), 0 reads it from the span.
template <int C>
__global__ void __launch_bounds__(256) lsb_paper_embed_rows_kernel(PaperSpan p) {
    extern __shared__ __attribute__((aligned(16))) uint8_t paper_chunk[];
    const PaperRow r = paper_row(p, blockIdx.x);
    if (r.L == 0) {
        if (!p.inplace) paper_row_copy(p, r, threadIdx.x, blockDim.x);
        return;
    }
    paper_row_stage(p, r, paper_chunk + kPaperGuard, threadIdx.x, blockDim.x);
    __syncthreads();
    if constexpr (C == 1 || C == 3 || C == 4) {
        if (r.L >= PaperWindow<C>::len) {
            paper_row_update<C, true>(p, r, paper_chunk, threadIdx.x, blockDim.x);
            return;
        }
    }
    paper_row_update<C, false>(p, r, paper_chunk, threadIdx.x, blockDim.x);
}

}  // namespace lsb

using namespace lsb;

// Largest data chunk per row staged in LDS by the row kernel.
static constexpr uint64_t kPaperRowChunkMax = 60 * 1024;
static_assert(paper_row_lds_bytes(kPaperRowChunkMax) <= 64 * 1024, "row kernel LDS within 64 KiB");

static int paper_check(uint32_t h, uint32_t w, uint32_t c, uint32_t plane, uint64_t len, const char *who) {
    if (c == 0 || plane >= c) return fail(LSB_E_ARG, "%s: plane %u outside 0..%u", who, plane, c ? c - 1 : 0);
    if ((uint64_t)h * w > (1ull << 48) / c) return fail(LSB_E_ARG, "%s: h*w*c above 2^48 bytes", who);
    const uint64_t cap = (uint64_t)h * (w / 4);
    if (len > cap)
        return fail(LSB_E_CAPACITY, "%s: %llu data bytes exceed the capacity h*floor(w/4) = %llu", who,
                    (unsigned long long)len, (unsigned long long)cap);
    return LSB_OK;
}

extern "C" {

int64_t lsb_paper_capacity(uint32_t h, uint32_t w) { return (int64_t)h * (w / 4); }

int lsb_paper_embed(const uint8_t *cover, uint8_t *stego, uint32_t h, uint32_t w, uint32_t c, uint32_t plane,
                    const uint8_t *data, uint64_t len, void *stream) {
    const TimedCall timed_call;
    int rc = paper_check(h, w, c, plane, len, "lsb_paper_embed");
    if (rc) return rc;
    const uint64_t n = (uint64_t)h * w * c;
    if (n == 0) return LSB_OK;
    if (!cover || !stego) return fail(LSB_E_ARG, "lsb_paper_embed: null cover/stego");
    if (len && !data) return fail(LSB_E_ARG, "lsb_paper_embed: null data");
    if (cover != stego && overlaps(cover, n, stego, n))
        return fail(LSB_E_ARG, "lsb_paper_embed: cover and stego overlap (only stego == cover is allowed)");
    if (overlaps(data, len, stego, n)) return fail(LSB_E_ARG, "lsb_paper_embed: data overlaps stego");
    PaperSpan p{};
    p.src = cover;
    p.dst = stego;
    p.data = data;
    p.n = n;
    p.len = len;
    p.rowbytes = (uint64_t)w * c;
    p.w = w;
    p.c = c;
    p.plane = plane;
    p.q = w / 4;
    p.inplace = cover == stego;
    if (p.rowbytes >= (1ull << 31)) return fail(LSB_E_ARG, "lsb_paper_embed: rows of 2^31 bytes or more");
    const bool aligned = (((uintptr_t)cover | (uintptr_t)stego) & 15u) == 0;
    if (aligned && p.rowbytes % 16 == 0 && p.q + 4 <= kPaperRowChunkMax && h < (1u << 31)) {
        // rows past the last data-carrying one: copied out-of-place, untouched in-place
        const uint64_t rows_with_data = p.q ? ceil_div(len, p.q) : 0;
        const uint64_t rows = p.inplace ? rows_with_data : h;
        if (rows == 0) return LSB_OK;
        const size_t lds = (size_t)paper_row_lds_bytes(p.q);
        hipEvent_t e0, e1;
        take_launch_events(&e0, &e1);
        void (*fn)(PaperSpan) = c == 1 ? lsb_paper_embed_rows_kernel<1>
                                : c == 3 ? lsb_paper_embed_rows_kernel<3>
                                : c == 4 ? lsb_paper_embed_rows_kernel<4>
                                         : lsb_paper_embed_rows_kernel<0>;
        hipExtLaunchKernelGGL(fn, dim3((unsigned)rows), dim3(256), lds, (hipStream_t)stream, e0, e1, 0, p);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? LSB_OK : hip_fail(e, "paper row embed kernel launch");
    }
    const bool vec = aligned && p.rowbytes >= 16;
    const uint64_t items = vec ? ceil_div(n, 16) : n;
    uint64_t blocks = ceil_div(items, 256);
    const uint64_t cap = (uint64_t)device_cus() * 16;
    if (blocks > cap) blocks = cap;
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    if (vec)
        hipExtLaunchKernelGGL(lsb_paper_embed_kernel<true>, dim3((unsigned)blocks), dim3(256), 0,
                              (hipStream_t)stream, e0, e1, 0, p);
    else
        hipExtLaunchKernelGGL(lsb_paper_embed_kernel<false>, dim3((unsigned)blocks), dim3(256), 0,
                              (hipStream_t)stream, e0, e1, 0, p);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "paper embed kernel launch");
}

int lsb_paper_extract(const uint8_t *stego, uint32_t h, uint32_t w, uint32_t c, uint32_t plane, uint8_t *data_out,
                      uint64_t len, void *stream) {
    const TimedCall timed_call;
    int rc = paper_check(h, w, c, plane, len, "lsb_paper_extract");
    if (rc) return rc;
    if (len == 0) return LSB_OK;
    const uint64_t n = (uint64_t)h * w * c;
    if (!stego || !data_out) return fail(LSB_E_ARG, "lsb_paper_extract: null stego/data_out");
    if (overlaps(data_out, len, stego, n)) return fail(LSB_E_ARG, "lsb_paper_extract: data_out overlaps stego");
    PaperSpan p{};
    p.src = stego;
    p.out = data_out;
    p.n = n;
    p.len = len;
    p.rowbytes = (uint64_t)w * c;
    p.w = w;
    p.c = c;
    p.plane = plane;
    p.q = w / 4;
    uint64_t blocks = ceil_div(len, 256);
    const uint64_t cap = (uint64_t)device_cus() * 16;
    if (blocks > cap) blocks = cap;
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    hipExtLaunchKernelGGL(lsb_paper_extract_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, e0,
                          e1, 0, p);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "paper extract kernel launch");
}

}  // extern "C"
