// lsb_verify.hip -- one-launch check that a stego buffer is exactly the
// embedding of a message into a cover (arXiv:0912.0947, Section VI step 7
// recomputed; by the round-trip property, Section VII step 6 then returns
// the message).  Reads cover, stego and stream once (2n + |S| bytes) and
// counts the stego bytes that differ from the recomputed embedding; zero
// means verified.  Serving code can run it after an embed without copying
// anything back but one counter.
#include <hip/hip_ext.h>

#include "lsb_host.hpp"

namespace lsb {

// Expected stego byte t (the value an embed writes there).
__device__ __forceinline__ uint32_t verify_expected(const Span &s, uint64_t t) {
    const uint32_t k = (uint32_t)s.k;
    const uint64_t first = (uint64_t)k * (s.t0 + t);
    const uint32_t c = s.src[t];
    if (first >= s.bits) return c;
    const uint64_t left = s.bits - first;
    const uint32_t nb = left < k ? (uint32_t)left : k;
    const uint64_t byte = first >> 3;
    const uint32_t bit = (uint32_t)(first & 7);
    uint32_t pair = stream_byte(s, byte) << 8;
    if (bit + nb > 8) pair |= stream_byte(s, byte + 1);
    const uint32_t v = (pair >> (16 - bit - nb)) & ((1u << nb) - 1u);
    const uint32_t shift = k - nb;
    const uint32_t mask = ((1u << nb) - 1u) << shift;
    return (c & ~mask) | (v << shift);
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

// s.src = cover, s.dst = stego (read only here).
template <int K>
__global__ void __launch_bounds__(256) lsb_verify_kernel(Span s, unsigned long long *mismatches) {
    const Ranges r = embed_ranges<K>(s);  // inplace = 0: every vector is visited
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uintptr_t body_base = (uintptr_t)s.body - s.hdr_len;
    uint32_t bad = 0;
    for (uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; u < r.count; u += stride) {
        if (u >= r.fast_begin && u < r.fast_end) {
            uint32_t w[Chunk<K>::NW];
            const uint8_t *p = reinterpret_cast<const uint8_t *>(body_base + 2 * K * u);
            if (s.words) load_chunk_words<K>(p, w);
            else load_chunk_bytes<K>(p, 0, w);
            bad += bytes_differ(embed_vec<K>(load16<true>(s.src + 16 * u), w), load16<true>(s.dst + 16 * u));
        } else if (u >= r.copy_begin && u < r.copy_end) {
            bad += bytes_differ(load16<true>(s.src + 16 * u), load16<true>(s.dst + 16 * u));
        } else {
            const uint64_t t_end = 16 * u + 16 < s.n ? 16 * u + 16 : s.n;
            for (uint64_t t = 16 * u; t < t_end; ++t) bad += verify_expected(s, t) != s.dst[t];
        }
    }
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
    __shared__ uint32_t part[4];
    if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t sum = part[0] + part[1] + part[2] + part[3];
        if (sum) atomicAdd(mismatches, (unsigned long long)sum);
    }
}

// Per-byte form for misaligned buffers.
__global__ void __launch_bounds__(256) lsb_verify_bytes_kernel(Span s, unsigned long long *mismatches) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < s.n; t += stride)
        bad += verify_expected(s, t) != s.dst[t];
    for (int off = 32; off > 0; off >>= 1) bad += __shfl_xor(bad, off);
    if ((threadIdx.x & 63u) == 0 && bad) atomicAdd(mismatches, (unsigned long long)bad);
}

__global__ void lsb_verify_zero_kernel(unsigned long long *p) { *p = 0; }

typedef void (*VerifyFn)(Span, unsigned long long *);
static VerifyFn verify_fn(int k) {
    switch (k) {
        case 1: return lsb_verify_kernel<1>;
        case 2: return lsb_verify_kernel<2>;
        case 3: return lsb_verify_kernel<3>;
        case 4: return lsb_verify_kernel<4>;
        case 5: return lsb_verify_kernel<5>;
        case 6: return lsb_verify_kernel<6>;
        case 7: return lsb_verify_kernel<7>;
        default: return lsb_verify_kernel<8>;
    }
}

}  // namespace lsb

using namespace lsb;

extern "C" int lsb_verify(const uint8_t *cover, const uint8_t *stego, uint64_t n, const uint8_t *msg, uint32_t len,
                          int k, uint64_t *mismatches_dev, void *stream) {
    const TimedCall timed_call;
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_verify: k=%d outside 1..8", k);
    const int64_t cap = lsb_capacity(n, k);
    if (cap < 0) return (int)cap;
    if ((uint64_t)len > (uint64_t)cap)
        return fail(LSB_E_CAPACITY, "lsb_verify: message of %u bytes exceeds capacity %lld", len, (long long)cap);
    if (!cover || !stego || !mismatches_dev) return fail(LSB_E_ARG, "lsb_verify: null pointer");
    if (len && !msg) return fail(LSB_E_ARG, "lsb_verify: null msg");
    if (overlaps(mismatches_dev, 8, cover, n) || overlaps(mismatches_dev, 8, stego, n))
        return fail(LSB_E_ARG, "lsb_verify: counter overlaps a buffer");
    Span s{};
    s.src = cover;
    s.dst = const_cast<uint8_t *>(stego);  // read only
    s.body = msg;
    s.n = n;
    s.bits = 8 * (4 + (uint64_t)len);
    s.hdr = len;
    s.hdr_len = 4;
    s.k = k;
    s.inplace = 0;
    s.words = (((uintptr_t)msg - 4) & 3u) == 0;
    hipStream_t st = (hipStream_t)stream;
    unsigned long long *cnt = (unsigned long long *)mismatches_dev;
    hipLaunchKernelGGL(lsb_verify_zero_kernel, dim3(1), dim3(1), 0, st, cnt);
    const bool vec = (((uintptr_t)cover | (uintptr_t)stego) & 15u) == 0;
    const uint64_t items = vec ? ceil_div(n, 16) : n;
    uint64_t blocks = ceil_div(items ? items : 1, 256);
    const uint64_t capb = (uint64_t)device_cus() * 8;
    if (blocks > capb) blocks = capb;
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    if (vec)
        hipExtLaunchKernelGGL(verify_fn(k), dim3((unsigned)blocks), dim3(256), 0, st, e0, e1, 0, s, cnt);
    else
        hipExtLaunchKernelGGL(lsb_verify_bytes_kernel, dim3((unsigned)blocks), dim3(256), 0, st, e0, e1, 0, s, cnt);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "verify kernel launch");
}
