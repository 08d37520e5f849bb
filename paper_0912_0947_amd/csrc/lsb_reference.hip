// lsb_reference.hip -- reference streaming kernels: plain streams with the
// traffic mixes of the embed and extract kernels, so that their durations
// can be set against what a stream of the same bytes achieves on this device
// (a measurement aid; none of the method is computed here).
//
// Each lane moves whole 16-byte vectors in a grid-stride loop; an unrolled
// lane keeps `UNR` loads in flight, one grid stride apart.
#include <hip/hip_ext.h>

#include "lsb_host.hpp"

namespace lsb {

// KIND 0: dst[i] = src[i].
// KIND 1: dst[i] = src[i] with side[i] (16 bits) XORed into its first dword
//         (reads n + n/8 bytes, writes n: the k = 1 embed mix).
// KIND 2: out2[i] = low 16 bits of the XOR of src[i]'s four dwords (reads n,
//         writes n/8: the k = 1 extract mix).
template <int KIND>
__device__ __forceinline__ void ref_one(const u32x4 *src, u32x4 *dst, const uint16_t *side, uint16_t *out2,
                                        uint64_t i, u32x4 v, uint32_t w) {
    if constexpr (KIND == 0) {
        __builtin_nontemporal_store(v, dst + i);
    } else if constexpr (KIND == 1) {
        v[0] ^= w;
        __builtin_nontemporal_store(v, dst + i);
    } else {
        out2[i] = (uint16_t)(v[0] ^ v[1] ^ v[2] ^ v[3]);
    }
}

template <int KIND, int UNR>
__global__ void __launch_bounds__(1024)
    lsb_stream_ref_kernel(const u32x4 *src, u32x4 *dst, const uint16_t *side, uint16_t *out2, uint64_t nv) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (UNR - 1) * stride < nv; i += UNR * stride) {
        u32x4 v[UNR];
        uint32_t w[UNR];
#pragma unroll
        for (int j = 0; j < UNR; ++j) {
            v[j] = __builtin_nontemporal_load(src + i + j * stride);
            w[j] = KIND == 1 ? (uint32_t)side[i + j * stride] : 0u;
        }
#pragma unroll
        for (int j = 0; j < UNR; ++j) ref_one<KIND>(src, dst, side, out2, i + j * stride, v[j], w[j]);
    }
    for (; i < nv; i += stride) ref_one<KIND>(src, dst, side, out2, i, src[i], KIND == 1 ? (uint32_t)side[i] : 0u);
}

typedef void (*RefFn)(const u32x4 *, u32x4 *, const uint16_t *, uint16_t *, uint64_t);

template <int KIND>
static RefFn ref_fn(int unroll) {
    return unroll == 1 ? lsb_stream_ref_kernel<KIND, 1>
           : unroll == 2 ? lsb_stream_ref_kernel<KIND, 2>
                         : lsb_stream_ref_kernel<KIND, 4>;
}

}  // namespace lsb

using namespace lsb;

extern "C" int lsb_stream_reference(int kind, const uint8_t *src, uint8_t *dst, const uint8_t *side, uint64_t n,
                                    int block, int unroll, uint32_t grid, void *stream) {
    clear_error();
    if (kind < LSB_REF_COPY || kind > LSB_REF_EXTRACT_MIX)
        return fail(LSB_E_ARG, "lsb_stream_reference: kind %d unknown", kind);
    if (block != 256 && block != 512 && block != 1024)
        return fail(LSB_E_ARG, "lsb_stream_reference: block %d not 256, 512 or 1024", block);
    if (unroll != 1 && unroll != 2 && unroll != 4)
        return fail(LSB_E_ARG, "lsb_stream_reference: unroll %d not 1, 2 or 4", unroll);
    if (n % 16) return fail(LSB_E_ARG, "lsb_stream_reference: n = %llu not a multiple of 16", (unsigned long long)n);
    if (n == 0) return LSB_OK;
    if (!src || !dst || (kind == LSB_REF_EMBED_MIX && !side))
        return fail(LSB_E_ARG, "lsb_stream_reference: null pointer");
    const uint64_t nv = n / 16;
    const uint64_t dst_bytes = kind == LSB_REF_EXTRACT_MIX ? 2 * nv : n;
    if (((uintptr_t)src & 15u) || (kind != LSB_REF_EXTRACT_MIX && ((uintptr_t)dst & 15u)) || ((uintptr_t)dst & 1u) ||
        (kind == LSB_REF_EMBED_MIX && ((uintptr_t)side & 1u)))
        return fail(LSB_E_ARG, "lsb_stream_reference: misaligned pointer");
    if (overlaps(src, n, dst, dst_bytes) || (kind == LSB_REF_EMBED_MIX && overlaps(side, 2 * nv, dst, dst_bytes)))
        return fail(LSB_E_ARG, "lsb_stream_reference: output overlaps an input");
    const uint64_t full = ceil_div(nv, (uint64_t)block * unroll);
    uint64_t g = grid ? grid : full;
    if (g > full) g = full;
    if (g > 0x7FFFFFFFull) g = 0x7FFFFFFFull;
    RefFn fn = kind == LSB_REF_COPY ? ref_fn<0>(unroll) : kind == LSB_REF_EMBED_MIX ? ref_fn<1>(unroll) : ref_fn<2>(unroll);
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    hipExtLaunchKernelGGL(fn, dim3((unsigned)g), dim3(block), 0, (hipStream_t)stream, e0, e1, 0,
                          reinterpret_cast<const u32x4 *>(src), reinterpret_cast<u32x4 *>(dst),
                          reinterpret_cast<const uint16_t *>(side), reinterpret_cast<uint16_t *>(dst), nv);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "stream reference kernel launch");
}
