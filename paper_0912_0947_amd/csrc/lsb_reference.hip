// lsb_reference.hip -- reference streaming kernels: plain streams with the
// traffic mixes of the embed and extract kernels, so that their durations
// can be set against what a stream of the same bytes achieves on this device
// (a measurement aid; none of the method is computed here).
//
// At k bits per cover byte a 16-byte cover vector goes with 2k stream bytes:
// the embed mix reads them beside the vector, the extract mix writes them.
// Each lane moves whole 16-byte vectors in a grid-stride loop; an unrolled
// lane keeps `UNR` loads in flight, one grid stride apart.
#include <hip/hip_ext.h>

#include "lsb_host.hpp"

namespace lsb {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// The 2k side bytes of one vector.
template <int K> struct RefSide;
template <> struct RefSide<1> { typedef uint16_t T; };
template <> struct RefSide<2> { typedef uint32_t T; };
template <> struct RefSide<4> { typedef u32x2 T; };

// Embed mix: the side bytes XORed into the vector's first dword(s).
template <int K>
__device__ __forceinline__ u32x4 ref_fold(u32x4 v, typename RefSide<K>::T w) {
    if constexpr (K == 4) {
        v[0] ^= w[0];
        v[1] ^= w[1];
    } else {
        v[0] ^= (uint32_t)w;
    }
    return v;
}

// Extract mix: 2k bytes made from the vector (k = 1: low half of the XOR of
// its four dwords; k = 2: that XOR; k = 4: {v0 ^ v1, v2 ^ v3}).
template <int K>
__device__ __forceinline__ typename RefSide<K>::T ref_pack(u32x4 v) {
    if constexpr (K == 4) {
        u32x2 r;
        r[0] = v[0] ^ v[1];
        r[1] = v[2] ^ v[3];
        return r;
    } else {
        return (typename RefSide<K>::T)(v[0] ^ v[1] ^ v[2] ^ v[3]);
    }
}

// KIND 0: dst[i] = src[i].
// KIND 1: dst[i] = ref_fold(src[i], side[i])  (reads n + nk/8, writes n)
// KIND 2: out[i] = ref_pack(src[i])           (reads n, writes nk/8)
template <int KIND, int K>
__device__ __forceinline__ void ref_one(u32x4 *dst, typename RefSide<K>::T *out, uint64_t i, u32x4 v,
                                        typename RefSide<K>::T w) {
    if constexpr (KIND == 0) {
        __builtin_nontemporal_store(v, dst + i);
    } else if constexpr (KIND == 1) {
        __builtin_nontemporal_store(ref_fold<K>(v, w), dst + i);
    } else {
        out[i] = ref_pack<K>(v);
    }
}

template <int KIND, int K, int UNR>
__global__ void __launch_bounds__(1024)
    lsb_stream_ref_kernel(const u32x4 *src, u32x4 *dst, const typename RefSide<K>::T *side,
                          typename RefSide<K>::T *out, uint64_t nv) {
    typedef typename RefSide<K>::T S;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (UNR - 1) * stride < nv; i += UNR * stride) {
        u32x4 v[UNR];
        S w[UNR];
#pragma unroll
        for (int j = 0; j < UNR; ++j) {
            v[j] = __builtin_nontemporal_load(src + i + j * stride);
            w[j] = KIND == 1 ? side[i + j * stride] : S{};
        }
#pragma unroll
        for (int j = 0; j < UNR; ++j) ref_one<KIND, K>(dst, out, i + j * stride, v[j], w[j]);
    }
    for (; i < nv; i += stride) ref_one<KIND, K>(dst, out, i, src[i], KIND == 1 ? side[i] : S{});
}

// Type-erased launch of one (KIND, K, UNR) kernel.
typedef void (*RefLaunch)(dim3, dim3, hipStream_t, hipEvent_t, hipEvent_t, const void *, void *, const void *,
                          uint64_t);

template <int KIND, int K, int UNR>
static void ref_launch(dim3 g, dim3 b, hipStream_t st, hipEvent_t e0, hipEvent_t e1, const void *src, void *dst,
                       const void *side, uint64_t nv) {
    typedef typename RefSide<K>::T S;
    hipExtLaunchKernelGGL((lsb_stream_ref_kernel<KIND, K, UNR>), g, b, 0, st, e0, e1, 0,
                          reinterpret_cast<const u32x4 *>(src), reinterpret_cast<u32x4 *>(dst),
                          reinterpret_cast<const S *>(side), reinterpret_cast<S *>(dst), nv);
}

template <int KIND, int K>
static RefLaunch ref_fn_k(int unroll) {
    return unroll == 1 ? ref_launch<KIND, K, 1> : unroll == 2 ? ref_launch<KIND, K, 2> : ref_launch<KIND, K, 4>;
}

template <int KIND>
static RefLaunch ref_fn(int k, int unroll) {
    return k == 1 ? ref_fn_k<KIND, 1>(unroll) : k == 2 ? ref_fn_k<KIND, 2>(unroll) : ref_fn_k<KIND, 4>(unroll);
}

}  // namespace lsb

using namespace lsb;

extern "C" int lsb_stream_reference(int kind, int k, const uint8_t *src, uint8_t *dst, const uint8_t *side,
                                    uint64_t n, int block, int unroll, uint32_t grid, void *stream) {
    const TimedCall timed_call;
    if (kind < LSB_REF_COPY || kind > LSB_REF_EXTRACT_MIX)
        return fail(LSB_E_ARG, "lsb_stream_reference: kind %d unknown", kind);
    if (k != 1 && k != 2 && k != 4) return fail(LSB_E_ARG, "lsb_stream_reference: k %d not 1, 2 or 4", k);
    if (block != 256 && block != 512 && block != 1024)
        return fail(LSB_E_ARG, "lsb_stream_reference: block %d not 256, 512 or 1024", block);
    if (unroll != 1 && unroll != 2 && unroll != 4)
        return fail(LSB_E_ARG, "lsb_stream_reference: unroll %d not 1, 2 or 4", unroll);
    if (n % 16) return fail(LSB_E_ARG, "lsb_stream_reference: n = %llu not a multiple of 16", (unsigned long long)n);
    if (n == 0) return LSB_OK;
    if (!src || !dst || (kind == LSB_REF_EMBED_MIX && !side))
        return fail(LSB_E_ARG, "lsb_stream_reference: null pointer");
    const uint64_t nv = n / 16;
    const uint64_t side_bytes = 2 * (uint64_t)k * nv;  // n*k/8
    const uint64_t dst_bytes = kind == LSB_REF_EXTRACT_MIX ? side_bytes : n;
    const uintptr_t side_align = 2u * (uintptr_t)k - 1u;
    if (((uintptr_t)src & 15u) || (kind != LSB_REF_EXTRACT_MIX && ((uintptr_t)dst & 15u)) ||
        (kind == LSB_REF_EXTRACT_MIX && ((uintptr_t)dst & side_align)) ||
        (kind == LSB_REF_EMBED_MIX && ((uintptr_t)side & side_align)))
        return fail(LSB_E_ARG, "lsb_stream_reference: misaligned pointer");
    if (overlaps(src, n, dst, dst_bytes) || (kind == LSB_REF_EMBED_MIX && overlaps(side, side_bytes, dst, dst_bytes)))
        return fail(LSB_E_ARG, "lsb_stream_reference: output overlaps an input");
    const uint64_t full = ceil_div(nv, (uint64_t)block * unroll);
    uint64_t g = grid ? grid : full;
    if (g > full) g = full;
    if (g > 0x7FFFFFFFull) g = 0x7FFFFFFFull;
    const RefLaunch fn = kind == LSB_REF_COPY        ? ref_fn<0>(1, unroll)
                         : kind == LSB_REF_EMBED_MIX ? ref_fn<1>(k, unroll)
                                                     : ref_fn<2>(k, unroll);
    hipEvent_t e0, e1;
    take_launch_events(&e0, &e1);
    fn(dim3((unsigned)g), dim3(block), (hipStream_t)stream, e0, e1, src, dst, side, nv);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LSB_OK : hip_fail(e, "stream reference kernel launch");
}
