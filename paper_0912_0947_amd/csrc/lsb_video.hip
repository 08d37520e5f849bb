// lsb_video.hip -- frames streamed from host memory through the GPU.
//
// The paper's MEX gateway copies each image row to the device, launches the
// kernel and copies the result back before MATLAB sends the next row
// (Sections III and V).  Here frames of a clip living in pinned host memory
// go round-robin over a few streams; each stream copies its frame into a
// ring slot, embeds it in place (raw slice at t0 = f * frame_bytes of one
// logical stream) and copies it back.  A slot is only reused by a later
// frame of the same stream, so stream order alone keeps the ring safe, and
// while one stream copies in another copies out: both PCIe directions stay
// busy.  (Splitting copy-in, embed and copy-out over three streams joined by
// events measured 33 GB/s each way against 43 GB/s for this layout.)
#include "lsb_host.hpp"

extern "C" int lsb_video_embed_host(const uint8_t *host_frames, uint8_t *host_stego, uint64_t frame_bytes,
                                    uint64_t frames, const uint8_t *stream_dev, uint64_t stream_bits, int k,
                                    uint8_t *dev_ring, uint32_t ring_slots, void *const *streams, int n_streams) {
    using namespace lsb;
    const TimedCall timed_call;
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_video_embed_host: k=%d outside 1..8", k);
    if (n_streams < 1 || n_streams > 16 || !streams)
        return fail(LSB_E_ARG, "lsb_video_embed_host: n_streams=%d outside 1..16", n_streams);
    for (int a = 0; a < n_streams; ++a)
        for (int b = a + 1; b < n_streams; ++b)
            if (streams[a] == streams[b]) return fail(LSB_E_ARG, "lsb_video_embed_host: streams must be distinct");
    if (ring_slots < 1 || ring_slots > 64 || ring_slots % (uint32_t)n_streams)
        return fail(LSB_E_ARG, "lsb_video_embed_host: ring_slots=%u must be a multiple of n_streams=%d in 1..64",
                    ring_slots, n_streams);
    if (!frames || !frame_bytes) return LSB_OK;
    if (!host_frames || !host_stego || !dev_ring) return fail(LSB_E_ARG, "lsb_video_embed_host: null buffer");
    if (stream_bits && !stream_dev) return fail(LSB_E_ARG, "lsb_video_embed_host: null stream");
    if (frame_bytes > (1ull << 40) || frames > (1ull << 24)) return fail(LSB_E_ARG, "lsb_video_embed_host: size");
    const lsb_launch_cfg cfg = tune_lookup(LSB_OP_EMBED, k, frame_bytes);
    for (uint64_t f = 0; f < frames; ++f) {
        hipStream_t st = (hipStream_t)streams[f % (uint64_t)n_streams];
        uint8_t *d = dev_ring + (f % ring_slots) * frame_bytes;
        hipError_t err = hipMemcpyAsync(d, host_frames + f * frame_bytes, frame_bytes, hipMemcpyHostToDevice, st);
        if (err != hipSuccess) return hip_fail(err, "video copy in");
        Span s{};
        s.src = d;
        s.dst = d;
        s.body = stream_dev;
        s.n = frame_bytes;
        s.t0 = f * frame_bytes;
        s.bits = stream_bits;
        s.hdr_len = 0;
        s.k = k;
        s.inplace = 1;
        const int rc = launch_embed(s, cfg, st);
        if (rc != LSB_OK) return rc;
        err = hipMemcpyAsync(host_stego + f * frame_bytes, d, frame_bytes, hipMemcpyDeviceToHost, st);
        if (err != hipSuccess) return hip_fail(err, "video copy out");
    }
    return LSB_OK;
}
