// lsb_video.hip -- frames streamed from host memory through the GPU.
//
// The paper's MEX gateway copies each image row to the device, launches the
// kernel and copies the result back before MATLAB sends the next row
// (Sections III and V).  Here frames of a clip living in pinned host memory
// flow through a ring of device slots on three streams -- copy in, embed in
// place (raw slice at t0 = f * frame_bytes of one logical stream), copy out
// -- so that the two PCIe directions and the kernels of different frames
// overlap.  Slot reuse is ordered by events, never by host waits.
#include <vector>

#include "lsb_host.hpp"

extern "C" int lsb_video_embed_host(const uint8_t *host_frames, uint8_t *host_stego, uint64_t frame_bytes,
                                    uint64_t frames, const uint8_t *stream_dev, uint64_t stream_bits, int k,
                                    uint8_t *dev_ring, uint32_t ring_slots, void *s_in, void *s_compute,
                                    void *s_out) {
    using namespace lsb;
    clear_error();
    if (k < 1 || k > 8) return fail(LSB_E_ARG, "lsb_video_embed_host: k=%d outside 1..8", k);
    if (!frames || !frame_bytes) return LSB_OK;
    if (!host_frames || !host_stego || !dev_ring) return fail(LSB_E_ARG, "lsb_video_embed_host: null buffer");
    if (ring_slots < 1 || ring_slots > 64) return fail(LSB_E_ARG, "lsb_video_embed_host: ring_slots 1..64");
    if (stream_bits && !stream_dev) return fail(LSB_E_ARG, "lsb_video_embed_host: null stream");
    if (frame_bytes > (1ull << 40) || frames > (1ull << 24)) return fail(LSB_E_ARG, "lsb_video_embed_host: size");
    hipStream_t sin = (hipStream_t)s_in, sc = (hipStream_t)s_compute, sout = (hipStream_t)s_out;
    if (sin == sc || sin == sout || sc == sout)
        return fail(LSB_E_ARG, "lsb_video_embed_host: the three streams must be distinct");
    std::vector<hipEvent_t> ev;  // per slot: copied in, embedded, copied out
    ev.resize(3 * (size_t)ring_slots, nullptr);
    int rc = LSB_OK;
    for (auto &e : ev) {
        hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
        if (err != hipSuccess) {
            rc = hip_fail(err, "hipEventCreate(video)");
            break;
        }
    }
    const lsb_launch_cfg cfg = tune_lookup(LSB_OP_EMBED, k, frame_bytes);
    for (uint64_t f = 0; f < frames && rc == LSB_OK; ++f) {
        const uint32_t slot = (uint32_t)(f % ring_slots);
        hipEvent_t e_in = ev[3 * slot], e_emb = ev[3 * slot + 1], e_out = ev[3 * slot + 2];
        uint8_t *d = dev_ring + (uint64_t)slot * frame_bytes;
        hipError_t err = hipSuccess;
        if (f >= ring_slots) err = hipStreamWaitEvent(sin, e_out, 0);  // slot drained by the copy out
        if (err == hipSuccess)
            err = hipMemcpyAsync(d, host_frames + f * frame_bytes, frame_bytes, hipMemcpyHostToDevice, sin);
        if (err == hipSuccess) err = hipEventRecord(e_in, sin);
        if (err == hipSuccess) err = hipStreamWaitEvent(sc, e_in, 0);
        if (err != hipSuccess) {
            rc = hip_fail(err, "video copy in");
            break;
        }
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
        rc = launch_embed(s, cfg, sc);
        if (rc != LSB_OK) break;
        err = hipEventRecord(e_emb, sc);
        if (err == hipSuccess) err = hipStreamWaitEvent(sout, e_emb, 0);
        if (err == hipSuccess)
            err = hipMemcpyAsync(host_stego + f * frame_bytes, d, frame_bytes, hipMemcpyDeviceToHost, sout);
        if (err == hipSuccess) err = hipEventRecord(e_out, sout);
        if (err != hipSuccess) rc = hip_fail(err, "video copy out");
    }
    // events may be destroyed while still pending: the runtime releases them
    // once they complete
    for (auto &e : ev)
        if (e) hipEventDestroy(e);
    return rc;
}
