// lsb_host.hpp -- host-side helpers shared by the translation units of
// liblsb.so: error reporting, device properties, launch-configuration table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/lsb.h"
#include "lsb_device.hpp"

namespace lsb {

// Thread-local message for lsb_last_error().
int fail(int code, const char *fmt, ...);
void clear_error();

// Map a HIP error to LSB_E_HIP with a message naming the call.
int hip_fail(hipError_t e, const char *what);

// Events set by lsb_time_next_launch for the calling thread; returns them
// and clears the request (both null when none is pending).
void take_launch_events(hipEvent_t *start, hipEvent_t *stop);
int set_launch_events(void *start, void *stop);

// Scope of an entry point that honours lsb_time_next_launch: clears the
// error message on entry and, on return, a timing request that no launch
// took (the call failed or had nothing to launch), so that the events never
// reach a later call.
struct TimedCall {
    TimedCall() { clear_error(); }
    ~TimedCall() { set_launch_events(nullptr, nullptr); }
    TimedCall(const TimedCall &) = delete;
    TimedCall &operator=(const TimedCall &) = delete;
};

// Compute units of the current device (cached per device).
int device_cus();

// true if [a, a+na) and [b, b+nb) share a byte.
inline bool overlaps(const void *a, uint64_t na, const void *b, uint64_t nb) {
    if (!na || !nb) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Launch configuration table, indexed by op (0 embed, 1 extract), k and
// size bucket floor(log2(n)).
constexpr int kBuckets = 64;
lsb_launch_cfg tune_lookup(int op, int k, uint64_t n);
bool cfg_valid(const lsb_launch_cfg &c);

// Grid size for `vectors` 16-byte vectors under configuration c.
inline unsigned grid_for(const lsb_launch_cfg &c, uint64_t vectors) {
    const uint64_t per_block = (uint64_t)c.block * (uint64_t)c.unroll;  // vectors per block step
    uint64_t blocks = ceil_div(vectors, per_block);
    if (blocks == 0) blocks = 1;
    if (c.blocks_per_cu > 0) {
        const uint64_t cap = (uint64_t)c.blocks_per_cu * (uint64_t)device_cus();
        if (blocks > cap) blocks = cap;
    }
    if (blocks > 0x7FFFFFFFull) blocks = 0x7FFFFFFFull;
    return (unsigned)blocks;
}

// Plain-kernel launchers (lsb_plain.hip); they validate nothing.
int launch_embed(const Span &s, const lsb_launch_cfg &c, hipStream_t stream);
int launch_extract(const Span &s, int header, uint64_t out_cap, uint32_t *len_out,
                   int32_t *status_out, uint64_t max_vectors, const lsb_launch_cfg &c,
                   hipStream_t stream);

}  // namespace lsb
