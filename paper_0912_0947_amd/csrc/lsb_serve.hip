// lsb_serve.hip -- open-loop serving with continuous batching over the
// batched kernel.
//
// One host thread runs the loop: arrivals whose scheduled time has come are
// admitted in order while the HBM budget (the caller's arena) has room for
// their outputs; admitted requests go into the next launch on any free slot
// (a slot = one embed plan + one extract plan + a stream + an event), so
// several launches overlap on the device and requests that arrive while
// others run join the next one.  Completions are found by polling the slot
// events; stego buffers stay resident until an extract consumes them or the
// budget needs their space (oldest first).
//
// The paper serves one image row per blocking MEX call (Section V: copy in,
// launch, copy out); the roles of that call -- validate, place on the
// device, run, return -- are kept, spread over many requests in flight.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <vector>

#include "lsb_host.hpp"

using namespace lsb;

namespace {

constexpr uint64_t kNone = ~0ull;
constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) in 256-byte granules.
class Arena {
   public:
    explicit Arena(uint64_t size) : size_(size) {
        if (size) free_[0] = size;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = align_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = align_up(bytes ? bytes : 1);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t peak() const { return peak_; }

   private:
    uint64_t size_;
    uint64_t used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

struct Slot {
    lsb_plan *plan[2] = {nullptr, nullptr};  // [op]
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint64_t status_off = 0;  // arena offset of 2 x max_batch int32 statuses
    uint64_t len_off = 0;     // arena offset of 2 x max_batch uint32 lengths
    int32_t *status_host = nullptr;
    uint32_t *len_host = nullptr;
    std::vector<int> reqs[2];
    bool busy = false;
};

struct Served {
    uint64_t out_bytes = 0;  // bytes of the output allocation
    bool live = false;       // embed: stego resident and not yet claimed
};

double embed_bytes(uint64_t n, uint32_t len) { return 2.0 * (double)n + 4.0 + (double)len; }
double extract_bytes(uint64_t n_unused, uint32_t len, int k) {
    (void)n_unused;
    return (double)ceil_div(8 * (4 + (uint64_t)len), (uint64_t)k) + (double)len;
}

}  // namespace

extern "C" int lsb_serve(const lsb_server_cfg *cfg, const lsb_request *req, int n_req, lsb_result *res,
                         lsb_serve_stats *stats) {
    clear_error();
    if (!cfg || (!req && n_req) || (!res && n_req) || n_req < 0)
        return fail(LSB_E_ARG, "lsb_serve: null argument");
    if (!cfg->arena || ((uintptr_t)cfg->arena & 255) || ((uintptr_t)cfg->cover_pool & 255) ||
        ((uintptr_t)cfg->msg_pool & 255))
        return fail(LSB_E_ARG, "lsb_serve: arena and pools must be 256-byte aligned device buffers");
    if (cfg->max_batch < 1 || cfg->max_batch > 65536 || cfg->n_slots < 1 || cfg->n_slots > 16 || cfg->reserved)
        return fail(LSB_E_ARG, "lsb_serve: max_batch 1..65536, n_slots 1..16, reserved 0");
    for (int i = 0; i < n_req; ++i) {
        const lsb_request &r = req[i];
        if (r.op != LSB_OP_EMBED && r.op != LSB_OP_EXTRACT) return fail(LSB_E_ARG, "request %d: bad op", i);
        if (r.k < 1 || r.k > 8) return fail(LSB_E_ARG, "request %d: k outside 1..8", i);
        if ((r.cover_off | r.msg_off) & 255) return fail(LSB_E_ARG, "request %d: offsets must be 256-aligned", i);
        if (i && r.arrival_s < req[i - 1].arrival_s) return fail(LSB_E_ARG, "requests must be sorted by arrival");
        if (r.target >= i) return fail(LSB_E_ARG, "request %d: target must be an earlier request", i);
        if (r.reserved) return fail(LSB_E_ARG, "request %d: reserved must be 0", i);
        const uint64_t room = room_bytes(r.n, r.k);
        if (room < 4 || r.len > room - 4) return fail(LSB_E_CAPACITY, "request %d: message exceeds capacity", i);
    }

    const int B = cfg->max_batch, S = cfg->n_slots;
    Arena arena(cfg->arena_bytes);
    std::vector<Slot> slots(S);
    int rc = LSB_OK;
    auto cleanup = [&]() {
        for (Slot &s : slots) {
            if (s.busy && s.done) hipEventSynchronize(s.done);
            for (lsb_plan *p : s.plan)
                if (p) lsb_plan_destroy(p);
            if (s.done) hipEventDestroy(s.done);
            if (s.stream) hipStreamDestroy(s.stream);
            if (s.status_host) hipHostFree(s.status_host);
            if (s.len_host) hipHostFree(s.len_host);
        }
    };
    for (Slot &s : slots) {
        if (!arena.alloc(sizeof(int32_t) * 2 * B, &s.status_off) || !arena.alloc(sizeof(uint32_t) * 2 * B, &s.len_off)) {
            cleanup();
            return fail(LSB_E_NOMEM, "lsb_serve: arena too small for per-slot status arrays");
        }
        hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s.status_host, sizeof(int32_t) * 2 * B, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&s.len_host, sizeof(uint32_t) * 2 * B, hipHostMallocDefault);
        if (e != hipSuccess) {
            cleanup();
            return hip_fail(e, "lsb_serve: slot setup");
        }
        for (int op = 0; op < 2 && rc == LSB_OK; ++op) rc = lsb_plan_create(&s.plan[op], B);
        if (rc != LSB_OK) {
            cleanup();
            return rc;
        }
    }

    std::vector<Served> sv(n_req);
    for (int i = 0; i < n_req; ++i) {
        lsb_result &r = res[i];
        memset(&r, 0, sizeof r);
        r.out_off = kNone;
        r.target = -1;
        r.status = 1;  // not finished
        r.k = req[i].k;
    }
    std::deque<int> waiting, ready, live;  // arrived / admitted / completed embeds with resident stego
    std::vector<lsb_job> jobs((size_t)B);
    std::vector<double> lat;
    lat.reserve(n_req);
    int next = 0, finished = 0;
    int64_t launches = 0, evictions = 0, stalls = 0, rejected = 0, batched = 0;
    bool stalled = false;
    double bytes = 0, first_arrival = n_req ? req[0].arrival_s : 0, last_done = 0;
    const auto t0 = std::chrono::steady_clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    auto in_flight = [&]() {
        for (const Slot &s : slots)
            if (s.busy) return true;
        return !ready.empty();
    };
    auto release_out = [&](int i) {
        if (res[i].out_off != kNone) {
            arena.release(res[i].out_off, sv[i].out_bytes);
            res[i].out_off = kNone;
        }
    };

    while (finished < n_req && rc == LSB_OK) {
        double now = now_s();
        while (next < n_req && req[next].arrival_s <= now) waiting.push_back(next++);

        // ---- admission, in arrival order, against the HBM budget
        while (!waiting.empty()) {
            const int i = waiting.front();
            const lsb_request &q = req[i];
            lsb_result &r = res[i];
            int target = -1;
            if (q.op == LSB_OP_EXTRACT) {
                if (q.target >= 0) {
                    if (sv[q.target].live) {
                        target = (int)q.target;
                        live.erase(std::find(live.begin(), live.end(), target));
                    }
                } else if (!live.empty()) {
                    target = live.front();
                    live.pop_front();
                }
                if (target >= 0) sv[target].live = false;  // claimed by this extract
            }
            const uint64_t need = target >= 0 ? res[target].len : q.n;
            uint64_t off = 0;
            bool ok = arena.alloc(need, &off);
            while (!ok && !cfg->keep_outputs && !live.empty()) {  // evict the oldest resident stego
                const int v = live.front();
                live.pop_front();
                sv[v].live = false;
                release_out(v);
                ++evictions;
                ok = arena.alloc(need, &off);
            }
            if (!ok) {
                if (target >= 0) {  // give the claim back
                    sv[target].live = true;
                    live.push_front(target);
                }
                if (in_flight()) {
                    if (!stalled) ++stalls;
                    stalled = true;
                    break;  // wait for completions to free memory
                }
                r.status = LSB_E_NOMEM;  // can never fit the budget
                r.done_s = now;
                ++rejected;
                ++finished;
                waiting.pop_front();
                continue;
            }
            stalled = false;
            waiting.pop_front();
            r.admit_s = now;
            r.out_off = off;
            sv[i].out_bytes = need;
            if (target >= 0) {
                r.op_run = LSB_OP_EXTRACT;
                r.target = target;
                r.k = res[target].k;
            } else {
                r.op_run = LSB_OP_EMBED;
                r.len = q.len;
            }
            ready.push_back(i);
        }

        // ---- launch admitted requests on free slots
        for (Slot &s : slots) {
            if (ready.empty() || rc != LSB_OK) break;
            if (s.busy) continue;
            s.reqs[0].clear();
            s.reqs[1].clear();
            for (int c = 0; c < B && !ready.empty(); ++c) {
                const int i = ready.front();
                ready.pop_front();
                s.reqs[res[i].op_run].push_back(i);
            }
            now = now_s();
            uint8_t *arena_p = cfg->arena;
            for (int op = 0; op < 2 && rc == LSB_OK; ++op) {
                const std::vector<int> &ids = s.reqs[op];
                if (ids.empty()) continue;
                for (size_t j = 0; j < ids.size(); ++j) {
                    const int i = ids[j];
                    lsb_job &J = jobs[j];
                    memset(&J, 0, sizeof J);
                    J.op = (uint8_t)op;
                    if (op == LSB_OP_EMBED) {
                        J.cover_off = req[i].cover_off;
                        J.stego_off = res[i].out_off;
                        J.msg_off = req[i].msg_off;
                        J.n = req[i].n;
                        J.len = req[i].len;
                        J.k = req[i].k;
                    } else {
                        const int t = (int)res[i].target;
                        J.stego_off = res[t].out_off;
                        J.msg_off = res[i].out_off;
                        J.n = req[t].n;
                        J.msg_cap = res[t].len;
                        J.k = res[t].k;
                    }
                    res[i].launch_s = now;
                }
                rc = lsb_plan_set_jobs(s.plan[op], jobs.data(), (int)ids.size());
                if (rc != LSB_OK) break;
                int32_t *st = (int32_t *)(arena_p + s.status_off) + op * B;
                uint32_t *ln = (uint32_t *)(arena_p + s.len_off) + op * B;
                rc = lsb_plan_run(s.plan[op], op == LSB_OP_EMBED ? cfg->cover_pool : nullptr, arena_p,
                                  op == LSB_OP_EMBED ? (uint8_t *)cfg->msg_pool : arena_p, ln, st, s.stream);
                if (rc != LSB_OK) break;
                hipError_t e = hipMemcpyAsync(s.status_host + op * B, st, sizeof(int32_t) * ids.size(),
                                              hipMemcpyDeviceToHost, s.stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(s.len_host + op * B, ln, sizeof(uint32_t) * ids.size(), hipMemcpyDeviceToHost,
                                       s.stream);
                if (e != hipSuccess) rc = hip_fail(e, "lsb_serve: status copy");
            }
            if (rc != LSB_OK) break;
            hipError_t e = hipEventRecord(s.done, s.stream);
            if (e != hipSuccess) {
                rc = hip_fail(e, "lsb_serve: event record");
                break;
            }
            s.busy = true;
            ++launches;
            batched += (int64_t)(s.reqs[0].size() + s.reqs[1].size());
        }

        // ---- completions
        for (Slot &s : slots) {
            if (!s.busy || rc != LSB_OK) continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                rc = hip_fail(q, "lsb_serve: event query");
                break;
            }
            s.busy = false;
            now = now_s();
            for (int op = 0; op < 2; ++op) {
                for (size_t j = 0; j < s.reqs[op].size(); ++j) {
                    const int i = s.reqs[op][j];
                    lsb_result &r = res[i];
                    r.status = s.status_host[op * B + j];
                    r.done_s = now;
                    ++finished;
                    last_done = now;
                    lat.push_back(now - req[i].arrival_s);
                    if (op == LSB_OP_EMBED) {
                        bytes += embed_bytes(req[i].n, req[i].len);
                        if (r.status == LSB_OK) {
                            sv[i].live = true;
                            live.push_back(i);
                        } else if (!cfg->keep_outputs) {
                            release_out(i);
                        }
                    } else {
                        const int t = (int)r.target;
                        r.len = s.len_host[op * B + j];
                        bytes += extract_bytes(req[t].n, res[t].len, res[t].k);
                        if (!cfg->keep_outputs) {
                            release_out(i);  // message delivered
                            release_out(t);  // its stego is consumed
                        }
                    }
                }
            }
        }
    }

    cleanup();
    if (rc != LSB_OK) return rc;
    if (stats) {
        memset(stats, 0, sizeof *stats);
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double p) {
            if (lat.empty()) return 0.0;
            size_t idx = (size_t)(p * (double)(lat.size() - 1) + 0.5);
            return lat[std::min(idx, lat.size() - 1)] * 1e3;
        };
        stats->makespan_s = last_done - first_arrival;
        stats->bytes = bytes;
        stats->gbps = stats->makespan_s > 0 ? bytes / stats->makespan_s / 1e9 : 0;
        stats->p50_ms = pct(0.50);
        stats->p99_ms = pct(0.99);
        stats->max_ms = lat.empty() ? 0 : lat.back() * 1e3;
        double sum = 0;
        for (double v : lat) sum += v;
        stats->mean_ms = lat.empty() ? 0 : sum / (double)lat.size() * 1e3;
        stats->launches = launches;
        stats->evictions = evictions;
        stats->admission_stalls = stalls;
        stats->rejected = rejected;
        stats->mean_batch = launches ? (double)batched / (double)launches : 0;
        stats->peak_arena_bytes = arena.peak();
    }
    return LSB_OK;
}
