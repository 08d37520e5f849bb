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
// The scheduler is written against an executor interface.  lsb_serve runs it
// with the HIP executor on the real clock; lsb_serve_simulate runs the same
// scheduler with a host-only executor whose launches finish after a modelled
// time on a virtual clock, so that admission, batching and eviction can be
// tested without a GPU.
//
// The paper serves one image row per blocking MEX call (Section V: copy in,
// launch, copy out); the roles of that call -- validate, place on the
// device, run, return -- are kept, spread over many requests in flight.
#include <string.h>

#include <algorithm>
#include <cstddef>
#include <chrono>
#include <deque>
#include <map>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "lsb_host.hpp"

using namespace lsb;

namespace {

// roctx range over one phase of a loop iteration (admission, launch,
// completion), so that a trace taken with rocprofv3 --marker-trace shows
// where the host thread spends its time.  Without a profiler attached a
// range costs two calls into the roctx library.
class PhaseRange {
   public:
    explicit PhaseRange(const char *name) { roctxRangePushA(name); }
    ~PhaseRange() { roctxRangePop(); }
    PhaseRange(const PhaseRange &) = delete;
    PhaseRange &operator=(const PhaseRange &) = delete;
};

constexpr uint64_t kNone = ~0ull;
constexpr uint64_t kAlign = 256;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) in 256-byte granules.
class Arena {
   public:
    explicit Arena(uint64_t size) {
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
    uint64_t used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

double embed_bytes(uint64_t n, uint32_t len) { return 2.0 * (double)n + 4.0 + (double)len; }
double extract_bytes(uint32_t len, int k) {
    return (double)ceil_div(8 * (4 + (uint64_t)len), (uint64_t)k) + (double)len;
}

// ---------------------------------------------------------------------------
// Executors.  launch() takes a slot's embed and extract job lists (either may
// be empty); poll() reports whether the slot's launch has finished and then
// fills the per-job status and decoded length.
struct Executor {
    virtual ~Executor() {}
    virtual int launch(int slot, const lsb_job *jobs_e, int ne, const lsb_job *jobs_x, int nx) = 0;
    virtual int poll(int slot, bool *done) = 0;
    virtual int32_t status(int slot, int op, int j) const = 0;
    virtual uint32_t length(int slot, int op, int j) const = 0;
    virtual double now() = 0;
    // Nothing can happen before `t` (next arrival) unless a launch finishes:
    // a virtual clock jumps there; the real clock just keeps running.
    virtual void idle(double t) = 0;
};

class HipExecutor : public Executor {
   public:
    HipExecutor(const lsb_server_cfg *cfg, int slots, int batch) : cfg_(cfg), B_(batch), s_(slots) {
        t0_ = std::chrono::steady_clock::now();
    }
    // The run's clock starts here, once the slots are set up, so that the
    // first arrivals are not charged for stream, event and plan creation.
    void start_clock() { t0_ = std::chrono::steady_clock::now(); }
    ~HipExecutor() override {
        for (S &s : s_) {
            // teardown: nothing useful can be done with a failure here.  A
            // launch that failed part-way may have left work on the stream
            // (a plan run, a status copy into status_host), so drain it first.
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            for (lsb_plan *p : s.plan)
                if (p) lsb_plan_destroy(p);
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.stream) (void)hipStreamDestroy(s.stream);
            if (s.status_host) (void)hipHostFree(s.status_host);
            if (s.len_host) (void)hipHostFree(s.len_host);
        }
    }
    // status_off / len_off: arena offsets of 2*B int32 / uint32 per slot.
    // Embed jobs report their status in status_dev[0, B); extract jobs their
    // decoded length in len_dev[0, B) and their status right after it, in
    // len_dev[B, 2B), so one copy brings an extract launch's results back.
    int init(const std::vector<uint64_t> &status_off, const std::vector<uint64_t> &len_off) {
        for (size_t i = 0; i < s_.size(); ++i) {
            S &s = s_[i];
            s.status_dev = (int32_t *)(cfg_->arena + status_off[i]);
            s.len_dev = (uint32_t *)(cfg_->arena + len_off[i]);
            hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
            if (e == hipSuccess) e = hipHostMalloc((void **)&s.status_host, sizeof(int32_t) * 2 * B_, hipHostMallocDefault);
            if (e == hipSuccess) e = hipHostMalloc((void **)&s.len_host, sizeof(uint32_t) * 2 * B_, hipHostMallocDefault);
            if (e != hipSuccess) return hip_fail(e, "lsb_serve: slot setup");
            for (int op = 0; op < 2; ++op) {
                const int rc = lsb_plan_create(&s.plan[op], nullptr, B_, op);
                if (rc != LSB_OK) return rc;
            }
        }
        return LSB_OK;
    }
    int launch(int slot, const lsb_job *jobs_e, int ne, const lsb_job *jobs_x, int nx) override {
        S &s = s_[slot];
        const lsb_job *jobs[2] = {jobs_e, jobs_x};
        const int cnt[2] = {ne, nx};
        for (int op = 0; op < 2; ++op) {
            if (!cnt[op]) continue;
            if (cnt[op] <= kDirectMax) {
                const int rc = launch_direct(s, op, jobs[op], cnt[op]);
                if (rc != LSB_OK) return rc;
                continue;
            }
            int rc = lsb_plan_update(s.plan[op], jobs[op], cnt[op]);
            if (rc != LSB_OK) return rc;
            const bool emb = op == LSB_OP_EMBED;
            int32_t *st = emb ? s.status_dev : (int32_t *)(s.len_dev + B_);
            uint32_t *ln = emb ? nullptr : s.len_dev;
            rc = lsb_plan_run(s.plan[op], emb ? cfg_->cover_pool : nullptr, cfg_->arena,
                              emb ? (uint8_t *)cfg_->msg_pool : cfg_->arena, ln, st, s.stream);
            if (rc != LSB_OK) return rc;
            // one copy per launch: embed statuses, or an extract's lengths
            // together with the statuses that follow them
            const hipError_t e =
                emb ? hipMemcpyAsync(s.status_host, st, sizeof(int32_t) * cnt[op], hipMemcpyDeviceToHost, s.stream)
                    : hipMemcpyAsync(s.len_host, ln, sizeof(uint32_t) * ((size_t)B_ + cnt[op]), hipMemcpyDeviceToHost,
                                     s.stream);
            if (e != hipSuccess) return hip_fail(e, "lsb_serve: status copy");
        }
        const hipError_t e = hipEventRecord(s.done, s.stream);
        if (e != hipSuccess) return hip_fail(e, "lsb_serve: event record");
        s.busy = true;
        return LSB_OK;
    }
    int poll(int slot, bool *done) override {
        S &s = s_[slot];
        const hipError_t q = hipEventQuery(s.done);
        if (q == hipErrorNotReady) {
            *done = false;
            return LSB_OK;
        }
        if (q != hipSuccess) return hip_fail(q, "lsb_serve: event query");
        s.busy = false;
        *done = true;
        return LSB_OK;
    }
    int32_t status(int slot, int op, int j) const override {
        const S &s = s_[slot];
        return op == LSB_OP_EMBED ? s.status_host[j] : (int32_t)s.len_host[B_ + j];
    }
    uint32_t length(int slot, int op, int j) const override {
        return op == LSB_OP_EXTRACT ? s_[slot].len_host[j] : 0u;
    }
    double now() override {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
    }
    void idle(double) override {}

   private:
    struct S;
    // A launch of at most kDirectMax jobs issues them through the plain entry
    // points, one kernel each, instead of a plan (no table upload or graph):
    // a plan's host-side cost is that of about five plain launches.  Results and statuses are those a plan reports.  An embed
    // over capacity is refused on the host and its status set here; extracts
    // report decoded lengths and statuses on the device, in the same places
    // as a plan's, and one copy brings them back.
    static constexpr int kDirectMax = 4;
    int launch_direct(S &s, int op, const lsb_job *jobs, int cnt) {
        if (op == LSB_OP_EMBED) {
            for (int j = 0; j < cnt; ++j) {
                const lsb_job &J = jobs[j];
                const int rc = lsb_embed(cfg_->cover_pool + J.cover_off, cfg_->arena + J.stego_off, J.n,
                                         cfg_->msg_pool + J.msg_off, J.len, J.k, s.stream);
                if (rc != LSB_OK && rc != LSB_E_CAPACITY) return rc;
                clear_error();  // a refused job is a status, not an error of the run
                s.status_host[j] = rc;
            }
            return LSB_OK;
        }
        uint32_t *ln = s.len_dev;
        int32_t *st = (int32_t *)(s.len_dev + B_);
        for (int j = 0; j < cnt; ++j) {
            const lsb_job &J = jobs[j];
            const int rc = lsb_extract(cfg_->arena + J.stego_off, J.n, J.k, cfg_->arena + J.msg_off, J.msg_cap, ln + j,
                                       st + j, s.stream);
            if (rc != LSB_OK) return rc;
        }
        const hipError_t e = hipMemcpyAsync(s.len_host, ln, sizeof(uint32_t) * ((size_t)B_ + cnt),
                                            hipMemcpyDeviceToHost, s.stream);
        return e == hipSuccess ? LSB_OK : hip_fail(e, "lsb_serve: status copy");
    }
    struct S {
        lsb_plan *plan[2] = {nullptr, nullptr};
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
        int32_t *status_dev = nullptr;
        uint32_t *len_dev = nullptr;
        int32_t *status_host = nullptr;
        uint32_t *len_host = nullptr;
        bool busy = false;
    };
    const lsb_server_cfg *cfg_;
    int B_;
    std::vector<S> s_;
    std::chrono::steady_clock::time_point t0_;
};

// Host-only executor on a virtual clock: a launch finishes
// fixed_us + bytes / gbps after it starts, slots run independently, every
// job succeeds (extract jobs report their message capacity as the decoded
// length).  Nothing is computed.
class SimExecutor : public Executor {
   public:
    SimExecutor(int slots, int batch, double fixed_us, double gbps)
        : B_(batch), fixed_(fixed_us * 1e-6), gbps_(gbps), s_(slots) {
        for (S &s : s_) s.len.assign(2 * (size_t)batch, 0);
    }
    int launch(int slot, const lsb_job *jobs_e, int ne, const lsb_job *jobs_x, int nx) override {
        S &s = s_[slot];
        double bytes = 0;
        for (int j = 0; j < ne; ++j) bytes += embed_bytes(jobs_e[j].n, jobs_e[j].len);
        for (int j = 0; j < nx; ++j) {
            bytes += extract_bytes((uint32_t)jobs_x[j].msg_cap, jobs_x[j].k);
            s.len[B_ + j] = (uint32_t)jobs_x[j].msg_cap;
        }
        for (int j = 0; j < ne; ++j) s.len[j] = jobs_e[j].len;
        s.finish = t_ + fixed_ + bytes / (gbps_ * 1e9);
        s.busy = true;
        return LSB_OK;
    }
    int poll(int slot, bool *done) override {
        S &s = s_[slot];
        *done = s.busy && t_ >= s.finish;
        if (*done) s.busy = false;
        return LSB_OK;
    }
    int32_t status(int, int, int) const override { return LSB_OK; }
    uint32_t length(int slot, int op, int j) const override { return s_[slot].len[op * B_ + j]; }
    double now() override { return t_; }
    void idle(double t) override {
        double next = t;
        for (const S &s : s_)
            if (s.busy) next = std::min(next, s.finish);
        if (next > t_ && next < 1e300) t_ = next;
    }

   private:
    struct S {
        double finish = 0;
        bool busy = false;
        std::vector<uint32_t> len;
    };
    int B_;
    double fixed_, gbps_, t_ = 0;
    std::vector<S> s_;
};

int check_args(const lsb_server_cfg *cfg, const lsb_request *req, int n_req, lsb_result *res, bool device) {
    if (!cfg || (!req && n_req) || (!res && n_req) || n_req < 0) return fail(LSB_E_ARG, "lsb_serve: null argument");
    // any request may be served as an embed (an extract with nothing resident
    // is), so both pools are always needed
    if (device && (!cfg->arena || !cfg->cover_pool || !cfg->msg_pool || ((uintptr_t)cfg->arena & 255) ||
                   ((uintptr_t)cfg->cover_pool & 255) || ((uintptr_t)cfg->msg_pool & 255)))
        return fail(LSB_E_ARG, "lsb_serve: arena and pools must be non-null, 256-byte aligned device buffers");
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
        if (r.n > (1ull << 48)) return fail(LSB_E_ARG, "request %d: n out of range", i);
    }
    return LSB_OK;
}

struct Served {
    uint64_t out_bytes = 0;  // bytes of the output allocation
    bool live = false;       // embed: stego resident and not yet claimed
};

// The scheduler.  `arena` already holds the per-slot status arrays.
int run_scheduler(const lsb_server_cfg *cfg, const lsb_request *req, int n_req, lsb_result *res,
                  lsb_serve_stats *stats, Executor &ex, Arena &arena) {
    const int B = cfg->max_batch, S = cfg->n_slots;
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
    std::vector<std::vector<int>> slot_reqs[2];
    for (int op = 0; op < 2; ++op) slot_reqs[op].resize(S);
    std::vector<bool> busy(S, false);
    std::vector<lsb_job> jobs[2] = {std::vector<lsb_job>((size_t)B), std::vector<lsb_job>((size_t)B)};
    std::vector<double> lat;
    lat.reserve(n_req);
    int next = 0, finished = 0, rc = LSB_OK;
    int64_t launches = 0, evictions = 0, stalls = 0, rejected = 0, batched = 0;
    bool stalled = false;
    bool released = false;  // a completion released memory since the last admission pass
    double bytes = 0, first_arrival = n_req ? req[0].arrival_s : 0, last_done = 0;
    auto in_flight = [&]() {
        for (int s = 0; s < S; ++s)
            if (busy[s]) return true;
        return !ready.empty();
    };
    auto release_out = [&](int i) {
        if (res[i].out_off != kNone) {
            arena.release(res[i].out_off, sv[i].out_bytes);
            res[i].out_off = kNone;
        }
    };

    while (finished < n_req && rc == LSB_OK) {
        double now = ex.now();
        bool progressed = false;
        while (next < n_req && req[next].arrival_s <= now) waiting.push_back(next++);

        // ---- admission, in arrival order, against the HBM budget.  After a
        // stall the head of the queue can only fit once a completion has
        // released memory, so admission waits for one.
        if (!waiting.empty() && !(stalled && !released)) {
            released = false;
            const PhaseRange admit_range("lsb_serve:admit");
            while (!waiting.empty()) {
                const int i = waiting.front();
                const lsb_request &q = req[i];
                lsb_result &r = res[i];
                int target = -1;
                size_t target_pos = 0;  // where the claimed stego sat in `live`
                if (q.op == LSB_OP_EXTRACT) {
                    if (q.target >= 0) {
                        if (sv[q.target].live) {
                            target = (int)q.target;
                            const auto it = std::find(live.begin(), live.end(), target);
                            target_pos = (size_t)(it - live.begin());
                            live.erase(it);
                        }
                    } else if (!live.empty()) {
                        target = live.front();
                        live.pop_front();
                    }
                    if (target >= 0) sv[target].live = false;  // claimed by this extract
                }
                if (target < 0) {  // served as an embed: its message must fit its cover
                    const uint64_t room = room_bytes(q.n, q.k);
                    if (room < 4 || q.len > room - 4) {  // fails alone, at admission
                        r.status = LSB_E_CAPACITY;
                        r.op_run = LSB_OP_EMBED;
                        r.done_s = now;
                        ++rejected;
                        ++finished;
                        waiting.pop_front();
                        progressed = true;
                        continue;
                    }
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
                    if (target >= 0) {  // give the claim back, at its place in the age order
                        sv[target].live = true;
                        live.insert(live.begin() + (std::ptrdiff_t)std::min(target_pos, live.size()), target);
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
                    progressed = true;
                    continue;
                }
                stalled = false;
                waiting.pop_front();
                progressed = true;
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
        }

        // ---- launch admitted requests on free slots
        for (int s = 0; s < S && !ready.empty() && rc == LSB_OK; ++s) {
            if (busy[s]) continue;
            const PhaseRange launch_range("lsb_serve:launch");
            slot_reqs[0][s].clear();
            slot_reqs[1][s].clear();
            for (int c = 0; c < B && !ready.empty(); ++c) {
                const int i = ready.front();
                ready.pop_front();
                slot_reqs[res[i].op_run][s].push_back(i);
            }
            now = ex.now();
            for (int op = 0; op < 2; ++op) {
                const std::vector<int> &ids = slot_reqs[op][s];
                for (size_t j = 0; j < ids.size(); ++j) {
                    const int i = ids[j];
                    lsb_job &J = jobs[op][j];
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
            }
            rc = ex.launch(s, jobs[0].data(), (int)slot_reqs[0][s].size(), jobs[1].data(),
                           (int)slot_reqs[1][s].size());
            if (rc != LSB_OK) break;
            busy[s] = true;
            progressed = true;
            ++launches;
            batched += (int64_t)(slot_reqs[0][s].size() + slot_reqs[1][s].size());
        }

        // ---- completions
        for (int s = 0; s < S && rc == LSB_OK; ++s) {
            if (!busy[s]) continue;
            bool done = false;
            rc = ex.poll(s, &done);
            if (rc != LSB_OK || !done) continue;
            const PhaseRange complete_range("lsb_serve:complete");
            busy[s] = false;
            released = true;
            progressed = true;
            now = ex.now();
            for (int op = 0; op < 2; ++op) {
                const std::vector<int> &ids = slot_reqs[op][s];
                for (size_t j = 0; j < ids.size(); ++j) {
                    const int i = ids[j];
                    lsb_result &r = res[i];
                    r.status = ex.status(s, op, (int)j);
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
                        r.len = ex.length(s, op, (int)j);
                        bytes += extract_bytes(res[t].len, res[t].k);
                        if (!cfg->keep_outputs) {
                            release_out(i);  // message delivered
                            release_out(t);  // its stego is consumed
                        }
                    }
                }
            }
        }
        if (!progressed && rc == LSB_OK) ex.idle(next < n_req ? req[next].arrival_s : 1e300);
    }
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

// Per-slot status arrays come out of the budget first (2 x B int32 + 2 x B
// uint32 per slot).
int reserve_status(const lsb_server_cfg *cfg, Arena &arena, std::vector<uint64_t> &st, std::vector<uint64_t> &ln) {
    st.resize(cfg->n_slots);
    ln.resize(cfg->n_slots);
    for (int s = 0; s < cfg->n_slots; ++s)
        if (!arena.alloc(sizeof(int32_t) * 2 * cfg->max_batch, &st[s]) ||
            !arena.alloc(sizeof(uint32_t) * 2 * cfg->max_batch, &ln[s]))
            return fail(LSB_E_NOMEM, "lsb_serve: arena too small for per-slot status arrays");
    return LSB_OK;
}

}  // namespace

extern "C" int lsb_serve(const lsb_server_cfg *cfg, const lsb_request *req, int n_req, lsb_result *res,
                         lsb_serve_stats *stats) {
    clear_error();
    int rc = check_args(cfg, req, n_req, res, true);
    if (rc != LSB_OK) return rc;
    Arena arena(cfg->arena_bytes);
    std::vector<uint64_t> st, ln;
    rc = reserve_status(cfg, arena, st, ln);
    if (rc != LSB_OK) return rc;
    HipExecutor ex(cfg, cfg->n_slots, cfg->max_batch);
    rc = ex.init(st, ln);
    if (rc != LSB_OK) return rc;
    ex.start_clock();
    return run_scheduler(cfg, req, n_req, res, stats, ex, arena);
}

extern "C" int lsb_serve_simulate(const lsb_server_cfg *cfg, const lsb_request *req, int n_req, lsb_result *res,
                                  lsb_serve_stats *stats, double launch_us, double device_gbps) {
    clear_error();
    int rc = check_args(cfg, req, n_req, res, false);
    if (rc != LSB_OK) return rc;
    if (!(launch_us >= 0) || !(device_gbps > 0)) return fail(LSB_E_ARG, "lsb_serve_simulate: bad timing model");
    Arena arena(cfg->arena_bytes);
    std::vector<uint64_t> st, ln;
    rc = reserve_status(cfg, arena, st, ln);
    if (rc != LSB_OK) return rc;
    SimExecutor ex(cfg->n_slots, cfg->max_batch, launch_us, device_gbps);
    return run_scheduler(cfg, req, n_req, res, stats, ex, arena);
}
