// Serving runtime: continuous batching of volume-term requests over
// device-resident meshes of mixed n (3D Euler, one GPU).
//
//  * Meshes are registered once; their state lives in a device buffer the
//    server owns.
//  * sf_submit queues a request (FIFO).  A scheduler thread admits queued
//    requests in order while the output buffer fits the HBM budget (a
//    first-fit arena carved out of one device allocation) and fewer than
//    max_inflight requests hold output memory; a request larger than the
//    whole budget is rejected at submission (SF_ERR_BUDGET).
//  * Every scheduler tick packs all admitted, not yet launched requests into
//    one batch on a free launch slot (two slots on two streams, so a new
//    batch starts while the previous one drains): one serving kernel launch
//    per (precision, n) variant present (one workgroup per block of
//    elements of its requests), each a pre-built one-node hipGraph
//    replayed with the batch's grid and arguments -- its requests'
//    descriptors in the kernel arguments (or, for large batches, copied once
//    to the device).  Requests that arrive while a batch runs go into the
//    next one.
//  * Completion is observed by querying each slot's event; latency runs from
//    sf_submit to that observation on the host's steady clock.  The output
//    stays owned by the server until sf_release returns it to the budget.
//
// A host-only simulation executor (sf_server_create_sim) runs the same
// scheduler with a modelled service time and no device, for tests and
// capacity planning.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include <sys/prctl.h>

#include "sfhad_internal.h"

namespace sfhad {
namespace serve {

using Clock = std::chrono::steady_clock;

constexpr size_t kAlign = 256;
constexpr int kSlots = 2;  // 3 and 4 measured no better (p50/p99 within run-to-run spread)

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit sub-allocator over [0, cap) with coalescing free list.
class Arena {
public:
    void reset(size_t cap) {
        cap_ = cap;
        free_.clear();
        if (cap) free_[0] = cap;
        used_ = 0;
    }
    bool alloc(size_t bytes, size_t &off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                used_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = free_.emplace(off, bytes).first;
        used_ -= bytes;
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
    size_t used() const { return used_; }
    size_t cap() const { return cap_; }

private:
    size_t cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;
};

struct Mesh {
    double *u = nullptr;  // device (HIP executor) or null (simulation)
    int64_t E = 0;
    int n = 0;
    int node_kind = 0;
    size_t out_bytes = 0;
    int outstanding = 0;  // requests not yet released
};

enum class State { Queued, Admitted, Running, Done };

struct Request {
    int64_t ticket = 0;
    int64_t mesh = 0;
    int prec = 0;
    size_t off = 0, bytes = 0;
    State state = State::Queued;
    int status = SF_OK;  // SF_ERR_HIP when its batch could not be launched
    Clock::time_point t_submit, t_done;
};

// What the scheduler needs from a device (or from the simulation).
class Executor {
public:
    virtual ~Executor() = default;
    virtual int init(size_t arena_bytes, int max_inflight) = 0;
    virtual char *arena_base() = 0;
    virtual int mesh_upload(const double *u_src, size_t bytes, double **u_dev) = 0;
    virtual void mesh_free(double *u_dev) = 0;
    // Launch a batch on slot s (asynchronous).
    virtual int launch(int s, const std::vector<ServeDesc> &descs) = 0;
    virtual bool done(int s) = 0;   // non-blocking
    virtual void drain(int s) = 0;  // blocking
    // Make the next `count` launches fail (simulation only, for tests).
    virtual int fail_launches(int) { return SF_ERR_UNSUPPORTED; }
};

class HipExecutor : public Executor {
public:
    ~HipExecutor() override {
        for (int s = 0; s < kSlots; ++s) {
            for (int v = 0; v < kServeVariants; ++v) {
                if (gexec_[s][v]) (void)hipGraphExecDestroy(gexec_[s][v]);
                if (graph_[s][v]) (void)hipGraphDestroy(graph_[s][v]);
            }
            if (ev_[s]) (void)hipEventDestroy(ev_[s]);
            if (st_[s]) (void)hipStreamDestroy(st_[s]);
            if (ddesc_[s]) (void)hipFree(ddesc_[s]);
            if (hdesc_[s]) (void)hipHostFree(hdesc_[s]);
        }
        if (optab_) (void)hipFree(optab_);
        if (arena_) (void)hipFree(arena_);
    }

    int init(size_t arena_bytes, int max_inflight) override {
        maxr_ = max_inflight;
        if (hipGetDevice(&device_) != hipSuccess) return fail_hip("hipGetDevice");
        if (arena_bytes && hipMalloc(&arena_, arena_bytes) != hipSuccess) {
            set_error("serving arena allocation failed");
            return SF_ERR_NOMEM;
        }
        std::vector<double> tab(serve_optable_doubles());
        serve_fill_optable(tab.data());
        if (hipMalloc(&optab_, tab.size() * sizeof(double)) != hipSuccess) return fail_hip("hipMalloc optable");
        if (hipMemcpy(optab_, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
            return fail_hip("optable upload");
        const size_t dbytes = sizeof(ServeDesc) * (size_t)maxr_;
        for (int s = 0; s < kSlots; ++s) {
            if (hipStreamCreateWithFlags(&st_[s], hipStreamNonBlocking) != hipSuccess) return fail_hip("stream");
            if (hipEventCreateWithFlags(&ev_[s], hipEventDisableTiming) != hipSuccess) return fail_hip("event");
            if (hipMalloc(&ddesc_[s], dbytes) != hipSuccess) return fail_hip("descriptor buffer");
            if (hipHostMalloc(&hdesc_[s], dbytes, hipHostMallocDefault) != hipSuccess)
                return fail_hip("pinned descriptor buffer");
            for (int v = 0; v < kServeVariants; ++v) {
                int st = build_graph(s, v);
                if (st != SF_OK) return st;
            }
        }
        return SF_OK;
    }

    char *arena_base() override { return reinterpret_cast<char *>(arena_); }

    int mesh_upload(const double *u_src, size_t bytes, double **u_dev) override {
        if (hipMalloc(u_dev, bytes) != hipSuccess) {
            set_error("mesh allocation failed");
            return SF_ERR_NOMEM;
        }
        // host or device source: the runtime tells them apart (unified addressing)
        if (hipMemcpy(*u_dev, u_src, bytes, hipMemcpyDefault) != hipSuccess) {
            (void)hipFree(*u_dev);
            return fail_hip("mesh upload");
        }
        return SF_OK;
    }

    void mesh_free(double *u_dev) override {
        if (u_dev) (void)hipFree(u_dev);
    }

    // One launch per (precision, n) variant of the batch, in order of
    // decreasing work, on the slot's stream, then the slot's event.  Each
    // (slot, variant) owns a one-node graph of its serving kernel; a
    // launch sets the node's grid and arguments and replays it.  A variant's
    // descriptors (grouped, blk_begin counted per variant) go in the kernel
    // arguments when there are at most kServeInline of them; otherwise the
    // batch's descriptors are copied once to the slot's device array.  (One
    // graph holding all 14 variants, with the unused nodes disabled per
    // batch, took about 0.26 ms of host time per launch.)
    int launch(int s, const std::vector<ServeDesc> &descs) override {
        int count[kServeVariants] = {0};
        for (const ServeDesc &d : descs) count[serve_variant(d.n, d.prec)]++;
        int first[kServeVariants];
        int acc = 0;
        for (int v = 0; v < kServeVariants; ++v) {
            first[v] = acc;
            acc += count[v];
        }
        int fill[kServeVariants] = {0};
        int64_t total[kServeVariants] = {0};
        for (const ServeDesc &d : descs) {
            const int v = serve_variant(d.n, d.prec);
            ServeDesc &slot = hdesc_[s][first[v] + fill[v]++];
            slot = d;
            slot.blk_begin = total[v];
            total[v] += d.nblk;
        }
        bool copy = false;
        int order[kServeVariants];
        int nv = 0;
        for (int v = 0; v < kServeVariants; ++v) {
            if (total[v] > 0x7fffffffLL) {
                set_error("batch too large for one launch");
                return SF_ERR_UNSUPPORTED;
            }
            if (total[v] > 0) order[nv++] = v;
            if (count[v] > kServeInline) copy = true;
        }
        std::sort(order, order + nv, [&](int a, int b) { return total[a] > total[b]; });
        if (copy && hipMemcpyAsync(ddesc_[s], hdesc_[s], sizeof(ServeDesc) * descs.size(), hipMemcpyHostToDevice,
                                   st_[s]) != hipSuccess)
            return fail_hip("descriptor copy");
        for (int k = 0; k < nv; ++k) {
            const int v = order[k];
            ServeArgs &a = args_[s][v];
            a.optab = optab_;
            a.ndesc = count[v];
            a.total = (int32_t)total[v];
            if (count[v] > kServeInline) {
                a.desc = ddesc_[s] + first[v];
            } else {
                a.desc = nullptr;
                std::memcpy(a.inl, hdesc_[s] + first[v], sizeof(ServeDesc) * count[v]);
            }
            hipKernelNodeParams p = params_[s][v];
            p.gridDim = dim3((unsigned)total[v]);  // one workgroup per block of elements
            if (hipGraphExecKernelNodeSetParams(gexec_[s][v], node_[s][v], &p) != hipSuccess)
                return fail_hip("graph node update");
            if (hipGraphLaunch(gexec_[s][v], st_[s]) != hipSuccess) return fail_hip("hipGraphLaunch");
        }
        if (hipEventRecord(ev_[s], st_[s]) != hipSuccess) return fail_hip("hipEventRecord");
        return SF_OK;
    }

    bool done(int s) override { return hipEventQuery(ev_[s]) == hipSuccess; }
    void drain(int s) override { (void)hipEventSynchronize(ev_[s]); }

private:
    int fail_hip(const char *what) {
        set_error(std::string("serving: ") + what + ": " + hipGetErrorString(hipGetLastError()));
        return SF_ERR_HIP;
    }

    int build_graph(int s, int v) {
        if (hipGraphCreate(&graph_[s][v], 0) != hipSuccess) return fail_hip("hipGraphCreate");
        std::memset(&args_[s][v], 0, sizeof(ServeArgs));
        kargs_[s][v][0] = &args_[s][v];
        hipKernelNodeParams &p = params_[s][v];
        std::memset(&p, 0, sizeof(p));
        p.func = const_cast<void *>(serve_variant_kernel(v));
        p.gridDim = dim3(1);
        p.blockDim = dim3(serve_threads(v));
        p.sharedMemBytes = 0;
        p.kernelParams = kargs_[s][v];
        p.extra = nullptr;
        if (hipGraphAddKernelNode(&node_[s][v], graph_[s][v], nullptr, 0, &p) != hipSuccess)
            return fail_hip("hipGraphAddKernelNode");
        if (hipGraphInstantiate(&gexec_[s][v], graph_[s][v], nullptr, nullptr, 0) != hipSuccess)
            return fail_hip("hipGraphInstantiate");
        return SF_OK;
    }

    int device_ = 0, maxr_ = 1;
    double *arena_ = nullptr, *optab_ = nullptr;
    hipStream_t st_[kSlots] = {};
    hipEvent_t ev_[kSlots] = {};
    ServeDesc *ddesc_[kSlots] = {}, *hdesc_[kSlots] = {};
    hipGraph_t graph_[kSlots][kServeVariants] = {};
    hipGraphExec_t gexec_[kSlots][kServeVariants] = {};
    hipGraphNode_t node_[kSlots][kServeVariants] = {};
    hipKernelNodeParams params_[kSlots][kServeVariants];
    ServeArgs args_[kSlots][kServeVariants];
    void *kargs_[kSlots][kServeVariants][1];
};

// Host-only executor: a batch completes `us_per_block` microseconds per
// block after its launch (or after the previous batch on the slot's device
// timeline, which is shared by both slots).
class SimExecutor : public Executor {
public:
    explicit SimExecutor(double us_per_block) : us_(us_per_block) {}
    int init(size_t, int) override { return SF_OK; }
    char *arena_base() override { return nullptr; }
    int mesh_upload(const double *, size_t, double **u_dev) override {
        *u_dev = nullptr;
        return SF_OK;
    }
    void mesh_free(double *) override {}
    int launch(int s, const std::vector<ServeDesc> &descs) override {
        if (fail_.load() > 0) {
            fail_--;
            set_error("simulated launch failure");
            return SF_ERR_HIP;
        }
        int64_t blocks = 0;
        for (const ServeDesc &d : descs) blocks += d.nblk;
        const auto now = Clock::now();
        const auto start = std::max(now, busy_until_);
        busy_until_ = start + std::chrono::nanoseconds((int64_t)(us_ * 1e3 * (double)blocks));
        done_at_[s] = busy_until_;
        return SF_OK;
    }
    bool done(int s) override { return Clock::now() >= done_at_[s]; }
    void drain(int s) override { std::this_thread::sleep_until(done_at_[s]); }
    int fail_launches(int count) override {
        fail_ = count;
        return SF_OK;
    }

private:
    std::atomic<int> fail_{0};
    double us_;
    Clock::time_point busy_until_{}, done_at_[kSlots]{};
};

class Server {
public:
    Server(std::unique_ptr<Executor> ex, size_t budget, int max_inflight)
        : ex_(std::move(ex)), budget_(budget), max_inflight_(max_inflight) {}

    int start() {
        int st = ex_->init(budget_, max_inflight_);
        if (st != SF_OK) return st;
        arena_.reset(budget_);
        thread_ = std::thread([this] { loop(); });
        return SF_OK;
    }

    ~Server() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        if (thread_.joinable()) thread_.join();
        for (int s = 0; s < kSlots; ++s)
            if (slot_busy_[s]) ex_->drain(s);
        for (auto &kv : meshes_) ex_->mesh_free(kv.second.u);
    }

    int register_mesh(const double *u_src, int64_t E, int n, int flux, int node_kind, int64_t *out) {
        if (!u_src || !out || E <= 0) return fail(SF_ERR_ARG, "null state or E <= 0");
        if (flux != SF_FLUX_EULER_CHANDRASHEKAR) return fail(SF_ERR_UNSUPPORTED, "serving is built for the Euler flux");
        if (node_kind != SF_NODES_GAUSS_LEGENDRE && node_kind != SF_NODES_GAUSS_LOBATTO)
            return fail(SF_ERR_ARG, "unknown node_kind");
        if (n < 2 || n > kServeMaxN) return fail(SF_ERR_UNSUPPORTED, "serving is built for 2 <= n <= 8");
        const size_t bytes = (size_t)5 * E * n * n * n * sizeof(double);
        Mesh m;
        m.E = E;
        m.n = n;
        m.node_kind = node_kind;
        m.out_bytes = align_up(bytes);
        int st = ex_->mesh_upload(u_src, bytes, &m.u);
        if (st != SF_OK) return st;
        std::lock_guard<std::mutex> lk(mu_);
        *out = next_mesh_++;
        meshes_[*out] = m;
        return SF_OK;
    }

    int unregister_mesh(int64_t id) {
        double *u = nullptr;
        {
            std::lock_guard<std::mutex> lk(mu_);
            auto it = meshes_.find(id);
            if (it == meshes_.end()) return fail(SF_ERR_NOT_FOUND, "unknown mesh");
            if (it->second.outstanding) return fail(SF_ERR_BUSY, "mesh has requests not yet released");
            u = it->second.u;
            meshes_.erase(it);
        }
        ex_->mesh_free(u);
        return SF_OK;
    }

    int submit(int64_t mesh, int prec, int64_t *ticket) {
        if (!ticket) return fail(SF_ERR_ARG, "null ticket");
        if (prec != SF_PREC_FP64 && prec != SF_PREC_FP32_SPLIT) return fail(SF_ERR_ARG, "unknown precision");
        std::lock_guard<std::mutex> lk(mu_);
        auto it = meshes_.find(mesh);
        if (it == meshes_.end()) return fail(SF_ERR_NOT_FOUND, "unknown mesh");
        if (it->second.out_bytes > budget_) return fail(SF_ERR_BUDGET, "request larger than the whole budget");
        Request r;
        r.ticket = next_ticket_++;
        r.mesh = mesh;
        r.prec = prec;
        r.bytes = it->second.out_bytes;
        r.t_submit = Clock::now();
        it->second.outstanding++;
        reqs_[r.ticket] = r;
        queue_.push_back(r.ticket);
        *ticket = r.ticket;
        cv_.notify_all();
        return SF_OK;
    }

    int poll(int64_t t) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return fail(SF_ERR_NOT_FOUND, "unknown ticket");
        return it->second.state == State::Done ? 1 : 0;
    }

    int wait(int64_t t, const double **y, double *latency) {
        std::unique_lock<std::mutex> lk(mu_);
        auto it = reqs_.find(t);
        // look the ticket up again after every wake-up: inserts may rehash
        while (it != reqs_.end() && it->second.state != State::Done && !stop_) {
            cv_.wait(lk);
            it = reqs_.find(t);
        }
        if (it == reqs_.end()) return fail(SF_ERR_NOT_FOUND, "unknown ticket");
        if (it->second.state != State::Done) return fail(SF_ERR_BUSY, "server stopping");
        if (it->second.status != SF_OK) {
            if (y) *y = nullptr;
            if (latency)
                *latency = std::chrono::duration<double>(it->second.t_done - it->second.t_submit).count();
            return fail(it->second.status, "the request's batch could not be launched");
        }
        if (y) {
            char *base = ex_->arena_base();
            *y = base ? reinterpret_cast<const double *>(base + it->second.off) : nullptr;
        }
        if (latency)
            *latency = std::chrono::duration<double>(it->second.t_done - it->second.t_submit).count();
        return SF_OK;
    }

    int release(int64_t t) {
        std::lock_guard<std::mutex> lk(mu_);
        auto it = reqs_.find(t);
        if (it == reqs_.end()) return fail(SF_ERR_NOT_FOUND, "unknown ticket");
        if (it->second.state != State::Done) return fail(SF_ERR_BUSY, "request not complete");
        arena_.release(it->second.off, it->second.bytes);
        inflight_--;
        auto m = meshes_.find(it->second.mesh);
        if (m != meshes_.end()) m->second.outstanding--;
        reqs_.erase(it);
        cv_.notify_all();
        return SF_OK;
    }

    int fail_launches(int count) { return ex_->fail_launches(count); }

    // introspection for tests: queued, admitted-or-running, budget bytes in use
    void stats(int64_t *queued, int64_t *inflight, int64_t *used) {
        std::lock_guard<std::mutex> lk(mu_);
        if (queued) *queued = (int64_t)queue_.size();
        if (inflight) *inflight = inflight_;
        if (used) *used = (int64_t)arena_.used();
    }

    // batches launched, the most requests in one batch, the most launch
    // slots running at once (continuous batching: > 1 means a batch started
    // while another was still on the device)
    void batch_stats(int64_t *batches, int64_t *max_reqs, int64_t *max_busy) {
        std::lock_guard<std::mutex> lk(mu_);
        if (batches) *batches = batches_;
        if (max_reqs) *max_reqs = max_batch_reqs_;
        if (max_busy) *max_busy = max_slots_busy_;
    }

private:
    static int fail(int st, const char *msg) {
        set_error(msg);
        return st;
    }

    // One scheduler pass under the lock: admit, launch, retire.  Returns true
    // if anything changed.
    bool step(std::unique_lock<std::mutex> &lk) {
        bool changed = false;
        // admission: FIFO, stop at the first request that does not fit
        while (!queue_.empty() && inflight_ < max_inflight_) {
            Request &r = reqs_[queue_.front()];
            size_t off;
            if (!arena_.alloc(r.bytes, off)) break;
            r.off = off;
            r.state = State::Admitted;
            pending_.push_back(r.ticket);
            queue_.pop_front();
            inflight_++;
            changed = true;
        }
        // launch everything admitted on a free slot
        if (!pending_.empty()) {
            int s = -1;
            for (int k = 0; k < kSlots; ++k)
                if (!slot_busy_[k]) { s = k; break; }
            if (s >= 0) {
                std::vector<ServeDesc> descs;
                descs.reserve(pending_.size());
                char *base = ex_->arena_base();
                for (int64_t t : pending_) {
                    Request &r = reqs_[t];
                    const Mesh &m = meshes_[r.mesh];
                    ServeDesc d{};
                    d.u = m.u;
                    d.out = base ? reinterpret_cast<double *>(base + r.off) : nullptr;
                    d.E = m.E;
                    d.n = m.n;
                    d.prec = r.prec;
                    d.node_kind = m.node_kind;
                    d.nblk = (int32_t)serve_blocks(m.n, r.prec, m.E);
                    d.gamma = 1.4;
                    descs.push_back(d);
                    r.state = State::Running;
                }
                slot_reqs_[s].swap(pending_);
                pending_.clear();
                slot_busy_[s] = true;
                batches_++;
                max_batch_reqs_ = std::max(max_batch_reqs_, (int64_t)descs.size());
                max_slots_busy_ = std::max(max_slots_busy_,
                                           (int64_t)std::count(slot_busy_, slot_busy_ + kSlots, true));
                lk.unlock();
                int st = ex_->launch(s, descs);
                lk.lock();
                if (st != SF_OK) {
                    // the batch never ran: its requests complete with the error
                    // (their output memory stays held until sf_release)
                    launch_error_ = st;
                    const auto now = Clock::now();
                    for (int64_t t : slot_reqs_[s]) {
                        auto it = reqs_.find(t);
                        if (it != reqs_.end()) {
                            it->second.state = State::Done;
                            it->second.status = st;
                            it->second.t_done = now;
                        }
                    }
                    slot_reqs_[s].clear();
                    slot_busy_[s] = false;
                }
                changed = true;
            }
        }
        // retire finished slots
        for (int s = 0; s < kSlots; ++s) {
            if (slot_busy_[s] && ex_->done(s)) {
                const auto now = Clock::now();
                for (int64_t t : slot_reqs_[s]) {
                    auto it = reqs_.find(t);
                    if (it != reqs_.end()) {
                        it->second.state = State::Done;
                        it->second.t_done = now;
                    }
                }
                slot_reqs_[s].clear();
                slot_busy_[s] = false;
                changed = true;
            }
        }
        return changed;
    }

    void loop() {
        // the completion poll below sleeps a few microseconds; the default
        // timer slack of a Linux thread (50 us) would stretch every such
        // sleep to about 55 us, and with it every request's latency
        (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
        std::unique_lock<std::mutex> lk(mu_);
        while (!stop_) {
            if (step(lk)) {
                cv_.notify_all();
                continue;
            }
            const bool busy = std::any_of(slot_busy_, slot_busy_ + kSlots, [](bool b) { return b; });
            if (busy) {
                // a batch is running: poll its completion without holding the lock
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(5));
                lk.lock();
            } else {
                cv_.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
    }

    std::unique_ptr<Executor> ex_;
    size_t budget_;
    int max_inflight_;
    Arena arena_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::thread thread_;
    bool stop_ = false;
    int launch_error_ = SF_OK;
    int64_t next_mesh_ = 1, next_ticket_ = 1;
    int inflight_ = 0;
    int64_t batches_ = 0, max_batch_reqs_ = 0, max_slots_busy_ = 0;
    std::unordered_map<int64_t, Mesh> meshes_;
    std::unordered_map<int64_t, Request> reqs_;
    std::deque<int64_t> queue_;
    std::vector<int64_t> pending_;
    std::vector<int64_t> slot_reqs_[kSlots];
    bool slot_busy_[kSlots] = {};
};

}  // namespace serve
}  // namespace sfhad

using sfhad::serve::Server;

struct sf_server {
    std::unique_ptr<Server> impl;
};

namespace {
int create(std::unique_ptr<sfhad::serve::Executor> ex, size_t budget, int max_inflight, sf_server **out) {
    if (!out) {
        sfhad::set_error("null out");
        return SF_ERR_ARG;
    }
    *out = nullptr;
    if (max_inflight < 1 || max_inflight > 1024) {
        sfhad::set_error("max_inflight must be in [1, 1024]");
        return SF_ERR_ARG;
    }
    auto srv = std::make_unique<sf_server>();
    srv->impl = std::make_unique<Server>(std::move(ex), budget, max_inflight);
    int st = srv->impl->start();
    if (st != SF_OK) return st;
    *out = srv.release();
    return SF_OK;
}
}  // namespace

extern "C" {

int sf_server_create(size_t hbm_budget_bytes, int max_inflight, sf_server **out) {
    return create(std::make_unique<sfhad::serve::HipExecutor>(), hbm_budget_bytes, max_inflight, out);
}

int sf_server_create_sim(size_t hbm_budget_bytes, int max_inflight, double us_per_block, sf_server **out) {
    if (!(us_per_block >= 0.0)) {
        sfhad::set_error("us_per_block must be >= 0");
        return SF_ERR_ARG;
    }
    return create(std::make_unique<sfhad::serve::SimExecutor>(us_per_block), hbm_budget_bytes, max_inflight, out);
}

int sf_mesh_register(sf_server *srv, const double *u_host_or_dev, int64_t E, int n, int flux_kind,
                     int node_kind, sf_mesh *out) {
    if (!srv) return SF_ERR_ARG;
    return srv->impl->register_mesh(u_host_or_dev, E, n, flux_kind, node_kind, out);
}

int sf_submit(sf_server *srv, sf_mesh mesh, int precision, sf_ticket *out) {
    if (!srv) return SF_ERR_ARG;
    return srv->impl->submit(mesh, precision, out);
}

int sf_poll(sf_server *srv, sf_ticket t) {
    if (!srv) return SF_ERR_ARG;
    return srv->impl->poll(t);
}

int sf_wait(sf_server *srv, sf_ticket t, const double **y_dev, double *latency_s) {
    if (!srv) return SF_ERR_ARG;
    return srv->impl->wait(t, y_dev, latency_s);
}

int sf_release(sf_server *srv, sf_ticket t) {
    if (!srv) return SF_ERR_ARG;
    return srv->impl->release(t);
}

int sf_mesh_unregister(sf_server *srv, sf_mesh mesh) {
    if (!srv) return SF_ERR_ARG;
    return srv->impl->unregister_mesh(mesh);
}

int sf_server_stats(sf_server *srv, int64_t *queued, int64_t *inflight, int64_t *budget_used) {
    if (!srv) return SF_ERR_ARG;
    srv->impl->stats(queued, inflight, budget_used);
    return SF_OK;
}

int sf_server_batch_stats(sf_server *srv, int64_t *batches, int64_t *max_batch_requests,
                          int64_t *max_slots_busy) {
    if (!srv) return SF_ERR_ARG;
    srv->impl->batch_stats(batches, max_batch_requests, max_slots_busy);
    return SF_OK;
}

int sf_server_sim_fail_launches(sf_server *srv, int count) {
    if (!srv || count < 0) return SF_ERR_ARG;
    const int st = srv->impl->fail_launches(count);
    if (st != SF_OK) sfhad::set_error("launch failures can only be injected into a simulated server");
    return st;
}

int sf_server_destroy(sf_server *srv) {
    if (!srv) return SF_ERR_ARG;
    delete srv;
    return SF_OK;
}

}  // extern "C"
