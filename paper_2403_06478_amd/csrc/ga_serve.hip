// ga_serve.hip -- native continuous-batching server over the C ABI of
// include/ga.h (host code only; every alignment step runs in the kernels of
// ga_kernels.hip, reached through ga_pack and ga_align_batch).
//
// Requests (one target/query pair each) arrive over time. Each lane (short
// requests, long requests) keeps a request ring in pinned, host-coherent
// memory that the packing kernel reads in place; requests are admitted when
// their bytes fit (admission by memory footprint), in groups of at most a
// batch, and until then wait in the lane's FIFO. A few execution slots per
// lane each own a context, a stream, pinned offset/length/result tables and
// device packed streams sized for the slot's capacity, and one HIP graph
// captured at that capacity (packing both sides out of the ring, aligning);
// a batch fills the tables (unused entries are empty pairs) and replays the
// graph. Slots run concurrently, so requests arriving while other batches
// are on the GPU are admitted and batched as memory and slots free up.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <chrono>
#include <deque>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ga.h"

namespace {

int64_t pad16(int64_t n) { return (n + 15) & ~int64_t(15); }

// Makes the server's device current for a call and restores the caller's.
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int device) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != device) (void)hipSetDevice(device);
    }
    ~DeviceScope() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Ring space handed out contiguously in arrival order (a request group that
// does not fit before the end starts again at 0, the skipped end counting
// as used) and released in any order; the oldest released regions are
// reclaimed once everything older is released too.
struct RingSpace {
    struct Region {
        int64_t off, size;
        bool released;
    };
    int64_t cap = 0, head = 0, used = 0;
    std::deque<Region> regions;
    uint64_t front_seq = 0;                       // sequence number of regions.front()
    std::unordered_map<int64_t, uint64_t> live;   // offset -> sequence number

    int64_t alloc(int64_t size) {
        if (size < 1) size = 1;
        if (size > cap) return -2;
        if (used == 0) head = 0;
        const int64_t tail = ((head - used) % cap + cap) % cap;
        int64_t off;
        if (used < cap && head >= tail) {
            if (cap - head >= size) {
                off = head;
            } else if (tail >= size) {
                push(head, cap - head, true);  // skip the end
                used += cap - head;
                off = 0;
            } else {
                return -1;
            }
        } else if (used < cap && tail - head >= size) {
            off = head;
        } else {
            return -1;
        }
        live[off] = front_seq + regions.size();
        push(off, size, false);
        head = (off + size) % cap;
        used += size;
        return off;
    }
    void push(int64_t off, int64_t size, bool released) { regions.push_back(Region{off, size, released}); }
    void release(int64_t off) {
        auto it = live.find(off);
        if (it == live.end()) return;
        regions[it->second - front_seq].released = true;
        live.erase(it);
        while (!regions.empty() && regions.front().released) {
            used -= regions.front().size;
            regions.pop_front();
            ++front_seq;
        }
    }
};

struct Req {
    int64_t tag;
    std::vector<uint8_t> t, q;
    int64_t off = -1, region = -1;
    double t_arrival = 0;
    int64_t bytes() const { return pad16((int64_t)t.size()) + pad16((int64_t)q.size()); }
};

struct Lane;

struct Slot {
    Lane *lane = nullptr;
    ga_context_t *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int64_t P = 0, W = 0;
    int32_t max_len = 0;
    int64_t *h_off[2] = {nullptr, nullptr};  // pinned
    int32_t *h_len[2] = {nullptr, nullptr};
    ga_result_t *h_out = nullptr;
    void *p_off[2] = {nullptr, nullptr}, *p_len[2] = {nullptr, nullptr}, *p_out = nullptr;  // their device addresses
    uint32_t *d_words[2] = {nullptr, nullptr};
    int64_t *d_woff[2] = {nullptr, nullptr};
    uint32_t *d_nmask[2] = {nullptr, nullptr};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<Req *> batch;
    bool busy = false;
};

struct Lane {
    RingSpace space;
    uint8_t *ring = nullptr;  // pinned
    void *ring_dev = nullptr;
    int64_t max_pairs = 0, max_bases = 0;
    std::unordered_map<int64_t, int64_t> refs;  // region -> requests not yet done
    std::deque<Req *> waiting, admitted;
    std::vector<Slot> slots;
};

}  // namespace

struct ga_server {
    int device = 0;
    ga_scoring_t sc{};
    int32_t w = 0, Z = 0;
    ga_server_config_t cfg{};
    Lane lanes[2];
    int64_t batches = 0;
    int64_t in_flight = 0;  // submitted, not yet finished
    int64_t max_capacity = 0;  // pairs of the largest slot
    int err = GA_OK;           // first error found while results were handed back
};

namespace {

int device_steps(ga_server *srv, Slot &s, hipStream_t st) {
    Lane &L = *s.lane;
    for (int side = 0; side < 2; ++side) {
        const int rc = ga_pack(s.ctx, (const uint8_t *)L.ring_dev, (const int64_t *)s.p_off[side],
                               (const int32_t *)s.p_len[side], s.P, s.W, s.d_words[side], s.d_woff[side],
                               s.d_nmask[side], st);
        if (rc != GA_OK) return rc;
    }
    ga_batch_t bt{};
    bt.n_pairs = s.P;
    bt.t_words_dev = s.d_words[0];
    bt.t_nwords = s.W;
    bt.q_words_dev = s.d_words[1];
    bt.q_nwords = s.W;
    bt.t_off_dev = s.d_woff[0];
    bt.q_off_dev = s.d_woff[1];
    bt.t_len_dev = (const int32_t *)s.p_len[0];
    bt.q_len_dev = (const int32_t *)s.p_len[1];
    bt.t_nmask_dev = s.d_nmask[0];
    bt.q_nmask_dev = s.d_nmask[1];
    bt.max_len = s.max_len;
    return ga_align_batch(s.ctx, &bt, &srv->sc, srv->w, srv->Z, (ga_result_t *)s.p_out, st);
}

int slot_init(ga_server *srv, Lane &L, Slot &s) {
    s.lane = &L;
    s.P = L.max_pairs;
    s.W = L.space.cap / 16 + s.P + 1;
    s.max_len = (int32_t)(L.space.cap < (1 << 20) ? L.space.cap : (1 << 20));
    int rc = ga_context_create(&s.ctx, srv->device);
    if (rc != GA_OK) return rc;
    if ((rc = ga_context_set_lanes(s.ctx, 1)) != GA_OK) return rc;
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return GA_EHIP;
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return GA_EHIP;
    for (int side = 0; side < 2; ++side) {
        if (hipHostMalloc((void **)&s.h_off[side], sizeof(int64_t) * s.P, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&s.h_len[side], sizeof(int32_t) * s.P, hipHostMallocDefault) != hipSuccess ||
            hipMalloc((void **)&s.d_words[side], sizeof(uint32_t) * s.W) != hipSuccess ||
            hipMalloc((void **)&s.d_woff[side], sizeof(int64_t) * s.P) != hipSuccess ||
            hipMalloc((void **)&s.d_nmask[side], sizeof(uint32_t) * ((s.W + 1) / 2)) != hipSuccess)
            return GA_ENOMEM;
        memset(s.h_off[side], 0, sizeof(int64_t) * s.P);  // empty pairs
        memset(s.h_len[side], 0, sizeof(int32_t) * s.P);
        if (ga_host_device_pointer(s.h_off[side], &s.p_off[side]) != GA_OK ||
            ga_host_device_pointer(s.h_len[side], &s.p_len[side]) != GA_OK)
            return GA_EHIP;
    }
    if (hipHostMalloc((void **)&s.h_out, sizeof(ga_result_t) * s.P, hipHostMallocDefault) != hipSuccess)
        return GA_ENOMEM;
    if (ga_host_device_pointer(s.h_out, &s.p_out) != GA_OK) return GA_EHIP;
    // one run on empty pairs sizes the context's workspace for the capacity
    if ((rc = device_steps(srv, s, s.stream)) != GA_OK) return rc;
    if ((rc = ga_context_check(s.ctx, s.stream)) != GA_OK) return rc;
    if (srv->cfg.graphs) {
        if (hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return GA_EHIP;
        rc = device_steps(srv, s, s.stream);
        hipGraph_t g = nullptr;
        const bool ended = hipStreamEndCapture(s.stream, &g) == hipSuccess;
        if (rc != GA_OK) return rc;
        if (!ended || !g) return GA_EHIP;
        s.graph = g;
        if (hipGraphInstantiate(&s.exec, g, nullptr, nullptr, 0) != hipSuccess) return GA_EHIP;
    }
    return GA_OK;
}

void slot_free(Slot &s) {
    if (s.stream) hipStreamSynchronize(s.stream);
    if (s.exec) hipGraphExecDestroy(s.exec);
    if (s.graph) hipGraphDestroy(s.graph);
    for (int side = 0; side < 2; ++side) {
        if (s.h_off[side]) hipHostFree(s.h_off[side]);
        if (s.h_len[side]) hipHostFree(s.h_len[side]);
        if (s.d_words[side]) hipFree(s.d_words[side]);
        if (s.d_woff[side]) hipFree(s.d_woff[side]);
        if (s.d_nmask[side]) hipFree(s.d_nmask[side]);
    }
    if (s.h_out) hipHostFree(s.h_out);
    if (s.done) hipEventDestroy(s.done);
    if (s.stream) hipStreamDestroy(s.stream);
    if (s.ctx) ga_context_destroy(s.ctx);
}

// Admit the longest prefix of the lane's waiting requests (at most a
// batch) that fits now into one region of the ring.
int64_t admit(Lane &L) {
    int64_t k = 0, total = 0;
    const int64_t free_bytes = L.space.cap - L.space.used;
    for (Req *r : L.waiting) {
        if (k >= L.max_pairs || total + r->bytes() > free_bytes) break;
        total += r->bytes();
        ++k;
    }
    int64_t off = -1;
    while (k > 0) {
        off = L.space.alloc(total);
        if (off >= 0) break;
        k /= 2;
        total = 0;
        for (int64_t i = 0; i < k; ++i) total += L.waiting[i]->bytes();
    }
    if (k == 0) return 0;
    int64_t pos = off;
    for (int64_t i = 0; i < k; ++i) {
        Req *r = L.waiting.front();
        L.waiting.pop_front();
        const int64_t nt = (int64_t)r->t.size(), nq = (int64_t)r->q.size();
        r->off = pos;
        r->region = off;
        if (nt) memcpy(L.ring + pos, r->t.data(), nt);
        if (pad16(nt) > nt) memset(L.ring + pos + nt, 0, pad16(nt) - nt);
        if (nq) memcpy(L.ring + pos + pad16(nt), r->q.data(), nq);
        if (pad16(nq) > nq) memset(L.ring + pos + pad16(nt) + nq, 0, pad16(nq) - nq);
        pos += r->bytes();
        L.admitted.push_back(r);
    }
    L.refs[off] = k;
    return k;
}

void release(Lane &L, Req *r) {
    auto it = L.refs.find(r->region);
    if (it == L.refs.end()) return;
    if (--it->second == 0) {
        L.refs.erase(it);
        L.space.release(r->region);
    }
}

int launch(ga_server *srv, Slot &s) {
    Lane &L = *s.lane;
    s.batch.clear();
    int64_t bases = 0;
    while (!L.admitted.empty() && (int64_t)s.batch.size() < s.P) {
        Req *r = L.admitted.front();
        const int64_t b = (int64_t)(r->t.size() + r->q.size());
        if (!s.batch.empty() && bases + b > L.max_bases) break;
        s.batch.push_back(r);
        L.admitted.pop_front();
        bases += b;
    }
    const int64_t n = (int64_t)s.batch.size();
    for (int64_t k = 0; k < n; ++k) {
        const Req *r = s.batch[k];
        s.h_off[0][k] = r->off;
        s.h_len[0][k] = (int32_t)r->t.size();
        s.h_off[1][k] = r->off + pad16((int64_t)r->t.size());
        s.h_len[1][k] = (int32_t)r->q.size();
    }
    for (int side = 0; side < 2; ++side) {
        memset(s.h_off[side] + n, 0, sizeof(int64_t) * (s.P - n));
        memset(s.h_len[side] + n, 0, sizeof(int32_t) * (s.P - n));
    }
    int rc = GA_OK;
    if (s.exec) {
        if (hipGraphLaunch(s.exec, s.stream) != hipSuccess) rc = GA_EHIP;
    } else {
        rc = device_steps(srv, s, s.stream);
    }
    if (rc == GA_OK && hipEventRecord(s.done, s.stream) != hipSuccess) rc = GA_EHIP;
    if (rc != GA_OK) {
        // nothing of this batch runs: its requests wait again, in order
        for (int64_t k = n - 1; k >= 0; --k) L.admitted.push_front(s.batch[k]);
        s.batch.clear();
        return rc;
    }
    s.busy = true;
    ++srv->batches;
    return GA_OK;
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

int ga_server_create(ga_server_t **out, int device, const ga_scoring_t *sc, int32_t w, int32_t Z,
                     const ga_server_config_t *cfg) {
    if (!out || !sc || !cfg) return GA_EINVAL;
    *out = nullptr;
    if (cfg->slots < 1 || cfg->long_slots < 1 || cfg->max_batch_pairs < 1 || cfg->long_batch_pairs < 1 ||
        cfg->max_batch_bases < 1 || cfg->long_batch_bases < 1 || cfg->ring_factor < 1 || cfg->long_bases < 0 ||
        !(cfg->replay_timeout_s >= 0))
        return GA_EINVAL;
    if (cfg->slots > GA_SERVER_MAX_SLOTS || cfg->long_slots > GA_SERVER_MAX_SLOTS ||
        cfg->max_batch_pairs > GA_SERVER_MAX_BATCH_PAIRS || cfg->long_batch_pairs > GA_SERVER_MAX_BATCH_PAIRS ||
        cfg->max_batch_bases > GA_SERVER_MAX_RING_BYTES / cfg->ring_factor ||
        cfg->long_batch_bases > GA_SERVER_MAX_RING_BYTES / cfg->ring_factor)
        return GA_EINVAL;
    ga_server *srv = new (std::nothrow) ga_server;
    if (!srv) return GA_ENOMEM;
    srv->device = device;
    srv->sc = *sc;
    srv->w = w;
    srv->Z = Z;
    srv->cfg = *cfg;
    srv->max_capacity = cfg->max_batch_pairs > cfg->long_batch_pairs ? cfg->max_batch_pairs : cfg->long_batch_pairs;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) {
        delete srv;
        return GA_EINVAL;
    }
    int rc = GA_OK;
    const int64_t pairs[2] = {cfg->max_batch_pairs, cfg->long_batch_pairs};
    const int64_t bases[2] = {cfg->max_batch_bases, cfg->long_batch_bases};
    const int nslots[2] = {cfg->slots, cfg->long_slots};
    for (int l = 0; l < 2 && rc == GA_OK; ++l) {
        Lane &L = srv->lanes[l];
        L.max_pairs = pairs[l];
        L.max_bases = bases[l];
        L.space.cap = pad16(cfg->ring_factor * bases[l]);
        if (hipHostMalloc((void **)&L.ring, L.space.cap, hipHostMallocDefault) != hipSuccess) {
            L.ring = nullptr;
            rc = GA_ENOMEM;
            break;
        }
        if (ga_host_device_pointer(L.ring, &L.ring_dev) != GA_OK) {
            rc = GA_EHIP;
            break;
        }
        L.slots.resize(nslots[l]);
        for (int k = 0; k < nslots[l] && rc == GA_OK; ++k) rc = slot_init(srv, L, L.slots[k]);
    }
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    if (rc != GA_OK) {
        ga_server_destroy(srv);
        return rc;
    }
    *out = srv;
    return GA_OK;
}

int ga_server_destroy(ga_server_t *srv) {
    if (!srv) return GA_EINVAL;
    DeviceScope ds(srv->device);
    for (Lane &L : srv->lanes) {
        for (Slot &s : L.slots) {
            for (Req *r : s.batch) delete r;
            s.batch.clear();
            slot_free(s);
        }
        for (Req *r : L.waiting) delete r;
        for (Req *r : L.admitted) delete r;
        if (L.ring) hipHostFree(L.ring);
    }
    delete srv;
    return GA_OK;
}

int ga_server_submit(ga_server_t *srv, int64_t tag, const uint8_t *target, int32_t n, const uint8_t *query,
                     int32_t m, double t_arrival) {
    if (!srv || n < 0 || m < 0 || (n > 0 && !target) || (m > 0 && !query)) return GA_EINVAL;
    const int l = (int64_t)n + m > srv->cfg.long_bases ? 1 : 0;
    Lane &L = srv->lanes[l];
    if (pad16(n) + pad16(m) > L.space.cap || n > L.slots[0].max_len || m > L.slots[0].max_len)
        return GA_EUNSUPPORTED;
    Req *r = new (std::nothrow) Req;
    if (!r) return GA_ENOMEM;
    r->tag = tag;
    r->t.assign(target, target + n);
    r->q.assign(query, query + m);
    r->t_arrival = t_arrival < 0 ? now_s() : t_arrival;
    L.waiting.push_back(r);
    ++srv->in_flight;
    return GA_OK;
}

int ga_server_poll(ga_server_t *srv, int64_t *tags, ga_result_t *results, double *t_done, int max_done) {
    if (!srv || max_done < 0 || (max_done > 0 && (!tags || !results))) return GA_EINVAL;
    // a batch is handed back whole: a buffer smaller than a slot's capacity
    // could leave that slot's results uncollected for ever
    if (max_done > 0 && max_done < srv->max_capacity) return GA_EINVAL;
    DeviceScope ds(srv->device);
    int nd = 0;
    auto latch = [srv](int code) {
        if (srv->err == GA_OK) srv->err = code;
    };
    for (Lane &L : srv->lanes) {
        for (Slot &s : L.slots) {
            if (!s.busy || (int64_t)(max_done - nd) < (int64_t)s.batch.size()) continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                latch(GA_EHIP);  // its results are not known to be complete: left in the slot
                continue;
            }
            // pairs outside the declared bounds got the sentinel result;
            // the rest of the batch is valid and is handed back
            const int crc = ga_context_check(s.ctx, s.stream);
            if (crc != GA_OK) latch(crc);
            const double t = now_s();
            for (size_t k = 0; k < s.batch.size(); ++k) {
                Req *r = s.batch[k];
                tags[nd] = r->tag;
                results[nd] = s.h_out[k];
                if (t_done) t_done[nd] = t;
                ++nd;
                release(L, r);
                delete r;
                --srv->in_flight;
            }
            s.batch.clear();
            s.busy = false;
        }
    }
    for (Lane &L : srv->lanes) {
        while (!L.waiting.empty() && admit(L) > 0) {
        }
        for (Slot &s : L.slots) {
            if (L.admitted.empty()) break;
            if (!s.busy) {
                const int lrc = launch(srv, s);
                if (lrc != GA_OK) {
                    latch(lrc);
                    break;
                }
            }
        }
    }
    if (nd > 0) return nd;
    const int e = srv->err;
    srv->err = GA_OK;
    return e;
}

int64_t ga_server_pending(const ga_server_t *srv) { return srv ? srv->in_flight : -1; }

int64_t ga_server_batches(const ga_server_t *srv) { return srv ? srv->batches : -1; }

int ga_server_replay(ga_server_t *srv, const uint8_t *t_ascii, const int64_t *t_off, const int32_t *t_len,
                     const uint8_t *q_ascii, const int64_t *q_off, const int32_t *q_len, const double *arrival_s,
                     int64_t n, ga_result_t *results, double *latency_s, double *wall_s) {
    if (!srv || n < 0 || !results || !latency_s || (n > 0 && (!t_ascii || !t_off || !t_len || !q_ascii ||
                                                                !q_off || !q_len || !arrival_s)))
        return GA_EINVAL;
    const double t0 = now_s();
    int64_t next = 0, finished = 0;
    // room for every slot's batch at once (ga_server_create bounds both)
    const int64_t cap64 = srv->cfg.slots * (int64_t)srv->cfg.max_batch_pairs +
                          srv->cfg.long_slots * (int64_t)srv->cfg.long_batch_pairs;
    const int cap = (int)cap64;
    std::vector<int64_t> tags(cap);
    std::vector<ga_result_t> res(cap);
    std::vector<double> td(cap);
    const double timeout = srv->cfg.replay_timeout_s > 0 ? srv->cfg.replay_timeout_s : GA_SERVER_REPLAY_TIMEOUT_S;
    double progress = now_s();  // the last submission or collection
    while (finished < n) {
        const double now = now_s() - t0;
        if (srv->in_flight > 0 && now_s() - progress > timeout) return GA_EHIP;  // no batch finished in time
        while (next < n && arrival_s[next] <= now) {
            const int rc = ga_server_submit(srv, next, t_ascii + t_off[next], t_len[next], q_ascii + q_off[next],
                                            q_len[next], t0 + arrival_s[next]);
            if (rc != GA_OK) return rc;
            ++next;
            progress = now_s();
        }
        const int nd = ga_server_poll(srv, tags.data(), res.data(), td.data(), cap);
        if (nd < 0) return nd;
        if (nd > 0) progress = now_s();
        for (int k = 0; k < nd; ++k) {
            const int64_t i = tags[k];
            results[i] = res[k];
            latency_s[i] = td[k] - (t0 + arrival_s[i]);
            ++finished;
        }
        if (nd == 0) {
            if (srv->in_flight == 0 && next < n) {
                // nothing in flight: wait for the next arrival (bounded)
                const double dt = arrival_s[next] - (now_s() - t0);
                if (dt > 0) std::this_thread::sleep_for(std::chrono::duration<double>(dt < 0.002 ? dt : 0.002));
            } else {
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        }
    }
    if (wall_s) *wall_s = now_s() - t0;
    return GA_OK;
}

}  // extern "C"
