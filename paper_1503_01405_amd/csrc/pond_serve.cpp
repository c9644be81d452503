// Real-time serving of many concurrent streams on one device.
//
// Each admitted stream owns a plan (its overlap tail and fold accumulators
// stay on the device between blocks), a non-blocking HIP stream, and a
// small ring of block slots (device staging for the int8 block, device and
// pinned host space for the profiles it completes).  A submitted block is
// dispatched at once when its stream has a free slot -- host-to-device copy,
// dedispersion + fold, profile copy back, completion event, all on the
// stream's HIP stream -- and otherwise waits in the stream's queue until
// poll() sees a slot free up.  Blocks of different streams therefore run
// concurrently on the device, each stream's blocks in order.  Streams are
// admitted against a device-memory budget; a stream that does not fit now
// waits, with the blocks submitted to it, in a first-come queue and is
// admitted by a later open, poll or close once closed streams have returned
// enough memory to the budget.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstring>
#include <deque>
#include <new>
#include <thread>
#include <vector>

#include "../../include/pond.h"
#include "pond_internal.hpp"

namespace {

constexpr int kSlots = 2;  // blocks of one stream on the device at once

double now_us() {
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

struct Block {
    int64_t ticket = 0;
    const int8_t* iq = nullptr;
    int64_t nsamp = 0;
    double t_submit = 0;
    int slot = -1;
    int64_t nprof = 0;
    int32_t status = POND_OK;
};

enum State { kWaiting = POND_STREAM_WAITING, kOpen = POND_STREAM_OPEN, kClosed = POND_STREAM_CLOSED };

struct Stream {
    pond_stream_desc d{};
    State state = kClosed;
    pond_plan* plan = nullptr;
    hipStream_t hs = nullptr;
    int64_t bytes = 0;            // charged against the budget
    int64_t max_prof = 0;         // profiles one block can complete
    int8_t* staging[kSlots] = {};
    float* dprof[kSlots] = {};
    float* hprof[kSlots] = {};    // pinned
    hipEvent_t ev_start[kSlots] = {};
    hipEvent_t ev_done[kSlots] = {};
    bool slot_busy[kSlots] = {};
    int next_slot = 0;
    std::deque<Block> pending;
    std::deque<Block> inflight;
    std::vector<float> profiles;  // completed, not yet taken (host)
    int32_t error = POND_OK;      // sticky stream error
};

int64_t profiles_per_block(const pond_stream_desc& d) {
    // A call appending n samples completes fewer than n + nfft outputs
    // (the blocks it finishes may have started in earlier calls), which
    // end at most (n + nfft) / S + 1 sub-integrations.
    return d.subint_nsamp > 0 ? (d.max_block_nsamp + d.nfft) / d.subint_nsamp + 2 : 1;
}

// Sub-integrations one call of at most max_block_nsamp samples can touch:
// the accumulator ring is created that large, so it never grows while the
// stream is served.
int64_t acc_slots_for(const pond_stream_desc& d) { return profiles_per_block(d) + 1; }

int64_t stream_bytes(const pond_stream_desc& d, int32_t max_batch) {
    const int64_t per_slot = d.max_block_nsamp * 2 + profiles_per_block(d) * (int64_t)d.nbins * 4;
    return pond::plan_footprint(d.nfft, d.nbins, d.precision, max_batch, acc_slots_for(d)) + kSlots * per_slot;
}

}  // namespace

struct pond_server {
    int device = 0;
    int64_t budget = 0;
    int64_t used = 0;
    int32_t max_streams = 0;
    int64_t next_ticket = 0;
    std::vector<Stream> streams;
    std::deque<int32_t> waiting;        // streams not yet admitted, first come first
    std::deque<pond_completion> ready;  // completions observed outside poll()
};

namespace {

void release_stream(Stream& s) {
    if (s.hs) (void)hipStreamSynchronize(s.hs);
    pond_plan_destroy(s.plan);
    s.plan = nullptr;
    for (int k = 0; k < kSlots; ++k) {
        if (s.staging[k]) (void)hipFree(s.staging[k]);
        if (s.dprof[k]) (void)hipFree(s.dprof[k]);
        if (s.hprof[k]) (void)hipHostFree(s.hprof[k]);
        if (s.ev_start[k]) (void)hipEventDestroy(s.ev_start[k]);
        if (s.ev_done[k]) (void)hipEventDestroy(s.ev_done[k]);
        s.staging[k] = nullptr;
        s.dprof[k] = nullptr;
        s.hprof[k] = nullptr;
        s.ev_start[k] = nullptr;
        s.ev_done[k] = nullptr;
    }
    if (s.hs) (void)hipStreamDestroy(s.hs);
    s.hs = nullptr;
    s.state = kClosed;
}

// Queue one block on its stream's HIP stream (the stream has a free slot).
void dispatch(Stream& s, Block& b) {
    int k = s.next_slot;
    s.next_slot = (k + 1) % kSlots;
    s.slot_busy[k] = true;
    b.slot = k;
    b.status = POND_OK;
    if (s.error != POND_OK) {
        b.status = s.error;
        return;
    }
    hipError_t e = hipEventRecord(s.ev_start[k], s.hs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s.staging[k], b.iq, (size_t)b.nsamp * 2, hipMemcpyHostToDevice, s.hs);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s.error = b.status = POND_EDEVICE;
        return;
    }
    const int64_t r = pond_dedisperse_fold(s.plan, s.staging[k], b.nsamp, s.d.subint_nsamp, s.dprof[k], s.max_prof,
                                           s.hs);
    if (r < 0) {
        s.error = b.status = (int32_t)r;
        return;
    }
    b.nprof = r;
    if (r > 0)
        e = hipMemcpyAsync(s.hprof[k], s.dprof[k], (size_t)r * s.d.nbins * 4, hipMemcpyDeviceToHost, s.hs);
    if (e == hipSuccess) e = hipEventRecord(s.ev_done[k], s.hs);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        s.error = b.status = POND_EDEVICE;
    }
}

// Move completed blocks of one stream, in order, to `out` and refill its
// slots from the queue.
void progress(pond_server* srv, int32_t id, std::deque<pond_completion>& out) {
    Stream& s = srv->streams[(size_t)id];
    while (!s.inflight.empty()) {
        Block& b = s.inflight.front();
        if (b.status == POND_OK) {
            const hipError_t q = hipEventQuery(s.ev_done[b.slot]);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) {
                (void)hipGetLastError();
                s.error = b.status = POND_EDEVICE;
            }
        }
        pond_completion c{};
        c.ticket = b.ticket;
        c.stream = id;
        c.status = b.status;
        c.n_profiles = b.status == POND_OK ? b.nprof : 0;
        c.latency_us = now_us() - b.t_submit;
        c.device_us = 0;
        if (b.status == POND_OK) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s.ev_start[b.slot], s.ev_done[b.slot]) == hipSuccess) c.device_us = ms * 1e3;
            const float* h = s.hprof[b.slot];
            s.profiles.insert(s.profiles.end(), h, h + (size_t)b.nprof * s.d.nbins);
        }
        s.slot_busy[b.slot] = false;
        out.push_back(c);
        s.inflight.pop_front();
    }
    while (!s.pending.empty() && (int)s.inflight.size() < kSlots) {
        Block b = s.pending.front();
        s.pending.pop_front();
        dispatch(s, b);
        s.inflight.push_back(b);
    }
}

bool valid_desc(const pond_stream_desc* d) {
    if (!d) return false;
    if (d->max_block_nsamp <= 0 || d->subint_nsamp < 0) return false;
    if (d->nbins < 1 || d->nbins > 65536) return false;
    if (d->nfft <= 0 || (d->nfft & (d->nfft - 1))) return false;
    return true;
}

// Blocks per launch for a stream that must fit `room` bytes: the default if
// it fits, else halved down to 1; 0 if even one block per launch does not.
int32_t fitting_batch(const pond_stream_desc& d, int64_t room) {
    int32_t mb = pond::plan_max_batch(d.nfft, d.precision, 0);
    while (mb > 1 && stream_bytes(d, mb) > room) mb /= 2;
    return stream_bytes(d, mb) <= room ? mb : 0;
}

// Create the stream's plan, HIP stream and slots (on the server's device).
int32_t admit(pond_server* srv, Stream& s, int32_t mb) {
    const pond_stream_desc& d = s.d;
    s.max_prof = profiles_per_block(d);
    s.plan = pond::plan_create_slots(d.f0_mhz, d.bw_mhz, d.dm, d.nfft, d.nbins, d.period_s, d.precision, mb,
                                     acc_slots_for(d));
    if (!s.plan) return pond_create_status() != POND_OK ? pond_create_status() : POND_EDEVICE;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess) e = x;
    };
    chk(hipStreamCreateWithFlags(&s.hs, hipStreamNonBlocking));
    for (int k = 0; k < kSlots; ++k) {
        chk(hipMalloc(reinterpret_cast<void**>(&s.staging[k]), (size_t)d.max_block_nsamp * 2));
        chk(hipMalloc(reinterpret_cast<void**>(&s.dprof[k]), (size_t)s.max_prof * d.nbins * 4));
        chk(hipHostMalloc(reinterpret_cast<void**>(&s.hprof[k]), (size_t)s.max_prof * d.nbins * 4,
                          hipHostMallocDefault));
        chk(hipEventCreate(&s.ev_start[k]));
        chk(hipEventCreate(&s.ev_done[k]));
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release_stream(s);
        return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? POND_ENOMEM : POND_EDEVICE;
    }
    s.state = kOpen;
    s.bytes = stream_bytes(d, mb);
    srv->used += s.bytes;
    return POND_OK;
}

// Complete every queued block of a stream with `status` (never run).
void drop_pending(Stream& s, int32_t id, int32_t status, std::deque<pond_completion>& out) {
    while (!s.pending.empty()) {
        pond_completion c{};
        c.ticket = s.pending.front().ticket;
        c.stream = id;
        c.status = status;
        c.latency_us = now_us() - s.pending.front().t_submit;
        out.push_back(c);
        s.pending.pop_front();
    }
}

// Admit waiting streams, first come first, while the first one fits the
// budget left.  Each admission is reported as a completion with ticket
// POND_TICKET_ADMITTED (status: POND_OK, or the error that ended the
// stream); an admitted stream's queued blocks are dispatched at once.
void admit_waiting(pond_server* srv, std::deque<pond_completion>& out) {
    while (!srv->waiting.empty()) {
        const int32_t id = srv->waiting.front();
        Stream& s = srv->streams[(size_t)id];
        const int32_t mb = fitting_batch(s.d, srv->budget - srv->used);
        if (mb == 0) break;
        srv->waiting.pop_front();
        const int32_t rc = admit(srv, s, mb);
        pond_completion c{};
        c.ticket = POND_TICKET_ADMITTED;
        c.stream = id;
        c.status = rc;
        out.push_back(c);
        if (rc != POND_OK) {
            s.state = kClosed;
            s.error = rc;
            drop_pending(s, id, rc, out);
            continue;
        }
        progress(srv, id, out);
    }
}

struct DeviceScope {
    int cur = -1, dev;
    explicit DeviceScope(int d) : dev(d) {
        (void)hipGetDevice(&cur);
        if (cur != dev) (void)hipSetDevice(dev);
    }
    ~DeviceScope() {
        if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    }
};

}  // namespace

extern "C" {

pond_server* pond_server_create(int64_t hbm_budget_bytes, int32_t max_streams) {
    if (hbm_budget_bytes <= 0 || max_streams < 1 || max_streams > 1024) return nullptr;
    pond_server* srv = new (std::nothrow) pond_server();
    if (!srv) return nullptr;
    if (hipGetDevice(&srv->device) != hipSuccess) {
        delete srv;
        return nullptr;
    }
    srv->budget = hbm_budget_bytes;
    srv->max_streams = max_streams;
    return srv;
}

int64_t pond_server_stream_bytes(const pond_stream_desc* d) {
    if (!valid_desc(d)) return POND_EINVAL;
    return stream_bytes(*d, 0);
}

int32_t pond_server_open(pond_server* srv, const pond_stream_desc* d) {
    if (!srv || !valid_desc(d)) return POND_EINVAL;
    int32_t live = 0;
    for (const Stream& s : srv->streams) live += s.state != kClosed ? 1 : 0;
    if (live >= srv->max_streams) return POND_EBUSY;
    // A stream that would not fit even an empty server is refused; one that
    // only needs others to close first waits for admission.
    if (fitting_batch(*d, srv->budget) == 0) return POND_EBUSY;
    DeviceScope ds(srv->device);
    Stream s;
    s.d = *d;
    s.state = kWaiting;
    srv->streams.push_back(std::move(s));
    const int32_t id = (int32_t)srv->streams.size() - 1;
    srv->waiting.push_back(id);
    admit_waiting(srv, srv->ready);
    const Stream& t = srv->streams[(size_t)id];
    if (t.state == kClosed) {
        // admission failed here: the admission completion of this stream
        // is not reported, the error is returned instead
        for (auto it = srv->ready.begin(); it != srv->ready.end(); ++it)
            if (it->stream == id && it->ticket == POND_TICKET_ADMITTED) {
                srv->ready.erase(it);
                break;
            }
        return t.error;
    }
    if (t.state == kOpen) {
        // admitted at once: no admission completion either
        for (auto it = srv->ready.begin(); it != srv->ready.end(); ++it)
            if (it->stream == id && it->ticket == POND_TICKET_ADMITTED) {
                srv->ready.erase(it);
                break;
            }
    }
    return id;
}

int32_t pond_server_stream_state(const pond_server* srv, int32_t id) {
    if (!srv || id < 0 || id >= (int32_t)srv->streams.size()) return POND_EINVAL;
    return (int32_t)srv->streams[(size_t)id].state;
}

int64_t pond_server_submit(pond_server* srv, int32_t id, const int8_t* host_iq, int64_t nsamp) {
    if (!srv || id < 0 || id >= (int32_t)srv->streams.size()) return POND_EINVAL;
    Stream& s = srv->streams[(size_t)id];
    if (s.state == kClosed || !host_iq || nsamp <= 0 || nsamp > s.d.max_block_nsamp) return POND_EINVAL;
    if (s.error != POND_OK) return s.error;
    Block b;
    b.ticket = srv->next_ticket++;
    b.iq = host_iq;
    b.nsamp = nsamp;
    b.t_submit = now_us();
    s.pending.push_back(b);
    if (s.state == kOpen) {
        DeviceScope ds(srv->device);
        progress(srv, id, srv->ready);
    }
    return b.ticket;
}

int32_t pond_server_poll(pond_server* srv, pond_completion* out, int32_t max_out, int32_t wait) {
    if (!srv || max_out < 0 || (max_out > 0 && !out)) return POND_EINVAL;
    {
        DeviceScope ds(srv->device);
        for (;;) {
            admit_waiting(srv, srv->ready);
            bool busy = false;
            for (int32_t id = 0; id < (int32_t)srv->streams.size(); ++id) {
                Stream& s = srv->streams[(size_t)id];
                if (s.state != kOpen) continue;
                progress(srv, id, srv->ready);
                busy = busy || !s.inflight.empty();
            }
            if (!srv->ready.empty() || !wait || !busy) break;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
    }
    int32_t n = 0;
    while (n < max_out && !srv->ready.empty()) {
        out[n++] = srv->ready.front();
        srv->ready.pop_front();
    }
    return n;
}

int64_t pond_server_take_profiles(pond_server* srv, int32_t id, float* host_out, int64_t max_profiles) {
    if (!srv || id < 0 || id >= (int32_t)srv->streams.size() || max_profiles < 0) return POND_EINVAL;
    Stream& s = srv->streams[(size_t)id];
    const int64_t have = (int64_t)(s.profiles.size() / (size_t)s.d.nbins);
    const int64_t n = have < max_profiles ? have : max_profiles;
    if (n > 0) {
        if (!host_out) return POND_EINVAL;
        std::memcpy(host_out, s.profiles.data(), (size_t)n * s.d.nbins * 4);
        s.profiles.erase(s.profiles.begin(), s.profiles.begin() + (size_t)n * s.d.nbins);
    }
    return n;
}

int32_t pond_server_close(pond_server* srv, int32_t id) {
    if (!srv || id < 0 || id >= (int32_t)srv->streams.size()) return POND_EINVAL;
    Stream& s = srv->streams[(size_t)id];
    if (s.state == kClosed) return POND_EINVAL;
    DeviceScope ds(srv->device);
    if (s.state == kWaiting) {
        // never admitted: its queued blocks are cancelled
        for (auto it = srv->waiting.begin(); it != srv->waiting.end(); ++it)
            if (*it == id) {
                srv->waiting.erase(it);
                break;
            }
        drop_pending(s, id, POND_ECANCELED, srv->ready);
        s.state = kClosed;
        admit_waiting(srv, srv->ready);
        return POND_OK;
    }
    // Drain the stream's queue, then end the stream (the open
    // sub-integration becomes the last profile).
    while (!s.pending.empty() || !s.inflight.empty()) {
        progress(srv, id, srv->ready);
        if (!s.inflight.empty() && s.inflight.front().status == POND_OK)
            (void)hipEventSynchronize(s.ev_done[s.inflight.front().slot]);
    }
    int32_t rc = s.error;
    if (rc == POND_OK) {
        const int64_t r = pond_dedisperse_fold(s.plan, nullptr, 0, s.d.subint_nsamp, s.dprof[0], 1, s.hs);
        hipError_t e = hipSuccess;
        if (r > 0) e = hipMemcpyAsync(s.hprof[0], s.dprof[0], (size_t)s.d.nbins * 4, hipMemcpyDeviceToHost, s.hs);
        if (e == hipSuccess) e = hipStreamSynchronize(s.hs);
        if (r < 0) {
            rc = (int32_t)r;
        } else if (e != hipSuccess) {
            (void)hipGetLastError();
            rc = POND_EDEVICE;
        } else if (r > 0) {
            s.profiles.insert(s.profiles.end(), s.hprof[0], s.hprof[0] + s.d.nbins);
        }
    }
    release_stream(s);
    srv->used -= s.bytes;
    s.bytes = 0;
    // the memory returned may admit waiting streams
    admit_waiting(srv, srv->ready);
    return rc;
}

int32_t pond_server_query(const pond_server* srv, int64_t* used_bytes, int64_t* budget_bytes, int32_t* open_streams,
                          int64_t* queued_blocks) {
    if (!srv) return POND_EINVAL;
    int32_t live = 0;
    int64_t q = 0;
    for (const Stream& s : srv->streams) {
        live += s.state == kOpen ? 1 : 0;
        q += (int64_t)(s.pending.size() + s.inflight.size());
    }
    if (used_bytes) *used_bytes = srv->used;
    if (budget_bytes) *budget_bytes = srv->budget;
    if (open_streams) *open_streams = live;
    if (queued_blocks) *queued_blocks = q;
    return POND_OK;
}

void pond_server_destroy(pond_server* srv) {
    if (!srv) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != srv->device) (void)hipSetDevice(srv->device);
    for (Stream& s : srv->streams)
        if (s.state == kOpen) release_stream(s);
    if (cur >= 0 && cur != srv->device) (void)hipSetDevice(cur);
    delete srv;
}

}  // extern "C"
