// smap_serve.hpp -- the serving loop behind simplex_serve_run (host code).
//
// A real-time replay of a request stream of automaton-step jobs on one GPU:
// jobs arrive at their arrival times, are admitted in arrival order when
// their output fits the memory budget (an arena the caller owns, managed
// here by a first-fit allocator), and are launched either one by one with
// the H map (the sequential baseline) or in continuous batches: whenever
// fewer than `max_inflight` batches are running, every admitted job that
// has not been launched goes out as one batched launch (or as one
// persistent work-queue launch), alternating between two streams so that
// consecutive batches overlap on the device.
// Completion times come from device events, so a job's latency is the
// time from its arrival to the end of the launch that ran it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <chrono>
#include <deque>
#include <map>
#include <vector>

#include "../../include/simplexmap.h"

namespace smap {

// First-fit allocator over [0, size) in 256-byte units; adjacent free
// ranges are merged on release.
class Arena {
public:
    explicit Arena(uint64_t size) { if (size >= 256) free_[0] = size & ~uint64_t(255); }
    static uint64_t round(uint64_t b) { return (b + 255) & ~uint64_t(255); }
    bool alloc(uint64_t bytes, uint64_t *off)
    {
        const uint64_t need = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= need) {
                *off = it->first;
                const uint64_t rest = it->second - need, at = it->first + need;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        uint64_t size = round(bytes);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += size;
                return;
            }
        }
        free_[off] = size;
    }

private:
    std::map<uint64_t, uint64_t> free_;
};

inline uint64_t serve_box_bytes(const simplex_serve_job &J)
{
    uint64_t b = 1;
    for (int k = 0; k < J.m; ++k) b *= (uint64_t)(J.n + 1);
    return b;
}

// The replay.  Arguments are validated by the caller (the C entry point).
inline int serve_run(const simplex_serve_job *jobs, int32_t njobs, uint8_t *arena, uint64_t arena_bytes,
                     int32_t mode, int32_t max_inflight, int32_t keep_outputs, simplex_serve_record *rec,
                     uint8_t *warm)
{
    using clock = std::chrono::steady_clock;
    struct Flight {
        hipEvent_t ev;
        std::vector<int32_t> jobs;
    };
    const int nstreams = mode == SMAP_SERVE_SEQUENTIAL ? 1 : 2;
    // a group of admitted jobs goes out as one launch group of the mode
    auto launch_group = [&](const simplex_job *b, int32_t cnt, hipStream_t s) {
        return mode == SMAP_SERVE_PERSISTENT ? simplex_queue_launch(b, cnt, 0, s) : simplex_batch_launch(b, cnt, s);
    };
    hipStream_t streams[2] = {nullptr, nullptr};
    std::vector<hipEvent_t> pool;  // events ready for reuse
    std::deque<Flight> flying[2];  // per stream, in issue order
    hipEvent_t ev0 = nullptr;
    int status = SMAP_OK;

    auto get_event = [&](hipEvent_t *e) -> bool {
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
            return true;
        }
        return hipEventCreate(e) == hipSuccess;
    };
    for (int i = 0; i < nstreams; ++i) {
        if (hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking) != hipSuccess) status = SMAP_EHIP;
    }
    if (status == SMAP_OK && hipEventCreate(&ev0) != hipSuccess) status = SMAP_EHIP;
    // Warm-up before the clock: the first launches in a process (and on a
    // new stream) load kernel and copy code and set up device queues, which
    // takes milliseconds.  One tiny step of each class runs on every stream,
    // on the library's own zeroed 16^3 boxes (`warm`, 2 x 8 KiB; the output
    // box stays all zero: a zero field stays zero).
    if (status == SMAP_OK && warm) {
        const simplex_job wj[2] = {{2, SMAP_OP_CA2, 15, warm, warm + 8192},
                                   {3, SMAP_OP_CA3, 15, warm, warm + 8192}};
        for (int i = 0; i < nstreams && status == SMAP_OK; ++i) {
            for (const simplex_job &w : wj) {
                const int rc = mode == SMAP_SERVE_SEQUENTIAL
                                   ? simplex_map_launch(w.m, w.n, 0, 0, w.op, w.buf_in, w.buf_out, streams[i])
                                   : launch_group(&w, 1, streams[i]);
                if (rc != SMAP_OK) status = rc;
            }
            if (status == SMAP_OK && hipStreamSynchronize(streams[i]) != hipSuccess) status = SMAP_EHIP;
        }
    }
    for (int i = 0; i < nstreams && status == SMAP_OK; ++i) {
        if (hipEventRecord(ev0, streams[i]) != hipSuccess || hipEventSynchronize(ev0) != hipSuccess)
            status = SMAP_EHIP;
    }
    // The run's clock starts at t0; the start event ev0 is placed at the
    // midpoint of its record-and-wait on that clock.
    const auto t0 = clock::now();
    if (status == SMAP_OK && hipEventRecord(ev0, streams[0]) != hipSuccess) status = SMAP_EHIP;
    if (status == SMAP_OK && hipEventSynchronize(ev0) != hipSuccess) status = SMAP_EHIP;
    auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };
    const double ev0_s = 0.5 * now_s();

    Arena heap(arena_bytes);
    std::deque<int32_t> waiting;    // arrived, not admitted
    std::vector<int32_t> admitted;  // admitted, not launched
    std::vector<simplex_job> batch;
    int32_t next = 0, done = 0, batch_id = 0, inflight = 0;

    while (status == SMAP_OK && done < njobs) {
        const double now = now_s();
        bool progress = false;
        while (next < njobs && jobs[next].arrival_s <= now) waiting.push_back(next++);
        // completions: the front of each stream's queue finishes first
        for (int si = 0; si < nstreams && status == SMAP_OK; ++si) {
            while (!flying[si].empty()) {
                Flight &f = flying[si].front();
                const hipError_t q = hipEventQuery(f.ev);
                if (q == hipErrorNotReady) break;
                if (q != hipSuccess) { status = SMAP_EHIP; break; }
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev0, f.ev) != hipSuccess) { status = SMAP_EHIP; break; }
                const double seen = now_s();
                for (int32_t j : f.jobs) {
                    rec[j].done_s = ev0_s + ms * 1e-3;
                    rec[j].release_s = seen;
                    if (!keep_outputs) heap.release(rec[j].out_offset, serve_box_bytes(jobs[j]));
                }
                done += (int32_t)f.jobs.size();
                --inflight;
                pool.push_back(f.ev);
                flying[si].pop_front();
                progress = true;
            }
        }
        if (status != SMAP_OK) break;
        // admission in arrival order (after this pass's releases)
        while (!waiting.empty()) {
            const int32_t j = waiting.front();
            uint64_t off = 0;
            if (!heap.alloc(serve_box_bytes(jobs[j]), &off)) break;
            rec[j].admit_s = now_s();
            rec[j].out_offset = off;
            admitted.push_back(j);
            waiting.pop_front();
            progress = true;
        }
        // launches
        if (mode == SMAP_SERVE_SEQUENTIAL) {
            for (int32_t j : admitted) {
                const simplex_serve_job &J = jobs[j];
                Flight f;
                if (!get_event(&f.ev)) { status = SMAP_EHIP; break; }
                rec[j].launch_s = now_s();
                rec[j].batch = batch_id++;
                const int rc = simplex_map_launch(J.m, J.n, 0, 0, J.op, J.buf_in, arena + rec[j].out_offset,
                                                  streams[0]);
                rec[j].status = rc;
                if (rc != SMAP_OK) { status = rc; pool.push_back(f.ev); break; }
                if (hipEventRecord(f.ev, streams[0]) != hipSuccess) { status = SMAP_EHIP; break; }
                f.jobs.push_back(j);
                flying[0].push_back(std::move(f));
                ++inflight;
            }
            admitted.clear();
        } else if (!admitted.empty() && inflight < max_inflight) {
            const int si = batch_id % 2;
            batch.clear();
            const double t = now_s();
            for (int32_t j : admitted) {
                const simplex_serve_job &J = jobs[j];
                batch.push_back({J.m, J.op, J.n, J.buf_in, arena + rec[j].out_offset});
                rec[j].launch_s = t;
                rec[j].batch = batch_id;
            }
            Flight f;
            if (!get_event(&f.ev)) { status = SMAP_EHIP; break; }
            const int rc = launch_group(batch.data(), (int32_t)batch.size(), streams[si]);
            for (int32_t j : admitted) rec[j].status = rc;
            if (rc != SMAP_OK) { status = rc; pool.push_back(f.ev); break; }
            if (hipEventRecord(f.ev, streams[si]) != hipSuccess) { status = SMAP_EHIP; break; }
            f.jobs = admitted;
            flying[si].push_back(std::move(f));
            ++inflight;
            ++batch_id;
            admitted.clear();
            progress = true;
        }
        (void)progress;  // the loop spins: arrivals are timed against the host clock
    }
    // drain whatever is still enqueued, then release the run's resources
    for (int i = 0; i < nstreams; ++i) {
        if (streams[i]) (void)hipStreamSynchronize(streams[i]);
    }
    for (int si = 0; si < nstreams; ++si)
        for (Flight &f : flying[si]) pool.push_back(f.ev);
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    if (ev0) (void)hipEventDestroy(ev0);
    for (int i = 0; i < nstreams; ++i) {
        if (streams[i]) (void)hipStreamDestroy(streams[i]);
    }
    return status;
}

}  // namespace smap
