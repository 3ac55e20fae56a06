// Streaming compressor (paper, Streaming): a distributor cuts the incoming
// bytes into fixed-size chunks; once a group of `lanes` chunks is full it is
// compressed into a shard (a complete .boa container) by one of `workers`
// host threads, while the caller keeps filling the next group.  Each worker
// compresses on its own HIP stream, so the host-to-device copy of one group
// overlaps the kernels of another on the GPU; at most `workers` groups wait
// for a worker, after which push() blocks (back-pressure).  Shards are handed
// out in input order.
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "boa_internal.h"

namespace {
struct Shard {
    int rc = BOA_OK;
    std::string err;
    uint8_t* data = nullptr;
    uint64_t len = 0;
};
}  // namespace

struct boa_stream {
    const boa_model* m = nullptr;
    boa_run_opts o{};
    uint64_t chunk = 0;
    uint32_t lanes = 0, workers = 0;
    std::vector<uint8_t> cur;                                   // the group being filled
    uint64_t submitted = 0, returned = 0;                       // shard sequence numbers
    bool finished = false, stopping = false;
    std::deque<std::pair<uint64_t, std::vector<uint8_t>>> work; // full groups waiting for a worker
    std::map<uint64_t, Shard> done;                             // compressed, not yet handed out
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_space;
    std::vector<std::thread> threads;

    uint64_t group_bytes() const { return chunk * lanes; }

    void worker() {
        for (;;) {
            std::pair<uint64_t, std::vector<uint8_t>> job;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] { return stopping || !work.empty(); });
                if (work.empty()) return;                       // stopping and drained
                job = std::move(work.front());
                work.pop_front();
                cv_space.notify_all();
            }
            const std::vector<uint8_t>& g = job.second;
            const uint64_t n = (g.size() + chunk - 1) / chunk;
            std::vector<uint64_t> lens(n, chunk);
            if (n) lens[n - 1] = g.size() - (n - 1) * chunk;
            Shard sh;
            sh.rc = boa_compress(m, g.data(), lens.data(), n, &o, &sh.data, &sh.len);
            if (sh.rc != BOA_OK) sh.err = boa_last_error();
            {
                std::lock_guard<std::mutex> lk(mu);
                done[job.first] = sh;
            }
            cv_done.notify_all();
        }
    }

    // hand the filled group to the workers (blocks while `workers` groups wait)
    void submit() {
        std::unique_lock<std::mutex> lk(mu);
        cv_space.wait(lk, [&] { return work.size() < workers; });
        work.emplace_back(submitted++, std::move(cur));
        cur = std::vector<uint8_t>();
        cur.reserve(group_bytes());
        cv_work.notify_one();
    }
};

extern "C" int boa_stream_open(const boa_model* m, uint64_t chunk_len, uint32_t lanes, uint32_t workers,
                               const boa_run_opts* opts, boa_stream** out) {
    if (!m || !out) return boa::report_error(BOA_E_ARG, "null argument");
    if (chunk_len < 1 || lanes < 1 || workers < 1 || workers > 8)
        return boa::report_error(BOA_E_ARG, "chunk_len and lanes must be >= 1, workers in [1, 8]");
    if (chunk_len > (1ULL << 32) || (uint64_t)lanes * chunk_len > (1ULL << 36))
        return boa::report_error(BOA_E_ARG, "group of lanes x chunk_len too large");
    boa_stream* st = new boa_stream;
    st->m = m;
    if (opts) st->o = *opts;
    st->chunk = chunk_len;
    st->lanes = lanes;
    st->workers = workers;
    st->cur.reserve(st->group_bytes());
    for (uint32_t i = 0; i < workers; ++i) st->threads.emplace_back([st] { st->worker(); });
    *out = st;
    return BOA_OK;
}

extern "C" int boa_stream_push(boa_stream* st, const uint8_t* h_data, uint64_t n) {
    if (!st || (n && !h_data)) return boa::report_error(BOA_E_ARG, "null argument");
    if (st->finished) return boa::report_error(BOA_E_ARG, "push after finish");
    while (n) {
        const uint64_t room = st->group_bytes() - st->cur.size();
        const uint64_t k = n < room ? n : room;
        st->cur.insert(st->cur.end(), h_data, h_data + k);
        h_data += k;
        n -= k;
        if (st->cur.size() == st->group_bytes()) st->submit();
    }
    return BOA_OK;
}

extern "C" int boa_stream_finish(boa_stream* st) {
    if (!st) return boa::report_error(BOA_E_ARG, "null argument");
    if (st->finished) return BOA_OK;
    if (!st->cur.empty()) st->submit();
    std::lock_guard<std::mutex> lk(st->mu);
    st->finished = true;
    st->cv_done.notify_all();
    return BOA_OK;
}

extern "C" int boa_stream_next_shard(boa_stream* st, int wait, uint8_t** out, uint64_t* out_len) {
    if (!st || !out || !out_len) return boa::report_error(BOA_E_ARG, "null argument");
    *out = nullptr;
    *out_len = 0;
    std::unique_lock<std::mutex> lk(st->mu);
    for (;;) {
        auto it = st->done.find(st->returned);
        if (it != st->done.end()) {
            Shard sh = it->second;
            st->done.erase(it);
            ++st->returned;
            lk.unlock();
            if (sh.rc != BOA_OK) {
                std::free(sh.data);
                return boa::report_error(sh.rc, "shard " + std::to_string(st->returned - 1) + ": " + sh.err);
            }
            *out = sh.data;
            *out_len = sh.len;
            return BOA_OK;
        }
        if (!wait || st->returned == st->submitted) return BOA_OK;   // none ready / none in flight
        st->cv_done.wait(lk);
    }
}

extern "C" void boa_stream_close(boa_stream* st) {
    if (!st) return;
    {
        std::lock_guard<std::mutex> lk(st->mu);
        st->stopping = true;
        st->work.clear();                       // groups no worker has started are dropped
    }
    st->cv_work.notify_all();
    st->cv_space.notify_all();
    for (auto& t : st->threads) t.join();
    for (auto& kv : st->done) std::free(kv.second.data);
    delete st;
}
