// Serving loop: continuous batching of partition requests on one GPU.
//
// submit() copies a request's graph into server memory and queues it.  Each
// of `slots` worker threads owns a HIP stream; an idle worker takes the
// longest prefix of the queue that the packing rule allows (plan_batch: the
// footprint fits the free budget, at most max_batch graphs, the union's node
// count within int32), partitions it as one batch and stores each request's
// result.  Requests that arrive while batches run are taken
// by the next idle worker, so their work overlaps on the device with the
// batches already running.  A batch uses graph-local ids in every hash and
// order, so a request's result does not depend on the requests it shares a
// batch with; it equals sclap_partition on that graph alone.
#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "driver.hpp"

namespace sclap {
namespace {

struct Request {
    uint64_t id = 0;
    int32_t n = 0;
    int32_t k = 1;
    double eps = 0;
    uint64_t seed = 0;
    std::vector<int64_t> xadj;
    std::vector<int32_t> adj, ew, vw;  // ew / vw empty: unit weights
    int64_t footprint = 0;
    // result
    bool done = false;
    int status = 0;
    std::string err;
    std::vector<int32_t> part;
    int64_t cut = 0;
    std::vector<int64_t> bw;
    double t_submit = 0, t_start = 0, t_done = 0;
    int32_t batch_size = 0;
};

using RequestPtr = std::shared_ptr<Request>;

// Device bytes a request may need while its batch runs (an upper bound): the
// graph (8 B per node for offsets, 4 for weights; 4 + 4 per slot), coarser
// levels of at most the same size, about 48 B per node of label propagation
// state (labels, weights, results, selection keys, boundary keys) and at most
// about 28 B per slot of contraction buffers (kept coarse ids, row entries,
// bucket staging).
int64_t footprint_of(int64_t n, int64_t S) { return 64 * n + 64 * S + (4LL << 20); }

}  // namespace

// How many of the queued requests (in queue order) one batch takes: the
// longest prefix, at most max_batch, whose summed footprint fits the free
// budget (the first request alone is always taken when nothing else runs)
// and whose summed node count stays within int32 (batch ids are int32).
// (Keeping the sizes in one batch within a factor 8 of each other was
// measured: it moved the p99 requests from small graphs batched behind a
// large one to the large graphs themselves but left p99 unchanged and raised
// p50, so sizes are mixed.)  `slots` is part of the interface for such rules.
int32_t plan_batch(const int64_t* nodes, const int64_t* slots, const int64_t* footprint, int32_t count,
                   int64_t free_budget, int32_t max_batch, bool idle) {
    (void)slots;
    int32_t taken = 0;
    int64_t bytes = 0, ntot = 0;
    for (int32_t i = 0; i < count && taken < max_batch; ++i) {
        if (taken == 0) {
            if (!idle && footprint[i] > free_budget) break;
        } else {
            if (bytes + footprint[i] > free_budget) break;
            if (ntot + nodes[i] > INT32_MAX) break;
        }
        bytes += footprint[i];
        ntot += nodes[i];
        ++taken;
    }
    return taken;
}

namespace {

}  // namespace
}  // namespace sclap

struct sclap_server {
    int32_t device = 0;
    int64_t budget = 0;
    int32_t max_batch = 64;
    int32_t max_queue = 1 << 16;
    sclap::Opts opts;
    sclap::Clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<sclap::RequestPtr> queue;
    std::unordered_map<uint64_t, sclap::RequestPtr> reqs;
    int64_t in_flight = 0;
    uint64_t next_id = 1;
    bool stop = false;
    std::vector<std::thread> workers;
};

namespace sclap {
namespace {

double now_ms(const sclap_server* sv) { return ms_since(sv->t0); }

void finish_error(const RequestPtr& r, int status, const std::string& msg) {
    r->status = status;
    r->err = msg;
}

// Partitions the requests as one batch on stream s; fills their results.
void run_batch(sclap_server* sv, std::vector<RequestPtr>& batch, hipStream_t s) {
    const int32_t G = static_cast<int32_t>(batch.size());
    std::vector<int32_t> nb(G + 1, 0), k(G);
    std::vector<double> eps(G);
    std::vector<uint64_t> seed(G);
    std::vector<int64_t> sb(G + 1, 0);
    bool any_ew = false, any_vw = false;
    for (int32_t i = 0; i < G; ++i) {
        const Request& r = *batch[i];
        nb[i + 1] = nb[i] + r.n;
        sb[i + 1] = sb[i] + (r.n > 0 ? r.xadj[r.n] : 0);
        k[i] = r.k;
        eps[i] = r.eps;
        seed[i] = r.seed;
        any_ew |= !r.ew.empty();
        any_vw |= !r.vw.empty();
    }
    const int32_t n = nb[G];
    const int64_t S = sb[G];
    std::vector<int64_t> xadj(static_cast<size_t>(n) + 1, 0);
    std::vector<int32_t> adj(static_cast<size_t>(std::max<int64_t>(S, 1)));
    std::vector<int32_t> ew(any_ew ? static_cast<size_t>(std::max<int64_t>(S, 1)) : 0);
    std::vector<int32_t> vw(any_vw ? static_cast<size_t>(std::max(n, 1)) : 0);
    for (int32_t i = 0; i < G; ++i) {
        const Request& r = *batch[i];
        for (int32_t v = 0; v < r.n; ++v) xadj[nb[i] + v + 1] = r.xadj[v + 1] + sb[i];
        const int64_t Si = sb[i + 1] - sb[i];
        for (int64_t j = 0; j < Si; ++j) adj[sb[i] + j] = r.adj[j] + nb[i];
        if (any_ew)
            for (int64_t j = 0; j < Si; ++j) ew[sb[i] + j] = r.ew.empty() ? 1 : r.ew[j];
        if (any_vw)
            for (int32_t v = 0; v < r.n; ++v) vw[nb[i] + v] = r.vw.empty() ? 1 : r.vw[v];
    }
    OwnedDevGraph d;
    d.n = n;
    d.S = S;
    d.xadj.alloc(static_cast<size_t>(n) + 1, s);
    d.adj.alloc(std::max<int64_t>(S, 1), s);
    HIPCHK(hipMemcpyAsync(d.xadj.get(), xadj.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (S > 0) HIPCHK(hipMemcpyAsync(d.adj.get(), adj.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (any_ew && S > 0) {
        d.ew.alloc(S, s);
        HIPCHK(hipMemcpyAsync(d.ew.get(), ew.data(), S * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    if (any_vw && n > 0) {
        d.vw.alloc(n, s);
        HIPCHK(hipMemcpyAsync(d.vw.get(), vw.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    DBuf<int32_t> part(std::max(n, 1), s);
    std::vector<int64_t> cut(G);
    std::vector<int64_t> bw(static_cast<size_t>(std::max(1, std::accumulate(k.begin(), k.end(), 0))));
    sclap_batch_stats st{};
    partition_batch_impl(d.view(), G, nb.data(), k.data(), eps.data(), seed.data(), sv->opts, part.get(), cut.data(),
                         bw.data(), &st, s);
    std::vector<int32_t> hpart(std::max(n, 1));
    if (n > 0) HIPCHK(hipMemcpyAsync(hpart.data(), part.get(), n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int64_t kb = 0;
    for (int32_t i = 0; i < G; ++i) {
        Request& r = *batch[i];
        r.part.assign(hpart.begin() + nb[i], hpart.begin() + nb[i + 1]);
        r.cut = cut[i];
        r.bw.assign(bw.begin() + kb, bw.begin() + kb + r.k);
        kb += r.k;
        // every node lies in some block, so the block weights sum to c(V)
        const int64_t Lmax = lmax_of(std::accumulate(r.bw.begin(), r.bw.end(), int64_t{0}), r.k, r.eps);
        r.status = SCLAP_OK;
        for (int64_t w : r.bw)
            if (w > Lmax) r.status = SCLAP_WARN_IMBALANCED;
        r.batch_size = G;
    }
}

void worker(sclap_server* sv) {
    hipStream_t s = nullptr;
    bool ok = hipSetDevice(sv->device) == hipSuccess && hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    while (true) {
        std::vector<RequestPtr> batch;
        int64_t bytes = 0;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_work.wait(lk, [&] {
                if (sv->stop) return true;
                if (sv->queue.empty()) return false;
                return sv->in_flight == 0 || sv->in_flight + sv->queue.front()->footprint <= sv->budget;
            });
            if (sv->stop) break;
            const int32_t look = static_cast<int32_t>(std::min<size_t>(sv->queue.size(), sv->max_batch));
            std::vector<int64_t> qn(look), qs(look), qf(look);
            for (int32_t i = 0; i < look; ++i) {
                const Request& r = *sv->queue[i];
                qn[i] = r.n;
                qs[i] = r.n > 0 ? r.xadj[r.n] : 0;
                qf[i] = r.footprint;
            }
            const int32_t take = plan_batch(qn.data(), qs.data(), qf.data(), look, sv->budget - sv->in_flight,
                                            sv->max_batch, sv->in_flight == 0);
            for (int32_t i = 0; i < take; ++i) {
                bytes += sv->queue.front()->footprint;
                batch.push_back(sv->queue.front());
                sv->queue.pop_front();
            }
            sv->in_flight += bytes;
            const double t = now_ms(sv);
            for (auto& r : batch) r->t_start = t;
        }
        if (!ok) {
            for (auto& r : batch) finish_error(r, SCLAP_ERR_HIP, "server stream creation failed");
        } else {
            try {
                try {
                    run_batch(sv, batch, s);
                } catch (const std::exception& e) {
                    // host failures (staging allocation, sizes) are retried alone too
                    if (dynamic_cast<const Error*>(&e)) throw;
                    throw Error(SCLAP_ERR_HIP, e.what());
                }
            } catch (const Error& e) {
                // attribute the failure: run every request of the batch alone
                if (batch.size() == 1) {
                    finish_error(batch[0], e.status, e.what());
                } else {
                    for (auto& r : batch) {
                        std::vector<RequestPtr> one{r};
                        try {
                            run_batch(sv, one, s);
                        } catch (const Error& e1) {
                            finish_error(r, e1.status, e1.what());
                        } catch (const std::exception& e1) {
                            finish_error(r, SCLAP_ERR_HIP, e1.what());
                        }
                    }
                }
            }
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->in_flight -= bytes;
            const double t = now_ms(sv);
            for (auto& r : batch) {
                r->t_done = t;
                r->done = true;
                r->xadj = {};
                r->adj = {};
                r->ew = {};
                r->vw = {};
            }
        }
        sv->cv_done.notify_all();
        sv->cv_work.notify_all();
    }
    if (s) {
        release_cached(s, false);  // this worker's cached blocks go back to the pool
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
}

}  // namespace

sclap_server* server_create(int32_t device, int64_t hbm_budget, int32_t slots, int32_t max_batch,
                            const sclap_options* opt) {
    int count = 0;
    HIPCHK(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) fail(SCLAP_ERR_INVALID, "no such device");
    if (slots < 1 || slots > 16) fail(SCLAP_ERR_INVALID, "slots must be in 1..16");
    if (max_batch < 1) fail(SCLAP_ERR_INVALID, "max_batch must be >= 1");
    auto sv = std::make_unique<sclap_server>();
    sv->device = device;
    sv->opts = resolve(opt);
    sv->opts.color_override = nullptr;
    sv->max_batch = max_batch;
    if (hbm_budget <= 0) {
        int prev = 0;
        HIPCHK(hipGetDevice(&prev));
        HIPCHK(hipSetDevice(device));
        size_t fr = 0, tot = 0;
        HIPCHK(hipMemGetInfo(&fr, &tot));
        HIPCHK(hipSetDevice(prev));
        hbm_budget = static_cast<int64_t>(fr / 10 * 8);
    }
    sv->budget = hbm_budget;
    sv->t0 = Clock::now();
    sclap_server* raw = sv.get();
    for (int32_t i = 0; i < slots; ++i) sv->workers.emplace_back(worker, raw);
    return sv.release();
}

uint64_t server_submit(sclap_server* sv, const sclap_graph* g, int32_t k, double eps, uint64_t seed) {
    if (!sv) fail(SCLAP_ERR_INVALID, "server is NULL");
    if (!g) fail(SCLAP_ERR_INVALID, "graph is NULL");
    check_k_eps(k, eps);
    if (g->n < 0) fail(SCLAP_ERR_INVALID, "n < 0");
    auto r = std::make_shared<Request>();
    r->n = g->n;
    r->k = k;
    r->eps = eps;
    r->seed = seed;
    if (g->n > 0) {
        if (!g->xadj) fail(SCLAP_ERR_INVALID, "xadj is NULL");
        const int64_t S = g->xadj[g->n];
        if (g->xadj[0] != 0 || S < 0) fail(SCLAP_ERR_INVALID, "bad xadj");
        if (S > 0 && !g->adjncy) fail(SCLAP_ERR_INVALID, "adjncy is NULL");
        r->xadj.assign(g->xadj, g->xadj + g->n + 1);
        r->adj.assign(g->adjncy, g->adjncy + S);
        for (int32_t v = 0; v < g->n; ++v)
            if (r->xadj[v + 1] < r->xadj[v]) fail(SCLAP_ERR_INVALID, "xadj must be non-decreasing");
        for (int64_t j = 0; j < S; ++j)
            if (r->adj[j] < 0 || r->adj[j] >= g->n) fail(SCLAP_ERR_INVALID, "neighbour id out of range");
        if (g->adjwgt) r->ew.assign(g->adjwgt, g->adjwgt + S);
        if (g->vwgt) r->vw.assign(g->vwgt, g->vwgt + g->n);
    } else {
        r->xadj.assign(1, 0);
    }
    r->footprint = footprint_of(r->n, r->xadj.back());
    std::lock_guard<std::mutex> lk(sv->mu);
    if (r->footprint > sv->budget) fail(SCLAP_ERR_NO_MEMORY, "request exceeds the server's device memory budget");
    if (static_cast<int32_t>(sv->queue.size()) >= sv->max_queue) fail(SCLAP_ERR_BUSY, "server queue is full");
    r->id = sv->next_id++;
    r->t_submit = now_ms(sv);
    sv->reqs[r->id] = r;
    sv->queue.push_back(r);
    sv->cv_work.notify_one();
    return r->id;
}

// Copies a finished request's outputs; returns its status.  *done = 0 and no
// output is written while it still runs.
int server_poll(sclap_server* sv, uint64_t id, int32_t timeout_ms, int32_t* done, int32_t* part, int64_t* cut,
                int64_t* block_w, sclap_request_info* info) {
    if (!sv) fail(SCLAP_ERR_INVALID, "server is NULL");
    if (!done) fail(SCLAP_ERR_INVALID, "done is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(id);
    if (it == sv->reqs.end()) fail(SCLAP_ERR_INVALID, "unknown request id");
    RequestPtr r = it->second;
    if (!r->done && timeout_ms != 0) {
        auto pred = [&] { return r->done; };
        if (timeout_ms < 0) sv->cv_done.wait(lk, pred);
        else sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
    }
    *done = r->done ? 1 : 0;
    if (!r->done) return SCLAP_OK;
    sv->reqs.erase(it);
    lk.unlock();
    if (info) {
        info->submit_ms = r->t_submit;
        info->start_ms = r->t_start;
        info->done_ms = r->t_done;
        info->batch_size = r->batch_size;
    }
    if (r->status < 0) fail(r->status, r->err);
    if (part && r->n > 0) std::memcpy(part, r->part.data(), r->n * sizeof(int32_t));
    if (cut) *cut = r->cut;
    if (block_w) std::memcpy(block_w, r->bw.data(), r->k * sizeof(int64_t));
    return r->status;
}

void server_destroy(sclap_server* sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_work.notify_all();
    for (auto& t : sv->workers) t.join();
    delete sv;
}

}  // namespace sclap
