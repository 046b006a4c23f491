// C ABI (include/sclap.h): argument checks and host/device staging around the
// gfx950 kernels and the multilevel drivers.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <climits>
#include <exception>
#include <thread>
#include <cmath>
#include <cstring>
#include <deque>
#include <mutex>
#include <queue>
#include <string>
#include <utility>
#include <vector>

#include "driver.hpp"
#include "profile.hpp"

namespace sclap {

thread_local std::string t_err;

void fail(int status, const std::string& msg) { throw Error(status, msg); }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
    if (e == hipSuccess) return;
    (void)hipGetLastError();
    const int st = e == hipErrorOutOfMemory ? SCLAP_ERR_NO_MEMORY : SCLAP_ERR_HIP;
    throw Error(st, std::string(what) + ": " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")");
}

// ------------------------------------------------------------ memory pool



namespace {

hipStream_t as_stream(void* p) { return reinterpret_cast<hipStream_t>(p); }

template <typename F>
int guarded(F&& f) {
    try {
        t_err.clear();
        return f();
    } catch (const Error& e) {
        t_err = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        t_err = "host allocation failed";
        return SCLAP_ERR_NO_MEMORY;
    } catch (const std::exception& e) {
        t_err = e.what();
        return SCLAP_ERR_HIP;
    }
}

// ------------------------------------------------ host <-> device staging

struct Staged {
    OwnedDevGraph own;
    DevGraph g;
};

Staged upload(const sclap_graph* h, hipStream_t s) {
    if (!h) fail(SCLAP_ERR_INVALID, "graph is NULL");
    if (h->n < 0) fail(SCLAP_ERR_INVALID, "n < 0");
    Staged st;
    const int32_t n = h->n;
    st.own.n = n;
    if (n > 0 && !h->xadj) fail(SCLAP_ERR_INVALID, "xadj is NULL");
    const int64_t S = n > 0 ? h->xadj[n] : 0;
    if (S < 0) fail(SCLAP_ERR_INVALID, "xadj[n] < 0");
    if (S > 0 && !h->adjncy) fail(SCLAP_ERR_INVALID, "adjncy is NULL");
    st.own.S = S;
    st.own.xadj.alloc(static_cast<size_t>(n) + 1, s);
    if (n > 0) HIPCHK(hipMemcpyAsync(st.own.xadj.get(), h->xadj, (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    else fill_i64(st.own.xadj.get(), 0, 1, s);
    if (S > 0) {
        st.own.adj.alloc(S, s);
        HIPCHK(hipMemcpyAsync(st.own.adj.get(), h->adjncy, S * sizeof(int32_t), hipMemcpyHostToDevice, s));
        if (h->adjwgt) {
            st.own.ew.alloc(S, s);
            HIPCHK(hipMemcpyAsync(st.own.ew.get(), h->adjwgt, S * sizeof(int32_t), hipMemcpyHostToDevice, s));
        }
    }
    if (n > 0 && h->vwgt) {
        st.own.vw.alloc(n, s);
        HIPCHK(hipMemcpyAsync(st.own.vw.get(), h->vwgt, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    st.g = st.own.view();
    return st;
}

template <typename T>
DBuf<T> upload_array(const T* h, int64_t count, hipStream_t s) {
    DBuf<T> d(std::max<int64_t>(count, 1), s);
    if (count > 0) HIPCHK(hipMemcpyAsync(d.get(), h, count * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

template <typename T>
void download(T* h, const T* d, int64_t count, hipStream_t s) {
    if (count > 0) HIPCHK(hipMemcpyAsync(h, d, count * sizeof(T), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
}

// ------------------------------------------------------ single operations

int cluster_impl(const DevGraph& g, int64_t U, int32_t rounds, uint64_t seed, int32_t level, const Opts& o,
                 const int32_t* color_dev, int32_t* labels, int32_t* rounds_run, hipStream_t s,
                 const int32_t* block = nullptr) {
    if (rounds < 0) fail(SCLAP_ERR_INVALID, "rounds < 0");
    if (U < 0) fail(SCLAP_ERR_INVALID, "U < 0");
    if (g.n > 0 && !labels) fail(SCLAP_ERR_INVALID, "labels is NULL");
    int64_t cV = 0, cmax = 0;
    check_graph(g, o.validate != 0, &cV, &cmax, s);
    if (color_dev && !all_in_range(color_dev, g.n, 0, o.nsub, s))
        fail(SCLAP_ERR_INVALID, "color_override value outside [0, subrounds)");
    DBuf<int32_t> w(std::max(g.n, 1), s);
    iota_u32(reinterpret_cast<uint32_t*>(labels), g.n, s);
    label_weights(g, labels, w.get(), g.n, s);
    OwnedDevGraph inside;
    DevGraph gc = g;
    if (block) {
        within_blocks(g, block, inside, s);
        gc = inside.view();
        gc.vw = g.vw;
    }
    DBuf<int32_t> dcol;
    if (o.degree_order && !color_dev && g.n > 0) {
        dcol.alloc(g.n, s);
        degree_colors(gc, 1, nullptr, nullptr, nullptr, o.nsub, dcol.get(), s);
        color_dev = dcol.get();
    }
    const LPResult r = run_lp(gc, kCluster, level, seed, o.nsub, rounds, U, labels, w.get(), g.n, color_dev, o.tune, s);
    HIPCHK(hipStreamSynchronize(s));
    if (rounds_run) *rounds_run = r.rounds_run;
    return SCLAP_OK;
}

int refine_impl(const DevGraph& g, int32_t k, int64_t Lmax, int32_t rounds, uint64_t seed, int32_t level,
                const Opts& o, const int32_t* color_dev, int32_t* part, int32_t* rounds_run, hipStream_t s) {
    if (k < 1) fail(SCLAP_ERR_INVALID, "k must be >= 1");
    if (rounds < 0) fail(SCLAP_ERR_INVALID, "rounds < 0");
    if (g.n > 0 && !part) fail(SCLAP_ERR_INVALID, "part is NULL");
    int64_t cV = 0, cmax = 0;
    check_graph(g, o.validate != 0, &cV, &cmax, s);
    if (!all_in_range(part, g.n, 0, k, s)) fail(SCLAP_ERR_INVALID, "part value outside [0, k)");
    if (color_dev && !all_in_range(color_dev, g.n, 0, o.nsub, s))
        fail(SCLAP_ERR_INVALID, "color_override value outside [0, subrounds)");
    DBuf<int32_t> w(k, s);
    label_weights(g, part, w.get(), k, s);
    const LPResult r = run_lp(g, kRefine, level, seed, o.nsub, rounds, Lmax, part, w.get(), k, color_dev, o.tune, s);
    HIPCHK(hipStreamSynchronize(s));
    if (rounds_run) *rounds_run = r.rounds_run;
    return SCLAP_OK;
}

}  // namespace
}  // namespace sclap

using namespace sclap;

// =================================================================== C ABI

extern "C" {

int sclap_default_options(sclap_options* opt) {
    if (!opt) return SCLAP_ERR_INVALID;
    std::memset(opt, 0, sizeof(*opt));
    opt->coarsen_rounds = 10;
    opt->refine_rounds = 10;
    opt->subrounds = 4;
    opt->cluster_divisor = 18;
    opt->coarsest_nodes = 10000;
    opt->max_levels = SCLAP_MAX_LEVELS;
    opt->validate = 1;
    opt->vcycles = 1;
    return SCLAP_OK;
}

const char* sclap_last_error(void) { return t_err.c_str(); }

int sclap_trim_memory(void) {
    return guarded([&] {
        release_cached(nullptr, true);
        HIPCHK(hipDeviceSynchronize());
        return SCLAP_OK;
    });
}

int64_t sclap_lmax(int64_t cV, int32_t k, double eps) {
    if (k < 1) return -1;
    return lmax_of(cV, k, eps);
}

int sclap_validate_dev(const sclap_graph* g, void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        const DevGraph d = dev_view(g, s);
        int64_t cV, cmax;
        const int st = validate_graph(d, &cV, &cmax, s);
        if (st != 0) t_err = "graph validation failed";
        return st;
    });
}

int sclap_validate(const sclap_graph* g) {
    return guarded([&]() -> int {
        if (!g || g->n < 0) fail(SCLAP_ERR_INVALID, "bad graph");
        const int32_t n = g->n;
        if (n == 0) return SCLAP_OK;
        if (!g->xadj || g->xadj[0] != 0) fail(SCLAP_ERR_INVALID, "xadj must start at 0");
        for (int32_t v = 0; v < n; ++v)
            if (g->xadj[v + 1] < g->xadj[v]) fail(SCLAP_ERR_INVALID, "xadj not monotone");
        const int64_t S = g->xadj[n];
        if (S > 0 && !g->adjncy) fail(SCLAP_ERR_INVALID, "adjncy is NULL");
        int64_t cV = 0, ws = 0;
        std::vector<std::pair<uint64_t, int32_t>> fwd(S), bwd(S);
        for (int32_t v = 0; v < n; ++v) {
            const int32_t c = g->vwgt ? g->vwgt[v] : 1;
            if (c < 0) fail(SCLAP_ERR_INVALID, "negative node weight");
            cV += c;
            for (int64_t i = g->xadj[v]; i < g->xadj[v + 1]; ++i) {
                const int32_t u = g->adjncy[i];
                const int32_t w = g->adjwgt ? g->adjwgt[i] : 1;
                if (u < 0 || u >= n || u == v) fail(SCLAP_ERR_INVALID, "neighbour id out of range or self-loop");
                if (w < 1) fail(SCLAP_ERR_INVALID, "edge weight < 1");
                ws += w;
                fwd[i] = {(static_cast<uint64_t>(v) << 32) | static_cast<uint32_t>(u), w};
                bwd[i] = {(static_cast<uint64_t>(u) << 32) | static_cast<uint32_t>(v), w};
            }
        }
        if (cV > 2147483647LL || ws / 2 > 2147483647LL) fail(SCLAP_ERR_OVERFLOW, "weight total exceeds 2^31-1");
        std::sort(fwd.begin(), fwd.end());
        std::sort(bwd.begin(), bwd.end());
        if (fwd != bwd) fail(SCLAP_ERR_NOT_SYMMETRIC, "graph is not symmetric");
        return SCLAP_OK;
    });
}

int sclap_cluster_dev(const sclap_graph* g, int64_t U, int32_t rounds, uint64_t seed, int32_t level,
                      const sclap_options* opt, int32_t* labels, int32_t* rounds_run, void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        const Opts o = resolve(opt);
        const DevGraph d = dev_view(g, s);
        return cluster_impl(d, U, rounds, seed, level, o, o.color_override, labels, rounds_run, s);
    });
}

int sclap_cluster(const sclap_graph* g, int64_t U, int32_t rounds, uint64_t seed, int32_t level,
                  const sclap_options* opt, int32_t* labels, int32_t* rounds_run) {
    return guarded([&] {
        hipStream_t s = nullptr;
        const Opts o = resolve(opt);
        Staged st = upload(g, s);
        DBuf<int32_t> col;
        if (o.color_override) col = upload_array(o.color_override, g->n, s);
        DBuf<int32_t> lab(std::max(g->n, 1), s);
        const int r = cluster_impl(st.g, U, rounds, seed, level, o, o.color_override ? col.get() : nullptr,
                                   lab.get(), rounds_run, s);
        download(labels, lab.get(), g->n, s);
        return r;
    });
}

int sclap_cluster_within_dev(const sclap_graph* g, const int32_t* block, int64_t U, int32_t rounds,
                             uint64_t seed, int32_t level, const sclap_options* opt, int32_t* labels,
                             int32_t* rounds_run, void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        const Opts o = resolve(opt);
        const DevGraph d = dev_view(g, s);
        if (d.n > 0 && !block) fail(SCLAP_ERR_INVALID, "block is NULL");
        return cluster_impl(d, U, rounds, seed, level, o, o.color_override, labels, rounds_run, s, block);
    });
}

int sclap_cluster_within(const sclap_graph* g, const int32_t* block, int64_t U, int32_t rounds, uint64_t seed,
                         int32_t level, const sclap_options* opt, int32_t* labels, int32_t* rounds_run) {
    return guarded([&] {
        hipStream_t s = nullptr;
        const Opts o = resolve(opt);
        Staged st = upload(g, s);
        if (g->n > 0 && !block) fail(SCLAP_ERR_INVALID, "block is NULL");
        DBuf<int32_t> col, blk = upload_array(block, g->n, s);
        if (o.color_override) col = upload_array(o.color_override, g->n, s);
        DBuf<int32_t> lab(std::max(g->n, 1), s);
        const int r = cluster_impl(st.g, U, rounds, seed, level, o, o.color_override ? col.get() : nullptr,
                                   lab.get(), rounds_run, s, blk.get());
        download(labels, lab.get(), g->n, s);
        return r;
    });
}

int sclap_refine_dev(const sclap_graph* g, int32_t k, int64_t Lmax, int32_t rounds, uint64_t seed, int32_t level,
                     const sclap_options* opt, int32_t* part, int32_t* rounds_run, void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        const Opts o = resolve(opt);
        const DevGraph d = dev_view(g, s);
        return refine_impl(d, k, Lmax, rounds, seed, level, o, o.color_override, part, rounds_run, s);
    });
}

int sclap_refine(const sclap_graph* g, int32_t k, int64_t Lmax, int32_t rounds, uint64_t seed, int32_t level,
                 const sclap_options* opt, int32_t* part, int32_t* rounds_run) {
    return guarded([&] {
        hipStream_t s = nullptr;
        const Opts o = resolve(opt);
        Staged st = upload(g, s);
        if (g->n > 0 && !part) fail(SCLAP_ERR_INVALID, "part is NULL");
        DBuf<int32_t> col;
        if (o.color_override) col = upload_array(o.color_override, g->n, s);
        DBuf<int32_t> p = upload_array(part, g->n, s);
        const int r = refine_impl(st.g, k, Lmax, rounds, seed, level, o, o.color_override ? col.get() : nullptr,
                                  p.get(), rounds_run, s);
        download(part, p.get(), g->n, s);
        return r;
    });
}

int sclap_contract_dev(const sclap_graph* g, const int32_t* labels, int32_t* C, sclap_graph_owned* coarse,
                       void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        if (!coarse) fail(SCLAP_ERR_INVALID, "coarse is NULL");
        const DevGraph d = dev_view(g, s);
        if (d.n > 0 && (!labels || !C)) fail(SCLAP_ERR_INVALID, "labels / C is NULL");
        if (!all_in_range(labels, d.n, 0, std::max(d.n, 1), s)) fail(SCLAP_ERR_INVALID, "label outside [0, n)");
        OwnedDevGraph cg;
        contract(d, labels, C, cg, s);
        HIPCHK(hipStreamSynchronize(s));
        coarse->n = cg.n;
        coarse->S = cg.S;
        coarse->xadj = cg.xadj.p;
        coarse->adjncy = cg.adj.p;
        coarse->adjwgt = cg.ew.p;
        coarse->vwgt = cg.vw.p;
        coarse->on_device = 1;
        cg.xadj.p = nullptr;
        cg.adj.p = nullptr;
        cg.ew.p = nullptr;
        cg.vw.p = nullptr;
        return SCLAP_OK;
    });
}

int sclap_contract(const sclap_graph* g, const int32_t* labels, int32_t* C, sclap_graph_owned* coarse) {
    return guarded([&] {
        hipStream_t s = nullptr;
        if (!coarse) fail(SCLAP_ERR_INVALID, "coarse is NULL");
        Staged st = upload(g, s);
        const int32_t n = st.g.n;
        if (n > 0 && (!labels || !C)) fail(SCLAP_ERR_INVALID, "labels / C is NULL");
        DBuf<int32_t> lab = upload_array(labels, n, s);
        if (!all_in_range(lab.get(), n, 0, std::max(n, 1), s)) fail(SCLAP_ERR_INVALID, "label outside [0, n)");
        DBuf<int32_t> dC(std::max(n, 1), s);
        OwnedDevGraph cg;
        contract(st.g, lab.get(), dC.get(), cg, s);
        download(C, dC.get(), n, s);
        sclap_graph_owned out{};
        out.n = cg.n;
        out.S = cg.S;
        out.on_device = 0;
        out.xadj = static_cast<int64_t*>(std::malloc((cg.n + 1) * sizeof(int64_t)));
        out.adjncy = static_cast<int32_t*>(std::malloc(std::max<int64_t>(cg.S, 1) * sizeof(int32_t)));
        out.adjwgt = static_cast<int32_t*>(std::malloc(std::max<int64_t>(cg.S, 1) * sizeof(int32_t)));
        out.vwgt = static_cast<int32_t*>(std::malloc(std::max(cg.n, 1) * sizeof(int32_t)));
        if (!out.xadj || !out.adjncy || !out.adjwgt || !out.vwgt) {
            std::free(out.xadj); std::free(out.adjncy); std::free(out.adjwgt); std::free(out.vwgt);
            throw std::bad_alloc();
        }
        download(out.xadj, cg.xadj.get(), cg.n + 1, s);
        download(out.adjncy, cg.adj.get(), cg.S, s);
        download(out.adjwgt, cg.ew.get(), cg.S, s);
        download(out.vwgt, cg.vw.get(), cg.n, s);
        *coarse = out;
        return SCLAP_OK;
    });
}

void sclap_graph_free(sclap_graph_owned* g) {
    if (!g) return;
    if (g->on_device) {
        if (g->xadj) (void)hipFreeAsync(g->xadj, nullptr);
        if (g->adjncy) (void)hipFreeAsync(g->adjncy, nullptr);
        if (g->adjwgt) (void)hipFreeAsync(g->adjwgt, nullptr);
        if (g->vwgt) (void)hipFreeAsync(g->vwgt, nullptr);
        (void)hipStreamSynchronize(nullptr);
    } else {
        std::free(g->xadj);
        std::free(g->adjncy);
        std::free(g->adjwgt);
        std::free(g->vwgt);
    }
    std::memset(g, 0, sizeof(*g));
}

int sclap_project_dev(int32_t n, int32_t n_coarse, const int32_t* C, const int32_t* coarse_part, int32_t* part,
                      void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        if (n < 0 || n_coarse < 0) fail(SCLAP_ERR_INVALID, "negative size");
        if (n == 0) return SCLAP_OK;
        if (!C || !coarse_part || !part) fail(SCLAP_ERR_INVALID, "NULL array");
        if (!all_in_range(C, n, 0, n_coarse, s)) fail(SCLAP_ERR_INVALID, "C value outside [0, n_coarse)");
        project(n, C, coarse_part, part, s);
        HIPCHK(hipStreamSynchronize(s));
        return SCLAP_OK;
    });
}

int sclap_project(int32_t n, int32_t n_coarse, const int32_t* C, const int32_t* coarse_part, int32_t* part) {
    return guarded([&] {
        hipStream_t s = nullptr;
        if (n < 0 || n_coarse < 0) fail(SCLAP_ERR_INVALID, "negative size");
        if (n == 0) return SCLAP_OK;
        if (!C || !coarse_part || !part) fail(SCLAP_ERR_INVALID, "NULL array");
        DBuf<int32_t> dC = upload_array(C, n, s);
        DBuf<int32_t> dcp = upload_array(coarse_part, n_coarse, s);
        DBuf<int32_t> dp(n, s);
        if (!all_in_range(dC.get(), n, 0, n_coarse, s)) fail(SCLAP_ERR_INVALID, "C value outside [0, n_coarse)");
        project(n, dC.get(), dcp.get(), dp.get(), s);
        download(part, dp.get(), n, s);
        return SCLAP_OK;
    });
}

int sclap_cut_dev(const sclap_graph* g, const int32_t* part, int32_t k, int64_t* cut, int64_t* block_w,
                  void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        if (k < 1 || !cut || !block_w) fail(SCLAP_ERR_INVALID, "bad k or NULL output");
        const DevGraph d = dev_view(g, s);
        if (d.n > 0 && !part) fail(SCLAP_ERR_INVALID, "part is NULL");
        if (!all_in_range(part, d.n, 0, k, s)) fail(SCLAP_ERR_INVALID, "part value outside [0, k)");
        cut_and_weights(d, part, k, cut, block_w, s);
        return SCLAP_OK;
    });
}

int sclap_cut_dev_noalloc(const sclap_graph* g, const int32_t* part, int32_t k, int64_t* cut, int64_t* block_w,
                          void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        if (k < 1 || !cut || !block_w) fail(SCLAP_ERR_INVALID, "bad k or NULL output");
        const DevGraph d = dev_view(g, s);
        if (d.n > 0 && !part) fail(SCLAP_ERR_INVALID, "part is NULL");
        cut_and_weights_noalloc(d, part, k, cut, block_w, s);
        return SCLAP_OK;
    });
}

int sclap_cut(const sclap_graph* g, const int32_t* part, int32_t k, int64_t* cut, int64_t* block_w) {
    return guarded([&] {
        hipStream_t s = nullptr;
        if (k < 1 || !cut || !block_w) fail(SCLAP_ERR_INVALID, "bad k or NULL output");
        Staged st = upload(g, s);
        if (st.g.n > 0 && !part) fail(SCLAP_ERR_INVALID, "part is NULL");
        DBuf<int32_t> p = upload_array(part, st.g.n, s);
        if (!all_in_range(p.get(), st.g.n, 0, k, s)) fail(SCLAP_ERR_INVALID, "part value outside [0, k)");
        cut_and_weights(st.g, p.get(), k, cut, block_w, s);
        return SCLAP_OK;
    });
}

int sclap_initial_partition(const sclap_graph* g, int32_t k, int32_t* part) {
    return guarded([&] {
        if (!g || g->n < 0 || k < 1) fail(SCLAP_ERR_INVALID, "bad arguments");
        if (g->n == 0) return SCLAP_OK;
        if (!g->xadj || !part || (g->xadj[g->n] > 0 && !g->adjncy)) fail(SCLAP_ERR_INVALID, "NULL array");
        int64_t cV = 0;
        for (int32_t v = 0; v < g->n; ++v) cV += g->vwgt ? g->vwgt[v] : 1;
        host_initial_partition(g->n, g->xadj, g->adjncy, g->vwgt, k, (cV + k - 1) / k, part);
        return SCLAP_OK;
    });
}

int sclap_initial_partition_lp_dev(const sclap_graph* g, int32_t k, int64_t T, int64_t Lmax, uint64_t seed,
                                   int32_t level, int32_t rounds, const sclap_options* opt, int32_t* part,
                                   int64_t* visits, void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        const Opts o = resolve(opt);
        const DevGraph d = dev_view(g, s);
        if (k < 1 || rounds < 0 || T < 0 || Lmax < 0) fail(SCLAP_ERR_INVALID, "bad k, rounds, T or Lmax");
        if (d.n > 0 && !part) fail(SCLAP_ERR_INVALID, "part is NULL");
        int64_t cV = 0, cmax = 0;
        check_graph(d, o.validate != 0, &cV, &cmax, s);
        const LPResult r = device_initial_partition(d, k, T, Lmax, seed, level, o.nsub, rounds, o.tune, part, s);
        HIPCHK(hipStreamSynchronize(s));
        if (visits) *visits = r.visits;
        return SCLAP_OK;
    });
}

int sclap_partition_dev(const sclap_graph* g, int32_t k, double eps, uint64_t seed, const sclap_options* opt,
                        int32_t* part, int64_t* cut, int64_t* block_w, sclap_stats* stats, void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        const Opts o = resolve(opt);
        const DevGraph d = dev_view(g, s);
        return partition_impl(d, k, eps, seed, o, part, cut, block_w, stats, s);
    });
}

int sclap_partition(const sclap_graph* g, int32_t k, double eps, uint64_t seed, const sclap_options* opt,
                    int32_t* part, int64_t* cut, int64_t* block_w, sclap_stats* stats) {
    return guarded([&] {
        hipStream_t s = nullptr;
        const Opts o = resolve(opt);
        check_k_eps(k, eps);
        Staged st = upload(g, s);
        if (st.g.n > 0 && !part) fail(SCLAP_ERR_INVALID, "part is NULL");
        DBuf<int32_t> p(std::max(st.g.n, 1), s);
        const int r = partition_impl(st.g, k, eps, seed, o, p.get(), cut, block_w, stats, s);
        download(part, p.get(), st.g.n, s);
        return r;
    });
}

int sclap_partition_batch_dev(const sclap_graph* g, int32_t count, const int32_t* node_base, const int32_t* k,
                              const double* eps, const uint64_t* seed, const sclap_options* opt, int32_t* part,
                              int64_t* cut, int64_t* block_w, sclap_batch_stats* stats, void* stream) {
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        const Opts o = resolve(opt);
        const DevGraph d = dev_view(g, s);
        return partition_batch_impl(d, count, node_base, k, eps, seed, o, part, cut, block_w, stats, s);
    });
}

int sclap_partition_batch(const sclap_graph* g, int32_t count, const int32_t* node_base, const int32_t* k,
                          const double* eps, const uint64_t* seed, const sclap_options* opt, int32_t* part,
                          int64_t* cut, int64_t* block_w, sclap_batch_stats* stats) {
    return guarded([&] {
        hipStream_t s = nullptr;
        const Opts o = resolve(opt);
        Staged st = upload(g, s);
        if (st.g.n > 0 && !part) fail(SCLAP_ERR_INVALID, "part is NULL");
        DBuf<int32_t> p(std::max(st.g.n, 1), s);
        const int r = partition_batch_impl(st.g, count, node_base, k, eps, seed, o, p.get(), cut, block_w, stats, s);
        download(part, p.get(), st.g.n, s);
        return r;
    });
}

sclap_server* sclap_server_create(int32_t device, int64_t hbm_budget, int32_t slots, int32_t max_batch,
                                  const sclap_options* opt) {
    sclap_server* sv = nullptr;
    guarded([&] {
        sv = server_create(device, hbm_budget, slots, max_batch, opt);
        return SCLAP_OK;
    });
    return sv;
}

int sclap_server_submit(sclap_server* sv, const sclap_graph* g, int32_t k, double eps, uint64_t seed,
                        uint64_t* req) {
    return guarded([&] {
        if (!req) fail(SCLAP_ERR_INVALID, "req is NULL");
        *req = server_submit(sv, g, k, eps, seed);
        return SCLAP_OK;
    });
}

int sclap_server_poll(sclap_server* sv, uint64_t req, int32_t timeout_ms, int32_t* done, int32_t* part,
                      int64_t* cut, int64_t* block_w, sclap_request_info* info) {
    return guarded([&] { return server_poll(sv, req, timeout_ms, done, part, cut, block_w, info); });
}

int32_t sclap_server_plan_batch(const int64_t* nodes, const int64_t* slots, const int64_t* footprint, int32_t count,
                                int64_t free_budget, int32_t max_batch, int32_t idle) {
    if (count < 0 || max_batch < 1 || (count > 0 && (!nodes || !slots || !footprint))) return SCLAP_ERR_INVALID;
    return plan_batch(nodes, slots, footprint, count, free_budget, max_batch, idle != 0);
}

void sclap_server_destroy(sclap_server* sv) {
    guarded([&] {
        server_destroy(sv);
        return SCLAP_OK;
    });
}

int sclap_autotune_dev(const sclap_graph* g, int32_t k, sclap_options* opt, void* stream) {
    return guarded([&] {
        if (!opt) fail(SCLAP_ERR_INVALID, "opt is NULL");
        hipStream_t s = as_stream(stream);
        const Opts o = resolve(opt);
        const DevGraph d = dev_view(g, s);
        const LPTuning t = autotune(d, k, o, s);
        opt->lane_max_degree = t.lane_max;
        opt->wave_max_degree = t.wave_max;
        opt->block_max_degree = t.block_max;
        opt->graph_capture = t.capture;
        opt->block_table = t.block_table;
        return SCLAP_OK;
    });
}

int sclap_gather_probe_dev(const sclap_graph* g, int32_t label_bytes, int32_t reps, double* ms, void* stream) {
    return guarded([&] {
        if (!ms || reps < 1) fail(SCLAP_ERR_INVALID, "ms is NULL or reps < 1");
        hipStream_t s = as_stream(stream);
        const DevGraph d = dev_view(g, s);
        *ms = gather_probe(d, label_bytes, reps, s);
        return SCLAP_OK;
    });
}

int sclap_profile_begin(void) { return sclap_profile_begin_only(nullptr); }

int sclap_profile_begin_only(const char* name) {
    return guarded([&] {
        profiler().reset();
        profiler().only = name ? name : "";
        profiler().on = true;
        return SCLAP_OK;
    });
}

int sclap_profile_end(sclap_kernel_stat* out, int32_t capacity, int32_t* count) {
    return guarded([&] {
        Profiler& p = profiler();
        p.collect();
        const int32_t m = static_cast<int32_t>(p.stats.size());
        for (int32_t i = 0; i < m && i < capacity && out; ++i) {
            std::memset(&out[i], 0, sizeof(out[i]));
            std::strncpy(out[i].name, p.stats[i].name.c_str(), sizeof(out[i].name) - 1);
            out[i].launches = p.stats[i].launches;
            out[i].ms = p.stats[i].ms;
            out[i].bytes = p.stats[i].bytes;
        }
        if (count) *count = m;
        p.stats.clear();
        p.on = false;
        return SCLAP_OK;
    });
}

}  // extern "C"
