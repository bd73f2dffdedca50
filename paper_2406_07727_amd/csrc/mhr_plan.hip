// Batched form around the query path: a captured HIP graph of one
// mhr_topk_paths call (replayed with one launch), and the autotuner that
// picks the tile length and probe-table size for a batch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "mhr.h"
#include "mhr_internal.h"

struct mhr_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace mhr;

extern "C" mhr_status mhr_plan_create(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq,
                                      const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                      uint32_t kmax, mhr_path *out, uint32_t *out_count, uint64_t *out_total,
                                      uint32_t *out_status, void *workspace, size_t ws_bytes, void *stream,
                                      mhr_plan **plan) {
    MHR_ARG_CHECK(plan != nullptr, "mhr_plan_create: null plan pointer");
    MHR_ARG_CHECK(nq >= 1, "mhr_plan_create: nq must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    bool own = false;
    if (st == nullptr) {
        MHR_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        own = true;
    }
    auto drop_stream = [&]() {
        if (own) (void)hipStreamDestroy(st);
    };
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        set_error(std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        drop_stream();
        return MHR_ERR_DEVICE;
    }
    const mhr_status rc = mhr_topk_paths(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status,
                                         workspace, ws_bytes, st);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (rc != MHR_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        drop_stream();
        if (rc != MHR_OK) return rc;   // the query call's own message stands
        set_error(std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        return MHR_ERR_DEVICE;
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    drop_stream();
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        return MHR_ERR_DEVICE;
    }
    mhr_plan *p = new (std::nothrow) mhr_plan;
    if (!p) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        set_error("mhr_plan_create: out of host memory");
        return MHR_ERR_OUT_OF_MEMORY;
    }
    p->graph = graph;
    p->exec = exec;
    *plan = p;
    return MHR_OK;
}

extern "C" mhr_status mhr_plan_launch(mhr_plan *plan, void *stream) {
    MHR_ARG_CHECK(plan != nullptr && plan->exec != nullptr, "mhr_plan_launch: null plan");
    MHR_HIP_TRY(hipGraphLaunch(plan->exec, static_cast<hipStream_t>(stream)));
    return MHR_OK;
}

extern "C" mhr_status mhr_plan_destroy(mhr_plan *plan) {
    if (!plan) return MHR_OK;
    hipError_t e1 = plan->exec ? hipGraphExecDestroy(plan->exec) : hipSuccess;
    hipError_t e2 = plan->graph ? hipGraphDestroy(plan->graph) : hipSuccess;
    delete plan;
    if (e1 != hipSuccess || e2 != hipSuccess) {
        set_error("mhr_plan_destroy: graph release failed");
        return MHR_ERR_DEVICE;
    }
    return MHR_OK;
}

namespace {

// Host copies of one call's outputs, for checking that a setting leaves the
// results unchanged.
struct Outputs {
    std::vector<unsigned char> paths, count, total, status;
};

hipError_t fetch(Outputs &o, uint32_t nq, uint32_t kmax, const mhr_path *out, const uint32_t *out_count,
                 const uint64_t *out_total, const uint32_t *out_status, hipStream_t st) {
    o.paths.resize(size_t(nq) * kmax * sizeof(mhr_path));
    o.count.resize(size_t(nq) * sizeof(uint32_t));
    o.total.resize(out_total ? size_t(nq) * sizeof(uint64_t) : 0);
    o.status.resize(out_status ? size_t(nq) * sizeof(uint32_t) : 0);
    hipError_t e = hipMemcpyAsync(o.paths.data(), out, o.paths.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(o.count.data(), out_count, o.count.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && out_total)
        e = hipMemcpyAsync(o.total.data(), out_total, o.total.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && out_status)
        e = hipMemcpyAsync(o.status.data(), out_status, o.status.size(), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

bool same(const Outputs &a, const Outputs &b) {
    return a.paths == b.paths && a.count == b.count && a.total == b.total && a.status == b.status;
}

}  // namespace

extern "C" mhr_status mhr_autotune(const mhr_graph *g, const mhr_query_opts *base, uint32_t nq,
                                   const uint32_t *src, const uint32_t *dst, const uint32_t *k, uint32_t kmax,
                                   mhr_path *out, uint32_t *out_count, uint64_t *out_total, uint32_t *out_status,
                                   void *workspace, size_t ws_bytes, void *stream, uint32_t reps,
                                   mhr_query_opts *tuned, float *best_ms) {
    MHR_ARG_CHECK(g != nullptr && tuned != nullptr, "mhr_autotune: null argument");
    MHR_ARG_CHECK(nq >= 1 && reps >= 1 && reps <= 1000, "mhr_autotune: nq >= 1 and 1 <= reps <= 1000");
    hipStream_t st = static_cast<hipStream_t>(stream);
    mhr_query_opts o{};
    if (base) o = *base;
    static const uint32_t kTiles[] = {8192, 16384, 32768, 65536, 131072, 262144, 524288};
    static const uint32_t kHash[] = {10, 11, 12};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MHR_HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        set_error("mhr_autotune: hipEventCreate failed");
        return MHR_ERR_DEVICE;
    }
    Outputs ref, cur;
    bool have_ref = false;
    float best = 0.0f;
    mhr_query_opts best_o{};
    mhr_status rc = MHR_OK;
    bool any = false;
    for (uint32_t te : kTiles) {
        for (uint32_t hl : kHash) {
            mhr_query_opts c = o;
            c.tile_edges = te;
            c.hash_log2 = hl;
            // settings whose workgroup does not fit are skipped, not errors
            mhr_status r = mhr_topk_paths(g, &c, nq, src, dst, k, kmax, out, out_count, out_total, out_status,
                                          workspace, ws_bytes, st);
            if (r == MHR_ERR_UNSUPPORTED) continue;
            if (r != MHR_OK) { rc = r; goto done; }
            if (fetch(cur, nq, kmax, out, out_count, out_total, out_status, st) != hipSuccess) {
                set_error("mhr_autotune: copying results failed");
                rc = MHR_ERR_DEVICE;
                goto done;
            }
            if (!have_ref) {
                ref = cur;
                have_ref = true;
            } else if (!same(ref, cur)) {
                set_error("mhr_autotune: tile_edges " + std::to_string(te) + ", hash_log2 " + std::to_string(hl) +
                          " changed the results");
                rc = MHR_ERR_INTERNAL;
                goto done;
            }
            if (hipEventRecord(e0, st) != hipSuccess) { rc = MHR_ERR_DEVICE; goto done; }
            for (uint32_t i = 0; i < reps; ++i) {
                r = mhr_topk_paths(g, &c, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace,
                                   ws_bytes, st);
                if (r != MHR_OK) { rc = r; goto done; }
            }
            float ms = 0.0f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                set_error("mhr_autotune: timing failed");
                rc = MHR_ERR_DEVICE;
                goto done;
            }
            ms /= static_cast<float>(reps);
            if (!any || ms < best) {
                best = ms;
                best_o = c;
                any = true;
            }
        }
    }
    if (!any) {
        set_error("mhr_autotune: no candidate setting fits this graph");
        rc = MHR_ERR_UNSUPPORTED;
    }
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == MHR_OK) {
        *tuned = best_o;
        if (best_ms) *best_ms = best;
    }
    return rc;
}
