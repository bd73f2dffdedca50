// Generic multi-hop search (paper section 5, the level-by-level algorithm
// with a per-parent top-K): from the source, every current path grows by
// each out-edge of its last vertex whose head is not on the path yet; an
// extension that reaches the target is recorded as a result and not grown
// further; of the other extensions each parent passes its best K to the
// next level.  After H levels the best K recorded paths are returned.
// Scores add the edge weights along the path.
//
// The paper parallelises each level over the current paths with as many
// threads as paths.  Here one workgroup expands one current path: its
// threads take the typed out-edges of the path's last vertex, score them
// and keep a running best K in LDS (bitonic merges of K + 256 entries);
// the level's paths sit at fixed slots (parent p's children at p*K ..
// p*K + K - 1), so no compaction pass is needed between levels, and every
// level is one launch on the stream with no host synchronisation.
//
// The beam keeps or drops paths by comparing scores, so the kernels score
// in FP64, in the definition's operation order (the edge weight's sum in
// ascending i, then the path's running sum), and take the same decisions as
// the FP64 definition: bit for bit for the TransE-L1 scorer (additions and
// absolute values only); for DistMult the FP64 exp and log1p of the device
// library may differ from another library's in the last bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mhr_device.h"
#include "mhr_internal.h"

namespace mhr {
namespace {

constexpr int kBeamThreads = 256;
constexpr uint32_t kMaxBeamK = 64;
constexpr uint32_t kMaxSlots = 1u << 20;   // paths of one level of one query
constexpr uint32_t kNoVertex = 0xFFFFFFFFu;
constexpr uint32_t kMergeN = 512;   // running best (<= kMaxBeamK) + one round of candidates, a power of two
static_assert(kMaxBeamK + kBeamThreads <= kMergeN, "merge buffer");

struct BP {
    double s;
    uint32_t len;                      // edges; 0 = the source alone
    uint32_t v[MHR_BEAM_MAX_HOPS];     // vertices after the source
    uint16_t r[MHR_BEAM_MAX_HOPS];
    uint32_t valid;
};

// Candidate of the running top-K: score, head vertex, relation, and (for
// results) the index of the recorded path.
struct BC {
    double s;
    uint32_t nb, r;
};

__device__ __forceinline__ bool bc_better(const BC &x, const BC &y) {
    if (x.s != y.s) return x.s > y.s;
    if (x.nb != y.nb) return x.nb < y.nb;
    return x.r < y.r;
}

__device__ __forceinline__ BC bc_none() {
    BC c;
    c.s = -__builtin_huge_val();
    c.nb = kNoVertex;
    c.r = 0xFFFFFFFFu;
    return c;
}

template <class T, class Better>
__device__ void bitonic_best_first(T *c, uint32_t n, Better better) {
    for (uint32_t k = 2; k <= n; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
                const uint32_t p = i ^ j;
                if (p > i) {
                    const T x = c[i], y = c[p];
                    const bool up = (i & k) == 0;
                    if (up ? better(y, x) : better(x, y)) {
                        c[i] = y;
                        c[p] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

#pragma clang fp contract(off)
// FP64 edge weight in the definition's operation order.
template <bool BF16, bool TE>
__device__ double edge_w64(const void *X, const void *Y, uint32_t d, double gamma, uint32_t u, uint32_t r, uint32_t v) {
    double acc = 0.0;
    const size_t du = static_cast<size_t>(u) * d, dr = static_cast<size_t>(r) * d, dv = static_cast<size_t>(v) * d;
    if (TE) {
        for (uint32_t i = 0; i < d; ++i)
            acc += fabs((static_cast<double>(load1<BF16>(X, du + i)) + static_cast<double>(load1<BF16>(Y, dr + i))) -
                        static_cast<double>(load1<BF16>(X, dv + i)));
        return gamma - acc;
    }
    for (uint32_t i = 0; i < d; ++i)
        acc += (static_cast<double>(load1<BF16>(X, du + i)) * static_cast<double>(load1<BF16>(Y, dr + i))) *
               static_cast<double>(load1<BF16>(X, dv + i));
    return fmin(acc, 0.0) - log1p(exp(-fabs(acc)));
}
#pragma clang fp contract(on)

struct BeamArgs {
    const uint32_t *rp, *col, *mask;    // forward CSR
    const void *X, *Y;
    uint32_t n, d;
    double gamma;
    const uint32_t *src, *dst;
    uint32_t nq, H, K, K2;
    BP *curr, *next;                    // [nq][slots]
    uint32_t curr_slots, next_slots;
    BP *res;                            // [nq][res_cap]
    uint32_t res_cap;
    uint32_t *res_n;                    // [nq]
    uint32_t *overflow;                 // [nq]
};

// Level start: the source alone in slot 0 of every query, the result
// counters cleared.
__global__ void beam_init_kernel(BeamArgs A) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= A.nq) return;
    BP root{};
    root.s = 0.0;
    root.len = 0;
    root.valid = A.src[q] < A.n && A.dst[q] < A.n;
    A.curr[static_cast<size_t>(q) * A.curr_slots] = root;
    A.res_n[q] = 0;
    A.overflow[q] = 0;
}

// grid (slots of this level, nq): expands one current path.  last: the
// final level (children are not kept).
template <bool BF16, bool TE>
__global__ __launch_bounds__(kBeamThreads) void beam_expand_kernel(BeamArgs A, uint32_t slots, int last) {
    __shared__ BC best[kMergeN];
    __shared__ BP par;
    __shared__ uint32_t ok;
    const uint32_t q = blockIdx.y, slot = blockIdx.x;
    if (threadIdx.x == 0) {
        par = A.curr[static_cast<size_t>(q) * A.curr_slots + slot];
        ok = slot < slots && par.valid;
    }
    __syncthreads();
    const uint32_t K = A.K, K2 = A.K2;
    if (!ok) {
        if (!last && slot < slots)
            for (uint32_t i = threadIdx.x; i < K; i += kBeamThreads)
                A.next[static_cast<size_t>(q) * A.next_slots + static_cast<size_t>(slot) * K + i].valid = 0;
        return;
    }
    const uint32_t s = A.src[q], t = A.dst[q];
    const uint32_t h = par.len ? par.v[par.len - 1] : s;
    for (uint32_t i = threadIdx.x; i < K2; i += kBeamThreads) best[i] = bc_none();
    const uint32_t beg = A.rp[h], end = A.rp[h + 1];
    // rounds of one out-pair per thread (a pair's relations handled by that
    // thread one after another); each round's candidates merge into best[]
    for (uint32_t base = beg; base < end; base += kBeamThreads) {
        __syncthreads();
        const uint32_t e = base + threadIdx.x;
        uint32_t nb = kNoVertex, msk = 0;
        if (e < end) {
            nb = A.col[e];
            msk = A.mask[e];
            bool on = nb == s;
            for (uint32_t i = 0; i < par.len; ++i) on |= par.v[i] == nb;
            if (on) msk = 0;
        }
        // each relation of the pair in turn: record or offer as a child
        uint32_t rest = msk;
        for (;;) {
            const bool have = rest != 0;
            BC c = bc_none();
            if (have) {
                const uint32_t r = static_cast<uint32_t>(__ffs(rest) - 1);
                rest &= rest - 1;
                c.s = par.s + edge_w64<BF16, TE>(A.X, A.Y, A.d, A.gamma, h, r, nb);
                c.nb = nb;
                c.r = r;
                if (nb == t) {
                    const uint32_t at = atomicAdd(&A.res_n[q], 1u);
                    if (at < A.res_cap) {
                        BP x = par;
                        x.v[x.len] = nb;
                        x.r[x.len] = static_cast<uint16_t>(r);
                        x.len += 1;
                        x.s = c.s;
                        x.valid = 1;
                        A.res[static_cast<size_t>(q) * A.res_cap + at] = x;
                    } else {
                        A.overflow[q] = 1;
                    }
                    c = bc_none();
                }
            }
            if (!last) {
                best[K2 + threadIdx.x] = c;
                for (uint32_t i = K2 + kBeamThreads + threadIdx.x; i < kMergeN; i += kBeamThreads) best[i] = bc_none();
            }
            const int any = __syncthreads_or(have ? 1 : 0);
            if (!any) break;
            if (!last) bitonic_best_first(best, kMergeN, bc_better);
        }
    }
    __syncthreads();
    if (last) return;
    for (uint32_t i = threadIdx.x; i < K; i += kBeamThreads) {
        BP x = par;
        const BC c = best[i];
        x.valid = c.nb != kNoVertex;
        if (x.valid) {
            x.v[x.len] = c.nb;
            x.r[x.len] = static_cast<uint16_t>(c.r);
            x.len += 1;
            x.s = c.s;
        }
        A.next[static_cast<size_t>(q) * A.next_slots + static_cast<size_t>(slot) * K + i] = x;
    }
}

// Recorded paths in the output order: score descending, then the vertex
// sequence (a proper prefix first), then the relation sequence.
__device__ __forceinline__ bool bp_better(const BP &x, const BP &y) {
    if (x.valid != y.valid) return x.valid > y.valid;
    if (x.s != y.s) return x.s > y.s;
    const uint32_t n = x.len < y.len ? x.len : y.len;
    for (uint32_t i = 0; i < n; ++i)
        if (x.v[i] != y.v[i]) return x.v[i] < y.v[i];
    if (x.len != y.len) return x.len < y.len;
    for (uint32_t i = 0; i < x.len; ++i)
        if (x.r[i] != y.r[i]) return x.r[i] < y.r[i];
    return false;
}

// grid (nq): the best K recorded paths (rounds of 256 merged into a running
// best K2 in LDS).
__global__ __launch_bounds__(kBeamThreads) void beam_final_kernel(BeamArgs A, mhr_beam_path *out, uint32_t *out_count,
                                                                  uint64_t *out_recorded) {
    __shared__ BP best[kMergeN];
    const uint32_t q = blockIdx.x;
    const uint32_t K = A.K, K2 = A.K2;
    const uint32_t nrec = A.res_n[q], nres = nrec < A.res_cap ? nrec : A.res_cap;
    for (uint32_t i = threadIdx.x; i < K2; i += kBeamThreads) best[i].valid = 0;
    const BP *res = A.res + static_cast<size_t>(q) * A.res_cap;
    for (uint32_t base = 0; base < nres; base += kBeamThreads) {
        __syncthreads();
        const uint32_t i = base + threadIdx.x;
        BP x{};
        x.valid = 0;
        if (i < nres) x = res[i];
        best[K2 + threadIdx.x] = x;
        for (uint32_t j = K2 + kBeamThreads + threadIdx.x; j < kMergeN; j += kBeamThreads) best[j].valid = 0;
        __syncthreads();
        bitonic_best_first(best, kMergeN, bp_better);
    }
    __syncthreads();
    const uint32_t cnt = nres < K ? nres : K;
    for (uint32_t i = threadIdx.x; i < K; i += kBeamThreads) {
        mhr_beam_path p{};
        if (i < cnt) {
            const BP &x = best[i];
            p.score = x.s;
            p.len = x.len;
            for (uint32_t j = 0; j < MHR_BEAM_MAX_HOPS; ++j) {
                p.v[j] = j < x.len ? x.v[j] : kNoVertex;
                p.r[j] = j < x.len ? x.r[j] : static_cast<uint16_t>(0xFFFF);
            }
        } else {
            p.score = -__builtin_huge_val();
            p.len = 0;
            for (uint32_t j = 0; j < MHR_BEAM_MAX_HOPS; ++j) {
                p.v[j] = kNoVertex;
                p.r[j] = 0xFFFF;
            }
        }
        out[static_cast<size_t>(q) * K + i] = p;
    }
    if (threadIdx.x == 0) {
        out_count[q] = cnt;
        if (out_recorded) out_recorded[q] = nrec;
    }
}

uint32_t ipow(uint32_t b, uint32_t e) {
    uint64_t v = 1;
    for (uint32_t i = 0; i < e; ++i) v = std::min<uint64_t>(v * b, 0xFFFFFFFFull);
    return static_cast<uint32_t>(v);
}

struct BeamLayout {
    uint32_t slots;      // the largest level's paths per query
    uint32_t res_cap;    // recorded paths per query
    size_t curr, next, res, res_n, overflow, total;
};

BeamLayout beam_layout(uint32_t R, uint32_t nq, uint32_t H, uint32_t K) {
    BeamLayout L{};
    L.slots = ipow(K, H - 1);
    // every path of every level can record one result per relation
    uint64_t paths = 0;
    for (uint32_t l = 0; l < H; ++l) paths += ipow(K, l);
    L.res_cap = static_cast<uint32_t>(std::min<uint64_t>(paths * R, 0xFFFFFFFull));
    auto al = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    size_t o = 0;
    L.curr = o; o = al(o + size_t(nq) * L.slots * sizeof(BP));
    L.next = o; o = al(o + size_t(nq) * L.slots * sizeof(BP));
    L.res = o; o = al(o + size_t(nq) * L.res_cap * sizeof(BP));
    L.res_n = o; o = al(o + size_t(nq) * 4);
    L.overflow = o; o = al(o + size_t(nq) * 4);
    L.total = o;
    return L;
}

}  // namespace
}  // namespace mhr

using namespace mhr;

extern "C" mhr_status mhr_beam_workspace_size(const mhr_graph *g, uint32_t nq, uint32_t hops, uint32_t k,
                                              size_t *bytes) {
    MHR_ARG_CHECK(g && bytes, "mhr_beam_workspace_size: null argument");
    MHR_ARG_CHECK(hops >= 1 && hops <= MHR_BEAM_MAX_HOPS, "hops must be in [1, MHR_BEAM_MAX_HOPS]");
    MHR_ARG_CHECK(k >= 1 && k <= kMaxBeamK, "k must be in [1, 64]");
    MHR_ARG_CHECK(ipow(k, hops - 1) <= kMaxSlots, "k^(hops-1) must not exceed 2^20 paths per level");
    *bytes = beam_layout(g->R, nq, hops, k).total;
    return MHR_OK;
}

extern "C" mhr_status mhr_beam_search(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                                      uint32_t hops, uint32_t k, mhr_beam_path *out, uint32_t *out_count,
                                      uint64_t *out_recorded, void *workspace, size_t ws_bytes, void *stream) {
    MHR_ARG_CHECK(g != nullptr, "mhr_beam_search: null graph");
    if (!g->X) {
        set_error("embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    MHR_ARG_CHECK(hops >= 1 && hops <= MHR_BEAM_MAX_HOPS, "hops must be in [1, MHR_BEAM_MAX_HOPS]");
    MHR_ARG_CHECK(k >= 1 && k <= kMaxBeamK, "k must be in [1, 64]");
    MHR_ARG_CHECK(ipow(k, hops - 1) <= kMaxSlots, "k^(hops-1) must not exceed 2^20 paths per level");
    if (nq == 0) return MHR_OK;
    MHR_ARG_CHECK(src && dst && out && out_count && workspace, "mhr_beam_search: null pointer");
    const BeamLayout L = beam_layout(g->R, nq, hops, k);
    if (ws_bytes < L.total) {
        set_error("mhr_beam_search: workspace too small");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(workspace);
    BeamArgs A{};
    A.rp = g->out.row_ptr;
    A.col = g->out.col;
    A.mask = g->out.rmask;
    A.X = g->X;
    A.Y = g->Y;
    A.n = g->n;
    A.d = g->dim;
    A.gamma = static_cast<double>(g->gamma);
    A.src = src;
    A.dst = dst;
    A.nq = nq;
    A.H = hops;
    A.K = k;
    A.K2 = next_pow2(k);
    A.curr = reinterpret_cast<BP *>(w + L.curr);
    A.next = reinterpret_cast<BP *>(w + L.next);
    A.curr_slots = L.slots;
    A.next_slots = L.slots;
    A.res = reinterpret_cast<BP *>(w + L.res);
    A.res_cap = L.res_cap;
    A.res_n = reinterpret_cast<uint32_t *>(w + L.res_n);
    A.overflow = reinterpret_cast<uint32_t *>(w + L.overflow);
    hipLaunchKernelGGL(beam_init_kernel, dim3((nq + 255) / 256), dim3(256), 0, st, A);
    const bool bf = g->dtype == MHR_DTYPE_BF16, te = g->scorer == MHR_SCORER_TRANSE_L1;
    uint32_t slots = 1;
    for (uint32_t level = 0; level < hops; ++level) {
        const int last = level + 1 == hops;
        const dim3 grid(slots, nq);
        if (bf) {
            if (te) hipLaunchKernelGGL((beam_expand_kernel<true, true>), grid, dim3(kBeamThreads), 0, st, A, slots, last);
            else hipLaunchKernelGGL((beam_expand_kernel<true, false>), grid, dim3(kBeamThreads), 0, st, A, slots, last);
        } else {
            if (te) hipLaunchKernelGGL((beam_expand_kernel<false, true>), grid, dim3(kBeamThreads), 0, st, A, slots, last);
            else hipLaunchKernelGGL((beam_expand_kernel<false, false>), grid, dim3(kBeamThreads), 0, st, A, slots, last);
        }
        std::swap(A.curr, A.next);
        slots *= k;
    }
    hipLaunchKernelGGL(beam_final_kernel, dim3(nq), dim3(kBeamThreads), 0, st, A, out, out_count, out_recorded);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}
