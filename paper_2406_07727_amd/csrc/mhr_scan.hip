// Candidate scan: the workload of the paper's three-hop award pipeline
// (section 3.2, the simple algorithm; section 3.3, the person, field and
// affiliation scoring).  For each query (head, relation) every candidate c
// of a list is scored with the TransE-L1 score
//     gamma - sum_i |(X[head,i] + Y[rel,i]) - X[c,i]|
// (the candidate as the tail) and the best K are kept under the total
// order (score descending, candidate id ascending).
//
// The paper scores candidates with thread-private K-heaps merged by a
// reduction tree.  Here a workgroup scores a chunk of kChunk candidates and
// keeps its best K2 = next_pow2(K) by a radix select in LDS (only those K2
// are sorted); a second kernel selects a query's best K the same way over
// its chunk lists.  A candidate costs
// one embedding row (d values) read from HBM: the scan is bandwidth-bound,
// and the scores are evaluated in FP64 in the oracle's operation order
// (head plus relation, minus the candidate, absolute value, summed in
// ascending i), so every comparison, including exact ties, is decided on the
// same values as the FP64 definition.  At d = 8 a candidate is 32 bytes and
// 24 FP64 operations: at 8 TB/s that asks for about 6 TFLOP/s of FP64, a
// small part of the chip's vector FP64 rate.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mhr_device.h"
#include "mhr_internal.h"

namespace mhr {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;
constexpr int kChunk = kScanThreads * kScanPer;   // candidates per workgroup (and per merge step)
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kMaxScanK = 256;
constexpr uint32_t kMaxScanDim = 512;

struct SC {
    double s;
    uint32_t id;
    uint32_t pad;
};

__device__ __forceinline__ bool sc_better(const SC &x, const SC &y) {
    if (x.s != y.s) return x.s > y.s;
    return x.id < y.id;
}

__device__ __forceinline__ SC sc_none() {
    SC c;
    c.s = -__builtin_huge_val();
    c.id = kNone;
    c.pad = 0;
    return c;
}

// Bitonic sort of n (a power of two) LDS entries, best first (whole block;
// ends with a barrier).
__device__ void sort_best_first(SC *c, uint32_t n) {
    for (uint32_t k = 2; k <= n; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
                const uint32_t p = i ^ j;
                if (p > i) {
                    const SC x = c[i], y = c[p];
                    const bool up = (i & k) == 0;
                    if (up ? sc_better(y, x) : sc_better(x, y)) {
                        c[i] = y;
                        c[p] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Order-preserving 64-bit key of a double (larger score, larger key).
__device__ __forceinline__ uint64_t dkey(double x) {
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

struct SelShared {
    uint32_t hist[256];
    uint32_t bin;     // the digit chosen by the last radix step
    uint32_t inbin;   // entries (matching the prefix) in that digit's bin
    uint32_t need;    // entries still to take among those matching the prefix
    uint32_t nsel;    // output slots used
    uint32_t neq;     // entries taken at the final key and id
};

// One step of a radix select over the values value(i, v) (i < n; entries
// for which value() returns false take no part) that match the prefix: the
// 8-bit digit at `shift` at which the count from the best end (the largest
// values when `largest`, else the smallest) reaches ss->need.  Sets ss->bin
// and ss->inbin, and lowers ss->need by the entries of better digits.
// Whole block; ends with a barrier.
template <class V, class F>
__device__ void radix_step(SelShared *ss, uint32_t n, F value, V prefix, V pmask, int shift, bool largest) {
    for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) ss->hist[i] = 0;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        V v;
        if (value(i, v) && (v & pmask) == prefix) atomicAdd(&ss->hist[static_cast<uint32_t>(v >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < static_cast<uint32_t>(kWave)) {
        // best-first position j = 0..255 is bin 255 - j (largest) or j;
        // lane l holds positions 4l..4l+3
        const uint32_t lane = threadIdx.x;
        uint32_t h[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t j = 4 * lane + k;
            h[k] = ss->hist[largest ? 255 - j : j];
        }
        const uint32_t own = h[0] + h[1] + h[2] + h[3];
        uint32_t incl = own;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t t = __shfl_up(incl, off, kWave);
            if (lane >= static_cast<uint32_t>(off)) incl += t;
        }
        uint32_t before = incl - own;
        const uint32_t need = ss->need;
        if (before < need && need <= incl) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (before + h[k] >= need) {
                    const uint32_t j = 4 * lane + k;
                    ss->bin = largest ? 255 - j : j;
                    ss->inbin = h[k];
                    ss->need = need - before;
                    break;
                }
                before += h[k];
            }
        }
    }
    __syncthreads();
}

// The best K2 of n entries get(i, e) under (score descending, id
// ascending), sorted best first into out[0..K2) (sentinels past the last
// when n < K2).  A radix select on the scores' 64-bit order keys finds the
// K2-th key; when several entries share it, a second radix select on the ids
// picks the smallest among them (equal entries are interchangeable).  Only
// the K2 chosen entries are then sorted.  Whole block; ends with a barrier.
template <class G>
__device__ void select_best(SelShared *ss, uint32_t n, uint32_t K2, G get, SC *out) {
    uint64_t prefix = 0, pmask = 0;
    uint32_t idprefix = 0, idmask = 0;
    bool all = n <= K2, done = false, iddone = false;
    if (threadIdx.x == 0) {
        ss->need = K2;
        ss->nsel = 0;
        ss->neq = 0;
    }
    __syncthreads();
    if (!all) {
        auto key = [&](uint32_t i, uint64_t &v) {
            SC e;
            get(i, e);
            v = dkey(e.s);
            return true;
        };
        for (int shift = 56; shift >= 0 && !done; shift -= 8) {
            radix_step<uint64_t>(ss, n, key, prefix, pmask, shift, true);
            prefix |= static_cast<uint64_t>(ss->bin) << shift;
            pmask |= 0xFFull << shift;
            done = ss->inbin == ss->need;   // the whole bin is taken
        }
        if (!done) {
            // entries at the K2-th key: the smallest ids
            auto tie_id = [&](uint32_t i, uint32_t &v) {
                SC e;
                get(i, e);
                v = e.id;
                return dkey(e.s) == prefix;
            };
            for (int shift = 24; shift >= 0 && !iddone; shift -= 8) {
                radix_step<uint32_t>(ss, n, tie_id, idprefix, idmask, shift, false);
                idprefix |= ss->bin << shift;
                idmask |= 0xFFu << shift;
                iddone = ss->inbin == ss->need;
            }
        }
    }
    const uint32_t need_eq = ss->need;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        SC e;
        get(i, e);
        bool take = all;
        if (!all) {
            const uint64_t v = dkey(e.s) & pmask;
            if (v > prefix) take = true;
            else if (v == prefix) {
                if (done) take = true;
                else {
                    const uint32_t id = e.id & idmask;
                    if (id < idprefix || (id == idprefix && iddone)) take = true;
                    else if (id == idprefix) take = atomicAdd(&ss->neq, 1u) < need_eq;
                }
            }
        }
        if (take) {
            const uint32_t slot = atomicAdd(&ss->nsel, 1u);
            if (slot < K2) out[slot] = e;   // exactly K2 are taken; the guard keeps LDS writes in bounds
        }
    }
    __syncthreads();
    for (uint32_t i = min(ss->nsel, K2) + threadIdx.x; i < K2; i += blockDim.x) out[i] = sc_none();
    __syncthreads();
    sort_best_first(out, K2);
}

#pragma clang fp contract(off)
// FP64 TransE-L1 score of candidate c against the anchor (head row h and
// relation row r held in LDS as FP64 sums h + r, formed in FP64 as the
// definition does).
template <bool BF16>
__device__ __forceinline__ double scan_score(const double *anchor, const void *X, uint32_t c, uint32_t d,
                                             double gamma) {
    double acc = 0.0;
    if (BF16) {
        const uint16_t *row = static_cast<const uint16_t *>(X) + static_cast<size_t>(c) * d;
        for (uint32_t i = 0; i < d; i += 8) {
            const uint4 u = *reinterpret_cast<const uint4 *>(row + i);
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                acc += fabs(anchor[i + 2 * k] - static_cast<double>(bf16_to_f32(w[k] & 0xFFFFu)));
                acc += fabs(anchor[i + 2 * k + 1] - static_cast<double>(bf16_to_f32(w[k] >> 16)));
            }
        }
    } else {
        const float *row = static_cast<const float *>(X) + static_cast<size_t>(c) * d;
        for (uint32_t i = 0; i < d; i += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(row + i);
            acc += fabs(anchor[i] - static_cast<double>(v.x));
            acc += fabs(anchor[i + 1] - static_cast<double>(v.y));
            acc += fabs(anchor[i + 2] - static_cast<double>(v.z));
            acc += fabs(anchor[i + 3] - static_cast<double>(v.w));
        }
    }
    return gamma - acc;
}
// The same score from a row already in registers (D values).
template <int D>
__device__ __forceinline__ double scan_score_row(const double *anchor, const float (&row)[D], double gamma) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) acc += fabs(anchor[i] - static_cast<double>(row[i]));
    return gamma - acc;
}

// Loads one candidate row of D values (D a multiple of 8) into registers.
template <bool BF16, int D>
__device__ __forceinline__ void scan_load_row(const void *X, uint32_t c, float (&row)[D]) {
    if (BF16) {
        const uint4 *p = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(X) + static_cast<size_t>(c) * D);
#pragma unroll
        for (int j = 0; j < D / 8; ++j) {
            const uint4 u = p[j];
            const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                row[8 * j + 2 * k] = bf16_to_f32(w[k] & 0xFFFFu);
                row[8 * j + 2 * k + 1] = bf16_to_f32(w[k] >> 16);
            }
        }
    } else {
        const float4 *p = reinterpret_cast<const float4 *>(static_cast<const float *>(X) + static_cast<size_t>(c) * D);
#pragma unroll
        for (int j = 0; j < D / 4; ++j) {
            const float4 v = p[j];
            row[4 * j] = v.x;
            row[4 * j + 1] = v.y;
            row[4 * j + 2] = v.z;
            row[4 * j + 3] = v.w;
        }
    }
}
#pragma clang fp contract(on)

struct ScanArgs {
    const void *X, *Y;
    uint32_t n, R, d, nq;
    const uint32_t *head, *rel;
    uint32_t rel_default;
    const uint32_t *cand;
    uint32_t ncand, cand_stride, K, K2, nblk;
    double gamma;
    SC *partial;              // [nq][nblk][K2]
    uint32_t *out_id;
    double *out_s;
    uint32_t *out_status;
};

// grid (nblk, nq): chunk blockIdx.x of query blockIdx.y.  D: the embedding
// dimension when it is small enough for a thread to hold all of its
// candidates' rows (their loads then all in flight together), else 0.
template <bool BF16, int D>
__global__ __launch_bounds__(kScanThreads) void scan_chunk_kernel(ScanArgs A) {
    __shared__ SC c[kChunk];
    __shared__ SC best[kMaxScanK];
    __shared__ SelShared ss;
    __shared__ double anchor[kMaxScanDim];
    __shared__ uint32_t bad;
    const uint32_t q = blockIdx.y, b = blockIdx.x;
    const uint32_t h = A.head[q];
    const uint32_t r = A.rel ? A.rel[q] : A.rel_default;
    const bool qok = h < A.n && r < A.R;
    if (threadIdx.x == 0) bad = 0;
    if (qok) {
        for (uint32_t i = threadIdx.x; i < A.d; i += kScanThreads)
            anchor[i] = static_cast<double>(load1<BF16>(A.X, static_cast<size_t>(h) * A.d + i)) +
                        static_cast<double>(load1<BF16>(A.Y, static_cast<size_t>(r) * A.d + i));
    }
    __syncthreads();
    const uint32_t *cand = A.cand + static_cast<size_t>(q) * A.cand_stride;
    const uint32_t base = b * kChunk;
    uint32_t ids[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        const uint32_t i = base + k * kScanThreads + threadIdx.x;
        ids[k] = (qok && i < A.ncand) ? cand[i] : kNone;
    }
    uint32_t nbad = 0;
    if constexpr (D > 0) {
        float rows[kScanPer][D > 0 ? D : 1];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) scan_load_row<BF16, D>(A.X, ids[k] < A.n ? ids[k] : 0u, rows[k]);
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            SC e = sc_none();
            if (ids[k] < A.n) {
                e.s = scan_score_row<D>(anchor, rows[k], A.gamma);
                e.id = ids[k];
            } else if (ids[k] != kNone) {
                ++nbad;   // an id out of range: skipped, reported in the status
            }
            c[k * kScanThreads + threadIdx.x] = e;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            SC e = sc_none();
            if (ids[k] < A.n) {
                e.s = scan_score<BF16>(anchor, A.X, ids[k], A.d, A.gamma);
                e.id = ids[k];
            } else if (ids[k] != kNone) {
                ++nbad;   // an id out of range: skipped, reported in the status
            }
            c[k * kScanThreads + threadIdx.x] = e;
        }
    }
    if (nbad) atomicAdd(&bad, nbad);
    __syncthreads();
    select_best(&ss, kChunk, A.K2, [&](uint32_t i, SC &e) { e = c[i]; }, best);
    SC *out = A.partial + (static_cast<size_t>(q) * A.nblk + b) * A.K2;
    for (uint32_t i = threadIdx.x; i < A.K2; i += kScanThreads) out[i] = best[i];
    if (threadIdx.x == 0 && A.out_status) {
        if (!qok && b == 0) atomicOr(&A.out_status[q], MHR_Q_BAD_ID);
        if (bad) atomicOr(&A.out_status[q], MHR_Q_BAD_ID);
    }
}

// Clears the status words before the chunk kernel sets bits.
__global__ void scan_status_clear_kernel(uint32_t *st, uint32_t nq) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nq) st[q] = 0;
}

// grid (nq): the best K over the query's chunk lists (nblk * K2 entries,
// read from memory in each radix pass).
__global__ __launch_bounds__(kScanThreads) void scan_merge_kernel(ScanArgs A) {
    __shared__ SC best[kMaxScanK];
    __shared__ SelShared ss;
    const uint32_t q = blockIdx.x;
    const uint32_t total = A.nblk * A.K2;
    const SC *in = A.partial + static_cast<size_t>(q) * total;
    select_best(&ss, total, A.K2, [&](uint32_t i, SC &e) { e = in[i]; }, best);
    for (uint32_t i = threadIdx.x; i < A.K; i += kScanThreads) {
        A.out_id[static_cast<size_t>(q) * A.K + i] = best[i].id;
        A.out_s[static_cast<size_t>(q) * A.K + i] = best[i].s;
    }
}

uint32_t scan_blocks(uint32_t ncand) { return std::max<uint32_t>(1u, (ncand + kChunk - 1) / kChunk); }

size_t scan_ws_bytes(uint32_t nq, uint32_t ncand, uint32_t K) {
    return static_cast<size_t>(nq) * scan_blocks(ncand) * next_pow2(K) * sizeof(SC);
}

mhr_status scan_impl(mhr_dtype dtype, uint32_t dim, const void *entity, const void *relation, uint32_t n,
                     uint32_t R, uint32_t nq, const uint32_t *head, const uint32_t *rel, uint32_t rel_default,
                     const uint32_t *cand, uint32_t ncand, uint32_t cand_stride, uint32_t K, float gamma,
                     uint32_t *out_id, double *out_s, uint32_t *out_status, void *ws, size_t ws_bytes,
                     hipStream_t st) {
    MHR_ARG_CHECK(dtype == MHR_DTYPE_F32 || dtype == MHR_DTYPE_BF16, "scan: dtype must be F32 or BF16");
    MHR_ARG_CHECK(dim >= 8 && dim <= kMaxScanDim && dim % 8 == 0, "scan: dim must be a multiple of 8 in [8, 512]");
    MHR_ARG_CHECK(K >= 1 && K <= kMaxScanK, "scan: K must be in [1, 256]");
    MHR_ARG_CHECK(gamma == gamma && gamma <= 3.0e38f && gamma >= -3.0e38f, "scan: gamma must be finite");
    if (nq == 0) return MHR_OK;
    MHR_ARG_CHECK(entity && relation && head && out_id && out_s && ws, "scan: null pointer");
    MHR_ARG_CHECK(ncand == 0 || cand, "scan: null candidate list");
    MHR_ARG_CHECK((reinterpret_cast<uintptr_t>(entity) & 15u) == 0, "scan: the entity table must be 16-byte aligned");
    if (ws_bytes < scan_ws_bytes(nq, ncand, K)) {
        set_error("scan: workspace too small");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    ScanArgs A{};
    A.X = entity;
    A.Y = relation;
    A.n = n;
    A.R = R;
    A.d = dim;
    A.nq = nq;
    A.head = head;
    A.rel = rel;
    A.rel_default = rel_default;
    A.cand = cand;
    A.ncand = ncand;
    A.cand_stride = cand_stride;
    A.K = K;
    A.K2 = next_pow2(K);
    A.nblk = scan_blocks(ncand);
    A.gamma = static_cast<double>(gamma);
    A.partial = static_cast<SC *>(ws);
    A.out_id = out_id;
    A.out_s = out_s;
    A.out_status = out_status;
    if (out_status) hipLaunchKernelGGL(scan_status_clear_kernel, dim3((nq + 255) / 256), dim3(256), 0, st, out_status, nq);
    const dim3 grid(A.nblk, nq);
    const bool bf = dtype == MHR_DTYPE_BF16;
    if (dim == 8) {
        if (bf) hipLaunchKernelGGL((scan_chunk_kernel<true, 8>), grid, dim3(kScanThreads), 0, st, A);
        else hipLaunchKernelGGL((scan_chunk_kernel<false, 8>), grid, dim3(kScanThreads), 0, st, A);
    } else if (dim == 16) {
        if (bf) hipLaunchKernelGGL((scan_chunk_kernel<true, 16>), grid, dim3(kScanThreads), 0, st, A);
        else hipLaunchKernelGGL((scan_chunk_kernel<false, 16>), grid, dim3(kScanThreads), 0, st, A);
    } else {
        if (bf) hipLaunchKernelGGL((scan_chunk_kernel<true, 0>), grid, dim3(kScanThreads), 0, st, A);
        else hipLaunchKernelGGL((scan_chunk_kernel<false, 0>), grid, dim3(kScanThreads), 0, st, A);
    }
    hipLaunchKernelGGL(scan_merge_kernel, dim3(nq), dim3(kScanThreads), 0, st, A);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

}  // namespace
}  // namespace mhr

using namespace mhr;

extern "C" mhr_status mhr_scan_workspace_size(uint32_t nq, uint32_t ncand, uint32_t k, size_t *bytes) {
    MHR_ARG_CHECK(bytes != nullptr, "mhr_scan_workspace_size: null argument");
    MHR_ARG_CHECK(k >= 1 && k <= kMaxScanK, "scan: K must be in [1, 256]");
    *bytes = scan_ws_bytes(nq, ncand, k);
    return MHR_OK;
}

extern "C" mhr_status mhr_scan_topk(mhr_dtype dtype, uint32_t dim, const void *entity, const void *relation,
                                    uint32_t num_entities, uint32_t num_relations, uint32_t nq, const uint32_t *head,
                                    const uint32_t *rel, uint32_t rel_default, const uint32_t *cand, uint32_t ncand,
                                    uint32_t cand_stride, uint32_t k, float gamma, uint32_t *out_id, double *out_score,
                                    uint32_t *out_status, void *workspace, size_t ws_bytes, void *stream) {
    return scan_impl(dtype, dim, entity, relation, num_entities, num_relations, nq, head, rel, rel_default, cand,
                     ncand, cand_stride, k, gamma, out_id, out_score, out_status, workspace, ws_bytes,
                     static_cast<hipStream_t>(stream));
}

extern "C" mhr_status mhr_scan_pipeline_workspace_size(uint32_t npipe, uint32_t npersons, uint32_t nuniv,
                                                       uint32_t k, size_t *bytes) {
    MHR_ARG_CHECK(bytes != nullptr, "mhr_scan_pipeline_workspace_size: null argument");
    MHR_ARG_CHECK(k >= 1 && k <= kMaxScanK, "scan: K must be in [1, 256]");
    *bytes = std::max({scan_ws_bytes(npipe, npersons, k), scan_ws_bytes(npipe, k, k),
                       scan_ws_bytes(npipe * k, nuniv, k)});
    return MHR_OK;
}

extern "C" mhr_status mhr_scan_pipeline(mhr_dtype dtype, uint32_t dim, const void *entity, const void *relation,
                                        uint32_t num_entities, uint32_t num_relations, uint32_t npipe,
                                        const uint32_t *award, const uint32_t *field, uint32_t r_award,
                                        uint32_t r_works, uint32_t r_affil, const uint32_t *persons,
                                        uint32_t npersons, const uint32_t *universities, uint32_t nuniv, uint32_t k,
                                        float gamma, uint32_t *hop1_id, double *hop1_score, uint32_t *hop2_id,
                                        double *hop2_score, uint32_t *hop3_id, double *hop3_score, void *workspace,
                                        size_t ws_bytes, void *stream) {
    MHR_ARG_CHECK(npipe == 0 || (award && field && hop1_id && hop1_score && hop2_id && hop2_score && hop3_id &&
                                 hop3_score),
                  "mhr_scan_pipeline: null pointer");
    MHR_ARG_CHECK(static_cast<uint64_t>(npipe) * k < (1ull << 31), "mhr_scan_pipeline: too many pipelines");
    hipStream_t st = static_cast<hipStream_t>(stream);
    // hop 1: persons against award + r_award
    mhr_status rc = scan_impl(dtype, dim, entity, relation, num_entities, num_relations, npipe, award, nullptr,
                              r_award, persons, npersons, 0, k, gamma, hop1_id, hop1_score, nullptr, workspace,
                              ws_bytes, st);
    if (rc != MHR_OK) return rc;
    // hop 2: each pipeline's K persons against field + r_works (absent
    // entries, when there are fewer than K persons, are skipped)
    rc = scan_impl(dtype, dim, entity, relation, num_entities, num_relations, npipe, field, nullptr, r_works, hop1_id,
                   k, k, k, gamma, hop2_id, hop2_score, nullptr, workspace, ws_bytes, st);
    if (rc != MHR_OK) return rc;
    // hop 3: each ranked person against every university
    return scan_impl(dtype, dim, entity, relation, num_entities, num_relations, npipe * k, hop2_id, nullptr, r_affil,
                     universities, nuniv, 0, k, gamma, hop3_id, hop3_score, nullptr, workspace, ws_bytes, st);
}
