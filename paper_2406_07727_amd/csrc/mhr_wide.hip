// Wide-relation graphs: three-hop top-K path search over knowledge graphs
// with up to 65,535 relations, the scale of the paper's experiments (section
// 4.1: 91.23M entities, 1,387 relations, 601.06M triples, 8-dimensional
// TransE embeddings).
//
// Layout (device memory, per direction):
//   row_ptr  uint32[n + 1]
//   col      uint32[m]   neighbour id of each distinct triple
//   rel      uint16[m]   its relation
// Rows are sorted by (neighbour, relation), so the relations joining one
// pair of vertices form a run of consecutive entries.
//
// Scoring: TransE-L1 (section 3.3) in FP64, w(u, r, v) = gamma -
// sum_i |(X[u,i] + Y[r,i]) - X[v,i]| accumulated in ascending i, and the
// path score S = w1 + w2 + w3 rounded once (the correctly rounded sum of
// the three FP64 weights).  Every step is a fixed sequence of correctly
// rounded FP64 operations, so scores are exact functions of the inputs and
// the ranking (S descending, then a, b, r1, r2, r3 ascending; section 3.1)
// needs no rescoring band.
//
// Query pipeline (one batch):
//   plan      per query: both rows, the scan cost of each direction
//             (sum of the scanned rows' lengths over distinct frontier
//             vertices), the cheaper direction, its tile count
//   offsets   exclusive scans over the batch (one workgroup)
//   table     per query: the distinct list-side vertices with their
//             scan-row prefix sums, and the tile map
//   gather    persistent workgroups take tiles of scan entries, look each
//             scanned neighbour up in the probe row (an LDS copy when it is
//             short, else the neighbour's own row), score the paths through
//             every match (edge weights computed where used) and keep
//             the tile's best K in LDS (staging buffer plus bitonic merges,
//             pruned by the query's best known K-th score)
//   merge     one wave per query: K-way merge of the tiles' sorted lists
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "mhr.h"
#include "mhr_device.h"
#include "mhr_internal.h"

#pragma clang fp contract(off)

struct mhr_wide_graph {
    uint32_t n = 0, R = 0;
    uint32_t id_bits = 1, rel_bits = 1;
    uint64_t m = 0;   // distinct triples
    struct Dir {
        uint32_t *row_ptr = nullptr;
        uint32_t *col = nullptr;
        uint16_t *rel = nullptr;
        // per vertex v: the scan cost of v's row as a frontier (the summed
        // row lengths, in this CSR, of the distinct neighbours of v) and the
        // number of those neighbours whose row is nonempty; both < 2^32
        // since each is at most the entry count
        uint32_t *cost = nullptr;
        uint32_t *ndist = nullptr;
        uint32_t max_degree = 0;
    } out, in;
    const void *X = nullptr;
    const void *Y = nullptr;
    uint32_t dim = 0;
    mhr_dtype dtype = MHR_DTYPE_F32;
    double gamma = 1.0;
    uint64_t device_bytes = 0;
    int device = 0;
};

namespace mhr {
namespace {

__host__ __device__ inline uint32_t wcdiv(uint64_t a, uint64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

struct WBuf {
    void *p = nullptr;
    ~WBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1); }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------
// LSD radix sort of (key, value) pairs, 8 bits per pass, stable.
// ---------------------------------------------------------------------------
constexpr int kWSortBlock = 256;
constexpr int kWSortItems = 16;
constexpr int kWSortTile = kWSortBlock * kWSortItems;
constexpr int kWBins = 256;

template <class K>
__global__ void wsort_hist_kernel(const K *keys, uint64_t n, int shift, uint32_t ntiles, uint32_t *counts) {
    __shared__ uint32_t hist[kWBins];
    for (int i = threadIdx.x; i < kWBins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kWSortTile;
    for (int k = 0; k < kWSortItems; ++k) {
        const uint64_t idx = base + static_cast<uint64_t>(k) * kWSortBlock + threadIdx.x;
        if (idx < n) atomicAdd(&hist[static_cast<uint32_t>(keys[idx] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kWBins; d += blockDim.x) counts[static_cast<uint64_t>(d) * ntiles + blockIdx.x] = hist[d];
}

// Items keep their input order within a digit: each row of 256 items is
// ranked by matching digits across the wave (eight ballots), then by the
// counts of the waves before it.
template <class K, class V>
__global__ void wsort_scatter_kernel(const K *keys, const V *vals, K *okeys, V *ovals, uint64_t n, int shift,
                                     uint32_t ntiles, const uint32_t *offsets) {
    constexpr int kWaves = kWSortBlock / kWave;
    __shared__ uint32_t base_off[kWBins];
    __shared__ uint32_t wcnt[kWaves][kWBins];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    for (int d = threadIdx.x; d < kWBins; d += blockDim.x)
        base_off[d] = offsets[static_cast<uint64_t>(d) * ntiles + blockIdx.x];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const uint64_t tile = static_cast<uint64_t>(blockIdx.x) * kWSortTile;
    for (int k = 0; k < kWSortItems; ++k) {
        for (int i = threadIdx.x; i < kWaves * kWBins; i += blockDim.x) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        const uint64_t idx = tile + static_cast<uint64_t>(k) * kWSortBlock + threadIdx.x;
        const bool valid = idx < n;
        const K key = valid ? keys[idx] : K(0);
        const V val = valid ? vals[idx] : V(0);
        const uint32_t dg = static_cast<uint32_t>(key >> shift) & 0xFFu;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot(((dg >> b) & 1u) != 0);
            peers &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && rank == 0) wcnt[wave][dg] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += wcnt[w][dg];
            const uint32_t dst = base_off[dg] + before + rank;
            okeys[dst] = key;
            ovals[dst] = val;
        }
        __syncthreads();
        for (int d = threadIdx.x; d < kWBins; d += blockDim.x) {
            uint32_t s = 0;
            for (int w = 0; w < kWaves; ++w) s += wcnt[w][d];
            base_off[d] += s;
        }
        __syncthreads();
    }
}

// Sorts n pairs by the low `bits` bits of the keys; on return keys / vals
// point at the sorted arrays (the other buffers hold scratch).
template <class K, class V>
mhr_status wsort_pairs(K *&keys, V *&vals, K *&tk, V *&tv, uint64_t n, int bits, hipStream_t st) {
    if (n <= 1) return MHR_OK;
    const uint32_t ntiles = wcdiv(n, kWSortTile);
    const uint64_t nc = static_cast<uint64_t>(ntiles) * kWBins;
    WBuf counts, scratch;
    MHR_HIP_TRY(counts.alloc(nc * sizeof(uint32_t)));
    MHR_HIP_TRY(scratch.alloc((wcdiv(nc, 2048) + 1) * sizeof(uint32_t)));
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(wsort_hist_kernel<K>, dim3(ntiles), dim3(kWSortBlock), 0, st, keys, n, shift, ntiles,
                           counts.as<uint32_t>());
        mhr_status s = device_exclusive_scan(counts.as<uint32_t>(), counts.as<uint32_t>(), nc, nullptr,
                                             scratch.as<uint32_t>(), st);
        if (s != MHR_OK) return s;
        hipLaunchKernelGGL((wsort_scatter_kernel<K, V>), dim3(ntiles), dim3(kWSortBlock), 0, st, keys, vals, tk, tv,
                           n, shift, ntiles, counts.as<uint32_t>());
        MHR_HIP_TRY(hipGetLastError());
        std::swap(keys, tk);
        std::swap(vals, tv);
    }
    MHR_HIP_TRY(hipStreamSynchronize(st));
    return MHR_OK;
}

// ---------------------------------------------------------------------------
// Ingest
// ---------------------------------------------------------------------------
// key = (other endpoint << rel_bits) | relation, value = row vertex
__global__ void wide_keys_kernel(const uint32_t *head, const uint32_t *rel, const uint32_t *tail, uint64_t m,
                                 uint32_t n, uint32_t R, int rel_bits, int reverse, uint64_t *keys, uint32_t *rows,
                                 uint32_t *err) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    uint32_t u = head[i], r = rel[i], v = tail[i];
    if (u >= n || v >= n || r >= R) {
        atomicOr(err, 1u);
        u = v = r = 0;
    }
    rows[i] = reverse ? v : u;
    keys[i] = (static_cast<uint64_t>(reverse ? u : v) << rel_bits) | r;
}

__global__ void wide_flags_kernel(const uint32_t *rows, const uint64_t *keys, uint64_t m, uint32_t *flag) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    flag[i] = (i == 0 || rows[i] != rows[i - 1] || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// Writes the distinct triples; row_ptr[x] for the rows from the previous
// triple's row + 1 up to this one start here.
__global__ void wide_fill_kernel(const uint32_t *rows, const uint64_t *keys, const uint32_t *flag,
                                 const uint32_t *pos, uint64_t m, int rel_bits, uint32_t n, uint32_t nd,
                                 uint32_t *row_ptr, uint32_t *col, uint16_t *rel) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t u = rows[i];
    if (i == m - 1)   // the rows after the last one end at nd (a duplicate may hold this slot)
        for (uint64_t x = static_cast<uint64_t>(u) + 1; x <= n; ++x) row_ptr[x] = nd;
    if (!flag[i]) return;
    const uint32_t p = pos[i];
    const uint64_t k = keys[i];
    col[p] = static_cast<uint32_t>(k >> rel_bits);
    rel[p] = static_cast<uint16_t>(k & ((1ull << rel_bits) - 1));
    const int64_t uprev = (i == 0) ? -1 : static_cast<int64_t>(rows[i - 1]);
    if (static_cast<int64_t>(u) != uprev)   // a new row starts a new triple
        for (int64_t x = uprev + 1; x <= static_cast<int64_t>(u); ++x) row_ptr[x] = p;
}

__global__ void wide_maxdeg_kernel(const uint32_t *row_ptr, uint32_t n, uint32_t *out) {
    uint32_t mx = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x)
        mx = max(mx, row_ptr[v + 1] - row_ptr[v]);
    for (int o = kWave / 2; o > 0; o >>= 1) mx = max(mx, static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), o, kWave)));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, mx);
}

__global__ void wide_cost_kernel(const uint32_t *row_ptr, const uint32_t *col, uint32_t n, uint32_t *cost,
                                 uint32_t *ndist);

mhr_status wide_build_direction(mhr_wide_graph *g, const mhr_graph_desc *d, int reverse, mhr_wide_graph::Dir &D,
                                hipStream_t st) {
    const uint64_t m = d->num_edges;
    const uint32_t n = g->n;
    WBuf kb, kt, vb, vt, err;
    MHR_HIP_TRY(kb.alloc(m * 8));
    MHR_HIP_TRY(kt.alloc(m * 8));
    MHR_HIP_TRY(vb.alloc(m * 4));
    MHR_HIP_TRY(vt.alloc(m * 4));
    MHR_HIP_TRY(err.alloc(4));
    MHR_HIP_TRY(hipMemsetAsync(err.p, 0, 4, st));
    uint64_t *keys = kb.as<uint64_t>(), *tkeys = kt.as<uint64_t>();
    uint32_t *rows = vb.as<uint32_t>(), *trows = vt.as<uint32_t>();
    if (m) {
        hipLaunchKernelGGL(wide_keys_kernel, dim3(wcdiv(m, 256)), dim3(256), 0, st, d->head, d->rel, d->tail, m, n,
                           g->R, static_cast<int>(g->rel_bits), reverse, keys, rows, err.as<uint32_t>());
        MHR_HIP_TRY(hipGetLastError());
    }
    uint32_t herr = 0;
    MHR_HIP_TRY(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipStreamSynchronize(st));
    if (herr) {
        set_error("edge list holds a vertex id >= num_vertices or a relation id >= num_relations");
        return MHR_ERR_BAD_EDGE;
    }
    // by (other endpoint, relation), then stably by row vertex
    mhr_status s = wsort_pairs<uint64_t, uint32_t>(keys, rows, tkeys, trows, m,
                                                   static_cast<int>(g->id_bits + g->rel_bits), st);
    if (s != MHR_OK) return s;
    s = wsort_pairs<uint32_t, uint64_t>(rows, keys, trows, tkeys, m, static_cast<int>(g->id_bits), st);
    if (s != MHR_OK) return s;
    WBuf flag, pos, scratch, total;
    MHR_HIP_TRY(flag.alloc(m * 4));
    MHR_HIP_TRY(pos.alloc(m * 4));
    MHR_HIP_TRY(scratch.alloc((wcdiv(m, 2048) + 1) * 4));
    MHR_HIP_TRY(total.alloc(4));
    if (m) {
        hipLaunchKernelGGL(wide_flags_kernel, dim3(wcdiv(m, 256)), dim3(256), 0, st, rows, keys, m,
                           flag.as<uint32_t>());
        MHR_HIP_TRY(hipGetLastError());
    }
    s = device_exclusive_scan(flag.as<uint32_t>(), pos.as<uint32_t>(), m, total.as<uint32_t>(),
                              scratch.as<uint32_t>(), st);
    if (s != MHR_OK) return s;
    uint32_t nd = 0;
    MHR_HIP_TRY(hipMemcpyAsync(&nd, total.p, 4, hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipStreamSynchronize(st));
    g->m = nd;
    MHR_HIP_TRY(hipMalloc(&D.row_ptr, (static_cast<size_t>(n) + 1) * 4));
    MHR_HIP_TRY(hipMalloc(&D.col, std::max<size_t>(nd, 1) * 4));
    MHR_HIP_TRY(hipMalloc(&D.rel, std::max<size_t>(nd, 1) * 2));
    g->device_bytes += (static_cast<uint64_t>(n) + 1) * 4 + static_cast<uint64_t>(nd) * 6;
    MHR_HIP_TRY(hipMemsetAsync(D.row_ptr, 0, (static_cast<size_t>(n) + 1) * 4, st));
    if (m) {
        hipLaunchKernelGGL(wide_fill_kernel, dim3(wcdiv(m, 256)), dim3(256), 0, st, rows, keys, flag.as<uint32_t>(),
                           pos.as<uint32_t>(), m, static_cast<int>(g->rel_bits), n, nd, D.row_ptr, D.col, D.rel);
        MHR_HIP_TRY(hipGetLastError());
    }
    WBuf mx;
    MHR_HIP_TRY(mx.alloc(4));
    MHR_HIP_TRY(hipMemsetAsync(mx.p, 0, 4, st));
    hipLaunchKernelGGL(wide_maxdeg_kernel, dim3(std::min<uint32_t>(wcdiv(n, 256), 4096)), dim3(256), 0, st, D.row_ptr,
                       n, mx.as<uint32_t>());
    MHR_HIP_TRY(hipGetLastError());
    MHR_HIP_TRY(hipMemcpyAsync(&D.max_degree, mx.p, 4, hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipMalloc(&D.cost, std::max<size_t>(n, 1) * 4));
    MHR_HIP_TRY(hipMalloc(&D.ndist, std::max<size_t>(n, 1) * 4));
    g->device_bytes += static_cast<uint64_t>(n) * 8;
    hipLaunchKernelGGL(wide_cost_kernel, dim3(std::min<uint32_t>(wcdiv(n, 4), 65535)), dim3(256), 0, st, D.row_ptr,
                       D.col, n, D.cost, D.ndist);
    MHR_HIP_TRY(hipGetLastError());
    MHR_HIP_TRY(hipStreamSynchronize(st));
    return MHR_OK;
}

void wide_free_dir(mhr_wide_graph::Dir &D) {
    if (D.row_ptr) (void)hipFree(D.row_ptr);
    if (D.col) (void)hipFree(D.col);
    if (D.rel) (void)hipFree(D.rel);
    if (D.cost) (void)hipFree(D.cost);
    if (D.ndist) (void)hipFree(D.ndist);
    D = mhr_wide_graph::Dir();
}

// ---------------------------------------------------------------------------
// Scores
// ---------------------------------------------------------------------------
template <bool BF16>
__device__ __forceinline__ double wide_weight(const void *X, const void *Y, uint32_t d, double gamma, uint32_t u,
                                              uint32_t r, uint32_t v) {
    double acc = 0.0;
    const size_t bu = static_cast<size_t>(u) * d, br = static_cast<size_t>(r) * d, bv = static_cast<size_t>(v) * d;
    for (uint32_t i = 0; i < d; ++i) {
        const double x = static_cast<double>(load1<BF16>(X, bu + i));
        const double y = static_cast<double>(load1<BF16>(Y, br + i));
        const double z = static_cast<double>(load1<BF16>(X, bv + i));
        acc += fabs((x + y) - z);
    }
    return gamma - acc;
}

__device__ __forceinline__ void two_sum_d(double a, double b, double &s, double &e) {
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// x + y rounded to odd: the neighbour of the exact sum whose last significand
// bit is 1 when the sum is inexact (Boldo and Melquiond, "Emulation of FMA
// and correctly rounded sums: proved algorithms using rounding to odd",
// IEEE Trans. Computers 57(4), 2008).
__device__ __forceinline__ double add_round_odd(double x, double y) {
    double s, e;
    two_sum_d(x, y, s, e);
    if (e != 0.0) {
        long long bits = __double_as_longlong(s);
        if ((bits & 1) == 0) bits += ((s > 0.0) == (e > 0.0)) ? 1 : -1;   // step toward the exact sum
        s = __longlong_as_double(bits);
    }
    return s;
}

// a + b + c rounded once to nearest (ties to even), by the same paper's
// algorithm: b + c and a + (b + c)_hi are split exactly, the two error terms
// are added rounded to odd, and the final addition rounds once.
__device__ __forceinline__ double sum3_rn(double a, double b, double c) {
    double uh, ul, th, tl;
    two_sum_d(b, c, uh, ul);
    two_sum_d(a, uh, th, tl);
    return th + add_round_odd(tl, ul);
}

// Order-preserving map of a double's bits to uint64 (larger double, larger
// key), for the atomic maximum of the per-query thresholds.
__device__ __forceinline__ uint64_t dkey(double x) {
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_inv(uint64_t k) {
    const uint64_t b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double(static_cast<long long>(b));
}

struct WCand {
    double s;
    uint32_t a, b;
    uint16_t r1, r2, r3, pad;
};

__device__ __forceinline__ WCand wcand_sentinel() {
    WCand c;
    c.s = -INFINITY;
    c.a = c.b = 0xFFFFFFFFu;
    c.r1 = c.r2 = c.r3 = 0xFFFFu;
    c.pad = 0;
    return c;
}

// x ranks before y: higher score, then smaller a, b, r1, r2, r3
__device__ __forceinline__ bool wbetter(const WCand &x, const WCand &y) {
    if (x.s != y.s) return x.s > y.s;
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    if (x.r1 != y.r1) return x.r1 < y.r1;
    if (x.r2 != y.r2) return x.r2 < y.r2;
    return x.r3 < y.r3;
}

// ---------------------------------------------------------------------------
// Query kernels
// ---------------------------------------------------------------------------
constexpr int kWBlock = 256;
constexpr uint32_t kWTile = 16384;      // scan entries per tile
constexpr uint32_t kWSub = 512;         // scan entries per staged sub-chunk
constexpr uint32_t kWProbeLds = 2048;   // probe rows up to this length may be copied to LDS
constexpr uint32_t kWPathsMin = 512;    // candidate buffer (list + staging) is max(512, 2K) rounded up to 2^j

struct WPlan {
    uint32_t s, t, k, status;
    uint32_t dir;                   // 1: forward (list out(s), scan out-rows, probe in(t)); 0: backward
    uint32_t list_beg, list_len;    // list row in the list CSR
    uint32_t probe_beg, probe_len;  // probe row in the probe CSR
    uint32_t out_len, in_len;       // |out(s)|, |in(t)| entries
    uint32_t nd;                    // distinct list vertices with a nonempty scan row
    uint32_t ntiles, tile_base;
    uint64_t cost;                  // scan entries
    uint64_t tab_off;
    uint32_t nchunks, chunk_base;   // kWChunk-entry chunks of the list row (table construction)
};

struct WTotals {
    unsigned long long nd, tiles, ctr, chunks;
};

struct WRow {
    uint64_t prefix;   // scan entries of the earlier rows
    uint32_t x, scan_beg, run_beg, run_len;
};

struct WArgs {
    const uint32_t *out_rp, *out_col, *in_rp, *in_col;
    const uint32_t *out_cost, *out_nd, *in_cost, *in_nd;   // per-vertex frontier scan costs (mhr_wide_graph::Dir)
    ulonglong2 *cpart;  // per list chunk: (distinct vertices, scan entries), then their exclusive prefix in the query
    const uint16_t *out_rel, *in_rel;
    const void *X, *Y;
    uint32_t n, d, nq, k_max;
    double gamma;
    WPlan *plans;
    WTotals *tot;
    uint64_t *gthr;     // per query: order key of the best known K-th score
    uint64_t *qtotal;   // per query: paths counted
    uint64_t *qmatch;   // per query: scanned entries found in the probe row
    WRow *tab;
    uint32_t *tile_q, *tile_n, *head;
    WCand *slots;       // [tile][k_max]
};

template <class T>
__device__ inline T wblock_sum(T v, T *red) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < static_cast<int>(blockDim.x / kWave); ++i) s += red[i];
    return s;
}

// Exclusive scan over the block (one value per thread); *total gets the sum.
template <class T>
__device__ inline T wblock_excl(T v, T *red, T *total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    T x = v;
    for (int o = 1; o < kWave; o <<= 1) {
        const T y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == kWave - 1) red[w] = x;
    __syncthreads();
    T base = 0, all = 0;
    for (int i = 0; i < static_cast<int>(blockDim.x / kWave); ++i) {
        if (i < w) base += red[i];
        all += red[i];
    }
    *total = all;
    return base + x - v;
}

constexpr uint32_t kWSeg = 16;                 // row entries per thread per planning step
constexpr uint32_t kWChunk = kWBlock * kWSeg;  // row entries per planning step

// Over the entries [i0, min(i0 + kWSeg, end)) of the row [beg, end): the
// scan lengths (rows of the same CSR) of the distinct vertices starting a
// run there, and how many of those are nonempty.
// All loads of the segment are issued together (ids first, then the row
// bounds of the run starts), so a thread waits for memory twice per segment.
__device__ __forceinline__ void seg_cost(const uint32_t *col, const uint32_t *rp, uint32_t beg, uint32_t end,
                                         uint32_t i0, unsigned long long &cost, unsigned long long &nd) {
    if (i0 >= end) return;
    uint32_t xs[kWSeg + 1];
    xs[0] = i0 > beg ? col[i0 - 1] : 0xFFFFFFFFu;
#pragma unroll
    for (uint32_t j = 0; j < kWSeg; ++j) xs[j + 1] = (i0 + j < end) ? col[i0 + j] : 0xFFFFFFFFu;
    uint32_t lo[kWSeg], hi[kWSeg];
#pragma unroll
    for (uint32_t j = 0; j < kWSeg; ++j) {
        const bool first = i0 + j < end && xs[j + 1] != xs[j];
        lo[j] = first ? rp[xs[j + 1]] : 0u;
        hi[j] = first ? rp[xs[j + 1] + 1] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kWSeg; ++j) {
        const uint32_t dg = hi[j] - lo[j];
        cost += dg;
        nd += dg ? 1 : 0;
    }
}

// One wave per row v: over the runs of equal neighbours x in v's row (16
// entries per lane per step, as seg_cost reads them), the sum of
// row_ptr[x + 1] - row_ptr[x] and the count of nonempty ones.
__global__ void wide_cost_kernel(const uint32_t *row_ptr, const uint32_t *col, uint32_t n, uint32_t *cost,
                                 uint32_t *ndist) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t waves = gridDim.x * (blockDim.x / kWave);
    for (uint32_t v = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; v < n; v += waves) {
        const uint32_t b = row_ptr[v], e = row_ptr[v + 1];
        unsigned long long c = 0, nd = 0;
        for (uint32_t i0 = b + lane * kWSeg; i0 < e; i0 += kWave * kWSeg) seg_cost(col, row_ptr, b, e, i0, c, nd);
        for (int o = kWave / 2; o > 0; o >>= 1) {
            c += static_cast<unsigned long long>(__shfl_xor(static_cast<long long>(c), o, kWave));
            nd += static_cast<unsigned long long>(__shfl_xor(static_cast<long long>(nd), o, kWave));
        }
        if (lane == 0) {
            cost[v] = static_cast<uint32_t>(c);
            ndist[v] = static_cast<uint32_t>(nd);
        }
    }
}

// One thread per query: both rows, the scan cost of each direction from the
// per-vertex costs computed at ingest, the cheaper direction (forward on a
// tie) and its tile count.  A query with an empty endpoint row has no path.
__global__ __launch_bounds__(kWBlock) void wide_plan_kernel(WArgs A, const uint32_t *src, const uint32_t *dst,
                                                            const uint32_t *kq) {
    __shared__ unsigned long long red[kWBlock / kWave];
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long add_nd = 0, add_tiles = 0;
    if (q < A.nq) {
        const uint32_t s = src[q], t = dst[q], k = kq ? kq[q] : A.k_max;
        WPlan P{};
        P.s = s;
        P.t = t;
        P.k = k;
        if (s >= A.n || t >= A.n) P.status |= MHR_Q_BAD_ID;
        if (k == 0 || k > A.k_max) P.status |= MHR_Q_BAD_K;
        uint32_t os0 = 0, os1 = 0, it0 = 0, it1 = 0;
        unsigned long long cf = 0, cb = 0, nf = 0, nb = 0;
        if (P.status == 0) {
            os0 = A.out_rp[s];
            os1 = A.out_rp[s + 1];
            it0 = A.in_rp[t];
            it1 = A.in_rp[t + 1];
            if (os1 > os0 && it1 > it0) {
                cf = A.out_cost[s];
                nf = A.out_nd[s];
                cb = A.in_cost[t];
                nb = A.in_nd[t];
            }
        }
        P.out_len = os1 - os0;
        P.in_len = it1 - it0;
        const bool fwd = cf <= cb;
        P.dir = fwd ? 1u : 0u;
        P.list_beg = fwd ? os0 : it0;
        P.list_len = fwd ? P.out_len : P.in_len;
        P.probe_beg = fwd ? it0 : os0;
        P.probe_len = fwd ? P.in_len : P.out_len;
        P.cost = fwd ? cf : cb;
        P.nd = static_cast<uint32_t>(fwd ? nf : nb);
        P.ntiles = P.cost ? wcdiv(P.cost, kWTile) : 0u;
        P.nchunks = (P.status == 0 && P.cost) ? wcdiv(P.list_len, kWChunk) : 0u;
        A.plans[q] = P;
        A.gthr[q] = 0;
        A.qtotal[q] = 0;
        A.qmatch[q] = 0;
        add_nd = P.nd;
        add_tiles = P.ntiles;
    }
    const unsigned long long bn = wblock_sum(add_nd, red);
    const unsigned long long bt = wblock_sum(add_tiles, red);
    if (threadIdx.x == 0) {
        atomicAdd(&A.tot->nd, bn);
        atomicAdd(&A.tot->tiles, bt);
    }
}

// Offsets of each query's distinct table and tiles.
__global__ __launch_bounds__(kWBlock) void wide_offsets_kernel(WArgs A) {
    __shared__ unsigned long long red[kWBlock / kWave];
    unsigned long long cn = 0, ct = 0, cc = 0;
    for (uint32_t b = 0; b < A.nq; b += kWBlock) {
        const uint32_t q = b + threadIdx.x;
        WPlan P{};
        if (q < A.nq) P = A.plans[q];
        unsigned long long tn, tt, tc;
        const unsigned long long en = wblock_excl<unsigned long long>(q < A.nq ? P.nd : 0, red, &tn);
        const unsigned long long et = wblock_excl<unsigned long long>(q < A.nq ? P.ntiles : 0, red, &tt);
        const unsigned long long ec = wblock_excl<unsigned long long>(q < A.nq ? P.nchunks : 0, red, &tc);
        if (q < A.nq) {
            A.plans[q].tab_off = cn + en;
            A.plans[q].tile_base = static_cast<uint32_t>(ct + et);
            A.plans[q].chunk_base = static_cast<uint32_t>(cc + ec);
        }
        cn += tn;
        ct += tt;
        cc += tc;
    }
    if (threadIdx.x == 0) {
        A.tot->ctr = 0;
        A.tot->chunks = cc;
    }
}

// The distinct table of the list side: for every distinct list vertex x
// with a nonempty scan row, in list order, its scan-row bounds, its run in
// the list row and the scan entries of the earlier ones.  Built over chunks
// of kWChunk list entries spread across the grid (a hub's list row of
// millions of entries takes many workgroups): the count pass sizes each
// chunk, the per-query scan turns the sizes into offsets, the fill pass
// writes the rows.

// The query owning list chunk c: the last query whose chunk_base <= c (a
// query without chunks shares its base with the next query, and only
// precedes the owner of that base).
__device__ inline uint32_t chunk_query(const WArgs &A, uint32_t c) {
    uint32_t lo = 0, hi = A.nq;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        const WPlan &P = A.plans[mid];
        if (P.chunk_base <= c) lo = mid; else hi = mid;
    }
    return lo;
}

// This thread's segment of chunk cc of query P: the run starts with a
// nonempty scan row among its kWSeg entries (xs[j + 1], scan row [lo, lo +
// dg)), their count and their summed lengths.
struct ChunkSeg {
    uint32_t i0;
    uint32_t xs[kWSeg + 1], lo[kWSeg], dg[kWSeg];
    unsigned long long cnt, sum;
};

__device__ inline void chunk_segment(const WArgs &A, const WPlan &P, uint32_t cc, ChunkSeg &S) {
    const bool fwd = P.dir != 0;
    const uint32_t *Lcol = (fwd ? A.out_col : A.in_col) + P.list_beg;
    const uint32_t *Srp = fwd ? A.out_rp : A.in_rp;   // the scanned rows live in the list CSR
    S.i0 = cc * kWChunk + threadIdx.x * kWSeg;
    const uint32_t i0 = S.i0;
    S.xs[0] = (i0 > 0 && i0 < P.list_len) ? Lcol[i0 - 1] : 0xFFFFFFFFu;
#pragma unroll
    for (uint32_t j = 0; j < kWSeg; ++j) S.xs[j + 1] = (i0 + j < P.list_len) ? Lcol[i0 + j] : 0xFFFFFFFFu;
    S.cnt = S.sum = 0;
#pragma unroll
    for (uint32_t j = 0; j < kWSeg; ++j) {
        const bool first = i0 + j < P.list_len && S.xs[j + 1] != S.xs[j];
        S.lo[j] = first ? Srp[S.xs[j + 1]] : 0u;
        S.dg[j] = first ? Srp[S.xs[j + 1] + 1] - S.lo[j] : 0u;
    }
#pragma unroll
    for (uint32_t j = 0; j < kWSeg; ++j) {
        S.cnt += S.dg[j] ? 1 : 0;
        S.sum += S.dg[j];
    }
}

__global__ __launch_bounds__(kWBlock) void wide_chunk_count_kernel(WArgs A, uint32_t nchunks) {
    __shared__ unsigned long long red[kWBlock / kWave];
    __shared__ uint32_t sq;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        if (threadIdx.x == 0) sq = chunk_query(A, c);
        __syncthreads();
        const WPlan P = A.plans[sq];
        ChunkSeg S;
        chunk_segment(A, P, c - P.chunk_base, S);
        const unsigned long long tc = wblock_sum(S.cnt, red);
        const unsigned long long ts = wblock_sum(S.sum, red);
        if (threadIdx.x == 0) A.cpart[c] = make_ulonglong2(tc, ts);
        __syncthreads();
    }
}

// Per query: the chunks' sizes become their exclusive prefixes; and the
// tile map.
__global__ __launch_bounds__(kWBlock) void wide_chunk_scan_kernel(WArgs A) {
    __shared__ unsigned long long red[kWBlock / kWave];
    const uint32_t q = blockIdx.x;
    const WPlan P = A.plans[q];
    if (P.status != 0) return;
    for (uint32_t j = threadIdx.x; j < P.ntiles; j += kWBlock) A.tile_q[P.tile_base + j] = q;
    unsigned long long r0 = 0, p0 = 0;
    for (uint32_t b = 0; b < P.nchunks; b += kWBlock) {
        const uint32_t j = b + threadIdx.x;
        const ulonglong2 v = j < P.nchunks ? A.cpart[P.chunk_base + j] : make_ulonglong2(0ull, 0ull);
        unsigned long long tr, tp;
        const unsigned long long er = wblock_excl<unsigned long long>(v.x, red, &tr);
        const unsigned long long ep = wblock_excl<unsigned long long>(v.y, red, &tp);
        if (j < P.nchunks) A.cpart[P.chunk_base + j] = make_ulonglong2(r0 + er, p0 + ep);
        r0 += tr;
        p0 += tp;
    }
}

__global__ __launch_bounds__(kWBlock) void wide_chunk_fill_kernel(WArgs A, uint32_t nchunks) {
    __shared__ unsigned long long red[kWBlock / kWave];
    __shared__ uint32_t sq;
    for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        if (threadIdx.x == 0) sq = chunk_query(A, c);
        __syncthreads();
        const WPlan P = A.plans[sq];
        const bool fwd = P.dir != 0;
        const uint32_t *Lcol = (fwd ? A.out_col : A.in_col) + P.list_beg;
        ChunkSeg S;
        chunk_segment(A, P, c - P.chunk_base, S);
        unsigned long long tc, ts;
        const unsigned long long rc = wblock_excl<unsigned long long>(S.cnt, red, &tc);
        const unsigned long long pc = wblock_excl<unsigned long long>(S.sum, red, &ts);
        const ulonglong2 base = A.cpart[c];
        unsigned long long rank = base.x + rc, pre = base.y + pc;
        WRow *tab = A.tab + P.tab_off;
#pragma unroll
        for (uint32_t j = 0; j < kWSeg; ++j) {
            if (S.dg[j]) {
                const uint32_t i = S.i0 + j;
                uint32_t len = 1;   // the run of x: its relations to the list anchor
                while (i + len < P.list_len && Lcol[i + len] == S.xs[j + 1]) ++len;
                WRow R;
                R.prefix = pre;
                R.x = S.xs[j + 1];
                R.scan_beg = S.lo[j];
                R.run_beg = i;
                R.run_len = len;
                tab[rank++] = R;
                pre += S.dg[j];
            }
        }
        __syncthreads();
    }
}

struct WShared {
    uint32_t tile, q, list_n, stage_n, nrows;
    unsigned long long paths;
    WCand thr;
};

// Lower bound of y in ids[0 .. len): the first index holding an id >= y.
__device__ __forceinline__ uint32_t wlower(const uint32_t *ids, uint32_t len, uint32_t y) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ids[mid] < y) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Sorts c[0 .. N) best first (N a power of two) by bitonic exchanges.
__device__ inline void wbitonic(WCand *c, uint32_t N) {
    for (uint32_t size = 2; size <= N; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < N / 2; i += blockDim.x) {
                const uint32_t lo = 2 * i - (i & (stride - 1));
                const uint32_t hi = lo + stride;
                const bool up = (lo & size) == 0;   // this run is sorted best first
                WCand x = c[lo], y = c[hi];
                if (wbetter(y, x) == up) {
                    c[lo] = y;
                    c[hi] = x;
                }
            }
            __syncthreads();
        }
    }
}

// Merges the staged candidates into the list (c[0 .. k) list, c[k .. N)
// staging) and refreshes the thresholds.
__device__ inline void wmerge(const WArgs &A, WCand *c, uint32_t N, uint32_t k, WShared *sh, uint32_t q) {
    __syncthreads();
    const uint32_t staged = min(sh->stage_n, N - k);
    const uint32_t listed = sh->list_n;
    if (listed + staged <= k) {
        // everything fits the list: move the staged candidates behind it and
        // sort only the next power of two above their count
        for (uint32_t i = threadIdx.x; i < staged; i += blockDim.x) c[listed + i] = c[k + i];
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < staged; i += blockDim.x) c[k + i] = wcand_sentinel();
        __syncthreads();
        uint32_t n2 = 2;
        while (n2 < listed + staged) n2 <<= 1;
        wbitonic(c, n2);
        if (threadIdx.x == 0) {
            sh->list_n = listed + staged;
            sh->stage_n = 0;
            if (listed + staged == k) {
                sh->thr = c[k - 1];
                atomicMax(reinterpret_cast<unsigned long long *>(&A.gthr[q]),
                          static_cast<unsigned long long>(dkey(c[k - 1].s)));
            }
        }
        __syncthreads();
        return;
    }
    wbitonic(c, N);
    const uint32_t nl = min(k, listed + staged);
    for (uint32_t i = k + threadIdx.x; i < N; i += blockDim.x) c[i] = wcand_sentinel();
    if (threadIdx.x == 0) {
        sh->list_n = nl;
        sh->stage_n = 0;
        if (nl == k) {
            sh->thr = c[k - 1];
            atomicMax(reinterpret_cast<unsigned long long *>(&A.gthr[q]),
                      static_cast<unsigned long long>(dkey(c[k - 1].s)));
        }
    }
    __syncthreads();
}

template <bool BF16>
__global__ __launch_bounds__(kWBlock) void wide_gather_kernel(WArgs A, uint32_t total_tiles, uint32_t N) {
    extern __shared__ __align__(16) unsigned char wsm[];
    WCand *cand = reinterpret_cast<WCand *>(wsm);                                    // N
    uint32_t *pid = reinterpret_cast<uint32_t *>(wsm + size_t(N) * sizeof(WCand));   // kWProbeLds
    uint64_t *rpre = reinterpret_cast<uint64_t *>(pid + kWProbeLds);                  // kWSub
    uint32_t *rx = reinterpret_cast<uint32_t *>(rpre + kWSub);
    uint32_t *rsb = rx + kWSub, *rrb = rsb + kWSub, *rrl = rrb + kWSub;
    __shared__ WShared sh;
    __shared__ unsigned long long red[kWBlock / kWave];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint32_t t = static_cast<uint32_t>(atomicAdd(&A.tot->ctr, 1ull));
            sh.tile = t;
            if (t < total_tiles) sh.q = A.tile_q[t];
        }
        __syncthreads();
        const uint32_t tile = sh.tile;
        if (tile >= total_tiles) break;
        const uint32_t q = sh.q;
        const WPlan P = A.plans[q];
        const uint32_t k = P.k, S = N - k;
        const bool fwd = P.dir != 0;
        const uint32_t *Lcol = fwd ? A.out_col : A.in_col;
        const uint16_t *Lrel = fwd ? A.out_rel : A.in_rel;
        const uint32_t *Pcol = fwd ? A.in_col : A.out_col;
        const uint16_t *Prel = fwd ? A.in_rel : A.out_rel;
        // Long probe rows are not searched: the probe edge between a scanned
        // neighbour y and the probe anchor is found in y's own row instead
        // (forward: t in out(y); backward: s in in(y)), usually a few entries.
        const uint32_t *Qrp = fwd ? A.out_rp : A.in_rp;
        const uint32_t *Qcol = fwd ? A.out_col : A.in_col;
        const uint16_t *Qrel = fwd ? A.out_rel : A.in_rel;
        const uint32_t anchor_p = fwd ? P.t : P.s;
        const WRow *tab = A.tab + P.tab_off;
        // the probe row is copied to LDS when it is short and the query scans
        // at least half as many entries (else each lookup uses y's own row)
        const bool plds = P.probe_len <= kWProbeLds && P.probe_len <= 2 * min<uint64_t>(P.cost, kWTile);
        if (plds)
            for (uint32_t i = threadIdx.x; i < P.probe_len; i += kWBlock) pid[i] = Pcol[P.probe_beg + i];
        for (uint32_t i = threadIdx.x; i < N; i += kWBlock) cand[i] = wcand_sentinel();
        if (threadIdx.x == 0) {
            sh.list_n = 0;
            sh.stage_n = 0;
        }
        const uint64_t t0 = static_cast<uint64_t>(tile - P.tile_base) * kWTile;
        const uint64_t t1 = min(P.cost, t0 + kWTile);
        unsigned long long mypaths = 0, mymatch = 0;
        for (uint64_t sb = t0; sb < t1; sb += kWSub) {
            const uint64_t se = min(t1, sb + kWSub);
            __syncthreads();   // the previous sub-chunk's staged rows are no longer read
            // the last table row with prefix <= sb, searched by the whole
            // workgroup: each round tests kWBlock evenly spaced rows of the
            // remaining range at once (the prefixes ascend, so the rows that
            // pass are a leading run and their count locates the answer)
            uint32_t lo = 0, hi = sb == 0 ? 1u : P.nd;
            while (hi - lo > 1) {
                const uint32_t stride = (hi - lo + kWBlock - 1) / kWBlock;
                const uint32_t pos = lo + threadIdx.x * stride;
                const bool ok = pos < hi && tab[pos].prefix <= sb;   // row lo always passes
                const uint32_t c = static_cast<uint32_t>(__syncthreads_count(ok));
                lo += (c - 1) * stride;
                hi = min(hi, lo + stride);
            }
            const uint32_t r0 = lo;
            uint32_t valid = 0;
            for (uint32_t i = threadIdx.x; i < kWSub; i += kWBlock) {
                const uint32_t r = r0 + i;
                if (r < P.nd) {
                    const WRow R = tab[r];
                    if (R.prefix < se) {
                        rpre[i] = R.prefix;
                        rx[i] = R.x;
                        rsb[i] = R.scan_beg;
                        rrb[i] = R.run_beg;
                        rrl[i] = R.run_len;
                        ++valid;
                    }
                }
            }
            const uint32_t nrows = static_cast<uint32_t>(wblock_sum<unsigned long long>(valid, red));
            for (uint64_t base = sb; base < se; base += kWBlock) {
                const uint64_t p = base + threadIdx.x;
                uint32_t ncombo = 0, nl = 0, x = 0, y = 0, r2 = 0, rb = 0;
                const uint16_t *prr = nullptr;   // relations of the probe run
                double w2 = 0.0;
                if (p < se) {
                    // the staged row holding p: the last with prefix <= p
                    uint32_t lo = 0, hi = nrows;
                    while (hi - lo > 1) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (rpre[mid] <= p) lo = mid; else hi = mid;
                    }
                    const uint32_t e = rsb[lo] + static_cast<uint32_t>(p - rpre[lo]);
                    x = rx[lo];
                    rb = rrb[lo];
                    nl = rrl[lo];
                    y = Lcol[e];
                    r2 = Lrel[e];
                    uint32_t np = 0;
                    if (plds) {
                        const uint32_t ix = wlower(pid, P.probe_len, y);
                        while (ix + np < P.probe_len && pid[ix + np] == y) ++np;
                        prr = Prel + P.probe_beg + ix;
                    } else {
                        // the shorter of y's own row (searched for the anchor)
                        // and the probe row (searched for y)
                        const uint32_t b0 = Qrp[y], b1 = Qrp[y + 1];
                        if (b1 - b0 <= P.probe_len) {
                            const uint32_t ix = b0 + wlower(Qcol + b0, b1 - b0, anchor_p);
                            while (ix + np < b1 && Qcol[ix + np] == anchor_p) ++np;
                            prr = Qrel + ix;
                        } else {
                            const uint32_t *pc = Pcol + P.probe_beg;
                            const uint32_t ix = wlower(pc, P.probe_len, y);
                            while (ix + np < P.probe_len && pc[ix + np] == y) ++np;
                            prr = Prel + P.probe_beg + ix;
                        }
                    }
                    if (np) {
                        ncombo = nl * np;
                        w2 = fwd ? wide_weight<BF16>(A.X, A.Y, A.d, A.gamma, x, r2, y)
                                 : wide_weight<BF16>(A.X, A.Y, A.d, A.gamma, y, r2, x);
                    }
                }
                mypaths += ncombo;
                mymatch += ncombo ? 1u : 0u;
                const uint64_t gk = A.gthr[q];   // best known K-th score of the query (0: none yet)
                const double floor_s = gk ? dkey_inv(gk) : -INFINITY;
                uint32_t combo = 0;
                for (;;) {
                    while (combo < ncombo) {
                        const uint32_t li = combo % nl, pi = combo / nl;
                        const uint16_t rl = Lrel[P.list_beg + rb + li], rp = prr[pi];
                        // list edge s -rl-> x (forward) or x -rl-> t; probe edge
                        // y -rp-> t (forward) or s -rp-> y
                        const double wL = fwd ? wide_weight<BF16>(A.X, A.Y, A.d, A.gamma, P.s, rl, x)
                                              : wide_weight<BF16>(A.X, A.Y, A.d, A.gamma, x, rl, P.t);
                        const double wP = fwd ? wide_weight<BF16>(A.X, A.Y, A.d, A.gamma, y, rp, P.t)
                                              : wide_weight<BF16>(A.X, A.Y, A.d, A.gamma, P.s, rp, y);
                        WCand c;
                        c.s = fwd ? sum3_rn(wL, w2, wP) : sum3_rn(wP, w2, wL);
                        c.a = fwd ? x : y;
                        c.b = fwd ? y : x;
                        c.r1 = fwd ? rl : rp;
                        c.r2 = static_cast<uint16_t>(r2);
                        c.r3 = fwd ? rp : rl;
                        c.pad = 0;
                        const bool keep = c.s >= floor_s && (sh.list_n < k || wbetter(c, sh.thr));
                        if (keep) {
                            const uint32_t slot = atomicAdd(&sh.stage_n, 1u);
                            if (slot >= S) break;   // staging full: retry after the merge
                            cand[k + slot] = c;
                        }
                        ++combo;
                    }
                    if (!__syncthreads_or(combo < ncombo)) break;
                    wmerge(A, cand, N, k, &sh, q);
                }
            }
        }
        const unsigned long long bp = wblock_sum<unsigned long long>(mypaths, red);
        const unsigned long long bm = wblock_sum<unsigned long long>(mymatch, red);
        if (sh.stage_n > 0) wmerge(A, cand, N, k, &sh, q);
        __syncthreads();
        const uint32_t nl = sh.list_n;
        for (uint32_t i = threadIdx.x; i < nl; i += kWBlock) A.slots[static_cast<size_t>(tile) * A.k_max + i] = cand[i];
        if (threadIdx.x == 0) {
            A.tile_n[tile] = nl;
            A.head[tile] = 0;
            atomicAdd(reinterpret_cast<unsigned long long *>(&A.qtotal[q]), bp);
            atomicAdd(reinterpret_cast<unsigned long long *>(&A.qmatch[q]), bm);
        }
    }
}

// One wave per query: K-way merge of the tiles' sorted lists.
__global__ __launch_bounds__(kWBlock) void wide_merge_kernel(WArgs A, mhr_wide_path *out, uint32_t *out_count,
                                                             uint64_t *out_total, uint32_t *out_status,
                                                             mhr_wide_work *out_work) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t q = blockIdx.x * (kWBlock / kWave) + threadIdx.x / kWave;
    if (q >= A.nq) return;
    const WPlan P = A.plans[q];
    mhr_wide_path *row = out + static_cast<size_t>(q) * A.k_max;
    const uint64_t total = P.status ? 0ull : A.qtotal[q];
    const uint32_t cnt = P.status ? 0u : static_cast<uint32_t>(min<uint64_t>(total, P.k));
    for (uint32_t i = 0; i < cnt; ++i) {
        WCand best = wcand_sentinel();
        uint32_t bt = 0xFFFFFFFFu;
        for (uint32_t j = lane; j < P.ntiles; j += kWave) {
            const uint32_t t = P.tile_base + j;
            const uint32_t h = __hip_atomic_load(&A.head[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (h < A.tile_n[t]) {
                const WCand c = A.slots[static_cast<size_t>(t) * A.k_max + h];
                if (bt == 0xFFFFFFFFu || wbetter(c, best)) {
                    best = c;
                    bt = t;
                }
            }
        }
        for (int o = kWave / 2; o > 0; o >>= 1) {
            WCand c;
            c.s = __shfl_xor(best.s, o, kWave);
            c.a = __shfl_xor(best.a, o, kWave);
            c.b = __shfl_xor(best.b, o, kWave);
            const uint32_t r12 = __shfl_xor(static_cast<uint32_t>(best.r1) | (static_cast<uint32_t>(best.r2) << 16), o, kWave);
            const uint32_t r3 = __shfl_xor(static_cast<uint32_t>(best.r3), o, kWave);
            const uint32_t t = __shfl_xor(bt, o, kWave);
            c.r1 = static_cast<uint16_t>(r12 & 0xFFFFu);
            c.r2 = static_cast<uint16_t>(r12 >> 16);
            c.r3 = static_cast<uint16_t>(r3);
            c.pad = 0;
            if (t != 0xFFFFFFFFu && (bt == 0xFFFFFFFFu || wbetter(c, best) || (!wbetter(best, c) && t < bt))) {
                best = c;
                bt = t;
            }
        }
        uint32_t old = 0;
        if (lane == 0) {
            mhr_wide_path o;
            o.score = best.s;
            o.a = best.a;
            o.b = best.b;
            o.r1 = best.r1;
            o.r2 = best.r2;
            o.r3 = best.r3;
            o.reserved = 0;
            row[i] = o;
            // the head moves at the device-coherent level; the returned value
            // is consumed below, so the add completes before the next round's
            // loads of the heads
            if (bt != 0xFFFFFFFFu)
                old = __hip_atomic_fetch_add(&A.head[bt], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        old = __shfl(old, 0, kWave);
        if (old == 0xFFFFFFFFu) break;   // never: a head stays below its list length
    }
    for (uint32_t i = cnt + lane; i < A.k_max; i += kWave) {
        mhr_wide_path o;
        o.score = -INFINITY;
        o.a = o.b = 0xFFFFFFFFu;
        o.r1 = o.r2 = o.r3 = 0xFFFFu;
        o.reserved = 0;
        row[i] = o;
    }
    if (lane == 0) {
        out_count[q] = cnt;
        if (out_total) out_total[q] = total;
        if (out_status) out_status[q] = P.status;
        if (out_work) {
            mhr_wide_work w;
            w.scanned = P.cost;
            w.matches = P.status ? 0ull : A.qmatch[q];
            w.paths = total;
            w.frontier = static_cast<uint64_t>(P.out_len) + P.in_len;
            w.distinct = P.nd;
            w.probe_len = P.probe_len;
            w.tiles = P.ntiles;
            w.forward = P.dir;
            out_work[q] = w;
        }
    }
}

// Workspace: a fixed part sized by the batch, then the parts sized by the
// plan's totals.
struct WLayout {
    size_t plans, tot, gthr, qtotal, qmatch, fixed, tab, tile_q, tile_n, head, slots, cpart, total;
};

WLayout wide_layout(uint32_t nq, uint32_t k_max, uint64_t nd, uint64_t tiles, uint64_t chunks) {
    WLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = (o + bytes + 255) & ~size_t(255);
        return r;
    };
    L.plans = take(size_t(nq) * sizeof(WPlan));
    L.tot = take(sizeof(WTotals));
    L.gthr = take(size_t(nq) * 8);
    L.qtotal = take(size_t(nq) * 8);
    L.qmatch = take(size_t(nq) * 8);
    L.fixed = o;
    L.tab = take(nd * sizeof(WRow));
    L.tile_q = take(tiles * 4);
    L.tile_n = take(tiles * 4);
    L.head = take(tiles * 4);
    L.slots = take(tiles * k_max * sizeof(WCand));
    L.cpart = take(chunks * sizeof(ulonglong2));
    L.total = o;
    return L;
}

uint32_t wide_cand_slots(uint32_t k_max) {
    uint32_t N = kWPathsMin;
    while (N < 2 * k_max) N <<= 1;
    return N;
}

size_t wide_lds_bytes(uint32_t k_max) {
    return size_t(wide_cand_slots(k_max)) * sizeof(WCand) + kWProbeLds * 4 + kWSub * (8 + 4 * 4);
}

WArgs wide_args(const mhr_wide_graph *g, uint32_t nq, uint32_t k_max, char *ws, const WLayout &L) {
    WArgs A{};
    A.out_rp = g->out.row_ptr;
    A.out_col = g->out.col;
    A.out_rel = g->out.rel;
    A.in_rp = g->in.row_ptr;
    A.in_col = g->in.col;
    A.in_rel = g->in.rel;
    A.X = g->X;
    A.Y = g->Y;
    A.n = g->n;
    A.d = g->dim;
    A.nq = nq;
    A.k_max = k_max;
    A.gamma = g->gamma;
    A.plans = reinterpret_cast<WPlan *>(ws + L.plans);
    A.tot = reinterpret_cast<WTotals *>(ws + L.tot);
    A.gthr = reinterpret_cast<uint64_t *>(ws + L.gthr);
    A.qtotal = reinterpret_cast<uint64_t *>(ws + L.qtotal);
    A.qmatch = reinterpret_cast<uint64_t *>(ws + L.qmatch);
    A.tab = reinterpret_cast<WRow *>(ws + L.tab);
    A.tile_q = reinterpret_cast<uint32_t *>(ws + L.tile_q);
    A.tile_n = reinterpret_cast<uint32_t *>(ws + L.tile_n);
    A.head = reinterpret_cast<uint32_t *>(ws + L.head);
    A.slots = reinterpret_cast<WCand *>(ws + L.slots);
    A.cpart = reinterpret_cast<ulonglong2 *>(ws + L.cpart);
    A.out_cost = g->out.cost;
    A.out_nd = g->out.ndist;
    A.in_cost = g->in.cost;
    A.in_nd = g->in.ndist;
    return A;
}

mhr_status wide_check(const mhr_wide_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                      uint32_t k_max) {
    MHR_ARG_CHECK(g && src && dst, "wide query: null argument");
    MHR_ARG_CHECK(nq >= 1, "wide query: nq must be >= 1");
    MHR_ARG_CHECK(k_max >= 1 && k_max <= MHR_WIDE_MAX_K, "wide query: k_max must be in [1, 256]");
    if (!g->X || !g->Y || g->dim == 0) {
        set_error("wide query: embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    return MHR_OK;
}

// Plans the batch into the fixed part of ws and returns the totals (the
// stream is synchronised).
mhr_status wide_plan(const mhr_wide_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                     const uint32_t *k, uint32_t k_max, char *ws, WTotals *tot, hipStream_t st) {
    const WLayout L0 = wide_layout(nq, k_max, 0, 0, 0);
    WArgs A = wide_args(g, nq, k_max, ws, L0);
    MHR_HIP_TRY(hipMemsetAsync(A.tot, 0, sizeof(WTotals), st));
    hipLaunchKernelGGL(wide_plan_kernel, dim3(wcdiv(nq, kWBlock)), dim3(kWBlock), 0, st, A, src, dst, k);
    hipLaunchKernelGGL(wide_offsets_kernel, dim3(1), dim3(kWBlock), 0, st, A);
    MHR_HIP_TRY(hipGetLastError());
    MHR_HIP_TRY(hipMemcpyAsync(tot, A.tot, sizeof(WTotals), hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipStreamSynchronize(st));
    return MHR_OK;
}

}  // namespace
}  // namespace mhr

using namespace mhr;

extern "C" mhr_status mhr_wide_graph_create(const mhr_graph_desc *d, void *stream, mhr_wide_graph **out) {
    MHR_ARG_CHECK(d != nullptr && out != nullptr, "mhr_wide_graph_create: null argument");
    MHR_ARG_CHECK(d->num_vertices >= 1 && d->num_vertices < 0xFFFFFFFFu, "num_vertices must be in [1, 2^32-2]");
    MHR_ARG_CHECK(d->num_relations >= 1 && d->num_relations <= MHR_WIDE_MAX_RELATIONS,
                  "num_relations must be in [1, 65535]");
    MHR_ARG_CHECK(d->num_edges < 0xFFFFFFFFull, "num_edges must be < 2^32");
    MHR_ARG_CHECK(d->num_edges == 0 || (d->head && d->rel && d->tail), "edge arrays must not be null");
    hipStream_t st = static_cast<hipStream_t>(stream);
    mhr_wide_graph *g = new (std::nothrow) mhr_wide_graph();
    if (!g) {
        set_error("host allocation failed");
        return MHR_ERR_OUT_OF_MEMORY;
    }
    g->n = d->num_vertices;
    g->R = d->num_relations;
    while (g->id_bits < 32 && (1ull << g->id_bits) < g->n) ++g->id_bits;
    while (g->rel_bits < 16 && (1ull << g->rel_bits) < g->R) ++g->rel_bits;
    (void)hipGetDevice(&g->device);
    mhr_status s = wide_build_direction(g, d, 0, g->out, st);
    if (s == MHR_OK) s = wide_build_direction(g, d, 1, g->in, st);
    if (s != MHR_OK) {
        wide_free_dir(g->out);
        wide_free_dir(g->in);
        delete g;
        return s;
    }
    *out = g;
    return MHR_OK;
}

extern "C" mhr_status mhr_wide_graph_destroy(mhr_wide_graph *g) {
    if (!g) return MHR_OK;
    wide_free_dir(g->out);
    wide_free_dir(g->in);
    delete g;
    return MHR_OK;
}

extern "C" mhr_status mhr_wide_graph_set_embeddings(mhr_wide_graph *g, mhr_dtype dtype, uint32_t dim,
                                                    const void *entity, const void *relation, double gamma) {
    MHR_ARG_CHECK(g && entity && relation, "mhr_wide_graph_set_embeddings: null argument");
    MHR_ARG_CHECK(dtype == MHR_DTYPE_F32 || dtype == MHR_DTYPE_BF16, "mhr_wide_graph_set_embeddings: bad dtype");
    MHR_ARG_CHECK(dim >= 1 && dim <= 1024, "mhr_wide_graph_set_embeddings: dim must be in [1, 1024]");
    MHR_ARG_CHECK(std::isfinite(gamma), "mhr_wide_graph_set_embeddings: gamma must be finite");
    g->dtype = dtype;
    g->dim = dim;
    g->X = entity;
    g->Y = relation;
    g->gamma = gamma;
    return MHR_OK;
}

extern "C" mhr_status mhr_wide_graph_get_stats(const mhr_wide_graph *g, mhr_wide_stats *o) {
    MHR_ARG_CHECK(g && o, "mhr_wide_graph_get_stats: null argument");
    o->num_vertices = g->n;
    o->num_relations = g->R;
    o->num_triples = g->m;
    o->max_out_degree = g->out.max_degree;
    o->max_in_degree = g->in.max_degree;
    o->dim = g->dim;
    o->dtype = static_cast<uint32_t>(g->dtype);
    o->device_bytes = g->device_bytes;
    return MHR_OK;
}

extern "C" mhr_status mhr_wide_graph_export_csr(const mhr_wide_graph *g, int reverse, uint32_t *row_ptr,
                                                uint32_t *col, uint16_t *rel, void *stream) {
    MHR_ARG_CHECK(g && row_ptr && col && rel, "mhr_wide_graph_export_csr: null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const mhr_wide_graph::Dir &D = reverse ? g->in : g->out;
    MHR_HIP_TRY(hipMemcpyAsync(row_ptr, D.row_ptr, (static_cast<size_t>(g->n) + 1) * 4, hipMemcpyDeviceToDevice, st));
    if (g->m) {
        MHR_HIP_TRY(hipMemcpyAsync(col, D.col, g->m * 4, hipMemcpyDeviceToDevice, st));
        MHR_HIP_TRY(hipMemcpyAsync(rel, D.rel, g->m * 2, hipMemcpyDeviceToDevice, st));
    }
    return MHR_OK;
}

extern "C" mhr_status mhr_wide_workspace_size(const mhr_wide_graph *g, uint32_t nq, const uint32_t *src,
                                              const uint32_t *dst, const uint32_t *k, uint32_t k_max, size_t *bytes,
                                              void *stream) {
    mhr_status rc = wide_check(g, nq, src, dst, k_max);
    if (rc != MHR_OK) return rc;
    MHR_ARG_CHECK(bytes != nullptr, "mhr_wide_workspace_size: null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const WLayout L0 = wide_layout(nq, k_max, 0, 0, 0);
    WBuf tmp;
    MHR_HIP_TRY(tmp.alloc(L0.fixed));
    WTotals tot{};
    rc = wide_plan(g, nq, src, dst, k, k_max, tmp.as<char>(), &tot, st);
    if (rc != MHR_OK) return rc;
    *bytes = wide_layout(nq, k_max, tot.nd, tot.tiles, tot.chunks).total;
    return MHR_OK;
}

extern "C" mhr_status mhr_wide_topk_paths(const mhr_wide_graph *g, uint32_t nq, const uint32_t *src,
                                          const uint32_t *dst, const uint32_t *k, uint32_t k_max, mhr_wide_path *out,
                                          uint32_t *out_count, uint64_t *out_total, uint32_t *out_status,
                                          mhr_wide_work *out_work, void *workspace, size_t ws_bytes, void *stream,
                                          const mhr_phase_events *ev) {
    mhr_status rc = wide_check(g, nq, src, dst, k_max);
    if (rc != MHR_OK) return rc;
    MHR_ARG_CHECK(out && out_count && workspace, "mhr_wide_topk_paths: null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const WLayout L0 = wide_layout(nq, k_max, 0, 0, 0);
    if (ws_bytes < L0.fixed) {
        set_error("mhr_wide_topk_paths: workspace too small for the batch's plans");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    char *ws = static_cast<char *>(workspace);
    auto mark = [&](void *e) -> hipError_t { return e ? hipEventRecord(static_cast<hipEvent_t>(e), st) : hipSuccess; };
    MHR_HIP_TRY(mark(ev ? ev->begin : nullptr));
    WTotals tot{};
    rc = wide_plan(g, nq, src, dst, k, k_max, ws, &tot, st);
    if (rc != MHR_OK) return rc;
    const WLayout L = wide_layout(nq, k_max, tot.nd, tot.tiles, tot.chunks);
    if (ws_bytes < L.total) {
        set_error("mhr_wide_topk_paths: workspace too small: need " + std::to_string(L.total) + " bytes");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    if (tot.tiles >= 0xFFFFFFFFull) {
        set_error("mhr_wide_topk_paths: too many tiles in one batch");
        return MHR_ERR_UNSUPPORTED;
    }
    const WArgs A = wide_args(g, nq, k_max, ws, L);
    const bool bf = g->dtype == MHR_DTYPE_BF16;
    if (tot.chunks >= 0xFFFFFFFFull) {
        set_error("mhr_wide_topk_paths: list rows too long for one batch");
        return MHR_ERR_UNSUPPORTED;
    }
    const uint32_t nchunks = static_cast<uint32_t>(tot.chunks);
    if (nchunks) {
        const uint32_t cgrid = std::min<uint32_t>(nchunks, 65535u);
        hipLaunchKernelGGL(wide_chunk_count_kernel, dim3(cgrid), dim3(kWBlock), 0, st, A, nchunks);
        hipLaunchKernelGGL(wide_chunk_scan_kernel, dim3(nq), dim3(kWBlock), 0, st, A);
        hipLaunchKernelGGL(wide_chunk_fill_kernel, dim3(cgrid), dim3(kWBlock), 0, st, A, nchunks);
    } else {
        hipLaunchKernelGGL(wide_chunk_scan_kernel, dim3(nq), dim3(kWBlock), 0, st, A);   // the tile map
    }
    MHR_HIP_TRY(hipGetLastError());
    const uint32_t tiles = static_cast<uint32_t>(tot.tiles);
    MHR_HIP_TRY(mark(ev ? ev->gather_begin : nullptr));
    if (tiles) {
        int cus = 0;
        MHR_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
        const uint32_t N = wide_cand_slots(k_max);
        const size_t lds = wide_lds_bytes(k_max);
        const uint32_t grid = std::min<uint32_t>(tiles, static_cast<uint32_t>(std::max(cus, 1)) * 4u);
        if (bf) hipLaunchKernelGGL(wide_gather_kernel<true>, dim3(grid), dim3(kWBlock), lds, st, A, tiles, N);
        else hipLaunchKernelGGL(wide_gather_kernel<false>, dim3(grid), dim3(kWBlock), lds, st, A, tiles, N);
        MHR_HIP_TRY(hipGetLastError());
    }
    MHR_HIP_TRY(mark(ev ? ev->gather_end : nullptr));
    hipLaunchKernelGGL(wide_merge_kernel, dim3(wcdiv(nq, kWBlock / kWave)), dim3(kWBlock), 0, st, A, out, out_count,
                       out_total, out_status, out_work);
    MHR_HIP_TRY(hipGetLastError());
    MHR_HIP_TRY(mark(ev ? ev->end : nullptr));
    return MHR_OK;
}
