// Exact three-hop top-K path search, plain FP32 form with compensated
// rescoring of the boundary band.
//
// Pipeline for a batch of queries (all on the caller's stream):
//   plan      one workgroup per query: validates ids, measures the two
//             meet-in-the-middle costs (backward: sum of in-degrees of
//             N-(t); forward: sum of out-degrees of N+(s)), picks the
//             cheaper direction and cuts the scan into tiles.
//   schedule  one workgroup: prefix of tile counts, tile -> query map, and
//             the order the gather takes tiles in (longest expected first).
//   gather    persistent workgroups pulling tiles from an atomic counter.
//             A tile builds a membership table of the probe side (LDS hash
//             or, for long rows, the graph's bucket directory), streams the
//             CSR rows of its list slice, tests each scanned vertex, scores
//             every matched middle edge and the two outer edges in FP32 with
//             a rigorous error bound, enumerates the paths through it and
//             keeps the best KC by fast-pass score.
//   merge     one workgroup per query: selects the best KC over the tile
//             lists, takes every
//             candidate whose score lies within twice the error bound of the
//             K-th, rescores them in float-float and writes the ranked
//             result.  If a truncated tile could still hold a path that
//             can be returned the query is marked for the exhaustive pass.
//   exact     gather again for marked queries, scoring in float-float every
//             path above the band threshold that can still be returned (its
//             fast score plus error bound reaches both the kept list and a
//             lower bound on the K-th score), then a merge of those lists.
//
// The paper's CPU design (thread-private K-heaps merged by a tree
// reduction, section 3.3; level-synchronous frontier expansion, section 5)
// is the prior art this replaces: here the per-thread heap becomes a
// per-workgroup LDS candidate list fed by block-wide threshold filtering
// and trimmed by radix selection, and the reduction tree becomes the
// per-query selection over tile lists.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "mhr_device.h"
#include "mhr_internal.h"

namespace mhr {

namespace {

constexpr int kBlock = 512;
constexpr int kEPT = 8;                   // scan entries per thread per chunk
constexpr int kChunk = kBlock * kEPT;     // scan entries per chunk
constexpr int kRowBatch = 32;             // list rows staged at a time
constexpr int kSlab = 8 * kBlock;               // scored edge values per sub-batch
constexpr int kQueue = kChunk + kBlock;    // queued matches: a partial sub-batch plus one chunk's hits
constexpr int kStage = 3 * kBlock / 2;               // staged candidates before a merge
constexpr uint32_t kItemRun = 16;           // item ranges longer than this are written by a whole wave
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kDefaultTileEdges = 32768;
constexpr uint32_t kDefaultHashLog2 = 12;

struct GArgs {
    const uint32_t *out_rp, *out_col, *out_mask, *out_dir_off, *out_dir_pool;
    const uint32_t *in_rp, *in_col, *in_mask, *in_dir_off, *in_dir_pool;
    const void *X, *Y;
    uint32_t n, R, d, id_bits;
    QueryPlan *plans;
    Control *ctrl;
    uint32_t *tile_q;
    uint32_t *tile_order;   // the order in which the gather takes the tiles
    uint2 *tile_start;
    TileHeader *hdr;
    Cand *cands;
    uint32_t *exact_list;
    uint32_t tcap, hash_log2, nq, kc, tile_edges;
    float band_abs;              // minimum rescoring band width below the K-th score
    float gamma;                 // TransE-L1 scorer: the constant the L1 distance is subtracted from
    const uint8_t *keep;         // pruned search: keep flags (nullptr: every entry kept)
    const uint64_t *keep_off;    // per query: offset of its flags in keep
};

// Keep flags of the pruned search: per query, one byte per entry of s's
// out-row, then one per entry of t's in-row (nonzero = kept).  A pruned-away
// entry removes that first (or last) edge pair from every path.  nullptr
// when the search is not pruned.
__device__ inline const uint8_t *keep_row(const GArgs &A, uint32_t q, uint32_t s, bool t_row) {
    if (!A.keep) return nullptr;
    uint64_t off = A.keep_off[q];
    if (t_row) off += A.out_rp[s + 1] - A.out_rp[s];
    return A.keep + off;
}

constexpr uint32_t kMaxTilesPerQuery = 4096;
constexpr uint32_t kMergeSlots = 2048;      // LDS candidates per merge step
constexpr uint32_t kSpan = 16;              // embedding elements a scoring lane holds per step
constexpr int kRescoreLanes = 16;           // lanes that rescore one band candidate together
constexpr int kMergeBlock = 256;            // threads of a per-query merge workgroup (>= the largest KC)

// Tiles the workspace holds for nq queries.
__host__ __device__ inline uint32_t tile_capacity(uint32_t nq) { return nq * 4u > 16384u ? nq * 4u : 16384u; }

// Block reductions / scans (blockDim.x == NT, kBlock unless stated).  The
// scratch `lds` is written only after a barrier, so a later call may reuse
// it without one at the end of this call (no other code writes it).
template <class T, int NT = kBlock>
__device__ inline T block_sum(T v, T *lds) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < NT / kWave; ++w) s += lds[w];
    return s;
}

template <int NT = kBlock>
__device__ inline float block_max(float v, float *lds) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    float s = lds[0];
    for (int w = 1; w < NT / kWave; ++w) s = fmaxf(s, lds[w]);
    return s;
}

// Inclusive scan over the block; *total receives the block total.
template <class T>
__device__ inline T block_incl_scan(T v, T *lds, T *total) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int off = 1; off < kWave; off <<= 1) {
        T t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    __syncthreads();
    if (lane == kWave - 1) lds[wave] = v;
    __syncthreads();
    T base = 0, tot = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
        T x = lds[w];
        if (w < wave) base += x;
        tot += x;
    }
    *total = tot;
    return v + base;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void plan_kernel(GArgs A, const uint32_t *src, const uint32_t *dst,
                                                      const uint32_t *kq, uint32_t kdef, uint32_t kmax) {
    __shared__ uint64_t red64[kBlock / kWave];
    const uint32_t q = blockIdx.x;
    QueryPlan P{};
    P.s = src[q];
    P.t = dst[q];
    P.k = kq ? kq[q] : kdef;
    uint32_t st = 0;
    if (P.s >= A.n || P.t >= A.n) st |= MHR_Q_BAD_ID;
    if (P.k == 0 || P.k > kmax) st |= MHR_Q_BAD_K;
    P.status = st;
    if (st) {
        if (threadIdx.x == 0) A.plans[q] = P;
        return;
    }
    // Summed degrees of a list row's neighbours (their scanned rows), over
    // entries [base, base + kPlanSpan) of the list: each thread loads its
    // entries' ids together, then their row bounds together.
    constexpr int kPlanU = 4;
    constexpr uint32_t kPlanSpan = kPlanU * kBlock;
    auto span_cost = [&](const uint32_t *rp, const uint32_t *col, uint32_t beg, uint32_t len, const uint8_t *keep,
                         uint32_t base) -> uint64_t {
        uint32_t x[kPlanU];
        bool ok[kPlanU];
#pragma unroll
        for (int u = 0; u < kPlanU; ++u) {
            const uint32_t i = base + u * kBlock + threadIdx.x;
            ok[u] = i < len && (!keep || keep[i]);
            x[u] = ok[u] ? col[beg + i] : 0u;
        }
        uint64_t p = 0;
#pragma unroll
        for (int u = 0; u < kPlanU; ++u)
            if (ok[u]) p += rp[x[u] + 1] - rp[x[u]];
        return p;
    };
    // the endpoints' rows: N-(t) in the reverse CSR, N+(s) in the forward CSR
    const uint32_t lb_beg = A.in_rp[P.t], lb_end = A.in_rp[P.t + 1];
    const uint32_t lf_beg = A.out_rp[P.s], lf_end = A.out_rp[P.s + 1];
    const uint32_t lb_len = lb_end - lb_beg, lf_len = lf_end - lf_beg;
    // backward: list N-(t), scanned rows in the reverse CSR
    const uint8_t *kb = keep_row(A, q, P.s, true), *kf = keep_row(A, q, P.s, false);
    uint64_t part = 0;
    for (uint32_t base = 0; base < lb_len; base += kPlanSpan) part += span_cost(A.in_rp, A.in_col, lb_beg, lb_len, kb, base);
    const uint64_t cost_b = block_sum<uint64_t>(part, red64);
    // forward: list N+(s), scanned rows in the forward CSR; stop once it
    // cannot beat the backward cost
    uint64_t cost_f = 0;
    for (uint32_t base = 0; base < lf_len && cost_f < cost_b; base += kPlanSpan)
        cost_f += block_sum<uint64_t>(span_cost(A.out_rp, A.out_col, lf_beg, lf_len, kf, base), red64);
    const bool fwd = cost_f < cost_b;
    P.dir = fwd ? 1u : 0u;
    P.cost = fwd ? cost_f : cost_b;
    P.list_beg = fwd ? lf_beg : lb_beg;
    P.list_len = fwd ? lf_len : lb_len;
    P.probe_beg = fwd ? lb_beg : lf_beg;
    P.probe_len = fwd ? lb_len : lf_len;
    // tile count from the scan cost; the schedule may coarsen it to fit the
    // workspace
    P.ntiles = (P.cost > 0 && P.probe_len > 0) ? 1u : 0u;
    if (threadIdx.x == 0) A.plans[q] = P;
}

// ---------------------------------------------------------------------------
// schedule (one workgroup)
// ---------------------------------------------------------------------------
// Tile length for a query: about `tile` scan entries, at most
// kMaxTilesPerQuery tiles.  The tile count is then ceil(cost / length), so
// every tile start j * length lies below cost.
// ceil(a / b), in 32-bit arithmetic when both fit
__device__ inline uint64_t div_up(uint64_t a, uint64_t b) {
    if (((a + b) >> 32) == 0) return (static_cast<uint32_t>(a) + static_cast<uint32_t>(b) - 1u) / static_cast<uint32_t>(b);
    return (a + b - 1) / b;
}

__device__ inline uint64_t tile_len_for(uint64_t cost, uint64_t tile) {
    uint64_t nt = div_up(cost, tile);
    if (nt > kMaxTilesPerQuery) nt = kMaxTilesPerQuery;
    return div_up(cost, nt);
}

__device__ inline uint32_t tiles_for(uint64_t cost, uint64_t tile) {
    if (cost == 0) return 0u;
    return static_cast<uint32_t>(div_up(cost, tile_len_for(cost, tile)));
}

// Order class of a query's tiles, larger for longer expected tiles.  A
// tile's time is mostly its matches, and the share of scanned entries that
// hit the probe side grows with the probe side's size, so the tile length
// times (probe length + 64) orders tiles by expected time.  Classes are
// quarter-octaves of that product.
constexpr uint32_t kOrderClasses = 256;
__device__ inline uint32_t order_class(uint64_t tile_len, uint32_t probe_len) {
    const uint64_t x = tile_len * (static_cast<uint64_t>(probe_len) + 64u);
    if (x < 4) return static_cast<uint32_t>(x);
    const int msb = 63 - __clzll(static_cast<long long>(x));
    const uint32_t c = 4u * static_cast<uint32_t>(msb) + static_cast<uint32_t>((x >> (msb - 2)) & 3u);
    return min(c, kOrderClasses - 1);
}

// One workgroup: per-query tile counts (tile size doubled until the batch
// fits the workspace's tile capacity), their prefix, the tile -> query map,
// and the order in which the gather takes the tiles: longest expected first,
// so that the last tiles to start are short ones (a counting sort over the
// order classes; tiles of one class in any order).
// Batches of up to kSchedCache queries keep each query's scan cost, probe
// length and tile fields in LDS, read from the plans in one round of loads;
// larger batches read the plans again in each pass.
constexpr uint32_t kSchedCache = 4096;
constexpr size_t kSchedLds = size_t(kSchedCache) * (8 + 4 * 4);

__global__ __launch_bounds__(kBlock) void schedule_kernel(GArgs A) {
    __shared__ uint32_t red[kBlock / kWave];
    __shared__ uint64_t red64[kBlock / kWave];
    __shared__ uint32_t carry;
    __shared__ uint32_t cls_base[kOrderClasses];
    extern __shared__ __align__(16) unsigned char sched_smem[];
    uint64_t *c_cost = reinterpret_cast<uint64_t *>(sched_smem);   // 0: no tiles
    uint32_t *c_probe = reinterpret_cast<uint32_t *>(c_cost + kSchedCache);
    uint32_t *c_nt = c_probe + kSchedCache, *c_tb = c_nt + kSchedCache, *c_len = c_tb + kSchedCache;
    const bool cached = A.nq <= kSchedCache;
    if (cached) {
        constexpr int U = kSchedCache / kBlock;
        uint64_t cs[U];
        uint32_t pl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t q = u * kBlock + threadIdx.x;
            cs[u] = 0;
            pl[u] = 0;
            if (q < A.nq) {
                const QueryPlan &P = A.plans[q];
                const bool has = P.status == 0 && P.ntiles;
                cs[u] = has ? P.cost : 0u;
                pl[u] = P.probe_len;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t q = u * kBlock + threadIdx.x;
            if (q < A.nq) {
                c_cost[q] = cs[u];
                c_probe[q] = pl[u];
            }
        }
        __syncthreads();
    }
    auto qcost = [&](uint32_t q) -> uint64_t {
        if (cached) return c_cost[q];
        const QueryPlan &P = A.plans[q];
        return (P.status == 0 && P.ntiles) ? P.cost : 0u;
    };
    uint64_t tile = A.tile_edges;
    for (;;) {
        uint64_t part = 0;
        for (uint32_t q = threadIdx.x; q < A.nq; q += kBlock) part += tiles_for(qcost(q), tile);
        const uint64_t tot = block_sum<uint64_t>(part, red64);
        if (tot <= A.tcap) break;
        tile *= 2;
    }
    if (threadIdx.x == 0) carry = 0;
    for (uint32_t i = threadIdx.x; i < kOrderClasses; i += kBlock) cls_base[i] = 0;   // tiles per class
    __syncthreads();
    for (uint32_t base = 0; base < A.nq; base += kBlock) {
        const uint32_t q = base + threadIdx.x;
        const uint64_t cost = q < A.nq ? qcost(q) : 0u;
        const uint32_t nt = tiles_for(cost, tile);
        uint32_t tot;
        const uint32_t incl = block_incl_scan<uint32_t>(nt, red, &tot);
        const uint32_t c = carry;
        if (q < A.nq) {
            const uint32_t tb = c + incl - nt;
            const uint32_t len = nt ? static_cast<uint32_t>(tile_len_for(cost, tile)) : 0u;
            A.plans[q].ntiles = nt;
            A.plans[q].tile_base = tb;
            A.plans[q].flags = 0;
            A.plans[q].pad[0] = len;  // tile length
            for (uint32_t j = 0; j < nt; ++j) A.tile_q[tb + j] = q;
            if (nt) {
                const uint32_t pl = cached ? c_probe[q] : A.plans[q].probe_len;
                atomicAdd(&cls_base[kOrderClasses - 1 - order_class(len, pl)], nt);
            }
            if (cached) {
                c_nt[q] = nt;
                c_tb[q] = tb;
                c_len[q] = len;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    // class bases, highest class first
    {
        static_assert(kOrderClasses <= kBlock, "one class per thread");
        const uint32_t v = threadIdx.x < kOrderClasses ? cls_base[threadIdx.x] : 0u;
        uint32_t tot;
        const uint32_t incl = block_incl_scan<uint32_t>(v, red, &tot);
        if (threadIdx.x < kOrderClasses) cls_base[threadIdx.x] = incl - v;
    }
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < A.nq; q += kBlock) {
        uint32_t nt, tb, len, pl;
        if (cached) {
            nt = c_nt[q];
            tb = c_tb[q];
            len = c_len[q];
            pl = c_probe[q];
        } else {
            const QueryPlan &P = A.plans[q];
            nt = P.status == 0 ? P.ntiles : 0u;
            tb = P.tile_base;
            len = P.pad[0];
            pl = P.probe_len;
        }
        if (nt) {
            const uint32_t at = atomicAdd(&cls_base[kOrderClasses - 1 - order_class(len, pl)], nt);
            for (uint32_t j = 0; j < nt; ++j) A.tile_order[at + j] = tb + j;
        }
    }
    if (threadIdx.x == 0) {
        A.ctrl->total_tiles = carry;
        A.ctrl->gather_ctr = 0;
        A.ctrl->exact_ctr = 0;
        A.ctrl->exact_n = 0;
    }
}

// One workgroup per query: tile j starts at position j * L of the
// concatenation of the query's scanned rows; record (row, offset).
__global__ __launch_bounds__(kBlock) void tile_starts_kernel(GArgs A) {
    __shared__ uint64_t red64[kBlock / kWave];
    const uint32_t q = blockIdx.x;
    const QueryPlan P = A.plans[q];
    if (P.status != 0 || P.ntiles == 0) return;
    const uint64_t L = P.pad[0];
    const bool fwd = P.dir != 0;
    const uint32_t *rp = fwd ? A.out_rp : A.in_rp;
    const uint32_t *col = fwd ? A.out_col : A.in_col;
    const uint8_t *kl = keep_row(A, q, P.s, !fwd);
    uint64_t run = 0;
    for (uint32_t base = 0; base < P.list_len; base += kBlock) {
        const uint32_t i = base + threadIdx.x;
        uint64_t deg = 0;
        if (i < P.list_len && (!kl || kl[i])) {
            const uint32_t x = col[P.list_beg + i];
            deg = rp[x + 1] - rp[x];
        }
        uint64_t tot;
        const uint64_t incl = block_incl_scan<uint64_t>(deg, red64, &tot);
        const uint64_t p0 = run + incl - deg;
        if (deg > 0) {
            const uint64_t jlo = (p0 + L - 1) / L;
            const uint64_t jhi = (p0 + deg - 1) / L;
            for (uint64_t j = jlo; j <= jhi && j < P.ntiles; ++j)
                A.tile_start[P.tile_base + j] = make_uint2(i, static_cast<uint32_t>(j * L - p0));
        }
        run += tot;
    }
}

// ---------------------------------------------------------------------------
// float-float scoring of one path (rescoring and the exhaustive pass)
// ---------------------------------------------------------------------------
// One term X[u,i]*Y[r,i]*X[v,i] in float-float: the relation factor times
// the smaller entity factor exactly (TwoProduct), then times the larger.
// Taking the entity factors in value order makes the term, and so the edge
// weight, bit-identical for (u,r,v) and (v,r,u), as the DistMult score is.
__device__ __forceinline__ ff distmult_term_ff(float xu, float yr, float xv, float *abs_t) {
    const float lo = fminf(xu, xv), hi = fmaxf(xu, xv);
    const ff p = two_prod(lo, yr);
    *abs_t = fabsf(p.hi * hi);
    return ff_mul_f(p, hi);
}

template <bool BF16>
__device__ inline ff edge_x_ff(const GArgs &A, uint32_t u, uint32_t r, uint32_t v, float *abs_sum) {
    ff acc = {0.0f, 0.0f};
    float as = 0.0f;
    // eight elements per 16-byte load (d is a power of two >= 8), summed in
    // ascending order as one at a time
    for (uint32_t i0 = 0; i0 < A.d; i0 += 8) {
        float xu[8], yr[8], xv[8];
        load8<BF16>(A.X, u, A.d, i0, xu);
        load8<BF16>(A.Y, r, A.d, i0, yr);
        load8<BF16>(A.X, v, A.d, i0, xv);
#pragma unroll
        for (int l = 0; l < 8; ++l) {
            float at;
            const ff t = distmult_term_ff(xu[l], yr[l], xv[l], &at);
            acc = ff_add(acc, t);
            as += at;
        }
    }
    *abs_sum = as;
    return acc;
}

// The same sum computed by an aligned group of G lanes (a power of two, at
// most a wave): lane l of the group takes the terms l, l + G, ..., and a
// butterfly combines the lane sums (ff_add is symmetric in its operands, so
// every lane of the group ends with the same bits).  No term passes through
// more than d float-float additions, so the error bound of the sequential
// sum holds.
template <bool BF16, int G>
__device__ inline ff group_edge_x_ff(const GArgs &A, uint32_t u, uint32_t r, uint32_t v, float *abs_sum) {
    ff acc = {0.0f, 0.0f};
    float as = 0.0f;
    const size_t d = A.d;
    for (uint32_t i = threadIdx.x & (G - 1); i < A.d; i += G) {
        float at;
        const ff t = distmult_term_ff(load1<BF16>(A.X, u * d + i), load1<BF16>(A.Y, r * d + i),
                                      load1<BF16>(A.X, v * d + i), &at);
        acc = ff_add(acc, t);
        as += at;
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const ff w = {__shfl_xor(acc.hi, o, kWave), __shfl_xor(acc.lo, o, kWave)};
        acc = ff_add(acc, w);
        as += __shfl_xor(as, o, kWave);
    }
    *abs_sum = as;
    return acc;
}

// TransE-L1 term |(X[u,i] + Y[r,i]) - X[v,i]| in float-float: TwoSum makes
// X[u,i] + Y[r,i] exact; subtracting X[v,i] (double-word plus float) errs by
// at most 2u^2 of the result; the absolute value is exact.
__device__ __forceinline__ ff transe_term_ff(float xu, float yr, float xv) {
    const ff t = ff_add_f(two_sum(xu, yr), -xv);
    return t.hi < 0.0f ? ff_neg(t) : t;
}

// The L1 distance sum_i |(X[u,i] + Y[r,i]) - X[v,i]| of the TransE score in
// float-float, in ascending i (the terms are non-negative, so each
// double-word addition errs by at most 3u^2 of a partial sum <= the total).
// *abs_sum receives the FP32 sum of the terms' leading parts (for bounds).
template <bool BF16>
__device__ inline ff edge_l1_ff(const GArgs &A, uint32_t u, uint32_t r, uint32_t v, float *abs_sum) {
    ff acc = {0.0f, 0.0f};
    float as = 0.0f;
    for (uint32_t i0 = 0; i0 < A.d; i0 += 8) {
        float xu[8], yr[8], xv[8];
        load8<BF16>(A.X, u, A.d, i0, xu);
        load8<BF16>(A.Y, r, A.d, i0, yr);
        load8<BF16>(A.X, v, A.d, i0, xv);
#pragma unroll
        for (int l = 0; l < 8; ++l) {
            const ff t = transe_term_ff(xu[l], yr[l], xv[l]);
            acc = ff_add(acc, t);
            as += t.hi;
        }
    }
    *abs_sum = as;
    return acc;
}

// The same distance computed by an aligned group of G lanes (strided terms,
// then a butterfly of symmetric float-float additions; every lane of the
// group ends with the same bits).
template <bool BF16, int G>
__device__ inline ff group_edge_l1_ff(const GArgs &A, uint32_t u, uint32_t r, uint32_t v, float *abs_sum) {
    ff acc = {0.0f, 0.0f};
    float as = 0.0f;
    const size_t d = A.d;
    for (uint32_t i = threadIdx.x & (G - 1); i < A.d; i += G) {
        const ff t = transe_term_ff(load1<BF16>(A.X, u * d + i), load1<BF16>(A.Y, r * d + i),
                                    load1<BF16>(A.X, v * d + i));
        acc = ff_add(acc, t);
        as += t.hi;
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const ff w = {__shfl_xor(acc.hi, o, kWave), __shfl_xor(acc.lo, o, kWave)};
        acc = ff_add(acc, w);
        as += __shfl_xor(as, o, kWave);
    }
    *abs_sum = as;
    return acc;
}

// S = w(s,r1,a) + w(a,r2,b) + w(b,r3,t) in float-float, with a bound on
// its error.  DistMult (TE = false): w = logsigmoid(x) of the dot product;
// per edge, the dot product (about 4 d u^2 sum|t|) plus the log-sigmoid.
// TransE-L1 (TE = true): w = gamma - L1 distance; per edge, the distance
// (at most (3d + 2) u^2 of its value) and the subtraction from gamma.  Then
// the two additions of the weights.
// G = 1: one thread alone; G > 1 (a power of two, >= 4): an aligned group
// of G lanes computes the score together and every lane returns it.
template <bool BF16, int G, bool TE>
__device__ inline ff path_score_ff(const GArgs &A, uint32_t s, uint32_t a, uint32_t b, uint32_t t, uint32_t r1,
                                   uint32_t r2, uint32_t r3, float *eps) {
    const float u2 = kUnit * kUnit;
    float as1, as2, as3;
    ff x1, x2, x3;
    if constexpr (TE) {
        if (G > 1) {
            x1 = group_edge_l1_ff<BF16, G>(A, s, r1, a, &as1);
            x2 = group_edge_l1_ff<BF16, G>(A, a, r2, b, &as2);
            x3 = group_edge_l1_ff<BF16, G>(A, b, r3, t, &as3);
        } else {
            x1 = edge_l1_ff<BF16>(A, s, r1, a, &as1);
            x2 = edge_l1_ff<BF16>(A, a, r2, b, &as2);
            x3 = edge_l1_ff<BF16>(A, b, r3, t, &as3);
        }
    } else if (G > 1) {
        x1 = group_edge_x_ff<BF16, G>(A, s, r1, a, &as1);
        x2 = group_edge_x_ff<BF16, G>(A, a, r2, b, &as2);
        x3 = group_edge_x_ff<BF16, G>(A, b, r3, t, &as3);
    } else {
        x1 = edge_x_ff<BF16>(A, s, r1, a, &as1);
        x2 = edge_x_ff<BF16>(A, a, r2, b, &as2);
        x3 = edge_x_ff<BF16>(A, b, r3, t, &as3);
    }
    ff w1, w2, w3;
    if constexpr (TE) {
        w1 = ff_add_f(ff_neg(x1), A.gamma);
        w2 = ff_add_f(ff_neg(x2), A.gamma);
        w3 = ff_add_f(ff_neg(x3), A.gamma);
    } else if (G > 1) {
        // the group's lanes 0, 1, 2 (mod 3) take one log-sigmoid each; every
        // lane then reads all three
        const int lane = static_cast<int>(threadIdx.x & (kWave - 1));
        const int g0 = lane & ~(G - 1);
        const int e = (lane - g0) % 3;
        const ff w = ff_logsigmoid(e == 0 ? x1 : (e == 1 ? x2 : x3));
        w1 = ff{__shfl(w.hi, g0, kWave), __shfl(w.lo, g0, kWave)};
        w2 = ff{__shfl(w.hi, g0 + 1, kWave), __shfl(w.lo, g0 + 1, kWave)};
        w3 = ff{__shfl(w.hi, g0 + 2, kWave), __shfl(w.lo, g0 + 2, kWave)};
    } else {
        w1 = ff_logsigmoid(x1);
        w2 = ff_logsigmoid(x2);
        w3 = ff_logsigmoid(x3);
    }
    // Sum in a canonical order (descending) so that the result depends only
    // on the multiset of weights: paths whose weights are permutations of
    // each other (DistMult is symmetric) then tie exactly, as their real
    // scores do.
    ff v1 = w1, v2 = w2, v3 = w3;
    auto order = [](ff &x, ff &y) {
        if (x.hi < y.hi || (x.hi == y.hi && x.lo < y.lo)) {
            ff t = x;
            x = y;
            y = t;
        }
    };
    order(v1, v2);
    order(v2, v3);
    order(v1, v2);
    ff S = ff_add(ff_add(v1, v2), v3);
    float dd = static_cast<float>(A.d);
    float e;
    if constexpr (TE) {
        const float g = fabsf(A.gamma);
        e = (3.0f * dd + 4.0f) * u2 * 1.01f * ((as1 + g) + (as2 + g) + (as3 + g)) +
            8.0f * u2 * (fabsf(w1.hi) + fabsf(w2.hi) + fabsf(w3.hi));
    } else {
        e = 4.04f * dd * u2 * (as1 + as2 + as3) * 1.01f + ff_logsigmoid_err(w1.hi) + ff_logsigmoid_err(w2.hi) +
            ff_logsigmoid_err(w3.hi) + 8.0f * u2 * (fabsf(w1.hi) + fabsf(w2.hi) + fabsf(w3.hi));
    }
    *eps = e;
    return S;
}

// ---------------------------------------------------------------------------
// gather
// ---------------------------------------------------------------------------
struct RowInfo {
    uint32_t x, mask, beg, len, pref, vbase;
    float fmax, famax, emax;   // largest centred weight, |weight| and error bound of the row's list edges
};

struct GatherShared {
    uint32_t tile, q, j;
    uint32_t qcount;      // match queue fill
    uint32_t stage_n;
    uint32_t list_n;
    uint32_t truncated;
    uint32_t E;           // entries in the current row batch
    uint32_t rowvals;
    uint32_t sel_prefix, sel_need, sel_hi, sel_eq;   // stage-merge selection
    uint32_t vn;          // values in the current sub-batch's slab
    uint32_t pad[2];
    Cand thr;             // current worst kept candidate (sentinel until the list fills)
    uint64_t red64[kBlock / kWave];
    uint32_t red32[kBlock / kWave];
    float redf[kBlock / kWave];
};

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~static_cast<size_t>(15); }

struct GatherLayout {
    size_t hkeys, hvals, Y, anc_p, anc_l, rows, rowval, roweps, qpos, qmp, sub, slab, list, stage,
        ymax, ysum, rowrel, slab_rel, mkeys, shared, total;
};

constexpr int kSubFields = 7;  // pos, y, mp, mm, row, voff, first item

__host__ __device__ inline GatherLayout gather_layout(uint32_t hash_log2, uint32_t R, uint32_t d, uint32_t kc) {
    GatherLayout L{};
    size_t o = 0;
    const size_t slots = size_t(1) << hash_log2;
    L.hkeys = o; o = align16(o + slots * 4);
    L.hvals = o; o = align16(o + slots * 4);
    L.Y = o; o = align16(o + size_t(R) * (d + 4) * 4);
    L.anc_p = o; o = align16(o + size_t(d) * 4);
    L.anc_l = o; o = align16(o + size_t(d) * 4);
    L.rows = o; o = align16(o + kRowBatch * sizeof(RowInfo));
    L.rowval = o; o = align16(o + size_t(kRowBatch) * R * 4);
    L.roweps = o; o = align16(o + size_t(kRowBatch) * R * 4);
    L.qpos = o; o = align16(o + kQueue * 4);
    L.qmp = o; o = align16(o + kQueue * 4);
    L.sub = o; o = align16(o + kBlock * kSubFields * 4);
    L.mkeys = o; o = align16(o + 256 * 4);
    L.slab = o; o = align16(o + kSlab * 4);
    L.list = o; o = align16(o + size_t(kc) * sizeof(Cand));
    L.stage = o; o = align16(o + size_t(next_pow2(kStage + kc)) * sizeof(Cand));
    L.ymax = o; o = align16(o + size_t(R) * 4);
    L.ysum = o; o = align16(o + size_t(R) * 4);
    L.rowrel = o; o = align16(o + size_t(kRowBatch) * R);
    L.slab_rel = o; o = align16(o + kSlab);
    L.shared = o; o = align16(o + sizeof(GatherShared));
    L.total = o;
    return L;
}

// Lanes per scored edge and elements per lane for dimension d.
__device__ __forceinline__ int lanes_per_edge(uint32_t d) {
    int g = static_cast<int>(d / 8);
    return g < 4 ? 4 : (g > 64 ? 64 : g);
}

template <bool BF16>
__device__ __forceinline__ void load_lane(const void *base, size_t row, uint32_t d, uint32_t off, int epl,
                                          float (&v)[8]) {
    if (epl == 8) {
        load8<BF16>(base, row, d, off, v);
    } else {
#pragma unroll
        for (int l = 0; l < 8; ++l) v[l] = (l < epl) ? load1<BF16>(base, row * d + off + l) : 0.0f;
    }
}

// Scores the edges of one match held by a group of G lanes (lane glane
// owns elements [glane*epl, glane*epl + epl) of the d-vectors).  For each
// relation r in maskA the value is x = sum_i a[i] Y[r][i], then for each r
// in maskB x = sum_i b[i] Y[r][i]; the centred log-sigmoid of x goes to
// out[k] (k = value index: maskA bits ascending, then maskB bits) with its
// error bound in out_eps[k].  Values are produced four at a time: four
// independent accumulators and reductions keep the lanes busy, and lane j
// of the group evaluates the transcendental of value j.
//
// Error bound: each product a[i]*Y carries one rounding beyond the rounding
// of a[i] itself and the sum adds epl - 1 + log2 G more, so
// |x_fp32 - x| <= gamma_{epl + log2 G + 4} sum_i |a_i Y_ri|
//              <= gamma_{...} max_i |Y_ri| * sum_i |a_i| (ymax, suma).
__device__ inline void score_values(const float (&a)[8], float suma, uint32_t maskA, const float (&b)[8], float sumb,
                                    uint32_t maskB, const float *Ys, const float *ymax, uint32_t ys, int G, int epl,
                                    int glane, float *out, float *out_eps, uint8_t *out_rel) {
    const int lg = 31 - __clz(G);
    const float gam = gamma_n(epl + lg + 4) * 1.001f;
    const uint32_t na = __popc(maskA), nv = na + __popc(maskB);
    uint32_t ra = maskA, rb = maskB;
    const int off = glane * epl;
    for (uint32_t c = 0; c < nv; c += 4) {
        float part[4];
        uint32_t rel[4];
        bool isa[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t v = c + j;
            part[j] = 0.0f;
            rel[j] = 0;
            isa[j] = false;
            if (v < nv) {
                if (v < na) {
                    rel[j] = static_cast<uint32_t>(__ffs(ra) - 1);
                    ra &= ra - 1;
                    isa[j] = true;
                } else {
                    rel[j] = static_cast<uint32_t>(__ffs(rb) - 1);
                    rb &= rb - 1;
                }
                const float *yr = Ys + rel[j] * ys + off;
                float acc = 0.0f;
#pragma unroll
                for (int l = 0; l < 8; ++l)
                    if (l < epl) acc = __builtin_fmaf(isa[j] ? a[l] : b[l], yr[l], acc);
                part[j] = acc;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j] = group_sum(part[j], G);
        if (glane < 4 && c + glane < nv) {
            const float x = glane == 0 ? part[0] : glane == 1 ? part[1] : glane == 2 ? part[2] : part[3];
            const uint32_t r = glane == 0 ? rel[0] : glane == 1 ? rel[1] : glane == 2 ? rel[2] : rel[3];
            const bool ia = glane == 0 ? isa[0] : glane == 1 ? isa[1] : glane == 2 ? isa[2] : isa[3];
            float fe;
            const float f = centred_logsigmoid_e(x, fe);
            out[c + glane] = f;
            out_eps[c + glane] = gam * ymax[r] * (ia ? suma : sumb) + fe;
            out_rel[c + glane] = static_cast<uint8_t>(r);
        }
    }
}

// TransE-L1 values of the edges of one match (or one list row) held by a
// group of G lanes, lane glane owning elements [glane*epl, glane*epl + epl).
// For each relation r in maskA the value is f = gamma - sum_i |(pa[i] +
// Y[r][i]) - qa[i]| (pa the head's slice, qa the tail's), then for each r in
// maskB the same with pb, qb; values go to out[k] in that order (maskA bits
// ascending, then maskB bits), their error bounds to out_eps[k] (unless
// out_eps is null).  Four
// values at a time, lane j of the group finishing value j.
//
// Error bound: per element, the rounded head + relation and the rounded
// difference err by at most 2u(1 + u)(|p_i| + |Y_ri| + |q_i|); the sum adds
// at most epl - 1 + log2 G roundings of non-negative terms, and subtracting
// from gamma one more, so
// |f_fp32 - f| <= gamma_{d+3} (sum|p| + sum|Y_r| + sum|q|) + 2u |f|
// with sum|p| + sum|q| in tsumA / tsumB and sum|Y_r| in ysum[r].
__device__ inline void score_values_te(const float (&pa)[8], const float (&qa)[8], float tsumA, uint32_t maskA,
                                       const float (&pb)[8], const float (&qb)[8], float tsumB, uint32_t maskB,
                                       const float *Ys, const float *ysum, uint32_t ys, float gamma, float gamT,
                                       int G, int epl, int glane, float *out, float *out_eps, uint8_t *out_rel) {
    const uint32_t na = __popc(maskA), nv = na + __popc(maskB);
    uint32_t ra = maskA, rb = maskB;
    const int off = glane * epl;
    for (uint32_t c = 0; c < nv; c += 4) {
        float part[4];
        uint32_t rel[4];
        bool isa[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t v = c + j;
            part[j] = 0.0f;
            rel[j] = 0;
            isa[j] = false;
            if (v < nv) {
                if (v < na) {
                    rel[j] = static_cast<uint32_t>(__ffs(ra) - 1);
                    ra &= ra - 1;
                    isa[j] = true;
                } else {
                    rel[j] = static_cast<uint32_t>(__ffs(rb) - 1);
                    rb &= rb - 1;
                }
                const float *yr = Ys + rel[j] * ys + off;
                float acc = 0.0f;
#pragma unroll
                for (int l = 0; l < 8; ++l)
                    if (l < epl) acc += fabsf(((isa[j] ? pa[l] : pb[l]) + yr[l]) - (isa[j] ? qa[l] : qb[l]));
                part[j] = acc;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j] = group_sum(part[j], G);
        if (glane < 4 && c + glane < nv) {
            const float x = glane == 0 ? part[0] : glane == 1 ? part[1] : glane == 2 ? part[2] : part[3];
            const uint32_t r = glane == 0 ? rel[0] : glane == 1 ? rel[1] : glane == 2 ? rel[2] : rel[3];
            const bool ia = glane == 0 ? isa[0] : glane == 1 ? isa[1] : glane == 2 ? isa[2] : isa[3];
            const float f = gamma - x;
            out[c + glane] = f;
            if (out_eps) out_eps[c + glane] = gamT * ((ia ? tsumA : tsumB) + ysum[r]) + 2.0f * kUnit * fabsf(f);
            out_rel[c + glane] = static_cast<uint8_t>(r);
        }
    }
}

// Merge the staged candidates into the kept list (whole block).
// Order-preserving integer key of an FP32 score.
__device__ __forceinline__ uint32_t fkey(float x) {
    const uint32_t b = __float_as_uint(x);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Bitonic sort of n2 (a power of two) 64-bit keys into descending order
// (whole workgroup; ends with a barrier).
__device__ inline void block_sort_keys_desc(uint64_t *keys, uint32_t n2) {
    for (uint32_t k = 2; k <= n2; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) {
                const uint32_t p = i ^ j;
                if (p > i) {
                    const uint64_t x = keys[i], y = keys[p];
                    const bool desc = (i & k) == 0;   // this half ends highest-first
                    if (desc ? (x < y) : (x > y)) {
                        keys[i] = y;
                        keys[p] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Merges the staged candidates into the tile's list.
// Fast pass: the best KC of list + stage by fast-pass score (ties at the
// KC-th score in any order: dropping one marks the tile truncated at that
// score, and the band is re-sorted by the total order after rescoring); see
// below.  `hist` is scratch of 256 words.
// Exhaustive pass (EXACT): the scores are final, so the list keeps the best
// KC under the total order (score, then ids) and the whole candidates are
// sorted.
template <int KC, bool EXACT, bool BF16, bool TE>
__device__ inline void merge_stage(Cand *list, Cand *stage, GatherShared *sh, uint32_t *hist, const GArgs &A,
                                   uint32_t s, uint32_t t) {
    const uint32_t ns = sh->stage_n;
    if (EXACT) {
        // staged candidates carry their fast-pass score: take the float-float
        // score of each, one candidate per thread
        for (uint32_t i = threadIdx.x; i < ns; i += blockDim.x) {
            Cand c = stage[i];
            float e;
            const ff sc = path_score_ff<BF16, 1, TE>(A, s, c.a, c.b, t, (c.rel >> 16) & 0xFF, (c.rel >> 8) & 0xFF,
                                                 c.rel & 0xFF, &e);
            c.s = sc.hi;
            c.s_lo = sc.lo;
            c.eps = e;
            stage[i] = c;
        }
        __syncthreads();
        const uint32_t tot = ns + KC;
        const uint32_t n2 = next_pow2(tot);
        for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) {
            if (i >= ns && i < tot) stage[i] = list[i - ns];
            else if (i >= tot) stage[i] = cand_sentinel();
        }
        __syncthreads();
        block_sort_cands(stage, static_cast<int>(n2));
        if (threadIdx.x == 0) {
            if (stage[KC].a != 0xFFFFFFFFu) sh->truncated = 1;  // a real candidate fell off
            uint32_t cnt = sh->list_n + ns;
            sh->list_n = cnt < static_cast<uint32_t>(KC) ? cnt : KC;
            sh->stage_n = 0;
            sh->thr = (sh->list_n == static_cast<uint32_t>(KC)) ? stage[KC - 1] : cand_sentinel();
        }
        for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(KC); i += blockDim.x) list[i] = stage[i];
        __syncthreads();
        return;
    }
    // fast pass: the best KC of the staged and kept candidates, in no
    // particular order except that the last slot holds a kept minimum (the
    // threshold for later candidates).  A radix select over the 32-bit score
    // keys, 8 bits per pass from the top, finds the KC-th largest key T; every
    // candidate above T is kept, and as many at T as fit.
    const uint32_t ln = sh->list_n;
    const uint32_t real = ns + ln;
    for (uint32_t i = threadIdx.x; i < ln; i += blockDim.x) stage[ns + i] = list[i];
    __syncthreads();
    if (real < static_cast<uint32_t>(KC)) {
        for (uint32_t i = threadIdx.x; i < real; i += blockDim.x) list[i] = stage[i];
        __syncthreads();
        if (threadIdx.x == 0) {
            sh->list_n = real;
            sh->stage_n = 0;
        }
        __syncthreads();
        return;
    }
    uint32_t prefix = 0, pmask = 0, need = KC;
    for (int shift = 24; shift >= 0; shift -= 8) {
        for (uint32_t i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < real; i += blockDim.x) {
            const uint32_t key = fkey(stage[i].s);
            if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (threadIdx.x < static_cast<uint32_t>(kWave)) {
            // lane l holds bins 4l..4l+3; the bin where the count from the top
            // reaches `need` fixes the next 8 bits
            const uint32_t lane = threadIdx.x;
            const uint32_t h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2],
                           h3 = hist[4 * lane + 3];
            const uint32_t own = h0 + h1 + h2 + h3;
            uint32_t incl = own;   // this lane's bins and all higher ones
            for (int off = 1; off < kWave; off <<= 1) {
                const uint32_t t = __shfl_down(incl, off, kWave);
                if (lane + off < static_cast<uint32_t>(kWave)) incl += t;
            }
            const uint32_t above = incl - own;
            if (above < need && need <= incl) {
                uint32_t acc = above, b;
                if (acc + h3 >= need) b = 3;
                else if (acc += h3, acc + h2 >= need) b = 2;
                else if (acc += h2, acc + h1 >= need) b = 1;
                else { acc += h1; b = 0; }
                sh->sel_prefix = prefix | ((4 * lane + b) << shift);
                sh->sel_need = need - acc;
            }
        }
        if (threadIdx.x == 0) {
            sh->sel_hi = 0;
            sh->sel_eq = 0;
        }
        __syncthreads();
        prefix = sh->sel_prefix;
        need = sh->sel_need;
        pmask |= 255u << shift;
    }
    // keys above T fill the list from the front, the kept ones at T from the back
    for (uint32_t i = threadIdx.x; i < real; i += blockDim.x) {
        const uint32_t key = fkey(stage[i].s);
        if (key > prefix) {
            list[atomicAdd(&sh->sel_hi, 1u)] = stage[i];
        } else if (key == prefix) {
            const uint32_t e = atomicAdd(&sh->sel_eq, 1u);
            if (e < need) list[KC - 1 - e] = stage[i];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (real > static_cast<uint32_t>(KC)) sh->truncated = 1;   // a real candidate fell off
        sh->list_n = KC;
        sh->stage_n = 0;
        sh->thr = list[KC - 1];
    }
    __syncthreads();
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// A product of two bfloat16 values (16 significant bits, exact in FP32)
// split into two bfloat16 halves whose sum is exact: the leading 8
// significant bits (truncation, so both halves carry the sign of v) and the
// remaining at most 8 bits.  Returned as bit patterns.
__device__ __forceinline__ void split_bf16(float v, uint32_t &hi, uint32_t &lo) {
    const uint32_t b = __float_as_uint(v);
    hi = b >> 16;
    lo = __float_as_uint(v - __uint_as_float(b & 0xFFFF0000u)) >> 16;
}

// Up to S consecutive elements [off, off + n) of an embedding row (zeros
// past n, or everywhere when !valid).  n is a multiple of 2 and off of n's
// alignment: the loads are 16-byte vectors when n == S.
template <bool BF16, int S>
__device__ __forceinline__ void load_span(const void *base, uint32_t row, uint32_t d, uint32_t off, uint32_t n,
                                          bool valid, float (&v)[S]) {
#pragma unroll
    for (int l = 0; l < S; ++l) v[l] = 0.0f;
    if (!valid) return;
    if (n == static_cast<uint32_t>(S)) {
#pragma unroll
        for (int c = 0; c < S / 8; ++c) {
            float t[8];
            load8<BF16>(base, row, d, off + 8 * c, t);
#pragma unroll
            for (int l = 0; l < 8; ++l) v[8 * c + l] = t[l];
        }
    } else {
#pragma unroll
        for (int l = 0; l < S; ++l)
            if (static_cast<uint32_t>(l) < n) v[l] = load1<BF16>(base, static_cast<size_t>(row) * d + off + l);
    }
}

// S consecutive LDS floats p[0 .. n) (zeros past n): 16-byte reads when
// n == S (p is then 16-byte aligned), single reads otherwise.
template <int S>
__device__ __forceinline__ void lds_span(const float *p, uint32_t n, float (&v)[S]) {
    if (n == static_cast<uint32_t>(S)) {
#pragma unroll
        for (int c = 0; c < S / 4; ++c) {
            const float4 t = *reinterpret_cast<const float4 *>(p + 4 * c);
            v[4 * c] = t.x; v[4 * c + 1] = t.y; v[4 * c + 2] = t.z; v[4 * c + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int l = 0; l < S; ++l) v[l] = static_cast<uint32_t>(l) < n ? p[l] : 0.0f;
    }
}

// Insertion sort of n (<= 32) values into descending order, carrying their
// relation ids.  Equal values keep their relation order.
__device__ inline void sort_desc(float *v, uint8_t *rel, uint32_t n) {
    for (uint32_t i = 1; i < n; ++i) {
        const float x = v[i];
        const uint8_t rx = rel[i];
        uint32_t j = i;
        while (j > 0 && v[j - 1] < x) {
            v[j] = v[j - 1];
            rel[j] = rel[j - 1];
            --j;
        }
        v[j] = x;
        rel[j] = rx;
    }
}

// Partial sums used for the path score and its pruning bounds.  The same
// association is used for a bound and for the score it bounds, so FP32
// rounding (monotone) keeps every bound >= the scores below it.
__device__ __forceinline__ float combine3(bool fwd, float fp, float fm, float fl) {
    return fwd ? (fl + fm) + fp : (fp + fm) + fl;
}

// Phase clocks (a build with MHR_PHASE_CLOCKS defined): thread 0 of each
// gather workgroup reads the constant-rate wall clock at phase boundaries
// (each right after a barrier, so the interval is the workgroup's time in
// the phase that ended) and the totals over all workgroups are added to
// g_phase_ticks at exit.  Other builds compile the marks away.
enum GatherPhase {
    kPhFetch = 0,    // taking a tile, and the previous tile's output
    kPhSetup,        // probe table, anchors
    kPhRows,         // list rows: edge values, sorting
    kPhProbe,        // chunks: row search, column loads, probes, compaction
    kPhForm,         // sub-batch formation (masks, rows, value offsets)
    kPhScore,        // edge scoring (matrix cores, or vector units for TransE)
    kPhLogsig,       // dense log-sigmoids
    kPhBounds,       // per-match maxima, error bounds, work-item scan
    kPhEnum,         // path enumeration and staging
    kPhMerge,        // stage merges into the tile list
    kPhEnd,          // final merge, tile list and header out
    kNumPhases
};
// Work counts of the phase-clock build, per tile kind (see g_phase_ticks).
enum GatherCount {
    kCtTiles = 0,     // tiles taken
    kCtRowBatches,    // list-row batches
    kCtChunks,        // chunks of scanned entries
    kCtScanned,       // scanned entries
    kCtSubBatches,    // scoring sub-batches
    kCtMatches,       // matched middle edges scored
    kCtValues,        // edge values scored (probe and middle edges, per relation)
    kCtItems,         // enumeration items (match, probe value, middle value)
    kCtStaged,        // candidates staged
    kCtMerges,        // stage merges
    kNumCounts
};
constexpr int kPhSlots = kNumPhases + kNumCounts;
#ifdef MHR_PHASE_CLOCKS
// Per tile kind (0: probe side in the LDS table, 1: probing through the row
// directory): the phases' summed ticks, then the work counts.
__device__ unsigned long long g_phase_ticks[2 * kPhSlots];
#define MHR_PHASE(p)                                                      \
    do {                                                                  \
        if (tid == 0) {                                                   \
            const unsigned long long now_ = wall_clock64();               \
            ph_acc[(p) + (ph_heavy ? kPhSlots : 0)] += now_ - ph_t;       \
            ph_t = now_;                                                  \
        }                                                                 \
    } while (0)
#define MHR_COUNT(c, v)                                                                   \
    do {                                                                                  \
        if (tid == 0) ph_acc[kNumPhases + (c) + (ph_heavy ? kPhSlots : 0)] += (v);       \
    } while (0)
#else
#define MHR_PHASE(p) \
    do {             \
    } while (0)
#define MHR_COUNT(c, v) \
    do {                \
    } while (0)
#endif

// TE: the TransE-L1 scorer (VALU); otherwise DistMult (matrix cores).
template <bool BF16, bool EXACT, int KC, bool TE>
__global__ __launch_bounds__(kBlock) void gather_kernel(GArgs A) {
#ifdef MHR_PHASE_CLOCKS
    __shared__ unsigned long long ph_acc[2 * kPhSlots];
    __shared__ unsigned long long ph_t;
    bool ph_heavy = false;   // the current tile probes through the directory
    if (threadIdx.x < 2 * kPhSlots) ph_acc[threadIdx.x] = 0;
    if (threadIdx.x == 0) ph_t = wall_clock64();
#endif
    extern __shared__ __align__(16) unsigned char smem[];
    const GatherLayout Lo = gather_layout(A.hash_log2, A.R, A.d, KC);
    uint32_t *hkeys = reinterpret_cast<uint32_t *>(smem + Lo.hkeys);
    uint32_t *hvals = reinterpret_cast<uint32_t *>(smem + Lo.hvals);   // probe-row index of each key
    float *Ys = reinterpret_cast<float *>(smem + Lo.Y);
    float *anc_p = reinterpret_cast<float *>(smem + Lo.anc_p);
    float *anc_l = reinterpret_cast<float *>(smem + Lo.anc_l);
    RowInfo *rows = reinterpret_cast<RowInfo *>(smem + Lo.rows);
    float *rowval = reinterpret_cast<float *>(smem + Lo.rowval);
    float *roweps = reinterpret_cast<float *>(smem + Lo.roweps);
    uint32_t *qpos = reinterpret_cast<uint32_t *>(smem + Lo.qpos);
    uint32_t *qmp = reinterpret_cast<uint32_t *>(smem + Lo.qmp);   // queued hit's index in the probe row
    uint32_t *sub = reinterpret_cast<uint32_t *>(smem + Lo.sub);
    float *slab = reinterpret_cast<float *>(smem + Lo.slab);
    Cand *list = reinterpret_cast<Cand *>(smem + Lo.list);
    Cand *stage = reinterpret_cast<Cand *>(smem + Lo.stage);
    GatherShared *sh = reinterpret_cast<GatherShared *>(smem + Lo.shared);
    float *ymax = reinterpret_cast<float *>(smem + Lo.ymax);
    float *ysum = reinterpret_cast<float *>(smem + Lo.ysum);   // sum_i |Y[r][i]| (TransE bounds)
    uint32_t *mkeys = reinterpret_cast<uint32_t *>(smem + Lo.mkeys);  // stage-merge histogram
    uint8_t *rowrel = reinterpret_cast<uint8_t *>(smem + Lo.rowrel);
    uint8_t *slab_rel = reinterpret_cast<uint8_t *>(smem + Lo.slab_rel);
    float *sub_su_p = reinterpret_cast<float *>(sub);   // sum_k |up_k| per match (scoring)
    float *sub_su_m = reinterpret_cast<float *>(sub + 6 * kBlock);   // sum_k |um_k| (scoring; then sub_item)
    uint32_t *sub_y = sub + kBlock, *sub_mp = sub + 2 * kBlock, *sub_mm = sub + 3 * kBlock,
             *sub_row = sub + 4 * kBlock, *sub_voff = sub + 5 * kBlock, *sub_item = sub + 6 * kBlock;

    const uint32_t tid = threadIdx.x;
    const uint32_t d = A.d, R = A.R;
    const uint32_t slots = 1u << A.hash_log2, smask = slots - 1;
    const uint32_t hcap = slots / 2;
    const int G = lanes_per_edge(d);
    const int epl = static_cast<int>(d) / G;
    const int gid = static_cast<int>(tid) / G, glane = static_cast<int>(tid) % G;
    const int ngroups = kBlock / G;

    if (EXACT && A.ctrl->exact_n == 0) return;   // no query needs the exhaustive pass
    const uint32_t ystr = d + 4;  // padded row stride of the relation table in LDS
    for (uint32_t i = tid; i < R * d; i += kBlock) Ys[(i / d) * ystr + i % d] = load1<BF16>(A.Y, i);
    __syncthreads();
    for (uint32_t r = tid; r < R; r += kBlock) {
        float m = 0.0f, sa = 0.0f;
        for (uint32_t i = 0; i < d; ++i) {
            m = fmaxf(m, fabsf(Ys[r * ystr + i]));
            sa += fabsf(Ys[r * ystr + i]);
        }
        ymax[r] = m;
        ysum[r] = sa * (1.0f + static_cast<float>(d) * kUnit * 1.01f);   // rounded up
    }
    const float gamT = gamma_n(static_cast<int>(d) + 3) * 1.001f;   // TransE value bounds

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            uint32_t t;
            if (EXACT) {
                // only the tiles of queries the merge marked
                t = kEmpty;
                if (A.ctrl->exact_n > 0) {
                    for (;;) {
                        const uint32_t u = atomicAdd(&A.ctrl->exact_ctr, 1u);
                        if (u >= A.ctrl->total_tiles) break;
                        const uint32_t tt = A.tile_order[u];   // longest expected first, as in the fast pass
                        const uint32_t q = A.tile_q[tt];
                        if (A.plans[q].flags & kNeedExact) { t = tt; sh->q = q; sh->j = tt - A.plans[q].tile_base; break; }
                    }
                }
            } else {
                t = atomicAdd(&A.ctrl->gather_ctr, 1u);
                if (t < A.ctrl->total_tiles) {
                    t = A.tile_order[t];
                    uint32_t q = A.tile_q[t];
                    sh->q = q;
                    sh->j = t - A.plans[q].tile_base;
                } else {
                    t = kEmpty;
                }
            }
            sh->tile = t;
        }
        __syncthreads();
        const uint32_t tile = sh->tile;
        MHR_PHASE(kPhFetch);
        if (tile == kEmpty) break;
        const uint32_t q = sh->q, j = sh->j;
        const QueryPlan P = A.plans[q];
        const bool fwd = P.dir != 0;
        const uint32_t *Lrp = fwd ? A.out_rp : A.in_rp;
        const uint32_t *Lcol = fwd ? A.out_col : A.in_col;
        const uint32_t *Lmask = fwd ? A.out_mask : A.in_mask;
        const uint32_t *Pcol = fwd ? A.in_col : A.out_col;
        const uint32_t *Pmask = fwd ? A.in_mask : A.out_mask;
        const uint32_t *Pdir_off = fwd ? A.in_dir_off : A.out_dir_off;
        const uint32_t *Pdir_pool = fwd ? A.in_dir_pool : A.out_dir_pool;
        const uint32_t anchor_l = fwd ? P.s : P.t;
        const uint32_t anchor_p = fwd ? P.t : P.s;
        const bool heavy = P.probe_len > hcap;
        const float thr_exact = P.thr;
#ifdef MHR_PHASE_CLOCKS
        ph_heavy = heavy;
#endif
        MHR_COUNT(kCtTiles, 1);

        // ---- tile setup
        for (uint32_t i = tid; i < d; i += kBlock) {
            anc_p[i] = load1<BF16>(A.X, static_cast<size_t>(anchor_p) * d + i);
            anc_l[i] = load1<BF16>(A.X, static_cast<size_t>(anchor_l) * d + i);
        }
        if (!heavy)
            for (uint32_t i = tid; i < slots; i += kBlock) hkeys[i] = kEmpty;
        for (uint32_t i = tid; i < static_cast<uint32_t>(KC); i += kBlock) list[i] = cand_sentinel();
        if (tid == 0) {
            sh->stage_n = 0;
            sh->list_n = 0;
            sh->truncated = 0;
            sh->thr = cand_sentinel();
        }
        __syncthreads();
        const uint8_t *kl = keep_row(A, q, P.s, !fwd), *kp = keep_row(A, q, P.s, fwd);
        if (!heavy) {
            for (uint32_t i = tid; i < P.probe_len; i += kBlock) {
                if (kp && !kp[i]) continue;   // pruned away
                uint32_t y = Pcol[P.probe_beg + i];
                uint32_t slot = (y * 0x9E3779B1u) >> (32 - A.hash_log2);
                for (;;) {
                    uint32_t old = atomicCAS(&hkeys[slot], kEmpty, y);
                    if (old == kEmpty) { hvals[slot] = i; break; }   // the entry's index in the probe row
                    slot = (slot + 1) & smask;
                }
            }
        }
        const uint32_t *dir = nullptr;
        int dsh = 0;
        if (heavy) {
            dir = Pdir_pool + Pdir_off[anchor_p];
            uint32_t nb = next_pow2(P.probe_len) / 2;
            dsh = static_cast<int>(A.id_bits) - (31 - __clz(nb));
        }
        const uint2 ts = A.tile_start[tile];
        const uint2 te = (j + 1 < P.ntiles) ? A.tile_start[tile + 1] : make_uint2(P.list_len, 0u);
        uint64_t npaths = 0;
        float eps_local = 0.0f;
        __syncthreads();
        MHR_PHASE(kPhSetup);

        // ---- row batches
        const uint32_t row_end = (te.y > 0) ? te.x + 1 : te.x;  // exclusive
        for (uint32_t rb = ts.x; rb < row_end; rb += kRowBatch) {
            const uint32_t nrows = min(static_cast<uint32_t>(kRowBatch), row_end - rb);
            uint32_t len = 0, nv = 0;
            if (tid < nrows) {
                uint32_t i = rb + tid;
                uint32_t x = Lcol[P.list_beg + i];
                uint32_t mask = Lmask[P.list_beg + i];
                uint32_t beg = Lrp[x], end = Lrp[x + 1];
                if (i == ts.x) beg += ts.y;
                if (i == te.x) end = Lrp[x] + te.y;
                len = end > beg ? end - beg : 0u;
                if (kl && !kl[i]) len = 0;   // pruned away
                nv = __popc(mask);
                rows[tid].x = x;
                rows[tid].mask = mask;
                rows[tid].beg = beg;
                rows[tid].len = len;
            }
            if (tid < kWave) {  // prefix over the batch (kRowBatch <= one wave)
                uint32_t v = len, w = nv;
                for (int off = 1; off < kWave; off <<= 1) {
                    uint32_t t1 = __shfl_up(v, off, kWave);
                    uint32_t t2 = __shfl_up(w, off, kWave);
                    if (static_cast<int>(tid) >= off) { v += t1; w += t2; }
                }
                if (tid < nrows) {
                    rows[tid].pref = v - len;
                    rows[tid].vbase = w - nv;
                }
                if (tid == nrows - 1) { sh->E = v; sh->rowvals = w; }
            }
            __syncthreads();
            // list-edge weights: one group per row, all of its relations
            for (uint32_t r = gid; r < nrows; r += ngroups) {
                float ex[8], z[8];
                load_lane<BF16>(A.X, rows[r].x, d, glane * epl, epl, ex);
                if constexpr (TE) {
                    // the list edge is x -r-> t (backward) or s -r-> x (forward)
                    float av[8], sz = 0.0f;
#pragma unroll
                    for (int l = 0; l < 8; ++l) {
                        av[l] = (l < epl) ? anc_l[glane * epl + l] : 0.0f;
                        sz += fabsf(av[l]) + fabsf(ex[l]);
                    }
                    sz = group_sum(sz, G) * (1.0f + static_cast<float>(2 * d + 2) * kUnit * 1.01f);   // rounded up
                    score_values_te(fwd ? av : ex, fwd ? ex : av, sz, rows[r].mask, av, ex, sz, 0u, Ys, ysum, ystr,
                                    A.gamma, gamT, G, epl, glane, rowval + rows[r].vbase, roweps + rows[r].vbase,
                                    rowrel + rows[r].vbase);
                } else {
                    float sz = 0.0f;
#pragma unroll
                    for (int l = 0; l < 8; ++l) {
                        z[l] = (l < epl) ? ex[l] * anc_l[glane * epl + l] : 0.0f;
                        sz += fabsf(z[l]);
                    }
                    sz = group_sum(sz, G);
                    score_values(z, sz, rows[r].mask, z, sz, 0u, Ys, ymax, ystr, G, epl, glane,
                                 rowval + rows[r].vbase, roweps + rows[r].vbase, rowrel + rows[r].vbase);
                }
            }
            __syncthreads();
            if (tid < nrows) {
                float fa = 0.0f, em = 0.0f;
                const uint32_t vb = rows[tid].vbase, nvr = __popc(rows[tid].mask);
                for (uint32_t k = 0; k < nvr; ++k) {
                    fa = fmaxf(fa, fabsf(rowval[vb + k]));
                    em = fmaxf(em, roweps[vb + k]);
                }
                sort_desc(rowval + vb, rowrel + vb, nvr);
                rows[tid].fmax = rowval[vb];
                rows[tid].famax = fa;
                rows[tid].emax = em;
            }
            __syncthreads();
            const uint32_t E = sh->E;
            MHR_PHASE(kPhRows);
            MHR_COUNT(kCtRowBatches, 1);
            MHR_COUNT(kCtScanned, E);

            // ---- chunks of scanned entries.  Matches queue up across chunks
            // until a full sub-batch is ready (all of them after the last
            // chunk of the row batch).
            if (tid == 0) sh->qcount = 0;
            __syncthreads();
            // positions and column ids of a chunk's entries; a chunk's ids are
            // loaded while the previous chunk is probed
            auto chunk_entries = [&](uint32_t cb, uint32_t (&ps)[kEPT], uint32_t (&ys)[kEPT]) {
                // the last row with pref <= e, by halving steps of fixed count
                // (kRowBatch = 32 rows) taken for all of the thread's entries
                // together
                uint32_t lo[kEPT];
#pragma unroll
                for (int k = 0; k < kEPT; ++k) lo[k] = 0;
#pragma unroll
                for (uint32_t step = kRowBatch / 2; step > 0; step >>= 1) {
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        const uint32_t e = cb + k * kBlock + tid;
                        const uint32_t c = lo[k] + step;
                        if (c < nrows && rows[c].pref <= e) lo[k] = c;
                    }
                }
#pragma unroll
                for (int k = 0; k < kEPT; ++k) {
                    const uint32_t e = cb + k * kBlock + tid;
                    ps[k] = e < E ? rows[lo[k]].beg + (e - rows[lo[k]].pref) : kEmpty;
                }
#pragma unroll
                for (int k = 0; k < kEPT; ++k) ys[k] = (ps[k] != kEmpty) ? Lcol[ps[k]] : kEmpty;
            };
            uint32_t ps_n[kEPT], ys_n[kEPT];
            chunk_entries(0, ps_n, ys_n);
            for (uint32_t cb = 0; cb < E; cb += kChunk) {
                const bool last = cb + kChunk >= E;
                uint32_t ys[kEPT], ps[kEPT], mps[kEPT];   // mps: index of the hit in the probe row
                bool hits[kEPT];
#pragma unroll
                for (int k = 0; k < kEPT; ++k) {
                    ps[k] = ps_n[k];
                    ys[k] = ys_n[k];
                }
                if (!last) chunk_entries(cb + kChunk, ps_n, ys_n);
                if (!heavy) {
                    // first probe of every entry together, then the rare
                    // collision chains
                    uint32_t slot[kEPT], key[kEPT];
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        slot[k] = (ys[k] * 0x9E3779B1u) >> (32 - A.hash_log2);
                        key[k] = ps[k] != kEmpty ? hkeys[slot[k]] : kEmpty;
                    }
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        const uint32_t y = ys[k];
                        hits[k] = false;
                        mps[k] = 0;
                        while (key[k] != kEmpty && key[k] != y) {
                            slot[k] = (slot[k] + 1) & smask;
                            key[k] = hkeys[slot[k]];
                        }
                        if (ps[k] != kEmpty && key[k] == y) {
                            hits[k] = true;
                            mps[k] = hvals[slot[k]];
                        }
                    }
                } else {
                    // Directory probes in stages, each stage's loads issued
                    // for all of the thread's entries before any is used: the
                    // bucket bounds, then the bucket's first two ids (a bucket
                    // holds two ids on average), then a walk over the rest of
                    // the rare longer buckets, then the masks of the hits.
                    const uint32_t *pc = Pcol + P.probe_beg;
                    uint32_t lo[kEPT], hi[kEPT], c0[kEPT], c1[kEPT], at[kEPT];
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        lo[k] = hi[k] = 0;
                        if (ps[k] != kEmpty) {
                            const uint32_t bk = ys[k] >> dsh;
                            lo[k] = dir[bk];
                            hi[k] = dir[bk + 1];
                        }
                    }
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        c0[k] = (lo[k] < hi[k]) ? pc[lo[k]] : kEmpty;
                        c1[k] = (lo[k] + 1 < hi[k]) ? pc[lo[k] + 1] : kEmpty;
                    }
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        const uint32_t y = ys[k];
                        at[k] = kEmpty;
                        if (lo[k] >= hi[k] || c0[k] > y) continue;   // empty bucket, or ids past y
                        if (c0[k] == y) { at[k] = lo[k]; continue; }
                        if (c1[k] == y) { at[k] = lo[k] + 1; continue; }
                        if (c1[k] > y) continue;                      // includes a bucket of one id
                        for (uint32_t i = lo[k] + 2; i < hi[k]; ++i) {
                            const uint32_t c = pc[i];
                            if (c == y) { at[k] = i; break; }
                            if (c > y) break;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        hits[k] = at[k] != kEmpty && (!kp || kp[at[k]]);
                        mps[k] = at[k];
                    }
                }
                {
                    // one queue reservation per wave for all of its hits
                    const int lane = tid & (kWave - 1);
                    uint64_t bal[kEPT];
                    uint32_t wtot = 0;
#pragma unroll
                    for (int k = 0; k < kEPT; ++k) {
                        bal[k] = __ballot(hits[k]);
                        wtot += static_cast<uint32_t>(__popcll(bal[k]));
                    }
                    if (wtot) {
                        uint32_t base = 0;
                        if (lane == 0) base = atomicAdd(&sh->qcount, wtot);
                        base = __shfl(base, 0, kWave);
                        const uint64_t lt = lane ? (~0ull >> (kWave - lane)) : 0ull;   // lanes below this one
#pragma unroll
                        for (int k = 0; k < kEPT; ++k) {
                            if (hits[k]) {
                                const uint32_t slotq = base + static_cast<uint32_t>(__popcll(bal[k] & lt));
                                qpos[slotq] = ps[k];
                                qmp[slotq] = mps[k];
                            }
                            base += static_cast<uint32_t>(__popcll(bal[k]));
                        }
                    }
                }
                __syncthreads();
                MHR_PHASE(kPhProbe);
                MHR_COUNT(kCtChunks, 1);
                const uint32_t nmatch = sh->qcount;

                // ---- sub-batches of at most kBlock matches (value slab permitting)
                uint32_t m0 = 0;
                while (m0 < nmatch && (last || nmatch - m0 >= static_cast<uint32_t>(kBlock))) {
                    const uint32_t mi = m0 + tid;
                    uint32_t pos = 0, y = 0, mp = 0, mm = 0, row = 0, nv2 = 0;
                    if (mi < nmatch) {
                        pos = qpos[mi];
                        // the probe edge's relation mask, the scanned entry's id
                        // and the middle edge's mask, in one round of loads
                        mp = Pmask[P.probe_beg + qmp[mi]];
                        y = Lcol[pos];
                        mm = Lmask[pos];
                        uint32_t lo = 0;  // row holding pos (the last with beg <= pos)
#pragma unroll
                        for (uint32_t step = kRowBatch / 2; step > 0; step >>= 1) {
                            const uint32_t c = lo + step;
                            if (c < nrows && rows[c].beg <= pos) lo = c;
                        }
                        row = lo;
                        nv2 = __popc(mp) + __popc(mm);
                    }
                    uint32_t vtot;
                    const uint32_t vincl = block_incl_scan<uint32_t>(nv2, sh->red32, &vtot);
                    const bool take = (mi < nmatch) && vincl <= static_cast<uint32_t>(kSlab);
                    const uint32_t ncnt = static_cast<uint32_t>(__syncthreads_count(take));
                    if (take) {
                        sub_y[tid] = y;
                        sub_mp[tid] = mp;
                        sub_mm[tid] = mm;
                        sub_row[tid] = row;
                        sub_voff[tid] = vincl - nv2;
                        if (tid + 1 == ncnt) sh->vn = vincl;   // the taken matches are a prefix
                    }
                    __syncthreads();
                    MHR_PHASE(kPhForm);
                    MHR_COUNT(kCtSubBatches, 1);
                    MHR_COUNT(kCtMatches, ncnt);
                    MHR_COUNT(kCtValues, sh->vn);
                    // scoring on the matrix cores: a wave takes 16 matches at a time.
                    // Lane (row m = lane & 15, k-quarter kq = lane >> 4) holds the
                    // d/4 elements [kq*d/4, (kq+1)*d/4) of match m's vectors
                    //   up = e_y * e_anchor_p   (the probe-side edge y -- anchor)
                    //   um = e_y * e_x          (the middle edge y -- x)
                    // and the same slice of relation row 16*rb + m.  FP32 tables: each
                    // v_mfma_f32_16x16x4f32 multiplies a 16x4 slice of up (or um) by a
                    // 4x16 slice of Y^T, so after d/4 steps D[m][r] = sum_k up[m][k]
                    // Y[r][k].  bfloat16 tables: up and um are exact in FP32 (16
                    // significant bits); each is split into two bfloat16 halves and
                    // v_mfma_f32_16x16x32_bf16 takes four elements of both halves per
                    // lane against the same four elements of Y twice, so every product
                    // is exact and only the FP32 accumulation rounds.  The rounding
                    // error is at most gamma_n sum_k |up_k Y_rk| <= gamma_n max_k |Y_rk|
                    // sum_k |up_k|, with n = d + 3 (FP32) or 2d + 3 (bfloat16).
                    //
                    // TransE-L1 (no products to batch): one group of G lanes per
                    // match computes the distances of its probe edge and middle edge
                    // for the relations in their masks on the vector units; the
                    // values go to the slab in relation order (probe edge, then
                    // middle edge), and the match's sums sum|head| + sum|tail| of both
                    // edges to sub_su_p / sub_su_m for the bounds.
                    if constexpr (TE) {
                        for (uint32_t m = static_cast<uint32_t>(gid); m < ncnt; m += static_cast<uint32_t>(ngroups)) {
                            float ey[8], ex[8], av[8];
                            load_lane<BF16>(A.X, sub_y[m], d, glane * epl, epl, ey);
                            load_lane<BF16>(A.X, rows[sub_row[m]].x, d, glane * epl, epl, ex);
                            float sy = 0.0f, sx = 0.0f, sa = 0.0f;
#pragma unroll
                            for (int l = 0; l < 8; ++l) {
                                av[l] = (l < epl) ? anc_p[glane * epl + l] : 0.0f;
                                sy += fabsf(ey[l]);
                                sx += fabsf(ex[l]);
                                sa += fabsf(av[l]);
                            }
                            const float up = static_cast<float>(2 * d + 2) * kUnit * 1.01f;   // rounding up the sums
                            sy = group_sum(sy, G);
                            sx = group_sum(sx, G);
                            sa = group_sum(sa, G);
                            const float tp = (sy + sa) * (1.0f + up), tm = (sy + sx) * (1.0f + up);
                            const uint32_t vo = sub_voff[m];
                            // backward: probe edge s -> y, middle edge y -> x;
                            // forward: probe edge y -> t, middle edge x -> y
                            score_values_te(fwd ? ey : av, fwd ? av : ey, tp, sub_mp[m], fwd ? ex : ey, fwd ? ey : ex, tm,
                                            sub_mm[m], Ys, ysum, ystr, A.gamma, gamT, G, epl, glane, slab + vo, nullptr,
                                            slab_rel + vo);
                            if (glane == 0) {
                                sub_su_p[m] = tp;
                                sub_su_m[m] = tm;
                            }
                        }
                    } else {
                        const int lane = static_cast<int>(tid) & (kWave - 1), wv = static_cast<int>(tid) / kWave;
                        const int mrow = lane & 15, kq = lane >> 4;
                        const uint32_t KCH = d >> 2;
                        const uint32_t nrb = (R + 15) / 16;
                        for (uint32_t t0 = static_cast<uint32_t>(wv) * 16; t0 < ncnt; t0 += (kBlock / kWave) * 16) {
                            const uint32_t mi = t0 + mrow;
                            const bool mval = mi < ncnt;
                            const uint32_t yrow = mval ? sub_y[mi] : 0u;
                            const uint32_t xrow = mval ? rows[sub_row[mi]].x : 0u;
                            f4 aP[2], aM[2];
#pragma unroll
                            for (int rb = 0; rb < 2; ++rb) {
                                aP[rb] = f4{0.f, 0.f, 0.f, 0.f};
                                aM[rb] = aP[rb];
                            }
                            float sup = 0.0f, sum_ = 0.0f;  // sum_k |up|, sum_k |um| over this lane's slice
                            for (uint32_t kb = 0; kb < KCH; kb += kSpan) {
                                const uint32_t off = static_cast<uint32_t>(kq) * KCH + kb;
                                const uint32_t kn = KCH - kb < kSpan ? KCH - kb : kSpan;
                                float ey[kSpan], ex[kSpan];
                                load_span<BF16, kSpan>(A.X, yrow, d, off, kn, mval, ey);
                                load_span<BF16, kSpan>(A.X, xrow, d, off, kn, mval, ex);
                                // this lane's slices of the anchor row and of its
                                // relation rows, from LDS into registers
                                float av[kSpan], yb[2][kSpan];
                                lds_span<kSpan>(anc_p + off, kn, av);
#pragma unroll
                                for (uint32_t rb = 0; rb < 2; ++rb) {
                                    const uint32_t rr = rb * 16 + static_cast<uint32_t>(mrow);
                                    if (rb < nrb && rr < R) {
                                        lds_span<kSpan>(Ys + rr * ystr + off, kn, yb[rb]);
                                    } else {
#pragma unroll
                                        for (int l = 0; l < static_cast<int>(kSpan); ++l) yb[rb][l] = 0.0f;
                                    }
                                }
                                if constexpr (BF16) {
                                    // four elements per lane per step: A = [hi(u) | lo(u)] and
                                    // B = [y | y] as 8 bfloat16 each, K = 32 per instruction
#pragma unroll
                                    for (uint32_t j = 0; j < kSpan; j += 4) {
                                        if (j < kn) {
                                            u32x4 wp, wm;
#pragma unroll
                                            for (uint32_t e = 0; e < 4; e += 2) {
                                                uint32_t ph[2], pl[2], mh[2], ml[2];
#pragma unroll
                                                for (uint32_t h = 0; h < 2; ++h) {
                                                    const bool ok = j + e + h < kn;
                                                    const float up = ok ? ey[j + e + h] * av[j + e + h] : 0.0f;
                                                    const float um = ok ? ey[j + e + h] * ex[j + e + h] : 0.0f;
                                                    sup += fabsf(up);
                                                    sum_ += fabsf(um);
                                                    split_bf16(up, ph[h], pl[h]);
                                                    split_bf16(um, mh[h], ml[h]);
                                                }
                                                wp[e / 2] = ph[0] | (ph[1] << 16);
                                                wp[2 + e / 2] = pl[0] | (pl[1] << 16);
                                                wm[e / 2] = mh[0] | (mh[1] << 16);
                                                wm[2 + e / 2] = ml[0] | (ml[1] << 16);
                                            }
                                            const bf16x8 ap = __builtin_bit_cast(bf16x8, wp);
                                            const bf16x8 am = __builtin_bit_cast(bf16x8, wm);
#pragma unroll
                                            for (uint32_t rb = 0; rb < 2; ++rb) {
                                                if (rb < nrb) {
                                                    const uint32_t rr = rb * 16 + static_cast<uint32_t>(mrow);
                                                    uint32_t ybits[4];
#pragma unroll
                                                    for (uint32_t e = 0; e < 4; ++e)
                                                        ybits[e] = (rr < R && j + e < kn)
                                                                       ? __float_as_uint(yb[rb][j + e]) >> 16
                                                                       : 0u;
                                                    u32x4 wy;
                                                    wy[0] = ybits[0] | (ybits[1] << 16);
                                                    wy[1] = ybits[2] | (ybits[3] << 16);
                                                    wy[2] = wy[0];
                                                    wy[3] = wy[1];
                                                    const bf16x8 bv = __builtin_bit_cast(bf16x8, wy);
                                                    aP[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ap, bv, aP[rb], 0, 0, 0);
                                                    aM[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am, bv, aM[rb], 0, 0, 0);
                                                }
                                            }
                                        }
                                    }
                                } else {
#pragma unroll
                                for (uint32_t j = 0; j < kSpan; ++j) {
                                    if (j < kn) {
                                        const float up = ey[j] * av[j];
                                        const float um = ey[j] * ex[j];
                                        sup += fabsf(up);
                                        sum_ += fabsf(um);
#pragma unroll
                                        for (uint32_t rb = 0; rb < 2; ++rb) {
                                            if (rb < nrb) {
                                                const float yv = yb[rb][j];
                                                aP[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(up, yv, aP[rb], 0, 0, 0);
                                                aM[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(um, yv, aM[rb], 0, 0, 0);
                                            }
                                        }
                                    }
                                }
                                }
                            }
                            // sum over the four k-quarters of each match (lanes m, m+16, m+32, m+48)
                            sup += __shfl_xor(sup, 16, kWave);
                            sup += __shfl_xor(sup, 32, kWave);
                            sum_ += __shfl_xor(sum_, 16, kWave);
                            sum_ += __shfl_xor(sum_, 32, kWave);
                            if (kq == 0 && mval) {
                                sub_su_p[mi] = sup;
                                sub_su_m[mi] = sum_;
                            }
                            // lane holds D[4*kq + i][mrow] of each relation block: match
                            // t0 + 4*kq + i, relation 16*rb + mrow.  The dot products of
                            // the relations in the match's masks go to the slab in
                            // relation order (probe edge, then middle edge).
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                const uint32_t m = t0 + 4 * static_cast<uint32_t>(kq) + static_cast<uint32_t>(i);
                                if (m >= ncnt) continue;
                                const uint32_t smp = sub_mp[m], smm = sub_mm[m];
                                const uint32_t vo = sub_voff[m], np = __popc(smp);
#pragma unroll
                                for (uint32_t rb = 0; rb < 2; ++rb) {
                                    const uint32_t r = rb * 16 + static_cast<uint32_t>(mrow);
                                    if (rb < nrb && r < R) {
                                        const uint32_t below = (1u << r) - 1u;   // relations before r
                                        if ((smp >> r) & 1u) {
                                            const uint32_t ix = vo + __popc(smp & below);
                                            slab[ix] = aP[rb][i];
                                            slab_rel[ix] = static_cast<uint8_t>(r);
                                        }
                                        if ((smm >> r) & 1u) {
                                            const uint32_t ix = vo + np + __popc(smm & below);
                                            slab[ix] = aM[rb][i];
                                            slab_rel[ix] = static_cast<uint8_t>(r);
                                        }
                                    }
                                }
                            }
                        }
                    }
                    __syncthreads();
                    MHR_PHASE(kPhScore);
                    // centred log-sigmoids of the sub-batch's dot products, dense
                    // over the block
                    if constexpr (!TE) {
                        const uint32_t vn = sh->vn;
                        for (uint32_t ix = tid; ix < vn; ix += kBlock) {
                            float fe;
                            slab[ix] = centred_logsigmoid_e(slab[ix], fe);
                        }
                    }
                    __syncthreads();
                    MHR_PHASE(kPhLogsig);

                    // ---- path enumeration.  A work item is one (match, probe value,
                    // mid value) triple; items are spread over the block so that a
                    // match with many relation combinations does not hold up the
                    // rest.  Each item walks the list row's values, which are sorted
                    // descending, and stops at the first path below the kept K-th
                    // score.  Every skip rests on a bound that uses the score's own
                    // association with the per-edge maxima in place of the values not
                    // yet fixed (FP32 addition is monotone, so the bound is >= every
                    // score it covers).  Skipped paths are counted, not listed.
                    {
                        uint32_t nitems = 0;
                        if (take) {
                            const RowInfo &ri = rows[sub_row[tid]];
                            const uint32_t np = __popc(sub_mp[tid]), nm = __popc(sub_mm[tid]);
                            const uint32_t vo = sub_voff[tid];
                            // per edge of the match: largest value, largest |value|, and
                            // the largest error bound.  A value's bound is
                            // gam * ymax[r] * sum_k |u_k| (the dot product) plus the
                            // log-sigmoid's own error, at most 24 u |f| + 1e-10 on
                            // either of its paths (the series path's
                            // 16 u (|x|/2 + x^2/4) + 1e-10 with |x|/2 <= 1.15 |f| and
                            // x^2/4 <= 0.29 |f| for |x| <= 1/2; the library path's
                            // 16 u |f|).
                            // (four values per step, their loads issued together)
                            float mxp = -__builtin_huge_valf(), axp = 0.0f, yp = 0.0f;
                            float mxm = -__builtin_huge_valf(), axm = 0.0f, ym = 0.0f;
                            for (uint32_t k0 = 0; k0 < np + nm; k0 += 4) {
                                float f[4], yv[4];
                                uint32_t rr[4];
#pragma unroll
                                for (int j = 0; j < 4; ++j) {
                                    const bool ok = k0 + j < np + nm;
                                    f[j] = ok ? slab[vo + k0 + j] : 0.0f;
                                    rr[j] = ok ? slab_rel[vo + k0 + j] : 0u;
                                }
#pragma unroll
                                for (int j = 0; j < 4; ++j) yv[j] = TE ? ysum[rr[j]] : ymax[rr[j]];
#pragma unroll
                                for (int j = 0; j < 4; ++j) {
                                    const uint32_t k = k0 + j;
                                    if (k < np) {
                                        mxp = fmaxf(mxp, f[j]);
                                        axp = fmaxf(axp, fabsf(f[j]));
                                        yp = fmaxf(yp, yv[j]);
                                    } else if (k < np + nm) {
                                        mxm = fmaxf(mxm, f[j]);
                                        axm = fmaxf(axm, fabsf(f[j]));
                                        ym = fmaxf(ym, yv[j]);
                                    }
                                }
                            }
                            // FP32 operands: d products, each rounded once, then the
                            // sum; bfloat16 operands: 2d exact products (hi and lo
                            // halves), then the sum
                            // (TransE-L1: gamma_{d+3} (sum|head| + sum|tail| + sum|Y_r|) +
                            // 2u |f| per value, with the largest sum|Y_r| of the edge's
                            // relations)
                            const float gam = gamma_n(static_cast<int>(BF16 ? 2 * d : d) + 3) * 1.001f;
                            const float ep = TE ? gamT * (sub_su_p[tid] + yp) + 2.0f * kUnit * axp
                                                : gam * yp * sub_su_p[tid] + 24.0f * kUnit * axp + 1e-10f;
                            const float em = TE ? gamT * (sub_su_m[tid] + ym) + 2.0f * kUnit * axm
                                                : gam * ym * sub_su_m[tid] + 24.0f * kUnit * axm + 1e-10f;
                            const float perr = ep + em + ri.emax + 2.01f * kUnit * (axp + axm + ri.famax);
                            eps_local = fmaxf(eps_local, perr);
                            sub_su_p[tid] = perr;   // now: the bound on a path's fast-score error
                            npaths += static_cast<uint64_t>(np) * nm * __popc(ri.mask);
                            // exhaustive pass: no path of this match can be returned
                            // unless its fast score plus the bound reaches the K-th
                            // score's lower bound
                            const float tS0 = EXACT ? fmaxf(thr_exact, P.kth_low - perr) : sh->thr.s;
                            if (combine3(fwd, mxp, mxm, ri.fmax) >= tS0)
                                nitems = np * nm;
                            else
                                sh->truncated = 1;   // no path through this match can be kept
                        }
                        uint32_t ntot;
                        const uint32_t iincl = block_incl_scan<uint32_t>(nitems, sh->red32, &ntot);
                        sub_item[tid] = iincl - nitems;
                        // Tiles probing through the directory leave the LDS hash table
                        // unused: it then maps each item to its match (16-bit ids), so
                        // the walk below reads the match instead of searching for it.
                        const bool item_tab = heavy && ntot <= 4 * slots;
                        uint16_t *item_match = reinterpret_cast<uint16_t *>(hkeys);   // hkeys and hvals: 4 * slots ids
                        if (item_tab) {
                            // short ranges by their own thread; long ones by the whole
                            // wave, one range at a time (a match can hold hundreds of
                            // items, which one thread would write while the rest wait)
                            const uint32_t beg = iincl - nitems;
                            const bool longr = nitems > kItemRun;
                            if (!longr)
                                for (uint32_t j = 0; j < nitems; ++j) item_match[beg + j] = static_cast<uint16_t>(tid);
                            const uint32_t lane = tid & (kWave - 1);
                            for (uint64_t lm = __ballot(longr); lm != 0; lm &= lm - 1) {
                                const int L = __ffsll(static_cast<unsigned long long>(lm)) - 1;
                                const uint32_t b = __shfl(beg, L, kWave), n = __shfl(nitems, L, kWave);
                                const uint16_t owner = static_cast<uint16_t>(tid - lane + static_cast<uint32_t>(L));
                                for (uint32_t j = lane; j < n; j += kWave) item_match[b + j] = owner;
                            }
                        }
                        __syncthreads();
                        MHR_PHASE(kPhBounds);
                        MHR_COUNT(kCtItems, ntot);
                        // Each thread walks the items tid, tid + kBlock, ...; its cursor
                        // (item, list position) survives the rounds.  A round runs until
                        // every thread has walked all its items or some path found the
                        // stage full; that path is retried after the stage is merged, so
                        // a round ends with a barrier only when the stage fills.
                        uint32_t it = tid;
                        bool have = false;
                        uint32_t il = 0, nl = 0, lb = 0, sx = 0, sy = 0, rp_ = 0, rm_ = 0;
                        float perr_it = 0.0f;   // fast-score error bound of the current item's paths
                        float fp = 0.0f, fm = 0.0f;
                        for (;;) {
                            const Cand thr = sh->thr;
                            const float tS = EXACT ? thr_exact : thr.s;
                            // exhaustive pass: a path whose fast score plus its error
                            // bound stays below the kept list's threshold cannot enter
                            // the list either
                            // (and none below the lower bound on the query's true K-th
                            // score can be returned)
                            const float tL = !EXACT ? -__builtin_huge_valf()
                                                    : fmaxf(P.kth_low, thr.a != 0xFFFFFFFFu
                                                                            ? thr.s - 1e-6f * fabsf(thr.s)
                                                                            : -__builtin_huge_valf());
                            bool dropped = false, full = false;
                            for (;;) {
                                if (!have) {
                                    if (it >= ntot) break;
                                    // the last match whose items start at or before `it`
                                    uint32_t lo = 0;
                                    if (item_tab) {
                                        lo = item_match[it];
                                    } else {
                                        uint32_t hi = ncnt;
                                        while (hi - lo > 1) {
                                            const uint32_t mid = (lo + hi) >> 1;
                                            if (sub_item[mid] <= it) lo = mid; else hi = mid;
                                        }
                                    }
                                    const uint32_t m = lo;
                                    const uint32_t np = __popc(sub_mp[m]), nm = __popc(sub_mm[m]);
                                    const uint32_t l = it - sub_item[m];
                                    const uint32_t ip = l / nm, im = l - ip * nm;
                                    const uint32_t vo = sub_voff[m];
                                    fp = slab[vo + ip];
                                    fm = slab[vo + np + im];
                                    const RowInfo &ri = rows[sub_row[m]];
                                    perr_it = sub_su_p[m];
                                    if (combine3(fwd, fp, fm, ri.fmax) < fmaxf(tS, tL - perr_it)) {
                                        dropped = true;   // every path of this pair of values
                                        it += kBlock;
                                        continue;
                                    }
                                    rp_ = slab_rel[vo + ip];
                                    rm_ = slab_rel[vo + np + im];
                                    lb = ri.vbase;
                                    nl = __popc(ri.mask);
                                    sx = ri.x;
                                    sy = sub_y[m];
                                    il = 0;
                                    have = true;
                                }
                                if (il >= nl) {
                                    have = false;
                                    it += kBlock;
                                    continue;
                                }
                                const float fl = rowval[lb + il];
                                const float S = combine3(fwd, fp, fm, fl);
                                if (S < fmaxf(tS, tL - perr_it)) {
                                    dropped = true;   // this and every later list value
                                    have = false;
                                    it += kBlock;
                                    continue;
                                }
                                const uint32_t rl_ = rowrel[lb + il];
                                Cand cd;
                                cd.a = fwd ? sx : sy;
                                cd.b = fwd ? sy : sx;
                                const uint32_t r1 = fwd ? rl_ : rp_, r3 = fwd ? rp_ : rl_;
                                cd.rel = (r1 << 16) | (rm_ << 8) | r3;
                                cd.s = S;
                                cd.s_lo = 0.0f;
                                cd.eps = 0.0f;
                                // exhaustive pass: the path is staged with its fast score
                                // unless even its error bound cannot reach the kept
                                // list's threshold (its float-float score is taken when
                                // the stage is merged); fast pass: the total order
                                const bool keep = EXACT || cand_better(cd, thr);
                                if (keep) {
                                    const uint32_t slot = atomicAdd(&sh->stage_n, 1u);
                                    if (slot >= static_cast<uint32_t>(kStage)) {
                                        full = true;   // this path again after the merge
                                        break;
                                    }
                                    stage[slot] = cd;
                                } else {
                                    dropped = true;
                                }
                                ++il;
                            }
                            if (dropped) sh->truncated = 1;
                            if (!__syncthreads_or(full)) break;   // every item walked
                            // the stage is full (the reservations past its end wrote nothing)
                            if (tid == 0) sh->stage_n = kStage;
                            __syncthreads();
                            MHR_PHASE(kPhEnum);
                            MHR_COUNT(kCtStaged, kStage);
                            MHR_COUNT(kCtMerges, 1);
                            merge_stage<KC, EXACT, BF16, TE>(list, stage, sh, mkeys, A, P.s, P.t);
                            MHR_PHASE(kPhMerge);
                        }
                    }
                    m0 += ncnt;
                    __syncthreads();
                    MHR_PHASE(kPhEnum);
                }
                // the remaining matches (fewer than a sub-batch) move to the
                // queue's front; the next chunk appends after them
                const uint32_t rem = nmatch - m0;
                if (rem > 0 && m0 > 0) {
                    uint32_t p_ = 0, mp_ = 0;
                    if (tid < rem) {
                        p_ = qpos[m0 + tid];
                        mp_ = qmp[m0 + tid];
                    }
                    __syncthreads();
                    if (tid < rem) {
                        qpos[tid] = p_;
                        qmp[tid] = mp_;
                    }
                }
                if (tid == 0) sh->qcount = rem;
                __syncthreads();
                MHR_PHASE(kPhProbe);
            }
            __syncthreads();  // rows[] and sh->E are rewritten by the next batch
        }
        // ---- tile end: final merge and output
        __syncthreads();
        MHR_COUNT(kCtStaged, sh->stage_n);
        MHR_COUNT(kCtMerges, sh->stage_n > 0 ? 1 : 0);
        if (sh->stage_n > 0) merge_stage<KC, EXACT, BF16, TE>(list, stage, sh, mkeys, A, P.s, P.t);
        float em = block_max<>(eps_local, sh->redf);
        uint64_t npt = block_sum<uint64_t>(npaths, sh->red64);
        MHR_PHASE(kPhEnd);
        Cand *out = A.cands + static_cast<uint64_t>(tile) * KC;
        for (uint32_t i = tid; i < static_cast<uint32_t>(KC); i += kBlock) out[i] = list[i];
        if (tid == 0) {
            TileHeader h{};
            h.count = sh->list_n;
            h.truncated = sh->truncated;
            h.cutoff = (sh->list_n == static_cast<uint32_t>(KC)) ? list[KC - 1].s : -__builtin_huge_valf();
            h.eps = em;
            h.npaths = npt;
            A.hdr[tile] = h;
        }
    }
#ifdef MHR_PHASE_CLOCKS
    __syncthreads();
    if (threadIdx.x < 2 * kPhSlots) atomicAdd(&g_phase_ticks[threadIdx.x], ph_acc[threadIdx.x]);
#endif
}
// ---------------------------------------------------------------------------
// merge
// ---------------------------------------------------------------------------
__device__ inline void write_sentinels(mhr_path *row, uint32_t from, uint32_t kmax) {
    for (uint32_t i = from + threadIdx.x; i < kmax; i += blockDim.x) {
        mhr_path p;
        p.a = 0xFFFFFFFFu; p.b = 0xFFFFFFFFu;
        p.r1 = 0xFFFF; p.r2 = 0xFFFF; p.r3 = 0xFFFF; p.flags = 0;
        p.score = -__builtin_huge_valf();
        p.err_bound = 0.0f;
        row[i] = p;
    }
}

// Writes the first kk of the rescored, sorted candidates c[0..nc).
__device__ inline void write_result(mhr_path *row, const Cand *c, uint32_t nc, uint32_t kk, uint32_t kmax) {
    for (uint32_t i = threadIdx.x; i < kk; i += blockDim.x) {
        const Cand x = c[i];
        mhr_path p;
        p.a = x.a;
        p.b = x.b;
        p.r1 = static_cast<uint16_t>((x.rel >> 16) & 0xFF);
        p.r2 = static_cast<uint16_t>((x.rel >> 8) & 0xFF);
        p.r3 = static_cast<uint16_t>(x.rel & 0xFF);
        uint16_t fl = MHR_PATH_RESCORED;
        if (i + 1 < nc) {
            const Cand y = c[i + 1];
            ff dlt = ff_add(ff{x.s, x.s_lo}, ff{-y.s, -y.s_lo});
            bool equal = (x.s == y.s && x.s_lo == y.s_lo);
            if (!equal && fabsf(dlt.hi) <= (x.eps + y.eps) * 1.01f) fl |= MHR_PATH_PRECISION_TIE;
        }
        p.flags = fl;
        p.score = x.s;  // the FP32 value nearest the float-float score
        p.err_bound = (x.eps + fabsf(x.s_lo)) * (1.0f + 4.0f * kUnit);
        row[i] = p;
    }
    write_sentinels(row, kk, kmax);
}

// Streams the query's tile lists through LDS (kMergeSlots candidates at a
// time) and leaves the best KC in c[0..KC), sorted by the total order (the
// exhaustive pass, whose scores are final).
template <int KC>
__device__ inline void collect_top_exact(const GArgs &A, const QueryPlan &P, Cand *c) {
    constexpr uint32_t per = (kMergeSlots - KC) / KC;  // tile lists per step
    if (P.ntiles == 1) {   // one tile: its list is already sorted and complete
        const uint32_t cnt = A.hdr[P.tile_base].count;
        for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(KC); i += blockDim.x)
            c[i] = i < cnt ? A.cands[static_cast<uint64_t>(P.tile_base) * KC + i] : cand_sentinel();
        __syncthreads();
        return;
    }
    for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(KC); i += blockDim.x) c[i] = cand_sentinel();
    __syncthreads();
    for (uint32_t j0 = 0; j0 < P.ntiles; j0 += per) {
        const uint32_t nt = min(per, P.ntiles - j0);
        const uint32_t n = next_pow2((nt + 1) * static_cast<uint32_t>(KC));   // <= kMergeSlots
        for (uint32_t i = threadIdx.x; i < n - KC; i += blockDim.x) {
            const uint32_t jt = i / KC, k = i % KC;
            Cand x = cand_sentinel();
            if (jt < nt) {
                const uint32_t tile = P.tile_base + j0 + jt;
                if (k < A.hdr[tile].count) x = A.cands[static_cast<uint64_t>(tile) * KC + k];
            }
            c[KC + i] = x;
        }
        __syncthreads();
        block_sort_cands(c, static_cast<int>(n));
    }
}

// Fast-pass selection state (shared memory).
struct SelShared {
    uint32_t prefix;    // radix select: key bits fixed so far
    uint32_t need;      // candidates still to take among keys matching the prefix
    uint32_t nsel;      // candidates gathered
    uint32_t neq;       // candidates seen at the threshold key
    uint32_t dropkey;   // best key left out (0: none)
    uint32_t hist[256];
};
constexpr uint32_t kSelCache = 8192;   // keys of the tile lists kept in LDS between passes

template <int KC>
__device__ __forceinline__ uint32_t list_key(const GArgs &A, const QueryPlan &P, uint32_t i) {
    const uint32_t tile = P.tile_base + i / KC, k = i % KC;
    return k < A.hdr[tile].count ? fkey(A.cands[static_cast<uint64_t>(tile) * KC + k].s) : 0u;
}

// The fast pass's best KC over the query's tile lists (nvalid candidates in
// all), into c[0..KC) sorted by score, highest first, sentinels after the
// last; returns the best score left out (-inf when none).  Scores are
// compared by their order-preserving 32-bit keys (never 0 for a real score;
// 0 marks an empty slot).  A radix select, 8 key bits per pass from the top,
// finds the KC-th largest key T; a last pass gathers every candidate above T
// and as many at T as fit (which of equal keys is arbitrary: the score decides
// everything that follows).
template <int KC>
__device__ float select_top(const GArgs &A, const QueryPlan &P, uint32_t nvalid, Cand *c, uint64_t *keys,
                            uint32_t *cache, SelShared *ss) {
    const uint32_t tid = threadIdx.x;
    const uint32_t N = P.ntiles * static_cast<uint32_t>(KC);
    const bool cached = N <= kSelCache;
    if (tid == 0) {
        ss->prefix = 0;
        ss->nsel = 0;
        ss->neq = 0;
        ss->dropkey = 0;
        ss->need = nvalid > static_cast<uint32_t>(KC) ? static_cast<uint32_t>(KC) : 0u;
    }
    __syncthreads();
    uint32_t T = 0;   // with nvalid <= KC every real key is above T
    if (nvalid > static_cast<uint32_t>(KC)) {
        uint32_t pmask = 0;
        for (int shift = 24; shift >= 0; shift -= 8) {
            for (uint32_t i = tid; i < 256; i += kMergeBlock) ss->hist[i] = 0;
            __syncthreads();
            const uint32_t prefix = ss->prefix;
            for (uint32_t i = tid; i < N; i += kMergeBlock) {
                uint32_t key;
                if (shift == 24) {
                    key = list_key<KC>(A, P, i);
                    if (cached) cache[i] = key;
                } else {
                    key = cached ? cache[i] : list_key<KC>(A, P, i);
                }
                if (key != 0 && (key & pmask) == prefix) atomicAdd(&ss->hist[(key >> shift) & 255u], 1u);
            }
            __syncthreads();
            if (tid < kWave) {
                // lane l holds bins 4l..4l+3; the bin where the count from the
                // top reaches `need` fixes the next 8 bits
                const uint32_t lane = tid;
                const uint32_t h0 = ss->hist[4 * lane], h1 = ss->hist[4 * lane + 1], h2 = ss->hist[4 * lane + 2],
                               h3 = ss->hist[4 * lane + 3];
                const uint32_t own = h0 + h1 + h2 + h3;
                uint32_t incl = own;   // count in this lane's bins and all higher ones
                for (int off = 1; off < kWave; off <<= 1) {
                    const uint32_t t = __shfl_down(incl, off, kWave);
                    if (lane + off < static_cast<uint32_t>(kWave)) incl += t;
                }
                const uint32_t above = incl - own;
                const uint32_t need = ss->need;
                if (above < need && need <= incl) {
                    uint32_t acc = above, b;
                    if (acc + h3 >= need) b = 3;
                    else if (acc += h3, acc + h2 >= need) b = 2;
                    else if (acc += h2, acc + h1 >= need) b = 1;
                    else { acc += h1; b = 0; }
                    ss->prefix = prefix | ((4 * lane + b) << shift);
                    ss->need = need - acc;
                }
            }
            pmask |= 255u << shift;
            __syncthreads();
        }
        T = ss->prefix;
    }
    const uint32_t need_eq = ss->need;   // candidates to take at key T
    uint32_t drop = 0;
    for (uint32_t i = tid; i < N; i += kMergeBlock) {
        const uint32_t key = cached && nvalid > static_cast<uint32_t>(KC) ? cache[i] : list_key<KC>(A, P, i);
        if (key == 0) continue;
        bool take = key > T;
        if (!take && key == T) take = atomicAdd(&ss->neq, 1u) < need_eq;
        if (take) {
            const uint32_t slot = atomicAdd(&ss->nsel, 1u);
            c[slot] = A.cands[static_cast<uint64_t>(P.tile_base + i / KC) * KC + i % KC];
        } else {
            drop = max(drop, key);
        }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) drop = max(drop, static_cast<uint32_t>(__shfl_xor(drop, off, kWave)));
    if ((tid & (kWave - 1)) == 0 && drop) atomicMax(&ss->dropkey, drop);
    __syncthreads();
    const uint32_t nsel = ss->nsel;
    // sort the KC by key, highest first
    if (tid < static_cast<uint32_t>(KC))
        keys[tid] = tid < nsel ? (static_cast<uint64_t>(fkey(c[tid].s)) << 32) | tid : 0ull;
    __syncthreads();
    block_sort_keys_desc(keys, KC);
    Cand x = cand_sentinel();
    if (tid < nsel) x = c[static_cast<uint32_t>(keys[tid])];
    __syncthreads();
    if (tid < static_cast<uint32_t>(KC)) c[tid] = x;
    const uint32_t dk = ss->dropkey;
    __syncthreads();
    if (dk == 0) return -__builtin_huge_valf();
    return __uint_as_float((dk & 0x80000000u) ? (dk & 0x7FFFFFFFu) : ~dk);
}

template <bool BF16, int KC, bool TE>
__global__ __launch_bounds__(kMergeBlock) void merge_kernel(GArgs A, mhr_path *out, uint32_t *out_count,
                                                       uint64_t *out_total, uint32_t *out_status, uint32_t kmax) {
    static_assert(KC <= kMergeBlock, "one thread per kept candidate");
    extern __shared__ __align__(16) unsigned char smem[];
    Cand *c = reinterpret_cast<Cand *>(smem);
    uint64_t *keys = reinterpret_cast<uint64_t *>(c + KC);
    uint32_t *cache = reinterpret_cast<uint32_t *>(keys + KC);
    __shared__ SelShared ss;
    __shared__ uint32_t red32[kBlock / kWave];
    __shared__ uint64_t red64[kBlock / kWave];
    __shared__ float redf[kBlock / kWave];
    const uint32_t q = blockIdx.x;
    const QueryPlan P = A.plans[q];
    mhr_path *row = out + static_cast<uint64_t>(q) * kmax;
    if (P.status != 0 || P.ntiles == 0) {
        if (threadIdx.x == 0) {
            out_count[q] = 0;
            if (out_total) out_total[q] = 0;
            if (out_status) out_status[q] = P.status;
        }
        write_sentinels(row, 0, kmax);
        return;
    }
    // tile headers: candidates, largest error bound, paths
    uint32_t n_part = 0;
    float e_part = 0.0f;
    uint64_t t_part = 0;
    for (uint32_t j = threadIdx.x; j < P.ntiles; j += kMergeBlock) {
        const TileHeader &h = A.hdr[P.tile_base + j];
        n_part += h.count;
        e_part = fmaxf(e_part, h.eps);
        t_part += h.npaths;
    }
    const uint32_t cnt = block_sum<uint32_t, kMergeBlock>(n_part, red32);
    const float eps = block_max<kMergeBlock>(e_part, redf);
    const uint64_t tot = block_sum<uint64_t, kMergeBlock>(t_part, red64);
    const float s_drop = select_top<KC>(A, P, cnt, c, keys, cache, &ss);
    const uint32_t kept = min(cnt, static_cast<uint32_t>(KC));
    const uint32_t kk = min(P.k, cnt);
    if (kk == 0) {
        if (threadIdx.x == 0) {
            out_count[q] = 0;
            if (out_total) out_total[q] = tot;
            if (out_status) out_status[q] = 0;
        }
        write_sentinels(row, 0, kmax);
        return;
    }
    const float theta = c[kk - 1].s;
    // band threshold, rounded down generously
    const float thr = (theta - fmaxf(2.0f * eps, A.band_abs)) - 4.0f * kUnit * fabsf(theta) - 1e-30f;
    // K candidates have fast scores >= theta and errors <= eps, so the true
    // K-th score is at least theta - eps; a path whose fast score is below
    // theta - 2 eps (rounded down generously) scores strictly less and can
    // never be returned.  Only such a path may be dropped unseen: the
    // exhaustive pass is needed when a tile list or this selection dropped a
    // candidate at or above that line, whatever the band's width (a wider
    // band only adds kept candidates to the rescoring below).
    const float thr_ret = (theta - 2.0f * eps) - 4.0f * kUnit * fabsf(theta) - 1e-30f;
    int over_part = (threadIdx.x == 0 && s_drop >= thr_ret) ? 1 : 0;
    for (uint32_t j = threadIdx.x; j < P.ntiles; j += kMergeBlock) {
        const TileHeader &h = A.hdr[P.tile_base + j];
        if (h.truncated && h.cutoff >= thr_ret) over_part = 1;
    }
    // the band: the sorted prefix at or above the threshold
    const uint32_t nb = static_cast<uint32_t>(__syncthreads_count(threadIdx.x < kept && c[threadIdx.x].s >= thr));
    if (__syncthreads_or(over_part)) {
        if (threadIdx.x == 0) {
            A.plans[q].flags = kNeedExact;
            A.plans[q].thr = thr;
            // the lower bound on the true K-th score, rounded down generously
            A.plans[q].kth_low = (theta - eps) - 4.0f * kUnit * fabsf(theta) - 1e-30f;
            A.plans[q].total = tot;
            atomicAdd(&A.ctrl->exact_n, 1u);
        }
        return;
    }
    // a group of kRescoreLanes lanes rescores one band candidate
    for (uint32_t i = threadIdx.x / kRescoreLanes; i < nb; i += blockDim.x / kRescoreLanes) {
        Cand x = c[i];
        const uint32_t r1 = (x.rel >> 16) & 0xFF, r2 = (x.rel >> 8) & 0xFF, r3 = x.rel & 0xFF;
        float e;
        ff sc = path_score_ff<BF16, kRescoreLanes, TE>(A, P.s, x.a, x.b, P.t, r1, r2, r3, &e);
        x.s = sc.hi;
        x.s_lo = sc.lo;
        x.eps = e;
        if ((threadIdx.x & (kRescoreLanes - 1)) == 0) c[i] = x;
    }
    const uint32_t nb2 = next_pow2(nb);
    for (uint32_t i = nb + threadIdx.x; i < nb2; i += blockDim.x) c[i] = cand_sentinel();
    __syncthreads();
    block_sort_cands(c, static_cast<int>(nb2));
    write_result(row, c, nb, kk, kmax);
    if (threadIdx.x == 0) {
        out_count[q] = kk;
        if (out_total) out_total[q] = tot;
        if (out_status) out_status[q] = 0;
    }
}

// Merge of the exhaustive pass: the tile lists already hold float-float
// scores of every path above the threshold.
template <int KC>
__global__ __launch_bounds__(kBlock) void merge_exact_kernel(GArgs A, mhr_path *out, uint32_t *out_count,
                                                             uint64_t *out_total, uint32_t *out_status,
                                                             uint32_t kmax) {
    extern __shared__ __align__(16) unsigned char smem[];
    Cand *c = reinterpret_cast<Cand *>(smem);
    __shared__ uint32_t s_n;
    const uint32_t q = blockIdx.x;
    const QueryPlan P = A.plans[q];
    if (P.status != 0 || !(P.flags & kNeedExact)) return;
    mhr_path *row = out + static_cast<uint64_t>(q) * kmax;
    if (threadIdx.x == 0) {
        uint32_t n = 0;
        for (uint32_t j = 0; j < P.ntiles; ++j) n += A.hdr[P.tile_base + j].count;
        s_n = n;
    }
    collect_top_exact<KC>(A, P, c);
    const uint32_t kept = min(s_n, static_cast<uint32_t>(KC));
    const uint32_t kk = min(P.k, kept);
    write_result(row, c, kept, kk, kmax);
    if (threadIdx.x == 0) {
        out_count[q] = kk;
        if (out_total) out_total[q] = P.total;
        if (out_status) out_status[q] = MHR_Q_EXACT_PASS;
    }
}

// ---------------------------------------------------------------------------
// edge weights (unit entry point)
// ---------------------------------------------------------------------------
template <bool BF16, bool TE>
__global__ void edge_weight_kernel(GArgs A, uint64_t ne, const uint32_t *u, const uint32_t *r, const uint32_t *v,
                                   float *w32, float *e32, float *whi, float *wlo) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const uint32_t uu = u[i], rr = r[i], vv = v[i];
    const size_t d = A.d;
    float w, err;
    if (TE) {
        // the fast pass's evaluation: gamma - sum_k |(X[u,k] + Y[r,k]) - X[v,k]|
        float l1 = 0.0f, ts = 0.0f;
        for (uint32_t k = 0; k < A.d; ++k) {
            const float xu = load1<BF16>(A.X, uu * d + k), yr = load1<BF16>(A.Y, rr * d + k);
            const float xv = load1<BF16>(A.X, vv * d + k);
            l1 += fabsf((xu + yr) - xv);
            ts += fabsf(xu) + fabsf(yr) + fabsf(xv);
        }
        w = A.gamma - l1;
        err = gamma_n(static_cast<int>(A.d) + 3) * 1.001f * ts * (1.0f + 3.0f * static_cast<float>(A.d) * kUnit) +
              2.0f * kUnit * fabsf(w);
        float asf;
        const ff wf = ff_add_f(ff_neg(edge_l1_ff<BF16>(A, uu, rr, vv, &asf)), A.gamma);
        if (whi) whi[i] = wf.hi;
        if (wlo) wlo[i] = wf.lo;
    } else {
        float x = 0.0f, as = 0.0f;
        for (uint32_t k = 0; k < A.d; ++k) {
            float z = load1<BF16>(A.X, uu * d + k) * load1<BF16>(A.Y, rr * d + k);
            float xv = load1<BF16>(A.X, vv * d + k);
            x = __builtin_fmaf(z, xv, x);
            as += fabsf(z * xv);
        }
        float fe;
        float f = centred_logsigmoid_e(x, fe);   // the fast pass's evaluation and bound
        w = f - kLn2f;
        err = gamma_n(static_cast<int>(A.d) + 2) * as + fe + kUnit * fabsf(w) + kUnit * kLn2f;
        float asf;
        ff wf = ff_logsigmoid(edge_x_ff<BF16>(A, uu, rr, vv, &asf));
        if (whi) whi[i] = wf.hi;
        if (wlo) wlo[i] = wf.lo;
    }
    if (w32) w32[i] = w;
    if (e32) e32[i] = err;
}

// The fast-pass FP32 weight of one edge (DistMult: the FMA dot product and
// the centred log-sigmoid less ln 2; TransE-L1: gamma minus the distance).
template <bool BF16, bool TE>
__device__ inline float edge_w32(const GArgs &A, uint32_t uu, uint32_t rr, uint32_t vv) {
    const size_t d = A.d;
    if (TE) {
        float l1 = 0.0f;
        for (uint32_t k = 0; k < A.d; ++k)
            l1 += fabsf((load1<BF16>(A.X, uu * d + k) + load1<BF16>(A.Y, rr * d + k)) - load1<BF16>(A.X, vv * d + k));
        return A.gamma - l1;
    }
    float x = 0.0f;
    for (uint32_t k = 0; k < A.d; ++k)
        x = __builtin_fmaf(load1<BF16>(A.X, uu * d + k) * load1<BF16>(A.Y, rr * d + k), load1<BF16>(A.X, vv * d + k), x);
    float fe;
    return centred_logsigmoid_e(x, fe) - kLn2f;
}

// The weight of each pruner candidate's own edge: s -r-> v for a first-hop
// candidate of query q, v -r-> t for a second-hop one (the ranking a
// per-level score beam would use).
template <bool BF16, bool TE>
__global__ void candidate_weight_kernel(GArgs A, uint64_t n, const uint32_t *src, const uint32_t *dst,
                                        const uint32_t *cq, const uint32_t *cv, const uint32_t *cr, float *w) {
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t qw = cq[i], q = qw & 0x7FFFFFFFu;
    const bool hop2 = (qw & 0x80000000u) != 0;
    const uint32_t u = hop2 ? cv[i] : src[q], v = hop2 ? dst[q] : cv[i];
    w[i] = edge_w32<BF16, TE>(A, u, cr[i], v);
}

GArgs make_args(const mhr_graph *g) {
    GArgs A{};
    A.out_rp = g->out.row_ptr; A.out_col = g->out.col; A.out_mask = g->out.rmask;
    A.out_dir_off = g->out.dir_off; A.out_dir_pool = g->out.dir_pool;
    A.in_rp = g->in.row_ptr; A.in_col = g->in.col; A.in_mask = g->in.rmask;
    A.in_dir_off = g->in.dir_off; A.in_dir_pool = g->in.dir_pool;
    A.X = g->X; A.Y = g->Y;
    A.n = g->n; A.R = g->R; A.d = g->dim; A.id_bits = g->id_bits;
    A.gamma = g->gamma;
    return A;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct WsLayout {
    size_t ctrl, plans, tile_start, tile_q, tile_order, exact_list, hdr, cands, total;
};

uint32_t kc_for(uint32_t kmax) {
    uint32_t kc = 64;
    while (kc < kmax + 32) kc <<= 1;
    return kc;
}

WsLayout ws_layout(uint32_t nq, uint32_t kc) {
    const uint32_t tcap = tile_capacity(nq);
    WsLayout W{};
    size_t o = 0;
    auto al = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    W.ctrl = o; o = al(o + sizeof(Control));
    W.plans = o; o = al(o + size_t(nq) * sizeof(QueryPlan));
    W.tile_start = o; o = al(o + size_t(tcap) * sizeof(uint2));
    W.tile_q = o; o = al(o + size_t(tcap) * sizeof(uint32_t));
    W.tile_order = o; o = al(o + size_t(tcap) * sizeof(uint32_t));
    W.exact_list = o; o = al(o + size_t(nq) * sizeof(uint32_t));
    W.hdr = o; o = al(o + size_t(tcap) * sizeof(TileHeader));
    W.cands = o; o = al(o + size_t(tcap) * kc * sizeof(Cand));
    W.total = o;
    return W;
}

int g_num_cus = 0;

constexpr size_t kLdsBytes = 160 * 1024;
// dynamic LDS a gather workgroup may take: the CU's LDS less a reserve for
// the kernels' own static shared variables (a few hundred bytes)
constexpr size_t kDynLdsBytes = kLdsBytes - 1024;

// The probe-table size: the caller's choice, else the largest table of at
// most 2^kDefaultHashLog2 slots whose gather workgroup fits in LDS (large
// embedding dimensions and relation counts leave less room for it).
uint32_t hash_log2_for(const mhr_graph *g, const mhr_query_opts *o, uint32_t kmax) {
    if (o && o->hash_log2) return o->hash_log2;
    uint32_t h = kDefaultHashLog2;
    while (h > 10 && gather_layout(h, g->R, g->dim, kc_for(kmax)).total > kDynLdsBytes) --h;
    return h;
}

template <bool BF16, int KC, bool TE>
mhr_status launch_all(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq, const uint32_t *src,
                      const uint32_t *dst, const uint32_t *k, uint32_t kmax, mhr_path *out, uint32_t *out_count,
                      uint64_t *out_total, uint32_t *out_status, void *ws, hipStream_t st,
                      const mhr_phase_events *ev, const uint8_t *keep, const uint64_t *keep_off) {
    GArgs A = make_args(g);
    A.band_abs = o ? o->band_abs : 0.0f;
    A.keep = keep;
    A.keep_off = keep_off;
    auto rec = [&](void *e) -> hipError_t {
        return e ? hipEventRecord(static_cast<hipEvent_t>(e), st) : hipSuccess;
    };
    const WsLayout W = ws_layout(nq, KC);
    char *base = static_cast<char *>(ws);
    A.ctrl = reinterpret_cast<Control *>(base + W.ctrl);
    A.plans = reinterpret_cast<QueryPlan *>(base + W.plans);
    A.tile_start = reinterpret_cast<uint2 *>(base + W.tile_start);
    A.tile_q = reinterpret_cast<uint32_t *>(base + W.tile_q);
    A.tile_order = reinterpret_cast<uint32_t *>(base + W.tile_order);
    A.exact_list = reinterpret_cast<uint32_t *>(base + W.exact_list);
    A.hdr = reinterpret_cast<TileHeader *>(base + W.hdr);
    A.cands = reinterpret_cast<Cand *>(base + W.cands);
    A.tcap = tile_capacity(nq);
    A.nq = nq;
    A.kc = KC;
    A.hash_log2 = hash_log2_for(g, o, kmax);
    const uint32_t tile_edges = (o && o->tile_edges) ? o->tile_edges : kDefaultTileEdges;
    A.tile_edges = tile_edges;
    if (g_num_cus == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) g_num_cus = prop.multiProcessorCount;
        if (g_num_cus <= 0) g_num_cus = 256;
    }
    const GatherLayout GL = gather_layout(A.hash_log2, A.R, A.d, KC);
    uint32_t grid = (o && o->grid_blocks) ? o->grid_blocks : 0u;
    if (grid == 0) {
        // persistent: as many workgroups as can be resident at once
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(
                                                             gather_kernel<BF16, false, KC, TE>),
                                                         kBlock, GL.total) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        grid = static_cast<uint32_t>(g_num_cus * per_cu);
    }
    const uint32_t kdef = o ? o->k : 0u;

    MHR_HIP_TRY(rec(ev ? ev->begin : nullptr));
    hipLaunchKernelGGL(plan_kernel, dim3(nq), dim3(kBlock), 0, st, A, src, dst, k, kdef, kmax);
    MHR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(schedule_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kSchedLds)));
    hipLaunchKernelGGL(schedule_kernel, dim3(1), dim3(kBlock), nq <= kSchedCache ? kSchedLds : 0, st, A);
    hipLaunchKernelGGL(tile_starts_kernel, dim3(nq), dim3(kBlock), 0, st, A);
    auto gk = gather_kernel<BF16, false, KC, TE>;
    MHR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(gk),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(GL.total)));
    MHR_HIP_TRY(rec(ev ? ev->gather_begin : nullptr));
    hipLaunchKernelGGL(gk, dim3(grid), dim3(kBlock), GL.total, st, A);
    MHR_HIP_TRY(rec(ev ? ev->gather_end : nullptr));
    const size_t msmem = size_t(kMergeSlots) * sizeof(Cand);
    // fast merge: KC candidates, their sort keys, the key cache
    const size_t msmem_keys = size_t(KC) * (sizeof(Cand) + sizeof(uint64_t)) + size_t(kSelCache) * sizeof(uint32_t);
    auto mk = merge_kernel<BF16, KC, TE>;
    MHR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(mk),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(msmem_keys)));
    hipLaunchKernelGGL(mk, dim3(nq), dim3(kMergeBlock), msmem_keys, st, A, out, out_count, out_total, out_status, kmax);
    auto xk = gather_kernel<BF16, true, KC, TE>;
    MHR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(xk),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(GL.total)));
    hipLaunchKernelGGL(xk, dim3(grid), dim3(kBlock), GL.total, st, A);
    auto mx = merge_exact_kernel<KC>;
    MHR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(mx),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(msmem)));
    hipLaunchKernelGGL(mx, dim3(nq), dim3(kBlock), msmem, st, A, out, out_count, out_total, out_status, kmax);
    MHR_HIP_TRY(hipGetLastError());
    MHR_HIP_TRY(rec(ev ? ev->end : nullptr));
    return MHR_OK;
}

}  // namespace

size_t gather_lds_bytes(const mhr_graph *g, uint32_t hash_log2, uint32_t kmax) {
    return gather_layout(hash_log2, g->R, g->dim, kc_for(kmax)).total;
}

}  // namespace mhr

using namespace mhr;

extern "C" mhr_status mhr_workspace_size(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq, uint32_t kmax,
                                         size_t *bytes) {
    MHR_ARG_CHECK(g && bytes, "mhr_workspace_size: null argument");
    if (!g->X) {
        set_error("embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    MHR_ARG_CHECK(kmax >= 1 && kmax <= MHR_MAX_K, "k_max must be in [1, MHR_MAX_K]");
    (void)o;
    *bytes = ws_layout(nq, kc_for(kmax)).total;
    return MHR_OK;
}

extern "C" mhr_status mhr_topk_paths(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq, const uint32_t *src,
                                     const uint32_t *dst, const uint32_t *k, uint32_t kmax, mhr_path *out,
                                     uint32_t *out_count, uint64_t *out_total, uint32_t *out_status,
                                     void *workspace, size_t ws_bytes, void *stream) {
    return mhr_topk_paths_profiled(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace,
                                   ws_bytes, stream, nullptr);
}

namespace {

mhr_status topk_impl(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq, const uint32_t *src,
                     const uint32_t *dst, const uint32_t *k, uint32_t kmax, mhr_path *out, uint32_t *out_count,
                     uint64_t *out_total, uint32_t *out_status, void *workspace, size_t ws_bytes, void *stream,
                     const mhr_phase_events *ev, const uint8_t *keep, const uint64_t *keep_off) {
    MHR_ARG_CHECK(g != nullptr, "mhr_topk_paths: null graph");
    if (!g->X) {
        set_error("embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    MHR_ARG_CHECK(kmax >= 1 && kmax <= MHR_MAX_K, "k_max must be in [1, MHR_MAX_K]");
    if (nq == 0) return MHR_OK;
    MHR_ARG_CHECK(src && dst && out && out_count && workspace, "mhr_topk_paths: null pointer");
    MHR_ARG_CHECK(k != nullptr || (o && o->k >= 1 && o->k <= kmax), "opts->k must be in [1, k_max] when k is NULL");
    if (o) {
        MHR_ARG_CHECK(o->hash_log2 == 0 || (o->hash_log2 >= 10 && o->hash_log2 <= 12), "hash_log2 must be 10..12");
        for (uint32_t v : o->reserved) MHR_ARG_CHECK(v == 0, "reserved option fields must be zero");
        MHR_ARG_CHECK(o->band_abs >= 0.0f && o->band_abs <= 1e30f, "band_abs must be finite and >= 0");
    }
    const uint32_t kc = kc_for(kmax);
    const size_t need = ws_layout(nq, kc).total;
    if (ws_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    const size_t lds = gather_lds_bytes(g, hash_log2_for(g, o, kmax), kmax);
    if (lds > kDynLdsBytes) {
        set_error("LDS demand " + std::to_string(lds) + " exceeds 159 KiB (reduce hash_log2)");
        return MHR_ERR_UNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool bf = g->dtype == MHR_DTYPE_BF16;
    const bool te = g->scorer == MHR_SCORER_TRANSE_L1;
#define MHR_LAUNCH(BF, KCV, TEV)                                                                                   \
    launch_all<BF, KCV, TEV>(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, st, ev, \
                             keep, keep_off)
    switch (kc) {
        case 64:
            return bf ? (te ? MHR_LAUNCH(true, 64, true) : MHR_LAUNCH(true, 64, false))
                      : (te ? MHR_LAUNCH(false, 64, true) : MHR_LAUNCH(false, 64, false));
        case 128:
            return bf ? (te ? MHR_LAUNCH(true, 128, true) : MHR_LAUNCH(true, 128, false))
                      : (te ? MHR_LAUNCH(false, 128, true) : MHR_LAUNCH(false, 128, false));
        default:
            return bf ? (te ? MHR_LAUNCH(true, 256, true) : MHR_LAUNCH(true, 256, false))
                      : (te ? MHR_LAUNCH(false, 256, true) : MHR_LAUNCH(false, 256, false));
    }
#undef MHR_LAUNCH
}

}  // namespace

extern "C" mhr_status mhr_topk_paths_profiled(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq,
                                              const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                              uint32_t kmax, mhr_path *out, uint32_t *out_count,
                                              uint64_t *out_total, uint32_t *out_status, void *workspace,
                                              size_t ws_bytes, void *stream, const mhr_phase_events *ev) {
    return topk_impl(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, ws_bytes, stream,
                     ev, nullptr, nullptr);
}

extern "C" mhr_status mhr_topk_paths_pruned(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq,
                                            const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                            uint32_t kmax, const uint8_t *keep, const uint64_t *keep_off,
                                            mhr_path *out, uint32_t *out_count, uint64_t *out_total,
                                            uint32_t *out_status, void *workspace, size_t ws_bytes,
                                            void *stream) {
    MHR_ARG_CHECK(keep != nullptr && keep_off != nullptr, "mhr_topk_paths_pruned: null keep flags");
    return topk_impl(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, ws_bytes, stream,
                     nullptr, keep, keep_off);
}

extern "C" mhr_status mhr_edge_weights(const mhr_graph *g, uint64_t ne, const uint32_t *u, const uint32_t *r,
                                       const uint32_t *v, float *w32, float *e32, float *whi, float *wlo,
                                       void *stream) {
    MHR_ARG_CHECK(g != nullptr, "mhr_edge_weights: null graph");
    if (!g->X) {
        set_error("embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    if (ne == 0) return MHR_OK;
    MHR_ARG_CHECK(u && r && v, "mhr_edge_weights: null edge arrays");
    GArgs A = make_args(g);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t blocks = static_cast<uint32_t>((ne + 255) / 256);
    const bool te = g->scorer == MHR_SCORER_TRANSE_L1;
    if (g->dtype == MHR_DTYPE_BF16) {
        if (te) hipLaunchKernelGGL((edge_weight_kernel<true, true>), dim3(blocks), dim3(256), 0, st, A, ne, u, r, v, w32, e32, whi, wlo);
        else hipLaunchKernelGGL((edge_weight_kernel<true, false>), dim3(blocks), dim3(256), 0, st, A, ne, u, r, v, w32, e32, whi, wlo);
    } else {
        if (te) hipLaunchKernelGGL((edge_weight_kernel<false, true>), dim3(blocks), dim3(256), 0, st, A, ne, u, r, v, w32, e32, whi, wlo);
        else hipLaunchKernelGGL((edge_weight_kernel<false, false>), dim3(blocks), dim3(256), 0, st, A, ne, u, r, v, w32, e32, whi, wlo);
    }
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free query entry point.  The workspace is a fixed device array
// of this library (one copy per GPU, held until the process ends) instead of
// a caller buffer.  Host code never passes the array's name to a kernel: its
// device address is looked up once per device with hipGetSymbolAddress and
// that address is used as the workspace.
// ---------------------------------------------------------------------------
namespace mhr {
namespace {

__device__ __align__(256) unsigned char scratch[MHR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

// The device address of `scratch` on the current device (resolved on the
// first call on each device), or nullptr with the error set.
void *scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxScratchDevices) {
        set_error("mhr_topk_paths_noalloc: device index out of range");
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace mhr

extern "C" mhr_status mhr_topk_paths_noalloc(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq,
                                             const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                             uint32_t kmax, mhr_path *out, uint32_t *out_count,
                                             uint64_t *out_total, uint32_t *out_status, void *stream) {
    MHR_ARG_CHECK(g != nullptr, "mhr_topk_paths_noalloc: null graph");
    if (!g->X) {
        set_error("embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    MHR_ARG_CHECK(kmax >= 1 && kmax <= MHR_MAX_K, "k_max must be in [1, MHR_MAX_K]");
    if (nq == 0) return MHR_OK;
    const size_t need = ws_layout(nq, kc_for(kmax)).total;
    if (need > MHR_NOALLOC_SCRATCH_BYTES) {
        set_error("mhr_topk_paths_noalloc: the batch needs a larger workspace than the fixed scratch array holds "
                  "(use mhr_topk_paths with a caller workspace, or fewer queries / a smaller k_max)");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    int dev = -1;
    MHR_HIP_TRY(hipGetDevice(&dev));
    MHR_ARG_CHECK(dev == g->device, "mhr_topk_paths_noalloc: the graph lives on another device than the current one");
    void *ws = scratch_address(dev);
    if (!ws) return MHR_ERR_DEVICE;
    return topk_impl(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, ws,
                     MHR_NOALLOC_SCRATCH_BYTES, stream, nullptr, nullptr, nullptr);
}

// Phase clocks of the gather kernel (see GatherPhase, GatherCount): copies,
// per tile kind (0: probe side in the LDS table, 1: probing through the row
// directory), the summed per-workgroup wall-clock ticks of every phase since
// the last reset and then the work counts, to out (host, n >= 2 (kNumPhases
// + kNumCounts) entries), the clock's rate in Hz to *rate_hz, and resets
// them if reset != 0.  Synchronises the device.  Only a build with
// MHR_PHASE_CLOCKS records them; other builds return MHR_ERR_UNSUPPORTED.
extern "C" mhr_status mhr_debug_phase_ticks(uint64_t *out, uint32_t n, double *rate_hz, int reset) {
#ifdef MHR_PHASE_CLOCKS
    MHR_ARG_CHECK(out != nullptr && n >= static_cast<uint32_t>(2 * kPhSlots), "mhr_debug_phase_ticks: bad output");
    MHR_HIP_TRY(hipDeviceSynchronize());
    unsigned long long h[2 * kPhSlots];
    MHR_HIP_TRY(hipMemcpyFromSymbol(h, HIP_SYMBOL(g_phase_ticks), sizeof(h)));
    for (int i = 0; i < 2 * kPhSlots; ++i) out[i] = h[i];
    if (rate_hz) {
        int dev = 0, khz = 0;
        MHR_HIP_TRY(hipGetDevice(&dev));
        MHR_HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        *rate_hz = 1e3 * static_cast<double>(khz);
    }
    if (reset) {
        const unsigned long long z[2 * kPhSlots] = {};
        MHR_HIP_TRY(hipMemcpyToSymbol(HIP_SYMBOL(g_phase_ticks), z, sizeof(z)));
        MHR_HIP_TRY(hipDeviceSynchronize());
    }
    return MHR_OK;
#else
    (void)out;
    (void)n;
    (void)rate_hz;
    (void)reset;
    set_error("this build records no phase clocks (build with MHR_PHASE_CLOCKS)");
    return MHR_ERR_UNSUPPORTED;
#endif
}

extern "C" mhr_status mhr_pruner_candidate_weights(const mhr_graph *g, uint64_t ncand, const uint32_t *src,
                                                   const uint32_t *dst, const uint32_t *cand_q, const uint32_t *cand_v,
                                                   const uint32_t *cand_r, float *w, void *stream) {
    MHR_ARG_CHECK(g != nullptr, "mhr_pruner_candidate_weights: null graph");
    if (!g->X) {
        set_error("embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    if (ncand == 0) return MHR_OK;
    MHR_ARG_CHECK(src && dst && cand_q && cand_v && cand_r && w, "mhr_pruner_candidate_weights: null pointer");
    GArgs A = make_args(g);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const dim3 grid(static_cast<uint32_t>((ncand + 255) / 256));
    const bool te = g->scorer == MHR_SCORER_TRANSE_L1;
    if (g->dtype == MHR_DTYPE_BF16) {
        if (te) hipLaunchKernelGGL((candidate_weight_kernel<true, true>), grid, dim3(256), 0, st, A, ncand, src, dst, cand_q, cand_v, cand_r, w);
        else hipLaunchKernelGGL((candidate_weight_kernel<true, false>), grid, dim3(256), 0, st, A, ncand, src, dst, cand_q, cand_v, cand_r, w);
    } else {
        if (te) hipLaunchKernelGGL((candidate_weight_kernel<false, true>), grid, dim3(256), 0, st, A, ncand, src, dst, cand_q, cand_v, cand_r, w);
        else hipLaunchKernelGGL((candidate_weight_kernel<false, false>), grid, dim3(256), 0, st, A, ncand, src, dst, cand_q, cand_v, cand_r, w);
    }
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}
