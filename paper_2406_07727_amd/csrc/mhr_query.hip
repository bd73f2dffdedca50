// Exact three-hop top-K path search, plain FP32 form with compensated
// rescoring of the boundary band.
//
// Pipeline for a batch of queries (all on the caller's stream):
//   plan      one workgroup per query: validates ids, measures the two
//             meet-in-the-middle costs (backward: sum of in-degrees of
//             N-(t); forward: sum of out-degrees of N+(s)), picks the
//             cheaper direction and cuts the scan into tiles.
//   schedule  one workgroup: prefix of tile counts, tile -> query map.
//   gather    persistent workgroups pulling tiles from an atomic counter.
//             A tile builds a membership table of the probe side (LDS hash
//             or, for long rows, the graph's bucket directory), streams the
//             CSR rows of its list slice, tests each scanned vertex, scores
//             every matched middle edge and the two outer edges in FP32 with
//             a rigorous error bound, enumerates the paths through it and
//             keeps the best KC by the total order.
//   merge     one workgroup per query: merges the tile lists, takes every
//             candidate whose score lies within twice the error bound of the
//             K-th, rescores them in float-float and writes the ranked
//             result.  If a truncated tile could still hold a band member
//             the query is marked for the exhaustive pass.
//   exact     gather again for marked queries, scoring every path above the
//             band threshold in float-float, then a merge of those lists.
//
// The paper's CPU design (thread-private K-heaps merged by a tree
// reduction, section 3.3; level-synchronous frontier expansion, section 5)
// is the prior art this replaces: here the per-thread heap becomes a
// per-workgroup LDS candidate list fed by block-wide threshold filtering,
// and the reduction tree becomes the per-query merge of tile lists.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mhr_device.h"
#include "mhr_internal.h"

namespace mhr {

namespace {

constexpr int kBlock = 256;
constexpr int kEPT = 8;                   // scan entries per thread per chunk
constexpr int kChunk = kBlock * kEPT;     // scan entries per chunk
constexpr int kRowBatch = 32;             // list rows staged at a time
constexpr int kSlab = 1024;               // scored edge values per sub-batch
constexpr int kStage = 512;               // staged candidates before a merge
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
    uint2 *tile_start;
    TileHeader *hdr;
    Cand *cands;
    uint32_t *exact_list;
    uint32_t maxt, hash_log2, nq, kc;
};

__host__ __device__ inline uint32_t max_tiles_for(uint32_t kc) { return 2048u / kc; }

__device__ inline uint32_t nth_bit(uint32_t m, uint32_t k) {
    for (uint32_t i = 0; i < k; ++i) m &= m - 1;
    return static_cast<uint32_t>(__ffs(m) - 1);
}

// Block reductions / scans (blockDim.x == kBlock).
template <class T>
__device__ inline T block_sum(T v, T *lds) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < kBlock / kWave; ++w) s += lds[w];
    __syncthreads();
    return s;
}

__device__ inline float block_max(float v, float *lds) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    float s = lds[0];
    for (int w = 1; w < kBlock / kWave; ++w) s = fmaxf(s, lds[w]);
    __syncthreads();
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
    __syncthreads();
    *total = tot;
    return v + base;
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void plan_kernel(GArgs A, const uint32_t *src, const uint32_t *dst,
                                                      const uint32_t *kq, uint32_t kdef, uint32_t kmax,
                                                      uint32_t tile_edges) {
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
    // backward: list N-(t) (reverse CSR row of t), scanned rows in the reverse CSR
    const uint32_t lb_beg = A.in_rp[P.t], lb_len = A.in_rp[P.t + 1] - lb_beg;
    uint64_t part = 0;
    for (uint32_t i = threadIdx.x; i < lb_len; i += kBlock) {
        uint32_t b = A.in_col[lb_beg + i];
        part += A.in_rp[b + 1] - A.in_rp[b];
    }
    const uint64_t cost_b = block_sum<uint64_t>(part, red64);
    // forward: list N+(s), scanned rows in the forward CSR; stop once it
    // cannot beat the backward cost
    const uint32_t lf_beg = A.out_rp[P.s], lf_len = A.out_rp[P.s + 1] - lf_beg;
    uint64_t cost_f = 0;
    for (uint32_t base = 0; base < lf_len && cost_f < cost_b; base += kBlock) {
        uint64_t p = 0;
        uint32_t i = base + threadIdx.x;
        if (i < lf_len) {
            uint32_t a = A.out_col[lf_beg + i];
            p = A.out_rp[a + 1] - A.out_rp[a];
        }
        cost_f += block_sum<uint64_t>(p, red64);
    }
    const bool fwd = cost_f < cost_b;
    P.dir = fwd ? 1u : 0u;
    P.cost = fwd ? cost_f : cost_b;
    P.list_beg = fwd ? lf_beg : lb_beg;
    P.list_len = fwd ? lf_len : lb_len;
    P.probe_beg = fwd ? A.in_rp[P.t] : A.out_rp[P.s];
    P.probe_len = fwd ? (A.in_rp[P.t + 1] - P.probe_beg) : (A.out_rp[P.s + 1] - P.probe_beg);
    uint32_t ntiles = 0;
    if (P.cost > 0 && P.probe_len > 0) {
        uint64_t nt = (P.cost + tile_edges - 1) / tile_edges;
        ntiles = static_cast<uint32_t>(nt < A.maxt ? nt : A.maxt);
    }
    P.ntiles = ntiles;
    if (ntiles > 0) {
        // tile j starts at concatenated position j * L: record (row, offset)
        const uint64_t L = (P.cost + ntiles - 1) / ntiles;
        ntiles = static_cast<uint32_t>((P.cost + L - 1) / L);  // every start j*L < cost
        P.ntiles = ntiles;
        const uint32_t *rp = fwd ? A.out_rp : A.in_rp;
        const uint32_t *col = fwd ? A.out_col : A.in_col;
        uint64_t run = 0;
        for (uint32_t base = 0; base < P.list_len; base += kBlock) {
            uint32_t i = base + threadIdx.x;
            uint64_t deg = 0;
            if (i < P.list_len) {
                uint32_t x = col[P.list_beg + i];
                deg = rp[x + 1] - rp[x];
            }
            uint64_t tot;
            uint64_t incl = block_incl_scan<uint64_t>(deg, red64, &tot);
            uint64_t p0 = run + incl - deg;
            if (deg > 0) {
                uint64_t jlo = (p0 + L - 1) / L;
                uint64_t jhi = (p0 + deg - 1) / L;
                for (uint64_t j = jlo; j <= jhi && j < ntiles; ++j)
                    A.tile_start[static_cast<uint64_t>(q) * A.maxt + j] =
                        make_uint2(i, static_cast<uint32_t>(j * L - p0));
            }
            run += tot;
        }
    }
    if (threadIdx.x == 0) A.plans[q] = P;
}

// ---------------------------------------------------------------------------
// schedule (one workgroup)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void schedule_kernel(GArgs A) {
    __shared__ uint32_t red[kBlock / kWave];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < A.nq; base += kBlock) {
        uint32_t q = base + threadIdx.x;
        uint32_t nt = q < A.nq ? A.plans[q].ntiles : 0u;
        uint32_t tot;
        uint32_t incl = block_incl_scan<uint32_t>(nt, red, &tot);
        uint32_t c = carry;
        if (q < A.nq) {
            uint32_t tb = c + incl - nt;
            A.plans[q].tile_base = tb;
            A.plans[q].flags = 0;
            for (uint32_t j = 0; j < nt; ++j) A.tile_q[tb + j] = q;
        }
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        A.ctrl->total_tiles = carry;
        A.ctrl->gather_ctr = 0;
        A.ctrl->exact_ctr = 0;
        A.ctrl->exact_n = 0;
    }
}

// ---------------------------------------------------------------------------
// float-float scoring of one path (rescoring and the exhaustive pass)
// ---------------------------------------------------------------------------
template <bool BF16>
__device__ inline ff edge_x_ff(const GArgs &A, uint32_t u, uint32_t r, uint32_t v, float *abs_sum) {
    ff acc = {0.0f, 0.0f};
    float as = 0.0f;
    const size_t d = A.d;
    for (uint32_t i = 0; i < A.d; ++i) {
        float xu = load1<BF16>(A.X, u * d + i);
        float yr = load1<BF16>(A.Y, r * d + i);
        float xv = load1<BF16>(A.X, v * d + i);
        ff p = two_prod(xu, yr);
        ff t = ff_mul_f(p, xv);
        acc = ff_add(acc, t);
        as += fabsf(p.hi * xv);
    }
    *abs_sum = as;
    return acc;
}

// S = w(s,r1,a) + w(a,r2,b) + w(b,r3,t) in float-float, with a bound on
// its error: per edge, the dot product (about 4 d u^2 sum|t|) plus the
// log-sigmoid; then the two additions.
template <bool BF16>
__device__ inline ff path_score_ff(const GArgs &A, uint32_t s, uint32_t a, uint32_t b, uint32_t t, uint32_t r1,
                                   uint32_t r2, uint32_t r3, float *eps) {
    const float u2 = kUnit * kUnit;
    float as1, as2, as3;
    ff w1 = ff_logsigmoid(edge_x_ff<BF16>(A, s, r1, a, &as1));
    ff w2 = ff_logsigmoid(edge_x_ff<BF16>(A, a, r2, b, &as2));
    ff w3 = ff_logsigmoid(edge_x_ff<BF16>(A, b, r3, t, &as3));
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
    float e = 4.04f * dd * u2 * (as1 + as2 + as3) * 1.01f + ff_logsigmoid_err(w1.hi) + ff_logsigmoid_err(w2.hi) +
              ff_logsigmoid_err(w3.hi) + 8.0f * u2 * (fabsf(w1.hi) + fabsf(w2.hi) + fabsf(w3.hi));
    *eps = e;
    return S;
}

// ---------------------------------------------------------------------------
// gather
// ---------------------------------------------------------------------------
struct RowInfo {
    uint32_t x, mask, beg, len, pref, vbase;
};

struct GatherShared {
    uint32_t tile, q, j;
    uint32_t qcount;      // match queue fill
    uint32_t stage_n;
    uint32_t list_n;
    uint32_t truncated;
    uint32_t nrows;
    uint32_t E;           // entries in the current row batch
    uint32_t nsub, nc;
    uint32_t rowvals;
    float eps_max;
    uint32_t pad;
    Cand thr;             // current worst kept candidate (sentinel until the list fills)
    uint64_t red64[kBlock / kWave];
    uint32_t red32[kBlock / kWave];
    float redf[kBlock / kWave];
};

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~static_cast<size_t>(15); }

struct GatherLayout {
    size_t hkeys, hvals, Y, anc_p, anc_l, rows, rowval, roweps, queue_pos, queue_mp, sub_info, slab, slab_eps,
        list, stage, shared, total;
};

__host__ __device__ inline GatherLayout gather_layout(uint32_t hash_log2, uint32_t R, uint32_t d, uint32_t kc) {
    GatherLayout L{};
    size_t o = 0;
    const size_t slots = size_t(1) << hash_log2;
    L.hkeys = o; o = align16(o + slots * 4);
    L.hvals = o; o = align16(o + slots * 4);
    L.Y = o; o = align16(o + size_t(R) * d * 4);
    L.anc_p = o; o = align16(o + size_t(d) * 4);
    L.anc_l = o; o = align16(o + size_t(d) * 4);
    L.rows = o; o = align16(o + kRowBatch * sizeof(RowInfo));
    L.rowval = o; o = align16(o + size_t(kRowBatch) * R * 4);
    L.roweps = o; o = align16(o + size_t(kRowBatch) * R * 4);
    L.queue_pos = o; o = align16(o + kChunk * 4);
    L.queue_mp = o; o = align16(o + kChunk * 4);
    L.sub_info = o; o = align16(o + kBlock * 6 * 4);
    L.slab = o; o = align16(o + kSlab * 4);
    L.slab_eps = o; o = align16(o + kSlab * 4);
    L.list = o; o = align16(o + size_t(kc) * sizeof(Cand));
    L.stage = o; o = align16(o + size_t(next_pow2(kStage + kc)) * sizeof(Cand));
    L.shared = o; o = align16(o + sizeof(GatherShared));
    L.total = o;
    return L;
}

// Elements per lane and lanes per edge for dimension d.
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
        for (int l = 0; l < epl; ++l) v[l] = load1<BF16>(base, row * d + off + l);
        for (int l = epl; l < 8; ++l) v[l] = 0.0f;
    }
}

// Centred weight of a scored edge and its error bound, from the lane
// partial sums of one group.
__device__ __forceinline__ void finish_edge(float part, float apart, int G, int epl, float *f, float *eps) {
    float x = group_sum(part, G);
    float as = group_sum(apart, G);
    int lg = 31 - __clz(G);
    float fx = centred_logsigmoid(x);
    *f = fx;
    *eps = gamma_n(epl + lg + 2) * as + centred_logsigmoid_err(fx);
}

// Merge the staged candidates into the kept list (whole block).
template <int KC>
__device__ inline void merge_stage(Cand *list, Cand *stage, GatherShared *sh) {
    const uint32_t ns = sh->stage_n;
    const uint32_t tot = ns + KC;
    const uint32_t n2 = next_pow2(tot);
    for (uint32_t i = threadIdx.x; i < n2; i += blockDim.x) {
        if (i >= ns && i < tot) stage[i] = list[i - ns];
        else if (i >= tot) stage[i] = cand_sentinel();
    }
    __syncthreads();
    block_sort_cands(stage, static_cast<int>(n2));
    // entries past KC that are real candidates are dropped
    if (threadIdx.x == 0) {
        Cand c = stage[KC];
        if (c.a != 0xFFFFFFFFu) sh->truncated = 1;
        uint32_t cnt = sh->list_n + ns;
        sh->list_n = cnt < static_cast<uint32_t>(KC) ? cnt : KC;
        sh->stage_n = 0;
        sh->thr = (sh->list_n == static_cast<uint32_t>(KC)) ? stage[KC - 1] : cand_sentinel();
    }
    for (uint32_t i = threadIdx.x; i < static_cast<uint32_t>(KC); i += blockDim.x) list[i] = stage[i];
    __syncthreads();
}

template <bool BF16, bool EXACT, int KC>
__global__ __launch_bounds__(kBlock) void gather_kernel(GArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const GatherLayout Lo = gather_layout(A.hash_log2, A.R, A.d, KC);
    uint32_t *hkeys = reinterpret_cast<uint32_t *>(smem + Lo.hkeys);
    uint32_t *hvals = reinterpret_cast<uint32_t *>(smem + Lo.hvals);
    float *Ys = reinterpret_cast<float *>(smem + Lo.Y);
    float *anc_p = reinterpret_cast<float *>(smem + Lo.anc_p);
    float *anc_l = reinterpret_cast<float *>(smem + Lo.anc_l);
    RowInfo *rows = reinterpret_cast<RowInfo *>(smem + Lo.rows);
    float *rowval = reinterpret_cast<float *>(smem + Lo.rowval);
    float *roweps = reinterpret_cast<float *>(smem + Lo.roweps);
    uint32_t *qpos = reinterpret_cast<uint32_t *>(smem + Lo.queue_pos);
    uint32_t *qmp = reinterpret_cast<uint32_t *>(smem + Lo.queue_mp);
    uint32_t *sub = reinterpret_cast<uint32_t *>(smem + Lo.sub_info);
    float *slab = reinterpret_cast<float *>(smem + Lo.slab);
    float *slab_eps = reinterpret_cast<float *>(smem + Lo.slab_eps);
    Cand *list = reinterpret_cast<Cand *>(smem + Lo.list);
    Cand *stage = reinterpret_cast<Cand *>(smem + Lo.stage);
    GatherShared *sh = reinterpret_cast<GatherShared *>(smem + Lo.shared);
    // per sub-batch match info (one match per thread)
    uint32_t *sub_pos = sub, *sub_mp = sub + kBlock, *sub_mm = sub + 2 * kBlock, *sub_row = sub + 3 * kBlock,
             *sub_voff = sub + 4 * kBlock, *sub_coff = sub + 5 * kBlock;

    const uint32_t tid = threadIdx.x;
    const uint32_t d = A.d, R = A.R;
    const uint32_t slots = 1u << A.hash_log2, smask = slots - 1;
    const uint32_t hcap = slots / 2;
    const int G = lanes_per_edge(d);
    const int epl = static_cast<int>(d) / G;
    const int gid = static_cast<int>(tid) / G, glane = static_cast<int>(tid) % G;
    const int ngroups = kBlock / G;

    for (uint32_t i = tid; i < R * d; i += kBlock) Ys[i] = load1<BF16>(A.Y, i);

    for (;;) {
        __syncthreads();
        if (tid == 0) {
            uint32_t t;
            if (EXACT) {
                // items enumerate (marked query, tile) pairs
                for (;;) {
                    uint32_t item = atomicAdd(&A.ctrl->exact_ctr, 1u);
                    uint32_t qi = item / A.maxt, j = item % A.maxt;
                    if (qi >= A.ctrl->exact_n) { t = kEmpty; break; }
                    uint32_t q = A.exact_list[qi];
                    if (j < A.plans[q].ntiles) { t = A.plans[q].tile_base + j; sh->q = q; sh->j = j; break; }
                }
            } else {
                t = atomicAdd(&A.ctrl->gather_ctr, 1u);
                if (t < A.ctrl->total_tiles) {
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
            sh->eps_max = 0.0f;
            sh->thr = cand_sentinel();
        }
        __syncthreads();
        if (!heavy) {
            for (uint32_t i = tid; i < P.probe_len; i += kBlock) {
                uint32_t y = Pcol[P.probe_beg + i];
                uint32_t m = Pmask[P.probe_beg + i];
                uint32_t slot = (y * 0x9E3779B1u) >> (32 - A.hash_log2);
                for (;;) {
                    uint32_t old = atomicCAS(&hkeys[slot], kEmpty, y);
                    if (old == kEmpty) { hvals[slot] = m; break; }
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
        const uint2 ts = A.tile_start[static_cast<uint64_t>(q) * A.maxt + j];
        const uint2 te = (j + 1 < P.ntiles) ? A.tile_start[static_cast<uint64_t>(q) * A.maxt + j + 1]
                                           : make_uint2(P.list_len, 0u);
        uint64_t npaths = 0;
        float eps_local = 0.0f;
        __syncthreads();

        // ---- row batches
        const uint32_t row_end = (te.y > 0) ? te.x + 1 : te.x;  // exclusive
        for (uint32_t rb = ts.x; rb < row_end; rb += kRowBatch) {
            const uint32_t nrows = min(static_cast<uint32_t>(kRowBatch), row_end - rb);
            // row info: scan range clipped to the tile
            uint32_t len = 0;
            if (tid < nrows) {
                uint32_t i = rb + tid;
                uint32_t x = Lcol[P.list_beg + i];
                uint32_t beg = Lrp[x], end = Lrp[x + 1];
                if (i == ts.x) beg += ts.y;
                if (i == te.x) end = Lrp[x] + te.y;
                len = end > beg ? end - beg : 0u;
                rows[tid].x = x;
                rows[tid].mask = Lmask[P.list_beg + i];
                rows[tid].beg = beg;
                rows[tid].len = len;
            }
            // prefix over the batch (wave 0 holds all kRowBatch rows)
            if (tid < kWave) {
                uint32_t v = len;
                uint32_t nv = (tid < nrows) ? __popc(Lmask[P.list_beg + rb + tid]) : 0u;
                for (int off = 1; off < kWave; off <<= 1) {
                    uint32_t t1 = __shfl_up(v, off, kWave);
                    uint32_t t2 = __shfl_up(nv, off, kWave);
                    if (static_cast<int>(tid) >= off) { v += t1; nv += t2; }
                }
                if (tid < nrows) {
                    rows[tid].pref = v - len;
                    rows[tid].vbase = nv - ((tid < nrows) ? __popc(Lmask[P.list_beg + rb + tid]) : 0u);
                }
                if (tid == nrows - 1) { sh->E = v; sh->rowvals = nv; }
            }
            __syncthreads();
            // list-edge weights: one group per (row, relation) pair
            const uint32_t nrv = sh->rowvals;
            for (uint32_t base = 0; base < nrv; base += ngroups) {
                uint32_t vi = base + gid;
                bool act = vi < nrv;
                uint32_t r = 0, k = 0;
                if (act) {
                    while (r + 1 < nrows && rows[r + 1].vbase <= vi) ++r;
                    k = vi - rows[r].vbase;
                }
                float part = 0.0f, apart = 0.0f;
                if (act) {
                    uint32_t rel = nth_bit(rows[r].mask, k);
                    float ex[8];
                    load_lane<BF16>(A.X, rows[r].x, d, glane * epl, epl, ex);
                    for (int l = 0; l < epl; ++l) {
                        uint32_t e = glane * epl + l;
                        float z = anc_l[e] * Ys[rel * d + e];
                        part = __builtin_fmaf(z, ex[l], part);
                        apart += fabsf(z * ex[l]);
                    }
                }
                float f, eps;
                finish_edge(part, apart, G, epl, &f, &eps);
                if (act && glane == 0) { rowval[vi] = f; roweps[vi] = eps; }
            }
            __syncthreads();
            const uint32_t E = sh->E;

            // ---- chunks of scanned entries
            for (uint32_t cb = 0; cb < E; cb += kChunk) {
                if (tid == 0) sh->qcount = 0;
                __syncthreads();
                uint32_t ys[kEPT], ps[kEPT];
#pragma unroll
                for (int k = 0; k < kEPT; ++k) {
                    uint32_t e = cb + k * kBlock + tid;
                    ps[k] = kEmpty;
                    ys[k] = kEmpty;
                    if (e < E) {
                        uint32_t lo = 0, hi = nrows;  // last row with pref <= e
                        while (hi - lo > 1) {
                            uint32_t mid = (lo + hi) >> 1;
                            if (rows[mid].pref <= e) lo = mid; else hi = mid;
                        }
                        ps[k] = rows[lo].beg + (e - rows[lo].pref);
                    }
                }
#pragma unroll
                for (int k = 0; k < kEPT; ++k)
                    if (ps[k] != kEmpty) ys[k] = Lcol[ps[k]];
#pragma unroll
                for (int k = 0; k < kEPT; ++k) {
                    bool hit = false;
                    uint32_t mp = 0;
                    if (ps[k] != kEmpty) {
                        const uint32_t y = ys[k];
                        if (!heavy) {
                            uint32_t slot = (y * 0x9E3779B1u) >> (32 - A.hash_log2);
                            for (;;) {
                                uint32_t key = hkeys[slot];
                                if (key == y) { hit = true; mp = hvals[slot]; break; }
                                if (key == kEmpty) break;
                                slot = (slot + 1) & smask;
                            }
                        } else {
                            uint32_t bk = y >> dsh;
                            uint32_t lo = dir[bk], hi = dir[bk + 1];
                            for (uint32_t i = lo; i < hi; ++i) {
                                uint32_t c = Pcol[P.probe_beg + i];
                                if (c == y) { hit = true; mp = Pmask[P.probe_beg + i]; break; }
                                if (c > y) break;
                            }
                        }
                    }
                    uint64_t bal = __ballot(hit);
                    if (bal) {
                        const int lane = tid & (kWave - 1);
                        uint32_t base = 0;
                        if (lane == 0) base = atomicAdd(&sh->qcount, static_cast<uint32_t>(__popcll(bal)));
                        base = __shfl(base, 0, kWave);
                        if (hit) {
                            uint64_t lt = lane ? (bal & (~0ull >> (kWave - lane))) : 0ull;
                            uint32_t slotq = base + __popcll(lt);
                            qpos[slotq] = ps[k];
                            qmp[slotq] = mp;
                        }
                    }
                }
                __syncthreads();
                const uint32_t nmatch = sh->qcount;

                // ---- sub-batches of at most kBlock matches
                for (uint32_t m0 = 0; m0 < nmatch;) {
                    uint32_t mi = m0 + tid;
                    uint32_t pos = 0, mp = 0, mm = 0, row = 0, nv = 0, nc = 0;
                    if (mi < nmatch) {
                        pos = qpos[mi];
                        mp = qmp[mi];
                        mm = Lmask[pos];
                        uint32_t lo = 0, hi = nrows;  // row holding pos
                        while (hi - lo > 1) {
                            uint32_t mid = (lo + hi) >> 1;
                            if (rows[mid].beg <= pos) lo = mid; else hi = mid;
                        }
                        row = lo;
                        uint32_t np = __popc(mp), nm = __popc(mm), nl = __popc(rows[row].mask);
                        nv = np + nm;
                        nc = np * nm * nl;
                    }
                    uint32_t vtot;
                    uint32_t vincl = block_incl_scan<uint32_t>(nv, sh->red32, &vtot);
                    bool take = (mi < nmatch) && vincl <= static_cast<uint32_t>(kSlab);
                    uint32_t ncnt = block_sum<uint32_t>(take ? 1u : 0u, sh->red32);
                    uint32_t ctot;
                    uint32_t cincl = block_incl_scan<uint32_t>(take ? nc : 0u, sh->red32, &ctot);
                    if (take) {
                        sub_pos[tid] = pos;
                        sub_mp[tid] = mp;
                        sub_mm[tid] = mm;
                        sub_row[tid] = row;
                        sub_voff[tid] = vincl - nv;
                        sub_coff[tid] = cincl - nc;
                    }
                    __syncthreads();
                    // scoring: one group of G lanes per match
                    for (uint32_t s = gid; s < ncnt; s += ngroups) {
                        const uint32_t spos = sub_pos[s], smp = sub_mp[s], smm = sub_mm[s];
                        const RowInfo &ri = rows[sub_row[s]];
                        const uint32_t y = Lcol[spos];
                        float ey[8], ex[8];
                        load_lane<BF16>(A.X, y, d, glane * epl, epl, ey);
                        load_lane<BF16>(A.X, ri.x, d, glane * epl, epl, ex);
                        uint32_t vo = sub_voff[s];
                        uint32_t np = __popc(smp);
                        for (uint32_t k = 0; k < np; ++k) {
                            uint32_t rel = nth_bit(smp, k);
                            float part = 0.0f, apart = 0.0f;
                            for (int l = 0; l < epl; ++l) {
                                uint32_t e = glane * epl + l;
                                float z = anc_p[e] * Ys[rel * d + e];
                                part = __builtin_fmaf(z, ey[l], part);
                                apart += fabsf(z * ey[l]);
                            }
                            float f, eps;
                            finish_edge(part, apart, G, epl, &f, &eps);
                            if (glane == 0) { slab[vo + k] = f; slab_eps[vo + k] = eps; }
                        }
                        uint32_t nm = __popc(smm);
                        for (uint32_t k = 0; k < nm; ++k) {
                            uint32_t rel = nth_bit(smm, k);
                            float part = 0.0f, apart = 0.0f;
                            for (int l = 0; l < epl; ++l) {
                                uint32_t e = glane * epl + l;
                                float z = ey[l] * Ys[rel * d + e];
                                part = __builtin_fmaf(z, ex[l], part);
                                apart += fabsf(z * ex[l]);
                            }
                            float f, eps;
                            finish_edge(part, apart, G, epl, &f, &eps);
                            if (glane == 0) { slab[vo + np + k] = f; slab_eps[vo + np + k] = eps; }
                        }
                    }
                    __syncthreads();
                    // candidates: one per thread per round
                    for (uint32_t c0 = 0; c0 < ctot; c0 += kBlock) {
                        const uint32_t c = c0 + tid;
                        bool pass = false;
                        Cand cd;
                        if (c < ctot) {
                            uint32_t lo = 0, hi = ncnt;  // match holding candidate c
                            while (hi - lo > 1) {
                                uint32_t mid = (lo + hi) >> 1;
                                if (sub_coff[mid] <= c) lo = mid; else hi = mid;
                            }
                            const uint32_t s = lo;
                            const uint32_t local = c - sub_coff[s];
                            const uint32_t smp = sub_mp[s], smm = sub_mm[s];
                            const RowInfo &ri = rows[sub_row[s]];
                            const uint32_t np = __popc(smp), nm = __popc(smm), nl = __popc(ri.mask);
                            const uint32_t il = local % nl, im = (local / nl) % nm, ip = local / (nl * nm);
                            const uint32_t vo = sub_voff[s];
                            const float fp = slab[vo + ip], fm = slab[vo + np + im];
                            const float fl = rowval[ri.vbase + il];
                            const float ep = slab_eps[vo + ip], em = slab_eps[vo + np + im];
                            const float el = roweps[ri.vbase + il];
                            const float S = fwd ? (fl + fm) + fp : (fp + fm) + fl;
                            const float eS = ep + em + el + 2.01f * kUnit * (fabsf(fp) + fabsf(fm) + fabsf(fl));
                            const uint32_t rp_ = nth_bit(smp, ip), rm_ = nth_bit(smm, im), rl_ = nth_bit(ri.mask, il);
                            const uint32_t y = Lcol[sub_pos[s]];
                            cd.a = fwd ? ri.x : y;
                            cd.b = fwd ? y : ri.x;
                            const uint32_t r1 = fwd ? rl_ : rp_, r3 = fwd ? rp_ : rl_;
                            cd.rel = (r1 << 16) | (rm_ << 8) | r3;
                            cd.s = S;
                            cd.s_lo = 0.0f;
                            cd.eps = eS;
                            eps_local = fmaxf(eps_local, eS);
                            npaths += 1;
                            bool consider = true;
                            if (EXACT) {
                                consider = S >= thr_exact;
                                if (consider) {
                                    float e2;
                                    ff sc = path_score_ff<BF16>(A, P.s, cd.a, cd.b, P.t, r1, rm_, r3, &e2);
                                    cd.s = sc.hi;
                                    cd.s_lo = sc.lo;
                                    cd.eps = e2;
                                }
                            }
                            if (consider) {
                                if (cand_better(cd, sh->thr)) pass = true;
                                else sh->truncated = 1;
                            }
                        }
                        if (pass) {
                            uint32_t slot = atomicAdd(&sh->stage_n, 1u);
                            stage[slot] = cd;
                        }
                        __syncthreads();
                        if (sh->stage_n > static_cast<uint32_t>(kStage - kBlock)) merge_stage<KC>(list, stage, sh);
                    }
                    m0 += ncnt;
                    __syncthreads();
                }
            }
            __syncthreads();  // rows[] and sh->E are rewritten by the next batch
        }
        // ---- tile end: final merge and output
        __syncthreads();
        if (sh->stage_n > 0) merge_stage<KC>(list, stage, sh);
        float em = block_max(eps_local, sh->redf);
        uint64_t npt = block_sum<uint64_t>(npaths, sh->red64);
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

template <bool BF16, int KC>
__global__ __launch_bounds__(kBlock) void merge_kernel(GArgs A, mhr_path *out, uint32_t *out_count,
                                                       uint64_t *out_total, uint32_t *out_status, uint32_t kmax) {
    extern __shared__ __align__(16) unsigned char smem[];
    Cand *c = reinterpret_cast<Cand *>(smem);
    __shared__ uint32_t s_n, s_over, s_nb;
    __shared__ float s_eps;
    __shared__ uint64_t s_tot;
    const uint32_t q = blockIdx.x;
    QueryPlan P = A.plans[q];
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
    if (threadIdx.x == 0) {
        uint32_t n = 0;
        float eps = 0.0f;
        uint64_t tot = 0;
        for (uint32_t j = 0; j < P.ntiles; ++j) {
            const TileHeader &h = A.hdr[P.tile_base + j];
            n += h.count;
            eps = fmaxf(eps, h.eps);
            tot += h.npaths;
        }
        s_n = n;
        s_eps = eps;
        s_tot = tot;
    }
    __syncthreads();
    // compact the tile lists into LDS
    const uint32_t ntot = P.ntiles * KC;
    for (uint32_t i = threadIdx.x; i < ntot; i += blockDim.x) {
        uint32_t jt = i / KC, k = i % KC;
        const TileHeader &h = A.hdr[P.tile_base + jt];
        c[i] = (k < h.count) ? A.cands[static_cast<uint64_t>(P.tile_base + jt) * KC + k] : cand_sentinel();
    }
    const uint32_t n2 = next_pow2(ntot);
    for (uint32_t i = ntot + threadIdx.x; i < n2; i += blockDim.x) c[i] = cand_sentinel();
    __syncthreads();
    block_sort_cands(c, static_cast<int>(n2));
    const uint32_t cnt = s_n;
    const uint32_t kk = min(P.k, cnt);
    if (kk == 0) {
        if (threadIdx.x == 0) {
            out_count[q] = 0;
            if (out_total) out_total[q] = s_tot;
            if (out_status) out_status[q] = 0;
        }
        write_sentinels(row, 0, kmax);
        return;
    }
    const float theta = c[kk - 1].s;
    const float eps = s_eps;
    // band threshold, rounded down generously
    const float thr = (theta - 2.0f * eps) - 4.0f * kUnit * fabsf(theta) - 1e-30f;
    if (threadIdx.x == 0) {
        uint32_t over = 0;
        for (uint32_t j = 0; j < P.ntiles; ++j) {
            const TileHeader &h = A.hdr[P.tile_base + j];
            if (h.truncated && h.cutoff >= thr) over = 1;
        }
        uint32_t nb = 0;
        while (nb < cnt && c[nb].s >= thr) ++nb;
        s_over = over;
        s_nb = nb;
    }
    __syncthreads();
    if (s_over) {
        if (threadIdx.x == 0) {
            A.plans[q].flags = kNeedExact;
            A.plans[q].thr = thr;
            A.plans[q].total = s_tot;
            uint32_t slot = atomicAdd(&A.ctrl->exact_n, 1u);
            A.exact_list[slot] = q;
        }
        return;
    }
    const uint32_t nb = s_nb;
    for (uint32_t i = threadIdx.x; i < nb; i += blockDim.x) {
        Cand x = c[i];
        const uint32_t r1 = (x.rel >> 16) & 0xFF, r2 = (x.rel >> 8) & 0xFF, r3 = x.rel & 0xFF;
        float e;
        ff sc = path_score_ff<BF16>(A, P.s, x.a, x.b, P.t, r1, r2, r3, &e);
        x.s = sc.hi;
        x.s_lo = sc.lo;
        x.eps = e;
        c[i] = x;
    }
    const uint32_t nb2 = next_pow2(nb);
    for (uint32_t i = nb + threadIdx.x; i < nb2; i += blockDim.x) c[i] = cand_sentinel();
    __syncthreads();
    block_sort_cands(c, static_cast<int>(nb2));
    write_result(row, c, nb, kk, kmax);
    if (threadIdx.x == 0) {
        out_count[q] = kk;
        if (out_total) out_total[q] = s_tot;
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
    const uint32_t ntot = P.ntiles * KC;
    for (uint32_t i = threadIdx.x; i < ntot; i += blockDim.x) {
        uint32_t jt = i / KC, k = i % KC;
        const TileHeader &h = A.hdr[P.tile_base + jt];
        c[i] = (k < h.count) ? A.cands[static_cast<uint64_t>(P.tile_base + jt) * KC + k] : cand_sentinel();
    }
    const uint32_t n2 = next_pow2(ntot);
    for (uint32_t i = ntot + threadIdx.x; i < n2; i += blockDim.x) c[i] = cand_sentinel();
    __syncthreads();
    block_sort_cands(c, static_cast<int>(n2));
    const uint32_t kk = min(P.k, s_n);
    write_result(row, c, s_n, kk, kmax);
    if (threadIdx.x == 0) {
        out_count[q] = kk;
        if (out_total) out_total[q] = P.total;
        if (out_status) out_status[q] = MHR_Q_EXACT_PASS;
    }
}

// ---------------------------------------------------------------------------
// edge weights (unit entry point)
// ---------------------------------------------------------------------------
template <bool BF16>
__global__ void edge_weight_kernel(GArgs A, uint64_t ne, const uint32_t *u, const uint32_t *r, const uint32_t *v,
                                   float *w32, float *e32, float *whi, float *wlo) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const uint32_t uu = u[i], rr = r[i], vv = v[i];
    const size_t d = A.d;
    float x = 0.0f, as = 0.0f;
    for (uint32_t k = 0; k < A.d; ++k) {
        float z = load1<BF16>(A.X, uu * d + k) * load1<BF16>(A.Y, rr * d + k);
        float xv = load1<BF16>(A.X, vv * d + k);
        x = __builtin_fmaf(z, xv, x);
        as += fabsf(z * xv);
    }
    float f = centred_logsigmoid(x);
    float w = f - kLn2f;
    float err = gamma_n(static_cast<int>(A.d) + 2) * as + centred_logsigmoid_err(f) + kUnit * fabsf(w) +
                kUnit * kLn2f;
    if (w32) w32[i] = w;
    if (e32) e32[i] = err;
    float asf;
    ff wf = ff_logsigmoid(edge_x_ff<BF16>(A, uu, rr, vv, &asf));
    if (whi) whi[i] = wf.hi;
    if (wlo) wlo[i] = wf.lo;
}

GArgs make_args(const mhr_graph *g) {
    GArgs A{};
    A.out_rp = g->out.row_ptr; A.out_col = g->out.col; A.out_mask = g->out.rmask;
    A.out_dir_off = g->out.dir_off; A.out_dir_pool = g->out.dir_pool;
    A.in_rp = g->in.row_ptr; A.in_col = g->in.col; A.in_mask = g->in.rmask;
    A.in_dir_off = g->in.dir_off; A.in_dir_pool = g->in.dir_pool;
    A.X = g->X; A.Y = g->Y;
    A.n = g->n; A.R = g->R; A.d = g->dim; A.id_bits = g->id_bits;
    return A;
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------
struct WsLayout {
    size_t ctrl, plans, tile_start, tile_q, exact_list, hdr, cands, total;
};

uint32_t kc_for(uint32_t kmax) {
    uint32_t kc = 64;
    while (kc < kmax + 32) kc <<= 1;
    return kc;
}

WsLayout ws_layout(uint32_t nq, uint32_t kc) {
    const uint32_t maxt = max_tiles_for(kc);
    WsLayout W{};
    size_t o = 0;
    auto al = [](size_t v) { return (v + 255) & ~static_cast<size_t>(255); };
    W.ctrl = o; o = al(o + sizeof(Control));
    W.plans = o; o = al(o + size_t(nq) * sizeof(QueryPlan));
    W.tile_start = o; o = al(o + size_t(nq) * maxt * sizeof(uint2));
    W.tile_q = o; o = al(o + size_t(nq) * maxt * sizeof(uint32_t));
    W.exact_list = o; o = al(o + size_t(nq) * sizeof(uint32_t));
    W.hdr = o; o = al(o + size_t(nq) * maxt * sizeof(TileHeader));
    W.cands = o; o = al(o + size_t(nq) * maxt * kc * sizeof(Cand));
    W.total = o;
    return W;
}

int g_num_cus = 0;

template <bool BF16, int KC>
mhr_status launch_all(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq, const uint32_t *src,
                      const uint32_t *dst, const uint32_t *k, uint32_t kmax, mhr_path *out, uint32_t *out_count,
                      uint64_t *out_total, uint32_t *out_status, void *ws, hipStream_t st,
                      const mhr_phase_events *ev) {
    GArgs A = make_args(g);
    auto rec = [&](void *e) -> hipError_t {
        return e ? hipEventRecord(static_cast<hipEvent_t>(e), st) : hipSuccess;
    };
    const WsLayout W = ws_layout(nq, KC);
    char *base = static_cast<char *>(ws);
    A.ctrl = reinterpret_cast<Control *>(base + W.ctrl);
    A.plans = reinterpret_cast<QueryPlan *>(base + W.plans);
    A.tile_start = reinterpret_cast<uint2 *>(base + W.tile_start);
    A.tile_q = reinterpret_cast<uint32_t *>(base + W.tile_q);
    A.exact_list = reinterpret_cast<uint32_t *>(base + W.exact_list);
    A.hdr = reinterpret_cast<TileHeader *>(base + W.hdr);
    A.cands = reinterpret_cast<Cand *>(base + W.cands);
    A.maxt = max_tiles_for(KC);
    A.nq = nq;
    A.kc = KC;
    A.hash_log2 = (o && o->hash_log2) ? o->hash_log2 : kDefaultHashLog2;
    const uint32_t tile_edges = (o && o->tile_edges) ? o->tile_edges : kDefaultTileEdges;
    if (g_num_cus == 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, g->device) == hipSuccess) g_num_cus = prop.multiProcessorCount;
        if (g_num_cus <= 0) g_num_cus = 256;
    }
    const GatherLayout GL = gather_layout(A.hash_log2, A.R, A.d, KC);
    const uint32_t grid = (o && o->grid_blocks) ? o->grid_blocks : static_cast<uint32_t>(g_num_cus) * 2;
    const uint32_t kdef = o ? o->k : 0u;

    MHR_HIP_TRY(rec(ev ? ev->begin : nullptr));
    hipLaunchKernelGGL(plan_kernel, dim3(nq), dim3(kBlock), 0, st, A, src, dst, k, kdef, kmax, tile_edges);
    hipLaunchKernelGGL(schedule_kernel, dim3(1), dim3(kBlock), 0, st, A);
    auto gk = gather_kernel<BF16, false, KC>;
    MHR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(gk),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(GL.total)));
    MHR_HIP_TRY(rec(ev ? ev->gather_begin : nullptr));
    hipLaunchKernelGGL(gk, dim3(grid), dim3(kBlock), GL.total, st, A);
    MHR_HIP_TRY(rec(ev ? ev->gather_end : nullptr));
    const size_t msmem = size_t(next_pow2(max_tiles_for(KC) * KC)) * sizeof(Cand);
    auto mk = merge_kernel<BF16, KC>;
    MHR_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(mk),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(msmem)));
    hipLaunchKernelGGL(mk, dim3(nq), dim3(kBlock), msmem, st, A, out, out_count, out_total, out_status, kmax);
    auto xk = gather_kernel<BF16, true, KC>;
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
    return gather_layout(hash_log2 ? hash_log2 : kDefaultHashLog2, g->R, g->dim, kc_for(kmax)).total;
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

extern "C" mhr_status mhr_topk_paths_profiled(const mhr_graph *g, const mhr_query_opts *o, uint32_t nq,
                                              const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                              uint32_t kmax, mhr_path *out, uint32_t *out_count,
                                              uint64_t *out_total, uint32_t *out_status, void *workspace,
                                              size_t ws_bytes, void *stream, const mhr_phase_events *ev) {
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
        MHR_ARG_CHECK(o->hash_log2 == 0 || (o->hash_log2 >= 10 && o->hash_log2 <= 13), "hash_log2 must be 10..13");
        for (uint32_t v : o->reserved) MHR_ARG_CHECK(v == 0, "reserved option fields must be zero");
    }
    const uint32_t kc = kc_for(kmax);
    const size_t need = ws_layout(nq, kc).total;
    if (ws_bytes < need) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    const size_t lds = gather_lds_bytes(g, o ? o->hash_log2 : 0, kmax);
    if (lds > 160 * 1024) {
        set_error("LDS demand " + std::to_string(lds) + " exceeds 160 KiB (reduce hash_log2)");
        return MHR_ERR_UNSUPPORTED;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool bf = g->dtype == MHR_DTYPE_BF16;
    switch (kc) {
        case 64: return bf ? launch_all<true, 64>(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, st, ev)
                           : launch_all<false, 64>(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, st, ev);
        case 128: return bf ? launch_all<true, 128>(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, st, ev)
                            : launch_all<false, 128>(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, st, ev);
        default: return bf ? launch_all<true, 256>(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, st, ev)
                           : launch_all<false, 256>(g, o, nq, src, dst, k, kmax, out, out_count, out_total, out_status, workspace, st, ev);
    }
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
    if (g->dtype == MHR_DTYPE_BF16)
        hipLaunchKernelGGL(edge_weight_kernel<true>, dim3(blocks), dim3(256), 0, st, A, ne, u, r, v, w32, e32, whi, wlo);
    else
        hipLaunchKernelGGL(edge_weight_kernel<false>, dim3(blocks), dim3(256), 0, st, A, ne, u, r, v, w32, e32, whi, wlo);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}
