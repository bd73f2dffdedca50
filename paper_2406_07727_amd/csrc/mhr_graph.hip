// One-time graph ingest on the device: the edge list (h, r, t) of the
// problem statement is turned into a forward and a reverse CSR of distinct
// vertex pairs with relation bitmasks (identical triples merge), plus bucket
// directories for long rows.  The sort is an LSD radix sort written here
// (8-bit digits, stable block-local ranking).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "mhr_device.h"
#include "mhr_internal.h"

namespace mhr {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanBlock * kScanItems;

// Inclusive scan of one value per thread over the block; returns the
// inclusive prefix, and the block total in *total.
__device__ inline uint32_t block_inclusive_scan(uint32_t v, uint32_t *lds_wave, uint32_t *total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    for (int off = 1; off < kWave; off <<= 1) {
        uint32_t t = __shfl_up(v, off, kWave);
        if (lane >= off) v += t;
    }
    if (lane == kWave - 1) lds_wave[wave] = v;
    __syncthreads();
    if (wave == 0) {
        uint32_t w = lane < nwaves ? lds_wave[lane] : 0u;
        for (int off = 1; off < kWave; off <<= 1) {
            uint32_t t = __shfl_up(w, off, kWave);
            if (lane >= off) w += t;
        }
        if (lane < nwaves) lds_wave[lane] = w;
    }
    __syncthreads();
    uint32_t base = wave > 0 ? lds_wave[wave - 1] : 0u;
    *total = lds_wave[nwaves - 1];
    __syncthreads();
    return v + base;
}

__global__ void scan_reduce_kernel(const uint32_t *in, uint64_t n, uint32_t *partial) {
    __shared__ uint32_t lw[kScanBlock / kWave];
    uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanChunk;
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        uint64_t idx = base + static_cast<uint64_t>(threadIdx.x) * kScanItems + i;
        if (idx < n) s += in[idx];
    }
    uint32_t tot;
    block_inclusive_scan(s, lw, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Exclusive scan of the per-block partial sums by one block; also writes the
// grand total.
__global__ void scan_partials_kernel(uint32_t *partial, uint32_t nparts, uint32_t *grand) {
    __shared__ uint32_t lw[kScanBlock / kWave];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t b = 0; b < nparts; b += kScanBlock) {
        uint32_t i = b + threadIdx.x;
        uint32_t v = i < nparts ? partial[i] : 0u;
        uint32_t tot;
        uint32_t inc = block_inclusive_scan(v, lw, &tot);
        uint32_t c = carry;
        if (i < nparts) partial[i] = c + inc - v;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0 && grand) *grand = carry;
}

__global__ void scan_apply_kernel(const uint32_t *in, uint64_t n, const uint32_t *partial, uint32_t *out) {
    __shared__ uint32_t lw[kScanBlock / kWave];
    uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanChunk + static_cast<uint64_t>(threadIdx.x) * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t inc = block_inclusive_scan(s, lw, &tot);
    uint32_t run = partial[blockIdx.x] + inc - s;
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// ---------------------------------------------------------------------------
// LSD radix sort of 64-bit keys, 8 bits per pass.
// ---------------------------------------------------------------------------
constexpr int kSortBlock = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kBins = 256;

__global__ void radix_hist_kernel(const uint64_t *keys, uint64_t n, int shift, uint32_t ntiles, uint32_t *counts) {
    __shared__ uint32_t hist[kBins];
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        uint64_t idx = base + static_cast<uint64_t>(k) * kSortBlock + threadIdx.x;
        if (idx < n) atomicAdd(&hist[(keys[idx] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kBins; d += blockDim.x)
        counts[static_cast<uint64_t>(d) * ntiles + blockIdx.x] = hist[d];
}

// Stable scatter: items are ranked in their original order (row k of the
// tile holds items k*256 .. k*256+255).  Within a row, a wave finds the
// lanes sharing its digit with 8 ballots; wave totals per digit give the
// cross-wave offsets.
__global__ void radix_scatter_kernel(const uint64_t *keys, uint64_t *out, uint64_t n, int shift,
                                     uint32_t ntiles, const uint32_t *offsets) {
    constexpr int kWaves = kSortBlock / kWave;
    __shared__ uint32_t base_off[kBins];
    __shared__ uint32_t wcnt[kWaves][kBins];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    for (int d = threadIdx.x; d < kBins; d += blockDim.x)
        base_off[d] = offsets[static_cast<uint64_t>(d) * ntiles + blockIdx.x];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    uint64_t tile = static_cast<uint64_t>(blockIdx.x) * kSortTile;
    for (int k = 0; k < kSortItems; ++k) {
        for (int i = threadIdx.x; i < kWaves * kBins; i += blockDim.x) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        uint64_t idx = tile + static_cast<uint64_t>(k) * kSortBlock + threadIdx.x;
        const bool valid = idx < n;
        uint64_t key = valid ? keys[idx] : 0ull;
        uint32_t dg = static_cast<uint32_t>((key >> shift) & 0xFF);
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot(((dg >> b) & 1u) != 0);
            peers &= ((dg >> b) & 1u) ? bal : ~bal;
        }
        uint32_t rank_in_wave = __popcll(peers & lt_mask);
        uint32_t cnt_in_wave = __popcll(peers);
        if (valid && rank_in_wave == 0) wcnt[wave][dg] = cnt_in_wave;
        __syncthreads();
        if (valid) {
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += wcnt[w][dg];
            out[base_off[dg] + before + rank_in_wave] = key;
        }
        __syncthreads();
        for (int d = threadIdx.x; d < kBins; d += blockDim.x) {
            uint32_t s = 0;
            for (int w = 0; w < kWaves; ++w) s += wcnt[w][d];
            base_off[d] += s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Graph kernels
// ---------------------------------------------------------------------------
__global__ void make_keys_kernel(const uint32_t *head, const uint32_t *rel, const uint32_t *tail, uint64_t m,
                                 uint32_t n, uint32_t R, int id_bits, int reverse, uint64_t *keys, uint32_t *err) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    uint32_t u = head[i], r = rel[i], v = tail[i];
    if (u >= n || v >= n || r >= R) {
        atomicOr(err, 1u);
        u = 0; v = 0; r = 0;
    }
    uint32_t a = reverse ? v : u, b = reverse ? u : v;
    keys[i] = (((static_cast<uint64_t>(a) << id_bits) | b) << 5) | r;
}

__global__ void pair_flags_kernel(const uint64_t *keys, uint64_t m, uint32_t *newpair, uint32_t *newtriple) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    uint64_t k = keys[i];
    uint64_t p = i ? keys[i - 1] : ~0ull;
    newpair[i] = (i == 0 || (k >> 5) != (p >> 5)) ? 1u : 0u;
    newtriple[i] = (i == 0 || k != p) ? 1u : 0u;
}

__global__ void fill_csr_kernel(const uint64_t *keys, uint64_t m, const uint32_t *newpair, const uint32_t *pexcl,
                                int id_bits, uint32_t n, uint32_t num_pairs, uint32_t *row_ptr, uint32_t *col,
                                uint32_t *rmask) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint64_t vmask = (1ull << id_bits) - 1;
    uint64_t k = keys[i];
    uint32_t r = static_cast<uint32_t>(k & 31u);
    uint32_t v = static_cast<uint32_t>((k >> 5) & vmask);
    uint32_t u = static_cast<uint32_t>(k >> (5 + id_bits));
    uint32_t p = pexcl[i] + newpair[i] - 1;
    atomicOr(&rmask[p], 1u << r);
    if (newpair[i]) {
        col[p] = v;
        int64_t uprev = (i == 0) ? -1 : static_cast<int64_t>(keys[i - 1] >> (5 + id_bits));
        for (int64_t x = uprev + 1; x <= static_cast<int64_t>(u); ++x) row_ptr[x] = p;
    }
    if (i == m - 1)
        for (uint64_t x = static_cast<uint64_t>(u) + 1; x <= n; ++x) row_ptr[x] = num_pairs;
}

__global__ void dir_sizes_kernel(const uint32_t *row_ptr, uint32_t n, uint32_t *sizes, uint32_t *maxdeg,
                                 uint32_t *heavy_list, uint32_t *heavy_n) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    uint32_t deg = row_ptr[v + 1] - row_ptr[v];
    atomicMax(maxdeg, deg);
    uint32_t sz = 0;
    if (deg > kDirMinDegree) {
        sz = next_pow2(deg) / 2 + 1;
        uint32_t slot = atomicAdd(heavy_n, 1u);
        heavy_list[slot] = v;
    }
    sizes[v] = sz;
}

__global__ void dir_off_kernel(const uint32_t *sizes, const uint32_t *excl, uint32_t n, uint32_t *dir_off) {
    uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    dir_off[v] = sizes[v] ? excl[v] : 0xFFFFFFFFu;
}

__global__ void dir_fill_kernel(const uint32_t *heavy_list, const uint32_t *row_ptr, const uint32_t *col,
                                const uint32_t *dir_off, int id_bits, uint32_t *pool) {
    uint32_t v = heavy_list[blockIdx.x];
    uint32_t beg = row_ptr[v];
    uint32_t deg = row_ptr[v + 1] - beg;
    uint32_t nb = next_pow2(deg) / 2;
    int B = 31 - __clz(nb);
    int sh = id_bits - B;
    uint32_t *dir = pool + dir_off[v];
    for (uint32_t i = threadIdx.x; i < deg; i += blockDim.x) {
        int64_t k = col[beg + i] >> sh;
        int64_t kp = i ? static_cast<int64_t>(col[beg + i - 1] >> sh) : -1;
        for (int64_t kk = kp + 1; kk <= k; ++kk) dir[kk] = i;
        if (i == deg - 1)
            for (int64_t kk = k + 1; kk <= static_cast<int64_t>(nb); ++kk) dir[kk] = deg;
    }
}

inline uint32_t cdiv(uint64_t a, uint64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

}  // namespace

// Exclusive scan of n uint32 (out may equal in); optional total.
mhr_status device_exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *d_total,
                                 uint32_t *scratch, hipStream_t st) {
    if (n == 0) {
        if (d_total) MHR_HIP_TRY(hipMemsetAsync(d_total, 0, sizeof(uint32_t), st));
        return MHR_OK;
    }
    uint32_t nb = cdiv(n, kScanChunk);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(kScanBlock), 0, st, in, n, scratch);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(kScanBlock), 0, st, scratch, nb, d_total);
    hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(kScanBlock), 0, st, in, n, scratch, out);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

namespace {

// Device memory of one graph build.  Every buffer comes from one of two
// places: the caller's buffers (bump allocation in 256-byte pieces, in the
// order of the calls below, which is the order mhr_graph_buffer_sizes
// counts), or hipMalloc when the caller gave none.  Temporaries allocated
// with hipMalloc are freed when the build ends; CSR arrays allocated with
// hipMalloc belong to the handle.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
};

constexpr size_t kPiece = 256;
inline size_t piece(size_t bytes) { return (std::max<size_t>(bytes, 1) + kPiece - 1) / kPiece * kPiece; }

struct BuildMem {
    Arena *tmp = nullptr;   // null: temporaries by hipMalloc
    Arena *csr = nullptr;   // null: CSR arrays by hipMalloc (owned by the handle)
    std::vector<void *> tmp_owned;
    ~BuildMem() {
        for (void *p : tmp_owned) (void)hipFree(p);
    }
    static hipError_t take(Arena *a, void **p, size_t bytes) {
        const size_t b = piece(bytes);
        if (a->used + b > a->cap) return hipErrorOutOfMemory;
        *p = a->base + a->used;
        a->used += b;
        return hipSuccess;
    }
    template <class T>
    hipError_t temp(T **p, size_t count) {
        void *v = nullptr;
        hipError_t e;
        if (tmp) {
            e = take(tmp, &v, count * sizeof(T));
        } else {
            e = hipMalloc(&v, piece(count * sizeof(T)));
            if (e == hipSuccess) tmp_owned.push_back(v);
        }
        *p = static_cast<T *>(v);
        return e;
    }
    template <class T>
    hipError_t keep(T **p, size_t count) {
        void *v = nullptr;
        hipError_t e = csr ? take(csr, &v, count * sizeof(T)) : hipMalloc(&v, piece(count * sizeof(T)));
        *p = static_cast<T *>(v);
        return e;
    }
};

// Element counts of the temporaries of one direction's build, in allocation
// order (both directions reuse the same temporaries).
struct TempCounts {
    uint64_t keys, tmp, err, counts, sort_scratch, newpair, newtriple, pexcl, scratch, totals, sizes, sexcl, heavy,
        hn, maxdeg, tot, scratch2;
};

TempCounts temp_counts(uint32_t n, uint64_t m) {
    TempCounts c{};
    const uint64_t nc = static_cast<uint64_t>(cdiv(m, kSortTile)) * kBins;
    c.keys = m;            // uint64
    c.tmp = m;             // uint64
    c.err = 1;
    c.counts = nc;
    c.sort_scratch = cdiv(nc, kScanChunk) + 1;
    c.newpair = m;
    c.newtriple = m;
    c.pexcl = m;
    c.scratch = cdiv(m, kScanChunk) + 1;
    c.totals = 2;
    c.sizes = n;
    c.sexcl = n;
    c.heavy = n;
    c.hn = c.maxdeg = c.tot = 1;
    c.scratch2 = cdiv(n, kScanChunk) + 1;
    return c;
}

size_t temp_bytes(uint32_t n, uint64_t m) {
    const TempCounts c = temp_counts(n, m);
    return piece(c.keys * 8) + piece(c.tmp * 8) + piece(c.err * 4) + piece(c.counts * 4) +
           piece(c.sort_scratch * 4) + piece(c.newpair * 4) + piece(c.newtriple * 4) + piece(c.pexcl * 4) +
           piece(c.scratch * 4) + piece(c.totals * 4) + piece(c.sizes * 4) + piece(c.sexcl * 4) +
           piece(c.heavy * 4) + piece(c.hn * 4) + piece(c.maxdeg * 4) + piece(c.tot * 4) + piece(c.scratch2 * 4);
}

// Upper bound on the directory pool of one direction: a row of degree deg
// > kDirMinDegree takes next_pow2(deg) / 2 + 1 <= deg + 1 words.
uint64_t dir_pool_bound(uint64_t m) { return m + m / (kDirMinDegree + 1) + 1; }

// CSR bytes of one direction when the pair count and pool length are known
// (the caller-buffer form uses the bounds num_pairs <= m and
// dir_pool_bound(m)).
size_t csr_bytes(uint32_t n, uint64_t pairs, uint64_t pool) {
    return piece((static_cast<uint64_t>(n) + 1) * 4) + 2 * piece(pairs * 4) + piece(static_cast<uint64_t>(n) * 4) +
           piece(pool * 4);
}

mhr_status radix_sort(uint64_t *&keys, uint64_t *&tmp, uint64_t n, int bits, uint32_t *counts,
                      uint32_t *scratch, hipStream_t st) {
    if (n <= 1) return MHR_OK;
    uint32_t ntiles = cdiv(n, kSortTile);
    uint64_t nc = static_cast<uint64_t>(ntiles) * kBins;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(radix_hist_kernel, dim3(ntiles), dim3(kSortBlock), 0, st, keys, n, shift, ntiles, counts);
        mhr_status s = device_exclusive_scan(counts, counts, nc, nullptr, scratch, st);
        if (s != MHR_OK) return s;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(ntiles), dim3(kSortBlock), 0, st, keys, tmp, n, shift, ntiles,
                           counts);
        MHR_HIP_TRY(hipGetLastError());
        std::swap(keys, tmp);
    }
    MHR_HIP_TRY(hipStreamSynchronize(st));
    return MHR_OK;
}

// Builds one direction.  Temporaries come from mem (the same pieces for
// both directions: `t` is reused), the CSR arrays too; when the CSR lives in
// the caller's buffer its arrays take the bounds (m pairs, dir_pool_bound).
struct Temps {
    uint64_t *keys = nullptr, *tmp = nullptr;
    uint32_t *err = nullptr, *counts = nullptr, *sort_scratch = nullptr, *newpair = nullptr, *newtriple = nullptr,
             *pexcl = nullptr, *scratch = nullptr, *totals = nullptr, *sizes = nullptr, *sexcl = nullptr,
             *heavy = nullptr, *hn = nullptr, *maxdeg = nullptr, *tot = nullptr, *scratch2 = nullptr;
};

mhr_status alloc_temps(BuildMem &mem, uint32_t n, uint64_t m, Temps &t) {
    const TempCounts c = temp_counts(n, m);
    MHR_HIP_TRY(mem.temp(&t.keys, c.keys));
    MHR_HIP_TRY(mem.temp(&t.tmp, c.tmp));
    MHR_HIP_TRY(mem.temp(&t.err, c.err));
    MHR_HIP_TRY(mem.temp(&t.counts, c.counts));
    MHR_HIP_TRY(mem.temp(&t.sort_scratch, c.sort_scratch));
    MHR_HIP_TRY(mem.temp(&t.newpair, c.newpair));
    MHR_HIP_TRY(mem.temp(&t.newtriple, c.newtriple));
    MHR_HIP_TRY(mem.temp(&t.pexcl, c.pexcl));
    MHR_HIP_TRY(mem.temp(&t.scratch, c.scratch));
    MHR_HIP_TRY(mem.temp(&t.totals, c.totals));
    MHR_HIP_TRY(mem.temp(&t.sizes, c.sizes));
    MHR_HIP_TRY(mem.temp(&t.sexcl, c.sexcl));
    MHR_HIP_TRY(mem.temp(&t.heavy, c.heavy));
    MHR_HIP_TRY(mem.temp(&t.hn, c.hn));
    MHR_HIP_TRY(mem.temp(&t.maxdeg, c.maxdeg));
    MHR_HIP_TRY(mem.temp(&t.tot, c.tot));
    MHR_HIP_TRY(mem.temp(&t.scratch2, c.scratch2));
    return MHR_OK;
}

mhr_status build_direction(mhr_graph *g, const mhr_graph_desc *d, int reverse, Csr &csr, BuildMem &mem,
                           const Temps &t, hipStream_t st) {
    const uint64_t m = d->num_edges;
    const uint32_t n = g->n;
    MHR_HIP_TRY(hipMemsetAsync(t.err, 0, sizeof(uint32_t), st));
    uint64_t *keys = t.keys, *tmp = t.tmp;
    if (m) {
        hipLaunchKernelGGL(make_keys_kernel, dim3(cdiv(m, 256)), dim3(256), 0, st, d->head, d->rel, d->tail, m, n,
                           g->R, static_cast<int>(g->id_bits), reverse, keys, t.err);
        MHR_HIP_TRY(hipGetLastError());
    }
    uint32_t herr = 0;
    MHR_HIP_TRY(hipMemcpyAsync(&herr, t.err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipStreamSynchronize(st));
    if (herr) {
        set_error("edge list holds a vertex id >= num_vertices or a relation id >= num_relations");
        return MHR_ERR_BAD_EDGE;
    }
    mhr_status s = radix_sort(keys, tmp, m, 2 * static_cast<int>(g->id_bits) + 5, t.counts, t.sort_scratch, st);
    if (s != MHR_OK) return s;

    if (m) {
        hipLaunchKernelGGL(pair_flags_kernel, dim3(cdiv(m, 256)), dim3(256), 0, st, keys, m, t.newpair, t.newtriple);
        MHR_HIP_TRY(hipGetLastError());
    }
    s = device_exclusive_scan(t.newpair, t.pexcl, m, t.totals, t.scratch, st);
    if (s != MHR_OK) return s;
    // triples: reuse newtriple as its own scan output; only the total matters
    s = device_exclusive_scan(t.newtriple, t.newtriple, m, t.totals + 1, t.scratch, st);
    if (s != MHR_OK) return s;
    uint32_t ht[2] = {0, 0};
    MHR_HIP_TRY(hipMemcpyAsync(ht, t.totals, sizeof(ht), hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipStreamSynchronize(st));
    const uint32_t num_pairs = ht[0];
    g->num_pairs = num_pairs;
    g->num_triples = ht[1];

    const uint64_t cap_pairs = mem.csr ? m : num_pairs;   // caller buffer: sized before the pair count is known
    const size_t used0 = mem.csr ? mem.csr->used : 0;
    MHR_HIP_TRY(mem.keep(&csr.row_ptr, static_cast<size_t>(n) + 1));
    MHR_HIP_TRY(mem.keep(&csr.col, cap_pairs));
    MHR_HIP_TRY(mem.keep(&csr.rmask, cap_pairs));
    MHR_HIP_TRY(hipMemsetAsync(csr.rmask, 0, std::max<size_t>(num_pairs, 1) * sizeof(uint32_t), st));
    MHR_HIP_TRY(hipMemsetAsync(csr.row_ptr, 0, (static_cast<size_t>(n) + 1) * sizeof(uint32_t), st));
    if (m) {
        hipLaunchKernelGGL(fill_csr_kernel, dim3(cdiv(m, 256)), dim3(256), 0, st, keys, m, t.newpair, t.pexcl,
                           static_cast<int>(g->id_bits), n, num_pairs, csr.row_ptr, csr.col, csr.rmask);
        MHR_HIP_TRY(hipGetLastError());
    }

    // directories of long rows
    MHR_HIP_TRY(hipMemsetAsync(t.hn, 0, sizeof(uint32_t), st));
    MHR_HIP_TRY(hipMemsetAsync(t.maxdeg, 0, sizeof(uint32_t), st));
    hipLaunchKernelGGL(dir_sizes_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, csr.row_ptr, n, t.sizes, t.maxdeg,
                       t.heavy, t.hn);
    MHR_HIP_TRY(hipGetLastError());
    s = device_exclusive_scan(t.sizes, t.sexcl, n, t.tot, t.scratch2, st);
    if (s != MHR_OK) return s;
    uint32_t hv[3] = {0, 0, 0};
    MHR_HIP_TRY(hipMemcpyAsync(&hv[0], t.hn, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipMemcpyAsync(&hv[1], t.maxdeg, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipMemcpyAsync(&hv[2], t.tot, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipStreamSynchronize(st));
    csr.heavy_rows = hv[0];
    csr.max_degree = hv[1];
    csr.dir_pool_len = hv[2];
    if (mem.csr && csr.dir_pool_len > dir_pool_bound(m)) {   // cannot happen (each row takes <= deg + 1 words)
        set_error("directory pool exceeds its bound");
        return MHR_ERR_DEVICE;
    }
    MHR_HIP_TRY(mem.keep(&csr.dir_off, n));
    MHR_HIP_TRY(mem.keep(&csr.dir_pool, mem.csr ? dir_pool_bound(m) : csr.dir_pool_len));
    g->device_bytes += mem.csr ? mem.csr->used - used0 : csr_bytes(n, num_pairs, csr.dir_pool_len);
    hipLaunchKernelGGL(dir_off_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, t.sizes, t.sexcl, n, csr.dir_off);
    if (csr.heavy_rows)
        hipLaunchKernelGGL(dir_fill_kernel, dim3(csr.heavy_rows), dim3(256), 0, st, t.heavy, csr.row_ptr, csr.col,
                           csr.dir_off, static_cast<int>(g->id_bits), csr.dir_pool);
    MHR_HIP_TRY(hipGetLastError());
    MHR_HIP_TRY(hipStreamSynchronize(st));
    return MHR_OK;
}

void free_csr(mhr::Csr &c, bool owned) {
    if (!owned) {
        c = mhr::Csr();
        return;
    }
    if (c.row_ptr) (void)hipFree(c.row_ptr);
    if (c.col) (void)hipFree(c.col);
    if (c.rmask) (void)hipFree(c.rmask);
    if (c.dir_off) (void)hipFree(c.dir_off);
    if (c.dir_pool) (void)hipFree(c.dir_pool);
    c = mhr::Csr();
}

}  // namespace
}  // namespace mhr

using namespace mhr;

namespace {

mhr_status check_desc(const mhr_graph_desc *d) {
    MHR_ARG_CHECK(d != nullptr, "graph descriptor is null");
    MHR_ARG_CHECK(d->num_vertices >= 1 && d->num_vertices < 0xFFFFFFFFu, "num_vertices must be in [1, 2^32-2]");
    MHR_ARG_CHECK(d->num_relations >= 1 && d->num_relations <= MHR_MAX_RELATIONS, "num_relations must be in [1, 32]");
    MHR_ARG_CHECK(d->num_edges < 0xFFFFFFFFull, "num_edges must be < 2^32");
    MHR_ARG_CHECK(d->num_edges == 0 || (d->head && d->rel && d->tail), "edge arrays must not be null");
    return MHR_OK;
}

uint32_t id_bits_for(uint32_t n) {
    uint32_t bits = 1;
    while (bits < 32 && (1ull << bits) < n) ++bits;
    return bits;
}

// Both directions of the build; mem says where the memory comes from.
mhr_status create_graph(const mhr_graph_desc *d, BuildMem &mem, hipStream_t st, mhr_graph **out) {
    mhr_graph *g = new (std::nothrow) mhr_graph();
    if (!g) {
        set_error("host allocation failed");
        return MHR_ERR_OUT_OF_MEMORY;
    }
    g->n = d->num_vertices;
    g->R = d->num_relations;
    g->id_bits = id_bits_for(g->n);
    g->owns_csr = mem.csr == nullptr;
    if (2 * g->id_bits + 5 > 64) {
        delete g;
        set_error("too many vertices for the 64-bit sort key");
        return MHR_ERR_UNSUPPORTED;
    }
    (void)hipGetDevice(&g->device);
    Temps t;
    mhr_status s = alloc_temps(mem, g->n, d->num_edges, t);
    if (s == MHR_OK) s = build_direction(g, d, 0, g->out, mem, t, st);
    if (s == MHR_OK) s = build_direction(g, d, 1, g->in, mem, t, st);
    if (s != MHR_OK) {
        free_csr(g->out, g->owns_csr);
        free_csr(g->in, g->owns_csr);
        delete g;
        return s;
    }
    *out = g;
    return MHR_OK;
}

}  // namespace

extern "C" mhr_status mhr_graph_buffer_sizes(uint32_t num_vertices, uint32_t num_relations, uint64_t num_edges,
                                             size_t *csr_buffer_bytes, size_t *tmp_buffer_bytes) {
    MHR_ARG_CHECK(csr_buffer_bytes && tmp_buffer_bytes, "mhr_graph_buffer_sizes: null argument");
    mhr_graph_desc d{};
    d.num_vertices = num_vertices;
    d.num_relations = num_relations;
    d.num_edges = num_edges;
    d.head = d.rel = d.tail = reinterpret_cast<const uint32_t *>(kPiece);   // shape check only
    mhr_status s = check_desc(&d);
    if (s != MHR_OK) return s;
    *csr_buffer_bytes = 2 * csr_bytes(num_vertices, num_edges, dir_pool_bound(num_edges));
    *tmp_buffer_bytes = temp_bytes(num_vertices, num_edges);
    return MHR_OK;
}

extern "C" mhr_status mhr_graph_create(const mhr_graph_desc *d, void *stream, mhr_graph **out) {
    MHR_ARG_CHECK(out != nullptr, "mhr_graph_create: null argument");
    mhr_status s = check_desc(d);
    if (s != MHR_OK) return s;
    BuildMem mem;
    return create_graph(d, mem, static_cast<hipStream_t>(stream), out);
}

extern "C" mhr_status mhr_graph_create_in(const mhr_graph_desc *d, void *csr_buffer, size_t csr_buffer_bytes,
                                          void *tmp_buffer, size_t tmp_buffer_bytes, void *stream, mhr_graph **out) {
    MHR_ARG_CHECK(out != nullptr && csr_buffer != nullptr && tmp_buffer != nullptr,
                  "mhr_graph_create_in: null argument");
    mhr_status s = check_desc(d);
    if (s != MHR_OK) return s;
    MHR_ARG_CHECK((reinterpret_cast<uintptr_t>(csr_buffer) % kPiece) == 0 &&
                      (reinterpret_cast<uintptr_t>(tmp_buffer) % kPiece) == 0,
                  "graph buffers must be 256-byte aligned");
    size_t need_csr = 0, need_tmp = 0;
    s = mhr_graph_buffer_sizes(d->num_vertices, d->num_relations, d->num_edges, &need_csr, &need_tmp);
    if (s != MHR_OK) return s;
    if (csr_buffer_bytes < need_csr || tmp_buffer_bytes < need_tmp) {
        set_error("graph buffers smaller than mhr_graph_buffer_sizes: csr " + std::to_string(csr_buffer_bytes) +
                  " < " + std::to_string(need_csr) + " or tmp " + std::to_string(tmp_buffer_bytes) + " < " +
                  std::to_string(need_tmp));
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    Arena csr{static_cast<char *>(csr_buffer), csr_buffer_bytes, 0};
    Arena tmp{static_cast<char *>(tmp_buffer), tmp_buffer_bytes, 0};
    BuildMem mem;
    mem.csr = &csr;
    mem.tmp = &tmp;
    return create_graph(d, mem, static_cast<hipStream_t>(stream), out);
}

extern "C" mhr_status mhr_graph_destroy(mhr_graph *g) {
    if (!g) return MHR_OK;
    free_csr(g->out, g->owns_csr);
    free_csr(g->in, g->owns_csr);
    delete g;
    return MHR_OK;
}

extern "C" mhr_status mhr_graph_set_scorer(mhr_graph *g, mhr_scorer scorer, float gamma) {
    MHR_ARG_CHECK(g != nullptr, "mhr_graph_set_scorer: null graph");
    MHR_ARG_CHECK(scorer == MHR_SCORER_DISTMULT || scorer == MHR_SCORER_TRANSE_L1, "unknown scorer");
    MHR_ARG_CHECK(gamma == gamma && gamma <= 3.0e38f && gamma >= -3.0e38f, "gamma must be finite");
    g->scorer = scorer;
    g->gamma = gamma;
    return MHR_OK;
}

extern "C" mhr_status mhr_graph_get_stats(const mhr_graph *g, mhr_graph_stats *o) {
    MHR_ARG_CHECK(g && o, "mhr_graph_get_stats: null argument");
    mhr_graph_stats s{};
    s.num_vertices = g->n;
    s.num_relations = g->R;
    s.num_triples = g->num_triples;
    s.num_pairs = g->num_pairs;
    s.max_out_degree = g->out.max_degree;
    s.max_in_degree = g->in.max_degree;
    s.dim = g->dim;
    s.dtype = g->dtype;
    s.device_bytes = g->device_bytes;
    s.heavy_rows_out = g->out.heavy_rows;
    s.heavy_rows_in = g->in.heavy_rows;
    *o = s;
    return MHR_OK;
}

extern "C" mhr_status mhr_graph_export_csr(const mhr_graph *g, int reverse, uint32_t *row_ptr, uint32_t *col,
                                           uint32_t *rmask, void *stream) {
    MHR_ARG_CHECK(g && row_ptr && col && rmask, "mhr_graph_export_csr: null argument");
    const Csr &c = reverse ? g->in : g->out;
    hipStream_t st = static_cast<hipStream_t>(stream);
    MHR_HIP_TRY(hipMemcpyAsync(row_ptr, c.row_ptr, (static_cast<size_t>(g->n) + 1) * sizeof(uint32_t),
                               hipMemcpyDeviceToDevice, st));
    if (g->num_pairs) {
        MHR_HIP_TRY(hipMemcpyAsync(col, c.col, g->num_pairs * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
        MHR_HIP_TRY(hipMemcpyAsync(rmask, c.rmask, g->num_pairs * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    }
    return MHR_OK;
}

extern "C" mhr_status mhr_graph_set_embeddings(mhr_graph *g, mhr_dtype dtype, uint32_t dim, const void *entity,
                                               const void *relation, void *stream) {
    (void)stream;
    MHR_ARG_CHECK(g && entity && relation, "mhr_graph_set_embeddings: null argument");
    MHR_ARG_CHECK(dtype == MHR_DTYPE_F32 || dtype == MHR_DTYPE_BF16, "dtype must be F32 or BF16");
    MHR_ARG_CHECK(dim >= 8 && dim <= 512 && (dim & (dim - 1)) == 0, "dim must be a power of two in [8, 512]");
    MHR_ARG_CHECK((reinterpret_cast<uintptr_t>(entity) & 15u) == 0 && (reinterpret_cast<uintptr_t>(relation) & 15u) == 0,
                  "embedding tables must be 16-byte aligned");
    g->X = entity;
    g->Y = relation;
    g->dim = dim;
    g->dtype = dtype;
    return MHR_OK;
}
