// Host-side internals of the library: the graph handle, the per-query plan
// record shared by the query kernels, error reporting helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "mhr.h"

namespace mhr {

// Thread-local message of the last error.
void set_error(const std::string &msg);
const std::string &last_error();

#define MHR_HIP_TRY(expr)                                                          \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::mhr::set_error(std::string(#expr) + ": " + hipGetErrorString(e_)); \
            return MHR_ERR_DEVICE;                                                 \
        }                                                                          \
    } while (0)

#define MHR_ARG_CHECK(cond, msg)                      \
    do {                                              \
        if (!(cond)) {                                \
            ::mhr::set_error(msg);                    \
            return MHR_ERR_INVALID_ARGUMENT;          \
        }                                             \
    } while (0)

// One compressed sparse row adjacency: rows are vertices, entries are the
// distinct neighbours in ascending id order, each with the bitmask of the
// relations that join the pair.  Rows longer than kDirMinDegree also carry
// a bucket directory (see dir_* below).
struct Csr {
    uint32_t *row_ptr = nullptr;  // n + 1
    uint32_t *col = nullptr;      // nnz
    uint32_t *rmask = nullptr;    // nnz
    // Directory of long rows: dir_off[v] = offset into dir_pool, or
    // 0xFFFFFFFF.  A row of degree deg gets nb = next_pow2(deg) / 2 buckets;
    // bucket k holds the entries whose id >> (id_bits - log2 nb) == k, and
    // dir_pool[dir_off[v] + k] is the index (relative to the row start) of
    // its first entry; dir_pool[dir_off[v] + nb] = deg.
    uint32_t *dir_off = nullptr;  // n
    uint32_t *dir_pool = nullptr;
    uint64_t dir_pool_len = 0;
    uint32_t max_degree = 0;
    uint32_t heavy_rows = 0;
};

constexpr uint32_t kDirMinDegree = 512;

// Exclusive scan of n uint32 on the device (out may equal in); the grand
// total goes to *d_total when it is not null.  scratch holds
// n / 2048 + 1 uint32.
mhr_status device_exclusive_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *d_total,
                                 uint32_t *scratch, hipStream_t st);

}  // namespace mhr

struct mhr_graph {
    uint32_t n = 0, R = 0;
    uint32_t id_bits = 1;  // ceil(log2(n)), at least 1
    uint64_t num_triples = 0;
    uint64_t num_pairs = 0;
    mhr::Csr out, in;
    // embeddings (borrowed)
    const void *X = nullptr;
    const void *Y = nullptr;
    uint32_t dim = 0;
    mhr_dtype dtype = MHR_DTYPE_F32;
    mhr_scorer scorer = MHR_SCORER_DISTMULT;
    float gamma = 1.0f;           // TransE-L1 constant
    uint64_t device_bytes = 0;
    int device = 0;
    bool owns_csr = true;         // false: the CSR arrays live in the caller's buffer
};

namespace mhr {

// Per-query plan written by the planning kernel and read by the later ones.
struct QueryPlan {
    uint32_t s, t, k, status;
    uint32_t dir;           // 0: backward (probe N+(s), scan in-rows of N-(t)); 1: forward
    uint32_t probe_beg;     // probe row start in the probe CSR
    uint32_t probe_len;
    uint32_t list_beg;      // list row start in the scan CSR
    uint32_t list_len;
    uint32_t ntiles;
    uint32_t tile_base;
    uint32_t flags;         // kNeedExact
    float thr;              // exact pass: centred-score threshold
    float kth_low;          // exhaustive pass: a lower bound on the query's true K-th score
    uint64_t cost;          // scan entries
    uint64_t total;         // |P(s,t)|
    uint32_t pad[2];
};
static_assert(sizeof(QueryPlan) == 80, "plan layout");

constexpr uint32_t kNeedExact = 1u;

struct TileHeader {
    uint32_t count;       // candidates kept (<= KC)
    uint32_t truncated;   // 1 if some candidate was dropped
    float cutoff;         // centred score of the last kept candidate when truncated
    float eps;            // largest error bound over the tile's scored paths
    uint64_t npaths;      // paths enumerated by the tile
    uint64_t pad;
};
static_assert(sizeof(TileHeader) == 32, "tile header layout");

struct Control {
    uint32_t total_tiles;
    uint32_t gather_ctr;
    uint32_t exact_ctr;
    uint32_t exact_n;
    uint32_t pad[60];
};

}  // namespace mhr
