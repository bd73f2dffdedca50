// Files of the library: the learned pruner's checkpoint (parameters and
// Adam state, for resuming training) and the autotuner's cache of tuned
// settings.  Both are little-endian binary files guarded by CRC-32
// checksums (the IEEE 802.3 polynomial, reflected form 0xEDB88320, as in
// zlib and PNG).  Files are written to a temporary name and renamed, so a
// reader never sees a half-written file.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mhr_internal.h"
#include "mhr_pruner_internal.h"

namespace mhr {
namespace {

// CRC-32, byte-wise with a 256-entry table (built once, thread-safely, on
// first use).
struct CrcTable {
    uint32_t t[256];
    CrcTable() {
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int k = 0; k < 8; ++k) c = (c & 1u) ? (0xEDB88320u ^ (c >> 1)) : (c >> 1);
            t[i] = c;
        }
    }
};

uint32_t crc32_update(uint32_t crc, const void *data, size_t n) {
    static const CrcTable table;
    const unsigned char *p = static_cast<const unsigned char *>(data);
    crc = ~crc;
    for (size_t i = 0; i < n; ++i) crc = table.t[(crc ^ p[i]) & 0xFFu] ^ (crc >> 8);
    return ~crc;
}

bool read_file(const char *path, std::vector<unsigned char> &out) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    out.clear();
    unsigned char buf[1 << 16];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) out.insert(out.end(), buf, buf + n);
    const bool ok = std::ferror(f) == 0;
    std::fclose(f);
    return ok;
}

bool write_file_atomic(const char *path, const std::vector<unsigned char> &data) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    const bool ok = std::fwrite(data.data(), 1, data.size(), f) == data.size();
    if (std::fclose(f) != 0 || !ok) {
        std::remove(tmp.c_str());
        return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

// ---------------------------------------------------------------------------
// pruner checkpoint
//   bytes  0..7   magic "MHRPRUN1"
//          8..11  format version (1)
//         12..15  embedding dimension
//         16..19  hidden width
//         20..23  Adam step count
//         24..31  parameter count n
//         32..35  CRC-32 of the payload
//         36..39  CRC-32 of bytes 0..35
//   payload       float32 parameters[n], first moments[n], second moments[n]
// ---------------------------------------------------------------------------
constexpr char kPrunerMagic[8] = {'M', 'H', 'R', 'P', 'R', 'U', 'N', '1'};
constexpr uint32_t kPrunerVersion = 1;
constexpr size_t kPrunerHeader = 40;

struct PrunerFileInfo {
    uint32_t dim, hidden, step;
    uint64_t n;
};

mhr_status parse_pruner_file(const std::vector<unsigned char> &f, PrunerFileInfo *info) {
    if (f.size() < kPrunerHeader || std::memcmp(f.data(), kPrunerMagic, 8) != 0) {
        set_error("pruner checkpoint: not a pruner checkpoint (bad magic)");
        return MHR_ERR_CORRUPT;
    }
    uint32_t version, hcrc, pcrc;
    std::memcpy(&version, f.data() + 8, 4);
    std::memcpy(&info->dim, f.data() + 12, 4);
    std::memcpy(&info->hidden, f.data() + 16, 4);
    std::memcpy(&info->step, f.data() + 20, 4);
    std::memcpy(&info->n, f.data() + 24, 8);
    std::memcpy(&pcrc, f.data() + 32, 4);
    std::memcpy(&hcrc, f.data() + 36, 4);
    if (crc32_update(0, f.data(), 36) != hcrc) {
        set_error("pruner checkpoint: header checksum mismatch");
        return MHR_ERR_CORRUPT;
    }
    if (version != kPrunerVersion) {
        set_error("pruner checkpoint: unsupported format version " + std::to_string(version));
        return MHR_ERR_UNSUPPORTED;
    }
    if (info->n != mhr_pruner_param_count(info->dim, info->hidden) || info->n == 0 ||
        f.size() != kPrunerHeader + 3 * info->n * 4) {
        set_error("pruner checkpoint: size does not match its dimensions");
        return MHR_ERR_CORRUPT;
    }
    if (crc32_update(0, f.data() + kPrunerHeader, f.size() - kPrunerHeader) != pcrc) {
        set_error("pruner checkpoint: payload checksum mismatch");
        return MHR_ERR_CORRUPT;
    }
    return MHR_OK;
}

// ---------------------------------------------------------------------------
// tuning cache: a sequence of 96-byte records
//   key    device architecture name (char[32], zero padded), num_vertices,
//          num_relations, num_pairs (u64), dim, dtype, scorer, nq, k_max
//   value  tile_edges, hash_log2, grid_blocks, ms per call (float)
//   crc    CRC-32 of the record's first 92 bytes
// ---------------------------------------------------------------------------
struct TuneRecord {
    char arch[32];
    uint32_t n, R;
    uint64_t pairs;
    uint32_t dim, dtype, scorer, nq, kmax;
    uint32_t tile_edges, hash_log2, grid_blocks;
    float ms;
    uint32_t reserved[2];
    uint32_t crc;
};
static_assert(sizeof(TuneRecord) == 96, "tuning record layout");

bool same_key(const TuneRecord &a, const TuneRecord &b) {
    return std::memcmp(a.arch, b.arch, sizeof(a.arch)) == 0 && a.n == b.n && a.R == b.R && a.pairs == b.pairs &&
           a.dim == b.dim && a.dtype == b.dtype && a.scorer == b.scorer && a.nq == b.nq && a.kmax == b.kmax;
}

mhr_status parse_tuning_file(const std::vector<unsigned char> &f, std::vector<TuneRecord> *recs) {
    if (f.size() % sizeof(TuneRecord) != 0) {
        set_error("tuning cache: size is not a whole number of records");
        return MHR_ERR_CORRUPT;
    }
    recs->resize(f.size() / sizeof(TuneRecord));
    if (!f.empty()) std::memcpy(recs->data(), f.data(), f.size());
    for (size_t i = 0; i < recs->size(); ++i) {
        const TuneRecord &r = (*recs)[i];
        if (crc32_update(0, &r, offsetof(TuneRecord, crc)) != r.crc) {
            set_error("tuning cache: checksum mismatch in record " + std::to_string(i));
            return MHR_ERR_CORRUPT;
        }
    }
    return MHR_OK;
}

mhr_status tuning_key(const mhr_graph *g, uint32_t nq, uint32_t kmax, TuneRecord *r) {
    std::memset(r, 0, sizeof(*r));
    hipDeviceProp_t prop;
    MHR_HIP_TRY(hipGetDeviceProperties(&prop, g->device));
    std::strncpy(r->arch, prop.gcnArchName, sizeof(r->arch) - 1);
    r->n = g->n;
    r->R = g->R;
    r->pairs = g->num_pairs;
    r->dim = g->dim;
    r->dtype = static_cast<uint32_t>(g->dtype);
    r->scorer = static_cast<uint32_t>(g->scorer);
    r->nq = nq;
    r->kmax = kmax;
    return MHR_OK;
}

}  // namespace
}  // namespace mhr

using namespace mhr;

extern "C" uint32_t mhr_crc32(uint32_t crc, const void *data, size_t n) { return crc32_update(crc, data, n); }

extern "C" mhr_status mhr_pruner_file_info(const char *path, uint32_t *dim, uint32_t *hidden, uint32_t *step) {
    MHR_ARG_CHECK(path != nullptr, "mhr_pruner_file_info: null path");
    std::vector<unsigned char> f;
    if (!read_file(path, f)) {
        set_error(std::string("cannot read ") + path);
        return MHR_ERR_IO;
    }
    PrunerFileInfo info{};
    const mhr_status rc = parse_pruner_file(f, &info);
    if (rc != MHR_OK) return rc;
    if (dim) *dim = info.dim;
    if (hidden) *hidden = info.hidden;
    if (step) *step = info.step;
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_save(const mhr_pruner *p, const char *path, void *stream) {
    MHR_ARG_CHECK(p != nullptr && path != nullptr, "mhr_pruner_save: null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = p->np;
    std::vector<unsigned char> f(kPrunerHeader + 3 * n * 4);
    unsigned char *pay = f.data() + kPrunerHeader;
    MHR_HIP_TRY(hipMemcpyAsync(pay, p->theta, n * 4, hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipMemcpyAsync(pay + n * 4, p->m, n * 4, hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipMemcpyAsync(pay + 2 * n * 4, p->v, n * 4, hipMemcpyDeviceToHost, st));
    MHR_HIP_TRY(hipStreamSynchronize(st));
    const uint64_t n64 = n;
    std::memcpy(f.data(), kPrunerMagic, 8);
    std::memcpy(f.data() + 8, &kPrunerVersion, 4);
    std::memcpy(f.data() + 12, &p->d, 4);
    std::memcpy(f.data() + 16, &p->H, 4);
    std::memcpy(f.data() + 20, &p->step, 4);
    std::memcpy(f.data() + 24, &n64, 8);
    const uint32_t pcrc = crc32_update(0, pay, 3 * n * 4);
    std::memcpy(f.data() + 32, &pcrc, 4);
    const uint32_t hcrc = crc32_update(0, f.data(), 36);
    std::memcpy(f.data() + 36, &hcrc, 4);
    if (!write_file_atomic(path, f)) {
        set_error(std::string("cannot write ") + path);
        return MHR_ERR_IO;
    }
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_load(mhr_pruner *p, const char *path, void *stream) {
    MHR_ARG_CHECK(p != nullptr && path != nullptr, "mhr_pruner_load: null argument");
    std::vector<unsigned char> f;
    if (!read_file(path, f)) {
        set_error(std::string("cannot read ") + path);
        return MHR_ERR_IO;
    }
    PrunerFileInfo info{};
    mhr_status rc = parse_pruner_file(f, &info);
    if (rc != MHR_OK) return rc;
    if (info.dim != p->d || info.hidden != p->H) {
        set_error("mhr_pruner_load: the checkpoint's dimensions differ from the pruner's");
        return MHR_ERR_INVALID_ARGUMENT;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = p->np;
    const unsigned char *pay = f.data() + kPrunerHeader;
    MHR_HIP_TRY(hipMemcpyAsync(p->theta, pay, n * 4, hipMemcpyHostToDevice, st));
    MHR_HIP_TRY(hipMemcpyAsync(p->m, pay + n * 4, n * 4, hipMemcpyHostToDevice, st));
    MHR_HIP_TRY(hipMemcpyAsync(p->v, pay + 2 * n * 4, n * 4, hipMemcpyHostToDevice, st));
    p->step = info.step;
    MHR_HIP_TRY(pruner_refresh_bf16(p, st));
    MHR_HIP_TRY(hipStreamSynchronize(st));   // the host buffer is released on return
    return MHR_OK;
}

extern "C" mhr_status mhr_tuning_file_records(const char *path, uint32_t *count) {
    MHR_ARG_CHECK(path != nullptr && count != nullptr, "mhr_tuning_file_records: null argument");
    std::vector<unsigned char> f;
    if (!read_file(path, f)) {
        set_error(std::string("cannot read ") + path);
        return MHR_ERR_IO;
    }
    std::vector<TuneRecord> recs;
    const mhr_status rc = parse_tuning_file(f, &recs);
    if (rc != MHR_OK) return rc;
    *count = static_cast<uint32_t>(recs.size());
    return MHR_OK;
}

extern "C" mhr_status mhr_tuning_save(const char *path, const mhr_graph *g, uint32_t nq, uint32_t k_max,
                                      const mhr_query_opts *tuned, float ms) {
    MHR_ARG_CHECK(path && g && tuned, "mhr_tuning_save: null argument");
    std::vector<TuneRecord> recs;
    std::vector<unsigned char> f;
    if (read_file(path, f)) {
        const mhr_status rc = parse_tuning_file(f, &recs);
        if (rc != MHR_OK) return rc;   // never overwrite a damaged cache silently
    }
    TuneRecord r;
    mhr_status rc = tuning_key(g, nq, k_max, &r);
    if (rc != MHR_OK) return rc;
    r.tile_edges = tuned->tile_edges;
    r.hash_log2 = tuned->hash_log2;
    r.grid_blocks = tuned->grid_blocks;
    r.ms = ms;
    r.crc = crc32_update(0, &r, offsetof(TuneRecord, crc));
    bool replaced = false;
    for (TuneRecord &x : recs)
        if (same_key(x, r)) {
            x = r;
            replaced = true;
        }
    if (!replaced) recs.push_back(r);
    f.resize(recs.size() * sizeof(TuneRecord));
    std::memcpy(f.data(), recs.data(), f.size());
    if (!write_file_atomic(path, f)) {
        set_error(std::string("cannot write ") + path);
        return MHR_ERR_IO;
    }
    return MHR_OK;
}

extern "C" mhr_status mhr_tuning_load(const char *path, const mhr_graph *g, uint32_t nq, uint32_t k_max,
                                      mhr_query_opts *tuned, float *ms) {
    MHR_ARG_CHECK(path && g && tuned, "mhr_tuning_load: null argument");
    std::vector<unsigned char> f;
    if (!read_file(path, f)) {
        set_error(std::string("cannot read ") + path);
        return MHR_ERR_IO;
    }
    std::vector<TuneRecord> recs;
    mhr_status rc = parse_tuning_file(f, &recs);
    if (rc != MHR_OK) return rc;
    TuneRecord key;
    rc = tuning_key(g, nq, k_max, &key);
    if (rc != MHR_OK) return rc;
    for (const TuneRecord &x : recs) {
        if (!same_key(x, key)) continue;
        mhr_query_opts o{};
        o.tile_edges = x.tile_edges;
        o.hash_log2 = x.hash_log2;
        o.grid_blocks = x.grid_blocks;
        *tuned = o;
        if (ms) *ms = x.ms;
        return MHR_OK;
    }
    set_error("mhr_tuning_load: no record for this device, graph, batch size and k_max");
    return MHR_ERR_NOT_FOUND;
}
