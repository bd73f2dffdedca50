// Learned frontier pruner: a small MLP that scores the first-hop candidates
// (s, r1, a) and second-hop candidates (b, r3, t) of a query, trained on
// labels from the exact search.  Its input is f = [X[u], X[w], X[v], Y[r]]
// with u the query endpoint the candidate edge touches (s, or t for the
// second hop), w the other endpoint, v the candidate vertex and r the
// edge's relation: the same functional form for both hops, as the DistMult
// weight w(b, r3, t) = w(t, r3, b) is symmetric.
//
//   h1 = relu(W1 f + b1),  h2 = relu(W2 h1 + b2),  z = w3 . h2 + b3
//
// Matrix products run on the matrix cores (v_mfma_f32_16x16x32_bf16:
// bfloat16 operands, FP32 accumulation); FP32 master weights and Adam.  The
// operands rounded to bfloat16 are the features, W1, W2, w3, h1, h2 and the
// back-propagated dz2, dz1; everything else is FP32.
#include <hip/hip_runtime.h>

#include <string>

#include "mhr.h"
#include "mhr_device.h"
#include <algorithm>
#include <vector>

#include "mhr_internal.h"
#include "mhr_pruner_internal.h"



namespace mhr {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kGemmThreads = 256;
constexpr int kBlock = 512;   // workgroup size of the reduction and candidate kernels
constexpr int BM = 64, BN = 64, BK = 32, BKP = BK + 8;

// Parameter offsets in the flat vector W1 [H][4d], b1, W2 [H][H], b2, w3, b3.
struct PLayout {
    size_t W1, b1, W2, b2, w3, b3, n;
};
__host__ __device__ inline PLayout play(uint32_t d, uint32_t H) {
    PLayout L{};
    size_t o = 0;
    L.W1 = o; o += size_t(H) * 4 * d;
    L.b1 = o; o += H;
    L.W2 = o; o += size_t(H) * H;
    L.b2 = o; o += H;
    L.w3 = o; o += H;
    L.b3 = o; o += 1;
    L.n = o;
    return L;
}

__device__ __forceinline__ uint16_t to_bf16(float x) {   // round to nearest even (finite x)
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return static_cast<uint16_t>(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// A matrix operand: up to four column segments, each a table whose rows may
// be gathered through an index array.  Element (row, col) lies in segment
// g = col / seg at table row idx[g][row] (or row), column col - g * seg.
// lim[g] (when nonzero) bounds the gathered row ids of segment g: a row id
// at or above it reads as zeros.
struct Mat {
    const void *p[4];
    const uint32_t *idx[4];
    uint32_t lim[4];
    uint32_t seg, ld, nseg, f32, vec;   // vec: 8-column chunks may load as one 16-byte vector
};

__device__ __forceinline__ uint16_t mat_elem(const Mat &M, uint32_t row, uint32_t col) {
    const uint32_t g = col / M.seg, c = col - g * M.seg;
    const uint32_t r = M.idx[g] ? M.idx[g][row] : row;
    if (M.lim[g] && r >= M.lim[g]) return 0;
    const size_t o = static_cast<size_t>(r) * M.ld + c;
    return M.f32 ? to_bf16(static_cast<const float *>(M.p[g])[o]) : static_cast<const uint16_t *>(M.p[g])[o];
}

// Eight consecutive columns [col, col + 8) of one row into dst (zero outside
// [0, nrows) x [0, cend)).
__device__ __forceinline__ void mat_row8(const Mat &M, uint32_t row, uint32_t col, uint32_t nrows, uint32_t cend,
                                         uint16_t *dst) {
    if (row >= nrows) {
#pragma unroll
        for (int e = 0; e < 8; ++e) dst[e] = 0;
        return;
    }
    if (M.vec && col + 8 <= cend) {
        const uint32_t g = col / M.seg, c = col - g * M.seg;
        const uint32_t r = M.idx[g] ? M.idx[g][row] : row;
        if (M.lim[g] && r >= M.lim[g]) {
#pragma unroll
            for (int e = 0; e < 8; ++e) dst[e] = 0;
            return;
        }
        const size_t o = static_cast<size_t>(r) * M.ld + c;
        if (M.f32) {
            const float4 a = *reinterpret_cast<const float4 *>(static_cast<const float *>(M.p[g]) + o);
            const float4 b = *reinterpret_cast<const float4 *>(static_cast<const float *>(M.p[g]) + o + 4);
            dst[0] = to_bf16(a.x); dst[1] = to_bf16(a.y); dst[2] = to_bf16(a.z); dst[3] = to_bf16(a.w);
            dst[4] = to_bf16(b.x); dst[5] = to_bf16(b.y); dst[6] = to_bf16(b.z); dst[7] = to_bf16(b.w);
        } else {
            *reinterpret_cast<uint4 *>(dst) = *reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(M.p[g]) + o);
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[e] = (col + e < cend) ? mat_elem(M, row, col + e) : uint16_t(0);
}

// C[M][N] = sum_k opA(m, k) opB(k, n) over k in this block's chunk
// [z * kchunk, (z + 1) * kchunk) of [0, K).
//   opA(m, k) = TA ? A(k, m) : A(m, k)      opB(k, n) = TB ? B(n, k) : B(k, n)
// Block tile 64 x 64, four waves of 32 x 32 (2 x 2 MFMA tiles of 16 x 16),
// 32 k per step staged in LDS with k contiguous.  part != nullptr (split K):
// the block stores its chunk's sum in part[z][M][N] and a second kernel adds
// the chunks in order, so the result does not depend on block timing; else
// the block stores C.
template <bool TA, bool TB>
__global__ __launch_bounds__(kGemmThreads) void gemm_kernel(Mat A, Mat B, float *C, uint32_t ldc, uint32_t M,
                                                            uint32_t N, uint32_t K, uint32_t kchunk, float *part) {
    __shared__ __align__(16) uint16_t As[BM][BKP];
    __shared__ __align__(16) uint16_t Bs[BN][BKP];
    const uint32_t m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const uint32_t kbeg = blockIdx.z * kchunk;
    const uint32_t kend = min(K, kbeg + kchunk);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    for (uint32_t k0 = kbeg; k0 < kend; k0 += BK) {
        if (!TA) {   // A rows are m, contiguous along k
            const int r = tid >> 2, c = (tid & 3) * 8;
            mat_row8(A, m0 + r, k0 + c, M, kend, &As[r][c]);
        } else {     // A rows are k, contiguous along m
            const int kk = tid >> 3, c = (tid & 7) * 8;
            const uint32_t k = k0 + kk;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t m = m0 + c + e;
                As[c + e][kk] = (m < M && k < kend) ? mat_elem(A, k, m) : uint16_t(0);
            }
        }
        if (TB) {    // B rows are n, contiguous along k
            const int r = tid >> 2, c = (tid & 3) * 8;
            mat_row8(B, n0 + r, k0 + c, N, kend, &Bs[r][c]);
        } else {     // B rows are k, contiguous along n
            const int kk = tid >> 3, c = (tid & 7) * 8;
            const uint32_t k = k0 + kk;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint32_t n = n0 + c + e;
                Bs[c + e][kk] = (n < N && k < kend) ? mat_elem(B, k, n) : uint16_t(0);
            }
        }
        __syncthreads();
        // lane (row = lane & 15, group g = lane >> 4) supplies k = 8g .. 8g + 7
        const int row = lane & 15, g = lane >> 4;
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[wm + 16 * i + row][8 * g]);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[wn + 16 * j + row][8 * g]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // D[row][col] of a 16 x 16 tile sits in lane col + 16 * (row / 4), element row % 4
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const uint32_t m = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
                const uint32_t n = n0 + wn + 16 * j + (lane & 15);
                if (m < M && n < N) {
                    if (part) part[(static_cast<size_t>(blockIdx.z) * M + m) * N + n] = acc[i][j][e];
                    else C[static_cast<size_t>(m) * ldc + n] = acc[i][j][e];
                }
            }
}

// ---- forward products: C[m][n] = sum_k A(m, k) B(n, k) -----------------------
//
// Both operands are rows contiguous along k (A: gathered feature or
// activation rows; B: a weight matrix [N][K] read as stored).  Block tile
// 128 x 128, four waves of 64 x 64 (4 x 4 MFMA tiles of 16 x 16), 32 k per
// step.  The next step's tiles are loaded into registers while the current
// one is multiplied out of LDS, and written to the other of two LDS buffers,
// so one barrier separates the steps.  The epilogue is fused:
//   kEpiF32        C[m][n] = acc                      (FP32 out, ldc)
//   kEpiBiasRelu   h[m][n] = bf16(relu(((acc + T1[i1(m)][n]) + T2[i2(m)][n]) + bias[n]))
//                  (the T terms only when given; the hoisted first layer)
//   kEpiBiasReluDot as kEpiBiasRelu, h optional, and zpart[blockIdx.x][m] =
//                  the tile's sum over n of h[m][n] w3[n] (the output layer)
constexpr int kNtM = 128, kNtN = 128, kNtK = 32, kNtKP = kNtK + 8, kNtThreads = 256;
enum NtEpi { kEpiF32 = 0, kEpiBiasRelu = 1, kEpiBiasReluDot = 2 };

struct NtEpilogue {
    float *C;                 // kEpiF32
    uint32_t ldc;
    uint16_t *h;              // bf16 activations [M][N] (may be null for kEpiBiasReluDot)
    const float *bias;        // [N]
    const float *T1;          // [*][N] rows added before the bias (or null), row T1i(m)
    const uint32_t *q1;       // per row m: query word (query index | hop flag); T1 row = 2 query + hop
    uint32_t t1_queries;      // queries of T1 (a query index at or above it reads row 0)
    const float *T2;          // [*][N] (or null), row r2[m]
    const uint32_t *r2;
    uint32_t t2_rows;         // rows of T2 (an id at or above it reads row 0)
    const uint16_t *w3;       // bf16 [N] (kEpiBiasReluDot)
    float *zpart;             // [gridDim.x][M]
};

constexpr uint32_t kHopFlag = 0x80000000u;   // second-hop flag of a sample's query word

template <int EPI>
__global__ __launch_bounds__(kNtThreads) void gemm_nt_kernel(Mat A, Mat B, uint32_t M, uint32_t N, uint32_t K,
                                                             NtEpilogue E) {
    __shared__ __align__(16) uint16_t As[2][kNtM][kNtKP];
    __shared__ __align__(16) uint16_t Bs[2][kNtN][kNtKP];
    __shared__ float zred[2][kNtM];
    const uint32_t m0 = blockIdx.y * kNtM, n0 = blockIdx.x * kNtN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
    // loader: thread t fills rows t / 4 and t / 4 + 64, k columns 8 (t % 4) .. + 8
    const int lr = tid >> 2, lc = (tid & 3) * 8;
    uint4 ra[2], rb[2];
    auto load = [&](uint32_t k0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            mat_row8(A, m0 + lr + 64 * h, k0 + lc, M, K, reinterpret_cast<uint16_t *>(&ra[h]));
            mat_row8(B, n0 + lr + 64 * h, k0 + lc, N, K, reinterpret_cast<uint16_t *>(&rb[h]));
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            *reinterpret_cast<uint4 *>(&As[buf][lr + 64 * h][lc]) = ra[h];
            *reinterpret_cast<uint4 *>(&Bs[buf][lr + 64 * h][lc]) = rb[h];
        }
    };
    f4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    load(0);
    store(0);
    __syncthreads();
    const int row = lane & 15, g = lane >> 4;
    int buf = 0;
    for (uint32_t k0 = 0; k0 < K; k0 += kNtK) {
        const bool more = k0 + kNtK < K;
        if (more) load(k0 + kNtK);
        bf16x8 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const bf16x8 *>(&As[buf][wm + 16 * i + row][8 * g]);
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const bf16x8 *>(&Bs[buf][wn + 16 * j + row][8 * g]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // D[row][col] of a 16 x 16 tile sits in lane col + 16 * (row / 4), element row % 4
    float zp[4][4];   // kEpiBiasReluDot: per (i, e) this lane's share of the tile's output dot
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) zp[i][e] = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t m = m0 + wm + 16 * i + 4 * g + e;
            if (m >= M) continue;
            const float *t1 = nullptr, *t2 = nullptr;
            if (EPI != kEpiF32) {
                // out-of-range ids read row 0 (the logit is then replaced by
                // NaN: zpart_reduce_kernel)
                if (E.T1) {
                    const uint32_t w = E.q1[m], qq = w & ~kHopFlag;
                    t1 = E.T1 + (2 * static_cast<size_t>(qq >= E.t1_queries ? 0 : qq) + ((w & kHopFlag) ? 1 : 0)) * N;
                }
                if (E.T2) {
                    const uint32_t rr = E.r2[m];
                    t2 = E.T2 + static_cast<size_t>(rr >= E.t2_rows ? 0 : rr) * N;
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t n = n0 + wn + 16 * j + row;
                if (n >= N) continue;
                const float x = acc[i][j][e];
                if (EPI == kEpiF32) {
                    E.C[static_cast<size_t>(m) * E.ldc + n] = x;
                } else {
                    float zv = x;
                    if (t1) zv += t1[n];
                    if (t2) zv += t2[n];
                    const uint16_t hb = to_bf16(fmaxf(zv + E.bias[n], 0.0f));
                    if (E.h) E.h[static_cast<size_t>(m) * N + n] = hb;
                    if (EPI == kEpiBiasReluDot) zp[i][e] += from_bf16(hb) * from_bf16(E.w3[n]);
                }
            }
        }
    if (EPI == kEpiBiasReluDot) {
        // sum over the 16 lanes holding one row's columns, then over the two
        // waves of the row (fixed order)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float v = zp[i][e];
#pragma unroll
                for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o, 64);
                if (row == 0) zred[wave & 1][wm + 16 * i + 4 * g + e] = v;
            }
        __syncthreads();
        for (int r = tid; r < kNtM; r += kNtThreads) {
            const uint32_t m = m0 + r;
            if (m < M) E.zpart[static_cast<size_t>(blockIdx.x) * M + m] = zred[0][r] + zred[1][r];
        }
    }
}

// z[m] = (sum over the column blocks b = 0, 1, ... of zpart[b][m]) + b3;
// NaN for a sample whose query index (q, when given) is not below nq or
// whose relation (r, when given) is not below R.
__global__ void zpart_reduce_kernel(const float *zpart, uint32_t nb, uint32_t M, const float *b3, float *z,
                                    const uint32_t *q, uint32_t nq, const uint32_t *r, uint32_t R) {
    for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < M; m += gridDim.x * blockDim.x) {
        float acc = 0.0f;
        for (uint32_t b = 0; b < nb; ++b) acc += zpart[static_cast<size_t>(b) * M + m];
        const bool bad = (q && (q[m] & ~kHopFlag) >= nq) || (r && r[m] >= R);
        z[m] = bad ? __builtin_nanf("") : acc + b3[0];
    }
}

// ---- elementwise and reduction kernels -------------------------------------
//
// Every reduction over samples sums per-block partials in a fixed order (no
// floating-point atomics), so a training step is a deterministic function of
// its inputs and a resumed run repeats the uninterrupted one bit for bit.

// C[m][n] = sum over z = 0, 1, ... of part[z][m][n]
__global__ void splitk_reduce_kernel(const float *part, uint32_t splits, uint32_t M, uint32_t N, float *C,
                                     uint32_t ldc) {
    const size_t MN = size_t(M) * N;
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < MN; i += size_t(gridDim.x) * blockDim.x) {
        float acc = 0.0f;
        for (uint32_t z = 0; z < splits; ++z) acc += part[z * MN + i];
        C[(i / N) * ldc + i % N] = acc;
    }
}

__global__ void fill_kernel(float *p, size_t n, float v) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) p[i] = v;
}

__global__ void to_bf16_kernel(const float *src, uint16_t *dst, size_t n) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        dst[i] = to_bf16(src[i]);
}

constexpr uint32_t kHop2 = 0x80000000u;   // second-hop flag in a sample's query word

// Per sample, the query endpoint its candidate edge touches (s for the first
// hop, t for the second) and the other endpoint: the first two feature slots.
__global__ void expand_query_kernel(const uint32_t *q, const uint32_t *src, const uint32_t *dst, uint32_t *s,
                                    uint32_t *t, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t w = q[i], qq = w & ~kHop2;
        const bool hop2 = (w & kHop2) != 0;
        s[i] = hop2 ? dst[qq] : src[qq];
        t[i] = hop2 ? src[qq] : dst[qq];
    }
}

// h = bfloat16(relu(Z + b)), row-major [n][H]
__global__ void bias_relu_kernel(const float *Z, const float *b, uint16_t *h, size_t total, uint32_t H) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x)
        h[i] = to_bf16(fmaxf(Z[i] + b[i % H], 0.0f));
}

// z_i = w3 . h2_i + b3, one wave per row
__global__ void output_kernel(const uint16_t *h2, const uint16_t *w3b, const float *b3, float *z, uint32_t n,
                              uint32_t H) {
    const uint32_t lane = threadIdx.x & (kWave - 1);
    const uint32_t row = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    if (row >= n) return;
    float acc = 0.0f;
    for (uint32_t j = lane; j < H; j += kWave)
        acc += from_bf16(h2[static_cast<size_t>(row) * H + j]) * from_bf16(w3b[j]);
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (lane == 0) z[row] = acc + b3[0];
}

// dz_i = (w y (p - 1) + (1 - y) p) / n, and this block's share of the mean
// loss in lpart[block]
__global__ void bce_kernel(const float *z, const float *y, uint32_t n, float w_pos, float *dz, float *lpart) {
    __shared__ float red[kBlock / kWave];
    float part = 0.0f;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float zi = z[i], yi = y[i];
        const float e = expf(-fabsf(zi));
        const float l1p = log1pf(e);
        const float p = zi >= 0.0f ? 1.0f / (1.0f + e) : e / (1.0f + e);
        const float logp = fminf(zi, 0.0f) - l1p;        // log sigmoid(z)
        const float log1mp = fminf(-zi, 0.0f) - l1p;     // log sigmoid(-z)
        dz[i] = (w_pos * yi * (p - 1.0f) + (1.0f - yi) * p) / static_cast<float>(n);
        part -= (w_pos * yi * logp + (1.0f - yi) * log1mp);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) s += red[w];
        lpart[blockIdx.x] = s / static_cast<float>(n);
    }
}

// part[y][j] = sum_i scale_i * M[i][j] (scale = nullptr: 1) over the rows of
// chunk y
__global__ void colsum_kernel(const uint16_t *Mv, const float *scale, float *part, uint32_t n, uint32_t H,
                              uint32_t rows_per_block) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= H) return;
    const uint32_t r0 = blockIdx.y * rows_per_block, r1 = min(n, r0 + rows_per_block);
    float acc = 0.0f;
    for (uint32_t i = r0; i < r1; ++i) acc += (scale ? scale[i] : 1.0f) * from_bf16(Mv[static_cast<size_t>(i) * H + j]);
    part[static_cast<size_t>(blockIdx.y) * H + j] = acc;
}

// out[j] = sum over y = 0, 1, ... of part[y][j]
__global__ void colsum_reduce_kernel(const float *part, uint32_t chunks, uint32_t H, float *out) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= H) return;
    float acc = 0.0f;
    for (uint32_t y = 0; y < chunks; ++y) acc += part[static_cast<size_t>(y) * H + j];
    out[j] = acc;
}

// *out = sum of x[0 .. n), one block: per-thread strided sums, then a fixed
// tree over the block
__global__ void sum_kernel(const float *x, uint32_t n, float *out) {
    __shared__ float red[kBlock / kWave];
    float part = 0.0f;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) part += x[i];
    for (int o = kWave / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane == 0) red[wave] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.0f;
        for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) s += red[w];
        *out = s;
    }
}

// dz2 = bfloat16(dz_i w3_j [h2_ij > 0]), in place over h2
__global__ void dz2_kernel(const float *dz, const uint16_t *w3b, uint16_t *h2, size_t total, uint32_t H) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x) {
        const float h = from_bf16(h2[i]);
        h2[i] = h > 0.0f ? to_bf16(dz[i / H] * from_bf16(w3b[i % H])) : uint16_t(0);
    }
}

// dz1 = bfloat16(dH1 [h1 > 0]), in place over h1
__global__ void dz1_kernel(const float *dH1, uint16_t *h1, size_t total) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < total; i += size_t(gridDim.x) * blockDim.x) {
        const float h = from_bf16(h1[i]);
        h1[i] = h > 0.0f ? to_bf16(dH1[i]) : uint16_t(0);
    }
}

__global__ void adam_kernel(float *theta, const float *g, float *m, float *v, size_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        theta[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// ---- host helpers ------------------------------------------------------------

inline uint32_t grid_for(size_t n, uint32_t block = 256) {
    size_t g = (n + block - 1) / block;
    return static_cast<uint32_t>(g < 1 ? 1 : (g > 65535 ? 65535 : g));
}

Mat plain(const void *p, uint32_t cols, bool f32 = false) {
    Mat M{};
    M.p[0] = p;
    M.seg = cols;
    M.ld = cols;
    M.nseg = 1;
    M.f32 = f32 ? 1u : 0u;
    M.vec = (cols % 8 == 0) ? 1u : 0u;
    return M;
}

// The feature rows [X[s_i], X[t_i], X[v_i], Y[r_i]] of n samples.
Mat features(const mhr_graph *g, const uint32_t *s, const uint32_t *t, const uint32_t *v, const uint32_t *r) {
    Mat F{};
    F.p[0] = g->X; F.idx[0] = s;
    F.p[1] = g->X; F.idx[1] = t;
    F.p[2] = g->X; F.idx[2] = v;
    F.p[3] = g->Y; F.idx[3] = r;
    F.lim[0] = F.lim[1] = F.lim[2] = g->n;
    F.lim[3] = g->R;
    F.seg = g->dim;
    F.ld = g->dim;
    F.nseg = 4;
    F.f32 = g->dtype == MHR_DTYPE_F32 ? 1u : 0u;
    F.vec = (g->dim % 8 == 0) ? 1u : 0u;
    return F;
}

// K chunk (a multiple of BK) and chunk count for a requested split count
struct Split {
    uint32_t kchunk, splits;
};
Split split_k(uint32_t K, uint32_t splits) {
    if (splits < 1) splits = 1;
    uint32_t kchunk = (K + splits - 1) / splits;
    kchunk = (kchunk + BK - 1) / BK * BK;
    if (kchunk == 0) kchunk = BK;
    splits = (K + kchunk - 1) / kchunk;
    return {kchunk, splits < 1 ? 1u : splits};
}

// part: split-K staging of at least splits * M * N floats (unused for one
// split)
template <bool TA, bool TB>
hipError_t gemm(const Mat &A, const Mat &B, float *C, uint32_t ldc, uint32_t M, uint32_t N, uint32_t K,
                uint32_t splits, float *part, hipStream_t st) {
    if (M == 0 || N == 0) return hipSuccess;
    const Split sp = split_k(K, splits);
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, sp.splits);
    float *pp = sp.splits > 1 ? part : nullptr;
    hipLaunchKernelGGL((gemm_kernel<TA, TB>), grid, dim3(kGemmThreads), 0, st, A, B, C, ldc, M, N, K, sp.kchunk, pp);
    if (pp) hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for(size_t(M) * N)), dim3(256), 0, st, pp, sp.splits,
                               M, N, C, ldc);
    return hipGetLastError();
}

template <int EPI>
hipError_t gemm_nt(const Mat &A, const Mat &B, uint32_t M, uint32_t N, uint32_t K, const NtEpilogue &E,
                   hipStream_t st) {
    if (M == 0 || N == 0) return hipSuccess;
    if ((M + kNtM - 1) / kNtM > 65535u) return hipErrorInvalidValue;
    dim3 grid((N + kNtN - 1) / kNtN, (M + kNtM - 1) / kNtM);
    hipLaunchKernelGGL((gemm_nt_kernel<EPI>), grid, dim3(kNtThreads), 0, st, A, B, M, N, K, E);
    return hipGetLastError();
}

// split count for a reduction over K samples into an M x N output
uint32_t splits_for(uint32_t M, uint32_t N, uint32_t K) {
    const uint32_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    uint32_t s = (1024 + tiles - 1) / tiles;
    const uint32_t kmax = (K + 255) / 256;   // at least 256 samples per split
    if (s > kmax) s = kmax;
    return s < 1 ? 1 : s;
}

// floats of split-K staging for an M x N weight gradient over K samples
size_t split_floats(uint32_t M, uint32_t N, uint32_t K) {
    const Split sp = split_k(K, splits_for(M, N, K));
    return sp.splits > 1 ? size_t(sp.splits) * M * N : 0;
}

constexpr uint32_t kColRows = 256;   // rows per column-sum chunk

struct PWs {
    size_t Z, h1, h2, z, dz, s, t, part, cpart, lpart, zpart, total;
};
PWs pws_layout(uint32_t n, uint32_t d, uint32_t H) {
    PWs L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = (o + bytes + 255) & ~size_t(255); return r; };
    L.Z = take(size_t(n) * H * 4);
    L.h1 = take(size_t(n) * H * 2);
    L.h2 = take(size_t(n) * H * 2);
    L.z = take(size_t(n) * 4);
    L.dz = take(size_t(n) * 4);
    L.s = take(size_t(n) * 4);
    L.t = take(size_t(n) * 4);
    L.part = take(std::max(split_floats(H, H, n), split_floats(H, 4 * d, n)) * 4);
    L.cpart = take(size_t((n + kColRows - 1) / kColRows) * H * 4);
    L.lpart = take(size_t(grid_for(n, kBlock)) * 4);
    L.zpart = take(size_t((H + kNtN - 1) / kNtN) * n * 4);
    L.total = o;
    return L;
}

hipError_t refresh_bf16(mhr_pruner *p, hipStream_t st) {
    const PLayout L = play(p->d, p->H);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(L.b1 - L.W1)), dim3(256), 0, st, p->theta + L.W1, p->W1b,
                       L.b1 - L.W1);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(L.b2 - L.W2)), dim3(256), 0, st, p->theta + L.W2, p->W2b,
                       L.b2 - L.W2);
    hipLaunchKernelGGL(to_bf16_kernel, dim3(1), dim3(256), 0, st, p->theta + L.w3, p->w3b, size_t(p->H));
    return hipGetLastError();
}

// forward pass over n samples; leaves Z1 / h1 / h2 / z in the workspace
mhr_status forward_impl(mhr_pruner *p, const mhr_graph *g, uint32_t n, const uint32_t *q, const uint32_t *src,
                        const uint32_t *dst, const uint32_t *v, const uint32_t *r, char *ws, hipStream_t st) {
    const PWs W = pws_layout(n, p->d, p->H);
    const PLayout L = play(p->d, p->H);
    const uint32_t H = p->H, d = p->d;
    float *Z = reinterpret_cast<float *>(ws + W.Z);
    uint16_t *h1 = reinterpret_cast<uint16_t *>(ws + W.h1), *h2 = reinterpret_cast<uint16_t *>(ws + W.h2);
    uint32_t *s = reinterpret_cast<uint32_t *>(ws + W.s), *t = reinterpret_cast<uint32_t *>(ws + W.t);
    (void)Z;
    hipLaunchKernelGGL(expand_query_kernel, dim3(grid_for(n)), dim3(256), 0, st, q, src, dst, s, t, n);
    const Mat F = features(g, s, t, v, r);
    NtEpilogue E1{};
    E1.h = h1;
    E1.bias = p->theta + L.b1;
    MHR_HIP_TRY(gemm_nt<kEpiBiasRelu>(F, plain(p->W1b, 4 * d), n, H, 4 * d, E1, st));
    NtEpilogue E2{};
    E2.h = h2;
    E2.bias = p->theta + L.b2;
    E2.w3 = p->w3b;
    E2.zpart = reinterpret_cast<float *>(ws + W.zpart);
    MHR_HIP_TRY(gemm_nt<kEpiBiasReluDot>(plain(h1, H), plain(p->W2b, H), n, H, H, E2, st));
    hipLaunchKernelGGL(zpart_reduce_kernel, dim3(grid_for(n)), dim3(256), 0, st, E2.zpart, (H + kNtN - 1) / kNtN, n,
                       p->theta + L.b3, reinterpret_cast<float *>(ws + W.z), static_cast<const uint32_t *>(nullptr),
                       0u, static_cast<const uint32_t *>(nullptr), 0u);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

// ---- candidates ----------------------------------------------------------------

// Per query: entries (deg+(s) + deg-(t)) and candidates (relations over both
// rows); then exclusive offsets over the queries, totals at [nq].
__global__ void cand_count_kernel(const uint32_t *out_rp, const uint32_t *out_mask, const uint32_t *in_rp,
                                  const uint32_t *in_mask, uint32_t n, const uint32_t *src, const uint32_t *dst,
                                  uint64_t *entries, uint64_t *cands) {
    __shared__ uint64_t red[kBlock / kWave];
    const uint32_t q = blockIdx.x;
    const uint32_t s = src[q], t = dst[q];
    uint64_t ne = 0, nc = 0;
    if (s < n && t < n) {
        const uint32_t b0 = out_rp[s], b1 = out_rp[s + 1], c0 = in_rp[t], c1 = in_rp[t + 1];
        ne = (b1 - b0) + (c1 - c0);
        uint64_t part = 0;
        for (uint32_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) part += __popc(out_mask[i]);
        for (uint32_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) part += __popc(in_mask[i]);
        for (int o = kWave / 2; o > 0; o >>= 1) part += __shfl_xor(part, o, kWave);
        const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
        if (lane == 0) red[wave] = part;
        __syncthreads();
        for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) nc += red[w];
    }
    if (threadIdx.x == 0) {
        entries[q] = ne;
        cands[q] = nc;
    }
}

// in-place exclusive scan of a[0..n) with the total at a[n] (one workgroup)
__global__ void excl_scan_kernel(uint64_t *a, uint32_t n) {
    __shared__ uint64_t red[kBlock / kWave];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += blockDim.x) {
        const uint32_t i = base + threadIdx.x;
        const uint64_t x = i < n ? a[i] : 0;
        uint64_t v = x;
        const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint64_t y = __shfl_up(v, off, kWave);
            if (lane >= off) v += y;
        }
        if (lane == kWave - 1) red[wave] = v;
        __syncthreads();
        uint64_t before = 0, tot = 0;
        for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) {
            if (w < wave) before += red[w];
            tot += red[w];
        }
        const uint64_t c = carry;
        if (i < n) a[i] = c + before + v - x;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) a[n] = carry;
}

// One workgroup per query: first-hop candidates (entries of s's out-row,
// each relation of the entry's mask in ascending order), then second-hop
// candidates (entries of t's in-row).
__global__ void cand_fill_kernel(const uint32_t *out_rp, const uint32_t *out_col, const uint32_t *out_mask,
                                 const uint32_t *in_rp, const uint32_t *in_col, const uint32_t *in_mask, uint32_t n,
                                 const uint32_t *src, const uint32_t *dst, const uint64_t *entry_off,
                                 const uint64_t *cand_off, uint64_t *cand_split, uint32_t *cq, uint32_t *cv,
                                 uint32_t *cr, uint64_t *ce) {
    __shared__ uint64_t red[kBlock / kWave];
    __shared__ uint64_t carry;
    const uint32_t q = blockIdx.x;
    const uint32_t s = src[q], t = dst[q];
    if (threadIdx.x == 0) carry = cand_off[q];
    __syncthreads();
    if (!(s < n && t < n)) {
        if (threadIdx.x == 0) cand_split[q] = cand_off[q];
        return;
    }
    const uint32_t degs = out_rp[s + 1] - out_rp[s];
    for (int hop = 0; hop < 2; ++hop) {
        const uint32_t beg = hop ? in_rp[t] : out_rp[s], end = hop ? in_rp[t + 1] : out_rp[s + 1];
        const uint32_t *col = hop ? in_col : out_col, *mask = hop ? in_mask : out_mask;
        if (hop == 1 && threadIdx.x == 0) cand_split[q] = carry;
        __syncthreads();
        for (uint32_t base = beg; base < end; base += blockDim.x) {
            const uint32_t i = base + threadIdx.x;
            const uint32_t m = i < end ? mask[i] : 0u;
            const uint64_t x = __popc(m);
            uint64_t v = x;
            const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
            for (int off = 1; off < kWave; off <<= 1) {
                const uint64_t y = __shfl_up(v, off, kWave);
                if (lane >= off) v += y;
            }
            if (lane == kWave - 1) red[wave] = v;
            __syncthreads();
            uint64_t before = 0, tot = 0;
            for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) {
                if (w < wave) before += red[w];
                tot += red[w];
            }
            const uint64_t c = carry;
            if (i < end) {
                uint64_t o = c + before + v - x;
                const uint64_t e = entry_off[q] + (hop ? degs : 0u) + (i - beg);
                for (uint32_t mm = m; mm; mm &= mm - 1) {
                    cq[o] = hop ? (q | kHop2) : q;
                    cv[o] = col[i];
                    cr[o] = static_cast<uint32_t>(__ffs(mm) - 1);
                    ce[o] = e;
                    ++o;
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) carry = c + tot;
            __syncthreads();
        }
    }
}

// order-preserving key of a float score (NaN lowest)
__device__ __forceinline__ uint32_t score_key(float x) {
    if (x != x) return 0u;
    const uint32_t b = __float_as_uint(x);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

template <class T>
__device__ inline T wg_sum(T v, T *red) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) s += red[w];
    return s;
}

// An entry's score: the best score of its candidates (order-preserving key).
__global__ void entry_key_kernel(const float *score, const uint64_t *ce, uint64_t n, uint32_t *key) {
    for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x)
        atomicMax(&key[ce[i]], score_key(score[i]));
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) p[i] = v;
}

// One workgroup per (query, hop): keep the ceil(n * permille / 1000) entries
// (vertices) of the hop with the best entry scores, and every entry tied
// with the lowest kept one.  mass[2q + hop] = sum of sigmoid(score) over the
// candidates of kept entries / over all candidates (1 when there are none).
__global__ void select_kernel(const uint32_t *out_rp, const uint32_t *in_rp, uint32_t n, const uint32_t *src,
                              const uint32_t *dst, const uint64_t *entry_off, const uint64_t *cand_off,
                              const uint64_t *cand_split, const float *score, const uint64_t *ce, const uint32_t *ekey,
                              uint32_t permille, uint8_t *keep, float *mass) {
    __shared__ uint64_t red64[kBlock / kWave];
    __shared__ float redf[kBlock / kWave];
    const uint32_t q = blockIdx.x, hop = blockIdx.y;
    const uint32_t s = src[q], t = dst[q];
    if (!(s < n && t < n)) {
        if (threadIdx.x == 0 && mass) mass[2 * q + hop] = 1.0f;
        return;
    }
    const uint32_t degs = out_rp[s + 1] - out_rp[s], degt = in_rp[t + 1] - in_rp[t];
    const uint64_t e0 = entry_off[q] + (hop ? degs : 0u), ne = hop ? degt : degs;
    if (ne == 0) {
        if (threadIdx.x == 0 && mass) mass[2 * q + hop] = 1.0f;
        return;
    }
    const uint64_t m = (ne * permille + 999) / 1000 > 0 ? (ne * permille + 999) / 1000 : 1;
    // the m-th largest entry key: the largest T with #{key >= T} >= m, bit by bit
    uint32_t T = 0;
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t cand = T | (1u << bit);
        uint64_t cnt = 0;
        for (uint64_t i = threadIdx.x; i < ne; i += blockDim.x) cnt += ekey[e0 + i] >= cand ? 1u : 0u;
        cnt = wg_sum<uint64_t>(cnt, red64);
        if (cnt >= m) T = cand;
    }
    for (uint64_t i = threadIdx.x; i < ne; i += blockDim.x) keep[e0 + i] = ekey[e0 + i] >= T ? 1 : 0;
    const uint64_t c0 = hop ? cand_split[q] : cand_off[q], c1 = hop ? cand_off[q + 1] : cand_split[q];
    float pk = 0.0f, pa = 0.0f;
    for (uint64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
        const float x = score[i];
        const float p = (x != x) ? 0.0f : 1.0f / (1.0f + expf(-x));
        pa += p;
        if (ekey[ce[i]] >= T) pk += p;
    }
    pk = wg_sum<float>(pk, redf);
    pa = wg_sum<float>(pa, redf);
    if (threadIdx.x == 0 && mass) mass[2 * q + hop] = pa > 0.0f ? pk / pa : 1.0f;
}

// Positive flags per entry: an entry of s's out-row (t's in-row) is positive
// when its vertex is the a (the b) of one of the query's given paths.  The
// rows are sorted by vertex id, so each lookup is a binary search.
__device__ inline uint32_t row_find(const uint32_t *col, uint32_t beg, uint32_t end, uint32_t x) {
    uint32_t lo = beg, hi = end;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (col[mid] < x) lo = mid + 1; else hi = mid;
    }
    return (lo < end && col[lo] == x) ? lo : 0xFFFFFFFFu;
}

__global__ void label_kernel(const uint32_t *out_rp, const uint32_t *out_col, const uint32_t *in_rp,
                             const uint32_t *in_col, uint32_t n, const uint32_t *src, const uint32_t *dst,
                             const uint64_t *entry_off, const mhr_path *paths, const uint32_t *count, uint32_t kmax,
                             uint8_t *pos) {
    const uint32_t q = blockIdx.x;
    const uint32_t s = src[q], t = dst[q];
    if (!(s < n && t < n)) return;
    const uint32_t sb = out_rp[s], se = out_rp[s + 1], tb = in_rp[t], te = in_rp[t + 1];
    const uint64_t e0 = entry_off[q];
    for (uint32_t i = threadIdx.x; i < (se - sb) + (te - tb); i += blockDim.x) pos[e0 + i] = 0;
    __syncthreads();
    const uint32_t c = min(count[q], kmax);
    for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) {
        const mhr_path p = paths[static_cast<size_t>(q) * kmax + i];
        const uint32_t ja = row_find(out_col, sb, se, p.a);
        const uint32_t jb = row_find(in_col, tb, te, p.b);
        if (ja != 0xFFFFFFFFu) pos[e0 + (ja - sb)] = 1;
        if (jb != 0xFFFFFFFFu) pos[e0 + (se - sb) + (jb - tb)] = 1;
    }
}

// Counter-based uniform number in [0, 1) for (seed, i): the SplitMix64
// finaliser (Steele, Lea & Flood 2014) of seed + (i + 1) * golden gamma.
__device__ __forceinline__ float uniform01(uint64_t seed, uint64_t i) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return static_cast<float>(z >> 40) * (1.0f / 16777216.0f);
}

// Training-sample choice per candidate: every positive, and each negative
// with probability min(1, neg / negatives of its query and hop), so that
// about `neg` negatives per hop and query are drawn.
__global__ void sample_mask_kernel(const uint64_t *cand_off, const uint64_t *cand_split, uint64_t n,
                                   const uint32_t *cq, const uint64_t *ce, const uint8_t *pos, const uint32_t *npos,
                                   uint32_t neg, uint64_t seed, uint8_t *take) {
    for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * blockDim.x) {
        const uint32_t q = cq[i] & ~kHop2;
        const bool hop = i >= cand_split[q];
        const uint64_t nh = hop ? cand_off[q + 1] - cand_split[q] : cand_split[q] - cand_off[q];
        const uint64_t nneg = nh - npos[2 * q + (hop ? 1 : 0)];
        const bool p = pos[ce[i]] != 0;
        take[i] = (p || (nneg > 0 && uniform01(seed, i) * static_cast<float>(nneg) < static_cast<float>(neg))) ? 1 : 0;
    }
}

// positive candidates per (query, hop)
__global__ void count_pos_kernel(const uint64_t *cand_off, const uint64_t *cand_split, const uint64_t *ce,
                                 const uint8_t *pos, uint32_t *npos) {
    __shared__ uint64_t red[kBlock / kWave];
    const uint32_t q = blockIdx.x, hop = blockIdx.y;
    const uint64_t c0 = hop ? cand_split[q] : cand_off[q], c1 = hop ? cand_off[q + 1] : cand_split[q];
    uint64_t cnt = 0;
    for (uint64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) cnt += pos[ce[i]] ? 1u : 0u;
    cnt = wg_sum<uint64_t>(cnt, red);
    if (threadIdx.x == 0) npos[2 * q + hop] = static_cast<uint32_t>(cnt);
}

constexpr uint32_t kCompactChunk = 4096;   // flags per block in the compaction passes

__global__ void chunk_count_kernel(const uint8_t *flag, uint64_t n, uint64_t *cnt) {
    __shared__ uint64_t red[kBlock / kWave];
    const uint64_t b0 = blockIdx.x * uint64_t(kCompactChunk), b1 = min(n, b0 + kCompactChunk);
    uint64_t c = 0;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) c += flag[i] ? 1u : 0u;
    c = wg_sum<uint64_t>(c, red);
    if (threadIdx.x == 0) cnt[blockIdx.x] = c;
}

// In-order compaction of the taken candidates into training samples.
__global__ void sample_fill_kernel(const uint8_t *take, uint64_t n, const uint64_t *chunk_off, const uint32_t *cq,
                                   const uint32_t *cv, const uint32_t *cr, const uint64_t *ce, const uint8_t *pos,
                                   uint32_t *sq, uint32_t *sv, uint32_t *sr, float *sl) {
    __shared__ uint64_t red[kBlock / kWave];
    __shared__ uint64_t carry;
    const uint64_t b0 = blockIdx.x * uint64_t(kCompactChunk), b1 = min(n, b0 + kCompactChunk);
    if (threadIdx.x == 0) carry = chunk_off[blockIdx.x];
    __syncthreads();
    for (uint64_t base = b0; base < b1; base += blockDim.x) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t x = (i < b1 && take[i]) ? 1u : 0u;
        uint64_t v = x;
        const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint64_t y = __shfl_up(v, off, kWave);
            if (lane >= off) v += y;
        }
        if (lane == kWave - 1) red[wave] = v;
        __syncthreads();
        uint64_t before = 0, tot = 0;
        for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) {
            if (w < wave) before += red[w];
            tot += red[w];
        }
        const uint64_t c = carry;
        if (x) {
            const uint64_t o = c + before + v - 1;
            sq[o] = cq[i];
            sv[o] = cv[i];
            sr[o] = cr[i];
            sl[o] = pos[ce[i]] ? 1.0f : 0.0f;
        }
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
}

// One workgroup: the queries to answer exactly, because the pruned search
// found fewer than k paths or kept less than tau of the predicted mass at
// either hop; compacted in order, their count in *nfb.
__global__ void fallback_kernel(uint32_t nq, const uint32_t *src, const uint32_t *dst, const uint32_t *kq,
                                uint32_t kdef, const uint32_t *count, const uint32_t *status, const float *mass,
                                float tau, uint32_t *fb_src, uint32_t *fb_dst, uint32_t *fb_k, uint32_t *fb_idx,
                                uint32_t *nfb) {
    __shared__ uint32_t red[kBlock / kWave];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nq; base += blockDim.x) {
        const uint32_t q = base + threadIdx.x;
        uint32_t x = 0;
        if (q < nq && status[q] == 0) {
            const uint32_t k = kq ? kq[q] : kdef;
            x = (count[q] < k || mass[2 * q] < tau || mass[2 * q + 1] < tau) ? 1u : 0u;
        }
        uint32_t v = x;
        const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t y = __shfl_up(v, off, kWave);
            if (lane >= off) v += y;
        }
        if (lane == kWave - 1) red[wave] = v;
        __syncthreads();
        uint32_t before = 0, tot = 0;
        for (int w = 0; w < static_cast<int>(blockDim.x / kWave); ++w) {
            if (w < wave) before += red[w];
            tot += red[w];
        }
        const uint32_t c = carry;
        if (x) {
            const uint32_t o = c + before + v - 1;
            fb_src[o] = src[q];
            fb_dst[o] = dst[q];
            fb_k[o] = kq ? kq[q] : kdef;
            fb_idx[o] = q;
        }
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *nfb = carry;
}

__global__ void scatter_kernel(uint32_t n, const uint32_t *idx, uint32_t kmax, const mhr_path *sp, const uint32_t *sc,
                               const uint64_t *st, const uint32_t *ss, mhr_path *dp, uint32_t *dc, uint64_t *dt,
                               uint32_t *ds) {
    const uint32_t i = blockIdx.x;
    if (i >= n) return;
    const uint32_t q = idx[i];
    for (uint32_t j = threadIdx.x; j < kmax; j += blockDim.x)
        dp[static_cast<size_t>(q) * kmax + j] = sp[static_cast<size_t>(i) * kmax + j];
    if (threadIdx.x == 0) {
        dc[q] = sc[i];
        if (dt && st) dt[q] = st[i];
        if (ds && ss) ds[q] = ss[i];
    }
}

}  // namespace

hipError_t pruner_refresh_bf16(mhr_pruner *p, hipStream_t st) { return refresh_bf16(p, st); }

}  // namespace mhr

using namespace mhr;

extern "C" size_t mhr_pruner_param_count(uint32_t dim, uint32_t hidden) { return play(dim, hidden).n; }

namespace {

constexpr size_t kPrunerPiece = 256;
inline size_t prpiece(size_t b) { return (std::max<size_t>(b, 1) + kPrunerPiece - 1) / kPrunerPiece * kPrunerPiece; }

// Byte sizes of the handle's arrays, in buffer order: theta, grad, m, v
// (FP32), then the bfloat16 copies of W1, W2 and w3.
void pruner_pieces(uint32_t dim, uint32_t hidden, size_t (&b)[7]) {
    const PLayout L = play(dim, hidden);
    b[0] = b[1] = b[2] = b[3] = L.n * 4;
    b[4] = (L.b1 - L.W1) * 2;
    b[5] = (L.b2 - L.W2) * 2;
    b[6] = size_t(hidden) * 2;
}

mhr_status check_shape(uint32_t dim, uint32_t hidden) {
    MHR_ARG_CHECK(dim >= 8 && dim <= 512 && dim % 8 == 0, "pruner: dim must be a multiple of 8 in [8, 512]");
    MHR_ARG_CHECK(hidden >= 16 && hidden <= 4096 && hidden % 16 == 0,
                  "pruner: hidden must be a multiple of 16 in [16, 4096]");
    return MHR_OK;
}

// buffer: the caller's (bytes from mhr_pruner_buffer_bytes), or null to
// allocate the arrays here.
mhr_status create_pruner(uint32_t dim, uint32_t hidden, void *buffer, hipStream_t st, mhr_pruner **out) {
    mhr_pruner *p = new (std::nothrow) mhr_pruner;
    if (!p) {
        set_error("mhr_pruner_create: out of host memory");
        return MHR_ERR_OUT_OF_MEMORY;
    }
    p->d = dim;
    p->H = hidden;
    const PLayout L = play(dim, hidden);
    p->np = L.n;
    p->owns = buffer == nullptr;
    size_t b[7];
    pruner_pieces(dim, hidden, b);
    void *ptr[7] = {};
    bool ok = true;
    char *at = static_cast<char *>(buffer);
    for (int i = 0; i < 7; ++i) {
        if (buffer) {
            ptr[i] = at;
            at += prpiece(b[i]);
        } else {
            ok = ok && hipMalloc(&ptr[i], prpiece(b[i])) == hipSuccess;
        }
    }
    p->theta = static_cast<float *>(ptr[0]);
    p->grad = static_cast<float *>(ptr[1]);
    p->m = static_cast<float *>(ptr[2]);
    p->v = static_cast<float *>(ptr[3]);
    p->W1b = static_cast<uint16_t *>(ptr[4]);
    p->W2b = static_cast<uint16_t *>(ptr[5]);
    p->w3b = static_cast<uint16_t *>(ptr[6]);
    if (!ok) {
        mhr_pruner_destroy(p);
        set_error("mhr_pruner_create: device allocation failed");
        return MHR_ERR_OUT_OF_MEMORY;
    }
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(L.n)), dim3(256), 0, st, p->theta, L.n, 0.0f);
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(L.n)), dim3(256), 0, st, p->grad, L.n, 0.0f);
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(L.n)), dim3(256), 0, st, p->m, L.n, 0.0f);
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(L.n)), dim3(256), 0, st, p->v, L.n, 0.0f);
    if (refresh_bf16(p, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        mhr_pruner_destroy(p);
        set_error("mhr_pruner_create: initialisation failed");
        return MHR_ERR_DEVICE;
    }
    *out = p;
    return MHR_OK;
}

}  // namespace

extern "C" mhr_status mhr_pruner_buffer_bytes(uint32_t dim, uint32_t hidden, size_t *bytes) {
    MHR_ARG_CHECK(bytes != nullptr, "mhr_pruner_buffer_bytes: null output");
    mhr_status s = check_shape(dim, hidden);
    if (s != MHR_OK) return s;
    size_t b[7], t = 0;
    pruner_pieces(dim, hidden, b);
    for (size_t x : b) t += prpiece(x);
    *bytes = t;
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_create(uint32_t dim, uint32_t hidden, mhr_pruner **out) {
    MHR_ARG_CHECK(out != nullptr, "mhr_pruner_create: null output");
    mhr_status s = check_shape(dim, hidden);
    if (s != MHR_OK) return s;
    return create_pruner(dim, hidden, nullptr, nullptr, out);
}

extern "C" mhr_status mhr_pruner_create_in(uint32_t dim, uint32_t hidden, void *buffer, size_t bytes, void *stream,
                                           mhr_pruner **out) {
    MHR_ARG_CHECK(out != nullptr && buffer != nullptr, "mhr_pruner_create_in: null argument");
    MHR_ARG_CHECK(reinterpret_cast<uintptr_t>(buffer) % kPrunerPiece == 0,
                  "mhr_pruner_create_in: buffer must be 256-byte aligned");
    size_t need = 0;
    mhr_status s = mhr_pruner_buffer_bytes(dim, hidden, &need);
    if (s != MHR_OK) return s;
    if (bytes < need) {
        set_error("mhr_pruner_create_in: buffer of " + std::to_string(bytes) + " bytes, " + std::to_string(need) +
                  " needed");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    return create_pruner(dim, hidden, buffer, static_cast<hipStream_t>(stream), out);
}

extern "C" mhr_status mhr_pruner_destroy(mhr_pruner *p) {
    if (!p) return MHR_OK;
    if (p->owns) {
        (void)hipFree(p->theta);
        (void)hipFree(p->grad);
        (void)hipFree(p->m);
        (void)hipFree(p->v);
        (void)hipFree(p->W1b);
        (void)hipFree(p->W2b);
        (void)hipFree(p->w3b);
    }
    delete p;
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_set_params(mhr_pruner *p, const float *params, void *stream) {
    MHR_ARG_CHECK(p && params, "mhr_pruner_set_params: null argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    MHR_HIP_TRY(hipMemcpyAsync(p->theta, params, p->np * 4, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(p->np)), dim3(256), 0, st, p->m, p->np, 0.0f);
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(p->np)), dim3(256), 0, st, p->v, p->np, 0.0f);
    p->step = 0;
    MHR_HIP_TRY(refresh_bf16(p, st));
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_get_params(const mhr_pruner *p, float *params, float *grad, void *stream) {
    MHR_ARG_CHECK(p != nullptr, "mhr_pruner_get_params: null pruner");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (params) MHR_HIP_TRY(hipMemcpyAsync(params, p->theta, p->np * 4, hipMemcpyDeviceToDevice, st));
    if (grad) MHR_HIP_TRY(hipMemcpyAsync(grad, p->grad, p->np * 4, hipMemcpyDeviceToDevice, st));
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_workspace_size(const mhr_pruner *p, uint32_t n, size_t *bytes) {
    MHR_ARG_CHECK(p && bytes, "mhr_pruner_workspace_size: null argument");
    *bytes = pws_layout(n, p->d, p->H).total;
    return MHR_OK;
}

static mhr_status check_model(const mhr_pruner *p, const mhr_graph *g, uint32_t n, size_t ws_bytes) {
    MHR_ARG_CHECK(p && g, "pruner: null argument");
    if (!g->X) {
        set_error("embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    MHR_ARG_CHECK(g->dim == p->d, "pruner: the graph's embedding dimension differs from the pruner's");
    if (ws_bytes < pws_layout(n, p->d, p->H).total) {
        set_error("pruner workspace too small: need " + std::to_string(pws_layout(n, p->d, p->H).total) + " bytes");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_forward(mhr_pruner *p, const mhr_graph *g, uint32_t n, const uint32_t *q,
                                         const uint32_t *src, const uint32_t *dst, const uint32_t *v,
                                         const uint32_t *r, float *logits, void *ws, size_t ws_bytes, void *stream) {
    mhr_status rc = check_model(p, g, n, ws_bytes);
    if (rc != MHR_OK) return rc;
    if (n == 0) return MHR_OK;
    MHR_ARG_CHECK(q && src && dst && v && r && logits && ws, "mhr_pruner_forward: null pointer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    rc = forward_impl(p, g, n, q, src, dst, v, r, w, st);
    if (rc != MHR_OK) return rc;
    MHR_HIP_TRY(hipMemcpyAsync(logits, w + pws_layout(n, p->d, p->H).z, size_t(n) * 4, hipMemcpyDeviceToDevice, st));
    return MHR_OK;
}

namespace mhr {
namespace {

// Per (query, hop) row j = 2 q + hop: the endpoint the candidate edge
// touches and the other one (hop 2 swaps them, as expand_query_kernel does).
__global__ void query_rows_kernel(const uint32_t *src, const uint32_t *dst, uint32_t nq, uint32_t *qs, uint32_t *qt) {
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < 2 * nq; j += gridDim.x * blockDim.x) {
        const uint32_t q = j >> 1;
        const bool hop2 = j & 1u;
        qs[j] = hop2 ? dst[q] : src[q];
        qt[j] = hop2 ? src[q] : dst[q];
    }
}

struct ScoreWs {
    size_t Zq, Zr, qs, qt, h1, zpart, total;
};

ScoreWs score_layout(uint32_t nq, uint32_t R, uint32_t H, uint32_t chunk) {
    ScoreWs L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = (o + std::max<size_t>(bytes, 1) + 255) & ~size_t(255); return r; };
    L.Zq = take(size_t(2) * nq * H * 4);
    L.Zr = take(size_t(R) * H * 4);
    L.qs = take(size_t(2) * nq * 4);
    L.qt = take(size_t(2) * nq * 4);
    L.h1 = take(size_t(chunk) * H * 2);
    L.zpart = take(size_t((H + kNtN - 1) / kNtN) * chunk * 4);
    L.total = o;
    return L;
}

// Column block [c0, c0 + K) of W1 (bf16 [H][4d]) as a B operand.
Mat w1_block(const mhr_pruner *p, uint32_t c0, uint32_t K) {
    Mat B{};
    B.p[0] = p->W1b + c0;
    B.seg = K;
    B.ld = 4 * p->d;
    B.nseg = 1;
    B.vec = 1;
    return B;
}

}  // namespace
}  // namespace mhr

extern "C" mhr_status mhr_pruner_score_workspace_size(const mhr_pruner *p, const mhr_graph *g, uint32_t nq,
                                                      uint32_t chunk, size_t *bytes) {
    MHR_ARG_CHECK(p && g && bytes, "mhr_pruner_score_workspace_size: null argument");
    MHR_ARG_CHECK(chunk >= 1 && (chunk + kNtM - 1) / kNtM <= 65535u, "mhr_pruner_score_workspace_size: bad chunk");
    *bytes = score_layout(nq, g->R, p->H, chunk).total;
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_score(mhr_pruner *p, const mhr_graph *g, uint32_t nq, const uint32_t *src,
                                       const uint32_t *dst, uint64_t ncand, const uint32_t *q, const uint32_t *v,
                                       const uint32_t *r, float *logits, uint32_t chunk, void *ws, size_t ws_bytes,
                                       void *stream) {
    MHR_ARG_CHECK(p && g, "mhr_pruner_score: null handle");
    MHR_ARG_CHECK(g->X && g->Y && g->dim == p->d, "mhr_pruner_score: graph embeddings missing or of another dimension");
    MHR_ARG_CHECK(chunk >= 1 && (chunk + kNtM - 1) / kNtM <= 65535u, "mhr_pruner_score: bad chunk");
    if (ncand == 0) return MHR_OK;
    MHR_ARG_CHECK(nq >= 1 && src && dst && q && v && r && logits && ws, "mhr_pruner_score: null pointer");
    const ScoreWs W = score_layout(nq, g->R, p->H, chunk);
    if (ws_bytes < W.total) {
        set_error("mhr_pruner_score: workspace of " + std::to_string(ws_bytes) + " bytes, " +
                  std::to_string(W.total) + " needed");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    const uint32_t d = p->d, H = p->H;
    const PLayout L = play(d, H);
    float *Zq = reinterpret_cast<float *>(w + W.Zq), *Zr = reinterpret_cast<float *>(w + W.Zr);
    uint32_t *qs = reinterpret_cast<uint32_t *>(w + W.qs), *qt = reinterpret_cast<uint32_t *>(w + W.qt);
    uint16_t *h1 = reinterpret_cast<uint16_t *>(w + W.h1);
    float *zpart = reinterpret_cast<float *>(w + W.zpart);
    const uint32_t f32 = g->dtype == MHR_DTYPE_F32 ? 1u : 0u;
    // the query endpoints' share of the first layer, once per (query, hop)
    hipLaunchKernelGGL(query_rows_kernel, dim3(grid_for(size_t(2) * nq)), dim3(256), 0, st, src, dst, nq, qs, qt);
    Mat Aq{};
    Aq.p[0] = g->X; Aq.idx[0] = qs; Aq.lim[0] = g->n;
    Aq.p[1] = g->X; Aq.idx[1] = qt; Aq.lim[1] = g->n;
    Aq.seg = d; Aq.ld = d; Aq.nseg = 2; Aq.f32 = f32; Aq.vec = 1;
    NtEpilogue Eq{};
    Eq.C = Zq;
    Eq.ldc = H;
    MHR_HIP_TRY(gemm_nt<kEpiF32>(Aq, w1_block(p, 0, 2 * d), 2 * nq, H, 2 * d, Eq, st));
    // the relations' share, once per relation
    Mat Ar = plain(g->Y, d, f32 != 0);
    NtEpilogue Er{};
    Er.C = Zr;
    Er.ldc = H;
    MHR_HIP_TRY(gemm_nt<kEpiF32>(Ar, w1_block(p, 3 * d, d), g->R, H, d, Er, st));
    // per candidate: its own share, then the second layer and the output
    const uint32_t nb = (H + kNtN - 1) / kNtN;
    for (uint64_t c0 = 0; c0 < ncand; c0 += chunk) {
        const uint32_t m = static_cast<uint32_t>(std::min<uint64_t>(chunk, ncand - c0));
        Mat Ac{};
        Ac.p[0] = g->X; Ac.idx[0] = v + c0; Ac.lim[0] = g->n;
        Ac.seg = d; Ac.ld = d; Ac.nseg = 1; Ac.f32 = f32; Ac.vec = 1;
        NtEpilogue E1{};
        E1.h = h1;
        E1.bias = p->theta + L.b1;
        E1.T1 = Zq; E1.q1 = q + c0; E1.t1_queries = nq;
        E1.T2 = Zr; E1.r2 = r + c0; E1.t2_rows = g->R;
        MHR_HIP_TRY(gemm_nt<kEpiBiasRelu>(Ac, w1_block(p, 2 * d, d), m, H, d, E1, st));
        NtEpilogue E2{};
        E2.bias = p->theta + L.b2;
        E2.w3 = p->w3b;
        E2.zpart = zpart;
        MHR_HIP_TRY(gemm_nt<kEpiBiasReluDot>(plain(h1, H), plain(p->W2b, H), m, H, H, E2, st));
        hipLaunchKernelGGL(zpart_reduce_kernel, dim3(grid_for(m)), dim3(256), 0, st, zpart, nb, m, p->theta + L.b3,
                           logits + c0, q + c0, nq, r + c0, g->R);
    }
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_train_step(mhr_pruner *p, const mhr_graph *g, uint32_t n, const uint32_t *q,
                                            const uint32_t *src, const uint32_t *dst, const uint32_t *v,
                                            const uint32_t *r, const float *label, float pos_weight, float lr,
                                            float beta1, float beta2, float eps, int update, float *loss,
                                            void *ws, size_t ws_bytes, void *stream) {
    mhr_status rc = check_model(p, g, n, ws_bytes);
    if (rc != MHR_OK) return rc;
    MHR_ARG_CHECK(n >= 1 && q && src && dst && v && r && label && ws, "mhr_pruner_train_step: null pointer or n = 0");
    MHR_ARG_CHECK(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f,
                  "mhr_pruner_train_step: bad Adam constants");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    rc = forward_impl(p, g, n, q, src, dst, v, r, w, st);
    if (rc != MHR_OK) return rc;
    const PWs W = pws_layout(n, p->d, p->H);
    const PLayout L = play(p->d, p->H);
    const uint32_t H = p->H, d = p->d;
    float *Z = reinterpret_cast<float *>(w + W.Z);
    uint16_t *h1 = reinterpret_cast<uint16_t *>(w + W.h1), *h2 = reinterpret_cast<uint16_t *>(w + W.h2);
    float *z = reinterpret_cast<float *>(w + W.z), *dz = reinterpret_cast<float *>(w + W.dz);
    uint32_t *s = reinterpret_cast<uint32_t *>(w + W.s), *t = reinterpret_cast<uint32_t *>(w + W.t);
    const size_t nh = size_t(n) * H;
    float *part = reinterpret_cast<float *>(w + W.part), *cpart = reinterpret_cast<float *>(w + W.cpart);
    float *lpart = reinterpret_cast<float *>(w + W.lpart);
    const uint32_t nblk = grid_for(n, kBlock), chunks = (n + kColRows - 1) / kColRows;
    const dim3 cgrid((H + 255) / 256, chunks);
    hipLaunchKernelGGL(bce_kernel, dim3(nblk), dim3(kBlock), 0, st, z, label, n, pos_weight, dz, lpart);
    if (loss) hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kBlock), 0, st, lpart, nblk, loss);
    // output layer
    hipLaunchKernelGGL(colsum_kernel, cgrid, dim3(256), 0, st, h2, dz, cpart, n, H, kColRows);
    hipLaunchKernelGGL(colsum_reduce_kernel, dim3((H + 255) / 256), dim3(256), 0, st, cpart, chunks, H,
                       p->grad + L.w3);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kBlock), 0, st, dz, n, p->grad + L.b3);
    // second layer: dz2 over h2, then dW2 = dz2^T h1, db2, dH1 = dz2 W2
    hipLaunchKernelGGL(dz2_kernel, dim3(grid_for(nh)), dim3(256), 0, st, dz, p->w3b, h2, nh, H);
    MHR_HIP_TRY((gemm<true, false>(plain(h2, H), plain(h1, H), p->grad + L.W2, H, H, H, n, splits_for(H, H, n), part,
                                   st)));
    hipLaunchKernelGGL(colsum_kernel, cgrid, dim3(256), 0, st, h2, nullptr, cpart, n, H, kColRows);
    hipLaunchKernelGGL(colsum_reduce_kernel, dim3((H + 255) / 256), dim3(256), 0, st, cpart, chunks, H,
                       p->grad + L.b2);
    MHR_HIP_TRY((gemm<false, false>(plain(h2, H), plain(p->W2b, H), Z, H, n, H, H, 1, nullptr, st)));
    // first layer: dz1 over h1, then dW1 = dz1^T F, db1
    hipLaunchKernelGGL(dz1_kernel, dim3(grid_for(nh)), dim3(256), 0, st, Z, h1, nh);
    const Mat F = features(g, s, t, v, r);
    MHR_HIP_TRY((gemm<true, false>(plain(h1, H), F, p->grad + L.W1, 4 * d, H, 4 * d, n, splits_for(H, 4 * d, n),
                                   part, st)));
    hipLaunchKernelGGL(colsum_kernel, cgrid, dim3(256), 0, st, h1, nullptr, cpart, n, H, kColRows);
    hipLaunchKernelGGL(colsum_reduce_kernel, dim3((H + 255) / 256), dim3(256), 0, st, cpart, chunks, H,
                       p->grad + L.b1);
    if (update) {
        p->step += 1;
        const float bc1 = 1.0f - powf(beta1, static_cast<float>(p->step));
        const float bc2 = 1.0f - powf(beta2, static_cast<float>(p->step));
        hipLaunchKernelGGL(adam_kernel, dim3(grid_for(p->np)), dim3(256), 0, st, p->theta, p->grad, p->m, p->v, p->np,
                           lr, beta1, beta2, eps, bc1, bc2);
        MHR_HIP_TRY(refresh_bf16(p, st));
    }
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_count(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                                       uint64_t *entry_off, uint64_t *cand_off, void *stream) {
    MHR_ARG_CHECK(g && src && dst && entry_off && cand_off, "mhr_pruner_count: null argument");
    MHR_ARG_CHECK(nq >= 1, "mhr_pruner_count: nq must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(cand_count_kernel, dim3(nq), dim3(kBlock), 0, st, g->out.row_ptr, g->out.rmask, g->in.row_ptr,
                       g->in.rmask, g->n, src, dst, entry_off, cand_off);
    hipLaunchKernelGGL(excl_scan_kernel, dim3(1), dim3(kBlock), 0, st, entry_off, nq);
    hipLaunchKernelGGL(excl_scan_kernel, dim3(1), dim3(kBlock), 0, st, cand_off, nq);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_enumerate(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                                           const uint64_t *entry_off, const uint64_t *cand_off, uint64_t *cand_split,
                                           uint32_t *cand_q, uint32_t *cand_v, uint32_t *cand_r, uint64_t *cand_e,
                                           void *stream) {
    MHR_ARG_CHECK(g && src && dst && entry_off && cand_off && cand_split && cand_q && cand_v && cand_r && cand_e,
                  "mhr_pruner_enumerate: null argument");
    MHR_ARG_CHECK(nq >= 1, "mhr_pruner_enumerate: nq must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(cand_fill_kernel, dim3(nq), dim3(kBlock), 0, st, g->out.row_ptr, g->out.col, g->out.rmask,
                       g->in.row_ptr, g->in.col, g->in.rmask, g->n, src, dst, entry_off, cand_off, cand_split, cand_q,
                       cand_v, cand_r, cand_e);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_select(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                                        const uint64_t *entry_off, const uint64_t *cand_off,
                                        const uint64_t *cand_split, const float *score, const uint64_t *cand_e,
                                        uint64_t ncand, uint64_t nentries, uint32_t keep_permille, uint8_t *keep,
                                        float *mass, uint32_t *entry_key, void *stream) {
    MHR_ARG_CHECK(g && src && dst && entry_off && cand_off && cand_split && keep && entry_key,
                  "mhr_pruner_select: null argument");
    MHR_ARG_CHECK(ncand == 0 || (score && cand_e), "mhr_pruner_select: null scores");
    MHR_ARG_CHECK(nq >= 1 && keep_permille >= 1 && keep_permille <= 1000,
                  "mhr_pruner_select: nq >= 1 and keep_permille in [1, 1000]");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nentries) {
        hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(nentries)), dim3(256), 0, st, entry_key, nentries, 0u);
        if (ncand)
            hipLaunchKernelGGL(entry_key_kernel, dim3(grid_for(ncand)), dim3(256), 0, st, score, cand_e, ncand,
                               entry_key);
    }
    hipLaunchKernelGGL(select_kernel, dim3(nq, 2), dim3(kBlock), 0, st, g->out.row_ptr, g->in.row_ptr, g->n, src, dst,
                       entry_off, cand_off, cand_split, score, cand_e, entry_key, keep_permille, keep, mass);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_label(const mhr_graph *g, uint32_t nq, const uint32_t *src, const uint32_t *dst,
                                       const uint64_t *entry_off, const mhr_path *paths, const uint32_t *count,
                                       uint32_t kmax, uint8_t *pos, void *stream) {
    MHR_ARG_CHECK(g && src && dst && entry_off && paths && count && pos, "mhr_pruner_label: null argument");
    MHR_ARG_CHECK(nq >= 1 && kmax >= 1, "mhr_pruner_label: nq >= 1 and kmax >= 1");
    hipLaunchKernelGGL(label_kernel, dim3(nq), dim3(256), 0, static_cast<hipStream_t>(stream), g->out.row_ptr,
                       g->out.col, g->in.row_ptr, g->in.col, g->n, src, dst, entry_off, paths, count, kmax, pos);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

extern "C" size_t mhr_pruner_sample_workspace(uint32_t nq, uint64_t ncand) {
    const size_t chunks = static_cast<size_t>((ncand + kCompactChunk - 1) / kCompactChunk);
    return ((ncand + 255) & ~uint64_t(255)) + (size_t(2) * nq * 4 + 255) / 256 * 256 + (chunks + 1) * 8;
}

extern "C" mhr_status mhr_pruner_sample(uint32_t nq, const uint64_t *cand_off, const uint64_t *cand_split,
                                        uint64_t ncand, const uint32_t *cand_q, const uint32_t *cand_v,
                                        const uint32_t *cand_r, const uint64_t *cand_e, const uint8_t *pos,
                                        uint32_t neg_per_hop, uint64_t seed, uint32_t *sq, uint32_t *sv,
                                        uint32_t *sr, float *slabel, uint64_t *nsamples, void *ws, size_t ws_bytes,
                                        void *stream) {
    MHR_ARG_CHECK(cand_off && cand_split && pos && sq && sv && sr && slabel && nsamples && ws,
                  "mhr_pruner_sample: null argument");
    MHR_ARG_CHECK(nq >= 1, "mhr_pruner_sample: nq must be >= 1");
    if (ws_bytes < mhr_pruner_sample_workspace(nq, ncand)) {
        set_error("mhr_pruner_sample: workspace too small");
        return MHR_ERR_WORKSPACE_TOO_SMALL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    uint8_t *take = reinterpret_cast<uint8_t *>(w);
    uint32_t *npos = reinterpret_cast<uint32_t *>(w + ((ncand + 255) & ~uint64_t(255)));
    uint64_t *chunk = reinterpret_cast<uint64_t *>(w + ((ncand + 255) & ~uint64_t(255)) +
                                                   (size_t(2) * nq * 4 + 255) / 256 * 256);
    const uint32_t chunks = static_cast<uint32_t>((ncand + kCompactChunk - 1) / kCompactChunk);
    if (ncand == 0) {
        hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<float *>(nsamples), size_t(2), 0.0f);
        MHR_HIP_TRY(hipGetLastError());
        return MHR_OK;
    }
    hipLaunchKernelGGL(count_pos_kernel, dim3(nq, 2), dim3(kBlock), 0, st, cand_off, cand_split, cand_e, pos, npos);
    hipLaunchKernelGGL(sample_mask_kernel, dim3(grid_for(ncand)), dim3(256), 0, st, cand_off, cand_split, ncand,
                       cand_q, cand_e, pos, npos, neg_per_hop, seed, take);
    hipLaunchKernelGGL(chunk_count_kernel, dim3(chunks), dim3(kBlock), 0, st, take, ncand, chunk);
    hipLaunchKernelGGL(excl_scan_kernel, dim3(1), dim3(kBlock), 0, st, chunk, chunks);
    hipLaunchKernelGGL(sample_fill_kernel, dim3(chunks), dim3(kBlock), 0, st, take, ncand, chunk, cand_q, cand_v,
                       cand_r, cand_e, pos, sq, sv, sr, slabel);
    MHR_HIP_TRY(hipMemcpyAsync(nsamples, chunk + chunks, 8, hipMemcpyDeviceToDevice, st));
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

extern "C" mhr_status mhr_pruner_fallback(uint32_t nq, const uint32_t *src, const uint32_t *dst, const uint32_t *k,
                                          uint32_t kdef, const uint32_t *count, const uint32_t *status,
                                          const float *mass, float tau, uint32_t *fb_src, uint32_t *fb_dst,
                                          uint32_t *fb_k, uint32_t *fb_idx, uint32_t *nfb, void *stream) {
    MHR_ARG_CHECK(src && dst && count && status && mass && fb_src && fb_dst && fb_k && fb_idx && nfb,
                  "mhr_pruner_fallback: null argument");
    MHR_ARG_CHECK(nq >= 1 && (k || kdef >= 1), "mhr_pruner_fallback: nq >= 1 and a K");
    hipLaunchKernelGGL(fallback_kernel, dim3(1), dim3(kBlock), 0, static_cast<hipStream_t>(stream), nq, src, dst, k,
                       kdef, count, status, mass, tau, fb_src, fb_dst, fb_k, fb_idx, nfb);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

extern "C" mhr_status mhr_scatter_results(uint32_t n, const uint32_t *idx, uint32_t kmax, const mhr_path *src_paths,
                                          const uint32_t *src_count, const uint64_t *src_total,
                                          const uint32_t *src_status, mhr_path *paths, uint32_t *count,
                                          uint64_t *total, uint32_t *status, void *stream) {
    if (n == 0) return MHR_OK;
    MHR_ARG_CHECK(idx && src_paths && src_count && paths && count && kmax >= 1, "mhr_scatter_results: null argument");
    hipLaunchKernelGGL(scatter_kernel, dim3(n), dim3(64), 0, static_cast<hipStream_t>(stream), n, idx, kmax, src_paths,
                       src_count, src_total, src_status, paths, count, total, status);
    MHR_HIP_TRY(hipGetLastError());
    return MHR_OK;
}

// ---------------------------------------------------------------------------
// Whole training run (the sequence a caller would otherwise drive): batches
// of queries in a shuffled order, each labelled by the exact search, sampled
// and trained on in steps.
// ---------------------------------------------------------------------------
namespace mhr {
namespace {

__global__ void gather_u32_kernel(const uint32_t *src, const uint32_t *idx, uint32_t n, uint32_t *out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = src[idx[i]];
}

inline uint64_t splitmix64(uint64_t &x) {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Device buffers owned by one training run (freed on every exit).
struct TrainBuffers {
    std::vector<void *> owned;
    ~TrainBuffers() {
        for (void *p : owned) (void)hipFree(p);
    }
    template <class T>
    hipError_t get(T *&p, size_t count) {
        void *q = nullptr;
        const hipError_t e = hipMalloc(&q, (count ? count : 1) * sizeof(T));
        if (e == hipSuccess) owned.push_back(q);
        p = static_cast<T *>(q);
        return e;
    }
};

}  // namespace
}  // namespace mhr

extern "C" mhr_status mhr_pruner_train(mhr_pruner *p, const mhr_graph *g, const mhr_train_opts *opts, uint32_t nq,
                                       const uint32_t *src, const uint32_t *dst, float *losses, uint32_t max_losses,
                                       uint32_t *nsteps, void *stream) {
    MHR_ARG_CHECK(p && g && opts && nsteps, "mhr_pruner_train: null argument");
    MHR_ARG_CHECK(nq == 0 || (src && dst), "mhr_pruner_train: null query arrays");
    MHR_ARG_CHECK(max_losses == 0 || losses, "mhr_pruner_train: null loss array");
    for (uint32_t v : opts->reserved) MHR_ARG_CHECK(v == 0, "mhr_pruner_train: reserved fields must be zero");
    if (!g->X) {
        set_error("embeddings not set");
        return MHR_ERR_NO_EMBEDDINGS;
    }
    MHR_ARG_CHECK(g->dim == p->d, "mhr_pruner_train: the graph's embedding dimension differs from the pruner's");
    const uint32_t K = opts->k;
    MHR_ARG_CHECK(K >= 1 && K <= MHR_MAX_K, "mhr_pruner_train: k must be in [1, MHR_MAX_K]");
    const uint32_t B = opts->batch_queries ? opts->batch_queries : 4096u;
    const uint32_t S = opts->step_samples ? opts->step_samples : 65536u;
    const uint32_t E = opts->epochs ? opts->epochs : 1u;
    const uint32_t neg = opts->neg_per_hop ? opts->neg_per_hop : 64u;
    const float lr = opts->lr > 0.0f ? opts->lr : 1e-3f;
    const float b1 = opts->beta1 > 0.0f ? opts->beta1 : 0.9f, b2 = opts->beta2 > 0.0f ? opts->beta2 : 0.999f;
    const float eps = opts->eps > 0.0f ? opts->eps : 1e-8f;
    hipStream_t st = static_cast<hipStream_t>(stream);
    *nsteps = 0;
    if (nq == 0) return MHR_OK;

    TrainBuffers tb;
    const uint32_t nb_max = std::min(B, nq);
    uint32_t *perm_d, *bsrc, *bdst, *cnt;
    mhr_path *paths;
    uint64_t *eo, *co, *cs, *nsamp;
    float *loss_d, *possum;
    MHR_HIP_TRY(tb.get(perm_d, nb_max));
    MHR_HIP_TRY(tb.get(bsrc, nb_max));
    MHR_HIP_TRY(tb.get(bdst, nb_max));
    MHR_HIP_TRY(tb.get(cnt, nb_max));
    MHR_HIP_TRY(tb.get(paths, size_t(nb_max) * K));
    MHR_HIP_TRY(tb.get(eo, size_t(nb_max) + 1));
    MHR_HIP_TRY(tb.get(co, size_t(nb_max) + 1));
    MHR_HIP_TRY(tb.get(cs, nb_max));
    MHR_HIP_TRY(tb.get(nsamp, 1));
    MHR_HIP_TRY(tb.get(possum, 1));
    mhr_query_opts qo{};
    qo.k = K;
    size_t ws_bytes = 0;
    mhr_status rc = mhr_workspace_size(g, &qo, nb_max, K, &ws_bytes);
    if (rc != MHR_OK) return rc;
    unsigned char *ws;
    MHR_HIP_TRY(tb.get(ws, ws_bytes));
    size_t pws_bytes = 0;
    rc = mhr_pruner_workspace_size(p, S, &pws_bytes);
    if (rc != MHR_OK) return rc;
    unsigned char *pws;
    MHR_HIP_TRY(tb.get(pws, pws_bytes));
    // candidate and sample buffers grow with the largest batch seen
    uint64_t cap_c = 0, cap_e = 0;
    uint32_t *cq = nullptr, *cv = nullptr, *cr = nullptr, *sq = nullptr, *sv = nullptr, *sr = nullptr;
    uint64_t *ce = nullptr;
    uint8_t *pos = nullptr;
    float *sl = nullptr;
    unsigned char *sws = nullptr;
    size_t sws_cap = 0;
    uint32_t loss_cap = 0;
    loss_d = nullptr;

    std::vector<uint32_t> perm(nq);
    uint64_t rng = opts->seed ^ 0x6D68725F74726169ull;
    uint32_t steps = 0;
    uint64_t batch_no = 0;
    for (uint32_t ep = 0; ep < E; ++ep) {
        for (uint32_t i = 0; i < nq; ++i) perm[i] = i;
        for (uint32_t i = nq - 1; i > 0; --i) {   // Fisher-Yates with SplitMix64
            const uint32_t j = static_cast<uint32_t>(splitmix64(rng) % (static_cast<uint64_t>(i) + 1));
            std::swap(perm[i], perm[j]);
        }
        for (uint32_t b0 = 0; b0 < nq; b0 += B, ++batch_no) {
            const uint32_t nb = std::min(B, nq - b0);
            MHR_HIP_TRY(hipMemcpyAsync(perm_d, perm.data() + b0, size_t(nb) * 4, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(gather_u32_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, src, perm_d, nb, bsrc);
            hipLaunchKernelGGL(gather_u32_kernel, dim3((nb + 255) / 256), dim3(256), 0, st, dst, perm_d, nb, bdst);
            // labels: the exact top-K
            rc = mhr_topk_paths(g, &qo, nb, bsrc, bdst, nullptr, K, paths, cnt, nullptr, nullptr, ws, ws_bytes, st);
            if (rc != MHR_OK) return rc;
            rc = mhr_pruner_count(g, nb, bsrc, bdst, eo, co, st);
            if (rc != MHR_OK) return rc;
            uint64_t tot[2];
            MHR_HIP_TRY(hipMemcpyAsync(&tot[0], eo + nb, 8, hipMemcpyDeviceToHost, st));
            MHR_HIP_TRY(hipMemcpyAsync(&tot[1], co + nb, 8, hipMemcpyDeviceToHost, st));
            MHR_HIP_TRY(hipStreamSynchronize(st));
            const uint64_t nent = tot[0], ncand = tot[1];
            if (ncand == 0) continue;
            if (ncand > cap_c) {
                cap_c = ncand + ncand / 4;
                MHR_HIP_TRY(tb.get(cq, cap_c));
                MHR_HIP_TRY(tb.get(cv, cap_c));
                MHR_HIP_TRY(tb.get(cr, cap_c));
                MHR_HIP_TRY(tb.get(ce, cap_c));
                MHR_HIP_TRY(tb.get(sq, cap_c));
                MHR_HIP_TRY(tb.get(sv, cap_c));
                MHR_HIP_TRY(tb.get(sr, cap_c));
                MHR_HIP_TRY(tb.get(sl, cap_c));
            }
            if (nent > cap_e) {
                cap_e = nent + nent / 4;
                MHR_HIP_TRY(tb.get(pos, cap_e));
            }
            const size_t swsb = mhr_pruner_sample_workspace(nb, ncand);
            if (swsb > sws_cap) {
                sws_cap = swsb;
                MHR_HIP_TRY(tb.get(sws, sws_cap));
            }
            rc = mhr_pruner_enumerate(g, nb, bsrc, bdst, eo, co, cs, cq, cv, cr, ce, st);
            if (rc != MHR_OK) return rc;
            rc = mhr_pruner_label(g, nb, bsrc, bdst, eo, paths, cnt, K, pos, st);
            if (rc != MHR_OK) return rc;
            rc = mhr_pruner_sample(nb, co, cs, ncand, cq, cv, cr, ce, pos, neg, opts->seed * 1000003ull + batch_no, sq, sv,
                                   sr, sl, nsamp, sws, sws_cap, st);
            if (rc != MHR_OK) return rc;
            uint64_t m = 0;
            MHR_HIP_TRY(hipMemcpyAsync(&m, nsamp, 8, hipMemcpyDeviceToHost, st));
            MHR_HIP_TRY(hipStreamSynchronize(st));
            if (m == 0) continue;
            hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, possum, size_t(1), 0.0f);
            hipLaunchKernelGGL(sum_kernel, dim3(grid_for(m)), dim3(256), 0, st, sl, static_cast<uint32_t>(m), possum);
            float npos = 0.0f;
            MHR_HIP_TRY(hipMemcpyAsync(&npos, possum, 4, hipMemcpyDeviceToHost, st));
            MHR_HIP_TRY(hipStreamSynchronize(st));
            const float wpos = (static_cast<float>(m) - npos) / std::max(npos, 1.0f);
            const uint32_t nst = static_cast<uint32_t>((m + S - 1) / S);
            if (nst > loss_cap) {
                loss_cap = nst;
                MHR_HIP_TRY(tb.get(loss_d, loss_cap));
            }
            for (uint32_t k = 0; k < nst; ++k) {
                const uint64_t a = uint64_t(k) * S;
                const uint32_t len = static_cast<uint32_t>(std::min<uint64_t>(S, m - a));
                rc = mhr_pruner_train_step(p, g, len, sq + a, bsrc, bdst, sv + a, sr + a, sl + a, wpos, lr, b1, b2, eps,
                                           1, loss_d + k, pws, pws_bytes, st);
                if (rc != MHR_OK) return rc;
            }
            const uint32_t room = steps < max_losses ? std::min(nst, max_losses - steps) : 0u;
            if (room) MHR_HIP_TRY(hipMemcpyAsync(losses + steps, loss_d, size_t(room) * 4, hipMemcpyDeviceToHost, st));
            MHR_HIP_TRY(hipStreamSynchronize(st));
            steps += nst;
        }
    }
    *nsteps = steps;
    return MHR_OK;
}
