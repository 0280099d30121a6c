// Learned surrogate: a bfloat16 multilayer perceptron trained and evaluated on
// the matrix cores of gfx950 (v_mfma_f32_16x16x32_bf16, FP32 accumulation).
// C-ABI in include/tled_surrogate.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tled_surrogate.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef short i16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) i16x4 lds_i16x4;

constexpr int kThreads = 256;
constexpr int kColChunk = 64;   // least rows per chunk of a column-sum pass
constexpr int BM = 64, BN = 64, BK = 64, BKP = BK + 8;   // LDS rows padded against bank conflicts

__device__ inline float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
// float -> bfloat16 bits by the hardware convert (v_cvt_pk_bf16_f32 on gfx950,
// round to nearest even).
__device__ inline uint16_t bf16_bits(float x) {
    const __bf16 h = static_cast<__bf16>(x);
    uint16_t u;
    __builtin_memcpy(&u, &h, 2);
    return u;
}

// Logistic function from the hardware base-2 exponential and reciprocal
// (v_exp_f32, v_rcp_f32; each within about 1 ulp, far below the bfloat16
// rounding the activations then take).  Every SiLU of the forward passes and its
// derivative in the backward pass use this one function.
__device__ __forceinline__ float sigmoidf_hw(float z) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * z));
}

// sin(2 pi t) or cos(2 pi t) for t in revolutions: reduced to [-1/2, 1/2] (exact
// for |t| < 2^22), then the hardware sine/cosine, which take revolutions.
__device__ __forceinline__ float fourier_feature(float t, bool sine) {
    const float r = t - rintf(t);
    return sine ? __builtin_amdgcn_sinf(r) : __builtin_amdgcn_cosf(r);
}

enum { EPI_F32 = 0, EPI_BIAS_SILU = 1, EPI_BIAS_F32 = 2, EPI_SILU_BACK = 3 };
// How an operand tile is read from global memory: element by element (any
// strides), 16-byte vectors along k (k contiguous), or 16-byte vectors along
// the tile's rows (rows contiguous).  Chosen on the host from strides and alignment.
enum { LD_SCALAR = 0, LD_KVEC = 1, LD_RVEC = 2 };

// One thread's share (8 values) of half h (k in [k0 + 32h, k0 + 32h + 32)) of a
// 64 x 64 operand tile X(r, k) = X[r*sr + k*sk], rows r0.., zero outside r < R, k < ke,
// packed two bfloat16 per 32-bit word (value i in the low half of word i/2 when even).
struct TileRegs {
    uint4 w;
};

__device__ inline uint4 pack8(const uint16_t (&e)[8]) {
    return make_uint4(uint32_t(e[0]) | (uint32_t(e[1]) << 16), uint32_t(e[2]) | (uint32_t(e[3]) << 16),
                      uint32_t(e[4]) | (uint32_t(e[5]) << 16), uint32_t(e[6]) | (uint32_t(e[7]) << 16));
}

// Value i of a thread's share, as a float.
__device__ inline float tile_value(const TileRegs &q, int i) {
    const uint32_t u = i < 2 ? q.w.x : i < 4 ? q.w.y : i < 6 ? q.w.z : q.w.w;
    return bf2f(uint16_t((i & 1) ? (u >> 16) : (u & 0xffffu)));
}

template <int MODE>
__device__ inline void tile_load(TileRegs &q, const uint16_t *__restrict__ X, long sr, long sk, int r0, int R,
                                 int k0, int ke, int t, int h) {
    uint16_t e[8];
    if (MODE == LD_KVEC) {
        const int r = r0 + (t >> 2), k = k0 + 32 * h + (t & 3) * 8;
        if (r < R && k + 8 <= ke) {
            q.w = *reinterpret_cast<const uint4 *>(X + r * sr + k);
            return;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = (r < R && k + i < ke) ? X[r * sr + k + i] : uint16_t(0);
    } else if (MODE == LD_RVEC) {
        const int k = k0 + 32 * h + (t >> 3), r = r0 + (t & 7) * 8;
        if (k < ke && r + 8 <= R) {
            q.w = *reinterpret_cast<const uint4 *>(X + k * sk + r);
            return;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = (k < ke && r + i < R) ? X[k * sk + r + i] : uint16_t(0);
    } else {
        const int r = r0 + (t >> 2), k = k0 + 32 * h + (t & 3) * 8;
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = (r < R && k + i < ke) ? X[r * sr + (k + i) * sk] : uint16_t(0);
    }
    q.w = pack8(e);
}

// Stores a thread's share of half h of the 64-deep tile at k offset koff into an
// LDS operand of row pitch P: S[r P + k], or, for tiles read with rows contiguous,
// S[k P + r] as loaded (one 16-byte store either way; the MFMA fragments of a
// k-major operand are then fetched with the transpose read, see frag()).
template <int MODE>
__device__ inline void tile_store(const TileRegs &q, uint16_t *S, int P, int koff, int t, int h) {
    if (MODE == LD_RVEC) {
        const int k = koff + 32 * h + (t >> 3), r = (t & 7) * 8;
        *reinterpret_cast<uint4 *>(&S[k * P + r]) = q.w;
    } else {
        const int r = t >> 2, k = koff + 32 * h + (t & 3) * 8;
        *reinterpret_cast<uint4 *>(&S[r * P + k]) = q.w;
    }
}

// The 16 x 32 MFMA operand fragment of rows r0..r0+15, k in [k0, k0 + 32), of an
// LDS operand of row pitch P: lane l gets X(r0 + l%16, k0 + 8(l/16) + 0..7).  From
// an r-major operand (S[r P + k]) that is one 16-byte read.  From a k-major one
// (S[k P + r]) it takes two ds_read_b64_tr_b16: each lane of a 16-lane group reads
// 4 consecutive values of one k row, and the instruction hands lane i of the group
// value i%4 of lane 4j + i/4's read as its value j; lane 4j + q therefore reads row
// k + j at columns r0 + 4q.., which gives lane i the 4 k values of column r0 + i.
template <int MODE>
__device__ inline bf16x8 frag(const uint16_t *S, int P, int r0, int k0, int l) {
    if (MODE == LD_RVEC) {
        const int k = k0 + 8 * (l >> 4) + ((l & 15) >> 2), r = r0 + 4 * (l & 3);
        const i16x4 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)(&S[k * P + r]));
        const i16x4 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_i16x4 *)(&S[(k + 4) * P + r]));
        const i16x8 v = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
        return __builtin_bit_cast(bf16x8, v);
    } else {
        return *reinterpret_cast<const bf16x8 *>(&S[(r0 + (l & 15)) * P + k0 + 8 * (l >> 4)]);
    }
}

// COLS: thread t holds rows 8(t%8) + i of the A tile summed over its staged k; the 32
// threads of a row group are combined in thread order into colsum[m0 + ..] (colsum:
// this k chunk's partials).  red: 8 KB of LDS no longer read by the MFMA loop.
__device__ inline void colsum_finish(const float (&cs)[8], float *red, int t, int m0, int M, float *colsum) {
#pragma unroll
    for (int i = 0; i < 8; ++i) red[(t >> 3) * 64 + 8 * (t & 7) + i] = cs[i];
    __syncthreads();
    if (t < 64 && m0 + t < M) {
        float a = 0.f;
        for (int g = 0; g < 32; ++g) a += red[g * 64 + t];
        colsum[m0 + t] = a;
    }
}

// The epilogue of a wavefront's 32 x 32 output block (see gemm_kernel).
template <int EPI>
__device__ inline void gemm_epilogue(const f32x4 (&acc)[2][2], int m0, int n0, int wm, int wn, int l, int M, int N,
                                     float *__restrict__ C, long scm, long scn, uint16_t *__restrict__ Act,
                                     const float *__restrict__ bias) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + 4 * (l >> 4) + r;
                const int n = n0 + wn + 16 * j + (l & 15);
                if (m >= M || n >= N) continue;
                float v = acc[i][j][r];
                if (EPI == EPI_F32) {
                    if (gridDim.z > 1) C[size_t(m) * N + n] = v;
                    else C[m * scm + n * scn] = v;
                } else if (EPI == EPI_BIAS_F32) {
                    C[m * scm + n * scn] = v + bias[n];
                } else if (EPI == EPI_SILU_BACK) {
                    const float z = bias[size_t(m) * N + n], sg = sigmoidf_hw(z);
                    Act[size_t(m) * N + n] = bf16_bits(v * sg * (1.0f + z * (1.0f - sg)));
                } else {
                    const float z = v + bias[n];
                    C[m * scm + n * scn] = z;
                    Act[size_t(m) * N + n] = bf16_bits(z * sigmoidf_hw(z));
                }
            }
}

// EPI_SILU_BACK through LDS: the workgroup's 64 x 64 FP32 products go to LDS, then
// each thread takes 16 consecutive columns of one row, so the pre-activations are read
// and dZ written in 16-byte vectors (the arithmetic of gemm_epilogue, element by
// element).  tile: at least 64 x 68 floats of LDS that the k loop no longer reads.
// (Split-K partials written the same way measured slower than gemm_epilogue's.)
__device__ inline void silu_back_epilogue(const f32x4 (&acc)[2][2], float *tile, int m0, int n0, int wm, int wn,
                                          int l, int t, int M, int N, uint16_t *__restrict__ Act,
                                          const float *__restrict__ Z) {
    constexpr int TP = BN + 4;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) tile[(wm + 16 * i + 4 * (l >> 4) + r) * TP + wn + 16 * j + (l & 15)] = acc[i][j][r];
    __syncthreads();
    const int row = t >> 2, c0 = 16 * (t & 3), m = m0 + row;
    if (m >= M) return;
#pragma unroll
    for (int q = 0; q < 16; q += 8) {
        const int n = n0 + c0 + q;
        const float *v = tile + row * TP + c0 + q;
        if (N % 8 == 0 && n + 8 <= N) {
            const float4 za = *reinterpret_cast<const float4 *>(Z + size_t(m) * N + n);
            const float4 zb = *reinterpret_cast<const float4 *>(Z + size_t(m) * N + n + 4);
            const float zz[8] = {za.x, za.y, za.z, za.w, zb.x, zb.y, zb.z, zb.w};
            uint16_t h[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const float z = zz[c], sg = sigmoidf_hw(z);
                h[c] = bf16_bits(v[c] * sg * (1.0f + z * (1.0f - sg)));
            }
            *reinterpret_cast<uint4 *>(Act + size_t(m) * N + n) = pack8(h);
        } else {
            for (int c = 0; c < 8 && n + c < N; ++c) {
                const float z = Z[size_t(m) * N + n + c], sg = sigmoidf_hw(z);
                Act[size_t(m) * N + n + c] = bf16_bits(v[c] * sg * (1.0f + z * (1.0f - sg)));
            }
        }
    }
}

// XCD-aware tile order.  The hardware hands workgroup H (x fastest, then y, then z)
// to XCD H mod 8; with the tile count a multiple of 8, each XCD takes one contiguous
// range of the tiles in that order instead, so the workgroups that share operand rows
// (the column tiles of one row block; all tiles of one k chunk) run on the same XCD
// and read them through its L2 once.  Only which workgroup computes a tile changes.
constexpr int kNumXcd = 8;
__device__ inline void tile_of_block(int &bx, int &by, int &bz) {
    const int nx = int(gridDim.x), ny = int(gridDim.y), T = nx * ny * int(gridDim.z);
    int H = int(blockIdx.x) + nx * (int(blockIdx.y) + ny * int(blockIdx.z));
    if (T % kNumXcd == 0) H = (H % kNumXcd) * (T / kNumXcd) + H / kNumXcd;
    bx = H % nx;
    by = (H / nx) % ny;
    bz = H / (nx * ny);
}

// C = A B with A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn] (bfloat16 bits).
// 64x64 output tile per workgroup of four wavefronts, each wavefront 32x32 as
// 2x2 MFMA 16x16x32 tiles.  Lane l of a 16x16x32 MFMA supplies A[l%16][8(l/16)..+7]
// and B[8(l/16)..+7][l%16] and receives D[4(l/16)+r][l%16], r = 0..3.  k runs in
// 64-deep LDS tiles (two 32-deep MFMA steps each, in increasing k).
// Epilogues: EPI_F32 C(m,n) = acc; EPI_BIAS_F32 C = acc + bias[n];
// EPI_BIAS_SILU Z = acc + bias[n] (FP32 into C) and Act[m*N+n] = bf16(Z sigmoid(Z));
// EPI_SILU_BACK (backward through a SiLU; `bias` then points at the layer's FP32
// pre-activations z, row-major M x N): Act[m*N+n] = bf16(acc s (1 + z (1 - s))),
// s = sigmoid(z).
// Split-K: workgroup z covers k in [z*kchunk, (z+1)*kchunk) and (EPI_F32 only)
// writes its partial tile to C + z*M*N (row-major M x N); a reduction follows.
// COLS (EPI_F32 with A read along rows): the workgroups of the first column tile
// also sum A over their k range, colsum[z*M + m] = sum_k A(m, k) (a layer's bias
// gradient beside its weight gradient): each thread adds the 8 values it stages,
// tile by tile in increasing k, and the 32 threads of a row group are combined in
// thread order.
// Four wavefronts per SIMD (four workgroups per CU, which is also what the 36.9 KB of
// LDS allows): the k loop waits on global memory, so occupancy is what hides the
// latency (64-68 VGPRs with the staged values packed two per register).
template <int EPI, int AM, int BMODE, bool COLS = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void gemm_kernel(
    int M, int N, int K, const uint16_t *__restrict__ A, long sam, long sak, const uint16_t *__restrict__ B, long sbk,
    long sbn, float *__restrict__ C, long scm, long scn, uint16_t *__restrict__ Act, const float *__restrict__ bias,
    int kchunk, float *__restrict__ colsum) {
    static_assert(!COLS || (EPI == EPI_F32 && AM == LD_RVEC), "column sums of an A tile staged along rows");
    static_assert(BM == BK && BN == BK, "a k-major tile reuses the r-major tile's array");
    __shared__ __attribute__((aligned(16))) uint16_t As[2][BM][BKP];
    __shared__ __attribute__((aligned(16))) uint16_t Bt[2][BN][BKP];
    int bx, by, bz;
    tile_of_block(bx, by, bz);
    const int m0 = by * BM, n0 = bx * BN;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kb = bz * kchunk, ke = min(K, kb + kchunk);
    if (gridDim.z > 1) C += size_t(bz) * M * N;
    const int ntiles = ke > kb ? (ke - kb + BK - 1) / BK : 0;
    const bool cols = COLS && bx == 0;
    float cs[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    TileRegs qa[2], qb[2];
    // double-buffered 64-deep k tiles: tile t + 1 is read from global memory into
    // registers while tile t is multiplied out of LDS; one barrier per tile
    if (ntiles > 0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            tile_load<AM>(qa[h], A, sam, sak, m0, M, kb, ke, t, h);
            tile_load<BMODE>(qb[h], B, sbn, sbk, n0, N, kb, ke, t, h);
            tile_store<AM>(qa[h], &As[0][0][0], BKP, 0, t, h);
            tile_store<BMODE>(qb[h], &Bt[0][0][0], BKP, 0, t, h);
            if (cols)
#pragma unroll
                for (int i = 0; i < 8; ++i) cs[i] += tile_value(qa[h], i);
        }
    }
    __syncthreads();
    for (int tk = 0; tk < ntiles; ++tk) {
        const int k0 = kb + tk * BK, cur = tk & 1;
        const bool more = tk + 1 < ntiles;
        if (more) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                tile_load<AM>(qa[h], A, sam, sak, m0, M, k0 + BK, ke, t, h);
                tile_load<BMODE>(qb[h], B, sbn, sbk, n0, N, k0 + BK, ke, t, h);
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (k0 + 32 * h >= ke) break;        // the same 32-deep MFMA steps as a 32-deep loop
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const bf16x8 a = frag<AM>(&As[cur][0][0], BKP, wm + 16 * i, 32 * h, l);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf16x8 b = frag<BMODE>(&Bt[cur][0][0], BKP, wn + 16 * j, 32 * h, l);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
                }
            }
        }
        if (more) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                tile_store<AM>(qa[h], &As[cur ^ 1][0][0], BKP, 0, t, h);
                tile_store<BMODE>(qb[h], &Bt[cur ^ 1][0][0], BKP, 0, t, h);
                if (cols)
#pragma unroll
                    for (int i = 0; i < 8; ++i) cs[i] += tile_value(qa[h], i);
            }
        }
        __syncthreads();
    }
    if (cols) colsum_finish(cs, reinterpret_cast<float *>(&As[0][0][0]), t, m0, M, colsum + size_t(bz) * M);
    if constexpr (EPI == EPI_SILU_BACK) {
        static_assert(sizeof(As) >= sizeof(float) * BM * (BN + 4), "the FP32 tile fits in the A tiles' LDS");
        silu_back_epilogue(acc, reinterpret_cast<float *>(&As[0][0][0]), m0, n0, wm, wn, l, t, M, N, Act, bias);
    } else {
        gemm_epilogue<EPI>(acc, m0, n0, wm, wn, l, M, N, C, scm, scn, Act, bias);
    }
}

// Fixed-order sum of split-K partials (nz x M x N, row-major) into C(m, n); with
// bout, the elements past M x N are the column-sum partials (nz x M), summed into
// bout[m].  A block takes 64 elements; wavefront w adds partials w, w + 4, ... in
// order (64 consecutive elements per load), and the four sums are combined as
// (s0 + s1) + (s2 + s3).
__global__ __launch_bounds__(kThreads) void splitk_reduce_kernel(int nz, int M, int N, const float *__restrict__ part,
                                                                 float *__restrict__ C, long scm, long scn,
                                                                 const float *__restrict__ bpart,
                                                                 float *__restrict__ bout) {
    __shared__ float sh[4][64];
    const long MN = long(M) * N, E = MN + (bout ? M : 0);
    const int w = threadIdx.x >> 6, c = threadIdx.x & 63;
    const long i = long(blockIdx.x) * 64 + c;
    float s = 0.f;
    if (i < MN) {
#pragma unroll 8
        for (int z = w; z < nz; z += 4) s += part[size_t(z) * MN + i];   // loads in flight, additions in order
    } else if (i < E) {
#pragma unroll 8
        for (int z = w; z < nz; z += 4) s += bpart[size_t(z) * M + (i - MN)];
    }
    sh[w][c] = s;
    __syncthreads();
    if (w == 0 && i < E) {
        const float v = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
        if (i < MN) {
            const long m = i / N, n = i % N;
            C[m * scm + n * scn] = v;
        } else {
            bout[i - MN] = v;
        }
    }
}

// Output layer's gradient for n_out <= kOutMax, one pass over the last hidden
// activations: part[c][o W + j] = sum over the rows r of chunk c of dY(r, o) a(r, j),
// and part[c][n_out W + o] = sum_r dY(r, o) (the bias).  Products of two bfloat16
// values are exact in FP32.  A thread takes four adjacent columns and every fourth
// row of a block of 64 (its 16 loads in flight at once, dY of the block in LDS);
// rows in increasing order per thread, then the four row phases combined in order.
constexpr int kOutMax = 8;
__global__ __launch_bounds__(kThreads) void out_grad_partial_kernel(long n, int W, int no, long rows,
                                                                    const uint16_t *__restrict__ dY,
                                                                    const uint16_t *__restrict__ Aact,
                                                                    float *__restrict__ part) {
    __shared__ float dys[64][kOutMax];
    __shared__ float red[4][64][4 * kOutMax + kOutMax];
    const int t = threadIdx.x, cq = t & 63, ph = t >> 6;
    const long r0 = long(blockIdx.x) * rows, r1 = min(n, r0 + rows);
    float *out = part + size_t(blockIdx.x) * no * (W + 1);
    for (int cb = 0; cb < W; cb += 256) {
        const int j = cb + 4 * cq;
        const bool on = j < W;
        float acc[4][kOutMax], bacc[kOutMax];
#pragma unroll
        for (int o = 0; o < kOutMax; ++o) {
            bacc[o] = 0.f;
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c][o] = 0.f;
        }
        for (long b0 = r0; b0 < r1; b0 += 64) {
            const int nb = int(min(64L, r1 - b0));
            __syncthreads();
            for (int e = t; e < 64 * kOutMax; e += kThreads) {
                const int rr = e / kOutMax, o = e % kOutMax;
                dys[rr][o] = (rr < nb && o < no) ? bf2f(dY[(b0 + rr) * no + o]) : 0.f;
            }
            __syncthreads();
            uint2 av[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int rr = ph + 4 * i;
                av[i] = (on && rr < nb) ? *reinterpret_cast<const uint2 *>(Aact + (b0 + rr) * W + j) : uint2{0u, 0u};
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int rr = ph + 4 * i;
                const float a[4] = {bf2f(uint16_t(av[i].x & 0xffffu)), bf2f(uint16_t(av[i].x >> 16)),
                                    bf2f(uint16_t(av[i].y & 0xffffu)), bf2f(uint16_t(av[i].y >> 16))};
#pragma unroll
                for (int o = 0; o < kOutMax; ++o) {
                    const float d = dys[rr][o];   // zero past the block's rows and n_out
                    bacc[o] += d;
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c][o] += d * a[c];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < kOutMax; ++o) {
#pragma unroll
            for (int c = 0; c < 4; ++c) red[ph][cq][c * kOutMax + o] = acc[c][o];
            red[ph][cq][4 * kOutMax + o] = bacc[o];
        }
        __syncthreads();
        // the 64 column quads' 5 kOutMax values each, finished by the threads in turn
        for (int e = t; e < 64 * 5 * kOutMax; e += kThreads) {
            const int q = e / (5 * kOutMax), v = e % (5 * kOutMax);
            const float sum = ((red[0][q][v] + red[1][q][v]) + red[2][q][v]) + red[3][q][v];
            if (v < 4 * kOutMax) {
                const int c = v / kOutMax, o = v % kOutMax, jj = cb + 4 * q + c;
                if (o < no && jj < W) out[size_t(o) * W + jj] = sum;
            } else if (cb == 0 && q == 0 && v - 4 * kOutMax < no) {
                out[size_t(no) * W + (v - 4 * kOutMax)] = sum;
            }
        }
    }
}

// Fixed-order sum of nparts partial vectors of length L: sixteen threads per
// element, thread q adding parts q, q + 16, ... in order, the sixteen sums then
// added in thread order.
__global__ __launch_bounds__(kThreads) void parts_reduce_kernel(int nparts, long L, const float *__restrict__ part,
                                                                float *__restrict__ out) {
    __shared__ float sh[16][17];
    const int q = threadIdx.x & 15, el = threadIdx.x >> 4;
    const long e = long(blockIdx.x) * 16 + el;
    float a = 0.f;
    if (e < L) {
#pragma unroll 8
        for (int c = q; c < nparts; c += 16) a += part[size_t(c) * L + e];
    }
    sh[el][q] = a;
    __syncthreads();
    if (q == 0 && e < L) {
        float sum = 0.f;
        for (int k = 0; k < 16; ++k) sum += sh[el][k];
        out[e] = sum;
    }
}

// Row chunks of the output layer's gradient: (rows per chunk, chunks), at least
// kColChunk rows and at most 1024 chunks.
std::pair<long, long> out_grad_chunks(long n) {
    const long rows = std::max<long>(kColChunk, (n + 1023) / 1024);
    return {rows, (n + rows - 1) / rows};
}

// dZ of the last hidden layer for n_out <= kOutMax: (dY W_O)(r, j) = sum_o dY(r, o) W_O(o, j)
// in increasing o, through the SiLU at z(r, j) (the arithmetic of the GEMM epilogue).
// Eight columns per thread (W is a multiple of 64): 16-byte weight loads and dZ stores.
__global__ void out_back_kernel(long n, int W, int no, const uint16_t *__restrict__ dY,
                                const uint16_t *__restrict__ WO, const float *__restrict__ Z,
                                uint16_t *__restrict__ dZ) {
    const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x;
    const int q = W / 8;
    if (idx >= n * q) return;
    const long r = idx / q;
    const int j = 8 * int(idx % q);
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int o = 0; o < kOutMax; ++o)
        if (o < no) {
            const float d = bf2f(dY[r * no + o]);
            const TileRegs wv{*reinterpret_cast<const uint4 *>(WO + size_t(o) * W + j)};
#pragma unroll
            for (int c = 0; c < 8; ++c) v[c] += d * tile_value(wv, c);
        }
    const float4 za = *reinterpret_cast<const float4 *>(Z + r * W + j);
    const float4 zb = *reinterpret_cast<const float4 *>(Z + r * W + j + 4);
    const float zz[8] = {za.x, za.y, za.z, za.w, zb.x, zb.y, zb.z, zb.w};
    uint16_t h[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float z = zz[c], sg = sigmoidf_hw(z);
        h[c] = bf16_bits(v[c] * sg * (1.0f + z * (1.0f - sg)));
    }
    *reinterpret_cast<uint4 *>(dZ + r * W + j) = pack8(h);
}

// Features of sample i: [sin(2 pi B x_i), cos(2 pi B x_i), p_i, 0 ...] as bfloat16 (row of K0).
__global__ void features_kernel(long n, const float *__restrict__ x, const float *__restrict__ p,
                                const float *__restrict__ Bf, int nf, int np, int K0, uint16_t *__restrict__ out) {
    const long idx = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * K0) return;
    const long i = idx / K0;
    const int j = int(idx % K0);
    float v = 0.f;
    if (j < 2 * nf) {
        const int f = j < nf ? j : j - nf;
        v = fourier_feature(Bf[3 * f] * x[3 * i] + Bf[3 * f + 1] * x[3 * i + 1] + Bf[3 * f + 2] * x[3 * i + 2],
                            j < nf);
    } else if (j < 2 * nf + np) {
        v = p[i * np + (j - 2 * nf)];
    }
    out[idx] = bf16_bits(v);
}

// dY = 2 (Y - T) / (n n_out) (bfloat16) and per-block sums of (Y - T)^2.
__global__ void loss_grad_kernel(long n, int nout, const float *__restrict__ Y, const float *__restrict__ T,
                                 uint16_t *__restrict__ dY, float *__restrict__ part) {
    __shared__ float sh[kThreads];
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    float e2 = 0.f;
    if (i < n * nout) {
        const float d = Y[i] - T[i];
        e2 = d * d;
        dY[i] = bf16_bits(2.0f * d / float(n * nout));
    }
    sh[threadIdx.x] = e2;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Fixed-order sum of nparts partials, times scale, into out[0].
__global__ void sum_kernel(int nparts, const float *__restrict__ part, float scale, float *__restrict__ out) {
    __shared__ float sh[kThreads];
    float s = 0.f;
    for (int i = threadIdx.x; i < nparts; i += kThreads) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = kThreads / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0] * scale;
}

// Column sums of a bfloat16 M x N matrix in chunks of rows (at least kColChunk
// rows each): part[c][j] (short chunks: enough workgroups to keep the loads in flight).
__global__ void colsum_partial_kernel(long M, int N, const uint16_t *__restrict__ X, float *__restrict__ part,
                                      long chunk) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const long r0 = long(blockIdx.y) * chunk;
    if (j >= N) return;
    float s = 0.f;
    const long r1 = std::min(M, r0 + chunk);
#pragma unroll 8
    for (long r = r0; r < r1; ++r) s += bf2f(X[r * N + j]);        // loads in flight, additions in order
    part[size_t(blockIdx.y) * N + j] = s;
}

// Fixed-order sum of the chunk partials: a block covers 64 columns with four
// threads per column; thread q sums chunks q, q + 4, q + 8, ... in order, and the
// four sums are combined as (s0 + s1) + (s2 + s3).
__global__ __launch_bounds__(kThreads) void colsum_final_kernel(int nchunks, int N, const float *__restrict__ part,
                                                                float *__restrict__ out) {
    __shared__ float sh[4][64];
    const int c = blockIdx.x * 64 + (threadIdx.x & 63), q = threadIdx.x >> 6;
    float a = 0.f;
    if (c < N) {
#pragma unroll 8
        for (int ch = q; ch < nchunks; ch += 4) a += part[size_t(ch) * N + c];
    }
    sh[q][threadIdx.x & 63] = a;
    __syncthreads();
    if (q == 0 && c < N) {
        const int j = threadIdx.x & 63;
        out[c] = (sh[0][j] + sh[1][j]) + (sh[2][j] + sh[3][j]);
    }
}

// Adam on the FP32 master parameters; refreshes the bfloat16 copy.
__global__ void adam_kernel(long P, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, float lr, float c1, float c2, uint16_t *__restrict__ wb) {
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    w[i] = wi;
    wb[i] = bf16_bits(wi);
}

__global__ void to_bf16_kernel(long n, const float *__restrict__ x, uint16_t *__restrict__ y) {
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) y[i] = bf16_bits(x[i]);
}

// Whole-network inference, 64 samples per workgroup of four wavefronts; the
// activations never leave LDS.  Features are formed in LDS as in
// features_kernel.  Each hidden layer computes its output transposed,
// Z^T = W A^T + b, with W (bfloat16, row-major out x in) streamed from global
// memory straight into the MFMA A operand (8 consecutive k of one unit per lane)
// and A (64 x K) read from LDS as the B operand; wavefront w owns units
// [w W/4, (w+1) W/4), and each lane ends with 4 consecutive units of one sample,
// written back as one 8-byte store of bf16(SiLU(z)).  All waves finish reading A
// before any writes over it.  The output layer gives wavefront w samples
// [16w, 16w + 16).  Every output is the same k-ordered sum of the same products
// as in gemm_kernel, with the same epilogue arithmetic, so the result equals the
// layer-by-layer forward pass bit for bit (tested).  Registers are capped for
// three waves per SIMD (152 VGPRs for width 256, no spills): at millions of
// samples the extra wave hides more of the weight-load latency.
constexpr int kFusedRows = 64;
constexpr int kFusedMaxDepth = 8;
struct NetOffsets {
    long w[kFusedMaxDepth + 1];
    long b[kFusedMaxDepth + 1];
};
// The training forward keeps what the backward pass reads: the features (bf16,
// n x K0) and every hidden layer's FP32 pre-activation and bf16 activation
// (n x W, row-major), the same arrays the layer-by-layer GEMMs write.
struct TrainStore {
    uint16_t *x0;
    float *z[kFusedMaxDepth];
    uint16_t *a[kFusedMaxDepth];
};

// Z^T (16 NT units x 64 samples per wavefront) = W A^T with A (64 x K, LDS), K
// in steps of 32: the weights are the MFMA A operand and the activations the B
// operand, so each lane ends with 4 consecutive units of one sample.  The
// weight fragments of step k + 32 are requested before the MFMAs of step k.
template <int NT>
__device__ __forceinline__ void fused_k_step(f32x4 (&acc)[4][NT], const uint16_t *act, int P, const uint16_t *wrow,
                                             int K, int ldw, int k0, bf16x8 (&bn)[NT], int l) {
    bf16x8 b[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) b[j] = bn[j];
    if (k0 + 32 < K) {
#pragma unroll
        for (int j = 0; j < NT; ++j) bn[j] = *reinterpret_cast<const bf16x8 *>(wrow + long(16 * j) * ldw + k0 + 32);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&act[(16 * i + (l & 15)) * P + k0 + 8 * (l >> 4)]);
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b[j], a, acc[i][j], 0, 0, 0);
    }
}

// Z^T (16 NT units x 64 samples per wavefront) = W A^T with A (64 x K, LDS), K
// in steps of 32: the weights are the MFMA A operand and the activations the B
// operand, so each lane ends with 4 consecutive units of one sample.  The
// weight fragments of step k + 32 are requested before the MFMAs of step k.
// KFIX > 0: K = KFIX known at compile time (the loop unrolls fully).
template <int NT, int KFIX>
__device__ __forceinline__ void fused_layer_k(f32x4 (&acc)[4][NT], const uint16_t *act, int P, const uint16_t *Wl,
                                              int K, int nb, int l) {
    const int ldw = KFIX > 0 ? KFIX : K;
    const uint16_t *wrow = Wl + long(nb + (l & 15)) * ldw + 8 * (l >> 4);
    bf16x8 bn[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) bn[j] = *reinterpret_cast<const bf16x8 *>(wrow + long(16 * j) * ldw);
    if constexpr (KFIX > 0) {
#pragma unroll
        for (int k0 = 0; k0 < KFIX; k0 += 32) fused_k_step<NT>(acc, act, P, wrow, KFIX, KFIX, k0, bn, l);
    } else {
        for (int k0 = 0; k0 < K; k0 += 32) fused_k_step<NT>(acc, act, P, wrow, K, K, k0, bn, l);
    }
}

// TRAIN: also stores the features, pre-activations and activations (TrainStore)
// for the backward pass.
template <int W, bool TRAIN, int NW = 4>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(3))) void fused_forward_kernel(long n, const float *__restrict__ x,
                                                                 const float *__restrict__ p,
                                                                 const float *__restrict__ Bf, int nf, int np,
                                                                 int K0, int depth, int nout,
                                                                 const uint16_t *__restrict__ wb,
                                                                 const float *__restrict__ wf, NetOffsets off,
                                                                 float *__restrict__ out, TrainStore ts) {
    extern __shared__ __attribute__((aligned(16))) uint16_t act[];
    const int P = (K0 > W ? K0 : W) + 8;          // LDS row pitch (elements)
    const long r0 = long(blockIdx.x) * kFusedRows;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    for (int idx = t; idx < kFusedRows * K0; idx += 64 * NW) {
        const int row = idx / K0, j = idx % K0;
        const long i = r0 + row;
        float v = 0.f;
        if (i < n) {
            if (j < 2 * nf) {
                const int f = j < nf ? j : j - nf;
                v = fourier_feature(
                    Bf[3 * f] * x[3 * i] + Bf[3 * f + 1] * x[3 * i + 1] + Bf[3 * f + 2] * x[3 * i + 2], j < nf);
            } else if (j < 2 * nf + np) {
                v = p[i * np + (j - 2 * nf)];
            }
        }
        const uint16_t bits = bf16_bits(v);
        act[row * P + j] = bits;
        if (TRAIN && i < n) ts.x0[i * K0 + j] = bits;
    }
    __syncthreads();
    constexpr int NT = W / (16 * NW);              // 16-column tiles per wavefront
    static_assert(NT >= 1, "at least one 16-unit tile per wavefront");
    const int nb = w * (W / NW);
    for (int layer = 0; layer < depth; ++layer) {
        const uint16_t *Wl = wb + off.w[layer];
        f32x4 acc[4][NT];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        if (layer == 0) {
            fused_layer_k<NT, 0>(acc, act, P, Wl, K0, nb, l);
        } else {
            fused_layer_k<NT, W>(acc, act, P, Wl, W, nb, l);
        }
        __syncthreads();
        const float *bias = wf + off.b[layer];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int u0 = nb + 16 * j + 4 * (l >> 4);              // 4 consecutive units
            const float4 bc = *reinterpret_cast<const float4 *>(bias + u0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * i + (l & 15);                  // sample
                const float z0 = acc[i][j][0] + bc.x, z1 = acc[i][j][1] + bc.y;
                const float z2 = acc[i][j][2] + bc.z, z3 = acc[i][j][3] + bc.w;
                uint2 q;
                q.x = uint32_t(bf16_bits(z0 * sigmoidf_hw(z0))) | (uint32_t(bf16_bits(z1 * sigmoidf_hw(z1))) << 16);
                q.y = uint32_t(bf16_bits(z2 * sigmoidf_hw(z2))) | (uint32_t(bf16_bits(z3 * sigmoidf_hw(z3))) << 16);
                *reinterpret_cast<uint2 *>(&act[row * P + u0]) = q;
                if (TRAIN && r0 + row < n) {
                    const size_t o = size_t(r0 + row) * W + u0;
                    *reinterpret_cast<float4 *>(ts.z[layer] + o) = make_float4(z0, z1, z2, z3);
                    *reinterpret_cast<uint2 *>(ts.a[layer] + o) = q;
                }
            }
        }
        __syncthreads();
    }
    // output layer: rows [16w, 16w + 16) for the first four wavefronts, up to four 16-column tiles
    if (w >= 4) return;
    const uint16_t *Wo = wb + off.w[depth];
    const float *bo = wf + off.b[depth];
    f32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int ntile = (nout + 15) / 16;
    for (int k0 = 0; k0 < W; k0 += 32) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(&act[(16 * w + (l & 15)) * P + k0 + 8 * (l >> 4)]);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j >= ntile) break;
            const int col = 16 * j + (l & 15);
            bf16x8 b;
            if (col < nout) {
                b = *reinterpret_cast<const bf16x8 *>(Wo + long(col) * W + k0 + 8 * (l >> 4));
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) b[q] = __bf16(0.0f);
            }
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (j >= ntile) break;
        const int col = 16 * j + (l & 15);
        if (col >= nout) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const long row = r0 + 16 * w + 4 * (l >> 4) + r;
            if (row < n) out[row * nout + col] = acc[j][r] + bo[col];
        }
    }
}

// Ensemble statistics over K members' outputs (K x n x n_out, member-major):
// mean[i][o] = scale[o] (sum_k out[k][i][o]) / K and
// spread[i] = scale[0] (max_k out[k][i][0] - min_k out[k][i][0]); members summed in order.
__global__ void ensemble_stats_kernel(long n, int K, int nout, const float *__restrict__ outs,
                                      const float *__restrict__ scale, float *__restrict__ mean,
                                      float *__restrict__ spread) {
    const long i = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float invK = 1.0f / float(K);
    for (int o = 0; o < nout; ++o) {
        float s = 0.f, lo = INFINITY, hi = -INFINITY;
        for (int k = 0; k < K; ++k) {
            const float v = outs[(size_t(k) * n + i) * nout + o];
            s += v;
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
        }
        mean[i * nout + o] = scale[o] * s * invK;
        if (o == 0) spread[i] = scale[0] * (hi - lo);
    }
}

// Scenario of row r: the s with row_begin[s] <= r < row_begin[s + 1] (binary
// search over the n_scen + 1 offsets; rows of empty scenarios never occur).
__device__ inline int scenario_of(const int64_t *__restrict__ row_begin, int n_scen, int64_t r) {
    int lo = 0, hi = n_scen - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_begin[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Network inputs of many scenarios in one pass over their nodes: coordinates
// relative to the scenario's probe in units of its coordinate scale, and the
// parameter row (coordinates times p_scale, then the scenario's constants).
// The coordinate arithmetic is FP64, rounded once to FP32.
__global__ void scenario_inputs_kernel(int n_scen, int n_prm, const int64_t *__restrict__ row_begin,
                                       const double *__restrict__ X, const double *__restrict__ probe,
                                       const double *__restrict__ xi, double p_scale, const float *__restrict__ prm,
                                       float *__restrict__ x_out, float *__restrict__ p_out) {
#pragma clang fp contract(off)
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= row_begin[n_scen]) return;
    const int sc = scenario_of(row_begin, n_scen, r);
    const int w = 3 + n_prm;
    for (int i = 0; i < 3; ++i) {
        const double x = X[3 * r + i];
        const double rel = x - probe[3 * sc + i];
        x_out[3 * r + i] = float(rel * xi[sc]);
        p_out[w * r + i] = float(x * p_scale);
    }
    for (int k = 0; k < n_prm; ++k) p_out[w * r + 3 + k] = prm[size_t(n_prm) * sc + k];
}

// Ensemble mean and spread (scaled targets) to physical fields of each row's
// scenario, in FP32 with one rounding per operation (no fused multiply-add):
// T = T0 + sT * m0, u = su * m1..3, spread_K = sT * spread.
__global__ void scenario_outputs_kernel(int n_scen, const int64_t *__restrict__ row_begin,
                                        const float *__restrict__ mean, const float *__restrict__ spread,
                                        const float *__restrict__ T0, const float *__restrict__ sT,
                                        const float *__restrict__ su, float *__restrict__ T_out,
                                        float *__restrict__ u_out, float *__restrict__ spread_out) {
    // plain operators under contract(off): hipcc would otherwise form an FMA
    // (its rounding intrinsics are header functions the pragma does not reach)
#pragma clang fp contract(off)
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= row_begin[n_scen]) return;
    const int sc = scenario_of(row_begin, n_scen, r);
    const float rise = sT[sc] * mean[4 * r];
    T_out[r] = T0[sc] + rise;
    for (int i = 0; i < 3; ++i) u_out[3 * r + i] = su[sc] * mean[4 * r + 1 + i];
    spread_out[r] = sT[sc] * spread[r];
}

inline unsigned blocks(long n) { return unsigned((n + kThreads - 1) / kThreads); }

struct Layer {
    int in, out;      // in: padded input width
    long w_off, b_off;
};

}  // namespace

// Split-K partials of tled_mlp_gemm_static: a static device array (each GPU the
// library runs on holds its own copy for the life of the process).  Host code
// never passes `scratch` itself (on the host it names a stand-in, not a device
// address): its per-device address comes from hipGetSymbolAddress, taken once
// per device with that device current, when a handle is created there.  With
// the split rule of gemm() (nz x output tiles <= 512, 64 x 64 tiles) the
// partials never exceed 512 x 4096 floats, which is this array's size.
constexpr size_t kStaticSplitFloats = size_t(512) * 64 * 64;
static __device__ __align__(256) float scratch[kStaticSplitFloats];

namespace {
std::mutex g_scratch_mu;
std::vector<float *> g_scratch_addr;   // device ordinal -> address of `scratch` on that device

// Call with `device` current.
tled_status resolve_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (size_t(device) >= g_scratch_addr.size()) g_scratch_addr.resize(size_t(device) + 1, nullptr);
    if (g_scratch_addr[device]) return TLED_OK;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TLED_E_HIP;
    g_scratch_addr[device] = static_cast<float *>(p);
    return TLED_OK;
}
}  // namespace

struct tled_mlp {
    int device = 0;
    int cus = 256;                     // compute units of the device
    float *d_static_split = nullptr;   // this device's `scratch` (resolved at creation)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    tled_mlp_config cfg{};
    int K0 = 0;
    std::vector<Layer> layers;
    long P = 0;
    std::vector<float> freq;
    float *d_w = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr, *d_freq = nullptr;
    uint16_t *d_wb = nullptr;
    long adam_t = 0;
    // workspace for up to cap samples
    long cap = 0;
    uint16_t *d_x0 = nullptr;
    std::vector<float *> d_z;        // per hidden layer, cap x width
    std::vector<uint16_t *> d_a;     // per hidden layer, cap x width
    float *d_y = nullptr, *d_part = nullptr, *d_loss = nullptr, *d_cpart = nullptr;
    uint16_t *d_dy = nullptr, *d_dz = nullptr, *d_dz2 = nullptr;   // dZ of two adjacent layers
    std::vector<void *> ws;
    std::string err;
    float *d_split = nullptr;        // split-K partials
    size_t split_cap = 0;
    // timing
    bool timing = false;
    double gemm_ms = 0.0, fused_ms = 0.0, gemm_flops = 0.0, fused_flops = 0.0;
};

namespace {

tled_status mfail(tled_mlp *s, tled_status st, const std::string &m) {
    if (s) s->err = m;
    return st;
}

#define MCHK(s, expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return mfail(s, TLED_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MTRY(expr)                        \
    do {                                  \
        tled_status st_ = (expr);         \
        if (st_ != TLED_OK) return st_;   \
    } while (0)

uint64_t splitmix(uint64_t &s) {
    uint64_t z = (s += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
double uniform01(uint64_t &s) { return double(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

void free_ws(tled_mlp *s) {
    for (void *p : s->ws) (void)hipFree(p);
    s->ws.clear();
    s->d_z.clear();
    s->d_a.clear();
    s->cap = 0;
}

template <typename T>
tled_status walloc(tled_mlp *s, T **p, size_t n) {
    void *q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return mfail(s, TLED_E_OOM, "hipMalloc failed");
    s->ws.push_back(q);
    *p = static_cast<T *>(q);
    return TLED_OK;
}

tled_status ensure_workspace(tled_mlp *s, long n) {
    if (n <= s->cap) return TLED_OK;
    MCHK(s, hipStreamSynchronize(s->stream));
    free_ws(s);
    const long W = s->cfg.width, no = s->cfg.n_out;
    const long cap = std::max<long>(n, 1024);
    MTRY(walloc(s, &s->d_x0, size_t(cap) * s->K0));
    for (int l = 0; l < s->cfg.depth; ++l) {
        float *z;
        uint16_t *a;
        MTRY(walloc(s, &z, size_t(cap) * W));
        MTRY(walloc(s, &a, size_t(cap) * W));
        s->d_z.push_back(z);
        s->d_a.push_back(a);
    }
    MTRY(walloc(s, &s->d_y, size_t(cap) * no));
    MTRY(walloc(s, &s->d_dy, size_t(cap) * no));
    MTRY(walloc(s, &s->d_dz, size_t(cap) * W));
    MTRY(walloc(s, &s->d_dz2, size_t(cap) * W));
    MTRY(walloc(s, &s->d_part, size_t(blocks(cap * no))));
    MTRY(walloc(s, &s->d_loss, 1));
    MTRY(walloc(s, &s->d_cpart, std::max(size_t((cap + kColChunk - 1) / kColChunk) * std::max<long>(W, no),
                                         size_t(std::min<long>(1024, (cap + kColChunk - 1) / kColChunk)) * no *
                                             (W + 1))));   // the most chunks out_grad_chunks(n <= cap) makes
    s->cap = cap;
    return TLED_OK;
}

// Vector loads need 16-byte aligned vectors: base aligned and the strided axis a multiple of 8.
int load_mode(const uint16_t *X, long sr, long sk) {
    if (reinterpret_cast<uintptr_t>(X) % 16 != 0) return LD_SCALAR;
    if (sk == 1 && sr % 8 == 0) return LD_KVEC;
    if (sr == 1 && sk % 8 == 0) return LD_RVEC;
    return LD_SCALAR;
}

// split_ext: split-K partials in a caller-held buffer of split_ext_cap floats
// (nothing is allocated and no timing events are created); else the handle's
// buffer, grown on demand.  colsum (EPI_F32, both operands read along rows): also
// colsum[m] = sum_k A(m, k), from the same staged tiles.  Split-K (EPI_F32, fewer
// than 256 output tiles): about split_target workgroups (nz x tiles), at most 64 x
// split_target / 512 k chunks.  The entry points keep 512; the weight gradients
// of training ask for 1024 (their k loops are latency bound: more, shorter chunks
// measured faster despite the larger partials).
template <int EPI>
tled_status gemm(tled_mlp *s, int M, int N, int K, const uint16_t *A, long sam, long sak, const uint16_t *B,
                 long sbk, long sbn, float *C, long scm, long scn, uint16_t *Act, const float *bias,
                 float *split_ext = nullptr, size_t split_ext_cap = 0, float *colsum = nullptr,
                 int split_target = 512) {
    const long tiles = long((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    int nz = 1;
    if (EPI == EPI_F32 && tiles < 256 && K >= 4 * BK)
        nz = int(std::min<long>(64L * split_target / 512, std::max<long>(1, split_target / tiles)));
    int kchunk = ((K + nz - 1) / nz + BK - 1) / BK * BK;
    nz = (K + kchunk - 1) / kchunk;
    const int am = load_mode(A, sam, sak), bmode = load_mode(B, sbn, sbk);
    if (colsum && (EPI != EPI_F32 || am != LD_RVEC || bmode != LD_RVEC || split_ext))
        return mfail(s, TLED_E_ARG, "column sums need both operands read along rows");
    float *split = s->d_split;
    if (nz > 1 && split_ext) {
        const size_t need = size_t(nz) * M * N;
        if (need > split_ext_cap)
            return mfail(s, TLED_E_ARG, "split-K partials of " + std::to_string(need) + " floats exceed the " +
                                            std::to_string(split_ext_cap) + " of the static scratch array");
        split = split_ext;
    } else if (nz > 1) {
        const size_t need = size_t(nz) * M * N + (colsum ? size_t(nz) * M : 0);
        if (need > s->split_cap) {
            MCHK(s, hipStreamSynchronize(s->stream));   // earlier launches may still use the old buffer
            if (s->d_split) (void)hipFree(s->d_split);
            s->d_split = nullptr;
            s->split_cap = 0;
            void *p = nullptr;
            if (hipMalloc(&p, need * sizeof(float)) != hipSuccess) return mfail(s, TLED_E_OOM, "hipMalloc failed");
            s->d_split = static_cast<float *>(p);
            s->split_cap = need;
        }
        split = s->d_split;
    }
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, nz);
    float *cpart = colsum && nz > 1 ? split + size_t(nz) * M * N : colsum;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = s->timing && !split_ext;
    if (timed) {
        MCHK(s, hipEventCreate(&e0));
        MCHK(s, hipEventCreate(&e1));
        MCHK(s, hipEventRecord(e0, s->stream));
    }
    float *Cout = nz > 1 ? split : C;
#define TLED_GEMM_LAUNCH(AMODE, BMODE_, COLS)                                                                 \
    hipLaunchKernelGGL((gemm_kernel<EPI, AMODE, BMODE_, COLS>), grid, dim3(kThreads), 0, s->stream, M, N, K, A, sam, \
                       sak, B, sbk, sbn, Cout, scm, scn, Act, bias, kchunk, cpart)
    bool launched = false;
    if constexpr (EPI == EPI_F32) {
        if (colsum) {
            TLED_GEMM_LAUNCH(LD_RVEC, LD_RVEC, true);
            launched = true;
        }
    }
    if (launched) {
    } else if (am == LD_KVEC && bmode == LD_KVEC) TLED_GEMM_LAUNCH(LD_KVEC, LD_KVEC, false);
    else if (am == LD_KVEC && bmode == LD_RVEC) TLED_GEMM_LAUNCH(LD_KVEC, LD_RVEC, false);
    else if (am == LD_RVEC && bmode == LD_RVEC) TLED_GEMM_LAUNCH(LD_RVEC, LD_RVEC, false);
    else if (am == LD_RVEC && bmode == LD_KVEC) TLED_GEMM_LAUNCH(LD_RVEC, LD_KVEC, false);
    else TLED_GEMM_LAUNCH(LD_SCALAR, LD_SCALAR, false);
#undef TLED_GEMM_LAUNCH
    if (nz > 1)
        hipLaunchKernelGGL(splitk_reduce_kernel, dim3(unsigned((long(M) * N + (colsum ? M : 0) + 63) / 64)),
                           dim3(kThreads), 0, s->stream, nz, M, N, split, C, scm, scn, cpart, colsum);
    MCHK(s, hipGetLastError());
    if (timed) {
        MCHK(s, hipEventRecord(e1, s->stream));
        MCHK(s, hipEventSynchronize(e1));
        float ms = 0.f;
        MCHK(s, hipEventElapsedTime(&ms, e0, e1));
        s->gemm_ms += ms;
        s->gemm_flops += 2.0 * double(M) * N * K;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return TLED_OK;
}

// Fused inference applies to widths 64/128/256, depth <= 8, and LDS rows that fit.
size_t fused_lds_bytes(const tled_mlp *s) {
    return size_t(kFusedRows) * (std::max(s->K0, s->cfg.width) + 8) * sizeof(uint16_t);
}

bool fused_ok(const tled_mlp *s) {
    const int W = s->cfg.width;
    return !s->cfg.layerwise && (W == 64 || W == 128 || W == 256) && s->cfg.depth <= kFusedMaxDepth &&
           fused_lds_bytes(s) <= 64 * 1024;
}

// ts: the training forward (stores for the backward pass); null for inference.
tled_status fused_forward(tled_mlp *s, long n, const float *coords, const float *params, float *out,
                          const TrainStore *ts = nullptr) {
    NetOffsets off{};
    for (int l = 0; l <= s->cfg.depth; ++l) {
        off.w[l] = s->layers[l].w_off;
        off.b[l] = s->layers[l].b_off;
    }
    const unsigned grid = unsigned((n + kFusedRows - 1) / kFusedRows);
    const size_t lds = fused_lds_bytes(s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (s->timing) {
        MCHK(s, hipEventCreate(&e0));
        MCHK(s, hipEventCreate(&e1));
        MCHK(s, hipEventRecord(e0, s->stream));
    }
#define TLED_FUSED(WIDTH, TR, NW)                                                                           \
    hipLaunchKernelGGL((fused_forward_kernel<WIDTH, TR, NW>), dim3(grid), dim3(64 * NW), lds, s->stream, n,  \
                       coords, params, s->d_freq, s->cfg.n_freq, s->cfg.n_param, s->K0, s->cfg.depth,         \
                       s->cfg.n_out, s->d_wb, s->d_w, off, out, ts ? *ts : TrainStore{})
    // fewer than two workgroups per CU: eight wavefronts each (measured faster at 16k
    // samples, slower at 1M, same bits either way)
    const bool wide = long(grid) < 2L * s->cus;
    if (ts) {
        if (s->cfg.width == 64) TLED_FUSED(64, true, 4);
        else if (s->cfg.width == 128) { if (wide) TLED_FUSED(128, true, 8); else TLED_FUSED(128, true, 4); }
        else { if (wide) TLED_FUSED(256, true, 8); else TLED_FUSED(256, true, 4); }
    } else {
        if (s->cfg.width == 64) TLED_FUSED(64, false, 4);
        else if (s->cfg.width == 128) { if (wide) TLED_FUSED(128, false, 8); else TLED_FUSED(128, false, 4); }
        else { if (wide) TLED_FUSED(256, false, 8); else TLED_FUSED(256, false, 4); }
    }
#undef TLED_FUSED
    MCHK(s, hipGetLastError());
    if (s->timing) {
        MCHK(s, hipEventRecord(e1, s->stream));
        MCHK(s, hipEventSynchronize(e1));
        float ms = 0.f;
        MCHK(s, hipEventElapsedTime(&ms, e0, e1));
        const double W = s->cfg.width;
        const double fl = 2.0 * double(n) * (double(s->K0) * W + (s->cfg.depth - 1) * W * W + W * s->cfg.n_out);
        if (ts) {   // the training forward: counted with the step's GEMMs
            s->gemm_ms += ms;
            s->gemm_flops += fl;
        } else {
            s->fused_ms += ms;
            s->fused_flops += fl;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return TLED_OK;
}

// Forward pass for n samples: features, hidden layers (Z, activations kept), output into d_y.
// With the fused kernel available, one launch writes all of them (the same bits as the
// layer-by-layer GEMMs, whose epilogue arithmetic it repeats).
tled_status forward(tled_mlp *s, long n, const float *coords, const float *params) {
    MTRY(ensure_workspace(s, n));
    const int W = s->cfg.width;
    if (fused_ok(s)) {
        TrainStore ts{};
        ts.x0 = s->d_x0;
        for (int l = 0; l < s->cfg.depth; ++l) {
            ts.z[l] = s->d_z[l];
            ts.a[l] = s->d_a[l];
        }
        return fused_forward(s, n, coords, params, s->d_y, &ts);
    }
    hipLaunchKernelGGL(features_kernel, dim3(blocks(n * s->K0)), dim3(kThreads), 0, s->stream, n, coords, params,
                       s->d_freq, s->cfg.n_freq, s->cfg.n_param, s->K0, s->d_x0);
    MCHK(s, hipGetLastError());
    const uint16_t *a = s->d_x0;
    int in = s->K0;
    for (int l = 0; l < s->cfg.depth; ++l) {
        const Layer &L = s->layers[l];
        MTRY(gemm<EPI_BIAS_SILU>(s, int(n), W, in, a, in, 1, s->d_wb + L.w_off, 1, in, s->d_z[l], W, 1, s->d_a[l],
                                 s->d_w + L.b_off));
        a = s->d_a[l];
        in = W;
    }
    const Layer &O = s->layers.back();
    MTRY(gemm<EPI_BIAS_F32>(s, int(n), s->cfg.n_out, W, a, W, 1, s->d_wb + O.w_off, 1, W, s->d_y, s->cfg.n_out, 1,
                            nullptr, s->d_w + O.b_off));
    return TLED_OK;
}

// Loss and gradient into d_g (and *loss on the host if requested).
tled_status backward(tled_mlp *s, long n, const float *target, float *loss) {
    const int W = s->cfg.width, no = s->cfg.n_out, D = s->cfg.depth;
    const unsigned nb = blocks(n * no);
    hipLaunchKernelGGL(loss_grad_kernel, dim3(nb), dim3(kThreads), 0, s->stream, n, no, s->d_y, target, s->d_dy,
                       s->d_part);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kThreads), 0, s->stream, int(nb), s->d_part,
                       1.0f / float(n * no), s->d_loss);
    MCHK(s, hipGetLastError());
    // row chunks of at least kColChunk, few enough for the grid's y extent
    const long chunk = std::max<long>(kColChunk, (n + 65534) / 65535);
    const unsigned nchunk = unsigned((n + chunk - 1) / chunk);
    // output layer
    const Layer &O = s->layers.back();
    uint16_t *dz = s->d_dz, *dz_next = s->d_dz2;
    if (no <= kOutMax) {
        // weights and bias of the output layer are contiguous in the gradient
        const auto [rows, nc] = out_grad_chunks(n);
        hipLaunchKernelGGL(out_grad_partial_kernel, dim3(unsigned(nc)), dim3(kThreads), 0, s->stream, n, W, no, rows,
                           s->d_dy, s->d_a[D - 1], s->d_cpart);
        const long L = long(no) * (W + 1);
        hipLaunchKernelGGL(parts_reduce_kernel, dim3(unsigned((L + 15) / 16)), dim3(kThreads), 0, s->stream, int(nc),
                           L, s->d_cpart, s->d_g + O.w_off);
        // dZ of the last hidden layer = (dY W_O) through its SiLU
        hipLaunchKernelGGL(out_back_kernel, dim3(blocks(n * (W / 8))), dim3(kThreads), 0, s->stream, n, W, no,
                           s->d_dy, s->d_wb + O.w_off, s->d_z[D - 1], dz);
        MCHK(s, hipGetLastError());
    } else {
        MTRY(gemm<EPI_F32>(s, no, W, int(n), s->d_dy, 1, no, s->d_a[D - 1], W, 1, s->d_g + O.w_off, W, 1, nullptr,
                           nullptr));
        hipLaunchKernelGGL(colsum_partial_kernel, dim3((no + kThreads - 1) / kThreads, nchunk), dim3(kThreads), 0,
                           s->stream, n, no, s->d_dy, s->d_cpart, chunk);
        hipLaunchKernelGGL(colsum_final_kernel, dim3((no + 63) / 64), dim3(kThreads), 0, s->stream, int(nchunk), no,
                           s->d_cpart, s->d_g + O.b_off);
        // dZ of the last hidden layer = (dY W_O) through its SiLU, in the GEMM epilogue
        MTRY(gemm<EPI_SILU_BACK>(s, int(n), W, no, s->d_dy, no, 1, s->d_wb + O.w_off, W, 1, nullptr, W, 1, dz,
                                 s->d_z[D - 1]));
    }
    for (int l = D - 1; l >= 0; --l) {
        const Layer &L = s->layers[l];
        const uint16_t *ain = l > 0 ? s->d_a[l - 1] : s->d_x0;
        const int in = L.in;
        // the bias gradient (column sums of dZ) comes out of the weight-gradient GEMM
        // when both operands stage along rows (aligned rows, widths of multiples of 8)
        if (load_mode(dz, 1, W) == LD_RVEC && load_mode(ain, 1, in) == LD_RVEC) {
            MTRY(gemm<EPI_F32>(s, W, in, int(n), dz, 1, W, ain, in, 1, s->d_g + L.w_off, in, 1, nullptr, nullptr,
                               nullptr, 0, s->d_g + L.b_off, 1024));
        } else {
            MTRY(gemm<EPI_F32>(s, W, in, int(n), dz, 1, W, ain, in, 1, s->d_g + L.w_off, in, 1, nullptr, nullptr,
                               nullptr, 0, nullptr, 1024));
            hipLaunchKernelGGL(colsum_partial_kernel, dim3((W + kThreads - 1) / kThreads, nchunk), dim3(kThreads), 0,
                               s->stream, n, W, dz, s->d_cpart, chunk);
            hipLaunchKernelGGL(colsum_final_kernel, dim3((W + 63) / 64), dim3(kThreads), 0, s->stream, int(nchunk),
                               W, s->d_cpart, s->d_g + L.b_off);
        }
        if (l > 0) {
            // dZ of layer l - 1 = (dZ_l W_l) through layer l - 1's SiLU
            MTRY(gemm<EPI_SILU_BACK>(s, int(n), in, W, dz, W, 1, s->d_wb + L.w_off, in, 1, nullptr, in, 1, dz_next,
                                     s->d_z[l - 1]));
            std::swap(dz, dz_next);
        }
    }
    MCHK(s, hipGetLastError());
    if (loss) {
        MCHK(s, hipMemcpyAsync(loss, s->d_loss, sizeof(float), hipMemcpyDeviceToHost, s->stream));
        MCHK(s, hipStreamSynchronize(s->stream));
    }
    return TLED_OK;
}

}  // namespace

extern "C" {

const char *tled_mlp_last_error(const tled_mlp *mlp) { return mlp ? mlp->err.c_str() : "null handle"; }

tled_status tled_mlp_create(tled_mlp **out, int device, const tled_mlp_config *cfg) {
    if (!out || !cfg) return TLED_E_ARG;
    *out = nullptr;
    if (cfg->n_param < 0 || cfg->n_freq < 1 || cfg->width < 64 || cfg->width % 64 || cfg->depth < 1 ||
        cfg->n_out < 1 || cfg->n_out > 64 || !(cfg->sigma > 0))
        return TLED_E_ARG;
    int nd = 0;
    if (hipGetDeviceCount(&nd) != hipSuccess || device < 0 || device >= nd) return TLED_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return TLED_E_HIP;
    if (resolve_scratch(device) != TLED_OK) return TLED_E_HIP;
    tled_mlp *s = new (std::nothrow) tled_mlp();
    if (!s) return TLED_E_OOM;
    s->device = device;
    if (hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        delete s;
        return TLED_E_HIP;
    }
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        s->d_static_split = g_scratch_addr[device];
    }
    s->cfg = *cfg;
    s->K0 = ((2 * cfg->n_freq + cfg->n_param + 31) / 32) * 32;
    long off = 0;
    int in = s->K0;
    for (int l = 0; l <= cfg->depth; ++l) {
        const int o = l < cfg->depth ? cfg->width : cfg->n_out;
        Layer L{in, o, off, off + long(o) * in};
        off += long(o) * in + o;
        s->layers.push_back(L);
        in = cfg->width;
    }
    s->P = off;
    // frequencies ~ N(0, sigma^2) (Box-Muller) and uniform Glorot initial weights
    uint64_t rs = cfg->seed ^ 0x5eedf00dULL;
    s->freq.resize(3 * size_t(cfg->n_freq));
    for (auto &f : s->freq) {
        const double u1 = std::max(uniform01(rs), 1e-300), u2 = uniform01(rs);
        f = float(cfg->sigma * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
    std::vector<float> w(s->P, 0.f);
    const double scale = cfg->init_scale > 0 ? cfg->init_scale : 1.0;
    for (int l = 0; l <= cfg->depth; ++l) {
        const Layer &L = s->layers[l];
        const int fan_in = l == 0 ? 2 * cfg->n_freq + cfg->n_param : L.in;
        const double lim = scale * std::sqrt(6.0 / double(fan_in + L.out));
        for (int o = 0; o < L.out; ++o)
            for (int i = 0; i < L.in; ++i)
                w[L.w_off + long(o) * L.in + i] = (l == 0 && i >= fan_in) ? 0.f : float(lim * (2.0 * uniform01(rs) - 1.0));
    }
    auto fail_free = [&](tled_status st) {
        tled_mlp_destroy(s);
        return st;
    };
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) return fail_free(TLED_E_HIP);
    s->own_stream = true;
    void *p;
    if (hipMalloc(&p, sizeof(float) * s->P) != hipSuccess) return fail_free(TLED_E_OOM);
    s->d_w = static_cast<float *>(p);
    if (hipMalloc(&p, sizeof(float) * s->P) != hipSuccess) return fail_free(TLED_E_OOM);
    s->d_g = static_cast<float *>(p);
    if (hipMalloc(&p, sizeof(float) * s->P) != hipSuccess) return fail_free(TLED_E_OOM);
    s->d_m = static_cast<float *>(p);
    if (hipMalloc(&p, sizeof(float) * s->P) != hipSuccess) return fail_free(TLED_E_OOM);
    s->d_v = static_cast<float *>(p);
    if (hipMalloc(&p, sizeof(uint16_t) * s->P) != hipSuccess) return fail_free(TLED_E_OOM);
    s->d_wb = static_cast<uint16_t *>(p);
    if (hipMalloc(&p, sizeof(float) * s->freq.size()) != hipSuccess) return fail_free(TLED_E_OOM);
    s->d_freq = static_cast<float *>(p);
    if (hipMemcpy(s->d_freq, s->freq.data(), sizeof(float) * s->freq.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->d_m, 0, sizeof(float) * s->P) != hipSuccess ||
        hipMemset(s->d_v, 0, sizeof(float) * s->P) != hipSuccess)
        return fail_free(TLED_E_HIP);
    *out = s;
    if (tled_mlp_set_params(s, w.data()) != TLED_OK) {
        *out = nullptr;
        return fail_free(TLED_E_HIP);
    }
    return TLED_OK;
}

void tled_mlp_destroy(tled_mlp *s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_ws(s);
    if (s->d_split) (void)hipFree(s->d_split);
    for (void *p : {static_cast<void *>(s->d_w), static_cast<void *>(s->d_g), static_cast<void *>(s->d_m),
                    static_cast<void *>(s->d_v), static_cast<void *>(s->d_wb), static_cast<void *>(s->d_freq)})
        if (p) (void)hipFree(p);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

tled_status tled_mlp_set_stream(tled_mlp *s, void *hip_stream) {
    if (!s) return TLED_E_ARG;
    MCHK(s, hipStreamSynchronize(s->stream));
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    s->own_stream = false;
    s->stream = static_cast<hipStream_t>(hip_stream);
    if (!s->stream) {
        MCHK(s, hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    return TLED_OK;
}

tled_status tled_mlp_param_count(const tled_mlp *s, int64_t *n) {
    if (!s || !n) return TLED_E_ARG;
    *n = s->P;
    return TLED_OK;
}

tled_status tled_mlp_get_params(tled_mlp *s, float *host) {
    if (!s || !host) return TLED_E_ARG;
    MCHK(s, hipSetDevice(s->device));
    MCHK(s, hipMemcpyAsync(host, s->d_w, sizeof(float) * s->P, hipMemcpyDeviceToHost, s->stream));
    MCHK(s, hipStreamSynchronize(s->stream));
    return TLED_OK;
}

tled_status tled_mlp_set_params(tled_mlp *s, const float *host) {
    if (!s || !host) return TLED_E_ARG;
    MCHK(s, hipSetDevice(s->device));
    MCHK(s, hipMemcpyAsync(s->d_w, host, sizeof(float) * s->P, hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks(s->P)), dim3(kThreads), 0, s->stream, s->P, s->d_w, s->d_wb);
    MCHK(s, hipGetLastError());
    MCHK(s, hipStreamSynchronize(s->stream));
    return TLED_OK;
}

tled_status tled_mlp_get_frequencies(tled_mlp *s, float *host) {
    if (!s || !host) return TLED_E_ARG;
    std::memcpy(host, s->freq.data(), sizeof(float) * s->freq.size());
    return TLED_OK;
}

tled_status tled_mlp_forward(tled_mlp *s, int64_t n, const float *coords, const float *params, float *out) {
    if (!s || n < 0 || (n > 0 && (!coords || !out || (s->cfg.n_param > 0 && !params)))) return TLED_E_ARG;
    if (n == 0) return TLED_OK;
    MCHK(s, hipSetDevice(s->device));
    if (fused_ok(s)) return fused_forward(s, long(n), coords, params, out);
    MTRY(forward(s, long(n), coords, params));
    MCHK(s, hipMemcpyAsync(out, s->d_y, sizeof(float) * size_t(n) * s->cfg.n_out, hipMemcpyDeviceToDevice, s->stream));
    return TLED_OK;
}

tled_status tled_mlp_gradient(tled_mlp *s, int64_t n, const float *coords, const float *params, const float *target,
                              float *grad_host, float *loss) {
    if (!s || n <= 0 || !coords || !target || (s->cfg.n_param > 0 && !params)) return TLED_E_ARG;
    MCHK(s, hipSetDevice(s->device));
    MTRY(forward(s, long(n), coords, params));
    MTRY(backward(s, long(n), target, loss));
    if (grad_host) {
        MCHK(s, hipMemcpyAsync(grad_host, s->d_g, sizeof(float) * s->P, hipMemcpyDeviceToHost, s->stream));
        MCHK(s, hipStreamSynchronize(s->stream));
    }
    return TLED_OK;
}

tled_status tled_mlp_train_step(tled_mlp *s, int64_t n, const float *coords, const float *params,
                                const float *target, float lr, float *loss) {
    if (!s || n <= 0 || !coords || !target || (s->cfg.n_param > 0 && !params) || !(lr > 0)) return TLED_E_ARG;
    MCHK(s, hipSetDevice(s->device));
    MTRY(forward(s, long(n), coords, params));
    MTRY(backward(s, long(n), target, loss));
    s->adam_t += 1;
    const float c1 = float(1.0 / (1.0 - std::pow(0.9, double(s->adam_t))));
    const float c2 = float(1.0 / (1.0 - std::pow(0.999, double(s->adam_t))));
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(s->P)), dim3(kThreads), 0, s->stream, s->P, s->d_w, s->d_g, s->d_m,
                       s->d_v, lr, c1, c2, s->d_wb);
    MCHK(s, hipGetLastError());
    return TLED_OK;
}

tled_status tled_mlp_gemm(tled_mlp *s, int32_t m, int32_t n, int32_t k, const uint16_t *A, const uint16_t *B,
                          float *C) {
    if (!s || m <= 0 || n <= 0 || k <= 0 || !A || !B || !C) return TLED_E_ARG;
    MCHK(s, hipSetDevice(s->device));
    s->gemm_ms = s->fused_ms = s->gemm_flops = s->fused_flops = 0.0;
    MTRY(gemm<EPI_F32>(s, m, n, k, A, k, 1, B, n, 1, C, n, 1, nullptr, nullptr));
    return TLED_OK;
}

tled_status tled_mlp_gemm_static(tled_mlp *s, int32_t m, int32_t n, int32_t k, const uint16_t *A,
                                 const uint16_t *B, float *C) {
    if (!s || m <= 0 || n <= 0 || k <= 0 || !A || !B || !C) return TLED_E_ARG;
    if (!s->d_static_split) return mfail(s, TLED_E_STATE, "static scratch not resolved for this device");
    MCHK(s, hipSetDevice(s->device));
    return gemm<EPI_F32>(s, m, n, k, A, k, 1, B, n, 1, C, n, 1, nullptr, nullptr, s->d_static_split,
                         kStaticSplitFloats);
}

tled_status tled_mlp_ensemble_stats(int64_t n, int32_t members, int32_t n_out, const float *outs,
                                    const float *scale, float *mean, float *spread, void *hip_stream) {
    if (n < 0 || members < 1 || n_out < 1 || n_out > 64 || (n > 0 && (!outs || !scale || !mean || !spread)))
        return TLED_E_ARG;
    if (n == 0) return TLED_OK;
    hipLaunchKernelGGL(ensemble_stats_kernel, dim3(blocks(n)), dim3(kThreads), 0,
                       static_cast<hipStream_t>(hip_stream), long(n), int(members), int(n_out), outs, scale, mean,
                       spread);
    return hipGetLastError() == hipSuccess ? TLED_OK : TLED_E_HIP;
}

tled_status tled_mlp_scenario_inputs(int32_t n_scen, int32_t n_prm, int64_t n_rows, const int64_t *row_begin,
                                     const double *X, const double *probe, const double *xi, double p_scale,
                                     const float *prm, float *x_out, float *p_out, void *hip_stream) {
    if (n_scen < 1 || n_prm < 0 || n_prm > 64 || n_rows < 0 ||
        (n_rows > 0 && (!row_begin || !X || !probe || !xi || (n_prm > 0 && !prm) || !x_out || !p_out)))
        return TLED_E_ARG;
    if (n_rows == 0) return TLED_OK;
    hipLaunchKernelGGL(scenario_inputs_kernel, dim3(blocks(n_rows)), dim3(kThreads), 0,
                       static_cast<hipStream_t>(hip_stream), int(n_scen), int(n_prm), row_begin, X, probe, xi,
                       p_scale, prm, x_out, p_out);
    return hipGetLastError() == hipSuccess ? TLED_OK : TLED_E_HIP;
}

tled_status tled_mlp_scenario_outputs(int32_t n_scen, int64_t n_rows, const int64_t *row_begin, const float *mean,
                                      const float *spread, const float *T0, const float *sT, const float *su,
                                      float *T_out, float *u_out, float *spread_out, void *hip_stream) {
    if (n_scen < 1 || n_rows < 0 ||
        (n_rows > 0 && (!row_begin || !mean || !spread || !T0 || !sT || !su || !T_out || !u_out || !spread_out)))
        return TLED_E_ARG;
    if (n_rows == 0) return TLED_OK;
    hipLaunchKernelGGL(scenario_outputs_kernel, dim3(blocks(n_rows)), dim3(kThreads), 0,
                       static_cast<hipStream_t>(hip_stream), int(n_scen), row_begin, mean, spread, T0, sT, su, T_out,
                       u_out, spread_out);
    return hipGetLastError() == hipSuccess ? TLED_OK : TLED_E_HIP;
}

tled_status tled_mlp_set_timing(tled_mlp *s, int on) {
    if (!s) return TLED_E_ARG;
    s->timing = on != 0;
    s->gemm_ms = s->fused_ms = s->gemm_flops = s->fused_flops = 0.0;
    return TLED_OK;
}

tled_status tled_mlp_last_timing(tled_mlp *s, double ms[2], double flops[2]) {
    if (!s || !ms || !flops) return TLED_E_ARG;
    ms[0] = s->gemm_ms;
    ms[1] = s->fused_ms;
    flops[0] = s->gemm_flops;
    flops[1] = s->fused_flops;
    return TLED_OK;
}

}  // extern "C"
