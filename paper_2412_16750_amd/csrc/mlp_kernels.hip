// Learned warm start for the trajectory fit: a 150 -> 256 -> 256 -> 5 ReLU MLP
// that maps an observed trajectory window to normalised IDM parameters.
// Hand-written BF16 MFMA kernels for gfx950 (FP32 accumulate): the whole
// forward fused into one launch (v_mfma_f32_16x16x32_bf16), backward GEMMs
// (v_mfma_f32_16x16x16_bf16, up to three problems per launch) with a
// ReLU-mask epilogue and deterministic split-K for the weight gradients, the
// output layer's gradient on the VALU (5 nonzero columns), Adam on FP32
// master weights with BF16 copies (summing the split-K slabs), and the
// window-feature kernel.
//
// BF16 rounding points (mirrored by the CPU reference): the features X, the
// weight copies W1..W3, the hidden activations H1, H2 and the back-propagated
// gradients dY, dH2, dH1 are rounded to nearest-even BF16; every product is
// accumulated in FP32; biases, outputs Y and weight gradients stay FP32.
#include "idm.h"
#include "idm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

namespace idmx {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even, NaN quiet: gfx950's
// v_cvt_pk_bf16_f32 (one instruction converts two values).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f2bf(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){lo, hi}, bf16x2));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct Gemm {
    // C[m][n] = sum_k A[m][k] B[k][n]; element strides allow transposed operands
    const uint16_t *A;
    int64_t a_rs, a_cs;
    const uint16_t *B;
    int64_t b_rs, b_cs;
    int M, N, K;
    int k_chunk;             // split-K: block z handles k in [z*k_chunk, (z+1)*k_chunk)
    const uint16_t *mask;    // ReLU mask source (value > 0 keeps) or null
    int64_t mask_rs;
    float *C32;              // FP32 output (split-K: partial slab z at C32 + z*M*c32_rs)
    int64_t c32_rs;
    uint16_t *C16;           // BF16 output or null
    int64_t c16_rs;
    int ones_row;            // A's row that reads as all ones (not in memory), or -1
    int splits;              // k slabs (blocks along k)
};

// Up to three independent GEMMs in one launch: the blocks of problem p are
// the linear block indices [start[p], start[p + 1]), each problem's blocks
// ordered m-tile fastest, then n-tile, then k slab.
constexpr int MAX_GROUP = 3;
struct GemmGroup {
    Gemm g[MAX_GROUP];
    int n;
    int start[MAX_GROUP + 1];
};

// 256 threads = 4 waves; block tile 64 x 64; each wave 32 x 32 = 2 x 2 MFMA
// 16x16x16 tiles.  MFMA operand layout (16x16x16 bf16): lane l holds
// A[l % 16][4 (l / 16) + e] and B[4 (l / 16) + e][l % 16], e = 0..3, and the
// result D[4 (l / 16) + e][l % 16].
//
// K advances in stages of 32: the block stages A (64 x 32) and B (32 x 64)
// in LDS, both stored k-contiguous (As[m][k], Bs[n][k], row pitch 36 so the
// 16 rows one operand read touches fall in distinct banks), so each MFMA
// operand is one 8-byte LDS read.  (Stages of 128 were no faster: these
// GEMMs are small and latency-bound, and the larger tile halves occupancy.)  Global loads are 16-byte vectors of 8
// elements along whichever of the operand's dimensions is contiguous in
// memory (k for activations, m for a transposed activation, n or k for the
// weights); partial or misaligned vectors fall back to element loads, and
// elements outside the matrix or the block's k range read as 0.
constexpr int GK = 32;       // k per stage
constexpr int GPITCH = 36;   // LDS row pitch (elements): 16 consecutive rows hit distinct banks

typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));

constexpr uint16_t BF16_ONE = 0x3f80;

// Element (r, c) of a strided matrix, 0 outside [0, R) x [c_lo, c_hi); row
// `ones` reads as 1 without touching memory.
__device__ __forceinline__ uint16_t elem(const uint16_t *P, int64_t rs, int64_t cs, int r, int c,
                                         int R, int c_lo, int c_hi, int ones) {
    if (r >= R || c < c_lo || c >= c_hi) return 0;
    return r == ones ? BF16_ONE : P[(int64_t)r * rs + (int64_t)c * cs];
}

__device__ __forceinline__ void unpack8(const u32x4v &w, uint16_t (&v)[8]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        v[2 * i] = (uint16_t)(w[i] & 0xffffu);
        v[2 * i + 1] = (uint16_t)(w[i] >> 16);
    }
}

// Stage one 64 x GK operand tile into T[row][k] (row = m for A, n for B).
// s_row / s_k: element strides along the tile's row index and along k.  Each
// thread moves GK / 4 elements as GK / 32 vectors of 8; all of a thread's
// global loads are issued before its LDS stores.
__device__ __forceinline__ void stage_tile(const uint16_t *P, int64_t s_row, int64_t s_k,
                                           int row0, int rows, int k0, int k_lo, int k_hi,
                                           int ones, uint16_t (*T)[GPITCH]) {
    constexpr int NV = GK / 32;
    const int t = threadIdx.x;
    uint16_t v[NV][8];
    if (s_k == 1) {
        // k contiguous: thread -> (row, NV runs of 8 consecutive k)
        const int r = t >> 2, gr = row0 + r;
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const int gk = k0 + c * 32 + (t & 3) * 8;
            const uint16_t *src = P + (int64_t)gr * s_row + gk;
            if (gr < rows && gr != ones && gk >= k_lo && gk + 8 <= k_hi &&
                ((uintptr_t)src & 15) == 0) {
                unpack8(*reinterpret_cast<const u32x4v *>(src), v[c]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    v[c][i] = elem(P, s_row, 1, gr, gk + i, rows, k_lo, k_hi, ones);
            }
        }
#pragma unroll
        for (int c = 0; c < NV; ++c)
#pragma unroll
            for (int i = 0; i < 8; ++i) T[r][c * 32 + (t & 3) * 8 + i] = v[c][i];
    } else if (s_row == 1) {
        // row contiguous: thread -> (NV values of k, 8 consecutive rows)
        const int rq = (t & 7) * 8, gr = row0 + rq;
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            const int gk = k0 + c * 32 + (t >> 3);
            const uint16_t *src = P + (int64_t)gk * s_k + gr;
            if (gr + 8 <= rows && (ones < gr || ones >= gr + 8) && gk >= k_lo && gk < k_hi &&
                ((uintptr_t)src & 15) == 0) {
                unpack8(*reinterpret_cast<const u32x4v *>(src), v[c]);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    v[c][i] = elem(P, 1, s_k, gr + i, gk, rows, k_lo, k_hi, ones);
            }
        }
#pragma unroll
        for (int c = 0; c < NV; ++c)
#pragma unroll
            for (int i = 0; i < 8; ++i) T[rq + i][c * 32 + (t >> 3)] = v[c][i];
    } else {
        // general strides: element loads
        const int r = t >> 2;
#pragma unroll
        for (int c = 0; c < NV; ++c)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int kk = c * 32 + (t & 3) * 8 + i;
                T[r][kk] = elem(P, s_row, s_k, row0 + r, k0 + kk, rows, k_lo, k_hi, ones);
            }
    }
}

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmGroup G) {
    __shared__ __attribute__((aligned(16))) uint16_t As[64][GPITCH];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[64][GPITCH];
    int p = 0;
    while (p + 1 < G.n && (int)blockIdx.x >= G.start[p + 1]) ++p;
    const Gemm &g = G.g[p];
    const int local = (int)blockIdx.x - G.start[p];
    const int mt = (g.M + 63) / 64, nt = (g.N + 63) / 64;
    const int bz = local / (mt * nt);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tm = (local % mt) * 64, tn = ((local / mt) % nt) * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int bm = tm + wm, bn = tn + wn;
    const int kb = bz * g.k_chunk;
    const int ke = min(g.K, kb + g.k_chunk);
    const int li = lane & 15, lq = lane >> 4;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = kb; k0 < ke; k0 += GK) {
        __syncthreads();  // the previous stage's reads are done
        stage_tile(g.A, g.a_rs, g.a_cs, tm, g.M, k0, kb, ke, g.ones_row, As);
        stage_tile(g.B, g.b_cs, g.b_rs, tn, g.N, k0, kb, ke, -1, Bs);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; kk += 16) {
            if (k0 + kk >= ke) break;  // the rest of the stage is zero fill
            bf16x4 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *reinterpret_cast<const bf16x4 *>(&As[wm + i * 16 + li][kk + 4 * lq]);
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *reinterpret_cast<const bf16x4 *>(&Bs[wn + j * 16 + li][kk + 4 * lq]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    float *C32 = g.C32 ? g.C32 + (int64_t)bz * g.M * g.c32_rs : nullptr;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = bm + i * 16 + 4 * lq + e;
                const int n = bn + j * 16 + li;
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][e];
                if (g.mask && !(bf2f(g.mask[(int64_t)m * g.mask_rs + n]) > 0.0f)) v = 0.0f;
                if (C32) C32[(int64_t)m * g.c32_rs + n] = v;
                if (g.C16) g.C16[(int64_t)m * g.c16_rs + n] = f2bf(v);
            }
}

// ---------------------------------------------------------------- fused forward
// Y = MLP(X) for 64 rows per work-group in one launch.  The row tile of X is
// staged in LDS once; H1 and then H2 replace it there (a layer accumulates in
// registers, and its BF16 outputs overwrite the tile after a barrier that
// ends every wave's reads).  Weights come from their transposed BF16 copies
// (k contiguous, read through L2) straight into MFMA operands.  Each of the
// 4 waves owns 64 output columns of a hidden layer (4 x 4 tiles of 16 x 16)
// and 16 rows of the output layer.
//
// v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][k] and B[k][l % 16] for
// the 8 values of k of its lane group l / 16, and the result
// D[4 (l / 16) + e][l % 16].  The k-assignment is the same for both
// operands, so any fixed map of the 32 k of a chunk onto (group, element)
// gives the same sum; here group q holds k = 8 q .. 8 q + 7 (16-byte reads).
// The product is computed transposed, D = W^T-tile x act^T-tile (A = the
// weight rows, B = the activation rows: the same register contents as for
// act x W), so a lane's 4 results are 4 consecutive output columns of one
// row: one 8-byte LDS store of 4 BF16 values (or 4 adjacent FP32 outputs).
// Rounding points as in the oracle: H = bf16(relu(acc + b)), Y = acc + b in
// FP32.
constexpr int FT = 64;          // rows per work-group
constexpr int FPD = 2;          // hidden layers: weight chunks in flight ahead of the products
constexpr int FPITCH = 264;     // LDS row pitch (elements): 132 dwords, so the 16 rows one
                                // operand read touches start 4 banks apart
constexpr int MH = IDM_MLP_HIDDEN, MIN = IDM_MLP_IN_PAD, MOUT = IDM_MLP_OUT_PAD;
static_assert(MIN % 32 == 0 && MH % 32 == 0, "k in chunks of 32");
static_assert(MH == 4 * 64 && MOUT == 16 && FT % 64 == 0, "4 waves: 64 columns / FT/4 rows each");
static_assert(MIN <= FPITCH && MH <= FPITCH && (FPITCH * 2) % 16 == 0, "tile rows");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Work-group barrier that orders LDS accesses only: the global weight loads
// in flight (the next chunks' operands) need not drain at it.
__device__ __forceinline__ void tile_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// B operands of 32-k chunk c: Wt rows n0 + 16 j + l % 16, k = 32 c + 8 (l / 16) ..
// (Wt is [N][K], k contiguous, 16-byte aligned rows).
template <int K, int NJ>
__device__ __forceinline__ void load_b(const uint16_t *Wt, int n0, int c, bf16x8 (&b)[NJ]) {
    const int lane = threadIdx.x & 63, li = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        b[j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4v *>(
                                              Wt + (int64_t)(n0 + 16 * j + li) * K + 32 * c + 8 * lq));
}

// The first PD chunks of a layer's B operands (issued ahead of its products).
template <int K, int NJ, int PD>
__device__ __forceinline__ void load_b_head(const uint16_t *Wt, int n0, bf16x8 (&b)[PD][NJ]) {
#pragma unroll
    for (int d = 0; d < PD; ++d)
        if (d < K / 32) load_b<K, NJ>(Wt, n0, d, b[d]);
}

// Output rows m0 + 16 i .. 16 i + 15 (tile rows) times columns n0 + 16 j ..
// (Wt rows), over all K: lane l's acc[i][j][e] is row m0 + 16 i + l % 16,
// column n0 + 16 j + 4 (l / 16) + e.  On entry b[d] holds chunk d; chunk
// c's products run while chunks c + 1 .. c + PD are in flight.
template <int K, int NI, int NJ, int PD>
__device__ __forceinline__ void tile_product(const uint16_t *tile, int m0, const uint16_t *Wt,
                                             int n0, bf16x8 (&b)[PD][NJ], f32x4 (&acc)[NI][NJ]) {
    const int lane = threadIdx.x & 63, li = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < K / 32; ++c) {
        bf16x8 a[NI], bc[NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) bc[j] = b[c % PD][j];
        if (c + PD < K / 32) load_b<K, NJ>(Wt, n0, c + PD, b[c % PD]);
#pragma unroll
        for (int i = 0; i < NI; ++i)
            a[i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4v *>(
                                                  tile + (m0 + 16 * i + li) * FPITCH + 32 * c + 8 * lq));
#pragma unroll
        for (int i = 0; i < NI; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bc[j], a[i], acc[i][j], 0, 0, 0);
    }
}

// Hidden-layer epilogue: bf16(relu(acc + b)) into the wave's 64 columns of
// the tile; acc[i][j][e] is row 16 i + l % 16, column n0 + 16 j + 4 (l / 16) + e.
template <int NI>
__device__ __forceinline__ void hidden_out(const f32x4 (&acc)[NI][4], const float *bias, int n0,
                                           uint16_t *tile) {
    const int lane = threadIdx.x & 63, li = lane & 15, lq = lane >> 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int col = n0 + 16 * j + 4 * lq;
        const f32x4 bj = *reinterpret_cast<const f32x4 *>(bias + col);
#pragma unroll
        for (int i = 0; i < NI; ++i) {
            const uint2 h = make_uint2(f2bf2(fmaxf(acc[i][j][0] + bj[0], 0.0f), fmaxf(acc[i][j][1] + bj[1], 0.0f)),
                                       f2bf2(fmaxf(acc[i][j][2] + bj[2], 0.0f), fmaxf(acc[i][j][3] + bj[3], 0.0f)));
            *reinterpret_cast<uint2 *>(tile + (16 * i + li) * FPITCH + col) = h;
        }
    }
}

// The tile's first `rows` hidden rows to Hg [.][MH] (16-byte stores).
__device__ __forceinline__ void tile_to_global(const uint16_t *tile, int rows, int64_t r0,
                                               uint16_t *Hg) {
    for (int v = threadIdx.x; v < rows * (MH / 8); v += blockDim.x) {
        const int r = v / (MH / 8), c = (v % (MH / 8)) * 8;
        *reinterpret_cast<u32x4v *>(Hg + (r0 + r) * MH + c) =
            *reinterpret_cast<const u32x4v *>(tile + r * FPITCH + c);
    }
}

// X [B][MIN] BF16 (any alignment), W1t [MH][MIN], W2t [MH][MH], W3t [MOUT][MH]
// (16-byte aligned), biases FP32; Y [B][MOUT] FP32; H1g, H2g [B][MH] BF16
// (16-byte aligned) or null.
// One row tile; PD weight chunks of a hidden layer in flight ahead of its products.
template <int PD>
__device__ __forceinline__ void mlp_forward_tile(const uint16_t *X, int64_t B, const uint16_t *W1t,
                                                 const uint16_t *W2t, const uint16_t *W3t,
                                                 const float *b1, const float *b2, const float *b3,
                                                 float *Y, uint16_t *H1g, uint16_t *H2g) {
    constexpr int NI = FT / 16, NO = FT / 64;  // m-tiles per wave: hidden layers, output layer
    __shared__ __attribute__((aligned(16))) uint16_t tile[FT * FPITCH];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63, li = lane & 15, lq = lane >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * FT;
    const int rows = (int)min((int64_t)FT, B - r0);
    bf16x8 b[PD][4];
    load_b_head<MIN, 4, PD>(W1t, 64 * wave, b);
    // stage the X rows (zero beyond the batch)
    const bool vec = ((uintptr_t)X & 15) == 0;
    for (int v = t; v < FT * (MIN / 8); v += blockDim.x) {
        const int r = v / (MIN / 8), c = (v % (MIN / 8)) * 8;
        u32x4v w = {0u, 0u, 0u, 0u};
        if (r < rows) {
            const uint16_t *src = X + (r0 + r) * MIN + c;
            if (vec) {
                w = *reinterpret_cast<const u32x4v *>(src);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i) w[i] = (uint32_t)src[2 * i] | ((uint32_t)src[2 * i + 1] << 16);
            }
        }
        *reinterpret_cast<u32x4v *>(tile + r * FPITCH + c) = w;
    }
    tile_barrier();
    f32x4 acc[NI][4];
    tile_product<MIN, NI, 4, PD>(tile, 0, W1t, 64 * wave, b, acc);
    load_b_head<MH, 4, PD>(W2t, 64 * wave, b);
    tile_barrier();  // every wave has read X
    hidden_out<NI>(acc, b1, 64 * wave, tile);
    tile_barrier();
    if (H1g) tile_to_global(tile, rows, r0, H1g);
    tile_product<MH, NI, 4, PD>(tile, 0, W2t, 64 * wave, b, acc);
    // the output layer's weights (8 KB, the same for every wave): all of a
    // wave's chunks issued at once, since each feeds only NO products
    bf16x8 b3c[MH / 32][1];
    load_b_head<MH, 1, MH / 32>(W3t, 0, b3c);
    tile_barrier();  // every wave has read H1
    hidden_out<NI>(acc, b2, 64 * wave, tile);
    tile_barrier();
    if (H2g) tile_to_global(tile, rows, r0, H2g);
    f32x4 y[NO][1];
    tile_product<MH, NO, 1, MH / 32>(tile, 16 * NO * wave, W3t, 0, b3c, y);
#pragma unroll
    for (int i = 0; i < NO; ++i) {
        const int r = 16 * (NO * wave + i) + li;
        if (r < rows)
#pragma unroll
            for (int e = 0; e < 4; ++e) Y[(r0 + r) * MOUT + 4 * lq + e] = y[i][0][e] + b3[4 * lq + e];
    }
}

// Many row tiles: three waves per SIMD, the register budget that keeps 3
// work-groups per CU resident to overlap each other's latencies.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_mlp_forward(
    const uint16_t *X, int64_t B, const uint16_t *W1t, const uint16_t *W2t, const uint16_t *W3t,
    const float *b1, const float *b2, const float *b3, float *Y, uint16_t *H1g, uint16_t *H2g) {
    mlp_forward_tile<FPD>(X, B, W1t, W2t, W3t, b1, b2, b3, Y, H1g, H2g);
}

// At most one work-group per CU (a training batch): nothing overlaps a
// work-group's latencies but itself, so every chunk of a hidden layer's
// weights is in flight at once.
constexpr int FT_SMALL_TILES = 256;
__global__ __launch_bounds__(256) void k_mlp_forward_small(
    const uint16_t *X, int64_t B, const uint16_t *W1t, const uint16_t *W2t, const uint16_t *W3t,
    const float *b1, const float *b2, const float *b3, float *Y, uint16_t *H1g, uint16_t *H2g) {
    mlp_forward_tile<MH / 32>(X, B, W1t, W2t, W3t, b1, b2, b3, Y, H1g, H2g);
}

// Fixed-order sum of split-K partial slabs: out[i] = sum_z part[z][i].
__global__ __launch_bounds__(256) void k_sum_slabs(const float *part, int slabs, int64_t n,
                                                   float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int z = 0; z < slabs; ++z) s += part[(int64_t)z * n + i];
        out[i] = s;
    }
}

// Output layer's backward, 16 rows per step of a grid-stride loop:
// dY = 2 (Y - U) / (B n_out) on the first n_out columns (BF16, padding
// columns 0), the squared errors summed per work-group in FP64, and
// dH2 = (dY W3^T) * [H2 > 0] in BF16.  dY has only n_out nonzero columns, so
// dH2 is n_out FP32 products per element (exact: BF16 x BF16), accumulated
// in column order, one thread per hidden column.
constexpr int OG_ROWS = 256 / MOUT;  // rows per step: one thread per dY element
__global__ __launch_bounds__(256) void k_out_grad(const float *Y, const float *U, int B,
                                                  const uint16_t *W3, const uint16_t *H2,
                                                  uint16_t *dY, uint16_t *dH2, double *part) {
    constexpr int NOUT = IDM_MLP_OUT;
    static_assert(MH == 256 && OG_ROWS * MOUT == 256, "one thread per dY element and per column");
    __shared__ float sdy[OG_ROWS][NOUT];
    __shared__ double red[4];
    const int t = threadIdx.x;
    const float scale = 2.0f / ((float)B * (float)NOUT);
    float w[NOUT];  // column t of W3^T
#pragma unroll
    for (int c = 0; c < NOUT; ++c) w[c] = bf2f(W3[t * MOUT + c]);
    double se = 0.0;
    const int64_t groups = ((int64_t)B + OG_ROWS - 1) / OG_ROWS;
    for (int64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int64_t r0 = g * OG_ROWS;
        const int rows = (int)min((int64_t)OG_ROWS, (int64_t)B - r0);
        {
            const int r = t / MOUT, c = t % MOUT;
            float d = 0.0f;
            if (r < rows && c < NOUT) {
                const float res = Y[(r0 + r) * MOUT + c] - U[(r0 + r) * NOUT + c];
                se += (double)res * (double)res;
                d = scale * res;
            }
            const uint16_t h = f2bf(d);
            if (r < rows) dY[(r0 + r) * MOUT + c] = h;
            if (c < NOUT) sdy[r][c] = bf2f(h);
        }
        __syncthreads();
        for (int r = 0; r < rows; ++r) {
            float acc = 0.0f;
#pragma unroll
            for (int c = 0; c < NOUT; ++c) acc = fmaf(sdy[r][c], w[c], acc);
            const int64_t o = (r0 + r) * MH + t;
            dH2[o] = f2bf(bf2f(H2[o]) > 0.0f ? acc : 0.0f);
        }
        __syncthreads();  // sdy is rewritten by the next step
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) se += __shfl_down(se, off, 64);
    if ((t & 63) == 0) red[t >> 6] = se;
    __syncthreads();
    if (t == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Fixed-order sum of n FP64 partials: 256 threads take every 256th one, then
// a shared-memory tree (the same order on every call).
__global__ __launch_bounds__(256) void k_sum_f64(const double *part, int n, double scale,
                                                 double *out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Adam on the FP32 master parameters, then BF16 copies of the weights.
struct MlpAdam {
    float *p, *m, *v;
    const float *g;   // gradients, or null: then sums of the split-K slabs in `part`
    const float *part;
    int slabs;
    int64_t n;
    int32_t t;        // step number of this update (1-based)
    float lr, beta1, beta2, eps;
    // nullable: the step number is *t_dev + 1 (steps done before this one),
    // and the rate follows the cosine from lr0 to lr_final over total steps
    const int32_t *t_dev;
    float lr0, lr_final;
    int32_t total;
    uint16_t *w16;    // BF16 copies of the weight blocks
    int64_t w1_off, w1_n, w2_off, w2_n, w3_off, w3_n;  // ranges in p / w16 offsets
    int64_t w16_w2, w16_w3;
    int64_t t16_w1, t16_w2, t16_w3;  // transposed copies in w16
};

// BF16 value of weight element j (row-major [rows][cols]) into both copies.
__device__ __forceinline__ void put_w16(uint16_t *w16, int64_t plain, int64_t trans, int64_t j,
                                        int rows, int cols, uint16_t b) {
    w16[plain + j] = b;
    const int64_t r = j / cols, c = j % cols;
    w16[trans + c * rows + r] = b;
}

// Gradient of parameter i from the weight-gradient GEMMs' split-K slabs:
// layer block [b0, b1) (weights then bias) has its slabs at part + slabs * b0,
// [slab][b1 - b0]; summed in slab order, as k_sum_slabs does.
__device__ __forceinline__ float slab_grad(const MlpAdam &A, int64_t i) {
    const int64_t b0 = i >= A.w3_off ? A.w3_off : (i >= A.w2_off ? A.w2_off : A.w1_off);
    const int64_t b1 = i >= A.w3_off ? A.n : (i >= A.w2_off ? A.w3_off : A.w2_off);
    const int64_t nb = b1 - b0;
    const float *q = A.part + (int64_t)A.slabs * b0 + (i - b0);
    float s = 0.0f;
    for (int z = 0; z < A.slabs; ++z) s += q[(int64_t)z * nb];
    return s;
}

// Learning rate of scheduled step t: cosine from lr0 (t = 1) to lr_final
// (t = total + 1), in FP64, rounded once.
__device__ __forceinline__ float cosine_rate(int32_t t, float lr0, float lr_final, int32_t total) {
    const double c = cos(3.14159265358979323846 * (double)(t - 1) / (double)total);
    return (float)((double)lr_final + 0.5 * ((double)lr0 - (double)lr_final) * (1.0 + c));
}

__global__ __launch_bounds__(256) void k_mlp_adam(MlpAdam A) {
    if (A.t_dev) {
        A.t = *A.t_dev + 1;
        A.lr = cosine_rate(A.t, A.lr0, A.lr_final, A.total);
    }
    const float bc1 = 1.0f - powf(A.beta1, (float)A.t);
    const float bc2 = 1.0f - powf(A.beta2, (float)A.t);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float g = A.g ? A.g[i] : slab_grad(A, i);
        const float m = A.beta1 * A.m[i] + (1.0f - A.beta1) * g;
        const float v = A.beta2 * A.v[i] + (1.0f - A.beta2) * g * g;
        A.m[i] = m;
        A.v[i] = v;
        const float p = A.p[i] - A.lr * (m / bc1) / (sqrtf(v / bc2) + A.eps);
        A.p[i] = p;
        if (i >= A.w1_off && i < A.w1_off + A.w1_n)
            put_w16(A.w16, 0, A.t16_w1, i - A.w1_off, MIN, MH, f2bf(p));
        else if (i >= A.w2_off && i < A.w2_off + A.w2_n)
            put_w16(A.w16, A.w16_w2, A.t16_w2, i - A.w2_off, MH, MH, f2bf(p));
        else if (i >= A.w3_off && i < A.w3_off + A.w3_n)
            put_w16(A.w16, A.w16_w3, A.t16_w3, i - A.w3_off, MH, MOUT, f2bf(p));
    }
}

// BF16 copies of a row-major [rows][cols] weight block: y = x, yt = x^T.
__global__ __launch_bounds__(256) void k_to_bf16(const float *x, int rows, int cols, uint16_t *y,
                                                 uint16_t *yt) {
    const int64_t n = (int64_t)rows * cols;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint16_t b = f2bf(x[i]);
        y[i] = b;
        yt[(i % cols) * rows + i / cols] = b;
    }
}

// Batch rows of the scheduled step: row i of the batch is perm[b * B + i] with
// b = (t - 1) mod (rows per epoch / B); 16-byte pieces of the BF16 feature rows
// (IN_PAD * 2 = 320 B) and the 5 FP32 targets.  A permutation entry outside
// [0, n_rows) gives a zero row instead of a read outside the data.
__global__ __launch_bounds__(256) void k_mlp_gather(const uint4 *X_all, const float *U_all,
                                                    const int64_t *perm, int64_t n_rows,
                                                    int64_t n_batches, int B, const int32_t *step,
                                                    uint4 *Xb, float *Ub) {
    constexpr int XQ = IDM_MLP_IN_PAD * 2 / 16;  // 16-byte pieces per feature row
    const int64_t b = (int64_t)(*step) % n_batches;  // step t = *step + 1
    const int64_t total = (int64_t)B * (XQ + IDM_MLP_OUT);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = i / (XQ + IDM_MLP_OUT), c = i % (XQ + IDM_MLP_OUT);
        const int64_t src = perm[b * B + row];
        const bool in = src >= 0 && src < n_rows;
        if (c < XQ)
            Xb[row * XQ + c] = in ? X_all[src * XQ + c] : make_uint4(0u, 0u, 0u, 0u);
        else
            Ub[row * IDM_MLP_OUT + (c - XQ)] = in ? U_all[src * IDM_MLP_OUT + (c - XQ)] : 0.0f;
    }
}

// End of a scheduled step t = *step + 1: its loss into slot (t - 1) % len of
// the history, and the step counter advanced (the last kernel of the step, so
// every earlier kernel read the counter before this write).
__global__ void k_mlp_end_step(int32_t *step, const double *loss, double *hist, int32_t len) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int32_t t = *step + 1;
        hist[(t - 1) % len] = *loss;
        *step = t;
    }
}

__global__ __launch_bounds__(256) void k_fill_f32(float *x, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

// Window features of one vehicle from its observed positions (observation j
// at time t_j = (obs_first + j*obs_stride)*dt), its leader's observations and
// its initial state; row layout [IN_PAD] BF16:
//   [0, n_obs)         (p_j - p0) / 1000 m
//   [n_obs, 2 n_obs)   (p_j - p_{j-1}) / (t_j - t_{j-1}) / 30 m/s  (p_{-1} = p0 at t = 0)
//   [2 n_obs, 3 n_obs) (p_h,j - p_j - length_h) / 50 m, 200 m for a lane head
//   rest               0
//
// 64 vehicles per work-group: each thread builds its row in LDS, then the
// work-group writes the 64 rows out as consecutive 4-byte words (2-byte
// elements if X is not 4-byte aligned), so the stores are coalesced.
constexpr int FEAT_ROWS = 64;
constexpr int FEAT_PITCH = MIN + 2;  // 81 words: the 64 threads' rows start in distinct banks
__global__ __launch_bounds__(FEAT_ROWS) void k_features(const float *target, int n_obs,
                                                        int obs_first, int obs_stride, float dt,
                                                        const double *p0, const float *length,
                                                        const uint8_t *is_head, int64_t N,
                                                        uint16_t *X) {
    __shared__ __attribute__((aligned(4))) uint16_t rowbuf[FEAT_ROWS * FEAT_PITCH];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * FEAT_ROWS, i = i0 + t;
    const int rows = (int)min((int64_t)FEAT_ROWS, N - i0);
    uint16_t *row = rowbuf + t * FEAT_PITCH;
    if (i < N) {
        const bool head = is_head[i] != 0;
        const double p0i = p0[i];
        const float lh = head ? 0.0f : length[i - 1];
        double prev = p0i;
        float tprev = 0.0f;
        for (int j = 0; j < n_obs; ++j) {
            const double pj = (double)target[(int64_t)j * N + i];
            const float tj = (float)(obs_first + j * obs_stride) * dt;
            row[j] = f2bf((float)((pj - p0i) / 1000.0));
            row[n_obs + j] = f2bf((float)((pj - prev) / (double)(tj - tprev)) / 30.0f);
            float gap = 200.0f;
            if (!head) gap = (float)((double)target[(int64_t)j * N + i - 1] - pj - (double)lh);
            row[2 * n_obs + j] = f2bf(gap / 50.0f);
            prev = pj;
            tprev = tj;
        }
        for (int c = 3 * n_obs; c < MIN; ++c) row[c] = 0;
    }
    __syncthreads();
    if (((uintptr_t)X & 3) == 0) {
        const uint32_t *src = reinterpret_cast<const uint32_t *>(rowbuf);
        uint32_t *dst = reinterpret_cast<uint32_t *>(X + i0 * MIN);
        for (int w = t; w < rows * (MIN / 2); w += FEAT_ROWS)
            dst[w] = src[(w / (MIN / 2)) * (FEAT_PITCH / 2) + w % (MIN / 2)];
    } else {
        for (int e = t; e < rows * MIN; e += FEAT_ROWS)
            X[i0 * MIN + e] = rowbuf[(e / MIN) * FEAT_PITCH + e % MIN];
    }
}

int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

}  // namespace

hipError_t launch_gemms(const Gemm *gs, int n, hipStream_t s);

}  // namespace idmx

using namespace idmx;

// ---------------------------------------------------------------- C ABI

namespace {

idm_status mfail(idm_status st, const char *msg) { return idmx::set_error(st, msg); }

constexpr int H = IDM_MLP_HIDDEN, FIN = IDM_MLP_IN_PAD, FOUT = IDM_MLP_OUT_PAD;

// FP32 parameter blocks: W1 [FIN x H], b1 [H], W2 [H x H], b2 [H], W3 [H x FOUT], b3 [FOUT]
constexpr int64_t OFF_W1 = 0, N_W1 = (int64_t)FIN * H;
constexpr int64_t OFF_B1 = OFF_W1 + N_W1, N_B1 = H;
constexpr int64_t OFF_W2 = OFF_B1 + N_B1, N_W2 = (int64_t)H * H;
constexpr int64_t OFF_B2 = OFF_W2 + N_W2, N_B2 = H;
constexpr int64_t OFF_W3 = OFF_B2 + N_B2, N_W3 = (int64_t)H * FOUT;
constexpr int64_t OFF_B3 = OFF_W3 + N_W3, N_B3 = FOUT;
constexpr int64_t N_PARAMS = OFF_B3 + N_B3;
// weight_grad writes a layer's weight and bias gradients as one block
static_assert(OFF_B1 == OFF_W1 + N_W1 && OFF_B2 == OFF_W2 + N_W2 && OFF_B3 == OFF_W3 + N_W3,
              "each bias follows its weights");
// BF16 copies: W1, W2, W3 back to back, then their transposes W1^T [H x FIN],
// W2^T [H x H], W3^T [FOUT x H] (the fused forward's k-contiguous operands)
constexpr int64_t H16_W1 = 0, H16_W2 = N_W1, H16_W3 = N_W1 + N_W2;
constexpr int64_t T16_W1 = N_W1 + N_W2 + N_W3, T16_W2 = T16_W1 + N_W1, T16_W3 = T16_W2 + N_W2;
constexpr int64_t N_W16 = T16_W3 + N_W3;
static_assert(T16_W1 % 8 == 0 && T16_W2 % 8 == 0 && T16_W3 % 8 == 0, "16-byte aligned blocks");

constexpr int SPLIT_ROWS = 256;  // batch rows per split-K slab of a weight gradient
constexpr int MAX_SLABS = 64;    // larger batches get longer slabs (bounded workspace, grid z)

// Rows per split-K slab for a batch of B rows: SPLIT_ROWS, or longer (a
// multiple of the GEMM's k stage) so that at most MAX_SLABS slabs cover B.
int64_t slab_rows(int64_t B) {
    const int64_t slabs = std::max<int64_t>(1, std::min<int64_t>((B + SPLIT_ROWS - 1) / SPLIT_ROWS, MAX_SLABS));
    const int64_t rows = (B + slabs - 1) / slabs;
    return (rows + GK - 1) / GK * GK;
}

size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct MlpWs {
    size_t h1, h2, y, dy, dh2, dh1, part, lpart, sched, total;
};

MlpWs mlp_ws(int64_t B) {
    MlpWs w;
    size_t o = 0;
    w.h1 = o; o += al(2 * B * H);
    w.h2 = o; o += al(2 * B * H);
    w.y = o; o += al(4 * B * FOUT);
    w.dy = o; o += al(2 * B * FOUT);
    w.dh2 = o; o += al(2 * B * H);
    w.dh1 = o; o += al(2 * B * H);
    const int64_t slabs = (B + slab_rows(B) - 1) / slab_rows(B);
    // split-K slabs of the three weight gradients, one region per layer:
    // layer block [OFF_Wl, OFF_Wl + n_l) at part + slabs * OFF_Wl, [slab][n_l]
    w.part = o; o += al(4 * slabs * N_PARAMS);
    w.lpart = o; o += al(8 * 8192);
    w.sched = o; o += al(16);  // scheduled step: its loss (FP64)
    w.total = o;
    return w;
}

Gemm gemm(const uint16_t *A, int64_t a_rs, int64_t a_cs, const uint16_t *B, int64_t b_rs,
          int64_t b_cs, int M, int N, int K) {
    Gemm g;
    memset(&g, 0, sizeof g);
    g.A = A; g.a_rs = a_rs; g.a_cs = a_cs;
    g.B = B; g.b_rs = b_rs; g.b_cs = b_cs;
    g.M = M; g.N = N; g.K = K;
    g.k_chunk = ((K + 15) / 16) * 16;
    g.ones_row = -1;
    g.splits = 1;
    return g;
}

// Weight and bias gradients of one layer as one GEMM, [act^T; 1] dz, with
// split-K over slabs of slab_rows(rows) rows: slab z of the [in + 1][out]
// result (the weights, then the bias, as the parameters are laid out) at
// part + z (in + 1) out.  The all-ones row gives the bias gradient (column
// sums of dz).
Gemm weight_grad(const uint16_t *act, int64_t act_rs, int rows, int in, const uint16_t *dz,
                 int64_t dz_rs, int out, float *part) {
    Gemm g = gemm(act, 1, act_rs, dz, dz_rs, 1, in + 1, out, rows);
    g.ones_row = in;
    const int64_t sr = slab_rows(rows);
    g.k_chunk = (int)sr;
    g.splits = (int)((rows + sr - 1) / sr);
    g.C32 = part;
    g.c32_rs = out;
    return g;
}

// Fixed-order sum of a weight gradient's slabs into dst.
hipError_t sum_slabs(const Gemm &wg, float *dst, hipStream_t s) {
    const int64_t n = (int64_t)wg.M * wg.N;
    hipLaunchKernelGGL(k_sum_slabs, dim3(grid_for(n)), dim3(256), 0, s, wg.C32, wg.splits, n, dst);
    return hipGetLastError();
}

// Y = MLP(X) in one launch; H1 and H2 are kept only when the backward needs them.
hipError_t mlp_forward(const idm_mlp_state *st, const uint16_t *X, int64_t B, uint16_t *H1,
                       uint16_t *H2, float *Y, hipStream_t s) {
    const float *P = st->params;
    const uint16_t *W16 = st->weights_bf16;
    const int64_t tiles = (B + FT - 1) / FT;
    hipLaunchKernelGGL(tiles <= FT_SMALL_TILES ? k_mlp_forward_small : k_mlp_forward,
                       dim3((unsigned)tiles), dim3(256), 0, s, X, B, W16 + T16_W1, W16 + T16_W2,
                       W16 + T16_W3, P + OFF_B1, P + OFF_B2, P + OFF_B3, Y, H1, H2);
    return hipGetLastError();
}

// Forward + MSE + backward: gradients of every FP32 parameter into G, or
// (G null) left as per-layer split-K slabs in the workspace's `part`.
hipError_t mlp_backward(const idm_mlp_state *st, const uint16_t *X, const float *U, int64_t batch,
                        char *ws, float *G, double *loss_out, hipStream_t s) {
    const MlpWs w = mlp_ws(batch);
    const int B = (int)batch;
    float *Y = (float *)(ws + w.y);
    uint16_t *H1 = (uint16_t *)(ws + w.h1), *H2 = (uint16_t *)(ws + w.h2);
    hipError_t e = mlp_forward(st, X, batch, H1, H2, Y, s);
    if (e != hipSuccess) return e;
    uint16_t *dY = (uint16_t *)(ws + w.dy), *dH2 = (uint16_t *)(ws + w.dh2);
    uint16_t *dH1 = (uint16_t *)(ws + w.dh1);
    float *part = (float *)(ws + w.part);
    const int64_t slabs = (B + slab_rows(B) - 1) / slab_rows(B);
    float *part1 = part + slabs * OFF_W1, *part2 = part + slabs * OFF_W2, *part3 = part + slabs * OFF_W3;
    double *lpart = (double *)(ws + w.lpart);
    const uint16_t *W16 = st->weights_bf16;
    // output layer: dY, the loss partials and dH2 = (dY W3^T) * [H2 > 0]
    const int lgrid = (int)std::min<int64_t>(8192, ((int64_t)B + OG_ROWS - 1) / OG_ROWS);
    hipLaunchKernelGGL(k_out_grad, dim3(lgrid), dim3(256), 0, s, Y, U, B, W16 + H16_W3, H2, dY,
                       dH2, lpart);
    if (loss_out)
        hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(256), 0, s, lpart, lgrid,
                           1.0 / ((double)B * IDM_MLP_OUT), loss_out);
    // one launch: [dW3; db3] = [H2^T; 1] dY, [dW2; db2] = [H1^T; 1] dH2 and
    // dH1 = (dH2 W2^T) * [H1 > 0]
    Gemm grp[3];
    grp[0] = weight_grad(H2, H, B, H, dY, FOUT, FOUT, part3);
    grp[1] = weight_grad(H1, H, B, H, dH2, H, H, part2);
    grp[2] = gemm(dH2, H, 1, W16 + H16_W2, 1, H, B, H, H);
    grp[2].mask = H1; grp[2].mask_rs = H; grp[2].C16 = dH1; grp[2].c16_rs = H;
    e = launch_gemms(grp, 3, s);
    if (e != hipSuccess) return e;
    // [dW1; db1] = [X^T; 1] dH1
    const Gemm w1 = weight_grad(X, FIN, B, FIN, dH1, H, H, part1);
    e = launch_gemms(&w1, 1, s);
    if (e != hipSuccess || !G) return e;
    if ((e = sum_slabs(grp[0], G + OFF_W3, s)) != hipSuccess) return e;
    if ((e = sum_slabs(grp[1], G + OFF_W2, s)) != hipSuccess) return e;
    return sum_slabs(w1, G + OFF_W1, s);
}

idm_status check_state(const idm_mlp_state *st) {
    if (!st || !st->params || !st->weights_bf16) return mfail(IDM_ERR_INVALID_ARG, "mlp state: null pointer");
    if (((uintptr_t)st->weights_bf16 & 15) != 0 || ((uintptr_t)st->params & 15) != 0)
        return mfail(IDM_ERR_INVALID_ARG, "mlp state: params or weights_bf16 not 16-byte aligned");
    return IDM_OK;
}

}  // namespace

namespace idmx {
hipError_t launch_gemms(const Gemm *gs, int n, hipStream_t s) {
    GemmGroup G;
    memset(&G, 0, sizeof G);
    if (n < 1 || n > MAX_GROUP) return hipErrorInvalidValue;
    int64_t total = 0;
    for (int p = 0; p < n; ++p) {
        G.g[p] = gs[p];
        G.start[p] = (int)total;
        total += (int64_t)((gs[p].M + 63) / 64) * ((gs[p].N + 63) / 64) * gs[p].splits;
    }
    if (total > INT32_MAX) return hipErrorInvalidValue;
    G.n = n;
    G.start[n] = (int)total;
    hipLaunchKernelGGL(k_gemm_bf16, dim3((unsigned)total), dim3(256), 0, s, G);
    return hipGetLastError();
}
}  // namespace idmx

extern "C" {

int64_t idm_mlp_param_count(void) { return N_PARAMS; }
int64_t idm_mlp_weight_bf16_count(void) { return N_W16; }

size_t idm_mlp_workspace_bytes(int64_t batch) { return batch > 0 ? mlp_ws(batch).total : 0; }

idm_status idm_mlp_sync(const idm_mlp_state *st, void *stream) {
    idm_status r = check_state(st);
    if (r != IDM_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    uint16_t *w = st->weights_bf16;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(N_W1)), dim3(256), 0, s, st->params + OFF_W1, FIN, H,
                       w + H16_W1, w + T16_W1);
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(N_W2)), dim3(256), 0, s, st->params + OFF_W2, H, H,
                       w + H16_W2, w + T16_W2);
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(N_W3)), dim3(256), 0, s, st->params + OFF_W3, H, FOUT,
                       w + H16_W3, w + T16_W3);
    if (st->adam_m && st->adam_v) {
        hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(N_PARAMS)), dim3(256), 0, s, st->adam_m, N_PARAMS, 0.0f);
        hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(N_PARAMS)), dim3(256), 0, s, st->adam_v, N_PARAMS, 0.0f);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? IDM_OK : mfail(IDM_ERR_HIP, hipGetErrorString(e));
}

idm_status idm_mlp_features(idm_plan *plan, const float *target, int32_t n_obs, int32_t obs_first,
                            int32_t obs_stride, const double *p0, const float *length,
                            uint16_t *X, void *stream) {
    if (!plan || !target || !p0 || !length || !X) return mfail(IDM_ERR_INVALID_ARG, "null argument");
    if (n_obs < 1 || 3 * n_obs > FIN || obs_first < 1 || obs_stride < 1)
        return mfail(IDM_ERR_INVALID_ARG, "features: need 1 <= n_obs <= 53, obs_first >= 1, obs_stride >= 1");
    const uint8_t *head = idmx::plan_head_flags(plan);
    const int64_t N = idmx::plan_vehicles(plan);
    if (!head) return mfail(IDM_ERR_INVALID_ARG, "plan has no head flags");
    if ((int64_t)obs_first + (int64_t)(n_obs - 1) * obs_stride > idmx::plan_steps(plan))
        return mfail(IDM_ERR_INVALID_ARG, "features: last observed step beyond n_steps");
    hipLaunchKernelGGL(k_features, dim3((unsigned)((N + FEAT_ROWS - 1) / FEAT_ROWS)), dim3(FEAT_ROWS), 0,
                       (hipStream_t)stream,
                       target, n_obs, obs_first, obs_stride, idmx::plan_dt(plan), p0, length, head, N,
                       X);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? IDM_OK : mfail(IDM_ERR_HIP, hipGetErrorString(e));
}

idm_status idm_mlp_forward(const idm_mlp_state *st, const uint16_t *X, int64_t batch, float *Y,
                           void *workspace, void *stream) {
    idm_status r = check_state(st);
    if (r != IDM_OK) return r;
    (void)workspace;  // the fused forward keeps its activations on chip
    if (!X || !Y || batch < 1 || batch > (1 << 30))
        return mfail(IDM_ERR_INVALID_ARG, "mlp forward: bad arguments");
    hipError_t e = mlp_forward(st, X, batch, nullptr, nullptr, Y, (hipStream_t)stream);
    return e == hipSuccess ? IDM_OK : mfail(IDM_ERR_HIP, hipGetErrorString(e));
}

idm_status idm_mlp_gradients(const idm_mlp_state *st, const uint16_t *X, const float *U,
                             int64_t batch, float *grad_out, double *loss_out, void *workspace,
                             void *stream) {
    idm_status r = check_state(st);
    if (r != IDM_OK) return r;
    if (!X || !U || !workspace || !grad_out || batch < 1 || batch > (1 << 30))
        return mfail(IDM_ERR_INVALID_ARG, "mlp gradients: bad arguments");
    if (((uintptr_t)workspace & 15) != 0)
        return mfail(IDM_ERR_INVALID_ARG, "mlp gradients: workspace is not 16-byte aligned");
    hipError_t e = mlp_backward(st, X, U, batch, (char *)workspace, grad_out, loss_out,
                                (hipStream_t)stream);
    return e == hipSuccess ? IDM_OK : mfail(IDM_ERR_HIP, hipGetErrorString(e));
}

idm_status idm_mlp_train_step(const idm_mlp_state *st, const uint16_t *X, const float *U,
                              int64_t batch, int32_t t, double *loss_out, void *workspace,
                              void *stream) {
    idm_status r = check_state(st);
    if (r != IDM_OK) return r;
    if (!st->adam_m || !st->adam_v) return mfail(IDM_ERR_INVALID_ARG, "mlp state: no Adam moments");
    if (!X || !U || !workspace || batch < 1 || batch > (1 << 30) || t < 1)
        return mfail(IDM_ERR_INVALID_ARG, "mlp train step: bad arguments");
    if (((uintptr_t)workspace & 15) != 0)
        return mfail(IDM_ERR_INVALID_ARG, "mlp train step: workspace is not 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    hipError_t e = mlp_backward(st, X, U, batch, ws, nullptr, loss_out, s);
    if (e == hipSuccess) {
        MlpAdam A;
        A.p = st->params; A.m = st->adam_m; A.v = st->adam_v; A.g = nullptr; A.n = N_PARAMS;
        A.part = (const float *)(ws + mlp_ws(batch).part);
        A.slabs = (int)((batch + slab_rows(batch) - 1) / slab_rows(batch));
        A.t = t;
        A.lr = st->lr; A.beta1 = st->beta1; A.beta2 = st->beta2; A.eps = st->eps;
        A.t_dev = nullptr; A.lr0 = A.lr_final = 0.0f; A.total = 1;
        A.w16 = st->weights_bf16;
        A.w1_off = OFF_W1; A.w1_n = N_W1; A.w2_off = OFF_W2; A.w2_n = N_W2; A.w3_off = OFF_W3; A.w3_n = N_W3;
        A.w16_w2 = H16_W2; A.w16_w3 = H16_W3;
        A.t16_w1 = T16_W1; A.t16_w2 = T16_W2; A.t16_w3 = T16_W3;
        hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(N_PARAMS)), dim3(256), 0, s, A);
        e = hipGetLastError();
    }
    return e == hipSuccess ? IDM_OK : mfail(IDM_ERR_HIP, hipGetErrorString(e));
}

idm_status idm_mlp_train_step_scheduled(const idm_mlp_state *st, const uint16_t *X_all,
                                        const float *U_all, int64_t n_rows, const int64_t *perm,
                                        int64_t batch, const idm_mlp_schedule *sched,
                                        uint16_t *Xb, float *Ub, void *workspace, void *stream) {
    idm_status r = check_state(st);
    if (r != IDM_OK) return r;
    if (!st->adam_m || !st->adam_v) return mfail(IDM_ERR_INVALID_ARG, "mlp state: no Adam moments");
    if (!sched || !sched->step || !sched->loss_hist || sched->hist_len < 1 ||
        sched->total_steps < 1)
        return mfail(IDM_ERR_INVALID_ARG, "mlp schedule: bad arguments");
    if (!X_all || !U_all || !perm || !Xb || !Ub || !workspace || batch < 1 ||
        batch > (1 << 30) || n_rows < batch)
        return mfail(IDM_ERR_INVALID_ARG, "mlp scheduled step: bad arguments");
    if (((uintptr_t)workspace & 15) != 0 || ((uintptr_t)X_all & 15) != 0 || ((uintptr_t)Xb & 15) != 0)
        return mfail(IDM_ERR_INVALID_ARG, "mlp scheduled step: workspace and feature rows must be "
                                          "16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    const MlpWs w = mlp_ws(batch);
    double *loss = (double *)(ws + w.sched);
    hipLaunchKernelGGL(k_mlp_gather, dim3(grid_for(batch * (IDM_MLP_IN_PAD * 2 / 16 + IDM_MLP_OUT))),
                       dim3(256), 0, s, (const uint4 *)X_all, U_all, perm, n_rows,
                       n_rows / batch, (int)batch, (const int32_t *)sched->step, (uint4 *)Xb, Ub);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = mlp_backward(st, Xb, Ub, batch, ws, nullptr, loss, s);
    if (e == hipSuccess) {
        MlpAdam A;
        A.p = st->params; A.m = st->adam_m; A.v = st->adam_v; A.g = nullptr; A.n = N_PARAMS;
        A.part = (const float *)(ws + w.part);
        A.slabs = (int)((batch + slab_rows(batch) - 1) / slab_rows(batch));
        A.t = 1;
        A.lr = 0.0f; A.beta1 = st->beta1; A.beta2 = st->beta2; A.eps = st->eps;
        A.t_dev = sched->step;
        A.lr0 = sched->lr0; A.lr_final = sched->lr_final; A.total = sched->total_steps;
        A.w16 = st->weights_bf16;
        A.w1_off = OFF_W1; A.w1_n = N_W1; A.w2_off = OFF_W2; A.w2_n = N_W2; A.w3_off = OFF_W3; A.w3_n = N_W3;
        A.w16_w2 = H16_W2; A.w16_w3 = H16_W3;
        A.t16_w1 = T16_W1; A.t16_w2 = T16_W2; A.t16_w3 = T16_W3;
        hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(N_PARAMS)), dim3(256), 0, s, A);
        hipLaunchKernelGGL(k_mlp_end_step, dim3(1), dim3(64), 0, s, sched->step,
                           (const double *)loss, sched->loss_hist, sched->hist_len);
        e = hipGetLastError();
    }
    return e == hipSuccess ? IDM_OK : mfail(IDM_ERR_HIP, hipGetErrorString(e));
}

}  // extern "C"
