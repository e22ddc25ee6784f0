// Multi-right-hand-side apply of the assembled matrix: Y = A X as one real GEMM
// on the matrix cores.
//
// The complex64 matrix A (row-major [n][n], interleaved) is read as a real
// matrix A' [n][2n]; X (R right-hand sides) becomes X' [2n][2R] with
//   X'[2c][j] = Re X_j[c],  X'[2c+1][j] = -Im X_j[c],
//   X'[2c][R+j] = Im X_j[c], X'[2c+1][R+j] = Re X_j[c],
// so that Y' = A' X' holds [Re Y | Im Y].  X' is stored transposed (row j =
// column j of X', K contiguous) so both operands stream along K.
//
// Precisions:
//   split BF16 (3 terms): A' = A_hi + A_lo, X' = X_hi + X_lo (BF16 each);
//     Y' = A_hi X_hi + A_hi X_lo + A_lo X_hi with FP32 accumulation
//     (v_mfma_f32_16x16x32_bf16).
//   FP32: v_mfma_f32_16x16x4_f32 on A' and X' directly.
// Split-K over S slices fills the chip when 2R is small; slices are summed in
// a fixed order by the unpack kernel.
//
// The BF16 planes of A' and of X'^T are stored blocked: 16 rows x 32 K values
// per 1 KB block, blocks ordered (row block, K step), inside a block
// (K chunk of 8, row, 8 values).  One MFMA operand fragment of a row block and
// K step (lane l: row l % 16, K values 8 (l / 16) .. + 7) is then exactly the
// block, lane l reading bytes 16 l .. 16 l + 15: every fragment load is one
// contiguous 1 KB read of whole cache lines.
#include <algorithm>
#include <cmath>

#include "bem_internal.h"

namespace bem {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int GBM = 128;    // rows of a workgroup tile
constexpr int GBN = 128;    // columns of a workgroup tile
constexpr int GBK = 32;     // K step (one bf16 MFMA)
constexpr int GBKP = 40;    // padded LDS row, bf16 elements (80 B)
constexpr int FBKP = 36;    // padded LDS row, fp32 elements (144 B)

__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
    return uint16_t(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// element (r, k) of a blocked BF16 plane with Kp columns
__device__ __forceinline__ int64_t blocked_offset(int64_t r, int64_t k, int64_t Kp)
{
    return ((r >> 4) * (Kp >> 5) + (k >> 5)) * 512 + ((k & 31) >> 3) * 128 + (r & 15) * 8 + (k & 7);
}

// A' (n x 2n fp32 view of A) -> blocked hi/lo BF16 planes of Mr = n rounded up
// to 16 rows and Kp columns, zero-padded (grid-stride: Mr Kp exceeds the
// 32-bit work-item count of one dispatch beyond n ~ 46k).  Reads are along
// rows of A' (coalesced), writes are 16-byte runs inside the blocks.
__global__ void k_split_matrix(const float *__restrict__ A, int64_t n, int64_t Mr, int64_t Kp,
                               uint16_t *__restrict__ hi, uint16_t *__restrict__ lo)
{
    const int64_t total = Mr * Kp, step = int64_t(gridDim.x) * blockDim.x;
    for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total; idx += step) {
        const int64_t r = idx / Kp, k = idx - r * Kp;
        const float a = (r < n && k < 2 * n) ? A[r * 2 * n + k] : 0.0f;
        const uint16_t h = f32_to_bf16(a);
        const int64_t o = blocked_offset(r, k, Kp);
        hi[o] = h;
        lo[o] = f32_to_bf16(a - bf16_to_f32(h));
    }
}

// X (R vectors, complex128, RHS-major) -> X'^T [Np][Kp] (fp32 row-major, or
// blocked bf16 hi/lo planes)
template <bool BF16>
__global__ void k_pack_rhs(const double2 *__restrict__ X, int64_t n, int R, int64_t Np, int64_t Kp,
                           float *__restrict__ f32, uint16_t *__restrict__ hi, uint16_t *__restrict__ lo)
{
    const int64_t total = Np * Kp, step = int64_t(gridDim.x) * blockDim.x;
    for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total; idx += step) {
        const int64_t j = idx / Kp, k = idx - j * Kp;
        float v = 0.0f;
        if (k < 2 * n && j < 2 * R) {
            const int64_t c = k >> 1;
            const bool odd = k & 1;
            const double2 x = X[(j < R ? j : j - R) * n + c];
            if (j < R) v = odd ? float(-x.y) : float(x.x);
            else v = odd ? float(x.x) : float(x.y);
        }
        if (BF16) {
            const uint16_t h = f32_to_bf16(v);
            const int64_t o = blocked_offset(j, k, Kp);
            hi[o] = h;
            lo[o] = f32_to_bf16(v - bf16_to_f32(h));
        } else {
            f32[idx] = v;
        }
    }
}

// Tile order: the n-tiles and K slices of one m-tile sit on one XCD (workgroup
// ids differ by multiples of 8), so its A rows are shared through that L2.
__device__ __forceinline__ void tile_of(int id, int n_m, int n_n, int n_s, int &mt, int &nt, int &ks)
{
    const int per_m = n_n * n_s;
    const int xcd = id & 7, slot = id >> 3;
    const int group = slot / per_m, inner = slot - group * per_m;
    mt = group * 8 + xcd;
    nt = inner / n_s;
    ks = inner - nt * n_s;
    (void)n_m;
}

// Tile order of the split-BF16 GEMM: on each XCD the K slice varies slowest,
// then the XCD's m-tiles, then the n-tiles, so the workgroups resident at one
// time on an XCD read the same K range of X' and share A rows across n-tiles
// in that XCD's L2.
__device__ __forceinline__ void tile_of_kouter(int id, int n_m, int n_n, int &mt, int &nt, int &ks)
{
    const int per_x = (n_m + 7) / 8;
    const int xcd = id & 7, slot = id >> 3;
    ks = slot / (per_x * n_n);
    const int rem = slot - ks * per_x * n_n;
    const int loc = rem / n_n;
    nt = rem - loc * n_n;
    mt = loc * 8 + xcd;
}

// Split-BF16 GEMM.  Workgroup tile XBM x GBN (256 x 128): four waves stacked
// along M, each owning 64 rows x 128 columns (4 x 8 MFMA tiles of 16 x 16,
// 128 FP32 accumulators per lane).  A fragments are loaded from global memory
// straight into registers in the MFMA operand layout (each row block is read
// by exactly one wave, so staging it through LDS would only add LDS traffic);
// two register sets alternate so the loads of step t + 2 are in flight during
// step t + 1.  The X' tile (shared by the four waves) goes through a
// double-buffered LDS tile, one barrier per K step of 32.  K slices are
// multiples of 64, so every slice has an even number of steps.
constexpr int XBM = 256;    // rows of a split-BF16 workgroup tile
constexpr int XWB = 4;      // 16-row blocks per wave
constexpr int GKA = 192;    // alignment of Kp: K slices are multiples of 64 (4-wave shape) or 96 (8-wave shape)

// fragments of K offset k (a multiple of 32 inside the slice) from the blocked planes
template <int WB>
__device__ __forceinline__ void load_a_frags(const uint16_t *const *pah, const uint16_t *const *pal, int64_t k,
                                             bf16x8 (&ah)[WB], bf16x8 (&al)[WB])
{
    const int64_t o = (k / GBK) * 512;
#pragma unroll
    for (int i = 0; i < WB; ++i) {
        ah[i] = *reinterpret_cast<const bf16x8 *>(pah[i] + o);
        al[i] = *reinterpret_cast<const bf16x8 *>(pal[i] + o);
    }
}

// one K step of 32: 8 column blocks x (hi hi, hi lo, lo hi) x WB row blocks
template <int WB>
__device__ __forceinline__ void mfma_step(const uint16_t *sBh, const uint16_t *sBl, int frow, int fk,
                                          const bf16x8 (&ah)[WB], const bf16x8 (&al)[WB], f32x4 (&acc)[WB][8])
{
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const bf16x8 bh = *reinterpret_cast<const bf16x8 *>(&sBh[(16 * j + frow) * GBKP + fk]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(&sBl[(16 * j + frow) * GBKP + fk]);
#pragma unroll
        for (int i = 0; i < WB; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < WB; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl, acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < WB; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh, acc[i][j], 0, 0, 0);
    }
}

__global__ __launch_bounds__(256, 2) void k_gemm_bf16x3(const uint16_t *__restrict__ Ahi,
                                                        const uint16_t *__restrict__ Alo,
                                                        const uint16_t *__restrict__ Bhi,
                                                        const uint16_t *__restrict__ Blo, int64_t M, int64_t Kp,
                                                        int n_m, int n_n, int64_t kslice, float *__restrict__ C,
                                                        int64_t Np)
{
    constexpr int WM = 16 * XWB;
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][2][GBN * GBKP];   // [buffer][hi, lo]
    int mt, nt, ks;
    tile_of_kouter(blockIdx.x, n_m, n_n, mt, nt, ks);
    if (mt >= n_m) return;   // padding ids of the XCD-grouped order
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t m0 = int64_t(mt) * XBM, n0 = int64_t(nt) * GBN;
    const int64_t kb = int64_t(ks) * kslice, ke = std::min<int64_t>(Kp, kb + kslice);
    const int nk = int((ke - kb) / GBK);   // even, >= 2
    const int64_t klast = int64_t(nk - 1) * GBK;
    const int frow = lane & 15, fk = 8 * (lane >> 4);
    // A fragments of this lane in the blocked planes: block (row block, K step)
    // at ((row block) Kp / 32 + step) * 512, lane l at 8 l.  Row blocks past the
    // last one read the last one (valid memory; those rows are never stored).
    const int64_t ksteps = Kp / GBK, ks0 = kb / GBK, nrb = (M + 15) / 16;
    const uint16_t *pah[XWB], *pal[XWB];
#pragma unroll
    for (int i = 0; i < XWB; ++i) {
        const int64_t rb = std::min<int64_t>(nrb - 1, (m0 + WM * w + 16 * i) >> 4);
        pah[i] = Ahi + (rb * ksteps + ks0) * 512 + 8 * lane;
        pal[i] = Alo + (rb * ksteps + ks0) * 512 + 8 * lane;
    }
    // X' tile staging: 8 column blocks x 64 chunks of 16 B per plane and step,
    // two chunks per thread and plane, each stored to its (column, K chunk)
    // place of the padded LDS tile; loads past the slice are clamped to its
    // last step (valid memory, value unused)
    const uint16_t *pbh[2], *pbl[2];
    int soff[2];
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int c = tid + 256 * it;
        const int64_t cb = (n0 >> 4) + (c >> 6);   // column block, < Np / 16 (padded)
        pbh[it] = Bhi + (cb * ksteps + ks0) * 512 + 8 * (c & 63);
        pbl[it] = Blo + (cb * ksteps + ks0) * 512 + 8 * (c & 63);
        soff[it] = ((c >> 6) * 16 + (c & 15)) * GBKP + 8 * ((c & 63) >> 4);
    }
    uint4 b0h, b0l, b1h, b1l;
    auto load_b = [&](int64_t k) {
        const int64_t o = (std::min<int64_t>(k, klast) / GBK) * 512;
        b0h = *reinterpret_cast<const uint4 *>(pbh[0] + o);
        b0l = *reinterpret_cast<const uint4 *>(pbl[0] + o);
        b1h = *reinterpret_cast<const uint4 *>(pbh[1] + o);
        b1l = *reinterpret_cast<const uint4 *>(pbl[1] + o);
    };
    auto store_b = [&](int buf) {
        *reinterpret_cast<uint4 *>(&sB[buf][0][soff[0]]) = b0h;
        *reinterpret_cast<uint4 *>(&sB[buf][1][soff[0]]) = b0l;
        *reinterpret_cast<uint4 *>(&sB[buf][0][soff[1]]) = b1h;
        *reinterpret_cast<uint4 *>(&sB[buf][1][soff[1]]) = b1l;
    };
    f32x4 acc[XWB][8];
#pragma unroll
    for (int i = 0; i < XWB; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    bf16x8 xh[XWB], xl[XWB], yh[XWB], yl[XWB];
    load_b(0);
    load_a_frags<XWB>(pah, pal, 0, xh, xl);
    load_a_frags<XWB>(pah, pal, GBK, yh, yl);
    store_b(0);
    __syncthreads();
    for (int t = 0; t < nk; t += 2) {
        // even step: LDS buffer 0, registers x
        load_b(int64_t(t + 1) * GBK);
        mfma_step<XWB>(sB[0][0], sB[0][1], frow, fk, xh, xl, acc);
        load_a_frags<XWB>(pah, pal, std::min<int64_t>(int64_t(t + 2) * GBK, klast), xh, xl);
        store_b(1);
        __syncthreads();
        // odd step: LDS buffer 1, registers y
        load_b(int64_t(t + 2) * GBK);
        mfma_step<XWB>(sB[1][0], sB[1][1], frow, fk, yh, yl, acc);
        load_a_frags<XWB>(pah, pal, std::min<int64_t>(int64_t(t + 3) * GBK, klast), yh, yl);
        store_b(0);
        __syncthreads();
    }
    float *Cs = C + int64_t(ks) * M * Np;
#pragma unroll
    for (int i = 0; i < XWB; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = m0 + WM * w + 16 * i + 4 * (lane >> 4) + e;
                const int64_t col = n0 + 16 * j + frow;
                if (row < M) Cs[row * Np + col] = acc[i][j][e];
            }
}

// Split-BF16 GEMM, second tile shape: eight waves of 48 rows (3 x 8 MFMA tiles,
// 96 accumulators per lane) share one 384 x 128 workgroup tile, so the X' tile
// in LDS serves twice as many rows per byte staged, and the smaller per-wave
// A fragment set leaves registers for three sets: the loads of step t + 3 are
// issued as soon as step t has consumed its set.  K slices are multiples of 96
// (step count divisible by three).  The autotuner picks this shape or the
// four-wave one per problem size and right-hand-side bucket.
constexpr int YBM = 384;    // rows of the eight-wave tile
constexpr int YWB = 3;      // 16-row blocks per wave
constexpr int YNS = 3;      // A register sets in flight

__global__ __launch_bounds__(512, 1) void k_gemm_bf16x3_w8(const uint16_t *__restrict__ Ahi,
                                                           const uint16_t *__restrict__ Alo,
                                                           const uint16_t *__restrict__ Bhi,
                                                           const uint16_t *__restrict__ Blo, int64_t M, int64_t Kp,
                                                           int n_m, int n_n, int64_t kslice, float *__restrict__ C,
                                                           int64_t Np)
{
    constexpr int WM = 16 * YWB;
    __shared__ __attribute__((aligned(16))) uint16_t sB[2][2][GBN * GBKP];   // [buffer][hi, lo]
    int mt, nt, ks;
    tile_of_kouter(blockIdx.x, n_m, n_n, mt, nt, ks);
    if (mt >= n_m) return;   // padding ids of the XCD-grouped order
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t m0 = int64_t(mt) * YBM, n0 = int64_t(nt) * GBN;
    const int64_t kb = int64_t(ks) * kslice, ke = std::min<int64_t>(Kp, kb + kslice);
    const int nk = int((ke - kb) / GBK);   // multiple of YNS
    const int64_t klast = int64_t(nk - 1) * GBK;
    const int frow = lane & 15, fk = 8 * (lane >> 4);
    // blocked planes as in k_gemm_bf16x3 (row blocks past the last read the last)
    const int64_t ksteps = Kp / GBK, ks0 = kb / GBK, nrb = (M + 15) / 16;
    const uint16_t *pah[YWB], *pal[YWB];
#pragma unroll
    for (int i = 0; i < YWB; ++i) {
        const int64_t rb = std::min<int64_t>(nrb - 1, (m0 + WM * w + 16 * i) >> 4);
        pah[i] = Ahi + (rb * ksteps + ks0) * 512 + 8 * lane;
        pal[i] = Alo + (rb * ksteps + ks0) * 512 + 8 * lane;
    }
    // X' tile staging: 512 threads, one 16-byte chunk per thread and plane;
    // loads past the slice are clamped to its last step
    const int c = tid;
    const int64_t cb = (n0 >> 4) + (c >> 6);   // column block, < Np / 16 (padded)
    const uint16_t *pbh = Bhi + (cb * ksteps + ks0) * 512 + 8 * (c & 63);
    const uint16_t *pbl = Blo + (cb * ksteps + ks0) * 512 + 8 * (c & 63);
    const int soff = ((c >> 6) * 16 + (c & 15)) * GBKP + 8 * ((c & 63) >> 4);
    uint4 b0, b1;
    auto load_b = [&](int64_t k) {
        const int64_t o = (std::min<int64_t>(k, klast) / GBK) * 512;
        b0 = *reinterpret_cast<const uint4 *>(pbh + o);
        b1 = *reinterpret_cast<const uint4 *>(pbl + o);
    };
    auto store_b = [&](int buf) {
        *reinterpret_cast<uint4 *>(&sB[buf][0][soff]) = b0;
        *reinterpret_cast<uint4 *>(&sB[buf][1][soff]) = b1;
    };
    f32x4 acc[YWB][8];
#pragma unroll
    for (int i = 0; i < YWB; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    bf16x8 ah[YNS][YWB], al[YNS][YWB];
    load_b(0);
#pragma unroll
    for (int u = 0; u < YNS; ++u) load_a_frags<YWB>(pah, pal, int64_t(u) * GBK, ah[u], al[u]);
    store_b(0);
    __syncthreads();
    int buf = 0;
    for (int t = 0; t < nk; t += YNS) {
#pragma unroll
        for (int u = 0; u < YNS; ++u) {
            load_b(int64_t(t + u + 1) * GBK);
            mfma_step<YWB>(sB[buf][0], sB[buf][1], frow, fk, ah[u], al[u], acc);
            load_a_frags<YWB>(pah, pal, std::min<int64_t>(int64_t(t + u + YNS) * GBK, klast), ah[u], al[u]);
            // buffer buf ^ 1 was last read in the previous step, before the barrier
            store_b(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    float *Cs = C + int64_t(ks) * M * Np;
#pragma unroll
    for (int i = 0; i < YWB; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = m0 + WM * w + 16 * i + 4 * (lane >> 4) + e;
                const int64_t col = n0 + 16 * j + frow;
                if (row < M) Cs[row * Np + col] = acc[i][j][e];
            }
}

__global__ __launch_bounds__(256) void k_gemm_f32(const float *__restrict__ A, int64_t lda,
                                                  const float *__restrict__ B, int64_t M, int64_t K, int64_t Kp,
                                                  int n_m, int n_n, int n_s, int64_t kslice, float *__restrict__ C,
                                                  int64_t Np)
{
    __shared__ __attribute__((aligned(16))) float sA[GBM * FBKP];
    __shared__ __attribute__((aligned(16))) float sB[GBN * FBKP];
    int mt, nt, ks;
    tile_of(blockIdx.x, n_m, n_n, n_s, mt, nt, ks);
    if (mt >= n_m) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t m0 = int64_t(mt) * GBM, n0 = int64_t(nt) * GBN;
    const int64_t kb = int64_t(ks) * kslice, ke = std::min<int64_t>(Kp, kb + kslice);
    const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0, 0, 0, 0};
    const int frow = lane & 15, fk = 8 * (lane >> 4);
    for (int64_t k0 = kb; k0 < ke; k0 += GBK) {
        // 128 rows x 32 floats = 1024 chunks of 16 B; four per thread
#pragma unroll
        for (int it = 0; it < 4; ++it) {
            const int c = tid + 256 * it;
            const int row = c >> 3, ch = c & 7;
            const int64_t gr = m0 + row, kk = k0 + 4 * ch;
            float4 va = make_float4(0, 0, 0, 0);
            if (gr < M && kk < K) va = *reinterpret_cast<const float4 *>(A + gr * lda + kk);   // K is a multiple of 4
            *reinterpret_cast<float4 *>(&sA[row * FBKP + 4 * ch]) = va;
            *reinterpret_cast<float4 *>(&sB[row * FBKP + 4 * ch]) =
                *reinterpret_cast<const float4 *>(B + (n0 + row) * Kp + kk);
        }
        __syncthreads();
        // lane group g = lane/16 owns k = 8g .. 8g+7 of this step, in both operands
        float4 a0[4], a1[4], b0[4], b1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a0[i] = *reinterpret_cast<const float4 *>(&sA[(wm + 16 * i + frow) * FBKP + fk]);
            a1[i] = *reinterpret_cast<const float4 *>(&sA[(wm + 16 * i + frow) * FBKP + fk + 4]);
            b0[i] = *reinterpret_cast<const float4 *>(&sB[(wn + 16 * i + frow) * FBKP + fk]);
            b1[i] = *reinterpret_cast<const float4 *>(&sB[(wn + 16 * i + frow) * FBKP + fk + 4]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[i].x, b0[j].x, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[i].y, b0[j].y, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[i].z, b0[j].z, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0[i].w, b0[j].w, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[i].x, b1[j].x, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[i].y, b1[j].y, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[i].z, b1[j].z, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[i].w, b1[j].w, acc[i][j], 0, 0, 0);
            }
        __syncthreads();
    }
    float *Cs = C + int64_t(ks) * M * Np;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t row = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
                const int64_t col = n0 + wn + 16 * j + frow;
                if (row < M) Cs[row * Np + col] = acc[i][j][e];
            }
}

// Y_j[r] = (sum_s C_s[r][j], sum_s C_s[r][R + j])  (fixed slice order, FP64
// sums).  One workgroup per 32 x 32 tile of (r, j): the partials are read
// along j (rows of C are contiguous in j) and the sums written along r through
// an LDS transpose, so both sides are coalesced.
constexpr int UT = 32;
__global__ __launch_bounds__(256) void k_unpack_y(const float *__restrict__ C, int64_t M, int64_t Np, int R, int n_s,
                                                  double2 *__restrict__ Y)
{
    __shared__ double2 tile[UT][UT + 1];
    const int64_t r0 = int64_t(blockIdx.x) * UT;
    const int j0 = blockIdx.y * UT;
    const int t = threadIdx.x;
    {
        const int jj = t & (UT - 1);
        for (int rr = t / UT; rr < UT; rr += 256 / UT) {
            const int64_t r = r0 + rr;
            const int j = j0 + jj;
            double re = 0, im = 0;
            if (r < M && j < R) {
                // loads of 8 slices are issued together, then added in slice order
                const int64_t sstride = M * Np;
                const float *row = C + r * Np;
                for (int s0 = 0; s0 < n_s; s0 += 8) {
                    float vr[8], vi[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const int s = std::min(s0 + q, n_s - 1);
                        vr[q] = row[int64_t(s) * sstride + j];
                        vi[q] = row[int64_t(s) * sstride + R + j];
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (s0 + q < n_s) {
                            re += vr[q];
                            im += vi[q];
                        }
                }
            }
            tile[rr][jj] = make_double2(re, im);
        }
    }
    __syncthreads();
    const int rr = t & (UT - 1);
    for (int jj = t / UT; jj < UT; jj += 256 / UT) {
        const int64_t r = r0 + rr;
        const int j = j0 + jj;
        if (r < M && j < R) Y[int64_t(j) * M + r] = tile[rr][jj];
    }
}

static int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

void split_matrix_bf16(bem_problem &p)
{
    const int64_t Kp = round_up(2 * p.N, GKA), Mr = round_up(p.N, 16);
    dmalloc(reinterpret_cast<void **>(&p.d_Ahi), size_t(Mr) * Kp * sizeof(uint16_t));
    dmalloc(reinterpret_cast<void **>(&p.d_Alo), size_t(Mr) * Kp * sizeof(uint16_t));
    const int64_t tot = Mr * Kp;
    k_split_matrix<<<dim3(blocks_1d(tot, 256, true)), dim3(256), 0, p.stream>>>(
        reinterpret_cast<const float *>(p.d_A), p.N, Mr, Kp, p.d_Ahi, p.d_Alo);
    BEM_HIP(hipGetLastError());
}

GemmPlan gemm_plan(const bem_problem &p, int R, bool bf16, int force_slices, int shape)
{
    GemmPlan g{};
    g.R = R;
    g.bf16 = bf16;
    g.shape = bf16 ? std::max(0, std::min(shape, 1)) : 0;
    const int tile_m = !bf16 ? GBM : (g.shape == 1 ? YBM : XBM);
    const int64_t kalign = !bf16 ? 64 : (g.shape == 1 ? 96 : 64);   // divides GKA
    g.block = g.shape == 1 ? 512 : 256;
    g.Kp = round_up(2 * p.N, GKA);
    g.Np = round_up(2 * int64_t(R), GBN);
    g.n_m = int((p.N + tile_m - 1) / tile_m);
    g.n_n = int(g.Np / GBN);
    const int64_t ksteps = g.Kp / GBK;
    // enough workgroups to cover every CU several times
    int s = int(std::max<int64_t>(1, (2048 + int64_t(g.n_m) * g.n_n - 1) / (int64_t(g.n_m) * g.n_n)));
    s = int(std::min<int64_t>(s, std::max<int64_t>(1, ksteps / 8)));
    g.n_s = std::max(1, std::min(s, 64));
    if (force_slices > 0) g.n_s = int(std::min<int64_t>(force_slices, ksteps));
    g.kslice = round_up((g.Kp + g.n_s - 1) / g.n_s, kalign);
    g.n_s = int((g.Kp + g.kslice - 1) / g.kslice);
    const int groups = (g.n_m + 7) / 8;
    g.n_wg = groups * 8 * g.n_n * g.n_s;
    g.bytes_x = size_t(g.Np) * g.Kp * (bf16 ? 2 * sizeof(uint16_t) : sizeof(float));
    g.bytes_c = size_t(g.n_s) * p.N * g.Np * sizeof(float);
    return g;
}

void launch_gemm_kernel(bem_problem &p, const GemmPlan &g, void *xbuf, float *cbuf)
{
    const int64_t tot = g.Np * g.Kp;
    if (g.bf16) {
        uint16_t *hi = static_cast<uint16_t *>(xbuf), *lo = hi + tot;
        if (g.shape == 1)
            k_gemm_bf16x3_w8<<<dim3(unsigned(g.n_wg)), dim3(512), 0, p.stream>>>(p.d_Ahi, p.d_Alo, hi, lo, p.N, g.Kp,
                                                                                g.n_m, g.n_n, g.kslice, cbuf, g.Np);
        else
            k_gemm_bf16x3<<<dim3(unsigned(g.n_wg)), dim3(256), 0, p.stream>>>(p.d_Ahi, p.d_Alo, hi, lo, p.N, g.Kp,
                                                                             g.n_m, g.n_n, g.kslice, cbuf, g.Np);
    } else {
        k_gemm_f32<<<dim3(unsigned(g.n_wg)), dim3(256), 0, p.stream>>>(reinterpret_cast<const float *>(p.d_A), 2 * p.N,
                                                                      static_cast<float *>(xbuf), p.N, 2 * p.N, g.Kp,
                                                                      g.n_m, g.n_n, g.n_s, g.kslice, cbuf, g.Np);
    }
    BEM_HIP(hipGetLastError());
}

void launch_gemm(bem_problem &p, const GemmPlan &g, const double2 *X, double2 *Y, void *xbuf, float *cbuf)
{
    const int64_t tot = g.Np * g.Kp;
    if (g.bf16) {
        uint16_t *hi = static_cast<uint16_t *>(xbuf), *lo = hi + tot;
        k_pack_rhs<true><<<dim3(blocks_1d(tot, 256, true)), dim3(256), 0, p.stream>>>(X, p.N, g.R, g.Np, g.Kp,
                                                                                       nullptr, hi, lo);
        BEM_HIP(hipGetLastError());
        if (p.timed_gemm) BEM_HIP(hipEventRecord(p.ev[1], p.stream));
        if (g.shape == 1)
            k_gemm_bf16x3_w8<<<dim3(unsigned(g.n_wg)), dim3(512), 0, p.stream>>>(p.d_Ahi, p.d_Alo, hi, lo, p.N, g.Kp,
                                                                                g.n_m, g.n_n, g.kslice, cbuf, g.Np);
        else
            k_gemm_bf16x3<<<dim3(unsigned(g.n_wg)), dim3(256), 0, p.stream>>>(p.d_Ahi, p.d_Alo, hi, lo, p.N, g.Kp,
                                                                             g.n_m, g.n_n, g.kslice, cbuf, g.Np);
    } else {
        float *xf = static_cast<float *>(xbuf);
        k_pack_rhs<false><<<dim3(blocks_1d(tot, 256, true)), dim3(256), 0, p.stream>>>(X, p.N, g.R, g.Np, g.Kp, xf,
                                                                                        nullptr, nullptr);
        BEM_HIP(hipGetLastError());
        if (p.timed_gemm) BEM_HIP(hipEventRecord(p.ev[1], p.stream));
        k_gemm_f32<<<dim3(unsigned(g.n_wg)), dim3(256), 0, p.stream>>>(reinterpret_cast<const float *>(p.d_A), 2 * p.N,
                                                                      xf, p.N, 2 * p.N, g.Kp, g.n_m, g.n_n, g.n_s,
                                                                      g.kslice, cbuf, g.Np);
    }
    BEM_HIP(hipGetLastError());
    if (p.timed_gemm) BEM_HIP(hipEventRecord(p.ev[2], p.stream));
    launch_unpack(p, g, cbuf, Y);
}

void launch_unpack(bem_problem &p, const GemmPlan &g, const float *cbuf, double2 *Y)
{
    const dim3 ugrid(unsigned((p.N + UT - 1) / UT), unsigned((g.R + UT - 1) / UT));
    k_unpack_y<<<ugrid, dim3(256), 0, p.stream>>>(cbuf, p.N, g.Np, g.R, g.n_s, Y);
    BEM_HIP(hipGetLastError());
}

}  // namespace bem
