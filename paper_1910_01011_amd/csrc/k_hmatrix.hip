// Hierarchical matrix of the PMCHWT operator: the adaptive cross approximation
// of far blocks (build) and the blockwise apply.
//
// Block storage (HBlock): dense blocks column-major (2 m) x (2 n); low-rank
// blocks U (2 m) x r column-major and V r x (2 n) row-major, complex64, in the
// interleaved (vertex, D/N) order of the reordered vertices.
#include "bem_internal.h"

namespace bem {

constexpr int ACA_BLOCK = 256;
constexpr int HK_MAX = 128;   // largest rank of a low-rank block

__device__ __forceinline__ float2 cmulf(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// largest value over the workgroup with its index (ties: the smaller index)
__device__ void wg_argmax(float v, int64_t i, float *sv, int64_t *si, float &vmax, int64_t &imax)
{
    const int t = threadIdx.x;
    sv[t] = v;
    si[t] = i;
    __syncthreads();
    for (int s = ACA_BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) {
            const float a = sv[t], b = sv[t + s];
            const int64_t ia = si[t], ib = si[t + s];
            if (b > a || (b == a && ib < ia)) {
                sv[t] = b;
                si[t] = ib;
            }
        }
        __syncthreads();
    }
    vmax = sv[0];
    imax = si[0];
    __syncthreads();
}

// Adaptive cross approximation with complete pivoting, one dense block R per
// workgroup (overwritten by the residual): the pivot is the entry of largest
// modulus of R; the term is u = its column, v = its row / pivot; R -= u v.
// Stops when |pivot| <= eps |first pivot| (rank = terms taken) or after kmax
// terms (rank -1 unless the residual then meets eps).
__global__ __launch_bounds__(ACA_BLOCK) void k_aca(const HBlock *__restrict__ blocks, const int32_t *__restrict__ ids,
                                                   float2 *const *__restrict__ Rs, float2 *const *__restrict__ Us,
                                                   float2 *const *__restrict__ Vs, const int32_t *__restrict__ kmaxs,
                                                   float eps, int32_t *__restrict__ rank_out)
{
    __shared__ float sv[ACA_BLOCK];
    __shared__ int64_t si[ACA_BLOCK];
    const int b = blockIdx.x;
    const HBlock B = blocks[ids[b]];
    const int64_t m2 = 2 * int64_t(B.r1 - B.r0), n2 = 2 * int64_t(B.c1 - B.c0), tot = m2 * n2;
    float2 *R = Rs[b], *U = Us[b], *V = Vs[b];
    const int kmax = kmaxs[b];
    float best = -1.0f;
    int64_t bi = 0;
    for (int64_t e = threadIdx.x; e < tot; e += ACA_BLOCK) {
        const float2 r = R[e];
        const float a = r.x * r.x + r.y * r.y;
        if (a > best) {
            best = a;
            bi = e;
        }
    }
    float vmax;
    int64_t imax;
    wg_argmax(best, bi, sv, si, vmax, imax);
    if (!(vmax > 0.0f)) {
        if (threadIdx.x == 0) rank_out[b] = 0;
        return;
    }
    const float thr = eps * eps * vmax;   // squared moduli
    int k = 0;
    bool done = false;
    while (k < kmax) {
        if (vmax <= thr) {
            done = true;
            break;
        }
        const int64_t jc = imax / m2, ir = imax - jc * m2;   // column-major index
        const float2 piv = R[imax];
        const float d = piv.x * piv.x + piv.y * piv.y;
        const float2 ip = make_float2(piv.x / d, -piv.y / d);
        for (int64_t a = threadIdx.x; a < m2; a += ACA_BLOCK) U[int64_t(k) * m2 + a] = R[jc * m2 + a];
        for (int64_t c = threadIdx.x; c < n2; c += ACA_BLOCK) V[int64_t(k) * n2 + c] = cmulf(R[c * m2 + ir], ip);
        __syncthreads();
        const float2 *uk = U + int64_t(k) * m2, *vk = V + int64_t(k) * n2;
        best = -1.0f;
        bi = 0;
        int64_t a = threadIdx.x % m2, c = threadIdx.x / m2;
        for (int64_t e = threadIdx.x; e < tot; e += ACA_BLOCK) {
            const float2 uv = cmulf(uk[a], vk[c]);
            float2 r = R[e];
            r.x -= uv.x;
            r.y -= uv.y;
            R[e] = r;
            const float s = r.x * r.x + r.y * r.y;
            if (s > best) {
                best = s;
                bi = e;
            }
            a += ACA_BLOCK;
            while (a >= m2) {
                a -= m2;
                ++c;
            }
        }
        wg_argmax(best, bi, sv, si, vmax, imax);
        ++k;
    }
    if (!done && vmax <= thr) done = true;
    if (threadIdx.x == 0) rank_out[b] = done ? k : -1;
}

// copies of the listed arrays (one workgroup per item)
__global__ void k_copy_list(const float2 *const *__restrict__ src, float2 *const *__restrict__ dst,
                            const int64_t *__restrict__ count)
{
    const float2 *s = src[blockIdx.x];
    float2 *d = dst[blockIdx.x];
    const int64_t n = count[blockIdx.x];
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = s[i];
}

void launch_aca(hipStream_t s, const HBlock *blocks, const int32_t *ids, int n, float2 *const *R, float2 *const *U,
                float2 *const *V, const int32_t *kmax, float eps, int32_t *rank)
{
    if (n == 0) return;
    k_aca<<<dim3(unsigned(n)), dim3(ACA_BLOCK), 0, s>>>(blocks, ids, R, U, V, kmax, eps, rank);
    BEM_HIP(hipGetLastError());
}

void launch_copy_list(hipStream_t s, const float2 *const *src, float2 *const *dst, const int64_t *count, int n)
{
    if (n == 0) return;
    k_copy_list<<<dim3(unsigned(n)), dim3(256), 0, s>>>(src, dst, count);
    BEM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------

// xp[2 i + s] = x[row_s(perm[i])]: the vector in the reordered interleaved order
__global__ void k_h_gather(const int32_t *__restrict__ perm, const int32_t *__restrict__ rowD,
                           const int32_t *__restrict__ rowN, const double2 *__restrict__ x, int64_t NV,
                           double2 *__restrict__ xp)
{
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= 2 * NV) return;
    const int32_t g = perm[r >> 1];
    xp[r] = x[(r & 1) ? rowN[g] : rowD[g]];
}

// one workgroup per block: z[zoff + a] = (D x_J)[a], or (U (V x_J))[a] with the
// r values V x_J reduced per wave and kept in LDS; FP64 sums
__global__ __launch_bounds__(256) void k_h_blocks(const HBlock *__restrict__ blocks, const double2 *__restrict__ xp,
                                                  double2 *__restrict__ z)
{
    __shared__ double2 t[HK_MAX];
    const HBlock B = blocks[blockIdx.x];
    const int64_t m2 = 2 * int64_t(B.r1 - B.r0), n2 = 2 * int64_t(B.c1 - B.c0);
    const double2 *xj = xp + 2 * int64_t(B.c0);
    double2 *zb = z + B.zoff;
    if (B.rank < 0) {
        for (int64_t a = threadIdx.x; a < m2; a += blockDim.x) {
            double sr = 0.0, si = 0.0;
            for (int64_t c = 0; c < n2; ++c) {
                const float2 d = B.D[c * m2 + a];
                const double2 v = xj[c];
                sr += double(d.x) * v.x - double(d.y) * v.y;
                si += double(d.x) * v.y + double(d.y) * v.x;
            }
            zb[a] = make_double2(sr, si);
        }
        return;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int k = w; k < B.rank; k += nw) {
        double sr = 0.0, si = 0.0;
        const float2 *vk = B.V + int64_t(k) * n2;
        for (int64_t c = lane; c < n2; c += 64) {
            const float2 d = vk[c];
            const double2 v = xj[c];
            sr += double(d.x) * v.x - double(d.y) * v.y;
            si += double(d.x) * v.y + double(d.y) * v.x;
        }
        for (int off = 32; off > 0; off >>= 1) {
            sr += __shfl_xor(sr, off);
            si += __shfl_xor(si, off);
        }
        if (lane == 0) t[k] = make_double2(sr, si);
    }
    __syncthreads();
    for (int64_t a = threadIdx.x; a < m2; a += blockDim.x) {
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < B.rank; ++k) {
            const float2 u = B.U[int64_t(k) * m2 + a];
            const double2 v = t[k];
            sr += double(u.x) * v.x - double(u.y) * v.y;
            si += double(u.x) * v.y + double(u.y) * v.x;
        }
        zb[a] = make_double2(sr, si);
    }
}

// y[row_s(perm[i])] = sum of the block products of reordered row 2 i + s, in
// the fixed order of the row's list
__global__ void k_h_rows(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ rowz,
                         const double2 *__restrict__ z, const int32_t *__restrict__ perm,
                         const int32_t *__restrict__ rowD, const int32_t *__restrict__ rowN, int64_t NV,
                         double2 *__restrict__ y)
{
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= 2 * NV) return;
    double sr = 0.0, si = 0.0;
    for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
        const double2 v = z[rowz[e]];
        sr += v.x;
        si += v.y;
    }
    const int32_t g = perm[r >> 1];
    y[(r & 1) ? rowN[g] : rowD[g]] = make_double2(sr, si);
}

void launch_h_apply(hipStream_t s, const HBlock *blocks, int n_blocks, const int32_t *perm, const int32_t *rowD,
                    const int32_t *rowN, const int32_t *rowptr, const int32_t *rowz, int64_t NV, const double2 *x,
                    double2 *xp, double2 *z, double2 *y)
{
    k_h_gather<<<dim3(blocks_1d(2 * NV, 256)), dim3(256), 0, s>>>(perm, rowD, rowN, x, NV, xp);
    BEM_HIP(hipGetLastError());
    k_h_blocks<<<dim3(unsigned(n_blocks)), dim3(256), 0, s>>>(blocks, xp, z);
    BEM_HIP(hipGetLastError());
    k_h_rows<<<dim3(blocks_1d(2 * NV, 256)), dim3(256), 0, s>>>(rowptr, rowz, z, perm, rowD, rowN, NV, y);
    BEM_HIP(hipGetLastError());
}

}  // namespace bem
