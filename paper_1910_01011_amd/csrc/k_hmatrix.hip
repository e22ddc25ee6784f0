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

constexpr int HB_THREADS = 256;
constexpr int HB_XS_MAX = 1024;   // columns of x_J staged in LDS for V x_J

__device__ __forceinline__ void cmac(double &sr, double &si, float dx, float dy, double2 v)
{
    sr += double(dx) * v.x - double(dy) * v.y;
    si += double(dx) * v.y + double(dy) * v.x;
}

// zb = A v for a column-major (2 m) x ncol complex64 matrix A, rows taken in
// pairs (one 16-byte load holds rows 2 j and 2 j + 1 of a column).  With
// m <= 128 the columns are split over G = 256 / m thread groups whose FP64
// partial sums are added in group order through LDS; larger m loop over row
// pairs with all columns per thread.  Every thread of the workgroup calls it.
__device__ __forceinline__ void colmajor_apply(const float2 *__restrict__ A, int m, int64_t ncol, const double2 *vec,
                               double2 *__restrict__ zb, double2 *part)
{
    const int tid = threadIdx.x;
    const int P = min(m, HB_THREADS), G = HB_THREADS / P;
    const int j0 = tid % P, g = tid / P;
    if (G == 1) {
        if (g != 0) return;
        for (int j = j0; j < m; j += P) {
            double ar = 0, ai = 0, br = 0, bi = 0;
            int64_t c = 0;
            for (; c + 4 <= ncol; c += 4) {
                float4 d[4];
                double2 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    d[u] = load_streamed(A + 2 * ((c + u) * m + j));
                    v[u] = vec[c + u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    cmac(ar, ai, d[u].x, d[u].y, v[u]);
                    cmac(br, bi, d[u].z, d[u].w, v[u]);
                }
            }
            for (; c < ncol; ++c) {
                const float4 d = load_streamed(A + 2 * (c * m + j));
                const double2 v = vec[c];
                cmac(ar, ai, d.x, d.y, v);
                cmac(br, bi, d.z, d.w, v);
            }
            zb[2 * j] = make_double2(ar, ai);
            zb[2 * j + 1] = make_double2(br, bi);
        }
        return;
    }
    // m <= 128: one row pair per thread, G >= 2 column groups
    double ar = 0, ai = 0, br = 0, bi = 0;
    if (g < G) {
        int64_t c = g;
        for (; c + 3 * G < ncol; c += 4 * G) {
            float4 d[4];
            double2 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                d[u] = load_streamed(A + 2 * ((c + u * G) * m + j0));
                v[u] = vec[c + u * G];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                cmac(ar, ai, d[u].x, d[u].y, v[u]);
                cmac(br, bi, d[u].z, d[u].w, v[u]);
            }
        }
        for (; c < ncol; c += G) {
            const float4 d = load_streamed(A + 2 * (c * m + j0));
            const double2 v = vec[c];
            cmac(ar, ai, d.x, d.y, v);
            cmac(br, bi, d.z, d.w, v);
        }
    }
    part[2 * tid] = make_double2(ar, ai);
    part[2 * tid + 1] = make_double2(br, bi);
    __syncthreads();
    if (g == 0) {
        double sr0 = 0, si0 = 0, sr1 = 0, si1 = 0;
        for (int q = 0; q < G; ++q) {
            const double2 a = part[2 * (q * P + j0)], b = part[2 * (q * P + j0) + 1];
            sr0 += a.x;
            si0 += a.y;
            sr1 += b.x;
            si1 += b.y;
        }
        zb[2 * j0] = make_double2(sr0, si0);
        zb[2 * j0 + 1] = make_double2(sr1, si1);
    }
}

// t[k + i dk] (+)= row k + i dk of V (columns c0 ... c0 + 2 np - 1) times the
// staged x_J chunk, for i < NR rows at once so that the loads of one row are in
// flight while another is reduced; whole-wave call, lane 0 writes
template <int NR>
__device__ __forceinline__ void v_rows(const float2 *__restrict__ V, int64_t n2, int64_t c0, int np, int k, int dk,
                                       const double2 *xs, double2 *t)
{
    const int lane = threadIdx.x & 63;
    double sr[NR], si[NR];
    const float2 *vr[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        sr[i] = si[i] = 0.0;
        vr[i] = V + int64_t(k + i * dk) * n2 + c0;
    }
    int cp = lane;
    for (; cp + 64 < np; cp += 128) {
        float4 d0[NR], d1[NR];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            d0[i] = load_streamed(vr[i] + 2 * cp);
            d1[i] = load_streamed(vr[i] + 2 * (cp + 64));
        }
        const double2 x0 = xs[2 * cp], x1 = xs[2 * cp + 1], x2 = xs[2 * cp + 128], x3 = xs[2 * cp + 129];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            cmac(sr[i], si[i], d0[i].x, d0[i].y, x0);
            cmac(sr[i], si[i], d0[i].z, d0[i].w, x1);
            cmac(sr[i], si[i], d1[i].x, d1[i].y, x2);
            cmac(sr[i], si[i], d1[i].z, d1[i].w, x3);
        }
    }
    for (; cp < np; cp += 64) {
        const double2 x0 = xs[2 * cp], x1 = xs[2 * cp + 1];
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            const float4 d = load_streamed(vr[i] + 2 * cp);
            cmac(sr[i], si[i], d.x, d.y, x0);
            cmac(sr[i], si[i], d.z, d.w, x1);
        }
    }
#pragma unroll
    for (int i = 0; i < NR; ++i)
        for (int off = 32; off > 0; off >>= 1) {
            sr[i] += __shfl_xor(sr[i], off);
            si[i] += __shfl_xor(si[i], off);
        }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < NR; ++i) {
            double2 &o = t[k + i * dk];
            o = c0 == 0 ? make_double2(sr[i], si[i]) : make_double2(o.x + sr[i], o.y + si[i]);
        }
}

// one workgroup per block: z[zoff + a] = (D x_J)[a], or (U (V x_J))[a] with
// the r values V x_J (x_J staged in LDS, two columns per lane and load,
// reduced per wave) kept in LDS, then U t; FP64 sums in a fixed order
__global__ __launch_bounds__(HB_THREADS) void k_h_blocks(const HBlock *__restrict__ blocks,
                                                         const double2 *__restrict__ xp, double2 *__restrict__ z)
{
    __shared__ double2 t[HK_MAX];
    __shared__ double2 part[2 * HB_THREADS];
    __shared__ double2 xs[HB_XS_MAX];
    const HBlock B = blocks[blockIdx.x];
    const int m = B.r1 - B.r0, nc = B.c1 - B.c0;   // vertices on each side
    const int64_t n2 = 2 * int64_t(nc);
    const double2 *xj = xp + 2 * int64_t(B.c0);
    double2 *zb = z + B.zoff;
    if (B.rank < 0) {
        colmajor_apply(B.D, m, n2, xj, zb, part);
        return;
    }
    // t = V x_J over chunks of HB_XS_MAX columns of x_J staged in LDS; lane 0
    // of the wave that owns row k adds each chunk's sum to t[k] in chunk order
    const int w = threadIdx.x >> 6;
    for (int64_t c0 = 0; c0 < n2; c0 += HB_XS_MAX) {
        const int cn = int(min(int64_t(HB_XS_MAX), n2 - c0)), np = cn / 2;
        __syncthreads();
        for (int c = threadIdx.x; c < cn; c += HB_THREADS) xs[c] = xj[c0 + c];
        __syncthreads();
        int k = w;
        for (; k + HB_THREADS / 64 < B.rank; k += 2 * (HB_THREADS / 64))
            v_rows<2>(B.V, n2, c0, np, k, HB_THREADS / 64, xs, t);
        for (; k < B.rank; k += HB_THREADS / 64) v_rows<1>(B.V, n2, c0, np, k, HB_THREADS / 64, xs, t);
    }
    __syncthreads();
    colmajor_apply(B.U, m, B.rank, t, zb, part);
}

// y[row_s(perm[i])] = sum of the block products of reordered row 2 i + s:
// 16 lanes per row, each summing every 16th entry of the row's list, then a
// fixed shuffle tree (deterministic, no atomics)
__global__ void k_h_rows(const int32_t *__restrict__ rowptr, const int32_t *__restrict__ rowz,
                         const double2 *__restrict__ z, const int32_t *__restrict__ perm,
                         const int32_t *__restrict__ rowD, const int32_t *__restrict__ rowN, int64_t NV,
                         double2 *__restrict__ y)
{
    const int64_t r = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 4;
    const int sub = threadIdx.x & 15;
    double sr = 0.0, si = 0.0;
    if (r < 2 * NV)
        for (int32_t e = rowptr[r] + sub; e < rowptr[r + 1]; e += 16) {
            const double2 v = z[rowz[e]];
            sr += v.x;
            si += v.y;
        }
    for (int off = 8; off > 0; off >>= 1) {
        sr += __shfl_xor(sr, off);
        si += __shfl_xor(si, off);
    }
    if (sub == 0 && r < 2 * NV) {
        const int32_t g = perm[r >> 1];
        y[(r & 1) ? rowN[g] : rowD[g]] = make_double2(sr, si);
    }
}

void launch_h_apply(hipStream_t s, const HBlock *blocks, int n_blocks, const int32_t *perm, const int32_t *rowD,
                    const int32_t *rowN, const int32_t *rowptr, const int32_t *rowz, int64_t NV, const double2 *x,
                    double2 *xp, double2 *z, double2 *y)
{
    k_h_gather<<<dim3(blocks_1d(2 * NV, 256)), dim3(256), 0, s>>>(perm, rowD, rowN, x, NV, xp);
    BEM_HIP(hipGetLastError());
    k_h_blocks<<<dim3(unsigned(n_blocks)), dim3(HB_THREADS), 0, s>>>(blocks, xp, z);
    BEM_HIP(hipGetLastError());
    k_h_rows<<<dim3(blocks_1d(2 * NV * 16, 256)), dim3(256), 0, s>>>(rowptr, rowz, z, perm, rowD, rowN, NV, y);
    BEM_HIP(hipGetLastError());
}

}  // namespace bem
