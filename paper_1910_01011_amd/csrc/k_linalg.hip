// FP64 complex vector kernels for the GMRES driver: several inner products
// against one vector (two-stage, fixed-order reduction), multi-axpy and
// scaling.  Vectors are double2 (re, im).
#include "bem_internal.h"

namespace bem {

constexpr int LA_BLOCK = 256;

// partials[k][blk] = sum over the block's chunk of conj(V_k[i]) w[i]
__global__ __launch_bounds__(LA_BLOCK) void k_zdot_partial(const double2 *__restrict__ V, int64_t ld,
                                                           const double2 *__restrict__ w, int64_t n, int nblk,
                                                           double2 *__restrict__ partials)
{
    __shared__ double sr[LA_BLOCK], si[LA_BLOCK];
    const int k = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
    const double2 *v = V + int64_t(k) * ld;
    double ar = 0, ai = 0;
    for (int64_t i = int64_t(blk) * LA_BLOCK + tid; i < n; i += int64_t(nblk) * LA_BLOCK) {
        const double2 a = v[i], b = w[i];
        ar += a.x * b.x + a.y * b.y;
        ai += a.x * b.y - a.y * b.x;
    }
    sr[tid] = ar;
    si[tid] = ai;
    __syncthreads();
    for (int s = LA_BLOCK / 2; s > 0; s >>= 1) {
        if (tid < s) {
            sr[tid] += sr[tid + s];
            si[tid] += si[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) partials[int64_t(k) * nblk + blk] = make_double2(sr[0], si[0]);
}

__global__ void k_zdot_final(const double2 *__restrict__ partials, int nblk, int nvec, double2 *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nvec) return;
    double r = 0, im = 0;
    for (int b = 0; b < nblk; ++b) {
        r += partials[int64_t(k) * nblk + b].x;
        im += partials[int64_t(k) * nblk + b].y;
    }
    out[k] = make_double2(r, im);
}

void zdot_multi(hipStream_t s, const double2 *V, int64_t ld, int nvec, const double2 *w, int64_t n,
                double2 *partials, int nblk, double2 *out_dev)
{
    if (nvec <= 0) return;
    k_zdot_partial<<<dim3(unsigned(nblk), unsigned(nvec)), dim3(LA_BLOCK), 0, s>>>(V, ld, w, n, nblk, partials);
    BEM_HIP(hipGetLastError());
    k_zdot_final<<<dim3(blocks_1d(nvec, 64)), dim3(64), 0, s>>>(partials, nblk, nvec, out_dev);
    BEM_HIP(hipGetLastError());
}

// w += sign * sum_k h_k V_k
__global__ void k_zaxpy_multi(const double2 *__restrict__ V, int64_t ld, int nvec, const double2 *__restrict__ h,
                              double2 *__restrict__ w, int64_t n, double sign)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double r = 0, im = 0;
    for (int k = 0; k < nvec; ++k) {
        const double2 a = V[int64_t(k) * ld + i], c = h[k];
        r += c.x * a.x - c.y * a.y;
        im += c.x * a.y + c.y * a.x;
    }
    w[i] = make_double2(w[i].x + sign * r, w[i].y + sign * im);
}

void zaxpy_multi(hipStream_t s, const double2 *V, int64_t ld, int nvec, const double2 *h_dev, double2 *w, int64_t n,
                 double sign)
{
    if (nvec <= 0 || n <= 0) return;
    k_zaxpy_multi<<<dim3(blocks_1d(n, 256)), dim3(256), 0, s>>>(V, ld, nvec, h_dev, w, n, sign);
    BEM_HIP(hipGetLastError());
}

__global__ void k_zscale_copy(const double2 *__restrict__ x, double2 *__restrict__ y, int64_t n, double2 a)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 v = x[i];
    y[i] = make_double2(a.x * v.x - a.y * v.y, a.x * v.y + a.y * v.x);
}

void zscale_copy(hipStream_t s, const double2 *x, double2 *y, int64_t n, double2 a)
{
    if (n <= 0) return;
    k_zscale_copy<<<dim3(blocks_1d(n, 256)), dim3(256), 0, s>>>(x, y, n, a);
    BEM_HIP(hipGetLastError());
}

__global__ void k_zaxpy(double2 *__restrict__ y, const double2 *__restrict__ x, int64_t n, double2 a)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 v = x[i];
    y[i] = make_double2(y[i].x + a.x * v.x - a.y * v.y, y[i].y + a.x * v.y + a.y * v.x);
}

void zaxpy(hipStream_t s, double2 *y, const double2 *x, int64_t n, double2 a)
{
    if (n <= 0) return;
    k_zaxpy<<<dim3(blocks_1d(n, 256)), dim3(256), 0, s>>>(y, x, n, a);
    BEM_HIP(hipGetLastError());
}

}  // namespace bem

namespace bem {

// ---------------------------------------------------------------------------
// batched kernels: R independent vectors of length n stored contiguously
// (vector r at offset r * n); Krylov bases as [i][R][n].
// ---------------------------------------------------------------------------

// partials[(r * nvec + i) * nchunk + c] = sum over chunk c of conj(V_i[r]) w[r].
// One workgroup per (chunk of BD_CHUNK elements, right-hand side): the chunk of
// w stays in registers while the basis vectors are streamed in groups of
// BD_G; each sum is reduced across the wave by shuffles and across the four
// waves through LDS, always in the same order (deterministic).
constexpr int BD_T = BD_CHUNK / LA_BLOCK;   // elements per thread
constexpr int BD_G = 8;                     // basis vectors per pass
__global__ __launch_bounds__(LA_BLOCK) void k_bdot_partial(const double2 *__restrict__ V, int64_t ldv,
                                                           const double2 *__restrict__ w, int64_t n, int R,
                                                           int nvec, int nchunk, double2 *__restrict__ partials)
{
    __shared__ double2 red[LA_BLOCK / 64][BD_G];
    const int c = blockIdx.x, r = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t base = int64_t(c) * BD_CHUNK + tid;
    const double2 *ww = w + int64_t(r) * n;
    double2 wl[BD_T];
#pragma unroll
    for (int t = 0; t < BD_T; ++t) {
        const int64_t k = base + int64_t(LA_BLOCK) * t;
        wl[t] = k < n ? ww[k] : make_double2(0.0, 0.0);
    }
    for (int i0 = 0; i0 < nvec; i0 += BD_G) {
        double ar[BD_G], ai[BD_G];
#pragma unroll
        for (int g = 0; g < BD_G; ++g) {
            ar[g] = 0.0;
            ai[g] = 0.0;
            if (i0 + g < nvec) {
                const double2 *v = V + int64_t(i0 + g) * ldv + int64_t(r) * n;
#pragma unroll
                for (int t = 0; t < BD_T; ++t) {
                    const int64_t k = base + int64_t(LA_BLOCK) * t;
                    const double2 a = k < n ? v[k] : make_double2(0.0, 0.0);
                    ar[g] += a.x * wl[t].x + a.y * wl[t].y;
                    ai[g] += a.x * wl[t].y - a.y * wl[t].x;
                }
            }
        }
#pragma unroll
        for (int g = 0; g < BD_G; ++g)
            for (int off = 32; off > 0; off >>= 1) {
                ar[g] += __shfl_down(ar[g], off);
                ai[g] += __shfl_down(ai[g], off);
            }
        if (lane == 0)
#pragma unroll
            for (int g = 0; g < BD_G; ++g) red[wv][g] = make_double2(ar[g], ai[g]);
        __syncthreads();
        if (tid < BD_G && i0 + tid < nvec) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int q = 0; q < LA_BLOCK / 64; ++q) {
                sr += red[q][tid].x;
                si += red[q][tid].y;
            }
            partials[(int64_t(r) * nvec + i0 + tid) * nchunk + c] = make_double2(sr, si);
        }
        __syncthreads();
    }
}

__global__ void k_bdot_final(const double2 *__restrict__ partials, int nblk, int total, double2 *__restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= total) return;
    double re = 0, im = 0;
    for (int b = 0; b < nblk; ++b) {
        re += partials[int64_t(k) * nblk + b].x;
        im += partials[int64_t(k) * nblk + b].y;
    }
    out[k] = make_double2(re, im);
}

void bdot(hipStream_t s, const double2 *V, int64_t ldv, int nvec, const double2 *w, int64_t n, int R,
          double2 *partials, int nblk, double2 *out_dev)
{
    if (nvec <= 0 || R <= 0) return;
    if (nblk != bdot_chunks(n)) throw Error{BEM_ERR_INVALID_ARG, "bdot: partial buffer sized for another length"};
    k_bdot_partial<<<dim3(unsigned(nblk), unsigned(R)), dim3(LA_BLOCK), 0, s>>>(V, ldv, w, n, R, nvec, nblk, partials);
    BEM_HIP(hipGetLastError());
    const int total = R * nvec;
    k_bdot_final<<<dim3(blocks_1d(total, 64)), dim3(64), 0, s>>>(partials, nblk, total, out_dev);
    BEM_HIP(hipGetLastError());
}

// w[r] += sign * sum_i h[r * nvec + i] V_i[r]
__global__ void k_baxpy(const double2 *__restrict__ V, int64_t ldv, int nvec, const double2 *__restrict__ h,
                        double2 *__restrict__ w, int64_t n, int R, double sign)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    const int64_t r = idx / n;
    double re = 0, im = 0;
#pragma unroll 4
    for (int i = 0; i < nvec; ++i) {
        const double2 a = V[int64_t(i) * ldv + idx], c = h[r * nvec + i];
        re += c.x * a.x - c.y * a.y;
        im += c.x * a.y + c.y * a.x;
    }
    w[idx] = make_double2(w[idx].x + sign * re, w[idx].y + sign * im);
}

void baxpy(hipStream_t s, const double2 *V, int64_t ldv, int nvec, const double2 *h_dev, double2 *w, int64_t n, int R,
           double sign)
{
    if (nvec <= 0 || n * R <= 0) return;
    k_baxpy<<<dim3(blocks_1d(n * R, 256)), dim3(256), 0, s>>>(V, ldv, nvec, h_dev, w, n, R, sign);
    BEM_HIP(hipGetLastError());
}

// y[r] = a[r] * x[r]   (complex per-vector scalars)
__global__ void k_bscale(const double2 *__restrict__ x, double2 *__restrict__ y, int64_t n, int R,
                         const double2 *__restrict__ a)
{
    const int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= n * R) return;
    const double2 c = a[idx / n], v = x[idx];
    y[idx] = make_double2(c.x * v.x - c.y * v.y, c.x * v.y + c.y * v.x);
}

void bscale(hipStream_t s, const double2 *x, double2 *y, int64_t n, int R, const double2 *a_dev)
{
    if (n * R <= 0) return;
    k_bscale<<<dim3(blocks_1d(n * R, 256)), dim3(256), 0, s>>>(x, y, n, R, a_dev);
    BEM_HIP(hipGetLastError());
}

}  // namespace bem
