// Lanczos iteration on the GPU (eigval0 / eigvals_lanczos, Sec. 3.7.1; the
// recurrence of Lanczos 1950):
//   w = H v_j;  alpha_j = Re<v_j, w>;  w -= alpha_j v_j + beta_j v_{j-1};
//   [optional: classical Gram-Schmidt against all v_i, twice];
//   beta_{j+1} = |w|;  v_{j+1} = w / beta_{j+1}.
// Vectors are stored in FP64 or FP32 (complex if the block is); every dot
// product, norm, coefficient and the three-term update are computed in FP64
// and rounded once on store.  Reductions use fixed-order block partials, so
// the scalars are bitwise reproducible.  The scalars live on the device
// (no host round trip per step); the host reads them back to test
// convergence and solves the tridiagonal problem with the implicit QL
// method (Bowdler, Martin, Reinsch and Wilkinson, 1968).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "xdg_internal.hpp"

namespace xdg {

namespace {
constexpr int RB = 256;    // threads per block of the vector kernels
constexpr int MAXC = 16;   // scalar columns per row (nvec <= 8, complex)

// Sum over threads that share a column (t = column mod cols, cols a power of
// two dividing RB); sh[0 .. cols) holds the block totals afterwards.
__device__ inline void block_col_reduce(double *sh, int cols) {
    for (int s = RB / 2; s >= cols; s >>= 1) {
        __syncthreads();
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    }
    __syncthreads();
}

// partials[block][c] = sum over the block's scalars of column c of a*b.
// The flat scalar index q has column q % cols because the grid stride is a
// multiple of cols.
template <class T>
__global__ __launch_bounds__(RB) void k_dot(const T *a, const T *b, uint64_t n, int cols,
                                            double *partials) {
    __shared__ double sh[RB];
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * RB;
    for (uint64_t q = (uint64_t)blockIdx.x * RB + threadIdx.x; q < n; q += stride)
        acc += (double)a[q] * (double)b[q];
    sh[threadIdx.x] = acc;
    block_col_reduce(sh, cols);
    if ((int)threadIdx.x < cols) partials[(size_t)blockIdx.x * cols + threadIdx.x] = sh[threadIdx.x];
}

// Fixed-order total of the partials, pairs of columns combined for complex
// vectors (Re<a,b> = sum re*re + im*im).  mode 0: out = s; 1: out = sqrt(s).
// hist (may be null) receives the value at row *jdev.
__global__ __launch_bounds__(RB) void k_finalize(const double *partials, int n_blocks, int cols,
                                                 int C, int mode, double *out, double *hist,
                                                 const int *jdev) {
    __shared__ double sh[RB];
    const int c = threadIdx.x % cols;
    double acc = 0.0;
    for (int blk = threadIdx.x / cols; blk < n_blocks; blk += RB / cols)
        acc += partials[(size_t)blk * cols + c];
    sh[threadIdx.x] = acc;
    block_col_reduce(sh, cols);
    if ((int)threadIdx.x < cols / C) {
        const int v = threadIdx.x;
        double s = sh[v * C];
        if (C == 2) s += sh[v * C + 1];
        const double r = mode == 1 ? sqrt(s) : s;
        out[v] = r;
        if (hist) hist[(size_t)(*jdev) * (cols / C) + v] = r;
    }
}

// w = w - alpha v - beta vprev (FP64, one rounding), partial |w|^2
template <class T>
__global__ __launch_bounds__(RB) void k_update(T *w, const T *v, const T *vprev, uint64_t n,
                                               int cols, int C, const double *alpha,
                                               const double *beta, double *partials) {
    __shared__ double sh[RB];
    double acc = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * RB;
    // cols divides RB, so every scalar of this thread is in column threadIdx.x % cols
    const int vec = (int)(threadIdx.x % cols) / C;
    const double a = alpha[vec], b = vprev ? beta[vec] : 0.0;
    for (uint64_t q = (uint64_t)blockIdx.x * RB + threadIdx.x; q < n; q += stride) {
        double x = (double)w[q] - a * (double)v[q];
        if (vprev) x -= b * (double)vprev[q];
        const T r = (T)x;
        w[q] = r;
        acc += (double)r * (double)r;
    }
    sh[threadIdx.x] = acc;
    block_col_reduce(sh, cols);
    if ((int)threadIdx.x < cols) partials[(size_t)blockIdx.x * cols + threadIdx.x] = sh[threadIdx.x];
}

// dst = src / beta  (zero where beta vanished: invariant subspace)
template <class T>
__global__ __launch_bounds__(RB) void k_scale(const T *src, T *dst, uint64_t n, int cols, int C,
                                              const double *beta) {
    const uint64_t stride = (uint64_t)gridDim.x * RB;
    // cols divides RB, so every scalar of this thread is in column threadIdx.x % cols
    const double bt = beta[(int)(threadIdx.x % cols) / C];
    for (uint64_t q = (uint64_t)blockIdx.x * RB + threadIdx.x; q < n; q += stride)
        dst[q] = bt > 0.0 ? (T)((double)src[q] / bt) : T(0);
}

// One column (a single real vector): four consecutive scalars per thread
// through one vector load each, the same arithmetic per scalar as the
// kernels above.  Scalars past the last full group of four go to block 0.
template <class T>
using Vec4 = T __attribute__((ext_vector_type(4)));

template <class T>
__global__ __launch_bounds__(RB) void k_dot1(const T *a, const T *b, uint64_t n,
                                             double *partials) {
    __shared__ double sh[RB];
    double acc = 0.0;
    const uint64_t n4 = n / 4, stride = (uint64_t)gridDim.x * RB;
    for (uint64_t q = (uint64_t)blockIdx.x * RB + threadIdx.x; q < n4; q += stride) {
        const Vec4<T> x = reinterpret_cast<const Vec4<T> *>(a)[q];
        const Vec4<T> y = reinterpret_cast<const Vec4<T> *>(b)[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) acc += (double)x[e] * (double)y[e];
    }
    if (blockIdx.x == 0)
        for (uint64_t q = 4 * n4 + threadIdx.x; q < n; q += RB) acc += (double)a[q] * (double)b[q];
    sh[threadIdx.x] = acc;
    block_col_reduce(sh, 1);
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

template <class T>
__global__ __launch_bounds__(RB) void k_update1(T *w, const T *v, const T *vprev, uint64_t n,
                                                const double *alpha, const double *beta,
                                                double *partials) {
    __shared__ double sh[RB];
    double acc = 0.0;
    const double a = alpha[0], b = vprev ? beta[0] : 0.0;
    const uint64_t n4 = n / 4, stride = (uint64_t)gridDim.x * RB;
    for (uint64_t q = (uint64_t)blockIdx.x * RB + threadIdx.x; q < n4; q += stride) {
        Vec4<T> x = reinterpret_cast<const Vec4<T> *>(w)[q];
        const Vec4<T> y = reinterpret_cast<const Vec4<T> *>(v)[q];
        Vec4<T> z = {};
        if (vprev) z = reinterpret_cast<const Vec4<T> *>(vprev)[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double t = (double)x[e] - a * (double)y[e];
            if (vprev) t -= b * (double)z[e];
            const T r = (T)t;
            x[e] = r;
            acc += (double)r * (double)r;
        }
        reinterpret_cast<Vec4<T> *>(w)[q] = x;
    }
    if (blockIdx.x == 0)
        for (uint64_t q = 4 * n4 + threadIdx.x; q < n; q += RB) {
            double t = (double)w[q] - a * (double)v[q];
            if (vprev) t -= b * (double)vprev[q];
            const T r = (T)t;
            w[q] = r;
            acc += (double)r * (double)r;
        }
    sh[threadIdx.x] = acc;
    block_col_reduce(sh, 1);
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

template <class T>
__global__ __launch_bounds__(RB) void k_scale1(const T *src, T *dst, uint64_t n,
                                               const double *beta) {
    const double bt = beta[0];
    const uint64_t n4 = n / 4, stride = (uint64_t)gridDim.x * RB;
    for (uint64_t q = (uint64_t)blockIdx.x * RB + threadIdx.x; q < n4; q += stride) {
        Vec4<T> x = reinterpret_cast<const Vec4<T> *>(src)[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) x[e] = bt > 0.0 ? (T)((double)x[e] / bt) : T(0);
        reinterpret_cast<Vec4<T> *>(dst)[q] = x;
    }
    if (blockIdx.x == 0)
        for (uint64_t q = 4 * n4 + threadIdx.x; q < n; q += RB)
            dst[q] = bt > 0.0 ? (T)((double)src[q] / bt) : T(0);
}

__global__ void k_step_end(int *jdev, double *prev_beta, const double *cur_beta, int nv) {
    for (int v = threadIdx.x; v < nv; v += blockDim.x) prev_beta[v] = cur_beta[v];
    __syncthreads();
    if (threadIdx.x == 0 && jdev) *jdev += 1;
}

__global__ void k_set_scalars(int *jdev, double *prev_beta, int nv) {
    for (int v = threadIdx.x; v < nv; v += blockDim.x) prev_beta[v] = 0.0;
    if (threadIdx.x == 0) *jdev = 0;
}

// Reorthogonalisation of one vector against the stored Krylov vectors V_i,
// i < k (classical Gram-Schmidt: the coefficients c_i = <V_i, w> first, then
// w -= sum_i c_i V_i; complex when C = 2, conj(V_i) in the product).  Both
// kernels stream row tiles: each thread owns ru 16-byte chunks of a tile
// (L = 16 / sizeof(T) scalars each, consecutive threads on consecutive
// chunks), so a block covers RB * ru * L scalars and a column is read with
// ru independent 16-byte loads per thread; RG columns are in flight at once.
// Sums are FP64 in a fixed order (bitwise reproducible).
// 16-byte chunks per thread and column: eight scalars per thread for both
// types (FP32 with four chunks held too many registers for enough waves)
template <class T>
constexpr int ru() { return sizeof(T) == 4 ? 2 : 4; }
constexpr int RG = 4;   // columns per step

template <class T> struct Chunk16;
template <> struct Chunk16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
};
template <> struct Chunk16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};

template <class T>
constexpr int tile_scalars() { return RB * ru<T>() * (16 / (int)sizeof(T)); }

// scalars [q, q + L) of column `col` (zero beyond n): one 16-byte load when
// the chunk is whole, scalar loads at the ragged end
template <class T>
__device__ __forceinline__ void load_chunk(const T *col, uint64_t q, uint64_t n, T *out) {
    constexpr int L = 16 / (int)sizeof(T);
    if (q + L <= n) {
        typedef typename Chunk16<T>::type V16;
        const V16 v = *(const __attribute__((address_space(1))) V16 *)(col + q);
#pragma unroll
        for (int e = 0; e < L; ++e) out[e] = v[e];
    } else {
#pragma unroll
        for (int e = 0; e < L; ++e) out[e] = q + e < n ? col[q + e] : T(0);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// N values per lane summed over the wave together: each exchange step first
// halves the values a lane keeps (the lanes of one half of the exchange keep
// the lower values, the others the upper ones), then the last value is
// summed over the remaining lane groups.  Lane l returns the wave total of
// value l / (64 / N): N - 1 + 6 - log2(N) exchanges of a double instead of 6 N.
template <int N>
__device__ __forceinline__ double wave_sum_n(double (&v)[N], int lane) {
    static_assert(N == 1 || N == 2 || N == 4 || N == 8, "N in {1, 2, 4, 8}");
    int o = 32;
#pragma unroll
    for (int n = N; n > 1; n >>= 1, o >>= 1) {
        const bool up = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < n / 2; ++i) {
            const double keep = up ? v[i + n / 2] : v[i];
            const double send = up ? v[i] : v[i + n / 2];
            v[i] = keep + __shfl_xor(send, o, 64);
        }
    }
    double r = v[0];
#pragma unroll
    for (; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
    return r;
}

// partials[(i C + c) nb + block] = the block's share of Re / Im <V_i, w>.
// skip (may be null): a device flag; when set the pass does nothing.
template <class T, int C>
__global__ __launch_bounds__(RB) void k_reorth_dots(const T *V, uint64_t ld, int k, const T *w,
                                                    uint64_t nsc, double *partials,
                                                    const int *skip) {
    if (skip && *skip) return;
    constexpr int RU = ru<T>(), L = 16 / (int)sizeof(T), S = RU * L;
    __shared__ double sh[RB / 64][RG * C];
    const int nb = gridDim.x, t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const uint64_t tile0 = (uint64_t)blockIdx.x * tile_scalars<T>();
    T wr[S];
#pragma unroll
    for (int u = 0; u < RU; ++u)
        load_chunk<T>(w, tile0 + ((uint64_t)u * RB + t) * L, nsc, wr + u * L);
    for (int i0 = 0; i0 < k; i0 += RG) {
        T vr[RG][S];
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            const int i = i0 + g < k ? i0 + g : k - 1;   // a repeated column is discarded
#pragma unroll
            for (int u = 0; u < RU; ++u)
                load_chunk<T>(V + (size_t)i * ld, tile0 + ((uint64_t)u * RB + t) * L, nsc,
                              vr[g] + u * L);
        }
        double part[RG * C];   // value g C + c: Re (c = 0) / Im of <V_{i0+g}, w>
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int e = 0; e < S; e += C) {
                if (C == 1) {
                    re = fma((double)vr[g][e], (double)wr[e], re);
                } else {
                    const double a = vr[g][e], b = vr[g][e + 1], x = wr[e], y = wr[e + 1];
                    re = fma(a, x, fma(b, y, re));       // conj(V) w
                    im = fma(a, y, fma(-b, x, im));
                }
            }
            part[g * C] = re;
            if (C == 2) part[g * C + 1] = im;
        }
        {
            constexpr int Q = 64 / (RG * C);   // lanes per value after the exchanges
            const double r = wave_sum_n<RG * C>(part, lane);
            if ((lane & (Q - 1)) == 0) sh[wave][lane / Q] = r;
        }
        __syncthreads();
        if (t < RG * C && i0 + t / C < k) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < RB / 64; ++q) s += sh[q][t];
            partials[((size_t)(i0 + t / C) * C + t % C) * nb + blockIdx.x] = s;
        }
        __syncthreads();
    }
}

// coef[2 i + c] = sum over blocks (fixed order) of the partials; one block
// per (i, c); coef[2 i + 1] = 0 for real vectors
template <int C>
__global__ __launch_bounds__(RB) void k_reorth_finalize(const double *partials, int n_blocks,
                                                        double *coef, const int *skip) {
    if (skip && *skip) return;
    __shared__ double sh[RB];
    const int e = blockIdx.x;   // i C + c
    double s = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += RB) s += partials[(size_t)e * n_blocks + b];
    sh[threadIdx.x] = s;
    block_col_reduce(sh, 1);
    if (threadIdx.x == 0) {
        const int i = e / C, c = e % C;
        coef[2 * i + c] = sh[0];
        if (C == 1) coef[2 * i + 1] = 0.0;
    }
}

// w -= sum_i c_i V_i, accumulated in FP64 and rounded once on store
template <class T, int C>
__global__ __launch_bounds__(RB) void k_reorth_sub(const T *V, uint64_t ld, int k,
                                                   const double *coef, T *w, uint64_t nsc,
                                                   const int *skip) {
    if (skip && *skip) return;
    constexpr int RU = ru<T>(), L = 16 / (int)sizeof(T), S = RU * L;
    const int t = threadIdx.x;
    const uint64_t tile0 = (uint64_t)blockIdx.x * tile_scalars<T>();
    double acc[S];
    {
        T w0[S];
#pragma unroll
        for (int u = 0; u < RU; ++u)
            load_chunk<T>(w, tile0 + ((uint64_t)u * RB + t) * L, nsc, w0 + u * L);
#pragma unroll
        for (int e = 0; e < S; ++e) acc[e] = (double)w0[e];
    }
    for (int i0 = 0; i0 < k; i0 += RG) {
        T vr[RG][S];
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            const int i = i0 + g < k ? i0 + g : k - 1;
#pragma unroll
            for (int u = 0; u < RU; ++u)
                load_chunk<T>(V + (size_t)i * ld, tile0 + ((uint64_t)u * RB + t) * L, nsc,
                              vr[g] + u * L);
        }
#pragma unroll
        for (int g = 0; g < RG; ++g) {
            if (i0 + g >= k) break;
            const double cr = coef[2 * (i0 + g)], ci = coef[2 * (i0 + g) + 1];
#pragma unroll
            for (int e = 0; e < S; e += C) {
                if (C == 1) {
                    acc[e] = fma(-cr, (double)vr[g][e], acc[e]);
                } else {
                    const double a = vr[g][e], b = vr[g][e + 1];
                    acc[e] = fma(-cr, a, fma(ci, b, acc[e]));
                    acc[e + 1] = fma(-cr, b, fma(-ci, a, acc[e + 1]));
                }
            }
        }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) {
        const uint64_t q = tile0 + ((uint64_t)u * RB + t) * L;
        if (q + L <= nsc) {
            typedef typename Chunk16<T>::type V16;
            V16 v;
#pragma unroll
            for (int e = 0; e < L; ++e) v[e] = (T)acc[u * L + e];
            *(__attribute__((address_space(1))) V16 *)(w + q) = v;
        } else {
#pragma unroll
            for (int e = 0; e < L; ++e)
                if (q + e < nsc) w[q + e] = (T)acc[u * L + e];
        }
    }
}

// Second Gram-Schmidt pass only where the first removed more than half of
// |w|^2 (Daniel, Gragg, Kaufman and Stewart 1976, eta = 1/sqrt 2): skip = 1
// when |w'|^2 >= |w|^2 / 2 (no cancellation, w' orthogonal to working
// precision).
__global__ void k_dgks(const double *n0, const double *n1, int *skip) {
    if (threadIdx.x == 0) *skip = (*n1 >= 0.5 * *n0) ? 1 : 0;
}

int vec_grid(uint64_t n) {
    const uint64_t want = (n + RB - 1) / RB;
    return (int)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)device_cu_count() * 8));
}

// One family of vector kernels for a dtype.
struct VecOps {
    bool single;
    int cols, C;
    uint64_t n;        // scalars per vector block
    int grid;
    double *partials;  // [grid][cols]
    hipStream_t st;

    // one column and vector-aligned buffers: the four-wide kernels
    bool vec4(const void *p) const {
        return cols == 1 && ((uintptr_t)p % (single ? 16 : 32)) == 0;
    }
    int dot(const void *a, const void *b) const {
        if (vec4(a) && vec4(b)) {
            if (single)
                hipLaunchKernelGGL(k_dot1<float>, dim3(grid), dim3(RB), 0, st, (const float *)a,
                                   (const float *)b, n, partials);
            else
                hipLaunchKernelGGL(k_dot1<double>, dim3(grid), dim3(RB), 0, st, (const double *)a,
                                   (const double *)b, n, partials);
            XDG_TRY_HIP(hipGetLastError());
            return XDG_OK;
        }
        if (single)
            hipLaunchKernelGGL(k_dot<float>, dim3(grid), dim3(RB), 0, st, (const float *)a,
                               (const float *)b, n, cols, partials);
        else
            hipLaunchKernelGGL(k_dot<double>, dim3(grid), dim3(RB), 0, st, (const double *)a,
                               (const double *)b, n, cols, partials);
        XDG_TRY_HIP(hipGetLastError());
        return XDG_OK;
    }
    int finalize(int mode, double *out, double *hist, const int *jdev) const {
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RB), 0, st, partials, grid, cols, C, mode,
                           out, hist, jdev);
        XDG_TRY_HIP(hipGetLastError());
        return XDG_OK;
    }
    int update(void *w, const void *v, const void *vprev, const double *alpha,
               const double *beta) const {
        if (vec4(w) && vec4(v) && (!vprev || vec4(vprev))) {
            if (single)
                hipLaunchKernelGGL(k_update1<float>, dim3(grid), dim3(RB), 0, st, (float *)w,
                                   (const float *)v, (const float *)vprev, n, alpha, beta,
                                   partials);
            else
                hipLaunchKernelGGL(k_update1<double>, dim3(grid), dim3(RB), 0, st, (double *)w,
                                   (const double *)v, (const double *)vprev, n, alpha, beta,
                                   partials);
            XDG_TRY_HIP(hipGetLastError());
            return XDG_OK;
        }
        if (single)
            hipLaunchKernelGGL(k_update<float>, dim3(grid), dim3(RB), 0, st, (float *)w,
                               (const float *)v, (const float *)vprev, n, cols, C, alpha, beta,
                               partials);
        else
            hipLaunchKernelGGL(k_update<double>, dim3(grid), dim3(RB), 0, st, (double *)w,
                               (const double *)v, (const double *)vprev, n, cols, C, alpha, beta,
                               partials);
        XDG_TRY_HIP(hipGetLastError());
        return XDG_OK;
    }
    int scale(const void *src, void *dst, const double *beta) const {
        if (vec4(src) && vec4(dst)) {
            if (single)
                hipLaunchKernelGGL(k_scale1<float>, dim3(grid), dim3(RB), 0, st,
                                   (const float *)src, (float *)dst, n, beta);
            else
                hipLaunchKernelGGL(k_scale1<double>, dim3(grid), dim3(RB), 0, st,
                                   (const double *)src, (double *)dst, n, beta);
            XDG_TRY_HIP(hipGetLastError());
            return XDG_OK;
        }
        if (single)
            hipLaunchKernelGGL(k_scale<float>, dim3(grid), dim3(RB), 0, st, (const float *)src,
                               (float *)dst, n, cols, C, beta);
        else
            hipLaunchKernelGGL(k_scale<double>, dim3(grid), dim3(RB), 0, st, (const double *)src,
                               (double *)dst, n, cols, C, beta);
        XDG_TRY_HIP(hipGetLastError());
        return XDG_OK;
    }
};

// acc += c v (FP64 accumulation of the Ritz vector)
template <class T>
__global__ __launch_bounds__(RB) void k_acc_axpy(double *acc, const T *v, uint64_t n, double c) {
    const uint64_t stride = (uint64_t)gridDim.x * RB;
    for (uint64_t q = (uint64_t)blockIdx.x * RB + threadIdx.x; q < n; q += stride)
        acc[q] = __builtin_fma(c, (double)v[q], acc[q]);
}

// out = acc / nrm[0], one rounding to T
template <class T>
__global__ __launch_bounds__(RB) void k_acc_out(const double *acc, T *out, uint64_t n,
                                                const double *nrm) {
    const double s = nrm[0] > 0.0 ? 1.0 / nrm[0] : 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * RB;
    for (uint64_t q = (uint64_t)blockIdx.x * RB + threadIdx.x; q < n; q += stride)
        out[q] = (T)(acc[q] * s);
}

thread_local double g_t_total = 0.0, g_t_apply = 0.0;

// XDG_LANCZOS_PROGRESS=n: print a line to stderr every n iterations (0 = off)
int progress_every() {
    static int every = -1;
    if (every < 0) {
        const char *e = getenv("XDG_LANCZOS_PROGRESS");
        every = e ? std::max(0, atoi(e)) : 0;
    }
    return every;
}

}  // namespace

// Implicit QL with shifts taken from the leading 2x2 block (Bowdler, Martin,
// Reinsch, Wilkinson 1968) on the symmetric tridiagonal matrix with alpha on
// the diagonal and beta[i] coupling i and i+1.  d receives the eigenvalues
// (unsorted); z0, if given, the first components of the eigenvectors (the
// rotations applied to the first row of the identity).
static void tridiag_ql(int m, const double *alpha, const double *beta, std::vector<double> &d,
                       std::vector<double> *z0) {
    d.assign(alpha, alpha + m);
    std::vector<double> e(m, 0.0);
    for (int i = 0; i + 1 < m; ++i) e[i] = beta[i];
    if (z0) {
        z0->assign(m, 0.0);
        (*z0)[0] = 1.0;
    }
    for (int l = 0; l < m; ++l) {
        for (int sweep = 0; sweep < 200; ++sweep) {
            int q = l;
            while (q < m - 1) {
                const double scale = std::fabs(d[q]) + std::fabs(d[q + 1]);
                if (std::fabs(e[q]) <= 1e-16 * scale) break;
                ++q;
            }
            if (q == l) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[q] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            bool split = false;
            for (int i = q - 1; i >= l; --i) {
                const double f = s * e[i], bb = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[q] = 0.0;
                    split = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * bb;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - bb;
                if (z0) {
                    double &zi = (*z0)[i], &zj = (*z0)[i + 1];
                    const double t = zj;
                    zj = s * zi + c * t;
                    zi = c * zi - s * t;
                }
            }
            if (split) continue;
            d[l] -= p;
            e[l] = g;
            e[q] = 0.0;
        }
    }
}

// Eigenvalues of the symmetric tridiagonal matrix, ascending.
void tridiag_eigenvalues(int m, const double *alpha, const double *beta, std::vector<double> &out) {
    std::vector<double> d;
    tridiag_ql(m, alpha, beta, d, nullptr);
    std::sort(d.begin(), d.end());
    out = d;
}

// Eigenvalues (ascending) and the squared first components of their
// eigenvectors: the nodes and weights of the Gauss quadrature that the
// Lanczos recurrence defines for the start vector.
void tridiag_spectral_weights(int m, const double *alpha, const double *beta,
                              std::vector<double> &evals, std::vector<double> &weights) {
    std::vector<double> d, z;
    tridiag_ql(m, alpha, beta, d, &z);
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return d[a] < d[b]; });
    evals.resize(m);
    weights.resize(m);
    for (int i = 0; i < m; ++i) {
        evals[i] = d[order[i]];
        weights[i] = z[order[i]] * z[order[i]];
    }
}

int lanczos_single(xdg_ham_s *h, const void *v0, int k, double tol, int max_iter, uint64_t seed,
                   int prec, double *evals, int *n_iter, double *alpha, double *beta,
                   hipStream_t st, double *t_total, double *t_apply) {
    const xdg_basis_s *b = h->basis;
    if (k < 1 || max_iter < 1 || !evals || !n_iter || !(tol >= 0.0)) {
        set_error("lanczos: need k >= 1, max_iter >= 1, tol >= 0 and output pointers");
        return XDG_EINVAL;
    }
    if (prec < XDG_PREC_F64 || prec > XDG_PREC_F64_REORTH) {
        set_error("unknown precision form %d", prec);
        return XDG_EINVAL;
    }
    const int64_t D = b->dim;
    if (D < 1) {
        set_error("lanczos on an empty block");
        return XDG_EINVAL;
    }
    const bool single = prec == XDG_PREC_F32VEC || prec == XDG_PREC_F32VEC_REORTH;
    const bool reorth = prec == XDG_PREC_F32VEC_REORTH || prec == XDG_PREC_F64_REORTH;
    const int C = b->is_complex ? 2 : 1;
    const int dtype = C == 2 ? (single ? XDG_C64 : XDG_C128) : (single ? XDG_F32 : XDG_F64);
    const size_t esz = (single ? 4 : 8) * C;
    const uint64_t nsc = (uint64_t)D * C;
    const size_t vbytes = (size_t)D * esz;
    // slots 256-byte aligned (the vector kernels load four scalars at a time)
    const size_t vstride = (vbytes + 255) & ~(size_t)255;
    const uint64_t ld = vstride / (single ? 4 : 8);   // slot stride in scalars

    DevBuf bufs, wbuf, scal, parts, rparts;
    // vectors: reorth keeps every v_j (column j of V); otherwise three rotate
    const int nstore = reorth ? max_iter + 1 : 3;
    XDG_RETURN_IF(bufs.alloc(vstride * nstore));
    XDG_RETURN_IF(wbuf.alloc(vbytes));
    // scalars: cur_alpha, cur_beta, prev_beta, |w|^2 before and after a first
    // reorthogonalisation pass, hist_alpha[max_iter], hist_beta[max_iter],
    // coef[2 (max_iter + 1)], then jdev and the skip flag of the second pass
    XDG_RETURN_IF(scal.alloc(sizeof(double) * (5 + 2 * (size_t)max_iter + 2 * (size_t)(max_iter + 1)) + 16));
    double *cur_alpha = scal.as<double>(), *cur_beta = cur_alpha + 1, *prev_beta = cur_alpha + 2;
    double *nrm0 = cur_alpha + 3, *nrm1 = cur_alpha + 4;
    double *hist_a = cur_alpha + 5, *hist_b = hist_a + max_iter;
    double *coef = hist_b + max_iter;
    int *jdev = reinterpret_cast<int *>(coef + 2 * (size_t)(max_iter + 1));
    int *skip2 = jdev + 1;
    VecOps ops{single, C, C, nsc, vec_grid(nsc), nullptr, st};
    XDG_RETURN_IF(parts.alloc(sizeof(double) * (size_t)ops.grid * MAXC));
    ops.partials = parts.as<double>();
    // reorthogonalisation: one block per row tile; partial sums per (column, block)
    const int rtile = single ? tile_scalars<float>() : tile_scalars<double>();
    const int rgrid = (int)((nsc + rtile - 1) / rtile);
    if (reorth)
        XDG_RETURN_IF(rparts.alloc(sizeof(double) * (size_t)C * rgrid * (max_iter + 1)));

    auto vec = [&](int i) -> char * { return bufs.as<char>() + vstride * i; };
    char *w = wbuf.as<char>();
    if (v0)
        XDG_TRY_HIP(hipMemcpyAsync(vec(0), v0, vbytes, hipMemcpyDeviceToDevice, st));
    else
        XDG_RETURN_IF(random_fill((int64_t)nsc, seed, 1, single, vec(0), st));
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, st, jdev, prev_beta, 1);
    XDG_RETURN_IF(ops.dot(vec(0), vec(0)));
    XDG_RETURN_IF(ops.finalize(1, cur_beta, nullptr, jdev));
    XDG_RETURN_IF(ops.scale(vec(0), vec(0), cur_beta));

    // one event pair per iteration around the apply; summed at the end
    std::vector<hipEvent_t> evs(2 * (size_t)max_iter, nullptr);
    struct EvGuard {
        std::vector<hipEvent_t> &e;
        ~EvGuard() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } ev_guard{evs};
    for (auto &e : evs) XDG_TRY_HIP(hipEventCreate(&e));
    std::vector<double> ha(max_iter), hb(max_iter), ritz;
    double prev_k = NAN;
    int m = 0, status = XDG_ENOCONV;
    bool stop = false;
    double apply_s = 0.0;
    XDG_TRY_HIP(hipStreamSynchronize(st));
    const auto t0 = std::chrono::steady_clock::now();
    int iv = 0, ip = -1, in = 1;   // rotating indices (v, vprev, next) when not reorth
    for (int j = 0; j < max_iter && !stop; ++j) {
        char *v = reorth ? vec(j) : vec(iv);
        char *vp = reorth ? (j ? vec(j - 1) : nullptr) : (ip >= 0 ? vec(ip) : nullptr);
        XDG_TRY_HIP(hipEventRecord(evs[2 * j], st));
        XDG_RETURN_IF(apply_tuned(h, v, w, 1, dtype, st));
        XDG_TRY_HIP(hipEventRecord(evs[2 * j + 1], st));
        XDG_RETURN_IF(ops.dot(v, w));
        XDG_RETURN_IF(ops.finalize(0, cur_alpha, hist_a, jdev));
        XDG_RETURN_IF(ops.update(w, v, vp, cur_alpha, prev_beta));
        if (reorth) {
            // classical Gram-Schmidt against v_0 .. v_j, FP64 coefficients; the
            // second pass runs only where the first removed more than half of |w|^2
            const int kk = j + 1;
            double *rp = rparts.as<double>();
            auto pass = [&](const int *skip) -> int {
                if (single) {
                    const float *Vf = (const float *)vec(0);
                    float *wf = (float *)w;
                    if (C == 1) {
                        hipLaunchKernelGGL((k_reorth_dots<float, 1>), dim3(rgrid), dim3(RB), 0, st,
                                           Vf, ld, kk, wf, nsc, rp, skip);
                        hipLaunchKernelGGL(k_reorth_finalize<1>, dim3(kk), dim3(RB), 0, st, rp,
                                           rgrid, coef, skip);
                        hipLaunchKernelGGL((k_reorth_sub<float, 1>), dim3(rgrid), dim3(RB), 0, st,
                                           Vf, ld, kk, coef, wf, nsc, skip);
                    } else {
                        hipLaunchKernelGGL((k_reorth_dots<float, 2>), dim3(rgrid), dim3(RB), 0, st,
                                           Vf, ld, kk, wf, nsc, rp, skip);
                        hipLaunchKernelGGL(k_reorth_finalize<2>, dim3(2 * kk), dim3(RB), 0, st,
                                           rp, rgrid, coef, skip);
                        hipLaunchKernelGGL((k_reorth_sub<float, 2>), dim3(rgrid), dim3(RB), 0, st,
                                           Vf, ld, kk, coef, wf, nsc, skip);
                    }
                } else {
                    const double *Vd = (const double *)vec(0);
                    double *wd = (double *)w;
                    if (C == 1) {
                        hipLaunchKernelGGL((k_reorth_dots<double, 1>), dim3(rgrid), dim3(RB), 0,
                                           st, Vd, ld, kk, wd, nsc, rp, skip);
                        hipLaunchKernelGGL(k_reorth_finalize<1>, dim3(kk), dim3(RB), 0, st, rp,
                                           rgrid, coef, skip);
                        hipLaunchKernelGGL((k_reorth_sub<double, 1>), dim3(rgrid), dim3(RB), 0,
                                           st, Vd, ld, kk, coef, wd, nsc, skip);
                    } else {
                        hipLaunchKernelGGL((k_reorth_dots<double, 2>), dim3(rgrid), dim3(RB), 0,
                                           st, Vd, ld, kk, wd, nsc, rp, skip);
                        hipLaunchKernelGGL(k_reorth_finalize<2>, dim3(2 * kk), dim3(RB), 0, st,
                                           rp, rgrid, coef, skip);
                        hipLaunchKernelGGL((k_reorth_sub<double, 2>), dim3(rgrid), dim3(RB), 0,
                                           st, Vd, ld, kk, coef, wd, nsc, skip);
                    }
                }
                XDG_TRY_HIP(hipGetLastError());
                return XDG_OK;
            };
            XDG_RETURN_IF(ops.finalize(0, nrm0, nullptr, jdev));   // |w|^2 from the update
            XDG_RETURN_IF(pass(nullptr));
            XDG_RETURN_IF(ops.dot(w, w));
            XDG_RETURN_IF(ops.finalize(0, nrm1, nullptr, jdev));
            hipLaunchKernelGGL(k_dgks, dim3(1), dim3(64), 0, st, nrm0, nrm1, skip2);
            XDG_TRY_HIP(hipGetLastError());
            XDG_RETURN_IF(pass(skip2));
            XDG_RETURN_IF(ops.dot(w, w));
        }
        XDG_RETURN_IF(ops.finalize(1, cur_beta, hist_b, jdev));
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, jdev, prev_beta, cur_beta, 1);
        XDG_TRY_HIP(hipGetLastError());
        m = j + 1;
        if (progress_every() && m % progress_every() == 0) {
            XDG_TRY_HIP(hipStreamSynchronize(st));
            fprintf(stderr, "[xdg] lanczos iteration %d / %d\n", m, max_iter);
        }
        const bool check = tol > 0.0 || m == max_iter || (m % 16) == 0;
        if (check) {
            XDG_RETURN_IF(copy_d2h(ha.data(), hist_a, sizeof(double) * m, st));
            XDG_RETURN_IF(copy_d2h(hb.data(), hist_b, sizeof(double) * m, st));
            float ms = 0;
            // breakdown anywhere since the last check truncates the run there
            for (int t = std::max(0, m - 16); t < m; ++t)
                if (hb[t] <= 1e-13 * std::max(1.0, std::fabs(ha[t])) || !std::isfinite(hb[t])) {
                    m = t + 1;
                    stop = true;
                    status = XDG_OK;
                    break;
                }
            if (!stop && tol > 0.0 && m >= k) {
                tridiag_eigenvalues(m, ha.data(), hb.data(), ritz);
                const double th = ritz[k - 1];
                if (std::isfinite(prev_k) && std::fabs(th - prev_k) <= tol * std::fabs(th)) {
                    stop = true;
                    status = XDG_OK;
                }
                prev_k = th;
            }
            (void)ms;
        }
        if (stop) break;
        if (reorth) {
            XDG_RETURN_IF(ops.scale(w, vec(j + 1), cur_beta));
        } else {
            XDG_RETURN_IF(ops.scale(w, vec(in), cur_beta));
            ip = iv;
            iv = in;
            in = (in + 1) % 3;
            if (in == ip) in = (in + 1) % 3;
        }
    }
    XDG_TRY_HIP(hipStreamSynchronize(st));
    const double total =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int j = 0; j < m; ++j) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, evs[2 * j], evs[2 * j + 1]) == hipSuccess) apply_s += 1e-3 * ms;
    }
    XDG_RETURN_IF(copy_d2h(ha.data(), hist_a, sizeof(double) * m, st));
    XDG_RETURN_IF(copy_d2h(hb.data(), hist_b, sizeof(double) * m, st));
    if (tol == 0.0 && !stop) status = XDG_OK;
    tridiag_eigenvalues(m, ha.data(), hb.data(), ritz);
    for (int e = 0; e < k; ++e) evals[e] = e < m ? ritz[e] : NAN;
    *n_iter = m;
    if (alpha) std::copy(ha.begin(), ha.begin() + m, alpha);
    if (beta) std::copy(hb.begin(), hb.begin() + m, beta);
    g_t_total = total;
    g_t_apply = apply_s;
    if (t_total) *t_total = total;
    if (t_apply) *t_apply = apply_s;
    return status;
}

// n blocks x nvec recurrences in lockstep; each step (batched apply, then
// per-block dot / update / norm / scale) is captured once per buffer
// rotation phase into a HIP graph and replayed.
// Eigenvector of the symmetric tridiagonal matrix for its eigenvalue number
// `which` (ascending), by inverse iteration: (T - theta) x = x_prev solved by
// Gaussian elimination with partial pivoting on the tridiagonal band, three
// sweeps.  Normalised, first nonzero component made positive.
void tridiag_eigvec(int m, const double *alpha, const double *beta, int which,
                    std::vector<double> &x, double &theta) {
    std::vector<double> ev;
    tridiag_eigenvalues(m, alpha, beta, ev);
    theta = ev[which];
    double tnorm = 0.0;
    for (int i = 0; i < m; ++i)
        tnorm = std::max(tnorm, std::fabs(alpha[i]) + (i ? std::fabs(beta[i - 1]) : 0.0) +
                                    (i + 1 < m ? std::fabs(beta[i]) : 0.0));
    const double tiny = std::max(tnorm, 1e-300) * 1e-15;
    // factor P (T - theta) = L U; U has diagonals d, u1, u2; L multipliers f
    std::vector<double> d(m), u1(m, 0.0), u2(m, 0.0), f(m, 0.0);
    std::vector<char> swp(m, 0);
    for (int i = 0; i < m; ++i) {
        d[i] = alpha[i] - theta;
        if (i + 1 < m) u1[i] = beta[i];
    }
    for (int i = 0; i + 1 < m; ++i) {
        const double sub = beta[i];   // row i+1, column i
        if (std::fabs(d[i]) >= std::fabs(sub)) {
            if (d[i] == 0.0) d[i] = tiny;
            f[i] = sub / d[i];
            d[i + 1] -= f[i] * u1[i];
        } else {
            // rows i and i+1 exchanged
            swp[i] = 1;
            f[i] = d[i] / sub;
            d[i] = sub;
            const double r1 = u1[i];       // old row i, column i+1
            u1[i] = d[i + 1];              // old row i+1, column i+1
            d[i + 1] = r1 - f[i] * u1[i];
            if (i + 2 < m) {
                u2[i] = u1[i + 1];         // old row i+1, column i+2
                u1[i + 1] = -f[i] * u2[i];
            }
        }
    }
    if (d[m - 1] == 0.0) d[m - 1] = tiny;
    x.assign(m, 1.0);
    for (int sweep = 0; sweep < 3; ++sweep) {
        // forward: apply P and L^-1
        for (int i = 0; i + 1 < m; ++i) {
            if (swp[i]) std::swap(x[i], x[i + 1]);
            x[i + 1] -= f[i] * x[i];
        }
        // back substitution with U
        for (int i = m - 1; i >= 0; --i) {
            double r = x[i];
            if (i + 1 < m) r -= u1[i] * x[i + 1];
            if (i + 2 < m) r -= u2[i] * x[i + 2];
            x[i] = r / (d[i] != 0.0 ? d[i] : tiny);
        }
        double nrm = 0.0;
        for (double v : x) nrm += v * v;
        nrm = std::sqrt(nrm);
        for (double &v : x) v /= nrm;
    }
    for (int i = 0; i < m; ++i)
        if (x[i] != 0.0) {
            if (x[i] < 0.0)
                for (double &v : x) v = -v;
            break;
        }
}

int lanczos_eigvec(xdg_ham_s *h, const void *v0, uint64_t seed, int prec, int m,
                   const double *alpha, const double *beta, int which, void *psi, double *ritz,
                   hipStream_t st) {
    const xdg_basis_s *b = h->basis;
    if (prec != XDG_PREC_F64 && prec != XDG_PREC_F32VEC) {
        set_error("second Lanczos pass: precision form %d not supported (no reorthogonalisation)",
                  prec);
        return XDG_EINVAL;
    }
    if (m < 1 || which < 0 || which >= m || !alpha || !beta || !psi || psi == v0) {
        set_error("second Lanczos pass: need n_iter >= 1, 0 <= which < n_iter, alpha, beta and a "
                  "psi distinct from v0");
        return XDG_EINVAL;
    }
    const int64_t D = b->dim;
    if (D < 1) {
        set_error("lanczos on an empty block");
        return XDG_EINVAL;
    }
    for (int j = 0; j + 1 < m; ++j)
        if (!(beta[j] > 0.0)) {
            set_error("second Lanczos pass: beta[%d] = %g ends the recurrence before n_iter", j,
                      beta[j]);
            return XDG_EINVAL;
        }
    std::vector<double> c;
    double theta = 0.0;
    tridiag_eigvec(m, alpha, beta, which, c, theta);
    if (ritz) *ritz = theta;

    const bool single = prec == XDG_PREC_F32VEC;
    const int C = b->is_complex ? 2 : 1;
    const int dtype = C == 2 ? (single ? XDG_C64 : XDG_C128) : (single ? XDG_F32 : XDG_F64);
    const size_t esz = (single ? 4 : 8) * C;
    const uint64_t nsc = (uint64_t)D * C;
    const size_t vbytes = (size_t)D * esz;
    const size_t vstride = (vbytes + 255) & ~(size_t)255;   // 256-byte aligned slots
    DevBuf bufs, wbuf, acc, scal, parts;
    XDG_RETURN_IF(bufs.alloc(vstride * 3));
    XDG_RETURN_IF(wbuf.alloc(vbytes));
    XDG_RETURN_IF(acc.alloc(sizeof(double) * nsc));
    // scalars: nrm, alpha[m], beta[m], zero
    XDG_RETURN_IF(scal.alloc(sizeof(double) * (2 + 2 * (size_t)m) + 16));
    double *nrm = scal.as<double>(), *zero = nrm + 1, *al_d = nrm + 2, *be_d = al_d + m;
    int *jdev = reinterpret_cast<int *>(be_d + m);
    XDG_TRY_HIP(hipMemsetAsync(scal.p, 0, scal.bytes, st));
    XDG_RETURN_IF(copy_h2d(al_d, alpha, sizeof(double) * m, st));
    XDG_RETURN_IF(copy_h2d(be_d, beta, sizeof(double) * m, st));
    XDG_TRY_HIP(hipMemsetAsync(acc.p, 0, acc.bytes, st));
    VecOps ops{single, C, C, nsc, vec_grid(nsc), nullptr, st};
    XDG_RETURN_IF(parts.alloc(sizeof(double) * (size_t)ops.grid * MAXC));
    ops.partials = parts.as<double>();
    auto vec = [&](int i) -> char * { return bufs.as<char>() + vstride * i; };
    char *w = wbuf.as<char>();
    // start vector exactly as in the first pass
    if (v0)
        XDG_TRY_HIP(hipMemcpyAsync(vec(0), v0, vbytes, hipMemcpyDeviceToDevice, st));
    else
        XDG_RETURN_IF(random_fill((int64_t)nsc, seed, 1, single, vec(0), st));
    XDG_RETURN_IF(ops.dot(vec(0), vec(0)));
    XDG_RETURN_IF(ops.finalize(1, nrm, nullptr, jdev));
    XDG_RETURN_IF(ops.scale(vec(0), vec(0), nrm));
    const int g = vec_grid(nsc);
    int iv = 0, ip = -1, in = 1;
    for (int j = 0; j < m; ++j) {
        char *v = vec(iv);
        if (single)
            hipLaunchKernelGGL(k_acc_axpy<float>, dim3(g), dim3(RB), 0, st, acc.as<double>(),
                               (const float *)v, nsc, c[j]);
        else
            hipLaunchKernelGGL(k_acc_axpy<double>, dim3(g), dim3(RB), 0, st, acc.as<double>(),
                               (const double *)v, nsc, c[j]);
        XDG_TRY_HIP(hipGetLastError());
        if (j + 1 == m) break;
        XDG_RETURN_IF(apply_tuned(h, v, w, 1, dtype, st));
        XDG_RETURN_IF(ops.update(w, v, ip >= 0 ? vec(ip) : nullptr, al_d + j, j ? be_d + j - 1 : zero));
        XDG_RETURN_IF(ops.scale(w, vec(in), be_d + j));
        ip = iv;
        iv = in;
        in = (in + 1) % 3;
        if (in == ip) in = (in + 1) % 3;
        if (progress_every() && (j + 1) % progress_every() == 0) {
            XDG_TRY_HIP(hipStreamSynchronize(st));
            fprintf(stderr, "[xdg] second lanczos pass %d / %d\n", j + 1, m);
        }
    }
    // psi = acc / |acc|
    VecOps dops{false, 1, 1, nsc, vec_grid(nsc), parts.as<double>(), st};
    XDG_RETURN_IF(dops.dot(acc.p, acc.p));
    XDG_RETURN_IF(dops.finalize(1, nrm, nullptr, jdev));
    if (single)
        hipLaunchKernelGGL(k_acc_out<float>, dim3(g), dim3(RB), 0, st, acc.as<double>(),
                           (float *)psi, nsc, nrm);
    else
        hipLaunchKernelGGL(k_acc_out<double>, dim3(g), dim3(RB), 0, st, acc.as<double>(),
                           (double *)psi, nsc, nrm);
    XDG_TRY_HIP(hipGetLastError());
    XDG_TRY_HIP(hipStreamSynchronize(st));
    return XDG_OK;
}

int lanczos_batched(int n, xdg_ham_s *const *hams, const void *const *v0s, int64_t nvec,
                    int n_iter, uint64_t seed, int prec, double *evals, double *alpha,
                    double *beta, hipStream_t user_st, double *t_total, double *t_apply) {
    if (n < 1 || n_iter < 1 || !evals) {
        set_error("batched lanczos: need n >= 1, n_iter >= 1 and evals");
        return XDG_EINVAL;
    }
    if (nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8) {
        set_error("batched lanczos: nvec must be 1, 2, 4 or 8");
        return XDG_EINVAL;
    }
    if (prec != XDG_PREC_F64 && prec != XDG_PREC_F32VEC) {
        set_error("batched lanczos supports XDG_PREC_F64 and XDG_PREC_F32VEC");
        return XDG_EINVAL;
    }
    bool any_c = false;
    for (int i = 0; i < n; ++i) {
        if (!hams[i] || hams[i]->basis->dim < 1) {
            set_error("batched lanczos: block %d is null or empty", i);
            return XDG_EINVAL;
        }
        any_c |= hams[i]->basis->is_complex;
    }
    const bool single = prec == XDG_PREC_F32VEC;
    const int C = any_c ? 2 : 1;
    const int dtype = any_c ? (single ? XDG_C64 : XDG_C128) : (single ? XDG_F32 : XDG_F64);
    const size_t ssz = single ? 4 : 8;
    const int cols = (int)nvec * C;

    hipStream_t st = user_st;
    hipStream_t own = nullptr;
    if (!st) {
        XDG_TRY_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        st = own;
    }
    struct Sec {
        DevBuf buf, parts, scal;
        uint64_t nsc;
        size_t slot;   // bytes between the vector slots of buf
        VecOps ops;
        double *cur_a, *cur_b, *prev_b, *hist_a, *hist_b;
    };
    std::vector<Sec> S(n);
    DevBuf jbuf;
    XDG_RETURN_IF(jbuf.alloc(16));
    int *jdev = jbuf.as<int>();
    for (int i = 0; i < n; ++i) {
        Sec &s = S[i];
        const int64_t D = hams[i]->basis->dim;
        s.nsc = (uint64_t)D * cols;
        s.slot = (ssz * s.nsc + 255) & ~(size_t)255;   // 256-byte aligned slots
        XDG_RETURN_IF(s.buf.alloc(s.slot * 4));   // v0, v1, v2 (rotating) + w
        s.ops = VecOps{single, cols, C, s.nsc, vec_grid(s.nsc), nullptr, st};
        XDG_RETURN_IF(s.parts.alloc(sizeof(double) * (size_t)s.ops.grid * MAXC));
        s.ops.partials = s.parts.as<double>();
        XDG_RETURN_IF(s.scal.alloc(sizeof(double) * (3 * nvec + 2 * (size_t)n_iter * nvec)));
        s.cur_a = s.scal.as<double>();
        s.cur_b = s.cur_a + nvec;
        s.prev_b = s.cur_b + nvec;
        s.hist_a = s.prev_b + nvec;
        s.hist_b = s.hist_a + (size_t)n_iter * nvec;
        char *v = s.buf.as<char>();
        if (v0s && v0s[i])
            XDG_TRY_HIP(hipMemcpyAsync(v, v0s[i], ssz * s.nsc, hipMemcpyDeviceToDevice, st));
        else
            XDG_RETURN_IF(random_fill((int64_t)s.nsc, seed + (uint64_t)i, 1, single, v, st));
        hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, st, jdev, s.prev_b, (int)nvec);
        XDG_RETURN_IF(s.ops.dot(v, v));
        XDG_RETURN_IF(s.ops.finalize(1, s.cur_b, nullptr, jdev));
        XDG_RETURN_IF(s.ops.scale(v, v, s.cur_b));
    }
    auto vecp = [&](int i, int slot) -> char * { return S[i].buf.as<char>() + S[i].slot * slot; };
    // phase p: v = slot p, vprev = slot (p+2)%3 (none at j = 0), next = slot (p+1)%3, w = slot 3
    std::vector<xdg_ham_s *> hv(hams, hams + n);
    auto prepare = [&](int p, BatchPlan *P, uint32_t tile) -> int {
        std::vector<const void *> xs(n);
        std::vector<void *> ys(n);
        for (int i = 0; i < n; ++i) {
            xs[i] = vecp(i, p);
            ys[i] = vecp(i, 3);
        }
        return batch_prepare(n, hv.data(), xs.data(), ys.data(), nvec, dtype, P, tile);
    };
    // launch shape of the batched apply (tuned once per set of blocks)
    BatchShape best_shape;
    {
        std::vector<const void *> xs(n);
        std::vector<void *> ys(n);
        for (int i = 0; i < n; ++i) {
            xs[i] = vecp(i, 0);
            ys[i] = vecp(i, 3);
        }
        XDG_RETURN_IF(batch_shape_tuned(n, hv.data(), xs.data(), ys.data(), nvec, dtype, st,
                                        &best_shape));
    }
    BatchPlan plans[3];
    for (int p = 0; p < 3; ++p) XDG_RETURN_IF(prepare(p, &plans[p], best_shape.tile));
    const int best_grid = best_shape.grid;
    auto enqueue_step = [&](int p, bool first) -> int {
        XDG_RETURN_IF(batch_launch(plans[p], best_grid, best_shape.nv, st));
        for (int i = 0; i < n; ++i) {
            Sec &s = S[i];
            char *v = vecp(i, p), *w = vecp(i, 3);
            char *vp = first ? nullptr : vecp(i, (p + 2) % 3);
            XDG_RETURN_IF(s.ops.dot(v, w));
            XDG_RETURN_IF(s.ops.finalize(0, s.cur_a, s.hist_a, jdev));
            XDG_RETURN_IF(s.ops.update(w, v, vp, s.cur_a, s.prev_b));
            XDG_RETURN_IF(s.ops.finalize(1, s.cur_b, s.hist_b, jdev));
            XDG_RETURN_IF(s.ops.scale(w, vecp(i, (p + 1) % 3), s.cur_b));
            hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, (int *)nullptr, s.prev_b,
                               s.cur_b, (int)nvec);
        }
        // one counter for all blocks; k_step_end with a null counter only copies beta
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, jdev, S[0].prev_b, S[0].cur_b,
                           (int)nvec);
        XDG_TRY_HIP(hipGetLastError());
        return XDG_OK;
    };
    XDG_TRY_HIP(hipStreamSynchronize(st));
    const auto t0 = std::chrono::steady_clock::now();
    // step 0 runs eagerly (it has no v_{j-1}); later steps replay graphs
    XDG_RETURN_IF(enqueue_step(0, true));
    hipGraphExec_t exec[3] = {nullptr, nullptr, nullptr};
    hipGraph_t graphs[3] = {nullptr, nullptr, nullptr};
    int rc = XDG_OK;
    for (int p = 0; p < 3 && rc == XDG_OK && n_iter > 1; ++p) {
        XDG_TRY_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        rc = enqueue_step(p, false);
        hipError_t e = hipStreamEndCapture(st, &graphs[p]);
        if (rc == XDG_OK && e != hipSuccess) {
            set_error("graph capture failed: %s", hipGetErrorString(e));
            rc = XDG_EHIP;
        }
        if (rc == XDG_OK) {
            e = hipGraphInstantiate(&exec[p], graphs[p], nullptr, nullptr, 0);
            if (e != hipSuccess) {
                set_error("graph instantiation failed: %s", hipGetErrorString(e));
                rc = XDG_EHIP;
            }
        }
    }
    for (int j = 1; j < n_iter && rc == XDG_OK; ++j) {
        hipError_t e = hipGraphLaunch(exec[j % 3], st);
        if (e != hipSuccess) {
            set_error("graph launch failed: %s", hipGetErrorString(e));
            rc = XDG_EHIP;
        }
        if (rc == XDG_OK && progress_every() && (j + 1) % progress_every() == 0) {
            (void)hipStreamSynchronize(st);
            fprintf(stderr, "[xdg] batched lanczos iteration %d / %d\n", j + 1, n_iter);
        }
    }
    if (rc == XDG_OK) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            set_error("batched lanczos: %s", hipGetErrorString(e));
            rc = XDG_EHIP;
        }
    }
    const double total =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int p = 0; p < 3; ++p) {
        if (exec[p]) (void)hipGraphExecDestroy(exec[p]);
        if (graphs[p]) (void)hipGraphDestroy(graphs[p]);
    }
    if (rc == XDG_OK) {
        std::vector<double> ha((size_t)n_iter * nvec), hb((size_t)n_iter * nvec), a1(n_iter),
            b1(n_iter), ritz;
        for (int i = 0; i < n && rc == XDG_OK; ++i) {
            if (copy_d2h(ha.data(), S[i].hist_a, sizeof(double) * ha.size(), st) != XDG_OK ||
                copy_d2h(hb.data(), S[i].hist_b, sizeof(double) * hb.size(), st) != XDG_OK) {
                set_error("batched lanczos: copy of the tridiagonal matrices failed");
                rc = XDG_EHIP;
                break;
            }
            for (int v = 0; v < nvec; ++v) {
                int m = n_iter;
                for (int j = 0; j < n_iter; ++j) {
                    a1[j] = ha[(size_t)j * nvec + v];
                    b1[j] = hb[(size_t)j * nvec + v];
                    if (alpha) alpha[((size_t)i * nvec + v) * n_iter + j] = a1[j];
                    if (beta) beta[((size_t)i * nvec + v) * n_iter + j] = b1[j];
                }
                for (int j = 0; j < n_iter; ++j)
                    if (b1[j] <= 1e-13 * std::max(1.0, std::fabs(a1[j])) || !std::isfinite(b1[j])) {
                        m = j + 1;
                        break;
                    }
                tridiag_eigenvalues(m, a1.data(), b1.data(), ritz);
                evals[(size_t)i * nvec + v] = ritz[0];
            }
        }
    }
    if (own) (void)hipStreamDestroy(own);
    g_t_total = total;
    g_t_apply = 0.0;
    if (t_total) *t_total = total;
    if (t_apply) *t_apply = 0.0;
    return rc;
}

// Microcanonical TPQ sequence (Sec. 4.6, after Sugiura and Shimizu 2012):
// |k+1> = (l - H/N)|k> / norm from a unit start vector; per step one H x,
// the FP64 products <k|H|k> and <H k|H k> into device histories, then the
// next vector H|k> - l N |k> (the sign drops out of every expectation value)
// normalised in place.  The histories reach the host once, at the end.
int tpq_micro(xdg_ham_s *h, const void *v0, uint64_t seed, int prec, double l, int n_steps,
              double *u, double *u2, hipStream_t st) {
    const xdg_basis_s *b = h->basis;
    if (n_steps < 1 || !u || !u2 || !std::isfinite(l)) {
        set_error("tpq: need n_steps >= 1, output arrays and a finite l");
        return XDG_EINVAL;
    }
    if (prec != XDG_PREC_F64 && prec != XDG_PREC_F32VEC) {
        set_error("tpq: precision form %d (XDG_PREC_F64 or XDG_PREC_F32VEC)", prec);
        return XDG_EINVAL;
    }
    const int64_t D = b->dim;
    if (D < 1) {
        set_error("tpq on an empty block");
        return XDG_EINVAL;
    }
    const bool single = prec == XDG_PREC_F32VEC;
    const int C = b->is_complex ? 2 : 1;
    const int dtype = C == 2 ? (single ? XDG_C64 : XDG_C128) : (single ? XDG_F32 : XDG_F64);
    const size_t esz = (single ? 4 : 8) * C;
    const uint64_t nsc = (uint64_t)D * C;
    const size_t vbytes = (size_t)D * esz;
    const size_t vstride = (vbytes + 255) & ~(size_t)255;
    const double N = (double)b->n_sites;

    DevBuf vbuf, scal, parts;
    XDG_RETURN_IF(vbuf.alloc(2 * vstride));
    // scalars: <v,Hv>, <Hv,Hv>, norm, l N, unused, histories [2][n_steps], jdev
    XDG_RETURN_IF(scal.alloc(sizeof(double) * (5 + 2 * (size_t)n_steps) + 16));
    double *s_vw = scal.as<double>(), *s_ww = s_vw + 1, *s_nrm = s_vw + 2, *s_ln = s_vw + 3;
    double *s_dummy = s_vw + 4, *h_vw = s_vw + 5, *h_ww = h_vw + n_steps;
    int *jdev = reinterpret_cast<int *>(h_ww + n_steps);
    VecOps ops{single, C, C, nsc, vec_grid(nsc), nullptr, st};
    XDG_RETURN_IF(parts.alloc(sizeof(double) * (size_t)ops.grid * MAXC));
    ops.partials = parts.as<double>();
    char *v = vbuf.as<char>(), *w = v + vstride;
    if (v0)
        XDG_TRY_HIP(hipMemcpyAsync(v, v0, vbytes, hipMemcpyDeviceToDevice, st));
    else
        XDG_RETURN_IF(random_fill((int64_t)nsc, seed, 1, single, v, st));
    const double ln = l * N;
    XDG_TRY_HIP(hipMemcpyAsync(s_ln, &ln, sizeof(double), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, st, jdev, s_dummy, 1);
    XDG_TRY_HIP(hipGetLastError());
    XDG_RETURN_IF(ops.dot(v, v));
    XDG_RETURN_IF(ops.finalize(1, s_nrm, nullptr, jdev));
    XDG_RETURN_IF(ops.scale(v, v, s_nrm));
    for (int k = 0; k < n_steps; ++k) {
        XDG_RETURN_IF(apply_tuned(h, v, w, 1, dtype, st));
        XDG_RETURN_IF(ops.dot(v, w));
        XDG_RETURN_IF(ops.finalize(0, s_vw, h_vw, jdev));
        XDG_RETURN_IF(ops.dot(w, w));
        XDG_RETURN_IF(ops.finalize(0, s_ww, h_ww, jdev));
        if (k + 1 < n_steps) {
            XDG_RETURN_IF(ops.update(w, v, nullptr, s_ln, nullptr));   // w = H v - l N v
            XDG_RETURN_IF(ops.finalize(1, s_nrm, nullptr, jdev));
            XDG_RETURN_IF(ops.scale(w, v, s_nrm));
        }
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, jdev, s_dummy, s_dummy, 1);
        XDG_TRY_HIP(hipGetLastError());
    }
    std::vector<double> hv(n_steps), hw(n_steps);
    XDG_RETURN_IF(copy_d2h(hv.data(), h_vw, sizeof(double) * n_steps, st));
    XDG_RETURN_IF(copy_d2h(hw.data(), h_ww, sizeof(double) * n_steps, st));
    for (int k = 0; k < n_steps; ++k) {
        u[k] = hv[k] / N;
        u2[k] = hw[k] / (N * N);
    }
    return XDG_OK;
}

// The same sequence for n blocks x nvec start vectors in lockstep: one
// batched H x per step over every block (the persistent launch), per-column
// FP64 products and updates; one captured step replayed n_steps times.
int tpq_micro_batched(int n, xdg_ham_s *const *hams, const void *const *v0s, int64_t nvec,
                      uint64_t seed, int prec, double l, int n_steps, double *u, double *u2,
                      hipStream_t user_st) {
    if (n < 1 || n_steps < 1 || !u || !u2 || !std::isfinite(l)) {
        set_error("batched tpq: need n >= 1, n_steps >= 1, output arrays and a finite l");
        return XDG_EINVAL;
    }
    if (nvec != 1 && nvec != 2 && nvec != 4 && nvec != 8) {
        set_error("batched tpq: nvec must be 1, 2, 4 or 8");
        return XDG_EINVAL;
    }
    if (prec != XDG_PREC_F64 && prec != XDG_PREC_F32VEC) {
        set_error("batched tpq: precision form %d (XDG_PREC_F64 or XDG_PREC_F32VEC)", prec);
        return XDG_EINVAL;
    }
    bool any_c = false;
    for (int i = 0; i < n; ++i) {
        if (!hams[i] || hams[i]->basis->dim < 1) {
            set_error("batched tpq: block %d is null or empty", i);
            return XDG_EINVAL;
        }
        any_c |= hams[i]->basis->is_complex;
    }
    const bool single = prec == XDG_PREC_F32VEC;
    const int C = any_c ? 2 : 1;
    const int dtype = any_c ? (single ? XDG_C64 : XDG_C128) : (single ? XDG_F32 : XDG_F64);
    const size_t ssz = single ? 4 : 8;
    const int cols = (int)nvec * C;

    hipStream_t st = user_st;
    hipStream_t own = nullptr;
    if (!st) {
        XDG_TRY_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        st = own;
    }
    struct OwnStream {
        hipStream_t s;
        ~OwnStream() {
            if (s) (void)hipStreamDestroy(s);
        }
    } own_guard{own};
    struct Sec {
        DevBuf buf, parts, scal;
        uint64_t nsc;
        size_t slot;
        VecOps ops;
        double *ln, *nrm, *vw, *ww, *h_vw, *h_ww;
    };
    std::vector<Sec> S(n);
    DevBuf jbuf;
    XDG_RETURN_IF(jbuf.alloc(16));
    int *jdev = jbuf.as<int>();
    for (int i = 0; i < n; ++i) {
        Sec &s = S[i];
        const int64_t D = hams[i]->basis->dim;
        s.nsc = (uint64_t)D * cols;
        s.slot = (ssz * s.nsc + 255) & ~(size_t)255;
        XDG_RETURN_IF(s.buf.alloc(s.slot * 2));   // v, w
        s.ops = VecOps{single, cols, C, s.nsc, vec_grid(s.nsc), nullptr, st};
        XDG_RETURN_IF(s.parts.alloc(sizeof(double) * (size_t)s.ops.grid * MAXC));
        s.ops.partials = s.parts.as<double>();
        // per vector: l N, norm, <v, Hv>, <Hv, Hv>; then the two histories
        XDG_RETURN_IF(s.scal.alloc(sizeof(double) * (4 * (size_t)nvec + 2 * (size_t)n_steps * nvec)));
        s.ln = s.scal.as<double>();
        s.nrm = s.ln + nvec;
        s.vw = s.nrm + nvec;
        s.ww = s.vw + nvec;
        s.h_vw = s.ww + nvec;
        s.h_ww = s.h_vw + (size_t)n_steps * nvec;
        const std::vector<double> lnv(nvec, l * (double)hams[i]->basis->n_sites);
        XDG_TRY_HIP(hipMemcpyAsync(s.ln, lnv.data(), sizeof(double) * nvec, hipMemcpyHostToDevice,
                                   st));
        char *v = s.buf.as<char>();
        if (v0s && v0s[i])
            XDG_TRY_HIP(hipMemcpyAsync(v, v0s[i], ssz * s.nsc, hipMemcpyDeviceToDevice, st));
        else
            XDG_RETURN_IF(random_fill((int64_t)s.nsc, seed + (uint64_t)i, 1, single, v, st));
        XDG_RETURN_IF(s.ops.dot(v, v));
        XDG_RETURN_IF(s.ops.finalize(1, s.nrm, nullptr, jdev));
        XDG_RETURN_IF(s.ops.scale(v, v, s.nrm));
    }
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, st, jdev, S[0].nrm, 0);
    XDG_TRY_HIP(hipGetLastError());
    std::vector<xdg_ham_s *> hv(hams, hams + n);
    std::vector<const void *> xs(n);
    std::vector<void *> ys(n);
    for (int i = 0; i < n; ++i) {
        xs[i] = S[i].buf.as<char>();
        ys[i] = S[i].buf.as<char>() + S[i].slot;
    }
    BatchShape shape;
    XDG_RETURN_IF(batch_shape_tuned(n, hv.data(), xs.data(), ys.data(), nvec, dtype, st, &shape));
    BatchPlan plan;
    XDG_RETURN_IF(batch_prepare(n, hv.data(), xs.data(), ys.data(), nvec, dtype, &plan, shape.tile));
    auto step = [&]() -> int {
        XDG_RETURN_IF(batch_launch(plan, shape.grid, shape.nv, st));
        for (int i = 0; i < n; ++i) {
            Sec &s = S[i];
            char *v = s.buf.as<char>(), *w = v + s.slot;
            XDG_RETURN_IF(s.ops.dot(v, w));
            XDG_RETURN_IF(s.ops.finalize(0, s.vw, s.h_vw, jdev));
            XDG_RETURN_IF(s.ops.dot(w, w));
            XDG_RETURN_IF(s.ops.finalize(0, s.ww, s.h_ww, jdev));
            XDG_RETURN_IF(s.ops.update(w, v, nullptr, s.ln, nullptr));   // H v - l N v
            XDG_RETURN_IF(s.ops.finalize(1, s.nrm, nullptr, jdev));
            XDG_RETURN_IF(s.ops.scale(w, v, s.nrm));
        }
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, jdev, S[0].nrm, S[0].nrm, 0);
        XDG_TRY_HIP(hipGetLastError());
        return XDG_OK;
    };
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int rc = XDG_OK;
    XDG_TRY_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    rc = step();
    hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc == XDG_OK && e != hipSuccess) {
        set_error("graph capture failed: %s", hipGetErrorString(e));
        rc = XDG_EHIP;
    }
    if (rc == XDG_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error("graph instantiation failed");
        rc = XDG_EHIP;
    }
    for (int k = 0; k < n_steps && rc == XDG_OK; ++k) {
        if (hipGraphLaunch(exec, st) != hipSuccess) {
            set_error("graph launch failed");
            rc = XDG_EHIP;
        }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc == XDG_OK) {
        std::vector<double> hv_((size_t)n_steps * nvec), hw_((size_t)n_steps * nvec);
        for (int i = 0; i < n && rc == XDG_OK; ++i) {
            rc = copy_d2h(hv_.data(), S[i].h_vw, sizeof(double) * hv_.size(), st);
            if (rc == XDG_OK) rc = copy_d2h(hw_.data(), S[i].h_ww, sizeof(double) * hw_.size(), st);
            const double N = (double)hams[i]->basis->n_sites;
            for (int v = 0; v < nvec && rc == XDG_OK; ++v)
                for (int k = 0; k < n_steps; ++k) {
                    u[((size_t)i * nvec + v) * n_steps + k] = hv_[(size_t)k * nvec + v] / N;
                    u2[((size_t)i * nvec + v) * n_steps + k] = hw_[(size_t)k * nvec + v] / (N * N);
                }
        }
    }
    return rc;
}

int last_timing(double *total, double *apply) {
    if (total) *total = g_t_total;
    if (apply) *apply = g_t_apply;
    return XDG_OK;
}

}  // namespace xdg
