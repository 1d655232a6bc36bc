// Expectation values of symmetrised Ising correlations on a block
// (measurements, Sec. 3.8; symmetrisation of an operator over the group,
// Sec. 3.13).  O_ab = (1/|G|) sum_g S^z_{g(a)} S^z_{g(b)} is diagonal on the
// symmetric basis, with value o_ab(s) = (1/|G|) sum_g sz_s(g(a)) sz_s(g(b)) on
// representative s, so <psi|O_ab|psi> = sum_s |psi_s|^2 o_ab(s).  The orbit
// of each pair under the group is folded on the host into distinct site
// pairs with weights; a lane owns a state and up to PB pairs; block sums and
// their total are taken in a fixed order.
#include <algorithm>
#include <map>
#include <utility>
#include <vector>

#include "device_common.hpp"

namespace xdg {

namespace {

constexpr int MB = 256;   // threads per block
constexpr int PB = 8;     // pairs per pass

struct OrbitEntry {
    uint8_t a, b;
    uint16_t pad;
    float unused;
    double w;   // multiplicity / |G|
};

template <class W, class T, int C>
__global__ __launch_bounds__(MB) void k_szsz(const W *reps, int64_t dim, const T *psi,
                                             const OrbitEntry *orb, const int *orb_off, int np,
                                             double *partials) {
    __shared__ double sh[PB][MB];
    double acc[PB];
#pragma unroll
    for (int k = 0; k < PB; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * MB;
    for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < dim; i += stride) {
        const W s = reps ? reps[i] : W(0);
        double p = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double v = (double)psi[i * C + c];
            p = __builtin_fma(v, v, p);
        }
#pragma unroll
        for (int k = 0; k < PB; ++k) {
            if (k >= np) break;
            double o = 0.0;
            for (int e = orb_off[k]; e < orb_off[k + 1]; ++e) {
                const OrbitEntry oe = orb[e];
                const bool eq = ((s >> oe.a) & 1) == ((s >> oe.b) & 1);
                o += eq ? 0.25 * oe.w : -0.25 * oe.w;
            }
            acc[k] = __builtin_fma(p, o, acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < PB; ++k) sh[k][threadIdx.x] = acc[k];
    for (int h = MB / 2; h > 0; h >>= 1) {
        __syncthreads();
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int k = 0; k < PB; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + h];
    }
    __syncthreads();
    if ((int)threadIdx.x < PB) partials[(size_t)blockIdx.x * PB + threadIdx.x] = sh[threadIdx.x][0];
}

// U(1) blocks: states by Lin rank, computed from the colex successor of the
// previous one would serialise; instead each lane unranks its state.
template <class W>
__device__ __forceinline__ W unrank_u1(uint64_t r, int N, int n_up, const uint64_t *binom) {
    W s = 0;
    int k = n_up;
    for (int p = N - 1; p >= 0 && k > 0; --p) {
        const uint64_t c = binom[p * 65 + k];
        if (r >= c) {
            s |= W(1) << p;
            r -= c;
            --k;
        }
    }
    return s;
}

template <class W, class T, int C>
__global__ __launch_bounds__(MB) void k_szsz_u1(int64_t dim, int N, int n_up, const uint64_t *binom,
                                                const T *psi, const OrbitEntry *orb,
                                                const int *orb_off, int np, double *partials) {
    __shared__ double sh[PB][MB];
    double acc[PB];
#pragma unroll
    for (int k = 0; k < PB; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * MB;
    for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < dim; i += stride) {
        const W s = unrank_u1<W>((uint64_t)i, N, n_up, binom);
        double p = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const double v = (double)psi[i * C + c];
            p = __builtin_fma(v, v, p);
        }
#pragma unroll
        for (int k = 0; k < PB; ++k) {
            if (k >= np) break;
            double o = 0.0;
            for (int e = orb_off[k]; e < orb_off[k + 1]; ++e) {
                const OrbitEntry oe = orb[e];
                const bool eq = ((s >> oe.a) & 1) == ((s >> oe.b) & 1);
                o += eq ? 0.25 * oe.w : -0.25 * oe.w;
            }
            acc[k] = __builtin_fma(p, o, acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < PB; ++k) sh[k][threadIdx.x] = acc[k];
    for (int h = MB / 2; h > 0; h >>= 1) {
        __syncthreads();
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int k = 0; k < PB; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + h];
    }
    __syncthreads();
    if ((int)threadIdx.x < PB) partials[(size_t)blockIdx.x * PB + threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace

int expect_szsz(xdg_basis_s *b, const void *psi, int dtype, int n_pairs, const int32_t *pairs,
                double *out, hipStream_t st) {
    if (n_pairs < 0 || (n_pairs > 0 && (!pairs || !out)) || (b->dim > 0 && n_pairs > 0 && !psi)) {
        set_error("expect_szsz: bad arguments");
        return XDG_EINVAL;
    }
    if (dtype < XDG_F64 || dtype > XDG_C64) {
        set_error("unknown dtype %d", dtype);
        return XDG_EINVAL;
    }
    if (b->is_complex && !dtype_complex(dtype)) {
        set_error("the block has complex characters: vectors must be XDG_C128 or XDG_C64");
        return XDG_EINVAL;
    }
    for (int k = 0; k < n_pairs; ++k)
        if (pairs[2 * k] < 0 || pairs[2 * k] >= b->n_sites || pairs[2 * k + 1] < 0 ||
            pairs[2 * k + 1] >= b->n_sites) {
            set_error("pair %d = (%d, %d) outside [0, %d)", k, pairs[2 * k], pairs[2 * k + 1],
                      b->n_sites);
            return XDG_EINVAL;
        }
    if (n_pairs == 0) return XDG_OK;
    if (b->dim == 0) {
        std::fill(out, out + n_pairs, 0.0);
        return XDG_OK;
    }
    const int N = b->n_sites, G = std::max(b->n_sym, 1);
    const bool single = dtype_single(dtype);
    const int C = dtype_complex(dtype) ? 2 : 1;
    const int grid = (int)std::min<int64_t>((b->dim + MB - 1) / MB, (int64_t)device_cu_count() * 8);
    DevBuf orb_d, off_d, parts, binom_d;
    XDG_RETURN_IF(parts.alloc(sizeof(double) * (size_t)grid * PB));
    if (b->plan.kind == K_U1) {
        std::vector<uint64_t> bt(65 * 65);
        for (int p = 0; p <= 64; ++p)
            for (int q = 0; q <= 64; ++q) bt[p * 65 + q] = binomial(p, q);
        XDG_RETURN_IF(binom_d.upload(bt.data(), bt.size() * 8));
    }
    std::vector<double> host_parts((size_t)grid * PB);
    for (int k0 = 0; k0 < n_pairs; k0 += PB) {
        const int np = std::min(PB, n_pairs - k0);
        // orbit of each pair: distinct unordered site pairs with multiplicity / |G|
        std::vector<OrbitEntry> orb;
        std::vector<int> off(PB + 1, 0);
        for (int k = 0; k < np; ++k) {
            const int a = pairs[2 * (k0 + k)], c = pairs[2 * (k0 + k) + 1];
            std::map<std::pair<int, int>, int> mult;
            for (int g = 0; g < G; ++g) {
                int ga = a, gc = c;
                if (b->n_sym) {
                    ga = b->perm[(size_t)g * N + a];
                    gc = b->perm[(size_t)g * N + c];
                }
                ++mult[{std::min(ga, gc), std::max(ga, gc)}];
            }
            for (auto &e : mult)
                orb.push_back(OrbitEntry{(uint8_t)e.first.first, (uint8_t)e.first.second, 0, 0.0f,
                                         (double)e.second / G});
            off[k + 1] = (int)orb.size();
        }
        for (int k = np; k < PB; ++k) off[k + 1] = off[np];
        XDG_RETURN_IF(orb_d.upload(orb.data(), orb.size() * sizeof(OrbitEntry)));
        XDG_RETURN_IF(off_d.upload(off.data(), off.size() * sizeof(int)));
        const OrbitEntry *o = orb_d.as<OrbitEntry>();
        const int *of = off_d.as<int>();
        double *pp = parts.as<double>();
#define XDG_SZSZ(W_, T_, C_)                                                                    \
    do {                                                                                        \
        if (b->plan.kind == K_U1)                                                               \
            hipLaunchKernelGGL((k_szsz_u1<W_, T_, C_>), dim3(grid), dim3(MB), 0, st, b->dim, N, \
                               b->n_up, binom_d.as<uint64_t>(), (const T_ *)psi, o, of, np, pp); \
        else                                                                                    \
            hipLaunchKernelGGL((k_szsz<W_, T_, C_>), dim3(grid), dim3(MB), 0, st,              \
                               b->reps.as<W_>(), b->dim, (const T_ *)psi, o, of, np, pp);       \
    } while (0)
        if (b->wide) {
            if (single) {
                if (C == 2) XDG_SZSZ(uint64_t, float, 2); else XDG_SZSZ(uint64_t, float, 1);
            } else {
                if (C == 2) XDG_SZSZ(uint64_t, double, 2); else XDG_SZSZ(uint64_t, double, 1);
            }
        } else {
            if (single) {
                if (C == 2) XDG_SZSZ(uint32_t, float, 2); else XDG_SZSZ(uint32_t, float, 1);
            } else {
                if (C == 2) XDG_SZSZ(uint32_t, double, 2); else XDG_SZSZ(uint32_t, double, 1);
            }
        }
#undef XDG_SZSZ
        XDG_TRY_HIP(hipGetLastError());
        XDG_RETURN_IF(copy_d2h(host_parts.data(), pp, sizeof(double) * host_parts.size(), st));
        for (int k = 0; k < np; ++k) {
            double s = 0.0;
            for (int blk = 0; blk < grid; ++blk) s += host_parts[(size_t)blk * PB + k];
            out[k0 + k] = s;
        }
    }
    return XDG_OK;
}

}  // namespace xdg
