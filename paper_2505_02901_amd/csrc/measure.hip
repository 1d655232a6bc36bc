// Expectation values of symmetrised Ising correlations on a block
// (measurements, Sec. 3.8; symmetrisation of an operator over the group,
// Sec. 3.13).  O_ab = (1/|G|) sum_g S^z_{g(a)} S^z_{g(b)} is diagonal on the
// symmetric basis, with value o_ab(s) = (1/|G|) sum_g sz_s(g(a)) sz_s(g(b)) on
// representative s, so <psi|O_ab|psi> = sum_s |psi_s|^2 o_ab(s).  The orbit
// of each pair under the group is folded on the host into distinct site
// pairs with weights; a lane owns a state and up to PB pairs; block sums and
// their total are taken in a fixed order.
#include <algorithm>
#include <complex>
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

__global__ __launch_bounds__(MB) void k_unrank_all(int64_t dim, int N, int n_up,
                                                   const uint64_t *binom, uint64_t *out) {
    const int64_t stride = (int64_t)gridDim.x * MB;
    for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < dim; i += stride)
        out[i] = unrank_u1<uint64_t>((uint64_t)i, N, n_up, binom);
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

// ---------------------------------------------------------------------------
// Diagonal one-site operators between blocks (the operator at a momentum of
// Sec. 3.13, used for dynamical structure factors, Sec. 4.4):
//   O = sum_j c_j S^z_j.  If c is covariant, c_{g^-1(i)} = mu(g) c_i with
//   mu(g) = chi_in(g) / chi_out(g), then O maps the symmetric state of
//   representative s in the input block to o(s) times the symmetric state of
//   s in the output block, o(s) = sum_j c_j sz_s(j) (zero when s has no state
//   in the output block).  y[r] = o(s_r) x[idx_in(s_r)] over the output rows.
namespace xdg {
namespace {

template <class W, class T, bool CPLX>
__global__ __launch_bounds__(MB) void k_diag_transfer(const W *reps_out, const uint64_t *reps_u1,
                                                      int64_t dim_out, int N, const int64_t *idx,
                                                      const double2 *c, const T *x, T *y) {
    __shared__ double2 sc[64];
    for (int j = threadIdx.x; j < N; j += MB) sc[j] = c[j];
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * MB;
    for (int64_t r = (int64_t)blockIdx.x * MB + threadIdx.x; r < dim_out; r += stride) {
        const uint64_t s = reps_out ? (uint64_t)reps_out[r] : reps_u1[r];
        double orr = 0.0, oi = 0.0;
        for (int j = 0; j < N; ++j) {
            const double sz = ((s >> j) & 1) ? 0.5 : -0.5;
            orr = __builtin_fma(sc[j].x, sz, orr);
            oi = __builtin_fma(sc[j].y, sz, oi);
        }
        const int64_t q = idx[r];
        if constexpr (CPLX) {
            double yr = 0.0, yi = 0.0;
            if (q >= 0) {
                const double xr = (double)x[2 * q], xi = (double)x[2 * q + 1];
                yr = orr * xr - oi * xi;
                yi = orr * xi + oi * xr;
            }
            y[2 * r] = (T)yr;
            y[2 * r + 1] = (T)yi;
        } else {
            y[r] = q >= 0 ? (T)(orr * (double)x[q]) : T(0);
        }
    }
}

template <class W>
__global__ __launch_bounds__(MB) void k_widen(const W *in, int64_t n, uint64_t *out) {
    const int64_t stride = (int64_t)gridDim.x * MB;
    for (int64_t i = (int64_t)blockIdx.x * MB + threadIdx.x; i < n; i += stride) out[i] = in[i];
}

}  // namespace

int apply_diag_transfer(xdg_basis_s *bin, xdg_basis_s *bout, const double *coef, const void *x,
                        void *y, int dtype, hipStream_t st) {
    if (!coef || (bout->dim > 0 && (!y || (!x && bin->dim > 0))) || x == y) {
        set_error("diag transfer: bad arguments");
        return XDG_EINVAL;
    }
    if (dtype < XDG_F64 || dtype > XDG_C64) {
        set_error("unknown dtype %d", dtype);
        return XDG_EINVAL;
    }
    const int N = bin->n_sites;
    if (bout->n_sites != N || bout->n_up != bin->n_up || bout->n_sym != bin->n_sym ||
        bout->perm != bin->perm) {
        set_error("diag transfer: the blocks need the same sites, n_up and group");
        return XDG_EINVAL;
    }
    bool coef_cplx = false;
    for (int j = 0; j < N; ++j) coef_cplx |= std::fabs(coef[2 * j + 1]) > 0.0;
    const bool cplx = dtype_complex(dtype);
    if (!cplx && (coef_cplx || bin->is_complex || bout->is_complex)) {
        set_error("diag transfer: complex coefficients or blocks need XDG_C128 / XDG_C64");
        return XDG_EINVAL;
    }
    // covariance: c_{g^-1(i)} = mu(g) c_i with mu(g) = chi_in(g) / chi_out(g)
    if (bin->n_sym) {
        double cmax = 0.0;
        for (int j = 0; j < N; ++j) cmax = std::max(cmax, std::hypot(coef[2 * j], coef[2 * j + 1]));
        for (int g = 0; g < bin->n_sym; ++g) {
            const std::complex<double> ci(bin->chi[2 * g], bin->chi[2 * g + 1]);
            const std::complex<double> co(bout->chi[2 * g], bout->chi[2 * g + 1]);
            const std::complex<double> mu = ci / co;
            std::vector<int> inv(N);
            for (int i = 0; i < N; ++i) inv[bin->perm[(size_t)g * N + i]] = i;
            for (int i = 0; i < N; ++i) {
                const std::complex<double> a(coef[2 * inv[i]], coef[2 * inv[i] + 1]);
                const std::complex<double> b(coef[2 * i], coef[2 * i + 1]);
                if (std::abs(a - mu * b) > 1e-12 * std::max(1.0, cmax)) {
                    set_error("diag transfer: coefficients do not carry the character ratio of "
                              "the two blocks (element %d, site %d)", g, i);
                    return XDG_ENOTSYM;
                }
            }
        }
    }
    const int64_t Dout = bout->dim;
    if (Dout == 0) return XDG_OK;
    DevBuf states, idx, cd;
    XDG_RETURN_IF(idx.alloc(8 * (size_t)Dout));
    std::vector<double> c2(coef, coef + 2 * (size_t)N);
    XDG_RETURN_IF(cd.upload(c2.data(), c2.size() * 8));
    const int grid = (int)std::min<int64_t>((Dout + MB - 1) / MB, (int64_t)device_cu_count() * 16);
    const uint64_t *u1 = nullptr;
    if (bout->plan.kind == K_U1) {
        // U(1) rows: the states are the colex unranking of the row numbers
        std::vector<uint64_t> bt(65 * 65);
        for (int p = 0; p <= 64; ++p)
            for (int q = 0; q <= 64; ++q) bt[p * 65 + q] = binomial(p, q);
        DevBuf binom_d;
        XDG_RETURN_IF(binom_d.upload(bt.data(), bt.size() * 8));
        XDG_RETURN_IF(states.alloc(8 * (size_t)Dout));
        hipLaunchKernelGGL(k_unrank_all, dim3(grid), dim3(MB), 0, st, Dout, N, bout->n_up,
                           binom_d.as<uint64_t>(), states.as<uint64_t>());
        XDG_TRY_HIP(hipGetLastError());
        XDG_TRY_HIP(hipStreamSynchronize(st));
        u1 = states.as<uint64_t>();
    } else {
        XDG_RETURN_IF(states.alloc(8 * (size_t)Dout));
        if (bout->wide)
            hipLaunchKernelGGL(k_widen<uint64_t>, dim3(grid), dim3(MB), 0, st,
                               bout->reps.as<uint64_t>(), Dout, states.as<uint64_t>());
        else
            hipLaunchKernelGGL(k_widen<uint32_t>, dim3(grid), dim3(MB), 0, st,
                               bout->reps.as<uint32_t>(), Dout, states.as<uint64_t>());
        XDG_TRY_HIP(hipGetLastError());
        u1 = states.as<uint64_t>();
    }
    XDG_TRY_HIP(hipStreamSynchronize(st));
    XDG_RETURN_IF(basis_lookup(bin, states.as<uint64_t>(), Dout, idx.as<int64_t>(), st));
    const double2 *c = cd.as<double2>();
    const int64_t *ix = idx.as<int64_t>();
#define XDG_TRANSFER(T_, CPLX_)                                                                 \
    hipLaunchKernelGGL((k_diag_transfer<uint64_t, T_, CPLX_>), dim3(grid), dim3(MB), 0, st,   \
                       nullptr, u1, Dout, N, ix, c, (const T_ *)x, (T_ *)y)
    if (dtype == XDG_F64) XDG_TRANSFER(double, false);
    else if (dtype == XDG_F32) XDG_TRANSFER(float, false);
    else if (dtype == XDG_C128) XDG_TRANSFER(double, true);
    else XDG_TRANSFER(float, true);
#undef XDG_TRANSFER
    XDG_TRY_HIP(hipGetLastError());
    XDG_TRY_HIP(hipStreamSynchronize(st));
    return XDG_OK;
}

}  // namespace xdg
