// Sector basis on the GPU (Spinhalf(N, nup[, irrep]), Sec. 3.1 and 3.11):
// ascending enumeration of popcount-n_up states in independent chunks
// (colex unranking + next-same-popcount), representative and compatibility
// test per candidate, count -> scan -> ordered fill; then the device index
// (Lin tables for the U(1) block, Sec. 5.2; a line-bucketed hash for
// representatives).  Also the counter-based random state generator.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.hpp"

namespace xdg {

// ------------------------------------------------------------------ utils --
// Device memory held by the library's buffers, and the caller's limit on it
// (0 = none), see xdg_set_device_memory_limit.
static std::atomic<uint64_t> g_dev_bytes{0};
static std::atomic<uint64_t> g_dev_limit{0};

void set_device_memory_limit(uint64_t bytes) { g_dev_limit.store(bytes); }
uint64_t device_memory_in_use() { return g_dev_bytes.load(); }

void DevBuf::release() {
    if (p) {
        (void)hipFree(p);
        g_dev_bytes.fetch_sub(bytes);
    }
    p = nullptr;
    bytes = 0;
}

int DevBuf::alloc(size_t n) {
    release();
    if (n == 0) return XDG_OK;
    const uint64_t limit = g_dev_limit.load();
    const uint64_t held = g_dev_bytes.fetch_add(n) + n;
    if (limit && held > limit) {
        g_dev_bytes.fetch_sub(n);
        set_error("device memory limit: %zu more bytes would bring the library to %llu of %llu",
                  n, (unsigned long long)held, (unsigned long long)limit);
        return XDG_ENOMEM;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        g_dev_bytes.fetch_sub(n);
        p = nullptr;
        (void)hipGetLastError();
        set_error("hipMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
        return XDG_ENOMEM;
    }
    bytes = n;
    return XDG_OK;
}

int DevBuf::upload(const void *host, size_t n) {
    XDG_RETURN_IF(alloc(n));
    if (n) XDG_RETURN_IF(copy_h2d(p, host, n, nullptr));
    return XDG_OK;
}

// Host <-> device transfers go through a page-locked buffer owned by the
// library (per thread, grown on demand, chunks of at most 64 MiB) with an
// explicit wait after every chunk: no DMA ever targets pageable caller
// memory, and no transfer is still in flight when the call returns.
namespace {
// (kept until the process ends: freeing it from a thread-exit destructor
// could run after the HIP runtime has shut down)
struct PinnedStage {
    void *p = nullptr;
    size_t cap = 0;
    int reserve(size_t n) {
        if (n <= cap) return XDG_OK;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipHostMalloc(&p, n, hipHostMallocDefault);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            set_error("hipHostMalloc(%zu bytes) failed: %s", n, hipGetErrorString(e));
            return XDG_ENOMEM;
        }
        cap = n;
        return XDG_OK;
    }
};
thread_local PinnedStage g_stage;
constexpr size_t STAGE_CHUNK = (size_t)64 << 20;
}  // namespace

int copy_d2h(void *dst, const void *src, size_t n, hipStream_t st) {
    size_t done = 0;
    while (done < n) {
        const size_t len = std::min(STAGE_CHUNK, n - done);
        XDG_RETURN_IF(g_stage.reserve(len));
        XDG_TRY_HIP(hipMemcpyAsync(g_stage.p, static_cast<const char *>(src) + done, len,
                                   hipMemcpyDeviceToHost, st));
        XDG_TRY_HIP(hipStreamSynchronize(st));
        std::memcpy(static_cast<char *>(dst) + done, g_stage.p, len);
        done += len;
    }
    return XDG_OK;
}

int copy_h2d(void *dst, const void *src, size_t n, hipStream_t st) {
    size_t done = 0;
    while (done < n) {
        const size_t len = std::min(STAGE_CHUNK, n - done);
        XDG_RETURN_IF(g_stage.reserve(len));
        std::memcpy(g_stage.p, static_cast<const char *>(src) + done, len);
        XDG_TRY_HIP(hipMemcpyAsync(static_cast<char *>(dst) + done, g_stage.p, len,
                                   hipMemcpyHostToDevice, st));
        XDG_TRY_HIP(hipStreamSynchronize(st));
        done += len;
    }
    return XDG_OK;
}

int device_cu_count() {
    static int cached = 0;
    if (!cached) {
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            cu > 0)
            cached = cu;
        else
            cached = 256;
    }
    return cached;
}

size_t lds_limit() {
    static size_t cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            v > 0)
            cached = (size_t)v;
        else
            cached = 65536;
    }
    return cached;
}

__host__ __device__ static inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// ------------------------------------------------------------ enumeration --
template <class W>
struct EnumArgs {
    int N, n_up, n_sym;
    uint64_t total, n_chunks;
    uint32_t chunk_len;
    const uint64_t *binom;     // [65][65]
    uint32_t *counts;          // [n_chunks] (count pass)
    const uint64_t *offsets;   // [n_chunks] (fill pass; NULL = rank itself)
    W *reps;
    uint16_t *stab;
    const double2 *chi;
    const AffineElem *aff;
    const uint64_t *bytetab;
    int n_bchunks;
    const uint16_t *mintop;
    const uint32_t *cand_off;
    const uint16_t *cand_list;
    const uint32_t *sp;
    const uint16_t *tperm;
    int n_s, m, pb, n_perm;
    uint32_t n_cand;
    int stage_sub;
};

template <class W, int KIND, bool FILL>
__global__ __launch_bounds__(256) void k_enum(EnumArgs<W> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const double2 *chi = A.chi;
    const AffineElem *aff = A.aff;
    SubCtx C{A.mintop, A.cand_off, A.cand_list, A.sp, A.tperm, A.n_s, A.m, A.pb};
    if constexpr (KIND != K_U1) {
        double2 *lchi = reinterpret_cast<double2 *>(smem);
        size_t off = align16(sizeof(double2) * A.n_sym);
        for (int g = threadIdx.x; g < A.n_sym; g += blockDim.x) lchi[g] = A.chi[g];
        chi = lchi;
        if constexpr (KIND == K_AFF) {
            AffineElem *laff = reinterpret_cast<AffineElem *>(smem + off);
            for (int g = threadIdx.x; g < A.n_sym; g += blockDim.x) laff[g] = A.aff[g];
            aff = laff;
        }
        if constexpr (KIND == K_SUB) {
            if (A.stage_sub) {
                const uint32_t NV = (uint32_t)A.n_s << A.m;
                uint16_t *lmt = reinterpret_cast<uint16_t *>(smem + off);
                off = align16(off + 2 * NV);
                uint32_t *lco = reinterpret_cast<uint32_t *>(smem + off);
                off = align16(off + 4 * (NV + 1));
                uint16_t *lcl = reinterpret_cast<uint16_t *>(smem + off);
                for (uint32_t e = threadIdx.x; e < NV; e += blockDim.x) lmt[e] = A.mintop[e];
                for (uint32_t e = threadIdx.x; e <= NV; e += blockDim.x) lco[e] = A.cand_off[e];
                for (uint32_t e = threadIdx.x; e < A.n_cand; e += blockDim.x) lcl[e] = A.cand_list[e];
                off = align16(off + 2 * (size_t)A.n_cand);
                const uint32_t GS = (uint32_t)A.n_sym * A.n_s;
                uint32_t *lsp = reinterpret_cast<uint32_t *>(smem + off);
                off = align16(off + 4 * (size_t)GS);
                uint16_t *ltp = reinterpret_cast<uint16_t *>(smem + off);
                const uint32_t TP = (uint32_t)A.n_perm * 2u << A.pb;
                for (uint32_t e = threadIdx.x; e < GS; e += blockDim.x) lsp[e] = A.sp[e];
                for (uint32_t e = threadIdx.x; e < TP; e += blockDim.x) ltp[e] = A.tperm[e];
                C.mintop = lmt;
                C.cand_off = lco;
                C.cand_list = lcl;
                C.sp = lsp;
                C.tperm = ltp;
            }
        }
        __syncthreads();
    }
    const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= A.n_chunks) return;
    const uint64_t r0 = c * A.chunk_len;
    const uint64_t r1 = r0 + A.chunk_len < A.total ? r0 + A.chunk_len : A.total;
    W s = unrank_colex<W>(r0, A.N, A.n_up, A.binom);
    uint64_t pos = FILL ? (A.offsets ? A.offsets[c] : r0) : 0;
    uint32_t cnt = 0;
    for (uint64_t r = r0; r < r1; ++r) {
        bool keep = true;
        int st = 1;
        if constexpr (KIND != K_U1) {
            double cr, ci;
            bool rep;
            if constexpr (KIND == K_AFF)
                rep = aff_is_rep<W>(aff, A.n_sym, A.N, s, chi, st, cr, ci);
            else if constexpr (KIND == K_SUB)
                rep = sub_is_rep<W>(C, s, chi, st, cr, ci);
            else
                rep = tab_is_rep<W>(A.bytetab, A.n_bchunks, A.n_sym, s, chi, st, cr, ci);
            // the orbit carries a symmetric state iff the stabiliser sum of chi is nonzero
            keep = rep && (cr * cr + ci * ci > 0.25);
        }
        if (keep) {
            if constexpr (FILL) {
                A.reps[pos] = s;
                if constexpr (KIND != K_U1) A.stab[pos] = (uint16_t)st;
                ++pos;
            }
            ++cnt;
        }
        if (r + 1 < r1) s = next_same_popcount<W>(s);
    }
    if constexpr (!FILL) A.counts[c] = cnt;
}

// ------------------------------------------------------------------- scan --
// Exclusive scan of u32 counts into u64 offsets, three passes with
// 1024-element tiles; fixed order, no atomics.
__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *sh, uint64_t *total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int d = 1; d < (int)blockDim.x; d <<= 1) {
        uint64_t add = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    const uint64_t incl = sh[t];
    if (total) *total = sh[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(1024) void k_scan_tiles(const uint32_t *counts, uint64_t n,
                                                     uint64_t *tile_sums) {
    __shared__ uint64_t sh[1024];
    const uint64_t i = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
    uint64_t v = i < n ? counts[i] : 0;
    uint64_t tot;
    block_exclusive_scan(v, sh, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_sums(uint64_t *tile_sums, uint64_t n_tiles,
                                                    uint64_t *grand_total) {
    __shared__ uint64_t sh[1024];
    const uint64_t per = (n_tiles + 1023) / 1024;
    const uint64_t b0 = threadIdx.x * per;
    uint64_t local = 0;
    for (uint64_t b = b0; b < b0 + per && b < n_tiles; ++b) local += tile_sums[b];
    uint64_t tot;
    uint64_t base = block_exclusive_scan(local, sh, &tot);
    for (uint64_t b = b0; b < b0 + per && b < n_tiles; ++b) {
        uint64_t v = tile_sums[b];
        tile_sums[b] = base;
        base += v;
    }
    if (threadIdx.x == 0) *grand_total = tot;
}

__global__ __launch_bounds__(1024) void k_scan_apply(const uint32_t *counts, uint64_t n,
                                                     const uint64_t *tile_base, uint64_t *offsets) {
    __shared__ uint64_t sh[1024];
    const uint64_t i = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
    uint64_t v = i < n ? counts[i] : 0;
    uint64_t ex = block_exclusive_scan(v, sh, nullptr);
    if (i < n) offsets[i] = ex + tile_base[blockIdx.x];
}

// ------------------------------------------------------------------- hash --
template <class W>
__global__ __launch_bounds__(256) void k_hash_insert(const W *reps, uint64_t dim, void *table,
                                                     uint64_t n_lines, W empty) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dim) return;
    const W key = reps[i];
    uint64_t line = hash_line<W>(key, n_lines);
    for (;;) {
        if constexpr (sizeof(W) == 4) {
            Line32 *L = reinterpret_cast<Line32 *>(table) + line;
            for (int s = 0; s < 8; ++s) {
                uint32_t old = atomicCAS(&L->k[s], (uint32_t)empty, (uint32_t)key);
                if (old == (uint32_t)empty) {
                    L->v[s] = (uint32_t)i;
                    return;
                }
            }
        } else {
            Line64 *L = reinterpret_cast<Line64 *>(table) + line;
            for (int s = 0; s < 5; ++s) {
                unsigned long long old =
                    atomicCAS(reinterpret_cast<unsigned long long *>(&L->k[s]),
                              (unsigned long long)empty, (unsigned long long)key);
                if (old == (unsigned long long)empty) {
                    L->v[s] = (uint32_t)i;
                    return;
                }
            }
        }
        line = line + 1 == n_lines ? 0 : line + 1;
    }
}

// ------------------------------------------------------------------- rank --
// Sets the bit of every basis state; the first state of each word (the reps
// are ascending and the colex rank preserves their order) writes its index
// as the word's count.
template <class W>
__global__ __launch_bounds__(256) void k_rank_build(const W *reps, uint64_t dim, const void *T,
                                                    RankLayout L, uint2 *words) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dim) return;
    const uint64_t r = colex_rank<W>(T, L, reps[i]);
    const uint64_t w = r >> 5;
    atomicOr(&words[w].y, 1u << (uint32_t)(r & 31));
    if (i == 0 || (colex_rank<W>(T, L, reps[i - 1]) >> 5) != w) words[w].x = (uint32_t)i;
}

// index of arbitrary states (-1 when absent)
struct RankArgs {
    const uint2 *words;
    uint64_t n_words;   // 0: no rank index
    const void *tab;
    RankLayout L;
};

template <class W>
__global__ __launch_bounds__(256) void k_lookup(const uint64_t *states, int64_t n, int64_t *out,
                                                int N, int n_up, int u1, const uint32_t *lin,
                                                int nlo, const void *table, uint64_t n_lines,
                                                W empty, RankArgs R) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t s = states[i];
    int64_t r = -1;
    const bool in_range = N == 64 || (s >> N) == 0;
    if (in_range && __popcll(s) == n_up) {
        if (u1) {
            const uint64_t lo = s & ((1ull << nlo) - 1), hi = s >> nlo;
            r = (int64_t)lin[(1ull << nlo) + hi] + (int64_t)lin[lo];
        } else if (R.n_words) {
            r = rank_find(R.words, R.n_words, colex_rank<W>(R.tab, R.L, (W)s));
        } else if (n_lines) {
            r = hash_find<W>(table, n_lines, empty, (W)s);
        }
    }
    out[i] = r;
}

// ----------------------------------------------------------------- random --
__device__ __forceinline__ uint64_t splitmix_out(uint64_t seed, uint64_t n) {
    uint64_t z = seed + n * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double u53(uint64_t z) {
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

template <class T>
__global__ __launch_bounds__(256) void k_random(uint64_t n, uint64_t seed, int kind, T *out) {
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const double u1 = u53(splitmix_out(seed, 2 * q + 1));
        double v;
        if (kind == 0) {
            v = 2.0 * u1 - 1.0;
        } else {
            const double u2 = u53(splitmix_out(seed, 2 * q + 2));
            v = sqrt(-2.0 * log1p(-u1)) * cos(2.0 * M_PI * u2);
        }
        out[q] = (T)v;
    }
}

int random_fill(int64_t n_scalars, uint64_t seed, int kind, bool single, void *out,
                hipStream_t st) {
    if (n_scalars <= 0) return XDG_OK;
    const int block = 256;
    const uint64_t want = ((uint64_t)n_scalars + block - 1) / block;
    const int grid = (int)std::min<uint64_t>(want, (uint64_t)device_cu_count() * 16);
    if (single)
        hipLaunchKernelGGL(k_random<float>, dim3(grid), dim3(block), 0, st, (uint64_t)n_scalars,
                           seed, kind, (float *)out);
    else
        hipLaunchKernelGGL(k_random<double>, dim3(grid), dim3(block), 0, st,
                           (uint64_t)n_scalars, seed, kind, (double *)out);
    XDG_TRY_HIP(hipGetLastError());
    return XDG_OK;
}

// ------------------------------------------------------------- host side --
namespace {

template <class W>
int enumerate(xdg_basis_s *b, DevBuf &binom_d) {
    const int N = b->n_sites, n = b->n_up, kind = b->plan.kind;
    const uint64_t total = binomial(N, n);
    EnumArgs<W> A{};
    A.N = N;
    A.n_up = n;
    A.n_sym = b->n_sym;
    A.total = total;
    A.binom = binom_d.as<uint64_t>();
    A.chi = b->chi_d.as<double2>();
    A.aff = b->t_aff.as<AffineElem>();
    A.bytetab = b->t_bytes.as<uint64_t>();
    A.n_bchunks = b->plan.bytes.n_chunks;
    A.mintop = b->t_mintop.as<uint16_t>();
    A.cand_off = b->t_candoff.as<uint32_t>();
    A.cand_list = b->t_candlist.as<uint16_t>();
    A.sp = b->t_pid.as<uint32_t>();
    A.tperm = b->t_tperm.as<uint16_t>();
    A.n_s = b->plan.sub.n_s;
    A.m = b->plan.sub.m;
    A.pb = b->plan.sub.pb;
    A.n_perm = b->plan.sub.n_perm;
    A.n_cand = (uint32_t)b->plan.sub.cand_list.size();

    const uint64_t lanes_target = (uint64_t)device_cu_count() * 1024;
    uint64_t cl = total / lanes_target;
    cl = std::max<uint64_t>(16, std::min<uint64_t>(4096, cl));
    A.chunk_len = (uint32_t)cl;
    A.n_chunks = (total + cl - 1) / cl;

    size_t lds = 0;
    if (kind != K_U1) {
        lds = align16(sizeof(double2) * b->n_sym);
        if (kind == K_AFF) lds += align16(sizeof(AffineElem) * b->n_sym);
        if (kind == K_SUB) {
            const size_t NV = (size_t)A.n_s << A.m;
            const size_t GS = (size_t)A.n_sym * A.n_s;
            size_t need = align16(2 * NV) + align16(4 * (NV + 1)) + align16(2 * (size_t)A.n_cand) +
                          align16(4 * GS) +
                          align16(2 * ((size_t)A.n_perm * 2 << A.pb));
            if (lds + need <= lds_limit()) {
                A.stage_sub = 1;
                lds += need;
            }
        }
    }
    const int block = 256;
    const uint64_t grid = (A.n_chunks + block - 1) / block;
    if (grid > 0x7fffffffull) {
        set_error("enumeration grid too large");
        return XDG_EINVAL;
    }
    auto kcount = k_enum<W, K_U1, false>;
    auto kfill = k_enum<W, K_U1, true>;
    if (kind == K_AFF) {
        kcount = k_enum<W, K_AFF, false>;
        kfill = k_enum<W, K_AFF, true>;
    } else if (kind == K_SUB) {
        kcount = k_enum<W, K_SUB, false>;
        kfill = k_enum<W, K_SUB, true>;
    } else if (kind == K_TAB) {
        kcount = k_enum<W, K_TAB, false>;
        kfill = k_enum<W, K_TAB, true>;
    }
    if (lds > 65536) {
        XDG_TRY_HIP(hipFuncSetAttribute((const void *)kcount,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        XDG_TRY_HIP(hipFuncSetAttribute((const void *)kfill,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    }

    DevBuf counts, offsets, tiles, tot;
    uint64_t dim;
    if (kind == K_U1) {
        dim = total;
    } else {
        XDG_RETURN_IF(counts.alloc(sizeof(uint32_t) * A.n_chunks));
        XDG_RETURN_IF(offsets.alloc(sizeof(uint64_t) * A.n_chunks));
        const uint64_t n_tiles = (A.n_chunks + 1023) / 1024;
        XDG_RETURN_IF(tiles.alloc(sizeof(uint64_t) * n_tiles));
        XDG_RETURN_IF(tot.alloc(sizeof(uint64_t)));
        A.counts = counts.as<uint32_t>();
        hipLaunchKernelGGL(kcount, dim3((unsigned)grid), dim3(block), lds, 0, A);
        XDG_TRY_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)n_tiles), dim3(1024), 0, 0,
                           counts.as<uint32_t>(), A.n_chunks, tiles.as<uint64_t>());
        hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, 0, tiles.as<uint64_t>(),
                           n_tiles, tot.as<uint64_t>());
        hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)n_tiles), dim3(1024), 0, 0,
                           counts.as<uint32_t>(), A.n_chunks, tiles.as<uint64_t>(),
                           offsets.as<uint64_t>());
        XDG_TRY_HIP(hipGetLastError());
        XDG_RETURN_IF(copy_d2h(&dim, tot.p, sizeof dim, nullptr));
        A.offsets = offsets.as<uint64_t>();
    }
    if (dim >= 0xFFFFFFFFull) {
        set_error("block dimension %llu needs 64-bit indices (limit 2^32 - 1)",
                  (unsigned long long)dim);
        return XDG_EINVAL;
    }
    b->dim = (int64_t)dim;
    if (dim == 0) return XDG_OK;
    XDG_RETURN_IF(b->reps.alloc(sizeof(W) * dim));
    if (kind != K_U1) XDG_RETURN_IF(b->stab.alloc(sizeof(uint16_t) * dim));
    A.reps = b->reps.as<W>();
    A.stab = b->stab.as<uint16_t>();
    hipLaunchKernelGGL(kfill, dim3((unsigned)grid), dim3(block), lds, 0, A);
    XDG_TRY_HIP(hipGetLastError());
    XDG_TRY_HIP(hipDeviceSynchronize());
    return XDG_OK;
}

template <class W>
int build_hash(xdg_basis_s *b) {
    const uint64_t dim = (uint64_t)b->dim;
    const int slots = sizeof(W) == 4 ? 8 : 5;
    const double load = 0.5;   // mean occupied slots per slot
    uint64_t n_lines = (uint64_t)std::ceil((double)dim / (slots * load));
    n_lines = std::max<uint64_t>(n_lines, 1);
    if (n_lines >= (1ull << 32)) {
        set_error("hash index too large");
        return XDG_EINVAL;
    }
    XDG_RETURN_IF(b->hash.alloc(64 * n_lines));
    const W empty = b->n_up == b->n_sites ? W(0) : ~W(0);
    XDG_TRY_HIP(hipMemset(b->hash.p, empty ? 0xFF : 0x00, 64 * n_lines));
    b->hidx.n_lines = n_lines;
    b->hidx.slots = slots;
    const int block = 256;
    hipLaunchKernelGGL(k_hash_insert<W>, dim3((unsigned)((dim + block - 1) / block)), dim3(block),
                       0, 0, b->reps.as<W>(), dim, b->hash.p, n_lines, empty);
    XDG_TRY_HIP(hipGetLastError());
    XDG_TRY_HIP(hipDeviceSynchronize());
    return XDG_OK;
}

// Chunk tables of the colex rank (the layout read by colex_rank): the entry
// of chunk k, below set bits under it, chunk bits v is the sum over the set
// bits of v, the i-th (from the bottom) at site p = k cb + q, of
// C(p, below + i); sites beyond N contribute nothing.  Rows only for below
// in [rank_lo, rank_hi] of each chunk.  32-bit states: four chunks of 8
// sites, u32 entries.  Wider states: the widest chunk (fewest reads) whose
// table stays within 32 KiB (the apply kernels stage it in LDS), with u32
// entries saturating at 2^32 - 1 when max_rank, the largest rank the block
// must resolve, leaves room below that, u64 entries otherwise.
RankLayout rank_layout(int N, int n_up, bool wide, uint64_t max_rank) {
    RankLayout L{};
    auto rows_of = [&](int cb, int nc) {
        int rows = 0;
        for (int k = 0; k < nc; ++k) rows += rank_hi(n_up, cb, k) - rank_lo(N, n_up, cb, k) + 1;
        return rows;
    };
    if (!wide) {
        L.cb = RANK_CB32;
        L.nc = RANK_NC32;
        L.e32 = 1;
    } else {
        L.e32 = max_rank < 0xFFFFFFFFull - 64 ? 1 : 0;
        const size_t esz = L.e32 ? 4 : 8;
        for (L.cb = 8; L.cb > 4; --L.cb) {
            L.nc = (N + L.cb - 1) / L.cb;
            if (((size_t)rows_of(L.cb, L.nc) << L.cb) * esz <= 32768) break;
        }
        L.nc = (N + L.cb - 1) / L.cb;
    }
    int row = 0;
    for (int k = 0; k < L.nc; ++k) {
        const int lo = rank_lo(N, n_up, L.cb, k);
        L.rbase[k] = row - lo;
        row += rank_hi(n_up, L.cb, k) - lo + 1;
    }
    L.rows = row;
    return L;
}

template <class E>
void rank_tables(int N, int n_up, const RankLayout &L, std::vector<E> &T) {
    const int cb = L.cb;
    T.assign((size_t)L.rows << cb, 0);
    for (int k = 0; k < L.nc; ++k) {
        const int lo = rank_lo(N, n_up, cb, k), hi = rank_hi(n_up, cb, k);
        for (int below = lo; below <= hi; ++below) {
            const size_t row = (size_t)(L.rbase[k] + below);
            for (uint32_t v = 0; v < (1u << cb); ++v) {
                uint64_t r = 0;
                int c = below;
                for (int q = 0; q < cb; ++q) {
                    if (!((v >> q) & 1)) continue;
                    ++c;
                    const int p = k * cb + q;
                    if (p < N) r += binomial(p, c);
                }
                if (sizeof(E) == 4 && r > 0xFFFFFFFFull) r = 0xFFFFFFFFull;
                T[(row << cb) | v] = (E)r;
            }
        }
    }
}

uint64_t colex_rank_host(uint64_t s) {
    uint64_t r = 0;
    int c = 0;
    for (int p = 0; p < 64; ++p)
        if ((s >> p) & 1) r += binomial(p, ++c);
    return r;
}

// The rows of the chunk tables (layout L) for the chunks below B, in 4-byte
// entries: shares of sites below 32 are exact; larger ones (read only for
// bits above B, which the rank clears) saturate.
template <class E>
int xr_lower_rows(const RankLayout &L, const E *T, int B, int n_up, std::vector<uint32_t> &out) {
    const int nlc = (B + L.cb - 1) / L.cb;
    const int rows = L.rbase[nlc - 1] + rank_hi(n_up, L.cb, nlc - 1) + 1;
    out.resize((size_t)rows << L.cb);
    for (size_t e = 0; e < out.size(); ++e)
        out[e] = T[e] > (E)0xFFFFFFFFu ? 0xFFFFFFFFu : (uint32_t)T[e];
    return rows;
}

// First rank of every top block for rank-addressed vectors (top_rank): the
// blocks that are the minimal top of their own content, ascending, each
// followed by the colex ranks of the states of the remaining popcount on the
// B sites below it.  Not set up when the blocks do not tile the sites or B
// exceeds 31.  T: the block's chunk tables (u32 or u64 entries, layout L);
// first, last: its smallest and largest basis states.
template <class W>
int build_xr(xdg_basis_s *b, const void *T, const RankLayout &L, W first, W last) {
    const SublatticeTables &S = b->plan.sub;
    const int n_s = S.n_s, m = S.m, B = (n_s - 1) * m;
    if (n_s < 2 || n_s * m != b->n_sites || B < 1 || B > 31 || m > 16) return XDG_OK;
    const uint32_t V = 1u << m;
    std::vector<uint64_t> top(V, ~0ull);
    uint64_t acc = 0;
    for (uint32_t c = 0; c < V; ++c) {
        if (S.mintop[(size_t)(n_s - 1) * V + c] != c) continue;
        const int k = b->n_up - __builtin_popcount(c);
        if (k < 0 || k > B) continue;
        top[c] = acc;
        acc += binomial(B, k);
    }
    std::vector<uint32_t> low;
    const int rows = L.e32 ? xr_lower_rows(L, static_cast<const uint32_t *>(T), B, b->n_up, low)
                           : xr_lower_rows(L, static_cast<const uint64_t *>(T), B, b->n_up, low);
    const uint64_t r0 = top_rank<W>(low.data(), L, B, top.data(), first);
    const uint64_t r1 = top_rank<W>(low.data(), L, B, top.data(), last);
    if (r0 == ~0ull || r1 == ~0ull || r0 > r1 || r1 >= acc) {
        set_error("internal: a representative lies outside the top-block rank space");
        return XDG_EINVAL;
    }
    XDG_RETURN_IF(b->xr_top.upload(top.data(), sizeof(uint64_t) * V));
    if (acc < 0xFFFFFFFFull) {   // 4-byte first ranks for the kernels' LDS
        std::vector<uint32_t> t32(V);
        for (uint32_t c = 0; c < V; ++c) t32[c] = top[c] == ~0ull ? 0xFFFFFFFFu : (uint32_t)top[c];
        XDG_RETURN_IF(b->xr_top32.upload(t32.data(), sizeof(uint32_t) * V));
    }
    XDG_RETURN_IF(b->xr_rtab.upload(low.data(), sizeof(uint32_t) * low.size()));
    b->xr_rows = rows;
    b->xr_slots = r1 + 1;
    b->xr_bits = B;
    return XDG_OK;
}

// Rank index when it fits (see XDG_INDEX_RANK); returns XDG_OK with
// b->n_rwords = 0 when the hash index should be used instead.
template <class W>
int build_rank(xdg_basis_s *b) {
    const uint64_t dim = (uint64_t)b->dim;
    if (b->plan.flags & XDG_FLAG_HASH_INDEX) return XDG_OK;
    uint64_t last = 0;
    XDG_RETURN_IF(copy_d2h(&last, b->reps.as<W>() + (dim - 1), sizeof(W), nullptr));
    const uint64_t n_words = (colex_rank_host(last) >> 5) + 1;
    const int slots = sizeof(W) == 4 ? 8 : 5;
    const double hash_bytes = 64.0 * std::ceil((double)dim / (slots * 0.5));
    if ((double)n_words * 8.0 > 4.0 * hash_bytes + 64.0 * (1 << 20)) return XDG_OK;
    const RankLayout L = rank_layout(b->n_sites, b->n_up, sizeof(W) == 8, colex_rank_host(last));
    std::vector<uint32_t> T32;
    std::vector<uint64_t> T64;
    const void *T = nullptr;
    size_t tbytes = 0;
    if (L.e32) {
        rank_tables<uint32_t>(b->n_sites, b->n_up, L, T32);
        T = T32.data();
        tbytes = T32.size() * 4;
    } else {
        rank_tables<uint64_t>(b->n_sites, b->n_up, L, T64);
        T = T64.data();
        tbytes = T64.size() * 8;
    }
    // the table read of the device rank must give the plain colex rank
    if (colex_rank<W>(T, L, (W)last) != colex_rank_host(last)) {
        set_error("internal: colex chunk tables disagree with the colex rank");
        return XDG_EINVAL;
    }
    XDG_RETURN_IF(b->rtab.upload(T, tbytes));
    XDG_RETURN_IF(b->rwords.alloc(8 * n_words));
    XDG_TRY_HIP(hipMemset(b->rwords.p, 0, 8 * n_words));
    const int block = 256;
    hipLaunchKernelGGL(k_rank_build<W>, dim3((unsigned)((dim + block - 1) / block)), dim3(block), 0,
                       0, b->reps.as<W>(), dim, b->rtab.p, L, b->rwords.as<uint2>());
    XDG_TRY_HIP(hipGetLastError());
    XDG_TRY_HIP(hipDeviceSynchronize());
    b->n_rwords = n_words;
    b->rank = L;
    if (b->plan.kind == K_SUB) {
        W first = 0;
        XDG_RETURN_IF(copy_d2h(&first, b->reps.as<W>(), sizeof(W), nullptr));
        XDG_RETURN_IF(build_xr<W>(b, T, L, first, (W)last));
    }
    return XDG_OK;
}

int build_lin(xdg_basis_s *b) {
    // index(s) = L_hi[hi] + L_lo[lo]: L_lo = colex rank of lo among the
    // lo' with the same popcount, L_hi[hi] = number of basis states whose
    // high part is smaller than hi (Lin's two-table scheme, Sec. 5.2).
    const int N = b->n_sites, n = b->n_up;
    const int nlo = N / 2, nhi = N - nlo;
    std::vector<uint32_t> t((size_t)1 << nlo | 0, 0);
    t.assign(((size_t)1 << nlo) + ((size_t)1 << nhi), 0);
    for (uint64_t lo = 0; lo < (1ull << nlo); ++lo) {
        uint64_t r = 0;
        int k = 0;
        for (int p = 0; p < nlo; ++p)
            if ((lo >> p) & 1) {
                r += binomial(p, k + 1);
                ++k;
            }
        t[lo] = (uint32_t)r;
    }
    uint64_t acc = 0;
    for (uint64_t hi = 0; hi < (1ull << nhi); ++hi) {
        t[((size_t)1 << nlo) + hi] = (uint32_t)acc;
        const int rest = n - __builtin_popcountll(hi);
        if (rest >= 0 && rest <= nlo) acc += binomial(nlo, rest);
    }
    b->lin_nlo = nlo;
    b->lin_nhi = nhi;
    return b->lin.upload(t.data(), t.size() * sizeof(uint32_t));
}

}  // namespace

int basis_build_device(xdg_basis_s *b) {
    std::vector<uint64_t> bt(65 * 65);
    for (int a = 0; a <= 64; ++a)
        for (int c = 0; c <= 64; ++c) bt[a * 65 + c] = binomial(a, c);
    DevBuf binom_d;
    XDG_RETURN_IF(binom_d.upload(bt.data(), bt.size() * 8));

    const Plan &P = b->plan;
    if (b->n_sym) {
        XDG_RETURN_IF(b->chi_d.upload(b->chi.data(), b->chi.size() * sizeof(double)));
        b->chi_trivial = true;
        for (int g = 0; g < b->n_sym; ++g)
            b->chi_trivial &= b->chi[2 * g] == 1.0 && b->chi[2 * g + 1] == 0.0;
        std::vector<float> cf(b->chi.begin(), b->chi.end());
        XDG_RETURN_IF(b->chi_f.upload(cf.data(), cf.size() * sizeof(float)));
        std::vector<double> sq(2 * (b->n_sym + 1));
        std::vector<float> sqf(2 * (b->n_sym + 1));
        for (int c = 0; c <= b->n_sym; ++c) {
            sq[c] = c ? std::sqrt((double)c) : 0.0;
            sq[b->n_sym + 1 + c] = c ? 1.0 / std::sqrt((double)c) : 0.0;
            sqf[c] = (float)sq[c];
            sqf[b->n_sym + 1 + c] = (float)sq[b->n_sym + 1 + c];
        }
        XDG_RETURN_IF(b->sqrt_d.upload(sq.data(), sq.size() * sizeof(double)));
        XDG_RETURN_IF(b->sqrt_f.upload(sqf.data(), sqf.size() * sizeof(float)));
    }
    if (P.kind == K_AFF) {
        XDG_RETURN_IF(b->t_aff.upload(P.aff.data(), P.aff.size() * sizeof(AffineElem)));
        if (P.ring)
            XDG_RETURN_IF(b->t_ring.upload(P.ring_gidx.data(), P.ring_gidx.size() * 2));
    }
    if (P.kind == K_SUB) {
        // device form, one word per (element, block): the offset of the block
        // permutation's tables in tperm, shifted left by 8, or'ed with the
        // first bit of the source block
        const uint64_t E = 1ull << P.sub.pb;
        std::vector<uint32_t> sp(P.sub.pid.size());
        for (size_t e = 0; e < sp.size(); ++e) {
            const uint64_t to = (uint64_t)P.sub.pid[e] * 2u * E;
            const uint32_t so = (uint32_t)(P.sub.src[e] * P.sub.m);
            if (to >= (1ull << 24) || so > 255u) {
                set_error("sublattice tables too large for their packed offsets");
                return XDG_EINVAL;
            }
            sp[e] = (uint32_t)(to << 8) | so;
        }
        XDG_RETURN_IF(b->t_pid.upload(sp.data(), sp.size() * 4));
        XDG_RETURN_IF(b->t_tperm.upload(P.sub.tperm.data(), P.sub.tperm.size() * 2));
        XDG_RETURN_IF(b->t_mintop.upload(P.sub.mintop.data(), P.sub.mintop.size() * 2));
        XDG_RETURN_IF(b->t_candoff.upload(P.sub.cand_off.data(), P.sub.cand_off.size() * 4));
        XDG_RETURN_IF(b->t_candlist.upload(P.sub.cand_list.data(),
                                           std::max<size_t>(2, P.sub.cand_list.size() * 2)));
    }
    if (P.kind == K_TAB)
        XDG_RETURN_IF(b->t_bytes.upload(P.bytes.tab.data(), P.bytes.tab.size() * 8));

    if (b->wide) {
        XDG_RETURN_IF(enumerate<uint64_t>(b, binom_d));
    } else {
        XDG_RETURN_IF(enumerate<uint32_t>(b, binom_d));
    }
    if (P.kind == K_U1) {
        XDG_RETURN_IF(build_lin(b));
    } else if (b->dim > 0) {
        if (b->wide) {
            XDG_RETURN_IF(build_rank<uint64_t>(b));
            if (!b->n_rwords) XDG_RETURN_IF(build_hash<uint64_t>(b));
        } else {
            XDG_RETURN_IF(build_rank<uint32_t>(b));
            if (!b->n_rwords) XDG_RETURN_IF(build_hash<uint32_t>(b));
        }
    }
    return XDG_OK;
}

int basis_lookup(xdg_basis_s *b, const uint64_t *d_states, int64_t n, int64_t *d_idx,
                 hipStream_t st) {
    if (n <= 0) return XDG_OK;
    const int block = 256;
    const unsigned grid = (unsigned)((n + block - 1) / block);
    const int u1 = b->plan.kind == K_U1;
    const RankArgs R{b->rwords.as<uint2>(), b->n_rwords, b->rtab.p, b->rank};
    if (b->wide) {
        const uint64_t empty = b->n_up == b->n_sites ? 0ull : ~0ull;
        hipLaunchKernelGGL(k_lookup<uint64_t>, dim3(grid), dim3(block), 0, st, d_states, n, d_idx,
                           b->n_sites, b->n_up, u1, b->lin.as<uint32_t>(), b->lin_nlo, b->hash.p,
                           b->dim > 0 ? b->hidx.n_lines : 0, empty, R);
    } else {
        const uint32_t empty = b->n_up == b->n_sites ? 0u : ~0u;
        hipLaunchKernelGGL(k_lookup<uint32_t>, dim3(grid), dim3(block), 0, st, d_states, n, d_idx,
                           b->n_sites, b->n_up, u1, b->lin.as<uint32_t>(), b->lin_nlo, b->hash.p,
                           b->dim > 0 ? b->hidx.n_lines : 0, empty, R);
    }
    XDG_TRY_HIP(hipGetLastError());
    return XDG_OK;
}

}  // namespace xdg
