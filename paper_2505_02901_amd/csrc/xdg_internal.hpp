// Internal declarations of the MI355X library behind include/xdg.h.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "xdg.h"

namespace xdg {

// ---------------------------------------------------------------- errors --
void set_error(const char *fmt, ...);
const char *get_error();

#define XDG_TRY_HIP(expr)                                                          \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::xdg::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                  \
            return e_ == hipErrorOutOfMemory ? XDG_ENOMEM : XDG_EHIP;              \
        }                                                                          \
    } while (0)

#define XDG_RETURN_IF(err)        \
    do {                          \
        int r_ = (err);           \
        if (r_ != XDG_OK) return r_; \
    } while (0)

// Device allocation that owns its memory.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release();
    int alloc(size_t n);                      // XDG_OK / XDG_ENOMEM
    int upload(const void *host, size_t n);   // alloc + copy
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ------------------------------------------------------- search tables --
// Sublattice-coding tables (built on the host, uploaded once).
//   sites are blocks of m bits, block q = bits [q m, (q+1) m); top = n_s - 1.
//   src[g][a]      : block of t feeding block a of g.t
//   pid[g][a]      : which of the distinct block permutations maps it
//   tperm[p][h][u] : image bits of the half h (bits [h pb, (h+1) pb)) of a
//                    source chunk with value u under permutation p; the
//                    image chunk of v is tperm[p][0][v & lo] | tperm[p][1][v >> pb]
//   mintop[k][v]   : min over g with src[g][top] = k of the image of v
//   cand_off[k][v] : offsets into cand_list (size n_s*(2^m)+1)
//   cand_list      : group elements reaching mintop[k][v], ascending
struct SublatticeTables {
    int n_s = 0, m = 0, pb = 0, n_perm = 0;
    std::vector<uint8_t> src;        // [n_sym][n_s]
    std::vector<uint16_t> pid;       // [n_sym][n_s]
    std::vector<uint16_t> tperm;     // [n_perm][2][2^pb]
    std::vector<uint16_t> mintop;    // [n_s][2^m]
    std::vector<uint32_t> cand_off;  // [n_s * 2^m + 1]
    std::vector<uint16_t> cand_list; // [cand_off.back()]
};

// Generic byte tables: tab[g][c][v] = image bits of byte c of t having value v.
struct ByteTables {
    int n_chunks = 0;
    std::vector<uint64_t> tab;       // [n_sym][n_chunks][256]
};

// Affine (ring) elements: g(i) = (eps*i + a) mod N.
struct AffineElem {
    int32_t a;
    int32_t eps;
};

struct Plan {
    int kind = XDG_SEARCH_U1;
    SublatticeTables sub;
    ByteTables bytes;
    std::vector<AffineElem> aff;
    // affine groups holding every rotation (ring = 1) and also every
    // reflection (ring = 2): group index of rotation a at [a], of the
    // reflection with image rotr_N(rev_N(t), a) at [N + a]
    int ring = 0;
    std::vector<int16_t> ring_gidx;
    int flags = 0;   // XDG_FLAG_*
};

// The library's device memory: a caller-set limit on what its buffers may
// hold together (0 = none), and what they hold now.
void set_device_memory_limit(uint64_t bytes);
uint64_t device_memory_in_use();

// Transfers between host memory and the device through a page-locked
// staging buffer, complete on return.
int copy_d2h(void *dst, const void *src, size_t n, hipStream_t st);
int copy_h2d(void *dst, const void *src, size_t n, hipStream_t st);

int validate_group(int n_sites, int n_sym, const int32_t *perm, const double *chi);
int validate_bonds(int n_sites, int n_sym, const int32_t *perm, int n_bonds, const int32_t *sites,
                   const double *jz, const double *jxy);
int make_plan(int n_sites, int n_sym, const int32_t *perm, const xdg_basis_opts *opts, Plan *plan,
              bool build_tables);
uint64_t binomial(int n, int k);

// ---------------------------------------------------------------- basis --
struct DeviceSearch {
    // device copies of the search tables (pointers into DevBufs of the basis)
    const uint8_t *src = nullptr;
    const uint16_t *img = nullptr;
    const uint16_t *mintop = nullptr;
    const uint32_t *cand_off = nullptr;
    const uint16_t *cand_list = nullptr;
    const uint64_t *bytetab = nullptr;
    const AffineElem *aff = nullptr;
    int n_s = 0, m = 0, n_chunks = 0;
    uint32_t lds_sub_bytes = 0;   // bytes of mintop + cand_off + cand_list staged in LDS
};

// Layout of the colex-rank chunk tables of a block (see colex_rank).
constexpr int RANK_MAXC = 16;   // chunks of a wide state (cb >= 4 for N <= 64)
struct RankLayout {
    int cb, nc;
    int e32;                 // wide states: saturating 4-byte entries
    int rows;                // rows of the whole table
    int rbase[RANK_MAXC];    // chunk k, below b: row rbase[k] + b
};

struct HashIndex {
    uint64_t n_lines = 0;   // 64-byte lines
    int slots = 0;          // 8 (32-bit keys) or 5 (64-bit keys)
};

}  // namespace xdg

struct xdg_basis_s {
    std::atomic<int> refs{1};
    int device = 0;
    int n_sites = 0, n_up = 0, n_sym = 0;
    bool wide = false;          // 64-bit state words (n_sites > 32)
    bool is_complex = false;
    bool chi_trivial = false;   // every character is exactly 1
    int64_t dim = 0;
    std::vector<int32_t> perm;  // [n_sym][n_sites]
    std::vector<double> chi;    // [n_sym][2]
    xdg::Plan plan;
    // device data
    xdg::DevBuf reps;           // u32/u64 [dim]
    xdg::DevBuf stab;           // u16 [dim]  |Stab(s)|
    xdg::DevBuf hash;           // 64-byte lines
    xdg::HashIndex hidx;
    xdg::DevBuf lin;            // u32 [2^nlo + 2^nhi] Lin tables (U(1))
    // rank index (symmetric blocks): uint2 {count, bits} per 32 colex ranks,
    // and the chunk tables of the colex rank (u64 [nc][n_up + 1][2^cb])
    xdg::DevBuf rwords;
    uint64_t n_rwords = 0;      // 0: the hash index is used
    xdg::DevBuf rtab;
    xdg::RankLayout rank{};     // layout of rtab (chunks, entry size, row bases)
    // rank-addressed vectors (sublattice coding, see top_rank): first rank of
    // each top block (u64 [2^m], ~0 for a block that is never a minimal top),
    // the slots up to the last basis state and the sites below the top block
    xdg::DevBuf xr_top, xr_top32;   // xr_top32: u32 copy when every first rank fits
    xdg::DevBuf xr_rtab;        // u32 rows of the rank tables for the chunks below the top block
    uint64_t xr_slots = 0;      // 0: not available
    int xr_bits = 0;
    int xr_rows = 0;            // rows of xr_rtab
    int lin_nlo = 0, lin_nhi = 0;
    // sublattice tables on the device: t_pid = u32 [n_sym][n_s], the offset of
    // the block permutation's tables in t_tperm << 8 | first bit of the source block
    xdg::DevBuf t_pid, t_tperm, t_mintop, t_candoff, t_candlist, t_bytes, t_aff, t_ring;
    xdg::DevBuf chi_d;          // double2 [n_sym]
    xdg::DevBuf chi_f;          // float2 [n_sym]
    xdg::DevBuf sqrt_d;         // double [n_sym+1] sqrt(c), then [n_sym+1] 1/sqrt(c)
    xdg::DevBuf sqrt_f;         // float, same layout
    xdg::DeviceSearch dsearch;
};

namespace xdg {
struct TuneKey {
    int dtype;
    int64_t nvec;
    bool operator<(const TuneKey &o) const {
        return std::tie(dtype, nvec) < std::tie(o.dtype, o.nvec);
    }
};
struct LaunchCfg {
    int block = 256;       // threads per workgroup
    int grid = 0;          // workgroups (persistent grid); 0 = one row per lane
    int nv = 1;            // vectors per pass (<= nvec)
    int occ = -1;          // 64-VGPR copy at 8 waves per SIMD: 1 / 0 / -1 = when the LDS allows
    int compact = -1;      // table searches: 1 = wave-compacted term loop, 0 / -1 = row loop
    int sub_form = 0;      // sublattice coding: 0 = packed form where it applies, 2 = block form
    int xr = 0;            // sublattice coding: 1 = terms read a rank-addressed copy of x
};
}  // namespace xdg

struct xdg_ham_s {
    xdg_basis_s *basis = nullptr;
    uint64_t serial = 0;        // unique per created Hamiltonian (cache keys)
    int n_bonds = 0;
    std::vector<int32_t> sites;
    std::vector<double> jz, jxy;
    xdg::DevBuf bonds_d;        // BondD [n_bonds]
    xdg::DevBuf bonds_f;        // BondF [n_bonds]
    xdg::DevBuf bonds_x;        // BondX [n_bonds] (packed sublattice search only)
    int64_t nnz = -1;
    std::mutex tune_mu;         // guards `tuned` (and the tuning runs that fill it)
    std::map<xdg::TuneKey, xdg::LaunchCfg> tuned;
    // the rank-addressed copy of x (LaunchCfg::xr): slot bytes of its current
    // layout (slots outside the block hold zeros in it), and an event after
    // the last launch that read it (calls on other streams wait for it)
    std::mutex xr_mu;
    xdg::DevBuf xr_buf;
    size_t xr_slot_bytes = 0;
    hipEvent_t xr_ev = nullptr;
    ~xdg_ham_s() {
        if (xr_ev) (void)hipEventDestroy(xr_ev);
    }
};

namespace xdg {

struct BondD {
    uint32_t i, j;
    double jz, h;   // h = jxy / 2
};
struct BondF {
    uint32_t i, j;
    float jz, h;
};

// The packed form of the sublattice search applies to four blocks of at most
// 10 sites whose half-chunk tables have 2^pb entries, 3 <= pb <= 5.
__host__ __device__ constexpr bool sub_packed_ok(int n_s, int m, int pb) {
    return n_s == 4 && m <= 10 && pb >= 3 && pb <= 5 && m - pb <= pb;
}

// Per-bond data of the packed sublattice search, in device bond order, read
// with scalar loads: the two sites as a mask, and the bits that exchanging
// them flips in a state's packed words and in its four block-table indices.
struct BondX {
    uint64_t flip;
    uint32_t plo, phi;
    uint32_t ek[4];
};
// site i's share of those bits (block q = i / m, position p = i mod m)
inline void bondx_site(int i, int m, int pb, BondX &x) {
    const int q = i / m, p = i - q * m;
    x.flip |= 1ull << i;
    x.ek[q] |= 1u << p;
    if (p < pb)
        x.plo |= 1u << (7 * q + 1 + p);
    else
        x.phi |= 1u << (7 * q + 1 + p - pb);
}

int basis_build_device(xdg_basis_s *b);                 // enumerate + index
int basis_lookup(xdg_basis_s *b, const uint64_t *d_states, int64_t n, int64_t *d_idx,
                 hipStream_t st);
int ham_count_nnz(xdg_ham_s *h, int64_t *nnz);

int apply_launch(xdg_ham_s *h, const void *x, void *y, int64_t nvec, int dtype, hipStream_t st,
                 const LaunchCfg *cfg);
int apply_tuned(xdg_ham_s *h, const void *x, void *y, int64_t nvec, int dtype, hipStream_t st);
int apply_tuned_config(xdg_ham_s *h, int dtype, int64_t nvec, LaunchCfg *out);
int apply_batched_launch(int n, xdg_ham_s *const *hams, const void *const *xs, void *const *ys,
                         int64_t nvec, int dtype, hipStream_t st, uint32_t *d_queue,
                         int grid, int block);
// Shape of a batched persistent launch (host side, no device memory).
struct BatchMeta {
    int n = 0, kind = 0;
    bool wide = false, single = false, cplx = false, acc64 = true, tsingle = false;
    int64_t cols = 0;
    uint32_t n_tiles = 0, tile_rows = 0;
    size_t lds = 0;
    int stage_sub = 1;
};
// Batched persistent launch plan: device copies of the sector descriptors
// and the cumulative tile counts; the queue counter is zeroed by a kernel
// (not a memset) so that the launch can be captured into a graph.
struct BatchPlan : BatchMeta {
    DevBuf descs, prefix, queue;
};
struct SectorDesc;
// Host planning of a batch: fills M, and (when not null) descs[n] and
// prefix[n + 1] in host memory.  Allocates nothing.
int batch_plan_host(int n, xdg_ham_s *const *hams, const void *const *xs, void *const *ys,
                    int64_t nvec, int dtype, BatchMeta *M, SectorDesc *descs, uint32_t *prefix,
                    uint32_t tile_rows = 0);
int batch_prepare(int n, xdg_ham_s *const *hams, const void *const *xs, void *const *ys,
                  int64_t nvec, int dtype, BatchPlan *P, uint32_t tile_rows = 0);
int batch_launch(const BatchPlan &P, int grid, int nv_cap, hipStream_t st);
// The launch itself on device descriptors, tile prefix and queue counter.
int batch_launch_raw(const BatchMeta &M, const SectorDesc *d_descs, const uint32_t *d_prefix,
                     uint32_t *d_queue, int grid, int nv_cap, hipStream_t st);
int apply_batched_noalloc(int n, xdg_ham_s *const *hams, const void *const *xs,
                          void *const *ys, int64_t nvec, int dtype, hipStream_t st);
// Launch shape of a batched apply: persistent grid, rows per work item,
// vectors per pass.
struct BatchShape {
    int grid = 0;
    uint32_t tile = 4096;
    int nv = 8;
};
// The shape for this set of blocks (nvec, dtype): tuned on the first call by
// timing launches on xs -> ys (which it overwrites) and cached; locked.
int batch_shape_tuned(int n, xdg_ham_s *const *hams, const void *const *xs, void *const *ys,
                      int64_t nvec, int dtype, hipStream_t st, BatchShape *out);
// The cached shape, if any (no tuning, no allocation); false otherwise.
bool batch_shape_cached(int n, xdg_ham_s *const *hams, int64_t nvec, int dtype, BatchShape *out);
int lanczos_single(xdg_ham_s *h, const void *v0, int k, double tol, int max_iter, uint64_t seed,
                   int prec, double *evals, int *n_iter, double *alpha, double *beta,
                   hipStream_t st, double *t_total, double *t_apply);
int lanczos_batched(int n, xdg_ham_s *const *hams, const void *const *v0s, int64_t nvec,
                    int n_iter, uint64_t seed, int prec, double *evals, double *alpha,
                    double *beta, hipStream_t st, double *t_total, double *t_apply);
int tpq_micro(xdg_ham_s *h, const void *v0, uint64_t seed, int prec, double l, int n_steps,
              double *u, double *u2, hipStream_t st);
int tpq_micro_batched(int n, xdg_ham_s *const *hams, const void *const *v0s, int64_t nvec,
                      uint64_t seed, int prec, double l, int n_steps, double *u, double *u2,
                      hipStream_t st);
int tpq_thermo(int n_rec, int n_steps, const double *u, const double *u2, double l, int n_sites,
               const double *weight, int n_temp, const double *temps, double *energy,
               double *heat, double *log_z);
void tridiag_eigenvalues(int m, const double *alpha, const double *beta, std::vector<double> &out);
void tridiag_spectral_weights(int m, const double *alpha, const double *beta,
                              std::vector<double> &evals, std::vector<double> &weights);
int spectral_cf(int m, const double *alpha, const double *beta, double norm2, double e0,
                int n_w, const double *omega, double eta, double *out);
int apply_diag_transfer(xdg_basis_s *bin, xdg_basis_s *bout, const double *coef, const void *x,
                        void *y, int dtype, hipStream_t st);
int ftlm_thermo(int n_rec, int m, const double *alpha, const double *beta, const double *weight,
                int n_temp, const double *temps, double *energy, double *heat, double *log_z);
void tridiag_eigvec(int m, const double *alpha, const double *beta, int which,
                    std::vector<double> &x, double &theta);
int lanczos_eigvec(xdg_ham_s *h, const void *v0, uint64_t seed, int prec, int m,
                   const double *alpha, const double *beta, int which, void *psi, double *ritz,
                   hipStream_t st);
int expect_szsz(xdg_basis_s *b, const void *psi, int dtype, int n_pairs, const int32_t *pairs,
                double *out, hipStream_t st);

int random_fill(int64_t n_scalars, uint64_t seed, int kind, bool single, void *out,
                hipStream_t st);
int device_cu_count();
int apply_grid_for(int mult);

size_t dtype_size(int dtype);
bool dtype_complex(int dtype);
bool dtype_single(int dtype);

}  // namespace xdg
