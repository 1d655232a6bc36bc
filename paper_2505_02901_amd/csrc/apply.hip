// Host side of the matrix-free application: sector descriptors, launch
// shapes, the autotuner, the batched persistent launch and nnz counting.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "apply_impl.hpp"

namespace xdg {

size_t lds_limit();

// dynamic LDS available to the apply kernels: the device limit minus the
// static shared data (sector descriptor, tile counter)
static size_t lds_budget() {
    const size_t stat = sizeof(SectorDesc) + 64;
    return lds_limit() > stat ? lds_limit() - stat : 0;
}

// two workgroups of the apply kernel fit in one CU's LDS: run the variant
// limited to 64 VGPRs (8 waves per SIMD)
static int occ_for(size_t lds) {
    const size_t stat = sizeof(SectorDesc) + 64;
    return 2 * (lds + stat) <= lds_limit() ? 1 : 0;
}

size_t dtype_size(int dtype) {
    switch (dtype) {
        case XDG_F64: return 8;
        case XDG_F32: return 4;
        case XDG_C128: return 16;
        case XDG_C64: return 8;
    }
    return 0;
}
bool dtype_complex(int dtype) { return dtype == XDG_C128 || dtype == XDG_C64; }
bool dtype_single(int dtype) { return dtype == XDG_F32 || dtype == XDG_C64; }

// persistent apply grid of `mult` 1024-lane equivalents per compute unit
int apply_grid_for(int mult) { return device_cu_count() * mult * BLOCKS_PER_1024; }

namespace {

int launch_dispatch(int kind, bool wide, bool single, bool acc64, bool cplx, int nv,
                    const ApplyArgs &A, unsigned grid, unsigned block, size_t lds, hipStream_t st) {
    switch (kind) {
        case K_U1:
            return launch_kind<K_U1>(wide, single, acc64, cplx, nv, A, grid, block, lds, st);
        case K_AFF:
            return launch_kind<K_AFF>(wide, single, acc64, cplx, nv, A, grid, block, lds, st);
        case K_SUB:
            return launch_kind<K_SUB>(wide, single, acc64, cplx, nv, A, grid, block, lds, st);
        case K_TAB:
            return launch_kind<K_TAB>(wide, single, acc64, cplx, nv, A, grid, block, lds, st);
    }
    set_error("unknown search kind %d", kind);
    return XDG_EINVAL;
}

SectorDesc make_desc(const xdg_ham_s *h, bool single, const void *x, void *y) {
    const xdg_basis_s *b = h->basis;
    SectorDesc d{};
    d.reps = b->reps.p;
    d.stab = b->stab.as<uint16_t>();
    d.dim = b->dim;
    d.hash = b->hash.p;
    d.n_lines = b->hidx.n_lines;
    d.empty = b->wide ? (b->n_up == b->n_sites ? 0ull : ~0ull)
                      : (b->n_up == b->n_sites ? 0ull : 0xFFFFFFFFull);
    d.lin = b->lin.as<uint32_t>();
    d.nlo = b->lin_nlo;
    d.rwords = b->n_rwords ? b->rwords.as<uint2>() : nullptr;
    d.n_rwords = b->n_rwords;
    d.rtab = b->rtab.p;
    d.rl = b->rank;
    d.n_up = b->n_up;
    d.n_sites = b->n_sites;
    d.n_sym = b->n_sym;
    d.n_bonds = h->n_bonds;
    d.aff = b->t_aff.as<AffineElem>();
    d.ring = b->plan.ring;
    d.ring_gidx = b->t_ring.as<int16_t>();
    d.bytetab = b->t_bytes.as<uint64_t>();
    d.n_bchunks = b->plan.bytes.n_chunks;
    d.mintop = b->t_mintop.as<uint16_t>();
    d.cand_off = b->t_candoff.as<uint32_t>();
    d.cand_list = b->t_candlist.as<uint16_t>();
    d.sp = b->t_pid.as<uint32_t>();
    d.tperm = b->t_tperm.as<uint16_t>();
    d.n_s = b->plan.sub.n_s;
    d.m = b->plan.sub.m;
    d.pb = b->plan.sub.pb;
    d.n_perm = b->plan.sub.n_perm;
    d.n_cand = (uint32_t)b->plan.sub.cand_list.size();
    d.subf = b->plan.kind == K_SUB && sub_packed_ok(d.n_s, d.m, d.pb) && h->bonds_x.p;
    d.bx = d.subf ? h->bonds_x.as<BondX>() : nullptr;
    d.bonds = single ? h->bonds_f.p : h->bonds_d.p;
    d.chi = single ? b->chi_f.p : b->chi_d.p;
    d.sqrtt = single ? b->sqrt_f.p : b->sqrt_d.p;
    double jq = 0.0;
    for (double j : h->jz) jq += 0.25 * j;
    d.jz_quarter = jq;
    d.ring_bonds = h->n_bonds == b->n_sites;
    for (int i = 0; i < h->n_bonds && d.ring_bonds; ++i) {
        const int p = h->sites[2 * i], q = h->sites[2 * i + 1], r = (i + 1) % b->n_sites;
        d.ring_bonds = (p == i && q == r) || (p == r && q == i);
    }
    d.x = x;
    d.y = y;
    return d;
}

// Real-valued kernels serve complex vectors on a real block: the real and
// imaginary parts are independent columns of a [dim][2 nvec] real block.
struct Form {
    bool single, cplx_kernel;
    bool acc64;     // FP64 amplitudes and row accumulation
    bool tsingle;   // FP32 amplitude tables (single && !acc64)
    int64_t cols;   // columns seen by the kernel
};

int form_of(const xdg_basis_s *b, int dtype, int64_t nvec, Form *f) {
    if (dtype < XDG_F64 || dtype > XDG_C64) {
        set_error("unknown dtype %d", dtype);
        return XDG_EINVAL;
    }
    if (nvec < 1) {
        set_error("nvec = %lld must be >= 1", (long long)nvec);
        return XDG_EINVAL;
    }
    if (b->is_complex && !dtype_complex(dtype)) {
        set_error("the block (dimension %lld, %d group elements) has complex characters: "
                  "vectors must be XDG_C128 or XDG_C64 (got dtype %d)",
                  (long long)b->dim, b->n_sym, dtype);
        return XDG_EINVAL;
    }
    f->single = dtype_single(dtype);
    f->cplx_kernel = b->is_complex;
    f->acc64 = !f->single || !(b->plan.flags & XDG_FLAG_F32_ACCUMULATE);
    f->tsingle = f->single && !f->acc64;
    f->cols = (dtype_complex(dtype) && !b->is_complex) ? 2 * nvec : nvec;
    return XDG_OK;
}

// Rank-addressed x: row i of x goes to slot top_rank(reps[i]) of xr (spr
// scalars per row); the other slots hold zeros.
template <class W, class T>
__global__ __launch_bounds__(256) void k_xr_scatter(const W *reps, int64_t dim, int spr,
                                                   const T *x, T *xr, const uint32_t *rtab,
                                                   RankLayout L, int B, const uint64_t *top,
                                                   uint64_t slots) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < dim; i += stride) {
        const uint64_t r = top_rank<W>(rtab, L, B, top, reps[i]);
        if (r >= slots) continue;   // never for a basis state
        for (int c = 0; c < spr; ++c) xr[r * spr + c] = x[i * spr + c];
    }
}

__global__ __launch_bounds__(256) void k_zero32(uint32_t *p, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

// Fill the rank-addressed copy of x for this call (caller holds h->xr_mu):
// wait for the last launch that read it, (re)allocate and zero it when the
// layout changes (not under graph capture), then scatter x.
int xr_prepare(xdg_ham_s *h, const void *x, const Form &f, hipStream_t st, bool *capturing) {
    const xdg_basis_s *b = h->basis;
    const int spr = (int)f.cols * (f.cplx_kernel ? 2 : 1);
    const size_t tsz = f.single ? 4 : 8;
    const size_t slot_bytes = (size_t)spr * tsz;
    const size_t need = (size_t)b->xr_slots * slot_bytes;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    XDG_TRY_HIP(hipStreamIsCapturing(st, &cs));
    *capturing = cs != hipStreamCaptureStatusNone;
    if (!h->xr_ev) XDG_TRY_HIP(hipEventCreateWithFlags(&h->xr_ev, hipEventDisableTiming));
    if (!*capturing) XDG_TRY_HIP(hipStreamWaitEvent(st, h->xr_ev, 0));
    const int gcap = device_cu_count() * 32;
    if (h->xr_buf.bytes < need || h->xr_slot_bytes != slot_bytes) {
        if (*capturing) {
            set_error("the rank-addressed copy of x is set up by a first call outside graph capture");
            return XDG_EINVAL;
        }
        if (h->xr_buf.bytes < need) {
            h->xr_slot_bytes = 0;
            h->xr_buf.release();   // waits for the device
            XDG_RETURN_IF(h->xr_buf.alloc(need));
        }
        const uint64_t nw = need / 4;
        const unsigned g = (unsigned)std::min<uint64_t>((nw + 255) / 256, (uint64_t)gcap);
        hipLaunchKernelGGL(k_zero32, dim3(std::max(1u, g)), dim3(256), 0, st,
                           h->xr_buf.as<uint32_t>(), nw);
        XDG_TRY_HIP(hipGetLastError());
        h->xr_slot_bytes = slot_bytes;
    }
    const unsigned g =
        (unsigned)std::min<int64_t>((b->dim + 255) / 256, (int64_t)gcap);
    const uint64_t *top = b->xr_top.as<uint64_t>();
    if (b->wide) {
        if (f.single)
            hipLaunchKernelGGL((k_xr_scatter<uint64_t, float>), dim3(g), dim3(256), 0, st,
                               b->reps.as<uint64_t>(), b->dim, spr, (const float *)x,
                               h->xr_buf.as<float>(), b->xr_rtab.as<uint32_t>(), b->rank, b->xr_bits, top,
                               b->xr_slots);
        else
            hipLaunchKernelGGL((k_xr_scatter<uint64_t, double>), dim3(g), dim3(256), 0, st,
                               b->reps.as<uint64_t>(), b->dim, spr, (const double *)x,
                               h->xr_buf.as<double>(), b->xr_rtab.as<uint32_t>(), b->rank, b->xr_bits, top,
                               b->xr_slots);
    } else {
        if (f.single)
            hipLaunchKernelGGL((k_xr_scatter<uint32_t, float>), dim3(g), dim3(256), 0, st,
                               b->reps.as<uint32_t>(), b->dim, spr, (const float *)x,
                               h->xr_buf.as<float>(), b->xr_rtab.as<uint32_t>(), b->rank, b->xr_bits, top,
                               b->xr_slots);
        else
            hipLaunchKernelGGL((k_xr_scatter<uint32_t, double>), dim3(g), dim3(256), 0, st,
                               b->reps.as<uint32_t>(), b->dim, spr, (const double *)x,
                               h->xr_buf.as<double>(), b->xr_rtab.as<uint32_t>(), b->rank, b->xr_bits, top,
                               b->xr_slots);
    }
    XDG_TRY_HIP(hipGetLastError());
    return XDG_OK;
}

int pick_nv(int64_t remaining, int cap) {
    int nv = 8;
    while (nv > 1 && (nv > remaining || nv > cap)) nv >>= 1;
    return nv;
}

}  // namespace

// LDS bytes the apply kernel stages for this form, whether the sublattice
// tables fit with them, and whether two workgroups fit one compute unit
void apply_lds(const xdg_ham_s *h, int dtype, size_t *lds, int *stage_sub, int *occ_ok) {
    const xdg_basis_s *b = h->basis;
    const bool tsingle = dtype_single(dtype) && (b->plan.flags & XDG_FLAG_F32_ACCUMULATE);
    const SectorDesc d = make_desc(h, tsingle, nullptr, nullptr);
    size_t n = tsingle ? stage_bytes<float>(d, b->plan.kind, 1)
                       : stage_bytes<double>(d, b->plan.kind, 1);
    int st = 1;
    if (n > lds_budget()) {
        st = 0;
        n = tsingle ? stage_bytes<float>(d, b->plan.kind, 0) : stage_bytes<double>(d, b->plan.kind, 0);
    }
    *lds = n;
    *stage_sub = st;
    *occ_ok = st ? occ_for(n) : 0;
}

int apply_launch(xdg_ham_s *h, const void *x, void *y, int64_t nvec, int dtype, hipStream_t st,
                 const LaunchCfg *cfg) {
    const xdg_basis_s *b = h->basis;
    Form f;
    XDG_RETURN_IF(form_of(b, dtype, nvec, &f));
    if (b->dim == 0) return XDG_OK;
    if (!x || !y || x == y) {
        set_error("x and y must be distinct non-null device pointers");
        return XDG_EINVAL;
    }
    LaunchCfg c = cfg ? *cfg : LaunchCfg{};
    const unsigned block = APPLY_BLOCK;
    const int64_t need = (b->dim + block - 1) / block;
    const int64_t gmax = c.grid > 0 ? c.grid : (int64_t)apply_grid_for(2);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(need, gmax));
    ApplyArgs A{};
    A.one = make_desc(h, f.tsingle, x, y);
    if (c.sub_form == 2) {
        A.one.subf = 0;
        A.one.bx = nullptr;
    }
    // rank-addressed x: when its tables fit in LDS with the others
    bool xr_on = c.xr && b->xr_slots && b->plan.kind == K_SUB, capturing = false;
    if (xr_on) {
        A.one.xr = b->xr_top.p;   // the copy is set below; non-null for the LDS size
        A.one.xr_top = b->xr_top.as<uint64_t>();
        A.one.xr_top32 = b->xr_top32.as<uint32_t>();
        A.one.xr_slots = b->xr_slots;
        A.one.xr_bits = b->xr_bits;
        A.one.xr_rows = b->xr_rows;
        A.one.xr_rtab = b->xr_rtab.as<uint32_t>();
        const size_t lx = f.tsingle ? stage_bytes<float>(A.one, b->plan.kind, 1)
                                    : stage_bytes<double>(A.one, b->plan.kind, 1);
        if (lx > lds_budget()) {
            xr_on = false;
            A.one.xr = nullptr;
            A.one.xr_top = nullptr;
            A.one.xr_top32 = nullptr;
        }
    }
    std::unique_lock<std::mutex> xr_lock;
    if (xr_on) {
        xr_lock = std::unique_lock<std::mutex>(h->xr_mu);
        XDG_RETURN_IF(xr_prepare(h, x, f, st, &capturing));
        A.one.xr = h->xr_buf.p;
    }
    A.nvec = f.cols;
    size_t lds = f.tsingle ? stage_bytes<float>(A.one, b->plan.kind, 1)
                           : stage_bytes<double>(A.one, b->plan.kind, 1);
    A.stage_sub = 1;
    if (lds > lds_budget()) {
        A.stage_sub = 0;
        lds = f.tsingle ? stage_bytes<float>(A.one, b->plan.kind, 0)
                        : stage_bytes<double>(A.one, b->plan.kind, 0);
    }
    A.occ = A.stage_sub ? (c.occ >= 0 ? (c.occ && occ_for(lds)) : occ_for(lds)) : 0;
    A.compact = c.compact > 0 && !xr_on ? 1 : 0;   // the compacted loop reads x itself
    const int cap = std::min(c.nv > 0 ? c.nv : 8, xr_on ? 2 : 8);
    for (int64_t v0 = 0; v0 < f.cols;) {
        const int nv = pick_nv(f.cols - v0, cap);
        A.v0 = (int)v0;
        if (xr_on && b->chi_trivial && !f.cplx_kernel)
            XDG_RETURN_IF(launch_sub_xr_trivial(b->wide, f.single, f.acc64, nv, A, grid, block,
                                                lds, st));
        else if (xr_on)
            XDG_RETURN_IF(launch_sub_xr(b->wide, f.single, f.acc64, f.cplx_kernel, nv, A, grid,
                                        block, lds, st));
        else
            XDG_RETURN_IF(launch_dispatch(b->plan.kind, b->wide, f.single, f.acc64,
                                          f.cplx_kernel, nv, A, grid, block, lds, st));
        v0 += nv;
    }
    if (xr_on && !capturing) XDG_TRY_HIP(hipEventRecord(h->xr_ev, st));
    return XDG_OK;
}

// Launch-shape autotuner, run on the first call for a (dtype, nvec) pair:
// first the persistent grid (1, 2, 4 or 8 workgroups per compute unit, or
// one row per lane) and, with several columns, the vectors per pass; then,
// at the best of those, the 8- or 4-waves-per-SIMD copy of the kernel (when
// two workgroups' LDS fit a CU) and, for the table searches, the row loop
// or the wave-compacted term loop.  Every candidate computes bitwise the
// same y, so the timing runs also leave the right y behind.  XDG_TUNE_LOG=1
// prints the timings to stderr.
static bool tune_log() {
    static int on = -1;
    if (on < 0) {
        const char *e = getenv("XDG_TUNE_LOG");
        on = e && atoi(e) > 0;
    }
    return on;
}

int apply_tuned(xdg_ham_s *h, const void *x, void *y, int64_t nvec, int dtype, hipStream_t st) {
    TuneKey key{dtype, nvec};
    std::unique_lock<std::mutex> lock(h->tune_mu);
    auto it = h->tuned.find(key);
    if (it != h->tuned.end()) {
        const LaunchCfg c = it->second;
        lock.unlock();
        return apply_launch(h, x, y, nvec, dtype, st, &c);
    }
    const xdg_basis_s *b = h->basis;
    Form f;
    XDG_RETURN_IF(form_of(b, dtype, nvec, &f));
    const int64_t need = (b->dim + APPLY_BLOCK - 1) / APPLY_BLOCK;
    if (b->dim < (int64_t)1024 * APPLY_BLOCK) {   // small blocks: one row per lane
        LaunchCfg c{APPLY_BLOCK, (int)std::min<int64_t>(need, 1 << 30), 8};
        h->tuned[key] = c;
        return apply_launch(h, x, y, nvec, dtype, st, &c);
    }
    hipEvent_t e0, e1;
    XDG_TRY_HIP(hipEventCreate(&e0));
    XDG_TRY_HIP(hipEventCreate(&e1));
    // one warm launch, then the mean of `reps` timed launches (one for large blocks)
    const int reps = b->dim > (int64_t)200000000 ? 1 : 2;
    auto time_cfg = [&](const LaunchCfg &c, float *ms) -> int {
        XDG_RETURN_IF(apply_launch(h, x, y, nvec, dtype, st, &c));
        XDG_TRY_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) XDG_RETURN_IF(apply_launch(h, x, y, nvec, dtype, st, &c));
        XDG_TRY_HIP(hipEventRecord(e1, st));
        XDG_TRY_HIP(hipEventSynchronize(e1));
        XDG_TRY_HIP(hipEventElapsedTime(ms, e0, e1));
        *ms /= reps;
        if (tune_log()) {
            size_t lds = 0;
            int stg = 0, occ_ok = 0;
            apply_lds(h, dtype, &lds, &stg, &occ_ok);
            fprintf(stderr, "[xdg tune] dim %lld dtype %d nvec %lld (LDS %zu B, tables staged %d, "
                    "8-wave copy possible %d): grid %d nv %d occ %d compact %d xr %d: %.3f ms\n",
                    (long long)b->dim, dtype, (long long)nvec, lds, stg, occ_ok, c.grid, c.nv,
                    c.occ, c.compact, c.xr, *ms);
        }
        return XDG_OK;
    };
    std::vector<LaunchCfg> cands;
    const int cu = device_cu_count();
    for (int mult : {1, 2, 4, 8}) {
        const int g = cu * mult * BLOCKS_PER_1024;
        cands.push_back({APPLY_BLOCK, g, 8});
        if (f.cols > 1) cands.push_back({APPLY_BLOCK, g, (int)std::max<int64_t>(1, f.cols / 2)});
    }
    cands.push_back({APPLY_BLOCK, (int)std::min<int64_t>(need, 1 << 30), 8});
    float best = 1e30f;
    LaunchCfg bestc = cands[0];
    int rc = XDG_OK;
    for (const LaunchCfg &c : cands) {
        float ms = 0;
        if ((rc = time_cfg(c, &ms)) != XDG_OK) break;
        if (ms < best) {
            best = ms;
            bestc = c;
        }
    }
    // second phase: kernel copy (occupancy) and, for table searches, the loop form
    if (rc == XDG_OK) {
        std::vector<LaunchCfg> more;
        const bool table = b->plan.kind == K_SUB || b->plan.kind == K_TAB;
        for (int occ : {0, 1})
            for (int cmp : {0, 1}) {
                if (cmp && !table) continue;
                LaunchCfg c = bestc;
                c.occ = occ;
                c.compact = cmp;
                more.push_back(c);
            }
        // sublattice coding: terms reading a rank-addressed copy of x
        if (b->xr_slots && b->plan.kind == K_SUB)
            for (int occ : {0, 1}) {
                LaunchCfg c = bestc;
                c.occ = occ;
                c.compact = 0;
                c.xr = 1;
                more.push_back(c);
            }
        for (const LaunchCfg &c : more) {
            float ms = 0;
            if ((rc = time_cfg(c, &ms)) != XDG_OK) {
                if (c.xr && rc == XDG_ENOMEM) {   // no room for the copy: not a candidate
                    rc = XDG_OK;
                    continue;
                }
                break;
            }
            if (ms < best) {
                best = ms;
                bestc = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    XDG_RETURN_IF(rc);
    h->tuned[key] = bestc;
    bool xr_used = false;
    for (const auto &kv : h->tuned) xr_used |= kv.second.xr != 0;
    if (!xr_used) {   // free the copy no tuned shape reads
        std::lock_guard<std::mutex> g(h->xr_mu);
        h->xr_slot_bytes = 0;
        h->xr_buf.release();
    }
    return apply_launch(h, x, y, nvec, dtype, st, &bestc);
}

int apply_tuned_config(xdg_ham_s *h, int dtype, int64_t nvec, LaunchCfg *out) {
    std::lock_guard<std::mutex> lock(h->tune_mu);
    auto it = h->tuned.find(TuneKey{dtype, nvec});
    if (it == h->tuned.end()) {
        set_error("no tuned launch shape yet for dtype %d, nvec %lld (apply once first)", dtype,
                  (long long)nvec);
        return XDG_EINVAL;
    }
    *out = it->second;
    return XDG_OK;
}

int ham_count_nnz(xdg_ham_s *h, int64_t *nnz) {
    if (h->nnz >= 0) {
        *nnz = h->nnz;
        return XDG_OK;
    }
    const xdg_basis_s *b = h->basis;
    if (b->dim == 0) {
        h->nnz = 0;
        *nnz = 0;
        return XDG_OK;
    }
    DevBuf cnt;
    XDG_RETURN_IF(cnt.alloc(sizeof(unsigned long long)));
    XDG_TRY_HIP(hipMemset(cnt.p, 0, sizeof(unsigned long long)));
    ApplyArgs A{};
    A.one = make_desc(h, false, nullptr, nullptr);
    A.count = cnt.as<unsigned long long>();
    A.stage_sub = 1;
    size_t lds = stage_bytes<double>(A.one, b->plan.kind, 1);
    if (lds > lds_budget()) {
        A.stage_sub = 0;
        lds = stage_bytes<double>(A.one, b->plan.kind, 0);
    }
    const unsigned block = APPLY_BLOCK;
    const unsigned grid =
        (unsigned)std::min<int64_t>((b->dim + block - 1) / block, (int64_t)apply_grid_for(2));
    int rc;
    switch (b->plan.kind) {
        case K_U1: rc = launch_count_kind<K_U1>(b->wide, A, grid, block, lds, 0); break;
        case K_AFF: rc = launch_count_kind<K_AFF>(b->wide, A, grid, block, lds, 0); break;
        case K_SUB: rc = launch_count_kind<K_SUB>(b->wide, A, grid, block, lds, 0); break;
        default: rc = launch_count_kind<K_TAB>(b->wide, A, grid, block, lds, 0); break;
    }
    XDG_RETURN_IF(rc);
    unsigned long long c = 0;
    XDG_RETURN_IF(copy_d2h(&c, cnt.p, sizeof c, nullptr));
    h->nnz = b->dim + (int64_t)c;
    *nnz = h->nnz;
    return XDG_OK;
}

int batch_plan_host(int n, xdg_ham_s *const *hams, const void *const *xs, void *const *ys,
                    int64_t nvec, int dtype, BatchMeta *P, SectorDesc *descs, uint32_t *prefix,
                    uint32_t tile_rows) {
    if (n < 1) {
        set_error("batched apply needs at least one block");
        return XDG_EINVAL;
    }
    const xdg_basis_s *b0 = hams[0]->basis;
    bool any_cplx = false;
    for (int i = 0; i < n; ++i) {
        const xdg_basis_s *b = hams[i]->basis;
        if (b->plan.kind != b0->plan.kind || b->wide != b0->wide) {
            set_error("batched blocks must share the search kind and the state word width");
            return XDG_EINVAL;
        }
        if (b->is_complex && !dtype_complex(dtype)) {
            set_error("block %d is complex: vectors must be complex", i);
            return XDG_EINVAL;
        }
        any_cplx |= b->is_complex;
    }
    if (dtype < XDG_F64 || dtype > XDG_C64 || nvec < 1) {
        set_error("bad dtype or nvec");
        return XDG_EINVAL;
    }
    P->n = n;
    P->kind = b0->plan.kind;
    P->wide = b0->wide;
    P->single = dtype_single(dtype);
    P->acc64 = !P->single || !(b0->plan.flags & XDG_FLAG_F32_ACCUMULATE);
    P->tsingle = P->single && !P->acc64;
    P->cplx = any_cplx;
    P->cols = (dtype_complex(dtype) && !any_cplx) ? 2 * nvec : nvec;
    // rows per work item: a multiple of the workgroup (default four rows per lane)
    P->tile_rows = tile_rows ? (tile_rows + APPLY_BLOCK - 1) / APPLY_BLOCK * APPLY_BLOCK
                             : 4 * APPLY_BLOCK;
    size_t lds_full = 0, lds_part = 0;
    uint64_t acc = 0;
    for (int i = 0; i < n; ++i) {
        const SectorDesc d = make_desc(hams[i], P->tsingle, xs[i], ys[i]);
        const uint64_t tiles = (hams[i]->basis->dim + P->tile_rows - 1) / P->tile_rows;
        if (acc + tiles >= 0xFFFFFFFFull) {
            set_error("too many row tiles in the batch");
            return XDG_EINVAL;
        }
        if (prefix) prefix[i] = (uint32_t)acc;
        acc += tiles;
        if (descs) descs[i] = d;
        const size_t f1 = P->tsingle ? stage_bytes<float>(d, P->kind, 1)
                                     : stage_bytes<double>(d, P->kind, 1);
        const size_t f0 = P->tsingle ? stage_bytes<float>(d, P->kind, 0)
                                     : stage_bytes<double>(d, P->kind, 0);
        lds_full = std::max(lds_full, f1);
        lds_part = std::max(lds_part, f0);
    }
    if (prefix) prefix[n] = (uint32_t)acc;
    P->n_tiles = (uint32_t)acc;
    P->stage_sub = lds_full <= lds_budget();
    P->lds = P->stage_sub ? lds_full : lds_part;
    return XDG_OK;
}

int batch_prepare(int n, xdg_ham_s *const *hams, const void *const *xs, void *const *ys,
                  int64_t nvec, int dtype, BatchPlan *P, uint32_t tile_rows) {
    if (n < 1) {
        set_error("batched apply needs at least one block");
        return XDG_EINVAL;
    }
    std::vector<SectorDesc> descs(n);
    std::vector<uint32_t> prefix(n + 1, 0);
    XDG_RETURN_IF(batch_plan_host(n, hams, xs, ys, nvec, dtype, P, descs.data(), prefix.data(),
                                  tile_rows));
    XDG_RETURN_IF(P->descs.upload(descs.data(), sizeof(SectorDesc) * n));
    XDG_RETURN_IF(P->prefix.upload(prefix.data(), sizeof(uint32_t) * (n + 1)));
    XDG_RETURN_IF(P->queue.alloc(sizeof(uint32_t)));
    return XDG_OK;
}

int batch_launch_raw(const BatchMeta &P, const SectorDesc *d_descs, const uint32_t *d_prefix,
                     uint32_t *d_queue, int grid, int nv_cap, hipStream_t st) {
    if (P.n_tiles == 0) return XDG_OK;
    ApplyArgs A{};
    A.descs = d_descs;
    A.tile_prefix = d_prefix;
    A.n_secs = P.n;
    A.n_tiles = P.n_tiles;
    A.tile_rows = P.tile_rows;
    A.queue = d_queue;
    A.nvec = P.cols;
    A.stage_sub = P.stage_sub;
    A.occ = P.stage_sub ? occ_for(P.lds) : 0;
    const unsigned g = (unsigned)(grid > 0 ? grid : apply_grid_for(2));
    for (int64_t v0 = 0; v0 < P.cols;) {
        const int nv = pick_nv(P.cols - v0, nv_cap > 0 ? nv_cap : 8);
        A.v0 = (int)v0;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, A.queue);
        XDG_TRY_HIP(hipGetLastError());
        XDG_RETURN_IF(
            launch_dispatch(P.kind, P.wide, P.single, P.acc64, P.cplx, nv, A, g, APPLY_BLOCK,
                            P.lds, st));
        v0 += nv;
    }
    return XDG_OK;
}

int batch_launch(const BatchPlan &P, int grid, int nv_cap, hipStream_t st) {
    return batch_launch_raw(P, P.descs.as<SectorDesc>(), P.prefix.as<uint32_t>(),
                            P.queue.as<uint32_t>(), grid, nv_cap, st);
}

// ------------------------------------------------- batched launch shape --
// Chosen once per set of blocks (and nvec, dtype) and remembered: the
// persistent grid (1, 2 or 4 workgroups per compute unit), then the rows per
// work item (1k - 16k), then the vectors per pass (8, 4, 2).  XDG_TUNE_LOG=1
// prints the timings.
namespace {
std::mutex g_shape_mu;
std::map<std::vector<const void *>, BatchShape> g_shape_cache;

std::vector<const void *> shape_key(int n, xdg_ham_s *const *hams, int64_t nvec, int dtype) {
    std::vector<const void *> key;
    for (int i = 0; i < n; ++i) {
        key.push_back(hams[i]);
        key.push_back(reinterpret_cast<const void *>((uintptr_t)hams[i]->serial));
    }
    key.push_back(reinterpret_cast<const void *>((intptr_t)(nvec * 8 + dtype)));
    return key;
}
}  // namespace

bool batch_shape_cached(int n, xdg_ham_s *const *hams, int64_t nvec, int dtype, BatchShape *out) {
    std::lock_guard<std::mutex> lock(g_shape_mu);
    auto it = g_shape_cache.find(shape_key(n, hams, nvec, dtype));
    if (it == g_shape_cache.end()) return false;
    *out = it->second;
    return true;
}

int batch_shape_tuned(int n, xdg_ham_s *const *hams, const void *const *xs, void *const *ys,
                      int64_t nvec, int dtype, hipStream_t st, BatchShape *out) {
    const auto key = shape_key(n, hams, nvec, dtype);
    std::lock_guard<std::mutex> lock(g_shape_mu);
    auto it = g_shape_cache.find(key);
    if (it != g_shape_cache.end()) {
        *out = it->second;
        return XDG_OK;
    }
    BatchShape best_shape{apply_grid_for(2), 4 * 1024, 8};
    hipEvent_t e0, e1;
    XDG_TRY_HIP(hipEventCreate(&e0));
    XDG_TRY_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int64_t cols = 1;
    auto time_shape = [&](const BatchShape &sh) -> int {
        BatchPlan P;
        XDG_RETURN_IF(batch_prepare(n, hams, xs, ys, nvec, dtype, &P, sh.tile));
        cols = P.cols;
        XDG_RETURN_IF(batch_launch(P, sh.grid, sh.nv, st));
        XDG_TRY_HIP(hipEventRecord(e0, st));
        XDG_RETURN_IF(batch_launch(P, sh.grid, sh.nv, st));
        XDG_TRY_HIP(hipEventRecord(e1, st));
        XDG_TRY_HIP(hipEventSynchronize(e1));
        float ms = 0;
        XDG_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (tune_log())
            fprintf(stderr, "[xdg tune] batched %d blocks nvec %lld: grid %d tile %u nv %d: "
                    "%.3f ms\n", n, (long long)nvec, sh.grid, sh.tile, sh.nv, ms);
        if (ms < best) {
            best = ms;
            best_shape = sh;
        }
        return XDG_OK;
    };
    int rc = XDG_OK;
    for (int mult : {1, 2, 4})
        if (rc == XDG_OK) rc = time_shape({apply_grid_for(mult), 4 * 1024, 8});
    const BatchShape g = best_shape;
    for (uint32_t tile : {1024u, 2048u, 8192u, 16384u})
        if (rc == XDG_OK) rc = time_shape({g.grid, tile, g.nv});
    const BatchShape t = best_shape;
    for (int nv : {4, 2})
        if (rc == XDG_OK && nv < cols) rc = time_shape({t.grid, t.tile, nv});
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    XDG_RETURN_IF(rc);
    g_shape_cache[key] = best_shape;
    *out = best_shape;
    return XDG_OK;
}

// ------------------------------------------------- allocation-free batch --
// One file-scope device array per GPU holds everything the batched launch
// needs beyond the caller's vectors: the queue counter, the tile prefix and
// the sector descriptors.  Its address is taken once per device with
// hipGetSymbolAddress (the array's name is a host-side stand-in, not a device
// address); descriptors reach it through the arguments of a small fill
// kernel, so nothing is allocated and no host buffer must outlive the call.
constexpr int NOALLOC_MAX_SECTORS = 128;
constexpr size_t NOALLOC_PREFIX_OFF = 256;
constexpr size_t NOALLOC_DESC_OFF =
    a16(NOALLOC_PREFIX_OFF + sizeof(uint32_t) * (NOALLOC_MAX_SECTORS + 1));
constexpr size_t NOALLOC_BYTES = NOALLOC_DESC_OFF + sizeof(SectorDesc) * NOALLOC_MAX_SECTORS;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int FILL_PER_LAUNCH = 4;
struct FillArgs {
    SectorDesc d[FILL_PER_LAUNCH];
    uint32_t prefix[FILL_PER_LAUNCH + 1];
    int first, count;
    int last;            // 1: also write prefix[first + count] (the total)
    unsigned char *base;
};
static_assert(sizeof(FillArgs) <= 2048, "fill kernel arguments");

static __global__ void k_fill_batch(FillArgs a) {
    const int i = threadIdx.x;
    if (i < a.count) {
        SectorDesc *d = reinterpret_cast<SectorDesc *>(a.base + NOALLOC_DESC_OFF);
        d[a.first + i] = a.d[i];
        reinterpret_cast<uint32_t *>(a.base + NOALLOC_PREFIX_OFF)[a.first + i] = a.prefix[i];
    }
    if (i == 0 && a.last)
        reinterpret_cast<uint32_t *>(a.base + NOALLOC_PREFIX_OFF)[a.first + a.count] =
            a.prefix[a.count];
}

static int scratch_address(unsigned char **out) {
    static std::mutex mu;
    static void *ptr[64] = {};
    int dev = 0;
    XDG_TRY_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device %d out of range for the allocation-free path", dev);
        return XDG_EINVAL;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        XDG_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned no address for the scratch array");
            return XDG_EHIP;
        }
        ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(ptr[dev]);
    return XDG_OK;
}

int apply_batched_noalloc(int n, xdg_ham_s *const *hams, const void *const *xs,
                          void *const *ys, int64_t nvec, int dtype, hipStream_t st) {
    if (n < 1 || n > NOALLOC_MAX_SECTORS) {
        set_error("allocation-free batched apply takes 1 to %d blocks (got %d); its scratch "
                  "array holds %zu bytes", NOALLOC_MAX_SECTORS, n, NOALLOC_BYTES);
        return XDG_EINVAL;
    }
    for (int i = 0; i < n; ++i)
        if (!hams[i] || !xs[i] || !ys[i] || xs[i] == ys[i]) {
            set_error("batched apply: null handle/pointer or x == y at %d", i);
            return XDG_EINVAL;
        }
    thread_local SectorDesc descs[NOALLOC_MAX_SECTORS];
    thread_local uint32_t prefix[NOALLOC_MAX_SECTORS + 1];
    BatchShape sh;     // a shape tuned earlier for these blocks, else the default
    const bool tuned = batch_shape_cached(n, hams, nvec, dtype, &sh);
    BatchMeta M;
    XDG_RETURN_IF(batch_plan_host(n, hams, xs, ys, nvec, dtype, &M, descs, prefix,
                                  tuned ? sh.tile : 0));
    unsigned char *base = nullptr;
    XDG_RETURN_IF(scratch_address(&base));
    for (int first = 0; first < n; first += FILL_PER_LAUNCH) {
        FillArgs a{};
        a.first = first;
        a.count = std::min(FILL_PER_LAUNCH, n - first);
        a.last = first + a.count == n;
        for (int i = 0; i < a.count; ++i) a.d[i] = descs[first + i];
        for (int i = 0; i <= a.count; ++i) a.prefix[i] = prefix[first + i];
        a.base = base;
        hipLaunchKernelGGL(k_fill_batch, dim3(1), dim3(64), 0, st, a);
        XDG_TRY_HIP(hipGetLastError());
    }
    return batch_launch_raw(M, reinterpret_cast<const SectorDesc *>(base + NOALLOC_DESC_OFF),
                            reinterpret_cast<const uint32_t *>(base + NOALLOC_PREFIX_OFF),
                            reinterpret_cast<uint32_t *>(base), tuned ? sh.grid : 0,
                            tuned ? sh.nv : 8, st);
}

int apply_batched_launch(int n, xdg_ham_s *const *hams, const void *const *xs, void *const *ys,
                         int64_t nvec, int dtype, hipStream_t st, uint32_t *, int grid, int) {
    for (int i = 0; i < n; ++i)
        if (!hams[i] || !xs[i] || !ys[i] || xs[i] == ys[i]) {
            set_error("batched apply: null handle/pointer or x == y at %d", i);
            return XDG_EINVAL;
        }
    // plans are cached by the exact argument tuple so that repeated calls
    // (iterative methods) upload nothing; a Hamiltonian enters the key by its
    // serial number too, since a new one may reuse a freed one's address
    struct Key {
        std::vector<const void *> p;
        int64_t nvec;
        int dtype;
        bool operator==(const Key &o) const { return p == o.p && nvec == o.nvec && dtype == o.dtype; }
    };
    thread_local std::vector<std::pair<Key, std::unique_ptr<BatchPlan>>> cache;
    Key k;
    for (int i = 0; i < n; ++i) {
        k.p.push_back(hams[i]);
        k.p.push_back(reinterpret_cast<const void *>((uintptr_t)hams[i]->serial));
        k.p.push_back(xs[i]);
        k.p.push_back(ys[i]);
    }
    k.nvec = nvec;
    k.dtype = dtype;
    BatchShape sh;
    XDG_RETURN_IF(batch_shape_tuned(n, hams, xs, ys, nvec, dtype, st, &sh));
    k.p.push_back(reinterpret_cast<const void *>((uintptr_t)sh.tile));
    BatchPlan *P = nullptr;
    for (auto &e : cache)
        if (e.first == k) P = e.second.get();
    if (!P) {
        auto up = std::make_unique<BatchPlan>();
        XDG_RETURN_IF(batch_prepare(n, hams, xs, ys, nvec, dtype, up.get(), sh.tile));
        if (cache.size() >= 8) cache.erase(cache.begin());
        cache.emplace_back(k, std::move(up));
        P = cache.back().second.get();
    }
    return batch_launch(*P, grid > 0 ? grid : sh.grid, sh.nv, st);
}

}  // namespace xdg
