// The matrix-free application y = H x on a sector (apply, Sec. 3.6; the
// on-the-fly element loop of Sec. 5.1 and the indexing of Sec. 5.2).
//
// Pull form: one lane owns one output row r (a basis state).  For every bond
// with unequal spins it forms t = r with both spins exchanged, finds the
// representative s of t, a group element u with u.t = s (the first one the
// search meets: when s is in the block, chi is 1 on Stab(s), so every such u
// has the same chi(u)) and the number of such elements (= |Stab(s)|), looks
// up the index of s, and adds
//      (Jxy/2) chi(u) sqrt(|Stab s| / |Stab r|) x[idx(s)]
// to the row, after the diagonal Sum_b Jz_b (+-1/4) x[r].  The row is
// written once: no atomics, bitwise reproducible for any launch shape.
// Up to NV vectors of the [dim][nvec] block share each search and lookup.
// Workgroups are up to 1024 lanes so that the tables staged in LDS (bonds,
// characters, search tables) are shared by 16 waves.
#pragma once

#include "device_common.hpp"

namespace xdg {

#ifndef XDG_APPLY_BLOCK
#define XDG_APPLY_BLOCK 1024
#endif
constexpr int APPLY_BLOCK = XDG_APPLY_BLOCK;
// Occupancy variant: at most 64 VGPRs (8 waves per SIMD, two 1024-lane
// workgroups per CU), chosen when two workgroups' LDS fit in one CU.
constexpr int OCC_WAVES = 8;
constexpr int BLOCKS_PER_1024 = 1024 / APPLY_BLOCK;   // grid scale for smaller workgroups

template <class T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <class T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
    if constexpr (sizeof(T) == 4)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_fma(a, b, c);
}

template <class T> struct BondT;
template <> struct BondT<float> { using type = BondF; };
template <> struct BondT<double> { using type = BondD; };

// Everything one sector needs on the device (type-erased pointers).
struct SectorDesc {
    const void *reps;            // u32 / u64 [dim]
    const uint16_t *stab;        // [dim]
    int64_t dim;
    const void *hash;
    uint64_t n_lines;
    uint64_t empty;
    const uint2 *rwords;         // rank index (null: hash)
    uint64_t n_rwords;
    const void *rtab;            // colex chunk tables (layout rl)
    RankLayout rl;
    int n_up;
    const uint32_t *lin;         // Lin tables (U(1))
    int nlo;
    int n_sites, n_sym, n_bonds;
    const AffineElem *aff;
    int ring;                    // 0, 1 (all rotations), 2 (and all reflections)
    const int16_t *ring_gidx;    // [2 n_sites]
    const uint64_t *bytetab;
    int n_bchunks;
    const uint16_t *mintop;
    const uint32_t *cand_off;
    const uint16_t *cand_list;
    const uint32_t *sp;
    const uint16_t *tperm;
    int n_s, m, pb, n_perm;
    uint32_t n_cand;
    int subf;                    // sublattice tables in the packed form (staged kernels)
    const BondX *bx;             // per-bond data of the packed form [n_bonds]
    const void *bonds;           // BondD / BondF [n_bonds]
    const void *chi;             // double2 / float2 [n_sym]
    const void *sqrtt;           // T [2 (n_sym + 1)]: sqrt(c), then 1/sqrt(c)
    double jz_quarter;           // (1/4) sum_b Jz_b: the diagonal of the all-aligned state
    int ring_bonds;              // 1: n_bonds = n_sites and bond b joins sites b and b + 1 mod N
    // rank-addressed x (sublattice coding): slot top_rank(s) of xr holds the
    // row of representative s when s is a basis state, zeros otherwise, so a
    // term reads x without the index lookup (null: through the rank index)
    const void *xr;
    const uint64_t *xr_top;      // [2^m] first rank of each top block, ~0 if none
    const uint32_t *xr_top32;    // the same in 4 bytes (0xFFFFFFFF if none), when all fit; or null
    uint64_t xr_slots;           // slots of xr (beyond the last one: not in the block)
    int xr_bits;                 // sites below the top block
    const uint32_t *xr_rtab;     // the rank tables' rows for the chunks below it, 4-byte entries
    int xr_rows;                 // rows of xr_rtab
    const void *x;
    void *y;
};

struct ApplyArgs {
    SectorDesc one;              // used when descs == nullptr
    const SectorDesc *descs;     // batched: device array [n_secs]
    const uint32_t *tile_prefix; // batched: [n_secs + 1] cumulative tile counts
    int n_secs;
    uint32_t n_tiles;
    uint32_t tile_rows;
    uint32_t *queue;             // batched: work counter, zero at launch
    int64_t nvec;
    int v0;                      // first vector of this pass
    int stage_sub;               // copy sublattice tables into LDS
    int occ;                     // use the 8-waves-per-SIMD variant
    int compact;                 // table searches: wave-compacted term loop
    unsigned long long *count;   // nnz counting mode (nullptr otherwise)
};

__host__ __device__ constexpr size_t a16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t sub_table_bytes(const SectorDesc &d) {
    const size_t NV = (size_t)d.n_s << d.m;
    return a16(2 * NV) + a16(4 * (NV + 1)) + a16(2 * (size_t)d.n_cand) +
           a16(4 * (size_t)d.n_sym * d.n_s) +
           a16(2 * (size_t)d.n_perm * 2 * ((size_t)1 << d.pb));
}

__host__ __device__ inline size_t rank_table_bytes(const SectorDesc &d) {
    if (!d.rwords) return 0;
    // the rank-addressed x reads only its 4-byte rows of the chunks below the top block
    if (d.xr) return ((size_t)d.xr_rows << d.rl.cb) * 4;
    return ((size_t)d.rl.rows << d.rl.cb) * (d.rl.e32 ? 4 : 8);
}

// bytes of the first-rank table of the rank-addressed x in LDS
__host__ __device__ inline size_t xr_top_bytes(const SectorDesc &d) {
    return ((size_t)1 << d.m) * (d.xr_top32 ? 4 : 8);
}

// LDS bytes needed to stage a sector's tables.
template <class T>
__host__ __device__ inline size_t stage_bytes(const SectorDesc &d, int kind, int stage_sub) {
    size_t n = a16(sizeof(typename BondT<T>::type) * d.n_bonds);
    if (kind != K_U1) {
        n += a16(sizeof(typename Vec2<T>::type) * d.n_sym);
        n += a16(sizeof(T) * 2 * (d.n_sym + 1));
        n += a16(rank_table_bytes(d));
        if (kind == K_AFF) n += a16(sizeof(AffineElem) * d.n_sym) + a16(4 * (size_t)d.n_sites);
        if (kind == K_SUB && stage_sub) n += sub_table_bytes(d);
        // packed form: alignment of the permutation tables
        if (kind == K_SUB && stage_sub && d.subf) n += 128;
        if (kind == K_SUB && stage_sub && d.xr) n += a16(xr_top_bytes(d));
    }
    return n;
}

template <class T>
struct Staged {
    const typename BondT<T>::type *bonds;
    const typename Vec2<T>::type *chi;
    const T *sq;       // sqrt(c)
    const T *rsq;      // 1/sqrt(c)
    const AffineElem *aff;
    const int16_t *ring_gidx;
    const void *rtab;
    SubCtx sub;
    bool subf;             // packed sublattice search (sub.sp holds the packed entries)
    uint32_t amask;        // ~(4E - 1)
    const uint64_t *xr_top;   // first rank of each top block (rank-addressed x)
    const uint32_t *xr_top32; // the same in 4 bytes (xr_w32) at the same place
    bool xr_w32;
};

template <class E>
__device__ inline E *stage_copy(unsigned char *smem, size_t &off, const E *src, size_t n) {
    E *dst = reinterpret_cast<E *>(smem + off);
    off = a16(off + sizeof(E) * n);
    for (size_t e = threadIdx.x; e < n; e += blockDim.x) dst[e] = src[e];
    return dst;
}

// STAGE: the sublattice tables go to LDS too (otherwise they are read from
// global memory); a compile-time choice so that every table pointer has a
// known address space.
template <int KIND, class T, bool STAGE>
__device__ inline void stage(const SectorDesc &d, unsigned char *smem, Staged<T> &S) {
    using B = typename BondT<T>::type;
    using T2 = typename Vec2<T>::type;
    size_t off = 0;
    S.bonds = stage_copy(smem, off, reinterpret_cast<const B *>(d.bonds), d.n_bonds);
    S.sub = SubCtx{d.mintop, d.cand_off, d.cand_list, d.sp, d.tperm, d.n_s, d.m, d.pb};
    S.subf = false;
    S.xr_top = d.xr_top;
    S.xr_top32 = d.xr_top32;
    S.xr_w32 = d.xr_top32 != nullptr;
    if constexpr (KIND != K_U1) {
        S.chi = stage_copy(smem, off, reinterpret_cast<const T2 *>(d.chi), d.n_sym);
        const T *ls = stage_copy(smem, off, reinterpret_cast<const T *>(d.sqrtt), 2 * (d.n_sym + 1));
        S.sq = ls;
        S.rsq = ls + d.n_sym + 1;
        S.rtab = stage_copy(smem, off,
                            reinterpret_cast<const uint32_t *>(d.xr ? d.xr_rtab : d.rtab),
                            rank_table_bytes(d) / 4);
        if constexpr (KIND == K_AFF) {
            S.aff = stage_copy(smem, off, d.aff, d.n_sym);
            int16_t *lg = reinterpret_cast<int16_t *>(smem + off);
            off = a16(off + 4 * (size_t)d.n_sites);
            if (d.ring)
                for (int e = threadIdx.x; e < 2 * d.n_sites; e += blockDim.x) lg[e] = d.ring_gidx[e];
            S.ring_gidx = lg;
        }
        if constexpr (KIND == K_SUB) {
            if constexpr (STAGE) {
                const size_t NV = (size_t)d.n_s << d.m;
                const size_t ntp = (size_t)d.n_perm * 2 * ((size_t)1 << d.pb);
                S.sub.mintop = stage_copy(smem, off, d.mintop, NV);
                S.sub.cand_off = stage_copy(smem, off, d.cand_off, NV + 1);
                S.sub.cand_list = stage_copy(smem, off, d.cand_list, d.n_cand);
                if (d.subf) {
                    // permutation tables at a 128-byte aligned LDS address,
                    // then the packed (element, block) entries pointing there
                    const uint32_t base =
                        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) unsigned char *)smem;
                    off += (128u - ((base + (uint32_t)off) & 127u)) & 127u;
                    const uint32_t tpa = base + (uint32_t)off;
                    S.sub.tperm = stage_copy(smem, off, d.tperm, ntp);
                    const size_t nsp = (size_t)d.n_sym * d.n_s;
                    uint32_t *sq = reinterpret_cast<uint32_t *>(smem + off);
                    off = a16(off + 4 * nsp);
                    for (size_t e = threadIdx.x; e < nsp; e += blockDim.x) {
                        const uint32_t w = d.sp[e];
                        sq[e] = (tpa + 2u * (w >> 8)) | (7u * ((w & 0xFFu) / (uint32_t)d.m));
                    }
                    S.sub.sp = sq;
                    S.amask = ~((4u << d.pb) - 1u);
                    S.subf = true;
                } else {
                    S.sub.sp = stage_copy(smem, off, d.sp, (size_t)d.n_sym * d.n_s);
                    S.sub.tperm = stage_copy(smem, off, d.tperm, ntp);
                }
                // the first-rank table at one LDS address whatever its entry
                // size (both pointers always address LDS here: LDS reads)
                unsigned char *tp = smem + off;
                if (d.xr) {
                    if (d.xr_top32)
                        stage_copy(smem, off, d.xr_top32, (size_t)1 << d.m);
                    else
                        stage_copy(smem, off, d.xr_top, (size_t)1 << d.m);
                }
                S.xr_top32 = reinterpret_cast<const uint32_t *>(tp);
                S.xr_top = reinterpret_cast<const uint64_t *>(tp);
            }
        }
    }
}

// Positions of 32-bit states are below C(32, 16) < 2^31: 32-bit indices.
template <class W> struct IndexT { using type = int64_t; };
template <> struct IndexT<uint32_t> { using type = int32_t; };

// Locate the representative of t and its index; returns -1 when the orbit
// is not in the block.  On success writes u and |Stab(s)|.  key: t's key for
// the packed sublattice search (computed here from t when null and that
// search is on).  XR: the position is the slot in the rank-addressed x
// (sublattice coding with d.xr set); XR = 2: every character is 1, so the
// search does not keep the element (u is left unset).
template <class W, int KIND, class T, int XR = 0>
__device__ __forceinline__ typename IndexT<W>::type locate(const SectorDesc &d, const Staged<T> &S,
                                                           W t, int &u, int &cnt,
                                                           const SubKey *key = nullptr) {
    using I = typename IndexT<W>::type;
    if constexpr (KIND == K_U1) {
        const uint64_t lo = (uint64_t)t & ((1ull << d.nlo) - 1);
        const uint64_t hi = (uint64_t)t >> d.nlo;
        const uint32_t *lin = d.lin;
        u = 0;
        cnt = 1;
        return (I)((int64_t)gld(lin + (1ull << d.nlo) + hi) + (int64_t)gld(lin + lo));
    } else {
        W rep;
        if constexpr (KIND == K_AFF) {
            if (d.ring)
                ring_search<W>(S.ring_gidx, d.ring, d.n_sites, t, rep, u, cnt);
            else
                aff_search<W>(S.aff, d.n_sym, d.n_sites, t, rep, u, cnt);
        } else if constexpr (KIND == K_SUB) {
            if (S.subf) {
                if (key)
                    sub_search_packed<W, XR != 2>(S.sub, S.amask, *key, rep, u, cnt);
                else
                    sub_search_packed<W, XR != 2>(S.sub, S.amask, sub_key<W>(t, d.m, d.pb), rep,
                                                  u, cnt);
            } else if (d.n_s == 4)
                sub_search<W, 4>(S.sub, t, rep, u, cnt);
            else
                sub_search<W, 0>(S.sub, t, rep, u, cnt);
        } else {
            tab_search<W>(d.bytetab, d.n_bchunks, d.n_sym, t, rep, u, cnt);
        }
        if constexpr (KIND == K_SUB && XR != 0) {
            // the slot of rep in the rank-addressed x (zeros unless rep is a basis state)
            const uint32_t *T32 = static_cast<const uint32_t *>(S.rtab);
            const uint64_t r = S.xr_w32
                                   ? top_rank32<W>(T32, d.rl, d.xr_bits, S.xr_top32, rep)
                                   : top_rank<W>(T32, d.rl, d.xr_bits, S.xr_top, rep);
            return r < d.xr_slots ? (I)r : (I)-1;
        }
        if (d.rwords) {
            if constexpr (sizeof(W) == 4) {
                const uint64_t r = colex_rank<W>(S.rtab, d.rl, rep);
                return rank_find32(d.rwords, (uint32_t)d.n_rwords, (uint32_t)r);
            } else {
                // 4-byte entries: every basis state's rank is below 2^32 - 1
                if (d.rl.e32) {
                    const uint32_t r =
                        colex_rank_sat<W>(static_cast<const uint32_t *>(S.rtab), d.rl, rep);
                    return r == 0xFFFFFFFFu ? -1
                                            : rank_find_r32(d.rwords, (uint32_t)d.n_rwords, r);
                }
                return rank_find(d.rwords, d.n_rwords, colex_rank<W>(S.rtab, d.rl, rep));
            }
        }
        return (I)hash_find<W>(d.hash, d.n_lines, (W)d.empty, rep);
    }
}

// T: storage type of x and y; A: type of the amplitudes and of the per-row
// accumulation (each output element is rounded to T once, at the store).
// XR: the terms read the rank-addressed x (sublattice coding, d.xr set);
// XR = 2: every character is 1 (the amplitude skips chi(u), a product by
// exactly 1).  PIPE: each term's gather is added at the next term of the row
// (or after its last bond), so that its latency overlaps the next search;
// the same fused multiply-adds in the same order.
template <class W, int KIND, class T, class A, bool CPLX, int NV, int XR = 0,
          bool PIPE = false>
__device__ __forceinline__ void process_row(const SectorDesc &d, const Staged<A> &S, int64_t row,
                                            int64_t nvec, int v0) {
    using B = typename BondT<A>::type;
    constexpr int C = CPLX ? 2 : 1;
    const W s = gld(reinterpret_cast<const W *>(d.reps) + row);
    const T *X = reinterpret_cast<const T *>(d.x);
    T *Y = reinterpret_cast<T *>(d.y);
    // the terms' x: rank-addressed (the same values at other places) or x itself
    const T *XT = XR != 0 ? reinterpret_cast<const T *>(d.xr) : X;
    static_assert(XR != 2 || (PIPE && !CPLX), "trivial characters: real blocks, pipelined loop");
    const int nb = d.n_bonds;
    // Diagonal: sum_b Jz_b (+1/4 if the spins of b are equal, -1/4 if not)
    // = (1/4) sum_b Jz_b - (1/2) sum over the unequal-spin bonds of Jz_b; the
    // second sum is taken in the walk over those bonds below.
    A junq = 0;
    A acc[NV * C];
#pragma unroll
    for (int v = 0; v < NV * C; ++v) acc[v] = 0;
    A rn = A(1);
    if constexpr (KIND != K_U1) rn = S.rsq[gld(d.stab + row)];
    // explicit fused multiply-adds: a complex kernel on a block with real
    // characters (ai = 0) rounds exactly like the real kernel
    auto add = [&](A ar, A ai, const T *xv) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (CPLX) {
                const A xr = xv[2 * v], xi = xv[2 * v + 1];
                acc[2 * v] = fmadd<A>(-ai, xi, fmadd<A>(ar, xr, acc[2 * v]));
                acc[2 * v + 1] = fmadd<A>(ai, xr, fmadd<A>(ar, xi, acc[2 * v + 1]));
            } else {
                acc[v] = fmadd<A>(ar, (A)xv[v], acc[v]);
            }
        }
    };
    bool p_ok = false;   // PIPE: the pending term
    A p_ar = 0, p_ai = 0;
    T p_x[NV * C];
#pragma unroll
    for (int v = 0; v < NV * C; ++v) p_x[v] = T(0);
    // key: the packed sublattice search's key of the term's state, if given
    auto term = [&](const B &bd, W t, const SubKey *key) {
        int u, cnt;
        const auto idx = locate<W, KIND, A, XR>(d, S, t, u, cnt, key);
        if constexpr (PIPE) {
            // the gather is issued for every term (row 0 when the orbit is
            // not in the block: a valid address, never added)
            const bool ok = idx >= 0;
            A ar = 0, ai = 0;
            if (ok) {
                const A f = bd.h * S.sq[cnt];
                if constexpr (XR == 2) {
                    ar = f;   // chi(u) = 1
                } else {
                    const auto c = S.chi[u];
                    ar = f * c.x;
                    if constexpr (CPLX) ai = f * c.y;
                }
            }
            // the previous gather (issued one search ago) is added first, so
            // that the new one can land in the same registers
            if (p_ok) add(p_ar, p_ai, p_x);
            const size_t xb = ((size_t)(ok ? idx : 0) * nvec + v0) * C;
#pragma unroll
            for (int v = 0; v < NV * C; ++v) p_x[v] = gld(XT + xb + v);
            p_ok = ok;
            p_ar = ar;
            p_ai = ai;
            return;
        }
        if (idx < 0) return;
        A ar = bd.h, ai = 0;
        if constexpr (KIND != K_U1) {
            const A f = bd.h * S.sq[cnt];   // times 1/sqrt|Stab r| once per row
            const auto c = S.chi[u];
            ar = f * c.x;
            if constexpr (CPLX) ai = f * c.y;
        }
        // 32-bit states: positions below 2^31, one 32 x 32 -> 64-bit multiply-add
        const size_t xb = sizeof(W) == 4
                              ? (uint64_t)(uint32_t)idx * (uint32_t)(nvec * C) + (uint64_t)(v0 * C)
                              : ((size_t)idx * nvec + v0) * C;
        // explicit fused multiply-adds: a complex kernel on a block with real
        // characters (ai = 0) rounds exactly like the real kernel
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (CPLX) {
                const A xr = gld(XT + xb + 2 * v), xi = gld(XT + xb + 2 * v + 1);
                acc[2 * v] = fmadd<A>(-ai, xi, fmadd<A>(ar, xr, acc[2 * v]));
                acc[2 * v + 1] = fmadd<A>(ai, xr, fmadd<A>(ar, xi, acc[2 * v + 1]));
            } else {
                acc[v] = fmadd<A>(ar, (A)gld(XT + xb + v), acc[v]);
            }
        }
    };
    if constexpr (KIND == K_AFF || KIND == K_U1) {
        // Cheap searches: per group of 32 bonds, a mask of the bonds with
        // unequal spins, walked lowest first (the order of the plain bond
        // loop), so that a wave iterates over its lanes' active bonds only.
        // Bonds b = (b, b + 1 mod N) in order: bit b of s ^ rotr(s, 1).
        const W walls = d.ring_bonds ? (s ^ rotr_n<W>(s, 1, d.n_sites)) : W(0);
        for (int b0 = 0; b0 < nb; b0 += 32) {
            const int bn = nb - b0 < 32 ? nb - b0 : 32;
            uint32_t act = 0;
            if (d.ring_bonds) {
                act = (uint32_t)(walls >> b0) & (bn == 32 ? ~0u : ((1u << bn) - 1u));
            } else {
                for (int k = 0; k < bn; ++k) {
                    const B bd = S.bonds[b0 + k];
                    act |= (((uint32_t)(s >> bd.i) ^ (uint32_t)(s >> bd.j)) & 1u) << k;
                }
            }
            while (act) {
                const int b = b0 + __builtin_ctz(act);
                act &= act - 1;
                const B bd = S.bonds[b];
                junq += bd.jz;
                term(bd, s ^ ((W(1) << bd.i) | (W(1) << bd.j)), nullptr);
            }
        }
    } else {
        // Table searches: all lanes take the same bond at the same time, so
        // that neighbouring rows walk similar table entries and look up
        // neighbouring index words.
        bool done = false;
        if constexpr (KIND == K_SUB) {
            if (S.subf && d.bx) {
                // packed form: the bond comes with scalar loads, the term's key
                // is the row's key with the bond's bits flipped
                const SubKey kr = sub_key<W>(s, d.m, d.pb);
                for (int b = 0; b < nb; ++b) {
                    const BondX x = sld(d.bx + b);
                    const B bd = sld(reinterpret_cast<const B *>(d.bonds) + b);
                    const W fl = (W)x.flip, sf = s & fl;
                    if (sf == 0 || sf == fl) continue;
                    junq += bd.jz;
                    const SubKey kt = sub_key_flip(kr, x);
                    term(bd, s ^ fl, &kt);
                }
                if constexpr (PIPE) {
                    if (p_ok) add(p_ar, p_ai, p_x);
                    p_ok = false;
                }
                done = true;
            }
        }
        if (!done) {
            for (int b = 0; b < nb; ++b) {
                const B bd = S.bonds[b];
                if (((s >> bd.i) & 1) == ((s >> bd.j) & 1)) continue;
                junq += bd.jz;
                term(bd, s ^ ((W(1) << bd.i) | (W(1) << bd.j)), nullptr);
            }
            if constexpr (PIPE) {
                if (p_ok) add(p_ar, p_ai, p_x);
                p_ok = false;
            }
        }
    }
    const size_t base = ((size_t)row * nvec + v0) * C;
    const A diag = (A)d.jz_quarter - A(0.5) * junq;
#pragma unroll
    for (int v = 0; v < NV * C; ++v) {
        const A off = KIND != K_U1 ? rn * acc[v] : acc[v];
        gst(Y + base + v, (T)fmadd<A>(diag, (A)gld(X + base + v), off));
    }
}

// ------------------------------------------------ wave-compacted term loop --
// For the table searches (sublattice coding, byte tables) the row loop above
// takes every bond with all lanes of the wave at once, so on each bond only
// the lanes whose spins differ there (about half) do a term.  Here a wave
// owns a window of 64 + CMP_EXTRA consecutive rows (a second row on the
// first CMP_EXTRA lanes) and, bond by bond, packs the unequal-spin terms of
// the window into passes of up to 64: every lane of a pass takes the same
// bond, as in the row loop, but most lanes have a term.  Terms move between
// lanes with cross-lane permutes (no LDS): each owner pushes its row to the
// lane that will do its term, that lane pulls the row state, computes the
// term, and the owner pulls the amplitude and the gathered x back and adds
// them with the same fused multiply-adds, in bond order, so that both loops
// give bitwise identical rows.
constexpr int CMP_EXTRA = 48;
constexpr int CMP_ROWS = 64 + CMP_EXTRA;   // rows per wave window

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ int rank_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ int pull32(int src_lane, int v) {
    return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}

template <class V>
__device__ __forceinline__ V pull(int src_lane, V v) {
    if constexpr (sizeof(V) == 4) {
        return __builtin_bit_cast(V, pull32(src_lane, __builtin_bit_cast(int, v)));
    } else {
        static_assert(sizeof(V) == 8, "8-byte value");
        const uint64_t u = __builtin_bit_cast(uint64_t, v);
        const int lo = pull32(src_lane, (int)(uint32_t)u);
        const int hi = pull32(src_lane, (int)(uint32_t)(u >> 32));
        return __builtin_bit_cast(V, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
    }
}

// Lanes with `mine` send `val` to lane `dest` (dest distinct, all inside the
// range [lo, hi)); every other lane sends to one of the lanes outside that
// range, so that the permute is a bijection (a lane that is not a
// destination of any sender would receive an undefined value).  Returns what
// this lane received.
__device__ __forceinline__ int push_range(bool mine, int dest, int lo, int hi, int val) {
    const uint64_t other = __ballot(!mine);
    const int d = mine ? dest : ((hi + rank_below(other)) & 63);
    (void)lo;
    return __builtin_amdgcn_ds_permute(d << 2, val);
}

template <class W, int KIND, class T, class A, bool CPLX, int NV>
__device__ __forceinline__ void process_window(const SectorDesc &d, const Staged<A> &S,
                                               int64_t w0, int64_t r1, int64_t nvec, int v0) {
    using B = typename BondT<A>::type;
    constexpr int C = CPLX ? 2 : 1;
    const int lane = lane_id();
    const int64_t row0 = w0 + lane, row1 = w0 + 64 + lane;
    const bool ok0 = row0 < r1, ok1 = lane < CMP_EXTRA && row1 < r1;
    const W *R = reinterpret_cast<const W *>(d.reps);
    const W s0 = ok0 ? gld(R + row0) : W(0);
    const W s1 = ok1 ? gld(R + row1) : W(0);
    const T *X = reinterpret_cast<const T *>(d.x);
    T *Y = reinterpret_cast<T *>(d.y);
    const int nb = d.n_bonds;
    A acc0[NV * C], acc1[NV * C];
#pragma unroll
    for (int v = 0; v < NV * C; ++v) acc0[v] = acc1[v] = 0;
    auto unequal = [](W s, const B &bd) -> bool {
        return (((uint32_t)(s >> bd.i)) ^ ((uint32_t)(s >> bd.j))) & 1u;
    };
    auto add = [&](A *acc, A ar, A ai, const T *xq) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (CPLX) {
                const A xr = xq[2 * v], xi = xq[2 * v + 1];
                acc[2 * v] = fmadd<A>(-ai, xi, fmadd<A>(ar, xr, acc[2 * v]));
                acc[2 * v + 1] = fmadd<A>(ai, xr, fmadd<A>(ar, xi, acc[2 * v + 1]));
            } else {
                acc[v] = fmadd<A>(ar, (A)xq[v], acc[v]);
            }
        }
    };
    for (int b = 0; b < nb; ++b) {
        const B bd = S.bonds[b];
        const bool a0 = ok0 && unequal(s0, bd), a1 = ok1 && unequal(s1, bd);
        const uint64_t M0 = __ballot(a0), M1 = __ballot(a1);
        const int n0 = __popcll(M0), n = n0 + __popcll(M1);
        // term index of this lane's row-0 and row-1 terms (row 0 terms first)
        const int e0 = rank_below(M0), e1 = n0 + rank_below(M1);
        const W flip = (W(1) << bd.i) | (W(1) << bd.j);
        for (int p = 0; p < n; p += 64) {
            const int take = n - p < 64 ? n - p : 64;
            // pass lanes [lo0, hi0) take row-0 terms, [hi0, take) row-1 terms
            const int lo0 = 0, hi0 = n0 - p < 0 ? 0 : (n0 - p < take ? n0 - p : take);
            const bool m0 = a0 && e0 >= p && e0 < p + take;
            const bool m1 = a1 && e1 >= p && e1 < p + take;
            const int g0 = push_range(m0, e0 - p, lo0, hi0, lane);
            const int g1 = push_range(m1, e1 - p, hi0, take, lane);
            const bool has = lane < take;
            const bool second = lane >= hi0;
            const int src = second ? g1 : g0;   // owner lane of this pass lane's term
            const W t0 = pull<W>(src, s0), t1 = pull<W>(src, s1);
            bool ok = false;
            A ar = 0, ai = 0;
            T xv[NV * C];
#pragma unroll
            for (int v = 0; v < NV * C; ++v) xv[v] = T(0);
            if (has) {
                const W t = (second ? t1 : t0) ^ flip;
                int u, cnt;
                const auto idx = locate<W, KIND, A>(d, S, t, u, cnt);
                if (idx >= 0) {
                    ok = true;
                    const A f = bd.h * S.sq[cnt];
                    const auto c = S.chi[u];
                    ar = f * c.x;
                    if constexpr (CPLX) ai = f * c.y;
                    const size_t xb = sizeof(W) == 4
                                          ? (uint64_t)(uint32_t)idx * (uint32_t)(nvec * C) +
                                                (uint64_t)(v0 * C)
                                          : ((size_t)idx * nvec + v0) * C;
#pragma unroll
                    for (int v = 0; v < NV * C; ++v) xv[v] = gld(X + xb + v);
                }
            }
            // owners pull their terms back: row 0, then row 1
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const bool mine = h == 0 ? m0 : m1;
                const int from = mine ? (h == 0 ? e0 : e1) - p : lane;
                const bool okq = pull32(from, (int)ok) != 0;
                const A arq = pull<A>(from, ar);
                A aiq = 0;
                if constexpr (CPLX) aiq = pull<A>(from, ai);
                T xq[NV * C];
#pragma unroll
                for (int v = 0; v < NV * C; ++v) xq[v] = pull<T>(from, xv[v]);
                if (mine && okq) add(h == 0 ? acc0 : acc1, arq, aiq, xq);
            }
        }
    }
    // the diagonal, (1/4) sum_b Jz_b - (1/2) sum over the unequal-spin bonds
    // (bond order, as in the row loop), and the stores
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const bool okh = h == 0 ? ok0 : ok1;
        if (!okh) continue;
        const W sh = h == 0 ? s0 : s1;
        const int64_t row = h == 0 ? row0 : row1;
        A junq = 0;
        for (int b = 0; b < nb; ++b) {
            const B bd = S.bonds[b];
            if (unequal(sh, bd)) junq += bd.jz;
        }
        const A rn = S.rsq[gld(d.stab + row)];
        const size_t base = ((size_t)row * nvec + v0) * C;
        const A diag = (A)d.jz_quarter - A(0.5) * junq;
        const A *acc = h == 0 ? acc0 : acc1;
#pragma unroll
        for (int v = 0; v < NV * C; ++v)
            gst(Y + base + v, (T)fmadd<A>(diag, (A)gld(X + base + v), rn * acc[v]));
    }
}

// rows [r0, r1) of a sector.  CMP: windows of CMP_ROWS rows per wave (every
// lane of a wave takes part in its permutes; `first` and `stride` count
// lanes, so wave w of the launch starts at window w); otherwise a lane per
// row, reading the rank-addressed x when XR.
template <class W, int KIND, class T, class A, bool CPLX, int NV, bool CMP, int XR, bool PIPE>
__device__ __forceinline__ void process_range(const SectorDesc &d, const Staged<A> &S, int64_t r0,
                                              int64_t r1, int64_t first, int64_t stride,
                                              int64_t nvec, int v0) {
    if constexpr (CMP) {
        const int64_t wave = (first - lane_id()) / 64, waves = stride / 64;
        for (int64_t w0 = r0 + wave * CMP_ROWS; w0 < r1; w0 += waves * CMP_ROWS)
            process_window<W, KIND, T, A, CPLX, NV>(d, S, w0, r1, nvec, v0);
    } else {
        for (int64_t row = r0 + first; row < r1; row += stride)
            process_row<W, KIND, T, A, CPLX, NV, XR, PIPE>(d, S, row, nvec, v0);
    }
}

// count of the off-diagonal terms of a row that land in the block
template <class W, int KIND>
__device__ __forceinline__ uint32_t count_row(const SectorDesc &d, const Staged<double> &S,
                                              int64_t row) {
    const W s = reinterpret_cast<const W *>(d.reps)[row];
    uint32_t n = 0;
    for (int b = 0; b < d.n_bonds; ++b) {
        const BondD bd = S.bonds[b];
        if (((s >> bd.i) & 1) == ((s >> bd.j) & 1)) continue;
        const W t = s ^ ((W(1) << bd.i) | (W(1) << bd.j));
        int u, cnt;
        if (locate<W, KIND, double>(d, S, t, u, cnt) >= 0) ++n;
    }
    return n;
}

template <class W, int KIND, class T, class AC, bool CPLX, int NV, bool STAGE, bool OCC,
          bool CMP, int XR>
__global__ __launch_bounds__(APPLY_BLOCK, OCC ? OCC_WAVES : 1) void k_apply(ApplyArgs A) {
    // the sublattice row loop pipelines its gathers
    constexpr bool PIPE = KIND == K_SUB && !CMP;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t s_tile;
    __shared__ SectorDesc s_desc;
    Staged<AC> S;
    if (A.descs == nullptr) {
        const SectorDesc &d = A.one;
        stage<KIND, AC, STAGE>(d, smem, S);
        __syncthreads();
        const int64_t stride = (int64_t)gridDim.x * blockDim.x;
        process_range<W, KIND, T, AC, CPLX, NV, CMP, XR, PIPE>(d, S, 0, d.dim,
                                                (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                                                stride, A.nvec, A.v0);
        return;
    }
    // persistent: (sector, row tile) items from one queue
    int cur = -1;
    for (;;) {
        if (threadIdx.x == 0) s_tile = atomicAdd(A.queue, 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= A.n_tiles) break;
        int lo = 0, hi = A.n_secs - 1;   // last sector with tile_prefix <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.tile_prefix[mid] <= tile) lo = mid; else hi = mid - 1;
        }
        if (lo != cur) {
            if (threadIdx.x == 0) s_desc = A.descs[lo];
            __syncthreads();
            stage<KIND, AC, STAGE>(s_desc, smem, S);
            __syncthreads();
            cur = lo;
        }
        const SectorDesc &d = s_desc;
        const int64_t r0 = (int64_t)(tile - A.tile_prefix[lo]) * A.tile_rows;
        int64_t r1 = r0 + A.tile_rows;
        r1 = r1 < d.dim ? r1 : d.dim;
        process_range<W, KIND, T, AC, CPLX, NV, CMP, XR, PIPE>(d, S, r0, r1, threadIdx.x, blockDim.x,
                                                     A.nvec, A.v0);
        __syncthreads();
    }
}

template <class W, int KIND, bool STAGE>
__global__ __launch_bounds__(APPLY_BLOCK) void k_count(ApplyArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ unsigned long long s_sum;
    Staged<double> S;
    const SectorDesc &d = A.one;
    stage<KIND, double, STAGE>(d, smem, S);
    if (threadIdx.x == 0) s_sum = 0;
    __syncthreads();
    unsigned long long n = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < d.dim; row += stride)
        n += count_row<W, KIND>(d, S, row);
    atomicAdd(&s_sum, n);
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(A.count, s_sum);
}

static __global__ void k_zero_u32(uint32_t *p) { *p = 0; }

// Host launcher for one search kind (instantiated in one translation unit per
// kind).  `single`: FP32 vectors; `acc64`: FP64 amplitudes and accumulation
// (always for FP64 vectors).
template <int KIND>
int launch_kind(bool wide, bool single, bool acc64, bool cplx, int nv, const ApplyArgs &A,
                unsigned grid, unsigned block, size_t lds, hipStream_t st);

template <int KIND>
int launch_count_kind(bool wide, const ApplyArgs &A, unsigned grid, unsigned block, size_t lds,
                      hipStream_t st);

// The sublattice kernels whose terms read the rank-addressed x: any
// characters, and every character 1 (one translation unit each).
int launch_sub_xr(bool wide, bool single, bool acc64, bool cplx, int nv, const ApplyArgs &A,
                  unsigned grid, unsigned block, size_t lds, hipStream_t st);
int launch_sub_xr_trivial(bool wide, bool single, bool acc64, int nv, const ApplyArgs &A,
                          unsigned grid, unsigned block, size_t lds, hipStream_t st);

// XR (the rank-addressed x): passes of at most two vectors.
template <class W, int KIND, class T, class AC, bool CPLX, bool STAGE, bool OCC, bool CMP,
          int XR = 0>
void (*apply_kernel(int nv))(ApplyArgs) {
    switch (nv) {
        case 1: return k_apply<W, KIND, T, AC, CPLX, 1, STAGE, OCC, CMP, XR>;
        case 2: return k_apply<W, KIND, T, AC, CPLX, 2, STAGE, OCC, CMP, XR>;
    }
    if constexpr (!CMP && XR == 0) {
        switch (nv) {
            case 4: return k_apply<W, KIND, T, AC, CPLX, 4, STAGE, OCC, false, 0>;
            case 8: return k_apply<W, KIND, T, AC, CPLX, 8, STAGE, OCC, false, 0>;
        }
    }
    return nullptr;
}

// The compacted term loop exists for the table searches (sublattice coding,
// byte tables) with at most two vectors per pass.
template <int KIND>
constexpr bool has_compact() { return KIND == K_SUB || KIND == K_TAB; }

template <class W, int KIND, class T, class AC, bool CPLX, bool STAGE, bool OCC>
void (*apply_kernel_loop(int nv, bool compact))(ApplyArgs) {
    if constexpr (has_compact<KIND>())
        if (compact && nv <= 2) return apply_kernel<W, KIND, T, AC, CPLX, STAGE, OCC, true>(nv);
    return apply_kernel<W, KIND, T, AC, CPLX, STAGE, OCC, false>(nv);
}

template <class W, int KIND, class T, class AC, bool CPLX, int XR>
int launch_nv(int nv, const ApplyArgs &A, unsigned grid, unsigned block, size_t lds,
              hipStream_t st) {
    void (*f)(ApplyArgs) = nullptr;
    // only the sublattice kind has tables that may stay in global memory
    // the 64-VGPR copy only while a lane holds at most two accumulator
    // scalars: with more it spills them (complex 8-vector passes: 200 bytes)
    const bool occ = A.occ && nv * (CPLX ? 2 : 1) <= 2;
    const bool cmp = A.compact != 0;
    if constexpr (XR == 2 && CPLX) {
        set_error("internal: the trivial-character kernels serve real blocks");
        return XDG_EINVAL;
    } else if constexpr (XR != 0) {   // row loop, tables in LDS
        if (A.stage_sub)
            f = occ ? apply_kernel<W, KIND, T, AC, CPLX, true, true, false, XR>(nv)
                    : apply_kernel<W, KIND, T, AC, CPLX, true, false, false, XR>(nv);
    } else if (KIND != K_SUB || A.stage_sub)
        f = occ ? apply_kernel_loop<W, KIND, T, AC, CPLX, true, true>(nv, cmp)
                : apply_kernel_loop<W, KIND, T, AC, CPLX, true, false>(nv, cmp);
    else if constexpr (KIND == K_SUB)
        f = apply_kernel_loop<W, KIND, T, AC, CPLX, false, false>(nv, cmp);
    if (!f) {
        set_error("vectors per pass %d not in {1, 2, 4, 8} (at most 2 with the rank-addressed x, "
                  "whose tables must be in LDS)", nv);
        return XDG_EINVAL;
    }
    if (lds > 65536)
        XDG_TRY_HIP(hipFuncSetAttribute((const void *)f,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(f, dim3(grid), dim3(block), lds, st, A);
    XDG_TRY_HIP(hipGetLastError());
    return XDG_OK;
}

template <class W, int KIND, bool CPLX, int XR>
int launch_prec(bool single, bool acc64, int nv, const ApplyArgs &A, unsigned grid,
                unsigned block, size_t lds, hipStream_t st) {
    if (!single) return launch_nv<W, KIND, double, double, CPLX, XR>(nv, A, grid, block, lds, st);
    if (acc64) return launch_nv<W, KIND, float, double, CPLX, XR>(nv, A, grid, block, lds, st);
    return launch_nv<W, KIND, float, float, CPLX, XR>(nv, A, grid, block, lds, st);
}

template <int KIND, int XR = 0>
int launch_kind_impl(bool wide, bool single, bool acc64, bool cplx, int nv, const ApplyArgs &A,
                     unsigned grid, unsigned block, size_t lds, hipStream_t st) {
    if constexpr (KIND == K_U1) {
        if (cplx) {
            set_error("complex kernel requested for a U(1) block");
            return XDG_EINVAL;
        }
        return wide ? launch_prec<uint64_t, KIND, false, XR>(single, acc64, nv, A, grid, block, lds, st)
                    : launch_prec<uint32_t, KIND, false, XR>(single, acc64, nv, A, grid, block, lds, st);
    } else {
        if (wide)
            return cplx ? launch_prec<uint64_t, KIND, true, XR>(single, acc64, nv, A, grid, block, lds, st)
                        : launch_prec<uint64_t, KIND, false, XR>(single, acc64, nv, A, grid, block, lds, st);
        return cplx ? launch_prec<uint32_t, KIND, true, XR>(single, acc64, nv, A, grid, block, lds, st)
                    : launch_prec<uint32_t, KIND, false, XR>(single, acc64, nv, A, grid, block, lds, st);
    }
}

template <int KIND>
int launch_count_impl(bool wide, const ApplyArgs &A, unsigned grid, unsigned block, size_t lds,
                      hipStream_t st) {
    void (*f)(ApplyArgs) = wide ? k_count<uint64_t, KIND, true> : k_count<uint32_t, KIND, true>;
    if constexpr (KIND == K_SUB)
        if (!A.stage_sub)
            f = wide ? k_count<uint64_t, KIND, false> : k_count<uint32_t, KIND, false>;
    if (lds > 65536)
        XDG_TRY_HIP(hipFuncSetAttribute((const void *)f,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(f, dim3(grid), dim3(block), lds, st, A);
    XDG_TRY_HIP(hipGetLastError());
    return XDG_OK;
}

}  // namespace xdg
