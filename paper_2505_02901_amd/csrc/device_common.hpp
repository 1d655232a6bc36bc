// Device-side building blocks shared by the basis and apply kernels:
// bit rotations of ring states, the hash index of the basis, and the three
// representative searches (ring bit operations, sublattice coding, generic
// byte tables).  gfx950, wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xdg_internal.hpp"

namespace xdg {

enum : int { K_U1 = XDG_SEARCH_U1, K_AFF = XDG_SEARCH_AFFINE, K_SUB = XDG_SEARCH_SUBLATTICE,
             K_TAB = XDG_SEARCH_TABLE };

// ------------------------------------------------- global memory access --
// Loads and stores through the global address space.  A generic (flat)
// access is counted by the LDS counter as well, so the wait for an LDS table
// read that follows it would also wait for the HBM access; these helpers are
// for pointers known to address device memory from the allocator.
template <class T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const __attribute__((address_space(1))) T *)p;
}
// uint4 is a class whose copy constructor takes a generic reference, which
// would turn the load back into a flat one: load a native vector instead.
__device__ __forceinline__ uint4 gld(const uint4 *p) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 v = *(const __attribute__((address_space(1))) u32x4 *)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <class T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(__attribute__((address_space(1))) T *)p = v;
}
// Loads of read-only data at a wave-uniform address (the caller's promise):
// the address is taken from the first active lane and read through the
// constant address space, so the load is a scalar one into scalar registers.
// Read dword by dword (a class type's copy constructor would take a generic
// reference); the dwords merge into one wide scalar load.
template <class T>
__device__ __forceinline__ T sld(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "whole dwords");
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const __attribute__((address_space(4))) uint32_t *q =
        (const __attribute__((address_space(4))) uint32_t *)(((uint64_t)hi << 32) | lo);
    struct Words {
        uint32_t w[sizeof(T) / 4];
    } v;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) v.w[i] = q[i];
    return __builtin_bit_cast(T, v);
}

// ------------------------------------------------------------ bit helpers --
// Rotations of the low N bits of t by 0 <= a < N sites.  FULL: N is the
// width of W (a plain rotate); otherwise N < width, t < 2^N and mask = 2^N - 1,
// so that no shift reaches the width of W.
template <class W, bool FULL>
__host__ __device__ __forceinline__ W rot_r(W t, int a, int N, W mask) {
    if constexpr (FULL) {
        if constexpr (sizeof(W) == 4)
            return __builtin_rotateright32(t, (uint32_t)a);
        else
            return __builtin_rotateright64(t, (uint64_t)a);
    } else {
        return ((t >> a) | (t << (N - a))) & mask;
    }
}
template <class W, bool FULL>
__host__ __device__ __forceinline__ W rot_l(W t, int a, int N, W mask) {
    if constexpr (FULL) {
        if constexpr (sizeof(W) == 4)
            return __builtin_rotateleft32(t, (uint32_t)a);
        else
            return __builtin_rotateleft64(t, (uint64_t)a);
    } else {
        return ((t << a) | (t >> (N - a))) & mask;
    }
}

template <class W>
__host__ __device__ __forceinline__ W rotr_n(W t, int a, int N) {
    if (N == 8 * (int)sizeof(W)) return rot_r<W, true>(t, a, N, ~W(0));
    return rot_r<W, false>(t, a, N, (W(1) << N) - 1);
}

template <class W>
__host__ __device__ __forceinline__ W rev_n(W t, int N) {
    if constexpr (sizeof(W) == 4)
        return __builtin_bitreverse32(t) >> (32 - N);
    else
        return __builtin_bitreverse64(t) >> (64 - N);
}

// ------------------------------------------------------------- rank index --
// Colex rank of a state among the states of its popcount: the i-th set bit
// (from the bottom, i = 1, 2, ...) at site p contributes C(p, i).  It is
// summed per chunk of cb sites from tables indexed by (chunk k, below = set
// bits under the chunk, v = the chunk's bits).  For states of n_up set bits
// on N sites, below lies in [rank_lo(k), rank_hi(k)] for chunk k, and only
// those rows are stored, chunk after chunk: chunk k's row for `below` is
// rbase[k] + below.
//  * 32-bit states: four chunks of 8 sites and 4-byte entries (C(32, 16) <
//    2^32); the four reads are independent and issued together.
//  * wider states: nc chunks of cb sites (the widest whose table stays small
//    enough for LDS), read chunk after chunk; 4-byte entries that saturate at
//    2^32 - 1 when every rank of the block's basis states is below that (a
//    rank read as >= 2^32 - 1 lies beyond every index word), 8-byte entries
//    otherwise.
constexpr int RANK_CB32 = 8, RANK_NC32 = 4;

template <class W> struct RankEntry { using type = uint64_t; };
template <> struct RankEntry<uint32_t> { using type = uint32_t; };

__host__ __device__ inline int rank_lo(int N, int n_up, int cb, int k) {
    const int a = n_up - (N - k * cb);
    return a < 0 ? 0 : (a > n_up ? n_up : a);
}
__host__ __device__ inline int rank_hi(int n_up, int cb, int k) {
    return k * cb < n_up ? k * cb : n_up;
}

// T: the table (u32 entries for 32-bit states or e32, u64 otherwise).
template <class W>
__host__ __device__ __forceinline__ uint64_t colex_rank(const void *T, const RankLayout &L, W s) {
    if constexpr (sizeof(W) == 4) {
        const uint32_t *T32 = static_cast<const uint32_t *>(T);
        uint32_t e[RANK_NC32];
        uint32_t below = 0;
#pragma unroll
        for (int k = 0; k < RANK_NC32; ++k) {
            const uint32_t v = (s >> (k * RANK_CB32)) & 0xFFu;
            e[k] = T32[((uint32_t)(L.rbase[k] + (int)below) << RANK_CB32) | v];
            below += (uint32_t)__builtin_popcount(v);
        }
        return (uint64_t)((e[0] + e[1]) + (e[2] + e[3]));
    } else {
        // one chunk after the other (a loop the compiler keeps rolled: few
        // live registers); 4-byte entries are summed in 64 bits, so a rank
        // from 2^32 - 1 on reads as a value >= 2^32 - 1 (exact below)
        const int cb = L.cb, nc = L.nc;
        const uint32_t mask = (1u << cb) - 1;
        uint32_t below = 0;
        uint64_t r = 0;
        if (L.e32) {
            const uint32_t *T32 = static_cast<const uint32_t *>(T);
            for (int k = 0; k < nc; ++k) {
                const uint32_t v = (uint32_t)(s >> (k * cb)) & mask;
                r += T32[((uint32_t)(L.rbase[k] + (int)below) << cb) | v];
                below += (uint32_t)__builtin_popcount(v);
            }
        } else {
            const uint64_t *T64 = static_cast<const uint64_t *>(T);
            for (int k = 0; k < nc; ++k) {
                const uint32_t v = (uint32_t)(s >> (k * cb)) & mask;
                r += T64[((uint32_t)(L.rbase[k] + (int)below) << cb) | v];
                below += (uint32_t)__builtin_popcount(v);
            }
        }
        return r;
    }
}

// The colex rank of a wide state from 4-byte entries (layout with e32),
// summed with unsigned saturation: a rank of 2^32 - 1 or more (never the
// rank of a basis state) reads as 0xFFFFFFFF, every smaller rank exactly.
// Chunks inside the low 32 bits come from that word with 32-bit shifts.
template <class W>
__host__ __device__ __forceinline__ uint32_t colex_rank_sat(const uint32_t *T32,
                                                            const RankLayout &L, W s) {
    const int cb = L.cb, nc = L.nc;
    const int nlo = nc < 32 / cb ? nc : 32 / cb;
    const uint32_t lo = (uint32_t)s, mask = (1u << cb) - 1u;
    uint32_t below = 0, r = 0;
    int k = 0;
    for (; k < nlo; ++k) {
        const uint32_t v = (lo >> (k * cb)) & mask;
        r = __builtin_elementwise_add_sat(r, T32[(((uint32_t)L.rbase[k] + below) << cb) | v]);
        below += (uint32_t)__builtin_popcount(v);
    }
    for (; k < nc; ++k) {
        const uint32_t v = (uint32_t)((uint64_t)s >> (k * cb)) & mask;
        r = __builtin_elementwise_add_sat(r, T32[(((uint32_t)L.rbase[k] + below) << cb) | v]);
        below += (uint32_t)__builtin_popcount(v);
    }
    return r;
}

// Rank of a sublattice representative in the space of the states whose top
// block c is the minimal top of its own content (every representative's
// is): states ordered by c, then by the colex rank of the B bits below the
// top block.  top[c] is the first rank of top block c, ~0 when c is never a
// minimal top (the result is then ~0).  The bits below the top block lie in
// the low 32 bits (B <= 31), and their colex rank comes from T32: the rows
// of the chunk tables for the chunks below B (layout L), in 4-byte entries
// (every share of a site below 32 fits; the chunk across the boundary is
// read with its upper bits cleared, since a set bit's share depends only on
// its site and on the set bits below it).  Ascending states keep ascending
// ranks.
template <class W>
__host__ __device__ __forceinline__ uint32_t below_top_rank(const uint32_t *T32,
                                                            const RankLayout &L, int B, W s) {
    const int cb = L.cb;
    const uint32_t lo = (uint32_t)s & ((1u << B) - 1u), mask = (1u << cb) - 1u;
    const int nlc = (B + cb - 1) / cb;
    uint32_t below = 0, q = 0;
    for (int k = 0; k < nlc; ++k) {
        const uint32_t v = (lo >> (k * cb)) & mask;
        q += T32[(((uint32_t)L.rbase[k] + below) << cb) | v];
        below += (uint32_t)__builtin_popcount(v);
    }
    return q;
}

template <class W>
__host__ __device__ __forceinline__ uint64_t top_rank(const uint32_t *T32, const RankLayout &L,
                                                      int B, const uint64_t *top, W s) {
    const uint64_t base = top[(uint32_t)((uint64_t)s >> B)];
    return base == ~0ull ? ~0ull : base + below_top_rank<W>(T32, L, B, s);
}

// The same with 4-byte first ranks (every rank below 2^32 - 1; 0xFFFFFFFF
// marks a top block that is never a minimal top).
template <class W>
__host__ __device__ __forceinline__ uint64_t top_rank32(const uint32_t *T32, const RankLayout &L,
                                                        int B, const uint32_t *top, W s) {
    const uint32_t base = top[(uint32_t)((uint64_t)s >> B)];
    return base == 0xFFFFFFFFu ? ~0ull : (uint64_t)base + below_top_rank<W>(T32, L, B, s);
}

// Position of the state of colex rank r, or -1: words[r / 32] holds the
// number of basis states of smaller rank (valid in words holding a state)
// and one bit per rank.
__device__ __forceinline__ int64_t rank_find(const uint2 *words, uint64_t n_words, uint64_t r) {
    const uint64_t w = r >> 5;
    if (w >= n_words) return -1;
    // one 8-byte read of {count, bits}, no branch on the bit: both halves
    // come back with the same load
    const uint64_t e = gld(reinterpret_cast<const uint64_t *>(words) + w);
    const uint32_t cnt = (uint32_t)e, bits = (uint32_t)(e >> 32);
    const uint32_t b = (uint32_t)r & 31u;
    const int64_t idx = (int64_t)cnt + __popc(bits & ((1u << b) - 1u));
    return ((bits >> b) & 1u) ? idx : -1;
}

// The same for ranks below 2^32 in 32-bit arithmetic (positions below 2^32).
__device__ __forceinline__ int64_t rank_find_r32(const uint2 *words, uint32_t n_words, uint32_t r) {
    const uint32_t w = r >> 5;
    if (w >= n_words) return -1;
    const uint64_t e = gld(reinterpret_cast<const uint64_t *>(words) + w);
    const uint32_t cnt = (uint32_t)e, bits = (uint32_t)(e >> 32);
    const uint32_t b = r & 31u;
    const uint32_t idx = cnt + __popc(bits & ((1u << b) - 1u));
    return ((bits >> b) & 1u) ? (int64_t)idx : -1;
}

// The same for ranks and positions below 2^31 (32-bit states: every colex
// rank is below C(32, 16)), in 32-bit arithmetic.
__device__ __forceinline__ int32_t rank_find32(const uint2 *words, uint32_t n_words, uint32_t r) {
    const uint32_t w = r >> 5;
    if (w >= n_words) return -1;
    const uint64_t e = gld(reinterpret_cast<const uint64_t *>(words) + w);
    const uint32_t cnt = (uint32_t)e, bits = (uint32_t)(e >> 32);
    const uint32_t b = r & 31u;
    const int32_t idx = (int32_t)(cnt + __popc(bits & ((1u << b) - 1u)));
    return ((bits >> b) & 1u) ? idx : -1;
}

// ------------------------------------------------------------- hash index --
// Open addressing over 64-byte lines; a lookup reads one line in the common
// case.  A line holds 8 (key u32, value u32) or 5 (key u64, value u32) pairs.
struct alignas(64) Line32 {
    uint32_t k[8];
    uint32_t v[8];
};
struct alignas(64) Line64 {
    uint64_t k[5];
    uint32_t v[5];
    uint32_t pad;
};
static_assert(sizeof(Line32) == 64 && sizeof(Line64) == 64, "line size");

template <class W>
__host__ __device__ __forceinline__ uint64_t hash_line(W key, uint64_t n_lines) {
    uint32_t h;
    if constexpr (sizeof(W) == 4)
        h = (uint32_t)key * 0x9E3779B1u;
    else
        h = (uint32_t)(((uint64_t)key * 0x9E3779B97F4A7C15ull) >> 32);
    return ((uint64_t)h * n_lines) >> 32;
}

template <class W>
__device__ __forceinline__ int64_t hash_find(const void *table, uint64_t n_lines, W empty, W key) {
    uint64_t line = hash_line<W>(key, n_lines);
    for (;;) {
        if constexpr (sizeof(W) == 4) {
            const uint4 *p = reinterpret_cast<const uint4 *>(
                reinterpret_cast<const Line32 *>(table) + line);
            const uint4 k0 = gld(p), k1 = gld(p + 1), v0 = gld(p + 2), v1 = gld(p + 3);
            const uint32_t ks[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
            const uint32_t vs[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
            int64_t found = -1;
            bool any_empty = false;
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                if (ks[s] == key) found = vs[s];
                any_empty |= ks[s] == empty;
            }
            if (found >= 0) return found;
            if (any_empty) return -1;
        } else {
            const uint4 *p = reinterpret_cast<const uint4 *>(
                reinterpret_cast<const Line64 *>(table) + line);
            const uint4 a = gld(p), b = gld(p + 1), c = gld(p + 2), d = gld(p + 3);
            const uint64_t ks[5] = {((uint64_t)a.y << 32) | a.x, ((uint64_t)a.w << 32) | a.z,
                                    ((uint64_t)b.y << 32) | b.x, ((uint64_t)b.w << 32) | b.z,
                                    ((uint64_t)c.y << 32) | c.x};
            const uint32_t vs[5] = {c.z, c.w, d.x, d.y, d.z};
            int64_t found = -1;
            bool any_empty = false;
#pragma unroll
            for (int s = 0; s < 5; ++s) {
                if (ks[s] == key) found = vs[s];
                any_empty |= ks[s] == empty;
            }
            if (found >= 0) return found;
            if (any_empty) return -1;
        }
        line = line + 1 == n_lines ? 0 : line + 1;
    }
}

// ---------------------------------------------------- search: ring (affine) --
// Element g: image = rotr_N(t, a) (eps = +1) or rotr_N(rev_N(t), a) (eps = -1).
template <class W>
__device__ __forceinline__ void aff_search(const AffineElem *aff, int n_sym, int N, W t, W &best,
                                           int &u, int &cnt) {
    const W rt = rev_n<W>(t, N);
    best = ~W(0);
    u = 0;
    cnt = 0;
    for (int g = 0; g < n_sym; ++g) {
        const AffineElem e = aff[g];
        const W img = rotr_n<W>(e.eps > 0 ? t : rt, e.a, N);
        if (img < best) {
            best = img;
            u = g;
            cnt = 1;
        } else if (img == best) {
            ++cnt;
        }
    }
}

// ---------------------------------------- search: full ring of rotations --
// For a group holding every rotation i -> i + a (and optionally every
// reflection i -> a - i), the image under rotation a is rotr_N(t, a); read
// from its top bit it is t read downward from site a - 1.  The smallest image
// therefore begins with a longest run of zeros of t, so only the tops of the
// maximal zero runs need a full comparison.  With z = ~t, let y_m have bit p
// set iff sites p, p-1, .., p-m+1 (cyclically) of t are all down: y_1 = z and
// y_{m+n} = y_m & rotl(y_n, m).  Doubling gives p_j = y_{2^j}; the longest
// run L and y_L then follow by binary lifting, y <- p_j & rotl(y, 2^j) while
// that stays nonzero, for j from high to low: a fixed number of steps, every
// rotation by a constant, no divergence.  All minimising rotations are among
// the set bits of y_L, so the first minimising element and the number of
// minimisers (= |Stab|) come out exact.
//
// Scans the rotations of t; merges into (best, u, cnt) using gidx[a] as the
// group index of rotation a.  FIRST: (best, u, cnt) hold nothing yet and are
// set from the first candidate.
template <class W, bool FULL, bool FIRST>
__host__ __device__ __forceinline__ void ring_scan_t(W t, int N, const int16_t *gidx, W &best,
                                                     int &u, int &cnt) {
    constexpr int J = sizeof(W) == 4 ? 5 : 6;   // 2^J > the longest run < N
    const W mask = FULL ? ~W(0) : ((W(1) << N) - 1);
    const W z = ~t & mask;
    W y;
    if (z == 0 || z == mask) {
        y = mask;                      // all rotations give the same image
    } else {
        W p[J];                        // p[j] = y_{2^j}
        p[0] = z;
#pragma unroll
        for (int j = 1; j < J; ++j) {
            const int h = 1 << (j - 1);
            p[j] = (FULL || h < N) ? (p[j - 1] & rot_l<W, FULL>(p[j - 1], h, N, mask)) : W(0);
        }
        y = mask;                      // y_0
#pragma unroll
        for (int j = J - 1; j >= 0; --j) {
            const int h = 1 << j;
            if (FULL || h < N) {
                const W c = p[j] & rot_l<W, FULL>(y, h, N, mask);
                y = c ? c : y;
            }
        }
    }
    auto take = [&](int pos, bool first) {
        const int a = pos + 1 == N ? 0 : pos + 1;
        const W img = rot_r<W, FULL>(t, a, N, mask);
        const int g = gidx[a];
        if (first) {
            best = img;
            u = g;
            cnt = 1;
        } else if (img < best) {
            best = img;
            u = g;
            cnt = 1;
        } else if (img == best) {
            ++cnt;
            u = g < u ? g : u;
        }
    };
    auto ctz = [](W v) -> int {
        if constexpr (sizeof(W) == 4)
            return __builtin_ctz(v);
        else
            return __builtin_ctzll(v);
    };
    if constexpr (FIRST) {             // y has at least one bit
        take(ctz(y), true);
        y &= y - 1;
    }
    while (y) {
        take(ctz(y), false);
        y &= y - 1;
    }
}

template <class W, bool FIRST>
__host__ __device__ __forceinline__ void ring_scan(W t, int N, const int16_t *gidx, W &best,
                                                   int &u, int &cnt) {
    if (N == 8 * (int)sizeof(W))
        ring_scan_t<W, true, FIRST>(t, N, gidx, best, u, cnt);
    else
        ring_scan_t<W, false, FIRST>(t, N, gidx, best, u, cnt);
}

// ring = 1: rotations only; ring = 2: rotations and reflections.
// gidx[a] (rotation a) and gidx[N + a] (reflection image rotr_N(rev_N(t), a)).
template <class W>
__host__ __device__ __forceinline__ void ring_search(const int16_t *gidx, int ring, int N, W t,
                                                     W &best, int &u, int &cnt) {
    ring_scan<W, true>(t, N, gidx, best, u, cnt);
    if (ring == 2) ring_scan<W, false>(rev_n<W>(t, N), N, gidx + N, best, u, cnt);
}

// Representative test for enumeration: false as soon as some image is smaller.
// On true, stab = |Stab(s)| and (cr, ci) = sum of chi over the stabiliser.
template <class W>
__device__ __forceinline__ bool aff_is_rep(const AffineElem *aff, int n_sym, int N, W s,
                                           const double2 *chi, int &stab, double &cr, double &ci) {
    const W rs = rev_n<W>(s, N);
    stab = 0;
    cr = 0.0;
    ci = 0.0;
    for (int g = 0; g < n_sym; ++g) {
        const AffineElem e = aff[g];
        const W img = rotr_n<W>(e.eps > 0 ? s : rs, e.a, N);
        if (img < s) return false;
        if (img == s) {
            ++stab;
            cr += chi[g].x;
            ci += chi[g].y;
        }
    }
    return true;
}

// ------------------------------------------------ search: sublattice coding --
// Sites come in n_s blocks of m bits; every group element maps blocks onto
// blocks, so the top block of g.t is a lookup of one block of t.  The
// smallest possible top block over the whole group is the minimum of
// mintop[k][chunk_k(t)] over the source blocks k; only the elements listed
// for the blocks reaching that minimum can produce the representative, and
// only for them is the full image assembled, block by block from the top,
// abandoning an element as soon as its image prefix exceeds the best one.
struct SubCtx {
    const uint16_t *mintop;    // [n_s][V]
    const uint32_t *cand_off;  // [n_s*V + 1]
    const uint16_t *cand_list;
    const uint32_t *sp;        // [n_sym][n_s]: (offset in tperm of the tables of the block
                               // permutation feeding block a) << 8 | first bit of its source block
    const uint16_t *tperm;     // [n_perm][2][E]
    int n_s, m, pb;            // E = 1 << pb
};

template <class W>
__device__ __forceinline__ uint32_t chunk_of(W t, int k, int m, uint32_t vmask) {
    return (uint32_t)(t >> (k * m)) & vmask;
}

// image bits of a block of g.t from its packed entry w = sp[g][a] (two
// half-chunk lookups)
template <class W>
__device__ __forceinline__ uint32_t sub_block(const SubCtx &C, uint32_t w, W t, uint32_t vmask) {
    const uint32_t v = (uint32_t)(t >> (w & 0xFFu)) & vmask;
    const uint16_t *tp = C.tperm + (w >> 8);
    const uint32_t lo = (1u << C.pb) - 1;
    return (uint32_t)tp[v & lo] | tp[lo + 1 + (v >> C.pb)];
}

// the n_s packed entries of element g; four blocks come in one 16-byte read
template <int NS>
struct SubEntries {
    uint32_t w[NS > 0 ? NS : 1];
    const uint32_t *p;
    __device__ __forceinline__ SubEntries(const SubCtx &C, int g, int ns) {
        p = C.sp + g * ns;
        if constexpr (NS == 4) {
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            const u32x4 q = *reinterpret_cast<const u32x4 *>(p);
            w[0] = q.x;
            w[1] = q.y;
            w[2] = q.z;
            w[3] = q.w;
        }
    }
    __device__ __forceinline__ uint32_t operator[](int a) const {
        if constexpr (NS == 4)
            return w[a];
        else
            return p[a];
    }
};

// NS > 0: the number of blocks is a compile-time constant (loops unrolled);
// NS = 0: taken from C.n_s.
template <class W, int NS>
__device__ __forceinline__ void sub_search(const SubCtx &C, W t, W &best, int &u, int &cnt) {
    const int m = C.m;
    const int ns = NS > 0 ? NS : C.n_s, top = ns - 1;
    const uint32_t V = 1u << m, vmask = V - 1;
    uint32_t mt = 0xFFFFu;
#pragma unroll
    for (int k = 0; k < ns; ++k) {
        const uint32_t v = C.mintop[k * V + chunk_of<W>(t, k, m, vmask)];
        mt = v < mt ? v : mt;
    }
    best = ~W(0);
    u = 0x7fffffff;
    cnt = 0;
#pragma unroll
    for (int k = 0; k < ns; ++k) {
        const uint32_t e = k * V + chunk_of<W>(t, k, m, vmask);
        if (C.mintop[e] != mt) continue;
        const uint32_t q1 = C.cand_off[e + 1];
        for (uint32_t q = C.cand_off[e]; q < q1; ++q) {
            const int g = C.cand_list[q];
            const SubEntries<NS> ent(C, g, ns);
            // blocks from the top down; while the image agrees with the best
            // one so far, each block is compared with the best one's block
            W img = (W)mt << (top * m);
            bool eq = true, lose = false;
#pragma unroll
            for (int a = top - 1; a >= 0; --a) {
                const uint32_t v = sub_block<W>(C, ent[a], t, vmask);
                img |= (W)v << (a * m);
                if (eq) {
                    const uint32_t bb = (uint32_t)(best >> (a * m)) & vmask;
                    if (v > bb) {
                        lose = true;
                        break;
                    }
                    eq = v == bb;
                }
            }
            if (lose) continue;
            if (img < best) {
                best = img;
                u = g;
                cnt = 1;
            } else if (img == best) {
                ++cnt;
            }
        }
    }
}

template <class W>
__device__ __forceinline__ bool sub_is_rep(const SubCtx &C, W s, const double2 *chi, int &stab,
                                           double &cr, double &ci) {
    const int m = C.m, ns = C.n_s, top = ns - 1;
    const uint32_t V = 1u << m, vmask = V - 1;
    const uint32_t ct = chunk_of<W>(s, top, m, vmask);
    for (int k = 0; k < ns; ++k)
        if (C.mintop[k * V + chunk_of<W>(s, k, m, vmask)] < ct) return false;
    stab = 0;
    cr = 0.0;
    ci = 0.0;
    for (int k = 0; k < ns; ++k) {
        const uint32_t e = k * V + chunk_of<W>(s, k, m, vmask);
        if (C.mintop[e] != ct) continue;
        const uint32_t q1 = C.cand_off[e + 1];
        for (uint32_t q = C.cand_off[e]; q < q1; ++q) {
            const int g = C.cand_list[q];
            const uint32_t *sp = C.sp + g * ns;
            int cmp = 0;   // -1: image < s, +1: image > s
            for (int a = top - 1; a >= 0; --a) {
                const uint32_t v = sub_block<W>(C, sp[a], s, vmask);
                const uint32_t sv = chunk_of<W>(s, a, m, vmask);
                if (v != sv) {
                    cmp = v < sv ? -1 : 1;
                    break;
                }
            }
            if (cmp < 0) return false;
            if (cmp == 0) {
                ++stab;
                cr += chi[g].x;
                ci += chi[g].y;
            }
        }
    }
    return true;
}

// ------------------------------------- sublattice coding, packed form --
// For four blocks of m <= 10 bits whose half-chunk tables (E = 2^pb entries,
// 3 <= pb <= 5) sit in LDS at a 4E-aligned address.  A state enters as two
// words of 7-bit fields: field k of lo2 is 2 (chunk_k mod E) and field k of
// hi2 is 2 (E + chunk_k / E), the byte offsets of block k's two half-table
// entries within one permutation's 4E bytes of tables.  Each (element,
// block) entry w holds the LDS address of the permutation's tables (a
// multiple of 4E) or'ed with 7 times the source block, so one bit-field
// extract of the packed word at w's low five bits and one and-or with w give
// a table address.  Every candidate's top block is the minimal top, so the
// three lower image blocks (at most 30 bits) decide as one 32-bit word.
typedef __attribute__((address_space(3))) const uint16_t lds_u16;

// A state's key for the packed search: its four block-table indices
// e_k = k 2^m + chunk_k and its two packed words.
struct SubKey {
    uint32_t e[4];
    uint32_t lo2, hi2;
};

template <class W>
__device__ __forceinline__ SubKey sub_key(W t, int m, int pb) {
    const uint32_t E = 1u << pb, V = 1u << m, vmask = V - 1;
    SubKey K;
    K.lo2 = 0;
    K.hi2 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t c = chunk_of<W>(t, k, m, vmask);
        K.e[k] = k * V + c;
        K.lo2 |= ((c & (E - 1)) << 1) << (7 * k);
        K.hi2 |= ((E + (c >> pb)) << 1) << (7 * k);
    }
    return K;
}

// the key of a state with two sites exchanged (x: that bond's bits)
__device__ __forceinline__ SubKey sub_key_flip(const SubKey &K, const BondX &x) {
    SubKey T;
#pragma unroll
    for (int k = 0; k < 4; ++k) T.e[k] = K.e[k] ^ x.ek[k];
    T.lo2 = K.lo2 ^ x.plo;
    T.hi2 = K.hi2 ^ x.phi;
    return T;
}

// C.sp holds the packed (element, block) entries; amask = ~(4E - 1).
// KEEP_U = false: the element reaching the minimum is not kept (u = 0).
template <class W, bool KEEP_U = true>
__device__ __forceinline__ void sub_search_packed(const SubCtx &C, uint32_t amask,
                                                  const SubKey &K, W &best, int &u, int &cnt) {
    const int m = C.m;
    const uint32_t *e = K.e;
    const uint32_t lo2 = K.lo2, hi2 = K.hi2;
    uint32_t mv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) mv[k] = C.mintop[e[k]];
    const uint32_t mt = min(min(mv[0], mv[1]), min(mv[2], mv[3]));
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    uint32_t bl = 0xFFFFFFFFu, bu = 0x7fffffffu, bc = 0;
    auto candidate = [&](uint32_t g) {
        const u32x4 w = *reinterpret_cast<const u32x4 *>(C.sp + 4 * g);
        uint32_t v[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // the fields are below 4E: bitop3 table 0xE4 takes wa's bits
            // under amask and the field's below it
            const uint32_t wa = w[a];
            const uint32_t la =
                __builtin_amdgcn_bitop3_b32(wa, __builtin_amdgcn_ubfe(lo2, wa, 7), amask, 0xE4);
            const uint32_t ha =
                __builtin_amdgcn_bitop3_b32(wa, __builtin_amdgcn_ubfe(hi2, wa, 7), amask, 0xE4);
            // the two halves set disjoint bits: an add keeps the sum in 32 bits
            v[a] = (uint32_t)*(lds_u16 *)la + (uint32_t)*(lds_u16 *)ha;
        }
        const uint32_t img = (((v[2] << m) | v[1]) << m) | v[0];
        const bool lt = img < bl, eq = img == bl;
        if constexpr (KEEP_U) bu = lt ? g : bu;
        bc = lt ? 1u : bc + (eq ? 1u : 0u);
        bl = lt ? img : bl;
    };
    // the list of the lowest block reaching mt (most terms have one such
    // block): one paired read of its offsets, then one loop
    const bool h0 = mv[0] == mt, h1 = mv[1] == mt, h2 = mv[2] == mt;
    const uint32_t ef = h0 ? e[0] : h1 ? e[1] : h2 ? e[2] : e[3];
    const uint32_t q0 = C.cand_off[ef], n = C.cand_off[ef + 1] - q0;
    const uint16_t *cl = C.cand_list + q0;
    for (uint32_t i = 0; i < n; ++i) candidate(cl[i]);
    // the lists of further blocks reaching mt
    const int kf = h0 ? 0 : h1 ? 1 : h2 ? 2 : 3;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        if (k > kf && mv[k] == mt) {
            const uint32_t r1 = C.cand_off[e[k] + 1];
            for (uint32_t q = C.cand_off[e[k]]; q < r1; ++q) candidate(C.cand_list[q]);
        }
    }
    best = ((W)mt << (3 * m)) | (W)bl;
    u = KEEP_U ? (int)bu : 0;
    cnt = (int)bc;
}

// ---------------------------------------------------- search: byte tables --
template <class W>
__device__ __forceinline__ W tab_image(const uint64_t *tab, int n_chunks, int g, W t) {
    W img = 0;
    const uint64_t *tg = tab + (size_t)g * n_chunks * 256;
    for (int c = 0; c < n_chunks; ++c) img |= (W)tg[c * 256 + ((uint32_t)(t >> (8 * c)) & 255u)];
    return img;
}

template <class W>
__device__ __forceinline__ void tab_search(const uint64_t *tab, int n_chunks, int n_sym, W t,
                                           W &best, int &u, int &cnt) {
    best = ~W(0);
    u = 0;
    cnt = 0;
    for (int g = 0; g < n_sym; ++g) {
        const W img = tab_image<W>(tab, n_chunks, g, t);
        if (img < best) {
            best = img;
            u = g;
            cnt = 1;
        } else if (img == best) {
            ++cnt;
        }
    }
}

template <class W>
__device__ __forceinline__ bool tab_is_rep(const uint64_t *tab, int n_chunks, int n_sym, W s,
                                           const double2 *chi, int &stab, double &cr, double &ci) {
    stab = 0;
    cr = 0.0;
    ci = 0.0;
    for (int g = 0; g < n_sym; ++g) {
        const W img = tab_image<W>(tab, n_chunks, g, s);
        if (img < s) return false;
        if (img == s) {
            ++stab;
            cr += chi[g].x;
            ci += chi[g].y;
        }
    }
    return true;
}

// Colexicographic unranking of popcount-n states (ascending integer order):
// rank r = sum_k C(p_k, k+1) over the set bits p_0 < p_1 < ...
template <class W>
__device__ __forceinline__ W unrank_colex(uint64_t r, int N, int n, const uint64_t *binom) {
    W s = 0;
    int p = N - 1;
    for (int k = n; k >= 1; --k) {
        while (binom[p * 65 + k] > r) --p;
        s |= W(1) << p;
        r -= binom[p * 65 + k];
        --p;
    }
    return s;
}

// next larger integer with the same popcount
template <class W>
__device__ __forceinline__ W next_same_popcount(W s) {
    const W lowest = s & (~s + 1);
    const W ripple = s + lowest;
    int tz;
    if constexpr (sizeof(W) == 4)
        tz = __builtin_ctz(s);
    else
        tz = __builtin_ctzll(s);
    return ripple | (((s ^ ripple) >> 2) >> tz);
}

}  // namespace xdg
