// Host-side checks of two integer building blocks of the apply and index
// kernels, compiled from the library's own sources and run on the CPU:
//  * the colex rank read from the chunk tables equals the plain colex rank
//    (sum over the i-th set bit at site p of C(p, i)) for every N <= 64 and
//    every n_up, on random states and the smallest and largest ones;
//  * the rank among the states with an admissible top block (rank-addressed
//    vectors) equals the position in the ascending list of those states;
//  * the ring representative search (longest zero run by doubling and
//    binary lifting, then the candidate rotations) equals a scan of all N
//    rotations (and N reflections) written with plain per-bit loops.
// Prints "bad <count>" and exits nonzero on any mismatch.
#include "basis.hip"

#include <cstdio>
#include <random>

using namespace xdg;

static uint64_t binom_plain(int n, int k) {
    if (k < 0 || k > n) return 0;
    unsigned __int128 r = 1;   // r = C(n - k + i, i) after step i; the product needs 128 bits
    for (int i = 1; i <= k; ++i) r = r * (unsigned)(n - k + i) / (unsigned)i;
    return (uint64_t)r;
}

static uint64_t colex_plain(uint64_t s) {
    uint64_t r = 0;
    int i = 0;
    for (int p = 0; p < 64; ++p)
        if ((s >> p) & 1) r += binom_plain(p, ++i);
    return r;
}

// one layout: 32-bit states; wide states with the layout chosen for the
// largest rank of the sector, forced 8-byte entries, and forced saturating
// 4-byte entries (ranks from 2^32 - 1 on must read as at least 2^32 - 1)
template <class W>
static int check_rank_layout(int N, int n_up, uint64_t max_rank, std::mt19937_64 &g) {
    const bool wide = sizeof(W) == 8;
    const RankLayout L = rank_layout(N, n_up, wide, max_rank);
    std::vector<uint32_t> T32;
    std::vector<uint64_t> T64;
    const void *T;
    if (L.e32) {
        rank_tables<uint32_t>(N, n_up, L, T32);
        T = T32.data();
    } else {
        rank_tables<uint64_t>(N, n_up, L, T64);
        T = T64.data();
    }
    int bad = 0;
    std::vector<int> perm(N);
    for (int it = 0; it < 200; ++it) {
        for (int i = 0; i < N; ++i) perm[i] = i;
        for (int i = 0; i < n_up; ++i) std::swap(perm[i], perm[i + (int)(g() % (uint64_t)(N - i))]);
        uint64_t s = 0;
        for (int i = 0; i < n_up; ++i) s |= 1ull << perm[i];
        const uint64_t low = n_up ? (~0ull >> (64 - n_up)) : 0;
        if (it == 0) s = low;
        if (it == 1) s = low << (N - n_up);
        const uint64_t want = colex_plain(s), got = colex_rank<W>(T, L, (W)s);
        // saturating 4-byte entries: exact below 2^32 - 1, at least that above;
        // the 32-bit saturating sum: exact below, 0xFFFFFFFF above
        if (wide && L.e32 && want >= 0xFFFFFFFFull) {
            if (got < 0xFFFFFFFFull) ++bad;
        } else if (got != want) {
            ++bad;
        }
        if (wide && L.e32) {
            const uint32_t sat = colex_rank_sat<W>(T32.data(), L, (W)s);
            if (sat != (want >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)want)) ++bad;
        }
    }
    return bad;
}

template <class W>
static int check_rank(int N, int n_up, std::mt19937_64 &g) {
    const uint64_t low = n_up ? (~0ull >> (64 - n_up)) : 0;
    const uint64_t top = colex_plain(low << (N - n_up));
    int bad = check_rank_layout<W>(N, n_up, top, g);
    if (sizeof(W) == 8) {
        bad += check_rank_layout<W>(N, n_up, ~0ull, g);   // 8-byte entries
        bad += check_rank_layout<W>(N, n_up, 0, g);       // saturating 4-byte entries
    }
    return bad;
}

static uint64_t rot_plain(uint64_t t, int a, int N) {   // site i -> i - a (cyclic)
    uint64_t r = 0;
    for (int i = 0; i < N; ++i)
        if ((t >> i) & 1) r |= 1ull << ((i - a + N) % N);
    return r;
}

static uint64_t rev_plain(uint64_t t, int N) {
    uint64_t r = 0;
    for (int i = 0; i < N; ++i)
        if ((t >> i) & 1) r |= 1ull << (N - 1 - i);
    return r;
}

template <class W>
static int check_ring(int N, std::mt19937_64 &g) {
    std::vector<int16_t> gidx(2 * N);
    for (int a = 0; a < 2 * N; ++a) gidx[a] = (int16_t)((a * 7 + 3) % (2 * N));
    int bad = 0;
    for (int it = 0; it < 600; ++it) {
        uint64_t t = g();
        if (it % 3 == 1) t &= g();
        if (it % 3 == 2) t |= g();
        if (N < 64) t &= (1ull << N) - 1;
        if (it == 0) t = 0;
        if (it == 1) t = N < 64 ? (1ull << N) - 1 : ~0ull;
        for (int ring = 1; ring <= 2; ++ring) {
            W best;
            int u, cnt;
            ring_search<W>(gidx.data(), ring, N, (W)t, best, u, cnt);
            uint64_t b = ~0ull;
            int bu = 1 << 30, bc = 0;
            for (int e = 0; e < ring * N; ++e) {
                const uint64_t img = rot_plain(e < N ? t : rev_plain(t, N), e % N, N);
                if (img < b) {
                    b = img;
                    bu = gidx[e];
                    bc = 1;
                } else if (img == b) {
                    ++bc;
                    bu = gidx[e] < bu ? gidx[e] : bu;
                }
            }
            if ((uint64_t)best != b || u != bu || cnt != bc) ++bad;
        }
    }
    return bad;
}

// The rank of a state among the states whose top block (the highest of four
// blocks of m = N / 4 sites) lies in an admissible set, read from the chunk
// tables: for N <= 20, every state of the popcount in ascending order, where
// the admissible ones must take the ranks 0, 1, 2, ... and the others ~0; for
// every N, random states against the first rank of their top block plus the
// plain colex rank of the bits below it.  The admissible set is random (the
// library's is the set of minimal tops); 4-byte and 8-byte table entries.
template <class W>
static int check_top_rank(int N, int n_up, uint64_t max_rank, std::mt19937_64 &g) {
    const int m = N / 4, B = 3 * m;
    if (m < 1 || 4 * m != N || B > 31) return 0;
    const RankLayout L = rank_layout(N, n_up, sizeof(W) == 8, max_rank);
    // the library's 4-byte rows of the chunks below B, from either entry size
    std::vector<uint32_t> T32, low;
    std::vector<uint64_t> T64;
    if (L.e32) {
        rank_tables<uint32_t>(N, n_up, L, T32);
        xr_lower_rows(L, T32.data(), B, n_up, low);
    } else {
        rank_tables<uint64_t>(N, n_up, L, T64);
        xr_lower_rows(L, T64.data(), B, n_up, low);
    }
    const uint32_t *T = low.data();
    const uint32_t V = 1u << m;
    std::vector<uint64_t> top(V, ~0ull);
    uint64_t total = 0;
    for (uint32_t c = 0; c < V; ++c) {
        if (g() % 3 == 0) continue;
        const int k = n_up - __builtin_popcount(c);
        if (k < 0 || k > B) continue;
        top[c] = total;
        total += binom_plain(B, k);
    }
    int bad = 0;
    if (N <= 20 && n_up > 0 && n_up < N) {
        uint64_t next = 0;
        for (uint64_t s = (1ull << n_up) - 1; s < (1ull << N);) {
            const uint64_t r = top_rank<W>(T, L, B, top.data(), (W)s);
            if (top[s >> B] == ~0ull)
                bad += r != ~0ull;
            else
                bad += r != next++;
            const uint64_t c = s & (~s + 1), q = s + c;   // next state of the popcount
            s = (((q ^ s) >> 2) / c) | q;
        }
        bad += next != total;
    }
    std::vector<int> perm(N);
    for (int it = 0; it < 200; ++it) {
        for (int i = 0; i < N; ++i) perm[i] = i;
        for (int i = 0; i < n_up; ++i) std::swap(perm[i], perm[i + (int)(g() % (uint64_t)(N - i))]);
        uint64_t s = 0;
        for (int i = 0; i < n_up; ++i) s |= 1ull << perm[i];
        const uint64_t base = top[s >> B];
        const uint64_t want = base == ~0ull ? ~0ull : base + colex_plain(s & ((1ull << B) - 1));
        uint64_t got = top_rank<W>(T, L, B, top.data(), (W)s);
        if (total < 0xFFFFFFFFull) {   // the 4-byte first ranks give the same
            std::vector<uint32_t> t32(V);
            for (uint32_t c = 0; c < V; ++c) t32[c] = top[c] == ~0ull ? 0xFFFFFFFFu : (uint32_t)top[c];
            if (top_rank32<W>(T, L, B, t32.data(), (W)s) != got) got = ~1ull;
        }
        if (got != want) {
            if (bad < 5)
                printf("top rank N %d n_up %d s %llx: %llu, want %llu\n", N, n_up,
                       (unsigned long long)s, (unsigned long long)got, (unsigned long long)want);
            ++bad;
        }
    }
    return bad;
}

int main() {
    std::mt19937_64 g(20250505);
    int bad = 0;
    for (int N = 1; N <= 64; ++N)
        for (int n = 0; n <= N; ++n)
            bad += N <= 32 ? check_rank<uint32_t>(N, n, g) : check_rank<uint64_t>(N, n, g);
    for (int N = 4; N <= 40; N += 4)
        for (int n = 0; n <= N; ++n)
            for (uint64_t mr : {0ull, ~0ull})   // 4-byte, then 8-byte entries (wide states)
                bad += N <= 32 ? (mr ? 0 : check_top_rank<uint32_t>(N, n, mr, g))
                               : check_top_rank<uint64_t>(N, n, mr, g);
    for (int N = 2; N <= 64; ++N) {
        if (N <= 32) bad += check_ring<uint32_t>(N, g);
        bad += check_ring<uint64_t>(N, g);
    }
    printf("bad %d\n", bad);
    return bad != 0;
}
