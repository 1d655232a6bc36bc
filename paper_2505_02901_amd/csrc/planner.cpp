// Host-side planning for a sector: validation of the permutation group and
// its characters (Sec. 3.10.1, 3.10.2), invariance of the bond list
// (well-defined quantum numbers, Sec. 3.6 / 3.10), choice of the
// representative-search kind and construction of its lookup tables
// (Sec. 5.1 backends, Sec. 5.2: lookup tables for the symmetry action,
// sublattice coding).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>

#include "xdg_internal.hpp"

namespace xdg {

namespace {
thread_local std::string g_err;

struct VecHash {
    size_t operator()(const std::vector<int32_t> &v) const {
        uint64_t h = 1469598103934665603ull;
        for (int32_t x : v) {
            h ^= (uint64_t)(uint32_t)x;
            h *= 1099511628211ull;
        }
        return (size_t)h;
    }
};
}  // namespace

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

const char *get_error() { return g_err.c_str(); }

uint64_t binomial(int n, int k) {
    static uint64_t t[65][65];
    static bool ready = false;
    if (!ready) {
        for (int a = 0; a <= 64; ++a) {
            t[a][0] = 1;
            for (int b = 1; b <= a; ++b) t[a][b] = t[a - 1][b - 1] + (b < a ? t[a - 1][b] : 0);
        }
        ready = true;
    }
    if (n < 0 || k < 0 || k > n || n > 64) return 0;
    return t[n][k];
}

// --------------------------------------------------------- group checks --
int validate_group(int n_sites, int n_sym, const int32_t *perm, const double *chi) {
    if (n_sites < 1 || n_sites > 64) {
        set_error("n_sites = %d outside [1, 64]", n_sites);
        return XDG_EINVAL;
    }
    if (n_sym == 0) return XDG_OK;
    if (n_sym < 0 || !perm) {
        set_error("n_sym = %d with perm %s", n_sym, perm ? "set" : "NULL");
        return XDG_EINVAL;
    }
    const int N = n_sites;
    std::unordered_map<std::vector<int32_t>, int, VecHash> where;
    std::vector<int32_t> row(N);
    for (int g = 0; g < n_sym; ++g) {
        std::vector<char> seen(N, 0);
        for (int i = 0; i < N; ++i) {
            int32_t v = perm[(size_t)g * N + i];
            if (v < 0 || v >= N || seen[v]) {
                set_error("permutation %d is not a bijection of the %d sites", g, N);
                return XDG_EINVAL;
            }
            seen[v] = 1;
        }
        row.assign(perm + (size_t)g * N, perm + (size_t)(g + 1) * N);
        if (where.count(row)) {
            set_error("permutation %d appears twice in the group", g);
            return XDG_EGROUP;
        }
        where[row] = g;
    }
    // identity
    for (int i = 0; i < N; ++i) row[i] = i;
    auto it = where.find(row);
    if (it == where.end()) {
        set_error("the group lacks the identity permutation");
        return XDG_EGROUP;
    }
    // inverses
    for (int g = 0; g < n_sym; ++g) {
        for (int i = 0; i < N; ++i) row[perm[(size_t)g * N + i]] = i;
        if (!where.count(row)) {
            set_error("the inverse of permutation %d is missing", g);
            return XDG_EGROUP;
        }
    }
    // closure and the homomorphism property of the characters
    const double tol = 1e-12;
    if (chi) {
        for (int g = 0; g < n_sym; ++g) {
            double a = std::hypot(chi[2 * g], chi[2 * g + 1]);
            if (!std::isfinite(a) || std::fabs(a - 1.0) > tol) {
                set_error("|chi(%d)| = %.17g is not 1", g, a);
                return XDG_ECHAR;
            }
        }
    }
    for (int f = 0; f < n_sym; ++f) {
        const int32_t *pf = perm + (size_t)f * N;
        for (int g = 0; g < n_sym; ++g) {
            const int32_t *pg = perm + (size_t)g * N;
            for (int i = 0; i < N; ++i) row[i] = pf[pg[i]];   // (f o g)(i)
            auto h = where.find(row);
            if (h == where.end()) {
                set_error("product of permutations %d and %d is not in the group", f, g);
                return XDG_EGROUP;
            }
            if (chi) {
                std::complex<double> cf(chi[2 * f], chi[2 * f + 1]);
                std::complex<double> cg(chi[2 * g], chi[2 * g + 1]);
                std::complex<double> ch(chi[2 * h->second], chi[2 * h->second + 1]);
                if (std::abs(cf * cg - ch) > tol) {
                    set_error("characters violate chi(f)chi(g) = chi(fg) for f=%d g=%d", f, g);
                    return XDG_ECHAR;
                }
            }
        }
    }
    return XDG_OK;
}

int validate_bonds(int n_sites, int n_sym, const int32_t *perm, int n_bonds, const int32_t *sites,
                   const double *jz, const double *jxy) {
    if (n_bonds < 0 || (n_bonds > 0 && (!sites || !jz || !jxy))) {
        set_error("bad bond arrays");
        return XDG_EINVAL;
    }
    std::map<std::pair<int, int>, std::pair<double, double>> agg;
    double scale = 0.0;
    for (int b = 0; b < n_bonds; ++b) {
        int i = sites[2 * b], j = sites[2 * b + 1];
        if (i < 0 || j < 0 || i >= n_sites || j >= n_sites || i == j) {
            set_error("bond %d = (%d, %d) is not a pair of distinct sites in [0, %d)", b, i, j,
                      n_sites);
            return XDG_EINVAL;
        }
        if (!std::isfinite(jz[b]) || !std::isfinite(jxy[b])) {
            set_error("bond %d has a non-finite coupling", b);
            return XDG_EINVAL;
        }
        auto &a = agg[{std::min(i, j), std::max(i, j)}];
        a.first += jz[b];
        a.second += jxy[b];
        scale = std::max(scale, std::max(std::fabs(jz[b]), std::fabs(jxy[b])));
    }
    const double tol = 1e-12 * std::max(scale, 1e-300);
    for (int g = 0; g < n_sym; ++g) {
        const int32_t *pg = perm + (size_t)g * n_sites;
        std::map<std::pair<int, int>, std::pair<double, double>> img;
        for (auto &kv : agg) {
            int i = pg[kv.first.first], j = pg[kv.first.second];
            auto &a = img[{std::min(i, j), std::max(i, j)}];
            a.first += kv.second.first;
            a.second += kv.second.second;
        }
        for (auto &kv : img) {
            auto f = agg.find(kv.first);
            double z = f == agg.end() ? 0.0 : f->second.first;
            double x = f == agg.end() ? 0.0 : f->second.second;
            if (std::fabs(z - kv.second.first) > tol || std::fabs(x - kv.second.second) > tol) {
                set_error("the bond list is not invariant under permutation %d", g);
                return XDG_ENOTSYM;
            }
        }
        for (auto &kv : agg) {
            if (!img.count(kv.first) &&
                (std::fabs(kv.second.first) > tol || std::fabs(kv.second.second) > tol)) {
                set_error("the bond list is not invariant under permutation %d", g);
                return XDG_ENOTSYM;
            }
        }
    }
    return XDG_OK;
}

// --------------------------------------------------------- search kinds --
namespace {

bool detect_affine(int N, int n_sym, const int32_t *perm, std::vector<AffineElem> *out) {
    std::vector<AffineElem> v;
    for (int g = 0; g < n_sym; ++g) {
        const int32_t *p = perm + (size_t)g * N;
        int a = p[0];
        bool plus = true, minus = true;
        for (int i = 0; i < N; ++i) {
            if (p[i] != (a + i) % N) plus = false;
            if (p[i] != ((a - i) % N + N) % N) minus = false;
        }
        if (!plus && !minus) return false;
        // (g.t)_i = t_{g(i)}:  plus  -> image = rotr_N(t, a)
        //                      minus -> image = rotr_N(rev_N(t), (N - 1 - a) mod N)
        if (plus)
            v.push_back({a, +1});
        else
            v.push_back({((N - 1 - a) % N + N) % N, -1});
    }
    if (out) *out = v;
    return true;
}

// Blocks q = sites [q m, (q+1) m).  Stable if every g maps the sites of
// each block onto the sites of one block.
bool detect_sublattice(int N, int n_sym, const int32_t *perm, int n_s, std::vector<uint8_t> *src) {
    if (n_s < 2 || N % n_s) return false;
    const int m = N / n_s;
    std::vector<uint8_t> s((size_t)n_sym * n_s);
    for (int g = 0; g < n_sym; ++g) {
        const int32_t *p = perm + (size_t)g * N;
        for (int a = 0; a < n_s; ++a) {
            int k = p[a * m] / m;
            for (int w = 0; w < m; ++w)
                if (p[a * m + w] / m != k) return false;
            s[(size_t)g * n_s + a] = (uint8_t)k;
        }
    }
    if (src) *src = s;
    return true;
}

void build_sublattice(int N, int n_sym, const int32_t *perm, int n_s, SublatticeTables *T) {
    const int m = N / n_s;
    const int V = 1 << m;
    const int pb = (m + 1) / 2, E = 1 << pb;
    T->n_s = n_s;
    T->m = m;
    T->pb = pb;
    detect_sublattice(N, n_sym, perm, n_s, &T->src);
    // distinct block permutations: image bit w of block a takes source bit
    // p[a m + w] - k m of block k = src[g][a]
    std::map<std::vector<int>, int> ids;
    std::vector<std::vector<int>> perms;
    T->pid.assign((size_t)n_sym * n_s, 0);
    for (int g = 0; g < n_sym; ++g) {
        const int32_t *p = perm + (size_t)g * N;
        for (int a = 0; a < n_s; ++a) {
            const int k = T->src[(size_t)g * n_s + a];
            std::vector<int> bw(m);
            for (int w = 0; w < m; ++w) bw[w] = p[a * m + w] - k * m;
            auto it = ids.find(bw);
            if (it == ids.end()) {
                it = ids.emplace(bw, (int)perms.size()).first;
                perms.push_back(bw);
            }
            T->pid[(size_t)g * n_s + a] = (uint16_t)it->second;
        }
    }
    T->n_perm = (int)perms.size();
    T->tperm.assign((size_t)T->n_perm * 2 * E, 0);
    for (int q = 0; q < T->n_perm; ++q) {
        std::vector<int> dst(m);   // source bit -> image bit
        for (int w = 0; w < m; ++w) dst[perms[q][w]] = w;
        for (int h = 0; h < 2; ++h)
            for (int u = 0; u < E; ++u) {
                uint32_t r = 0;
                for (int j = 0; j < pb; ++j) {
                    const int sb = h * pb + j;
                    if (sb < m && ((u >> j) & 1)) r |= 1u << dst[sb];
                }
                T->tperm[((size_t)q * 2 + h) * E + u] = (uint16_t)r;
            }
    }
    auto image = [&](int g, int a, int v) -> uint32_t {
        const uint16_t *tp = &T->tperm[(size_t)T->pid[(size_t)g * n_s + a] * 2 * E];
        return (uint32_t)tp[v & (E - 1)] | tp[E + (v >> pb)];
    };
    const int top = n_s - 1;
    T->mintop.assign((size_t)n_s * V, 0xFFFF);
    std::vector<std::vector<uint16_t>> lists((size_t)n_s * V);
    for (int g = 0; g < n_sym; ++g) {
        int k = T->src[(size_t)g * n_s + top];
        for (int v = 0; v < V; ++v) {
            const uint16_t im = (uint16_t)image(g, top, v);
            uint16_t &mt = T->mintop[(size_t)k * V + v];
            auto &L = lists[(size_t)k * V + v];
            if (im < mt) {
                mt = im;
                L.clear();
            }
            if (im == mt) L.push_back((uint16_t)g);
        }
    }
    T->cand_off.assign((size_t)n_s * V + 1, 0);
    T->cand_list.clear();
    for (size_t e = 0; e < lists.size(); ++e) {
        T->cand_off[e] = (uint32_t)T->cand_list.size();
        T->cand_list.insert(T->cand_list.end(), lists[e].begin(), lists[e].end());
    }
    T->cand_off.back() = (uint32_t)T->cand_list.size();
}

void build_bytes(int N, int n_sym, const int32_t *perm, ByteTables *B) {
    const int C = (N + 7) / 8;
    B->n_chunks = C;
    B->tab.assign((size_t)n_sym * C * 256, 0);
    std::vector<int> inv(N);
    for (int g = 0; g < n_sym; ++g) {
        const int32_t *p = perm + (size_t)g * N;
        for (int i = 0; i < N; ++i) inv[p[i]] = i;   // bit j of t lands on bit inv[j]
        for (int c = 0; c < C; ++c)
            for (int v = 0; v < 256; ++v) {
                uint64_t r = 0;
                for (int bit = 0; bit < 8; ++bit) {
                    int j = 8 * c + bit;
                    if (j < N && ((v >> bit) & 1)) r |= 1ull << inv[j];
                }
                B->tab[((size_t)g * C + c) * 256 + v] = r;
            }
    }
}

}  // namespace

int make_plan(int n_sites, int n_sym, const int32_t *perm, const xdg_basis_opts *opts, Plan *plan,
              bool build_tables) {
    const int want = opts ? opts->search : XDG_SEARCH_AUTO;
    const int want_ns = opts ? opts->n_sublattices : 0;
    if (opts) {
        for (int r : opts->reserved)
            if (r != 0) {
                set_error("xdg_basis_opts.reserved must be zero");
                return XDG_EINVAL;
            }
    }
    if (want < XDG_SEARCH_AUTO || want > XDG_SEARCH_TABLE) {
        set_error("unknown search kind %d", want);
        return XDG_EINVAL;
    }
    const int flags = opts ? opts->flags : 0;
    if (flags & ~(XDG_FLAG_F32_ACCUMULATE | XDG_FLAG_HASH_INDEX)) {
        set_error("unknown flags 0x%x", flags);
        return XDG_EINVAL;
    }
    Plan p;
    p.flags = flags;
    if (n_sym == 0) {
        if (want != XDG_SEARCH_AUTO && want != XDG_SEARCH_U1) {
            set_error("search kind %d needs a permutation group", want);
            return XDG_EINVAL;
        }
        p.kind = XDG_SEARCH_U1;
        *plan = std::move(p);
        return XDG_OK;
    }
    if (want == XDG_SEARCH_U1) {
        set_error("XDG_SEARCH_U1 given together with a permutation group");
        return XDG_EINVAL;
    }
    if (n_sym > 65535) {
        set_error("groups of more than 65535 elements are not supported");
        return XDG_EINVAL;
    }
    const int N = n_sites;
    if (want == XDG_SEARCH_AUTO || want == XDG_SEARCH_AFFINE) {
        if (detect_affine(N, n_sym, perm, &p.aff)) {
            p.kind = XDG_SEARCH_AFFINE;
            std::vector<int16_t> gi(2 * (size_t)N, -1);
            int n_rot = 0, n_ref = 0;
            for (int g = 0; g < n_sym; ++g) {
                const AffineElem &e = p.aff[g];
                int16_t &slot = gi[(e.eps > 0 ? 0 : N) + e.a];
                if (slot < 0) {
                    slot = (int16_t)g;
                    (e.eps > 0 ? n_rot : n_ref)++;
                }
            }
            if (n_rot == N && (n_ref == 0 || n_ref == N) && n_sym == n_rot + n_ref && N <= 64) {
                p.ring = n_ref ? 2 : 1;
                p.ring_gidx = gi;
            }
            *plan = std::move(p);
            return XDG_OK;
        }
        if (want == XDG_SEARCH_AFFINE) {
            set_error("the group is not made of ring translations/reflections i -> +-i + a");
            return XDG_EINVAL;
        }
    }
    if (want == XDG_SEARCH_AUTO || want == XDG_SEARCH_SUBLATTICE) {
        int chosen = 0;
        if (want_ns) {
            if (N % want_ns == 0 && N / want_ns <= 16 && detect_sublattice(N, n_sym, perm, want_ns, nullptr))
                chosen = want_ns;
        } else {
            for (int ns = 2; ns <= 8 && !chosen; ++ns)
                if (N % ns == 0 && N / ns <= 12 && detect_sublattice(N, n_sym, perm, ns, nullptr))
                    chosen = ns;
        }
        if (chosen) {
            p.kind = XDG_SEARCH_SUBLATTICE;
            if (build_tables) build_sublattice(N, n_sym, perm, chosen, &p.sub);
            p.sub.n_s = chosen;
            p.sub.m = N / chosen;
            *plan = std::move(p);
            return XDG_OK;
        }
        if (want == XDG_SEARCH_SUBLATTICE) {
            set_error("the labelling has no stable block partition into %d sublattices",
                      want_ns);
            return XDG_EINVAL;
        }
    }
    p.kind = XDG_SEARCH_TABLE;
    if (build_tables) build_bytes(N, n_sym, perm, &p.bytes);
    p.bytes.n_chunks = (N + 7) / 8;
    *plan = std::move(p);
    return XDG_OK;
}

}  // namespace xdg
