/*
 * CPU oracle for symmetry-adapted spin-1/2 exact diagonalisation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU library; the two meet only through seeded inputs.
 *
 * Everything is done the slow, plain way, in double / double complex:
 *   - the action of a permutation is applied bit by bit;
 *   - representatives and stabilisers come from scanning the whole group;
 *   - the basis is every popcount-n_up integer in ascending order, filtered;
 *   - the index of a state is a binary search in that list;
 *   - the Hamiltonian is applied row by row in pull form;
 *   - Lanczos is the textbook three-term recurrence, eigenvalues of the
 *     tridiagonal matrix by Sturm-sequence bisection.
 *
 * Paper: XDiag (arXiv 2505.02901).  Citations name sections / equations.
 *
 * Conventions (readings of the paper, stated once here):
 *   - a state is an integer; bit i is site i (0-based, as in the C++
 *     listings of Sec. 3.10.1); bit value 1 means spin up, so the number of
 *     up spins is the popcount.
 *   - action of a permutation g (Sec. 3.11, the equation defining g|sigma>):
 *     (g.s) has at site i the spin that s has at site g(i).
 *   - representative: the smallest integer in the orbit (Sec. 3.11).
 *   - symmetric state |s~> = N_s^{-1} sum_g chi(g)^* g|s>   (Sec. 3.11),
 *     unit normalised: N_s = sqrt(|G| |Stab(s)|).
 *   - an orbit whose stabiliser sum  sum_{h in Stab(s)} chi(h)  vanishes has
 *     no symmetric state and is not part of the basis.
 *   - Hamiltonian (Appendix A: SzSz and Exchange; SdotS = both with equal
 *     coupling):  H = sum_b [ Jz_b Sz_i Sz_j + (Jxy_b/2)(S+_i S-_j + S-_i S+_j) ].
 *
 * Parity status: every exported function here is pinned by the not-gpu tests
 * (dense diagonalisation from the definition, the worked k = pi example of
 * Sec. 3.11, the dimension formula, Bethe-ansatz energies, trace and
 * ferromagnetic-bound identities, brute-force small cases).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* Bits and binomials                                                        */
/* ------------------------------------------------------------------------ */

static int popcount64(uint64_t s) {
    int c = 0;
    while (s) { s &= s - 1; ++c; }
    return c;
}

/* binomial coefficient C(n, k) for n <= 64 by Pascal's rule (exact in uint64
   for every value needed here, n <= 64). */
static uint64_t binom(int n, int k) {
    static uint64_t table[65][65];
    static int ready = 0;
    if (!ready) {
        for (int a = 0; a <= 64; ++a) {
            table[a][0] = 1;
            for (int b = 1; b <= a; ++b)
                table[a][b] = table[a - 1][b - 1] + (b <= a - 1 ? table[a - 1][b] : 0);
        }
        ready = 1;
    }
    if (k < 0 || n < 0 || k > n) return 0;
    return table[n][k];
}

/* The popcount-n states in ascending integer order are the n-subsets of the
   sites in colexicographic order; rank r maps to the subset with
   r = sum_k C(p_k, k+1) (combinatorial number system).  Used only to split
   the ascending sweep into independent chunks. */
static uint64_t unrank_colex(uint64_t r, int n_sites, int n_up) {
    uint64_t s = 0;
    int p = n_sites - 1;
    for (int k = n_up; k >= 1; --k) {
        while (binom(p, k) > r) --p;
        s |= (uint64_t)1 << p;
        r -= binom(p, k);
        --p;
    }
    return s;
}

/* next larger integer with the same popcount (s != 0) */
static uint64_t next_same_popcount(uint64_t s) {
    uint64_t lowest = s & (~s + 1);
    uint64_t ripple = s + lowest;
    uint64_t ones = s ^ ripple;
    ones = (ones >> 2) / lowest;
    return ripple | ones;
}

/* ------------------------------------------------------------------------ */
/* Group action (Sec. 3.11, definition of g|sigma>)                          */
/* ------------------------------------------------------------------------ */

uint64_t orc_act(int n_sites, const int32_t *g, uint64_t s) {
    uint64_t out = 0;
    for (int i = 0; i < n_sites; ++i)
        if ((s >> g[i]) & 1u) out |= (uint64_t)1 << i;
    return out;
}

/* Scan the whole group.  Returns the representative min_g g.s; *u is the
   first group element (in the caller's order) reaching it and *n_min the
   number of elements reaching it (= |Stab(s)|). */
uint64_t orc_rep(int n_sites, int n_sym, const int32_t *perm, uint64_t s,
                 int32_t *u, int32_t *n_min) {
    uint64_t best = UINT64_MAX;
    int32_t bu = -1, cnt = 0;
    for (int g = 0; g < n_sym; ++g) {
        uint64_t img = orc_act(n_sites, perm + (size_t)g * n_sites, s);
        if (img < best) { best = img; bu = g; cnt = 1; }
        else if (img == best) ++cnt;
    }
    if (u) *u = bu;
    if (n_min) *n_min = cnt;
    return best;
}

/* sum of chi over the stabiliser of s (as a complex number) */
static cplx stab_char_sum(int n_sites, int n_sym, const int32_t *perm,
                          const double *chi, uint64_t s, int *stab_size) {
    cplx c = 0;
    int cnt = 0;
    for (int g = 0; g < n_sym; ++g)
        if (orc_act(n_sites, perm + (size_t)g * n_sites, s) == s) {
            c += chi[2 * g] + I * chi[2 * g + 1];
            ++cnt;
        }
    if (stab_size) *stab_size = cnt;
    return c;
}

/* s belongs to the symmetric basis: it is the smallest element of its orbit
   and the orbit carries a non-vanishing symmetric state. */
static int in_sym_basis(int n_sites, int n_sym, const int32_t *perm,
                        const double *chi, uint64_t s) {
    for (int g = 0; g < n_sym; ++g)
        if (orc_act(n_sites, perm + (size_t)g * n_sites, s) < s) return 0;
    int st;
    cplx c = stab_char_sum(n_sites, n_sym, perm, chi, s, &st);
    return cabs(c) > 0.5;
}

/* ------------------------------------------------------------------------ */
/* Basis: ascending list of states (U(1): all popcount-n_up states; with a   */
/* group: the representatives of compatible orbits).                         */
/* Returns the dimension; out may be NULL (count only).  Negative on bad     */
/* arguments or if cap is too small.                                         */
/* ------------------------------------------------------------------------ */

int64_t orc_basis(int n_sites, int n_up, int n_sym, const int32_t *perm,
                  const double *chi, uint64_t *out, int64_t cap) {
    if (n_sites < 1 || n_sites > 64 || n_up < 0 || n_up > n_sites) return -1;
    uint64_t total = binom(n_sites, n_up);
    if (n_up == 0) {
        /* the single state 0 */
        int keep = n_sym == 0 || in_sym_basis(n_sites, n_sym, perm, chi, 0);
        if (keep && out) { if (cap < 1) return -2; out[0] = 0; }
        return keep;
    }
    const int64_t n_chunks = total < 4096 ? (int64_t)total : 4096;
    const uint64_t per = (total + (uint64_t)n_chunks - 1) / (uint64_t)n_chunks;
    int64_t *counts = (int64_t *)calloc((size_t)n_chunks + 1, sizeof(int64_t));
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            int64_t acc = 0;
            for (int64_t c = 0; c < n_chunks; ++c) { int64_t t = counts[c]; counts[c] = acc; acc += t; }
            counts[n_chunks] = acc;
            if (!out) break;
            if (acc > cap) { free(counts); return -2; }
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t c = 0; c < n_chunks; ++c) {
            uint64_t r0 = (uint64_t)c * per;
            if (r0 >= total) continue;
            uint64_t r1 = r0 + per < total ? r0 + per : total;
            uint64_t s = unrank_colex(r0, n_sites, n_up);
            int64_t pos = pass ? counts[c] : 0;
            for (uint64_t r = r0; r < r1; ++r) {
                int keep = n_sym == 0 || in_sym_basis(n_sites, n_sym, perm, chi, s);
                if (keep) {
                    if (pass) out[pos] = s;
                    ++pos;
                }
                if (r + 1 < r1) s = next_same_popcount(s);
            }
            if (!pass) counts[c] = pos;
        }
    }
    int64_t dim = counts[n_chunks];
    free(counts);
    return dim;
}

/* The basis states lying in [lo, hi] (ascending), by the same sweep as
   orc_basis restricted to that range.  Returns their number, or -2 if cap is
   too small. */
int64_t orc_basis_range(int n_sites, int n_up, int n_sym, const int32_t *perm,
                        const double *chi, uint64_t lo, uint64_t hi, uint64_t *out, int64_t cap) {
    if (n_sites < 1 || n_sites > 64 || n_up < 1 || n_up > n_sites || lo > hi) return -1;
    const uint64_t top = n_sites == 64 ? UINT64_MAX : (((uint64_t)1 << n_sites) - 1);
    /* smallest popcount-n_up integer >= lo (plain upward scan) */
    uint64_t s = lo;
    const uint64_t first = n_up == 64 ? UINT64_MAX : (((uint64_t)1 << n_up) - 1);
    if (s < first) s = first;
    while (popcount64(s) != n_up && s < top) ++s;
    if (popcount64(s) != n_up) return 0;
    int64_t n = 0;
    while (s <= hi && s <= top) {
        int keep = n_sym == 0 || in_sym_basis(n_sites, n_sym, perm, chi, s);
        if (keep) {
            if (n >= cap) return -2;
            out[n++] = s;
        }
        uint64_t nx = next_same_popcount(s);
        if (nx <= s) break;
        s = nx;
    }
    return n;
}

/* position of s in the ascending basis list, -1 if absent */
int64_t orc_index(const uint64_t *basis, int64_t dim, uint64_t s) {
    int64_t lo = 0, hi = dim;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (basis[mid] < s) lo = mid + 1; else hi = mid;
    }
    return (lo < dim && basis[lo] == s) ? lo : -1;
}

/* ------------------------------------------------------------------------ */
/* One row of H in the symmetric basis, pull form.                           */
/*                                                                           */
/* With H commuting with every g, chi one-dimensional and real couplings,    */
/*   <r~|H|s~> = sum over the terms t of H|r> whose orbit is that of s of    */
/*               h_t chi(u_t) N_s / N_r,   where u_t . t = s.                */
/* (H|r~> = sum_t h_t chi(u_t)^* (N_s/N_r) |s~>, then Hermiticity.)          */
/* The diagonal Sz Sz part is returned separately in *diag.                  */
/* Writes up to cap (target state, complex amplitude) pairs; returns their   */
/* number (targets outside the basis are skipped), or -1 if cap is short.    */
/* With n_sym == 0 (U(1) only) every amplitude is Jxy/2.                     */
/* ------------------------------------------------------------------------ */

int orc_row_terms(int n_sites, int n_sym, const int32_t *perm, const double *chi,
                  int n_bonds, const int32_t *sites, const double *jz, const double *jxy,
                  uint64_t r, double *diag, uint64_t *targets, double *amps, int cap) {
    double d = 0.0;
    int n = 0;
    int stab_r = 1;
    if (n_sym > 0) stab_char_sum(n_sites, n_sym, perm, chi, r, &stab_r);
    for (int b = 0; b < n_bonds; ++b) {
        int i = sites[2 * b], j = sites[2 * b + 1];
        int bi = (int)((r >> i) & 1u), bj = (int)((r >> j) & 1u);
        d += (bi == bj ? 0.25 : -0.25) * jz[b];
        if (bi == bj) continue;
        uint64_t t = r ^ (((uint64_t)1 << i) | ((uint64_t)1 << j));
        double h = 0.5 * jxy[b];
        uint64_t s = t;
        cplx amp = h;
        if (n_sym > 0) {
            int32_t u, nmin;
            s = orc_rep(n_sites, n_sym, perm, t, &u, &nmin);
            int st;
            cplx c = stab_char_sum(n_sites, n_sym, perm, chi, s, &st);
            if (cabs(c) <= 0.5) continue;      /* orbit has no symmetric state */
            amp = h * (chi[2 * u] + I * chi[2 * u + 1]) * sqrt((double)st / (double)stab_r);
        }
        if (n >= cap) return -1;
        targets[n] = s;
        amps[2 * n] = creal(amp);
        amps[2 * n + 1] = cimag(amp);
        ++n;
    }
    *diag = d;
    return n;
}

/* y = H x on the basis list; x, y complex128 interleaved, layout [dim][nvec]. */
int orc_apply(int n_sites, int n_sym, const int32_t *perm, const double *chi,
              int n_bonds, const int32_t *sites, const double *jz, const double *jxy,
              const uint64_t *basis, int64_t dim, int64_t nvec,
              const double *x, double *y) {
    const cplx *xc = (const cplx *)x;
    cplx *yc = (cplx *)y;
    int err = 0;
#pragma omp parallel
    {
        uint64_t *tg = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_bonds + 1));
        double *am = (double *)malloc(sizeof(double) * 2 * (size_t)(n_bonds + 1));
        cplx *acc = (cplx *)malloc(sizeof(cplx) * (size_t)nvec);
#pragma omp for schedule(dynamic, 256)
        for (int64_t row = 0; row < dim; ++row) {
            double d;
            int nt = orc_row_terms(n_sites, n_sym, perm, chi, n_bonds, sites, jz, jxy,
                                   basis[row], &d, tg, am, n_bonds + 1);
            if (nt < 0) { err = 1; continue; }
            for (int64_t v = 0; v < nvec; ++v) acc[v] = d * xc[row * nvec + v];
            for (int k = 0; k < nt; ++k) {
                int64_t col = orc_index(basis, dim, tg[k]);
                if (col < 0) { err = 1; continue; }
                cplx a = am[2 * k] + I * am[2 * k + 1];
                for (int64_t v = 0; v < nvec; ++v) acc[v] += a * xc[col * nvec + v];
            }
            for (int64_t v = 0; v < nvec; ++v) yc[row * nvec + v] = acc[v];
        }
        free(tg); free(am); free(acc);
    }
    return err ? -1 : 0;
}

/* y[k] = (H x)[rows[k]] for selected rows only (same arithmetic as
   orc_apply, row by row); x complex128 [dim][nvec], y [n_rows][nvec]. */
int orc_apply_rows(int n_sites, int n_sym, const int32_t *perm, const double *chi,
                   int n_bonds, const int32_t *sites, const double *jz, const double *jxy,
                   const uint64_t *basis, int64_t dim, const int64_t *rows, int64_t n_rows,
                   int64_t nvec, const double *x, double *y) {
    const cplx *xc = (const cplx *)x;
    cplx *yc = (cplx *)y;
    int err = 0;
#pragma omp parallel
    {
        uint64_t *tg = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_bonds + 1));
        double *am = (double *)malloc(sizeof(double) * 2 * (size_t)(n_bonds + 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < n_rows; ++k) {
            const int64_t row = rows[k];
            if (row < 0 || row >= dim) { err = 1; continue; }
            double d;
            int nt = orc_row_terms(n_sites, n_sym, perm, chi, n_bonds, sites, jz, jxy,
                                   basis[row], &d, tg, am, n_bonds + 1);
            if (nt < 0) { err = 1; continue; }
            for (int64_t v = 0; v < nvec; ++v) {
                cplx acc = d * xc[row * nvec + v];
                for (int q = 0; q < nt; ++q) {
                    int64_t col = orc_index(basis, dim, tg[q]);
                    if (col < 0) { err = 1; continue; }
                    acc += (am[2 * q] + I * am[2 * q + 1]) * xc[col * nvec + v];
                }
                yc[k * nvec + v] = acc;
            }
        }
        free(tg); free(am);
    }
    return err ? -1 : 0;
}

/* Representatives of n states (orc_rep for each, OpenMP over states) and
   whether each representative is a basis state (its orbit carries a
   symmetric state). */
int orc_rep_many(int n_sites, int n_sym, const int32_t *perm, const double *chi,
                 const uint64_t *states, int64_t n, uint64_t *reps, int32_t *in_basis) {
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < n; ++k) {
        const uint64_t r = n_sym > 0 ? orc_rep(n_sites, n_sym, perm, states[k], NULL, NULL)
                                     : states[k];
        reps[k] = r;
        in_basis[k] = n_sym == 0 || in_sym_basis(n_sites, n_sym, perm, chi, r);
    }
    return 0;
}

/* orc_row_terms for each of n_rows row states (OpenMP over rows), plus the
   membership of each row state in the sector basis (a representative of an
   orbit that carries a symmetric state; always 1 without a group).
   Row k's terms occupy slots [k * n_bonds, k * n_bonds + cnt[k]) of targets
   and amps (complex interleaved); diag[k] is its Sz Sz part.  Nothing here
   needs the basis list: targets are states, not positions.  Returns 0, or
   -1 if a row state has the wrong number of sites set. */
int orc_rows_terms(int n_sites, int n_up, int n_sym, const int32_t *perm, const double *chi,
                   int n_bonds, const int32_t *sites, const double *jz, const double *jxy,
                   const uint64_t *rows, int64_t n_rows, double *diag, int32_t *cnt,
                   int32_t *in_basis, uint64_t *targets, double *amps) {
    int err = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_rows; ++k) {
        const uint64_t r = rows[k];
        if (popcount64(r) != n_up) { err = 1; cnt[k] = 0; in_basis[k] = 0; continue; }
        in_basis[k] = n_sym == 0 || in_sym_basis(n_sites, n_sym, perm, chi, r);
        int nt = orc_row_terms(n_sites, n_sym, perm, chi, n_bonds, sites, jz, jxy, r,
                               diag + k, targets + (size_t)k * n_bonds,
                               amps + 2 * (size_t)k * n_bonds, n_bonds);
        if (nt < 0) { err = 1; nt = 0; }
        cnt[k] = nt;
    }
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Symmetric tridiagonal eigenvalues by Sturm-sequence bisection.            */
/* T has diagonal a[0..m) and off-diagonal b[0..m-1) (b[i] couples i, i+1).  */
/* Writes the k smallest eigenvalues in ascending order.                     */
/* ------------------------------------------------------------------------ */

static int sturm_count_below(int m, const double *a, const double *b, double x) {
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
        double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
        q = (a[i] - x) - (i > 0 ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0) ++cnt;
    }
    return cnt;
}

int orc_tridiag_eigvals(int m, const double *a, const double *b, int k, double *out) {
    if (m < 1 || k < 1 || k > m) return -1;
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < m ? fabs(b[i]) : 0.0);
        if (a[i] - r < lo) lo = a[i] - r;
        if (a[i] + r > hi) hi = a[i] + r;
    }
    double span = hi - lo + 1e-300;
    lo -= 1e-12 * span + 1e-300;
    hi += 1e-12 * span + 1e-300;
    for (int e = 0; e < k; ++e) {
        /* eigenvalue number e (0-based): smallest x with count_below(x) > e */
        double l = lo, h = hi;
        for (int it = 0; it < 200; ++it) {
            double mid = 0.5 * (l + h);
            if (mid <= l || mid >= h) break;
            if (sturm_count_below(m, a, b, mid) > e) h = mid; else l = mid;
        }
        out[e] = 0.5 * (l + h);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Lanczos (Sec. 3.7.1; the recurrence of Lanczos 1950), double complex.     */
/*   v_0 = x0/|x0|, beta_0 = 0;  for j = 0, 1, ...:                          */
/*     w = H v_j;  alpha_j = Re<v_j, w>;  w -= alpha_j v_j + beta_j v_{j-1}; */
/*     [reorth: twice, w -= sum_i <v_i, w> v_i]                              */
/*     beta_{j+1} = |w|;  stop on convergence of the k-th lowest Ritz value  */
/*     (relative change <= tol), breakdown or max_iter; v_{j+1} = w/beta.    */
/* alpha[j], beta[j] (= beta_{j+1}) are written for j < *n_iter.             */
/* Returns 0 converged / invariant subspace, 1 if max_iter was reached,      */
/* negative on error.                                                        */
/* ------------------------------------------------------------------------ */

static double dot_re(int64_t n, const cplx *a, const cplx *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += creal(conj(a[i]) * b[i]);
    return s;
}

static cplx dot_c(int64_t n, const cplx *a, const cplx *b) {
    cplx s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += conj(a[i]) * b[i];
    return s;
}

int orc_lanczos(int n_sites, int n_sym, const int32_t *perm, const double *chi,
                int n_bonds, const int32_t *sites, const double *jz, const double *jxy,
                const uint64_t *basis, int64_t dim, const double *x0,
                int k, double tol, int max_iter, int reorth,
                double *alpha, double *beta, int *n_iter, double *evals) {
    if (dim < 1 || k < 1 || max_iter < 1) return -1;
    cplx *vprev = (cplx *)calloc((size_t)dim, sizeof(cplx));
    cplx *v = (cplx *)malloc(sizeof(cplx) * (size_t)dim);
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)dim);
    cplx *V = reorth ? (cplx *)malloc(sizeof(cplx) * (size_t)dim * (size_t)max_iter) : NULL;
    double *ritz = (double *)malloc(sizeof(double) * (size_t)k);
    double prev_k = NAN;
    memcpy(v, x0, sizeof(cplx) * (size_t)dim);
    double nrm = sqrt(dot_re(dim, v, v));
    for (int64_t i = 0; i < dim; ++i) v[i] /= nrm;
    double b_cur = 0.0;
    int status = 1, m = 0;
    for (int j = 0; j < max_iter; ++j) {
        if (V) memcpy(V + (size_t)j * dim, v, sizeof(cplx) * (size_t)dim);
        if (orc_apply(n_sites, n_sym, perm, chi, n_bonds, sites, jz, jxy, basis, dim, 1,
                      (const double *)v, (double *)w) != 0) { status = -2; break; }
        double a = dot_re(dim, v, w);
        for (int64_t i = 0; i < dim; ++i) w[i] -= a * v[i] + b_cur * vprev[i];
        if (V) {
            for (int pass = 0; pass < 2; ++pass)
                for (int i = 0; i <= j; ++i) {
                    cplx c = dot_c(dim, V + (size_t)i * dim, w);
                    for (int64_t q = 0; q < dim; ++q) w[q] -= c * V[(size_t)i * dim + q];
                }
        }
        double bn = sqrt(dot_re(dim, w, w));
        alpha[j] = a;
        beta[j] = bn;
        m = j + 1;
        int stop = 0;
        if (m >= k) {
            orc_tridiag_eigvals(m, alpha, beta, k, ritz);
            if (tol > 0 && !isnan(prev_k) && fabs(ritz[k - 1] - prev_k) <= tol * fabs(ritz[k - 1]))
                stop = 1;
            prev_k = ritz[k - 1];
        }
        if (bn <= 1e-13 * fmax(1.0, fabs(a))) stop = 1;
        if (stop) { status = 0; break; }
        for (int64_t i = 0; i < dim; ++i) { vprev[i] = v[i]; v[i] = w[i] / bn; }
        b_cur = bn;
    }
    if (status >= 0) {
        int kk = k <= m ? k : m;
        orc_tridiag_eigvals(m, alpha, beta, kk, evals);
        for (int e = kk; e < k; ++e) evals[e] = NAN;
    }
    *n_iter = m;
    free(vprev); free(v); free(w); free(V); free(ritz);
    return status;
}

/* thread count the OpenMP runtime will use (for reporting) */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
