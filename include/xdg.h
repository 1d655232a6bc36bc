/*
 * xdg.h - C ABI of the MI355X library for symmetry-adapted spin-1/2 exact
 * diagonalisation: sector bases, the matrix-free Hamiltonian application
 * y = H x, and the Lanczos iteration built on it.
 *
 * Paper: XDiag, "Exact Diagonalization for Quantum Many-Body Systems"
 * (arXiv 2505.02901).  Each entry point names the passage that defines the
 * operation it performs.
 *
 * General rules
 *   - Pure C ABI: plain integers, doubles and pointers; no exceptions cross it.
 *   - Every function returns XDG_OK (0) on success or a negative XDG_E* code;
 *     xdg_last_error() then returns a message (thread-local, valid until the
 *     next failing call on the same thread).  XDG_ENOCONV is the one
 *     "soft" failure: the outputs are written anyway.
 *   - Sites are 0-based (as in the C++ listings of Sec. 3.1 and 3.10.1).
 *     A product state is an integer whose bit i is site i, bit value 1 = up.
 *   - Permutations are rows perm[g * n_sites + i] = g(i); the action on a
 *     product state follows the definition in Sec. 3.11: (g.s) has at site i
 *     the spin of s at site g(i).
 *   - A sector basis is the ascending list of orbit representatives (the
 *     smallest integer of each orbit, Sec. 3.11) whose orbit carries a
 *     symmetric state for the chosen characters; with no group it is the
 *     ascending list of all states with n_up up spins (Sec. 3.1).
 *     Basis vectors are unit normalised: |s~> = N_s^-1 sum_g chi(g)^* g|s>,
 *     N_s = sqrt(|G| |Stab(s)|).
 *   - Vectors are device pointers in HBM laid out [dim][nvec] row-major
 *     (the nvec values of one basis index are contiguous); complex values
 *     are (re, im) interleaved.  The caller owns them.  Handles own every
 *     table and work buffer they allocate and free them on destroy.
 *   - All device work runs on the current HIP device.  Functions that take
 *     a `stream` (hipStream_t passed as void*; NULL = default stream) only
 *     enqueue work; the others synchronise before returning.
 *   - The C ABI cannot see the size of a device buffer: a vector shorter
 *     than the block's dim * nvec (complex counted twice) is read or written
 *     out of bounds.  The Python binding checks tensor sizes and dtypes
 *     against xdg_ham_dim / xdg_basis_dim before every call.
 *   - Thread safety: handles may be used from several host threads; the
 *     launch-shape caches inside a Hamiltonian and the batched-grid cache
 *     are locked.  Calls that write the same output vector concurrently race
 *     like any two writers.
 */
#ifndef XDG_H
#define XDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define XDG_OK        0
#define XDG_EINVAL   -1  /* bad argument: n_up outside [0, N], N > 64, bad site, bad dtype ... */
#define XDG_EGROUP   -2  /* permutations do not form a group (Sec. 3.10.1: identity, inverses, closure) */
#define XDG_ECHAR    -3  /* characters are not a 1-d representation (Sec. 3.10.2: |chi| = 1, homomorphism) */
#define XDG_ENOTSYM  -4  /* bond list not invariant under the group: no well-defined sector (Sec. 3.6, 3.10) */
#define XDG_ENOMEM   -5  /* device allocation failed */
#define XDG_EHIP     -6  /* HIP runtime error */
#define XDG_ENOCONV  -7  /* Lanczos reached max_iter before the tolerance; outputs still written */

/* ---- scalar types of vectors -------------------------------------------- */
#define XDG_F64   0   /* double */
#define XDG_F32   1   /* float */
#define XDG_C128  2   /* complex double, (re, im) */
#define XDG_C64   3   /* complex float, (re, im) */

/* ---- representative search kinds (Sec. 5.1 backends, Sec. 5.2) ---------- */
#define XDG_SEARCH_AUTO        0  /* pick the fastest kind that applies */
#define XDG_SEARCH_U1          1  /* no permutation group: Lin-table index (Sec. 5.2) */
#define XDG_SEARCH_AFFINE      2  /* every g is i -> (+-i + a) mod N: images by bit rotation/reversal */
#define XDG_SEARCH_SUBLATTICE  3  /* sublattice coding: sites labelled in n_s contiguous blocks, each g maps blocks onto blocks */
#define XDG_SEARCH_TABLE       4  /* any group: images from per-element byte lookup tables */

/* ---- Lanczos precision forms --------------------------------------------- */
#define XDG_PREC_F64          0  /* FP64 (or complex FP64) vectors */
#define XDG_PREC_F32VEC       1  /* FP32 (or complex FP32) vectors; FP64 dot products, norms, update, tridiagonal solve */
#define XDG_PREC_F32VEC_REORTH 2 /* as F32VEC plus full reorthogonalisation (classical Gram-Schmidt, FP64 coefficients, a second pass where the first removes more than half of the norm squared: Daniel, Gragg, Kaufman, Stewart 1976) */
#define XDG_PREC_F64_REORTH   3  /* FP64 vectors plus full reorthogonalisation */

typedef struct xdg_basis_s *xdg_basis;
typedef struct xdg_ham_s *xdg_ham;

/* Options for xdg_create_basis; pass NULL for defaults (all zero). */
typedef struct xdg_basis_opts {
    int search;          /* XDG_SEARCH_*; 0 = auto */
    int n_sublattices;   /* for XDG_SEARCH_SUBLATTICE: 2..8; 0 = detect */
    int flags;           /* XDG_FLAG_* bits */
    int reserved[5];     /* must be zero */
} xdg_basis_opts;

/* flags:
 * XDG_FLAG_F32_ACCUMULATE: with FP32 / complex-FP32 vectors, compute the
 *   amplitudes and accumulate each output row in FP32 (default: FP64
 *   amplitudes and accumulation, one rounding to FP32 when the row is
 *   stored; the vectors are FP32 in memory either way). */
#define XDG_FLAG_F32_ACCUMULATE 2
/* XDG_FLAG_HASH_INDEX: index a symmetric block with the hash table even when
 *   the rank bitmap (below) would fit. */
#define XDG_FLAG_HASH_INDEX 4

/* Index of a block (Sec. 5.2: state -> position in the ascending basis):
 * XDG_INDEX_LIN   no permutation group: Lin's two tables;
 * XDG_INDEX_HASH  open addressing over 64-byte lines of (state, position);
 * XDG_INDEX_RANK  rank bitmap: one (u32 count, u32 bits) pair per 32
 *                 consecutive colex ranks among the states with n_up up
 *                 spins, up to the rank of the largest representative; the
 *                 position of s is the count of its word plus the set bits
 *                 below s's bit.  Colex rank preserves numeric order, so the
 *                 lookups of neighbouring rows touch neighbouring words.
 *                 Chosen when it takes at most 4x the hash table's memory
 *                 plus 64 MiB, unless XDG_FLAG_HASH_INDEX is set. */
#define XDG_INDEX_LIN  1
#define XDG_INDEX_HASH 2
#define XDG_INDEX_RANK 3

/* Limit on the device memory the library's own buffers (bases, indices,
 * tables, Lanczos work vectors, batched plans) may hold together, in bytes;
 * 0 removes it.  An allocation beyond it fails with XDG_ENOMEM as if the
 * device were full (the caller's own vectors do not count).  Applies to
 * every thread.  `in_use` (may be NULL) receives what the buffers hold now.
 * Host only. */
int xdg_set_device_memory_limit(int64_t bytes, int64_t *in_use);

/* Version string of the library (cf. the version banner, Sec. 2). */
const char *xdg_version(void);

/* Message of the last failing call on this thread (cf. error traces, Sec. 2). */
const char *xdg_last_error(void);

/* Host-only validation of a permutation group and its characters, exactly as
 * xdg_create_basis performs it (Sec. 3.10.1: identity, inverse of every
 * element and closure under products must be present; Sec. 3.10.2:
 * f*g = h implies chi(f) chi(g) = chi(h), and |chi| = 1).
 * perm: host int32[n_sym * n_sites]; chi: host double[2 * n_sym] (re, im)
 * or NULL (all 1).  Needs no GPU.  Tolerance 1e-12 absolute on characters.
 * Returns XDG_OK, XDG_EINVAL, XDG_EGROUP or XDG_ECHAR. */
int xdg_check_group(int n_sites, int n_sym, const int32_t *perm, const double *chi);

/* Host-only check that a bond list (with couplings) is mapped onto itself by
 * every group element (a Hamiltonian with a well-defined sector, Sec. 3.6).
 * Bonds are unordered pairs; duplicate bonds add their couplings.
 * Relative tolerance 1e-12.  Returns XDG_OK, XDG_EINVAL or XDG_ENOTSYM. */
int xdg_check_bonds(int n_sites, int n_sym, const int32_t *perm, int n_bonds,
                    const int32_t *sites, const double *jz, const double *jxy);

/* Search kind that xdg_create_basis would pick (host only, no GPU).
 * Writes the XDG_SEARCH_* kind and, for sublattice coding, the number of
 * sublattices. */
int xdg_plan_search(int n_sites, int n_sym, const int32_t *perm, const xdg_basis_opts *opts,
                    int *kind, int *n_sublattices);

/* Block Spinhalf(N, nup) or Spinhalf(N, nup, irrep) (Sec. 3.1, 3.11).
 *   n_sites in [1, 64]; n_up in [0, n_sites];
 *   n_sym = 0 and perm = NULL for the U(1)-only block;
 *   perm: host int32[n_sym * n_sites]; chi: host double[2 * n_sym] or NULL.
 * Validates the group and characters (xdg_check_group), enumerates the basis
 * on the GPU and builds its device index.  The handle is immutable.
 * Errors: XDG_EINVAL, XDG_EGROUP, XDG_ECHAR, XDG_ENOMEM, XDG_EHIP.
 * A sector of dimension 0 is legal. */
int xdg_create_basis(int n_sites, int n_up, int n_sym, const int32_t *perm, const double *chi,
                     const xdg_basis_opts *opts, xdg_basis *out);

/* Release a basis (Hamiltonians hold their own reference; NULL is ignored). */
void xdg_destroy_basis(xdg_basis b);

/* Dimension of the block (size(block), Sec. 3.1). */
int xdg_basis_dim(xdg_basis b, int64_t *dim);

/* 1 if the characters are not all real, so that H is complex on the block
 * and vectors must be XDG_C128 / XDG_C64. */
int xdg_basis_is_complex(xdg_basis b, int *is_complex);

/* Search kind in use and its number of sublattices (0 unless sublattice). */
int xdg_basis_search_kind(xdg_basis b, int *kind, int *n_sublattices);

/* Index kind in use (XDG_INDEX_*) and its device memory in bytes. */
int xdg_basis_index_kind(xdg_basis b, int *kind, int64_t *bytes);

/* Copy basis states [begin, begin + count) (ascending representatives) to
 * host memory (iteration over a block, Sec. 3.1 / 3.11). */
int xdg_basis_copy_states(xdg_basis b, int64_t begin, int64_t count, uint64_t *host_out);

/* Copy the stabiliser sizes |Stab(s)| of basis states [begin, begin+count)
 * to host memory (int32; all 1 for the U(1) block). */
int xdg_basis_copy_stabilisers(xdg_basis b, int64_t begin, int64_t count, int32_t *host_out);

/* index(block, state) (Sec. 3.1): 0-based positions of n host states, -1
 * for a state that is not a basis state (not a representative, wrong
 * popcount, or an orbit without a symmetric state).  Runs the device index. */
int xdg_basis_index(xdg_basis b, const uint64_t *states, int64_t n, int64_t *idx_out);

/* Hamiltonian H = sum_b [ jz[b] Sz_i Sz_j + jxy[b]/2 (S+_i S-_j + S-_i S+_j) ]
 * on a block: Appendix A types SzSz and Exchange (real coupling); SdotS is
 * jz = jxy = J; the XXZ chain of Sec. 4 is jz = J Delta, jxy = J.
 *   sites: host int32[2 * n_bonds] (i, j) pairs, i != j, both < n_sites;
 *   jz, jxy: host double[n_bonds].
 * The bond list must be invariant under the block's group (XDG_ENOTSYM).
 * The handle keeps a reference to the basis. */
int xdg_create_hamiltonian(xdg_basis b, int n_bonds, const int32_t *sites, const double *jz,
                           const double *jxy, xdg_ham *out);

void xdg_destroy_hamiltonian(xdg_ham h);

/* Number of nonzero matrix elements one application touches per vector:
 * dim (the diagonal, counted once per row) plus the off-diagonal (row, bond)
 * terms whose target lies in the block.  Computed on the GPU once, cached. */
int xdg_ham_nnz(xdg_ham h, int64_t *nnz);

/* Dimension of the Hamiltonian's block and whether it is complex (so that
 * callers holding only the Hamiltonian can size vectors; size(block),
 * Sec. 3.1).  Either pointer may be NULL.  Host only. */
int xdg_ham_dim(xdg_ham h, int64_t *dim, int *is_complex);

/* y = H x, matrix-free (apply, Sec. 3.6 and Sec. 5.1: elements are computed
 * on the fly; several vectors at once as for a matrix of coefficients).
 *   x, y: device pointers, [dim][nvec], dtype XDG_F64/F32/C128/C64; x != y.
 *   Real dtypes need a real block (xdg_basis_is_complex == 0).
 * One lane owns each output row and writes it once: no atomics, and the
 * result is bitwise reproducible for any launch configuration.
 * Enqueued on `stream`. */
int xdg_apply(xdg_ham h, const void *x, void *y, int64_t nvec, int dtype, void *stream);

/* Launch shape of the apply kernel (what the autotuner chooses). */
typedef struct xdg_launch_cfg {
    int grid;          /* workgroups of 1024 lanes looping over the rows; 0 = one row per lane */
    int nv;            /* vectors per pass: 1, 2, 4 or 8 (0 = 8), capped by nvec */
    int occ;           /* 1: the copy limited to 64 VGPRs, 8 waves per SIMD (used only when
                          two workgroups' LDS tables fit a compute unit); 0: 4 waves; -1: auto */
    int compact;       /* sublattice / table searches: 1 = wave-compacted term loop (terms of
                          64 rows packed into full passes), 0 or -1 = row loop */
    int sub_form;      /* sublattice coding: 0 = automatic (the packed form wherever it
                          applies: four blocks of at most 10 sites, tables in LDS), 2 = the
                          block-by-block form (comparisons); both give bitwise the same y */
    int xr;            /* sublattice coding with a rank index: 1 = the terms read x from a
                          rank-addressed copy (slot = rank of the representative among the
                          states whose top block is a minimal top; zeros where the
                          representative is not a basis state), filled by a scatter before
                          the launch: one random read per term instead of an index word and
                          x.  The copy is device memory held by the Hamiltonian (slots x the
                          row's bytes; XDG_ENOMEM when it does not fit), set up by a first call
                          outside graph capture; calls on other streams wait for the last
                          launch that read it.  0 = through the rank index.  Elsewhere
                          ignored.  Both give the same y (up to the sign of zero sums) */
    int reserved[2];   /* must be zero */
} xdg_launch_cfg;

/* xdg_apply in a given launch shape (tuning and tests: every shape computes
 * bitwise the same y).  Errors: XDG_EINVAL for a shape outside the ranges. */
int xdg_apply_with_config(xdg_ham h, const void *x, void *y, int64_t nvec, int dtype,
                          const xdg_launch_cfg *cfg, void *stream);

/* The launch shape the autotuner chose for (dtype, nvec) on this Hamiltonian
 * (after a first xdg_apply with them; XDG_EINVAL before).  Host only. */
int xdg_apply_tuned_config(xdg_ham h, int dtype, int64_t nvec, xdg_launch_cfg *out);

/* Several blocks (of possibly different dimension) in one persistent fused
 * launch: y_i = H_i x_i for i < n, all with the same nvec and dtype.  Work
 * items are (block, row tile) pairs drawn from one queue. */
int xdg_apply_batched(int n, const xdg_ham *hams, const void *const *xs, void *const *ys,
                      int64_t nvec, int dtype, void *stream);

/* xdg_apply_batched for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results (bitwise) as
 * xdg_apply_batched, but it allocates nothing: the queue counter, the tile
 * prefix and the sector descriptors live in one file-scope device array of
 * the library (about 40 KB, held by each GPU the library runs on until the
 * process ends), written by small kernels on `stream` before the launch.
 * Limit: n <= 128 blocks (XDG_EINVAL beyond, before any launch).  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other host threads) race; calls in order on one stream do not. */
int xdg_apply_batched_noalloc(int n, const xdg_ham *hams, const void *const *xs,
                              void *const *ys, int64_t nvec, int dtype, void *stream);

/* Seeded random vector of `dim * nvec` scalars (random_state, Sec. 3.6):
 * SplitMix64 (Steele, Lea, Flood 2014), counter based: output n of seed
 * is mix(seed + n * 0x9E3779B97F4A7C15).  Scalar q (flat over [dim][nvec],
 * complex re/im interleaved) uses outputs 2q+1, 2q+2:
 *   kind 0: uniform on [-1, 1]: 2 u - 1;
 *   kind 1: Gaussian: sqrt(-2 log1p(-u1)) cos(2 pi u2)   (Box-Muller),
 * u = top 53 bits * 2^-53.  out: device pointer. */
int xdg_random_state(int64_t dim, int64_t nvec, uint64_t seed, int kind, int dtype, void *out,
                     void *stream);

/* Lowest eigenvalues by Lanczos (eigval0 / eigvals_lanczos, Sec. 3.7.1).
 *   v0: device start vector [dim] of the dtype the precision form uses
 *       (F64/C128 or F32/C64), or NULL for xdg_random_state(seed, Gaussian);
 *   k: number of lowest eigenvalues; tol: stop when the k-th lowest Ritz
 *       value changes by <= tol * |value| between iterations (0 = run
 *       max_iter iterations); breakdown (beta <= 1e-13 max(1,|alpha|)) stops;
 *   prec: XDG_PREC_*;
 *   evals: host double[k]; n_iter: host int (iterations done);
 *   alpha, beta: host double[max_iter] or NULL: the tridiagonal matrix,
 *       beta[j] couples j and j+1 (beta[n_iter-1] is the last residual norm).
 * Returns XDG_OK, or XDG_ENOCONV when tol > 0 was not reached. */
int xdg_lanczos_eigval(xdg_ham h, const void *v0, int k, double tol, int max_iter, uint64_t seed,
                       int prec, double *evals, int *n_iter, double *alpha, double *beta,
                       void *stream);

/* n blocks x nvec independent Lanczos recurrences advanced in lockstep; each
 * step is one batched application (xdg_apply_batched) plus batched vector
 * operations, replayed from a captured HIP graph.  Fixed iteration count.
 *   v0s: n device pointers [dim_i][nvec] or NULL (seeds seed + i);
 *   prec: XDG_PREC_F64 or XDG_PREC_F32VEC (vector dtype complex if any block
 *         is complex, so that all blocks share one dtype);
 *   evals: host double[n * nvec] lowest Ritz value of each recurrence
 *         (block-major); alpha, beta: host double[n * nvec * n_iter] or NULL. */
int xdg_lanczos_eigval_batched(int n, const xdg_ham *hams, const void *const *v0s, int64_t nvec,
                               int n_iter, uint64_t seed, int prec, double *evals, double *alpha,
                               double *beta, void *stream);

/* Second Lanczos pass: the Ritz vector of T (eig0 / eigs_lanczos, Sec. 3.7.1,
 * which run the iteration twice to build eigenvectors without storing the
 * Krylov basis).  The recurrence of xdg_lanczos_eigval is replayed from the
 * same start vector with the tridiagonal matrix it returned, and
 * psi = sum_j c_j v_j is accumulated in FP64, c the normalised eigenvector
 * (c_0 >= 0) of the Ritz value number `which` (0 = lowest) of the leading
 * n_iter x n_iter block of T.  The vectors v_j equal those of the first pass
 * bit for bit (same kernels, same scalars).
 *   v0, seed, prec: as passed to xdg_lanczos_eigval (prec XDG_PREC_F64 or
 *       XDG_PREC_F32VEC; the forms with reorthogonalisation are refused);
 *   alpha, beta: host double[n_iter] from xdg_lanczos_eigval;
 *   psi: device [dim] of the precision form's vector dtype, normalised
 *       (FP64 accumulation, one rounding); may not alias v0.
 *   ritz (may be NULL): host double, the Ritz value used. */
int xdg_lanczos_eigvec(xdg_ham h, const void *v0, uint64_t seed, int prec, int n_iter,
                       const double *alpha, const double *beta, int which, void *psi,
                       double *ritz, void *stream);

/* <psi| O |psi> (measurements, Sec. 3.8) for the symmetrised Ising
 * correlations O = (1/|G|) sum_g S^z_{g(a)} S^z_{g(b)} (symmetrisation of an
 * operator over the group, Sec. 3.13).  It is diagonal in the symmetric basis with
 * value (1/|G|) sum_g sz_s(g(a)) sz_s(g(b)) on state s (sz = +-1/2), and for a
 * state of the block it equals the expectation of the plain S^z_a S^z_b.
 * On a U(1) block O = S^z_a S^z_b.  psi is not normalised by the call.
 *   psi: device [dim] of dtype; pairs: host int32[2 n_pairs] (a, b) in [0, N);
 *   out: host double[n_pairs].  Fixed-order reductions (reproducible). */
int xdg_expect_szsz(xdg_basis b, const void *psi, int dtype, int n_pairs, const int32_t *pairs,
                    double *out, void *stream);

/* Finite-temperature Lanczos thermodynamics (the thermodynamics examples of
 * Sec. 4.6, after Jaklic and Prelovsek): from n_rec Lanczos recurrences of m
 * steps started at random unit vectors (e.g. xdg_lanczos_eigval_batched),
 *   Z(T) = sum_r weight[r] sum_j w_rj exp(-eps_rj / T),
 * eps_rj the Ritz values and w_rj the squared first components of the Ritz
 * vectors of recurrence r (the Gauss quadrature of <r|f(H)|r>); weight[r] =
 * block dimension / number of vectors in that block.  A breakdown
 * (beta_j <= 1e-13 max(1, |alpha_j|)) ends a recurrence at step j.
 *   alpha, beta: host double[n_rec][m] (layout of xdg_lanczos_eigval_batched);
 *   temps: host double[n_temp] > 0; outputs host double[n_temp]:
 *   energy <H>, heat (<H^2> - <H>^2) / T^2, log_z = ln Z.  Host only. */
int xdg_ftlm_thermo(int n_rec, int m, const double *alpha, const double *beta,
                    const double *weight, int n_temp, const double *temps, double *energy,
                    double *heat, double *log_z);

/* Microcanonical thermal pure quantum states (the thermodynamics examples of
 * Sec. 4.6; the construction of Sugiura and Shimizu 2012): from a unit start
 * vector |0> (v0 normalised by the call, or the seeded Gaussian vector of
 * xdg_random_vector kind 1 when v0 is NULL) the sequence
 *   |k+1> = (l - H/N)|k> / || (l - H/N)|k> ||,   N = number of sites,
 * one H x per step, recording for k = 0 .. n_steps - 1
 *   u[k] = <k|H|k> / N,   u2[k] = <k|H^2|k> / N^2   (FP64 products).
 * l must be at least the largest eigenvalue of H/N on the block for the
 * sequence to run from high to low energy.
 *   v0: device [dim] of the block's dtype for prec, or NULL; prec:
 *   XDG_PREC_F64 or XDG_PREC_F32VEC; u, u2: host double[n_steps].
 * Synchronises `stream` once, at the end. */
int xdg_tpq_micro(xdg_ham h, const void *v0, uint64_t seed, int prec, double l, int n_steps,
                  double *u, double *u2, void *stream);

/* xdg_tpq_micro for n blocks x nvec start vectors in lockstep: one batched
 * H x per step over every block (the persistent launch of
 * xdg_apply_batched), per-vector FP64 products, one captured step replayed
 * n_steps times.  Start blocks v0s[i]: device [dim_i][nvec] (complex if any
 * block is), normalised per vector by the call; v0s NULL: the seeded
 * Gaussian block of seed + i for block i.  nvec in {1, 2, 4, 8}; prec
 * XDG_PREC_F64 or XDG_PREC_F32VEC.  u, u2: host double[n][nvec][n_steps].
 * Synchronises `stream` (or a stream of its own when NULL) at the end. */
int xdg_tpq_micro_batched(int n, const xdg_ham *hams, const void *const *v0s, int64_t nvec,
                          uint64_t seed, int prec, double l, int n_steps, double *u, double *u2,
                          void *stream);

/* Canonical TPQ thermodynamics from n_rec microcanonical sequences of
 * n_steps (Sec. 4.6; Sugiura and Shimizu 2013): with h = H/N, the moments
 * M_n = <0|(l - h)^n|0> for n <= 2 n_steps follow from u and u2
 * (q_0 = 1, q_{k+1} = q_k (l^2 - 2 l u_k + u2_k), M_{2k} = q_k,
 * M_{2k+1} = q_k (l - u_k)); with x = N / T and S_j = sum_n M_{n+j} x^n / n!,
 * summed over the sequences with their weights,
 *   ln Z = ln sum_r weight[r] S_0 - x l,   <H> = N (l - S_1 / S_0),
 *   heat = x^2 (S_2 / S_0 - (S_1 / S_0)^2)   (= (<H^2> - <H>^2) / T^2).
 * weight[r] = block dimension / number of sequences in that block.  NaN at a
 * temperature where a truncated series has not converged (last kept term
 * not below 1e-12 of its sum): more steps are needed there.
 * XDG_EINVAL if l < u[k] anywhere, a weight or temperature is not > 0.
 *   u, u2: host double[n_rec][n_steps]; temps: host double[n_temp];
 *   energy, heat, log_z: host double[n_temp].  Host only. */
int xdg_tpq_thermo(int n_rec, int n_steps, const double *u, const double *u2, double l,
                   int n_sites, const double *weight, int n_temp, const double *temps,
                   double *energy, double *heat, double *log_z);

/* y = O x for the one-site diagonal operator O = sum_j c_j S^z_j taking a
 * vector of block `in` to block `out` (an operator at momentum q from the
 * symmetrisation of Sec. 3.13, e.g. c_j = e^{i q j} / sqrt(N); dynamical
 * structure factors, Sec. 4.4).  The blocks need the same sites, n_up and
 * group, and c must carry the character ratio:
 * c_{g^-1(i)} = (chi_in(g) / chi_out(g)) c_i for all g, i (else
 * XDG_ENOTSYM); then y[r] = o(s_r) x[index_in(s_r)] with
 * o(s) = sum_j c_j sz_s(j), and 0 where s_r has no state in `in`.
 *   coef: host double[2 n_sites] (re, im); x: device [dim_in], y: device
 *   [dim_out] of dtype (complex unless c and both blocks are real). */
int xdg_apply_sz_transfer(xdg_basis in, xdg_basis out, const double *coef, const void *x,
                          void *y, int dtype, void *stream);

/* Spectral function from a Lanczos recurrence started at phi / |phi| (the
 * continued fraction of <phi|(z - H)^-1|phi>, Sec. 4.4):
 *   S(omega) = -Im[ norm2 / (z - a_0 - b_0^2 / (z - a_1 - ...)) ] / pi,
 *   z = omega + e0 + i eta;  a breakdown ends the fraction.
 *   alpha, beta: host double[m]; norm2 = <phi|phi>; out: host double[n_omega].
 * Host only. */
int xdg_spectral_cf(int m, const double *alpha, const double *beta, double norm2, double e0,
                    int n_omega, const double *omega, double eta, double *out);

/* Timing of the last xdg_lanczos_eigval[_batched] call on this thread:
 * total seconds in the iteration loop and seconds spent in the apply
 * kernels (HIP events); either may be NULL. */
int xdg_last_lanczos_timing(double *total_s, double *apply_s);

#ifdef __cplusplus
}
#endif

#endif /* XDG_H */
