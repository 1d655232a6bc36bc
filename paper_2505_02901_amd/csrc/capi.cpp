// The C ABI of include/xdg.h: argument checks, handle lifetime, dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "xdg_internal.hpp"

using namespace xdg;

namespace xdg {
int last_timing(double *total, double *apply);
}

namespace {

void basis_release(xdg_basis_s *b) {
    if (b && b->refs.fetch_sub(1) == 1) delete b;
}

template <class F>
int guarded(F &&f) {
    try {
        return f();
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return XDG_ENOMEM;
    } catch (...) {
        set_error("unexpected C++ exception");
        return XDG_EINVAL;
    }
}

}  // namespace

extern "C" {

const char *xdg_version(void) { return "xdg-mi355x 0.1.0 (gfx950, HIP)"; }

const char *xdg_last_error(void) { return get_error(); }

int xdg_check_group(int n_sites, int n_sym, const int32_t *perm, const double *chi) {
    return guarded([&] { return validate_group(n_sites, n_sym, perm, chi); });
}

int xdg_check_bonds(int n_sites, int n_sym, const int32_t *perm, int n_bonds,
                    const int32_t *sites, const double *jz, const double *jxy) {
    return guarded([&] {
        XDG_RETURN_IF(validate_group(n_sites, n_sym, perm, nullptr));
        return validate_bonds(n_sites, n_sym, perm, n_bonds, sites, jz, jxy);
    });
}

int xdg_plan_search(int n_sites, int n_sym, const int32_t *perm, const xdg_basis_opts *opts,
                    int *kind, int *n_sublattices) {
    return guarded([&] {
        XDG_RETURN_IF(validate_group(n_sites, n_sym, perm, nullptr));
        Plan p;
        XDG_RETURN_IF(make_plan(n_sites, n_sym, perm, opts, &p, false));
        if (kind) *kind = p.kind;
        if (n_sublattices) *n_sublattices = p.kind == XDG_SEARCH_SUBLATTICE ? p.sub.n_s : 0;
        return XDG_OK;
    });
}

int xdg_create_basis(int n_sites, int n_up, int n_sym, const int32_t *perm, const double *chi,
                     const xdg_basis_opts *opts, xdg_basis *out) {
    return guarded([&]() -> int {
        if (!out) {
            set_error("out is NULL");
            return XDG_EINVAL;
        }
        *out = nullptr;
        if (n_sites < 1 || n_sites > 64) {
            set_error("n_sites = %d outside [1, 64]", n_sites);
            return XDG_EINVAL;
        }
        if (n_up < 0 || n_up > n_sites) {
            set_error("n_up = %d outside [0, %d]", n_up, n_sites);
            return XDG_EINVAL;
        }
        XDG_RETURN_IF(validate_group(n_sites, n_sym, perm, chi));
        auto *b = new xdg_basis_s();
        b->n_sites = n_sites;
        b->n_up = n_up;
        b->n_sym = n_sym;
        b->wide = n_sites > 32;
        if (n_sym) {
            b->perm.assign(perm, perm + (size_t)n_sym * n_sites);
            // a plain copy, then a separate scan of the imaginary parts: the
            // fused copy-and-test loop was vectorised by the host compiler
            // into code that tests one entry past the end of chi
            if (chi) {
                b->chi.assign(chi, chi + 2 * (size_t)n_sym);
            } else {
                b->chi.assign(2 * (size_t)n_sym, 0.0);
                for (int g = 0; g < n_sym; ++g) b->chi[2 * (size_t)g] = 1.0;
            }
            bool cplx = false;
            for (size_t e = 1; e < b->chi.size(); e += 2) cplx |= std::fabs(b->chi[e]) > 1e-13;
            b->is_complex = cplx;
        }
        int rc = make_plan(n_sites, n_sym, n_sym ? b->perm.data() : nullptr, opts, &b->plan, true);
        if (rc == XDG_OK) {
            hipError_t e = hipGetDevice(&b->device);
            if (e != hipSuccess) {
                set_error("no HIP device: %s", hipGetErrorString(e));
                rc = XDG_EHIP;
            }
        }
        if (rc == XDG_OK) rc = basis_build_device(b);
        if (rc != XDG_OK) {
            delete b;
            return rc;
        }
        *out = b;
        return XDG_OK;
    });
}

void xdg_destroy_basis(xdg_basis b) { basis_release(b); }

int xdg_basis_dim(xdg_basis b, int64_t *dim) {
    if (!b || !dim) {
        set_error("null argument");
        return XDG_EINVAL;
    }
    *dim = b->dim;
    return XDG_OK;
}

int xdg_basis_is_complex(xdg_basis b, int *is_complex) {
    if (!b || !is_complex) {
        set_error("null argument");
        return XDG_EINVAL;
    }
    *is_complex = b->is_complex ? 1 : 0;
    return XDG_OK;
}

int xdg_basis_search_kind(xdg_basis b, int *kind, int *n_sublattices) {
    if (!b) {
        set_error("null basis");
        return XDG_EINVAL;
    }
    if (kind) *kind = b->plan.kind;
    if (n_sublattices) *n_sublattices = b->plan.kind == XDG_SEARCH_SUBLATTICE ? b->plan.sub.n_s : 0;
    return XDG_OK;
}

int xdg_basis_index_kind(xdg_basis b, int *kind, int64_t *bytes) {
    if (!b) {
        set_error("null basis");
        return XDG_EINVAL;
    }
    int k = XDG_INDEX_LIN;
    size_t n = b->lin.bytes;
    if (b->plan.kind != XDG_SEARCH_U1) {
        k = b->n_rwords ? XDG_INDEX_RANK : XDG_INDEX_HASH;
        n = b->n_rwords ? b->rwords.bytes + b->rtab.bytes : b->hash.bytes;
    }
    if (kind) *kind = k;
    if (bytes) *bytes = (int64_t)n;
    return XDG_OK;
}

int xdg_basis_copy_states(xdg_basis b, int64_t begin, int64_t count, uint64_t *host_out) {
    return guarded([&]() -> int {
        if (!b || (count > 0 && !host_out) || begin < 0 || count < 0 || begin + count > b->dim) {
            set_error("bad range [%lld, +%lld) for dimension %lld", (long long)begin,
                      (long long)count, b ? (long long)b->dim : -1LL);
            return XDG_EINVAL;
        }
        if (count == 0) return XDG_OK;
        if (b->wide) {
            XDG_RETURN_IF(copy_d2h(host_out, b->reps.as<uint64_t>() + begin, 8 * (size_t)count,
                                   nullptr));
        } else {
            std::vector<uint32_t> tmp((size_t)count);
            XDG_RETURN_IF(copy_d2h(tmp.data(), b->reps.as<uint32_t>() + begin, 4 * (size_t)count,
                                   nullptr));
            for (int64_t i = 0; i < count; ++i) host_out[i] = tmp[(size_t)i];
        }
        return XDG_OK;
    });
}

int xdg_basis_copy_stabilisers(xdg_basis b, int64_t begin, int64_t count, int32_t *host_out) {
    return guarded([&]() -> int {
        if (!b || (count > 0 && !host_out) || begin < 0 || count < 0 || begin + count > b->dim) {
            set_error("bad range");
            return XDG_EINVAL;
        }
        if (count == 0) return XDG_OK;
        if (b->n_sym == 0) {
            std::fill(host_out, host_out + count, 1);
            return XDG_OK;
        }
        std::vector<uint16_t> tmp((size_t)count);
        XDG_RETURN_IF(copy_d2h(tmp.data(), b->stab.as<uint16_t>() + begin, 2 * (size_t)count,
                               nullptr));
        for (int64_t i = 0; i < count; ++i) host_out[i] = tmp[(size_t)i];
        return XDG_OK;
    });
}

int xdg_basis_index(xdg_basis b, const uint64_t *states, int64_t n, int64_t *idx_out) {
    return guarded([&]() -> int {
        if (!b || n < 0 || (n > 0 && (!states || !idx_out))) {
            set_error("bad arguments");
            return XDG_EINVAL;
        }
        if (n == 0) return XDG_OK;
        if (b->dim == 0) {
            std::fill(idx_out, idx_out + n, -1);
            return XDG_OK;
        }
        DevBuf ds, di;
        XDG_RETURN_IF(ds.upload(states, 8 * (size_t)n));
        XDG_RETURN_IF(di.alloc(8 * (size_t)n));
        XDG_RETURN_IF(basis_lookup(b, ds.as<uint64_t>(), n, di.as<int64_t>(), 0));
        XDG_RETURN_IF(copy_d2h(idx_out, di.p, 8 * (size_t)n, nullptr));
        return XDG_OK;
    });
}

int xdg_create_hamiltonian(xdg_basis b, int n_bonds, const int32_t *sites, const double *jz,
                           const double *jxy, xdg_ham *out) {
    return guarded([&]() -> int {
        if (!b || !out) {
            set_error("null argument");
            return XDG_EINVAL;
        }
        *out = nullptr;
        XDG_RETURN_IF(validate_bonds(b->n_sites, b->n_sym, b->perm.data(), n_bonds, sites, jz, jxy));
        static std::atomic<uint64_t> next_serial{1};
        auto *h = new xdg_ham_s();
        h->serial = next_serial.fetch_add(1);
        h->basis = b;
        b->refs.fetch_add(1);
        h->n_bonds = n_bonds;
        h->sites.assign(sites, sites + 2 * (size_t)n_bonds);
        h->jz.assign(jz, jz + n_bonds);
        h->jxy.assign(jxy, jxy + n_bonds);
        // device bond order: for sublattice coding, bonds joining the same pair
        // of blocks are kept together (stable), so that bonds taken one after
        // the other change the same two blocks of a state
        std::vector<int> order(n_bonds);
        for (int i = 0; i < n_bonds; ++i) order[i] = i;
        if (b->plan.kind == XDG_SEARCH_SUBLATTICE && b->plan.sub.m > 0) {
            const int m = b->plan.sub.m;
            auto key = [&](int k) {
                const int p = sites[2 * k] / m, q = sites[2 * k + 1] / m;
                return std::min(p, q) * 64 + std::max(p, q);
            };
            std::stable_sort(order.begin(), order.end(),
                             [&](int a, int c) { return key(a) < key(c); });
        }
        std::vector<BondD> bd(n_bonds);
        std::vector<BondF> bf(n_bonds);
        for (int e = 0; e < n_bonds; ++e) {
            const int i = order[e];
            bd[e] = BondD{(uint32_t)sites[2 * i], (uint32_t)sites[2 * i + 1], jz[i], 0.5 * jxy[i]};
            bf[e] = BondF{bd[e].i, bd[e].j, (float)jz[i], (float)(0.5 * jxy[i])};
        }
        int rc = h->bonds_d.upload(bd.data(), sizeof(BondD) * std::max(n_bonds, 1));
        if (rc == XDG_OK) rc = h->bonds_f.upload(bf.data(), sizeof(BondF) * std::max(n_bonds, 1));
        const auto &sp = b->plan.sub;
        if (rc == XDG_OK && b->plan.kind == XDG_SEARCH_SUBLATTICE &&
            sub_packed_ok(sp.n_s, sp.m, sp.pb)) {
            std::vector<BondX> bx(std::max(n_bonds, 1), BondX{});
            for (int e = 0; e < n_bonds; ++e) {
                bondx_site((int)bd[e].i, sp.m, sp.pb, bx[e]);
                bondx_site((int)bd[e].j, sp.m, sp.pb, bx[e]);
            }
            rc = h->bonds_x.upload(bx.data(), sizeof(BondX) * bx.size());
        }
        if (rc != XDG_OK) {
            basis_release(h->basis);
            delete h;
            return rc;
        }
        *out = h;
        return XDG_OK;
    });
}

void xdg_destroy_hamiltonian(xdg_ham h) {
    if (!h) return;
    basis_release(h->basis);
    delete h;
}

int xdg_ham_nnz(xdg_ham h, int64_t *nnz) {
    return guarded([&]() -> int {
        if (!h || !nnz) {
            set_error("null argument");
            return XDG_EINVAL;
        }
        return ham_count_nnz(h, nnz);
    });
}

int xdg_set_device_memory_limit(int64_t bytes, int64_t *in_use) {
    if (bytes < 0) {
        set_error("memory limit must be >= 0");
        return XDG_EINVAL;
    }
    set_device_memory_limit((uint64_t)bytes);
    if (in_use) *in_use = (int64_t)device_memory_in_use();
    return XDG_OK;
}

int xdg_ham_dim(xdg_ham h, int64_t *dim, int *is_complex) {
    return guarded([&]() -> int {
        if (!h) {
            set_error("null hamiltonian");
            return XDG_EINVAL;
        }
        if (dim) *dim = h->basis->dim;
        if (is_complex) *is_complex = h->basis->is_complex ? 1 : 0;
        return XDG_OK;
    });
}

int xdg_apply(xdg_ham h, const void *x, void *y, int64_t nvec, int dtype, void *stream) {
    return guarded([&]() -> int {
        if (!h) {
            set_error("null hamiltonian");
            return XDG_EINVAL;
        }
        return apply_tuned(h, x, y, nvec, dtype, (hipStream_t)stream);
    });
}

int xdg_apply_batched(int n, const xdg_ham *hams, const void *const *xs, void *const *ys,
                      int64_t nvec, int dtype, void *stream) {
    return guarded([&]() -> int {
        if (n < 1 || !hams || !xs || !ys) {
            set_error("bad batched arguments");
            return XDG_EINVAL;
        }
        std::vector<xdg_ham_s *> hv(hams, hams + n);
        return apply_batched_launch(n, hv.data(), xs, ys, nvec, dtype, (hipStream_t)stream,
                                    nullptr, 0, 256);
    });
}

int xdg_apply_with_config(xdg_ham h, const void *x, void *y, int64_t nvec, int dtype,
                          const xdg_launch_cfg *cfg, void *stream) {
    return guarded([&]() -> int {
        if (!h || !cfg) {
            set_error("null argument");
            return XDG_EINVAL;
        }
        const bool nv_ok = cfg->nv == 0 || cfg->nv == 1 || cfg->nv == 2 || cfg->nv == 4 ||
                           cfg->nv == 8;
        bool res_ok = true;
        for (int r : cfg->reserved) res_ok &= r == 0;
        if (cfg->grid < 0 || !nv_ok || cfg->occ < -1 || cfg->occ > 1 || cfg->compact < -1 ||
            cfg->compact > 1 || (cfg->sub_form != 0 && cfg->sub_form != 2) || cfg->xr < 0 ||
            cfg->xr > 1 || !res_ok) {
            set_error("launch shape out of range (grid %d, nv %d, occ %d, compact %d, sub_form %d, "
                      "xr %d)", cfg->grid, cfg->nv, cfg->occ, cfg->compact, cfg->sub_form,
                      cfg->xr);
            return XDG_EINVAL;
        }
        LaunchCfg c;
        c.grid = cfg->grid > 0 ? cfg->grid
                               : (int)std::max<int64_t>(1, (h->basis->dim + 1023) / 1024);
        c.nv = cfg->nv > 0 ? cfg->nv : 8;
        c.occ = cfg->occ;
        c.compact = cfg->compact;
        c.sub_form = cfg->sub_form;
        c.xr = cfg->xr;
        return apply_launch(h, x, y, nvec, dtype, (hipStream_t)stream, &c);
    });
}

int xdg_apply_tuned_config(xdg_ham h, int dtype, int64_t nvec, xdg_launch_cfg *out) {
    return guarded([&]() -> int {
        if (!h || !out) {
            set_error("null argument");
            return XDG_EINVAL;
        }
        LaunchCfg c;
        XDG_RETURN_IF(apply_tuned_config(h, dtype, nvec, &c));
        *out = xdg_launch_cfg{};
        out->grid = c.grid;
        out->nv = c.nv;
        out->occ = c.occ;
        out->compact = c.compact;
        out->sub_form = c.sub_form;
        out->xr = c.xr;
        return XDG_OK;
    });
}

int xdg_apply_batched_noalloc(int n, const xdg_ham *hams, const void *const *xs,
                              void *const *ys, int64_t nvec, int dtype, void *stream) {
    return guarded([&]() -> int {
        if (n < 1 || !hams || !xs || !ys) {
            set_error("bad batched arguments");
            return XDG_EINVAL;
        }
        return apply_batched_noalloc(n, const_cast<xdg_ham_s *const *>(hams), xs, ys, nvec,
                                     dtype, (hipStream_t)stream);
    });
}

int xdg_random_state(int64_t dim, int64_t nvec, uint64_t seed, int kind, int dtype, void *out,
                     void *stream) {
    return guarded([&]() -> int {
        if (dim < 0 || nvec < 1 || (kind != 0 && kind != 1) || dtype < XDG_F64 ||
            dtype > XDG_C64 || (dim > 0 && !out)) {
            set_error("bad random_state arguments");
            return XDG_EINVAL;
        }
        const int64_t n = dim * nvec * (dtype_complex(dtype) ? 2 : 1);
        return random_fill(n, seed, kind, dtype_single(dtype), out, (hipStream_t)stream);
    });
}

int xdg_lanczos_eigval(xdg_ham h, const void *v0, int k, double tol, int max_iter, uint64_t seed,
                       int prec, double *evals, int *n_iter, double *alpha, double *beta,
                       void *stream) {
    return guarded([&]() -> int {
        if (!h) {
            set_error("null hamiltonian");
            return XDG_EINVAL;
        }
        return lanczos_single(h, v0, k, tol, max_iter, seed, prec, evals, n_iter, alpha, beta,
                              (hipStream_t)stream, nullptr, nullptr);
    });
}

int xdg_lanczos_eigval_batched(int n, const xdg_ham *hams, const void *const *v0s, int64_t nvec,
                               int n_iter, uint64_t seed, int prec, double *evals, double *alpha,
                               double *beta, void *stream) {
    return guarded([&]() -> int {
        if (n < 1 || !hams) {
            set_error("bad batched arguments");
            return XDG_EINVAL;
        }
        std::vector<xdg_ham_s *> hv(hams, hams + n);
        return lanczos_batched(n, hv.data(), v0s, nvec, n_iter, seed, prec, evals, alpha, beta,
                               (hipStream_t)stream, nullptr, nullptr);
    });
}

int xdg_lanczos_eigvec(xdg_ham h, const void *v0, uint64_t seed, int prec, int n_iter,
                       const double *alpha, const double *beta, int which, void *psi,
                       double *ritz, void *stream) {
    return guarded([&]() -> int {
        if (!h) {
            set_error("null hamiltonian");
            return XDG_EINVAL;
        }
        return lanczos_eigvec(h, v0, seed, prec, n_iter, alpha, beta, which, psi, ritz,
                              (hipStream_t)stream);
    });
}

int xdg_expect_szsz(xdg_basis b, const void *psi, int dtype, int n_pairs, const int32_t *pairs,
                    double *out, void *stream) {
    return guarded([&]() -> int {
        if (!b) {
            set_error("null basis");
            return XDG_EINVAL;
        }
        return expect_szsz(b, psi, dtype, n_pairs, pairs, out, (hipStream_t)stream);
    });
}

int xdg_ftlm_thermo(int n_rec, int m, const double *alpha, const double *beta,
                    const double *weight, int n_temp, const double *temps, double *energy,
                    double *heat, double *log_z) {
    return guarded([&]() -> int {
        return ftlm_thermo(n_rec, m, alpha, beta, weight, n_temp, temps, energy, heat, log_z);
    });
}

int xdg_tpq_micro(xdg_ham h, const void *v0, uint64_t seed, int prec, double l, int n_steps,
                  double *u, double *u2, void *stream) {
    return guarded([&]() -> int {
        if (!h) {
            set_error("null hamiltonian");
            return XDG_EINVAL;
        }
        return tpq_micro(h, v0, seed, prec, l, n_steps, u, u2, (hipStream_t)stream);
    });
}

int xdg_tpq_micro_batched(int n, const xdg_ham *hams, const void *const *v0s, int64_t nvec,
                          uint64_t seed, int prec, double l, int n_steps, double *u, double *u2,
                          void *stream) {
    return guarded([&]() -> int {
        if (n < 1 || !hams) {
            set_error("batched tpq: need n >= 1 Hamiltonians");
            return XDG_EINVAL;
        }
        return tpq_micro_batched(n, hams, v0s, nvec, seed, prec, l, n_steps, u, u2,
                                 (hipStream_t)stream);
    });
}

int xdg_tpq_thermo(int n_rec, int n_steps, const double *u, const double *u2, double l,
                   int n_sites, const double *weight, int n_temp, const double *temps,
                   double *energy, double *heat, double *log_z) {
    return guarded([&]() -> int {
        return tpq_thermo(n_rec, n_steps, u, u2, l, n_sites, weight, n_temp, temps, energy, heat,
                          log_z);
    });
}

int xdg_apply_sz_transfer(xdg_basis in, xdg_basis out, const double *coef, const void *x,
                          void *y, int dtype, void *stream) {
    return guarded([&]() -> int {
        if (!in || !out) {
            set_error("null basis");
            return XDG_EINVAL;
        }
        return apply_diag_transfer(in, out, coef, x, y, dtype, (hipStream_t)stream);
    });
}

int xdg_spectral_cf(int m, const double *alpha, const double *beta, double norm2, double e0,
                    int n_omega, const double *omega, double eta, double *out) {
    return guarded([&]() -> int {
        return spectral_cf(m, alpha, beta, norm2, e0, n_omega, omega, eta, out);
    });
}

int xdg_last_lanczos_timing(double *total_s, double *apply_s) {
    return last_timing(total_s, apply_s);
}

}  // extern "C"
