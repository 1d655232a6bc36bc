// Instantiation of the sublattice apply kernels that read the rank-addressed x.
#include "apply_impl.hpp"

namespace xdg {

int launch_sub_xr(bool wide, bool single, bool acc64, bool cplx, int nv, const ApplyArgs &A,
                  unsigned grid, unsigned block, size_t lds, hipStream_t st) {
    return launch_kind_impl<K_SUB, 1>(wide, single, acc64, cplx, nv, A, grid, block, lds, st);
}

}  // namespace xdg
