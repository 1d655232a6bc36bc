// Instantiation of the sublattice apply kernels that read the rank-addressed x,
// for blocks whose characters are all 1 (real blocks).
#include "apply_impl.hpp"

namespace xdg {

int launch_sub_xr_trivial(bool wide, bool single, bool acc64, int nv, const ApplyArgs &A,
                          unsigned grid, unsigned block, size_t lds, hipStream_t st) {
    return wide ? launch_prec<uint64_t, K_SUB, false, 2>(single, acc64, nv, A, grid, block, lds, st)
                : launch_prec<uint32_t, K_SUB, false, 2>(single, acc64, nv, A, grid, block, lds, st);
}

}  // namespace xdg
