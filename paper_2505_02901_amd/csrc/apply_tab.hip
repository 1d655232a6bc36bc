// Instantiation of the apply / count kernels for one search kind.
#include "apply_impl.hpp"

namespace xdg {

template <>
int launch_kind<K_TAB>(bool wide, bool single, bool acc64, bool cplx, int nv, const ApplyArgs &A,
                    unsigned grid, unsigned block, size_t lds, hipStream_t st) {
    return launch_kind_impl<K_TAB>(wide, single, acc64, cplx, nv, A, grid, block, lds, st);
}

template <>
int launch_count_kind<K_TAB>(bool wide, const ApplyArgs &A, unsigned grid, unsigned block, size_t lds,
                          hipStream_t st) {
    return launch_count_impl<K_TAB>(wide, A, grid, block, lds, st);
}

}  // namespace xdg
