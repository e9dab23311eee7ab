// gibbs_tiles_a.hip -- compiled (L, R) variants of the Gibbs kernel, part a.
#include "gibbs_kernel.h"

namespace crbmlib {

#define TILE(l, r)                                              \
    if (L == l && R == r) {                                     \
        if (a) *err = gk::launch_tile<l, r>(*a, st);            \
        if (fn) *fn = gk::kernel_ptr<l, r>();                   \
        return true;                                            \
    }

bool tiles_a(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err,
             const void** fn) {
    TILE(4, 1)
    TILE(4, 2)
    TILE(6, 1)
    TILE(6, 3)
    TILE(8, 1)
    TILE(8, 2)
    TILE(8, 4)
    TILE(10, 1)
    TILE(10, 5)
    TILE(12, 1)
    TILE(12, 2)
    TILE(12, 3)
    TILE(12, 6)
    TILE(14, 1)
    TILE(14, 7)
    TILE(16, 1)
    TILE(16, 2)
    TILE(16, 4)
    TILE(16, 8)
    return false;
}

}  // namespace crbmlib
