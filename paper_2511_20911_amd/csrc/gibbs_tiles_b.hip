// gibbs_tiles_b.hip -- compiled (L, R) variants of the Gibbs kernel, part b.
#include "gibbs_kernel.h"

namespace crbmlib {

#define TILE(l, r)                                              \
    if (L == l && R == r) {                                     \
        if (a) *err = gk::launch_tile<l, r>(*a, st);            \
        if (fn) *fn = gk::kernel_ptr<l, r>();                   \
        return true;                                            \
    }

bool tiles_b(int L, int R, const GibbsArgs* a, hipStream_t st, hipError_t* err,
             const void** fn) {
    TILE(18, 1)
    TILE(18, 3)
    TILE(18, 9)
    TILE(20, 1)
    TILE(20, 2)
    TILE(20, 5)
    TILE(22, 1)
    TILE(22, 11)
    TILE(24, 1)
    TILE(24, 2)
    TILE(24, 3)
    TILE(24, 4)
    TILE(24, 6)
    TILE(26, 1)
    TILE(26, 13)
    return false;
}

}  // namespace crbmlib
